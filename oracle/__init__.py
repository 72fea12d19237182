"""FP64 CPU oracle of the matrix-free octree multigrid PCG solver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately
unoptimised restatement of the method of "Matrix-Free Multigrid with
Algebraically Consistent Coarsening on Adaptive Octrees" (Wang, Sun, Zhu):
explicit sparse matrices, explicit restriction/prolongation and explicit
Galerkin products.  Only the tests, the smoke entry point and the CPU-baseline
leg of the benchmark may import it; the product path (the HIP library and its
binding) never does, and it shares no code with that path.

Modules
  octree      node refinement, 2:1 face balance, canonical Morton leaf order
  discretize  faces, coefficients (Section 2.1, Eq. 2; Section 3.1), the
              composite leaf operator as CSR
  multigrid   level hierarchy, coarsening (Algorithm 3), level operators with
              T-junction ghosts (Eqs. 9-10), RBGS, the FAS-style cycle
              (Algorithm 4) and the standard cycle (Algorithm 2)
  krylov      PCG (Algorithm 1), adjoint solve, per-face gradient and the
              finite-difference reference

Readings where the paper is silent are listed in each module's docstring.
Parity pins that could not be tied to anything beyond the oracle itself are
marked "parity unpinned" in the docstring of the function concerned.
"""
