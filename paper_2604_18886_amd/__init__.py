"""MI355X-native matrix-free octree multigrid PCG solver.

The solver lives in libmfmg.so (HIP kernels for gfx950 behind the C ABI of
include/mfmg.h); ``paper_2604_18886_amd.mfmg`` is its ctypes binding and
``paper_2604_18886_amd.autograd`` wraps solve + adjoint as a
torch.autograd.Function.
"""

__all__ = ["mfmg"]
