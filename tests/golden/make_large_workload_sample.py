"""Writes large_workload_solution_sample.npz: the oracle's solution p* of the
large workload (leaf levels 7..10, 8 seeded refinement spheres and a solid
box, jittered face fractions, Dirichlet top wall, seeded zero-mean right-hand
side; about 26.3M leaves) at relative residual 1e-13, sampled at 32768 seeded
active leaves, with its full 2-norm and the solve's statistics.  The GPU
tests and the benchmark compare their solutions of that workload with this
sample (the full solve takes minutes on the host, the sample a few hundred
kilobytes).  Calls the oracle only.

    python tests/golden/make_large_workload_sample.py
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import problems  # noqa: E402
from oracle import discretize as D  # noqa: E402
from oracle import krylov as K  # noqa: E402
from oracle import multigrid as M  # noqa: E402
from oracle import octree as O  # noqa: E402

OUT = os.path.join(HERE, "large_workload_solution_sample.npz")
CFG = 4
N_SAMPLE = 32768
SEED = 4242
RTOL = 1e-13


def main():
    t0 = time.time()
    T = O.Octree(problems.config_spec(CFG))
    bc, th = problems.config_bc(CFG)
    disc = D.Discretization(T, None, bc, th)
    disc.set_beta(problems.face_beta(CFG, disc.face_level, disc.face_ijk, disc.face_dir))
    rhs = problems.rhs_random(CFG, T.level, T.ijk)
    H = M.Hierarchy(disc, coarsest=3)
    print(f"{T.n} leaves, {int(disc.active.sum())} active; set up in {time.time() - t0:.0f} s",
          flush=True)
    x, info = K.pcg(disc.A, rhs, H.vcycle, RTOL, 400, active=disc.active)
    print(f"oracle solve: {info['iters']} iterations, true residual {info['true']:.2e}, "
          f"status {info['status']}", flush=True)
    assert info["status"] == 0
    act = np.nonzero(disc.active)[0]
    rng = np.random.default_rng(SEED)
    idx = np.sort(rng.choice(act, size=N_SAMPLE, replace=False)).astype(np.int64)
    np.savez_compressed(OUT, idx=idx, val=x[idx], norm=np.linalg.norm(x),
                        n_leaves=T.n, n_active=len(act), iters=info["iters"],
                        true_resid=info["true"], rtol=RTOL)
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
