"""The static projection test with cut cells (Section 4.4) on the GPU at
small root sizes: a tank with solid floor and sides and an open top, a solid
sphere or star at the centre, u = (0, -1, 0), the mixed-precision W-cycle
(mu = 2) and PCG to relative residual 1e-6 as in the paper.

The discretisation reproduces linear fields exactly (pinned on the oracle's
direct solve in tests/test_oracle_projection.py), so the discrete pressure is
the hydrostatic p = y - 1 and the projected fluid is at rest; the library's
solution is checked against that closed form, the divergence left after the
update against the solve's residual, and the per-iteration residual
reduction against the paper's statement that it exceeds five (on the
sphere; the star's sliver faces slow the tail of the iteration here, the
oracle's FP64 cycle shows the same rate)."""

import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("obstacle", ["sphere", "star"])
def test_static_projection_small_grids(obstacle):
    import torch
    sys.path.insert(0, ROOT)
    import bench
    from paper_2604_18886_amd import mfmg
    runs = []
    for l0 in (3, 4, 5):
        r = bench.static_projection(mfmg, torch, obstacle, l0, sweep_iters=4)
        print(f"  {obstacle} root 1/{2 ** l0}: {r['leaves']} leaves, {r['iters']} iterations, "
              f"reduction {r['reduction_factor']:.2f}, RMS_V div {r['rms_div_before']:.3e} -> "
              f"{r['rms_div_after']:.3e}, max|p - (y-1)| {r['p_max_err_vs_exact']:.2e}, "
              f"max|u| {r['u_max_after']:.2e}", flush=True)
        runs.append(r)
        assert r["status"] == 0
        hist = np.asarray(r["residual_history"])
        assert hist[-1] <= 1e-6
        # the paper: the residual falls fast in the first iterations ...
        assert hist[min(3, len(hist) - 1)] <= 1e-2
        # ... and by more than five per iteration on its sphere grids (on the
        # star grids sliver faces, fractions down to 1e-8, slow the tail)
        if obstacle == "sphere":
            assert r["reduction_factor"] > 5.0
        # the divergence left is the solve's residual, far below the start
        assert r["rms_div_after"] <= 1e-5 * r["rms_div_before"]
        # the pressure approaches the hydrostatic closed form with the
        # iterations (the error of an iterate, not of the discretisation)
        per = r["per_iteration"]
        errs = [q["p_max_err_vs_exact"] for q in per] + [r["p_max_err_vs_exact"]]
        assert errs[-1] <= 1e-3 * errs[0]
    # a tight solve reaches the closed form to rounding
    r = bench.static_projection(mfmg, torch, obstacle, 4, rtol=1e-12, sweep_iters=0)
    print(f"  rtol 1e-12: max|p - (y-1)| {r['p_max_err_vs_exact']:.2e}, "
          f"max|u| {r['u_max_after']:.2e}", flush=True)
    assert r["status"] == 0
    assert r["p_max_err_vs_exact"] <= 1e-9 and r["u_max_after"] <= 1e-7
