"""The FAS right-hand side folded into the first pre-smoothing half-sweep
(k_smooth_fas) on levels above the coarsest with no leaf at or below them,
against k_fas_rhs followed by a plain half-sweep: the same preconditioner
output, both precisions, V- and W-cycles (the W-cycle's later visits of a
level keep the right-hand side of the first).  MFMG_FUSE_FAS=0 at hierarchy
build selects k_fas_rhs."""

import os

import numpy as np
import pytest

import problems
from gpu_fixtures import Case, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=["cut_sphere_5_7", "uniform32"])
def case(request):
    print(f"\n[case {request.param}]", flush=True)
    if request.param == "uniform32":
        return Case(1, problems.config_spec(1))
    return Case(3, problems.config_spec(3, 5, 7))


def _hierarchy(case, env, **kw):
    from paper_2604_18886_amd import mfmg
    saved = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        co = mfmg.assemble_coeffs(case.tree, case.device(case.beta), case.bc, case.theta)
        return mfmg.build_hierarchy(co, **kw)
    finally:
        for k, v in saved.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v


def test_cases_have_a_folded_level(case):
    """No leaf lies below level 5 in either case, so level 4 (above a
    coarsest level 2 with k_bottom at 3, or above a coarsest level 3 with
    the bottom in separate kernels) takes the folded half-sweep."""
    assert case.T.lmin == 5


@pytest.mark.parametrize("bottom,lc", [("1", 2), ("0", 3)])
@pytest.mark.parametrize("precision,mu", [(0, 1), (0, 2), (1, 1), (1, 2)])
def test_folded_fas_rhs_matches_separate_kernel(case, bottom, lc, precision, mu):
    from paper_2604_18886_amd import mfmg
    rng = np.random.default_rng(99)
    r = np.where(case.disc.active, rng.uniform(-1, 1, case.T.n), 0.0)
    z = []
    for fold in ("1", "0"):
        h = _hierarchy(case, {"MFMG_FUSE_FAS": fold, "MFMG_FUSE_BOTTOM": bottom},
                       coarsest_level=lc, precision=precision, mu=mu)
        z.append(mfmg.apply_precond(h, case.device(r)).cpu().numpy())
    assert np.abs(z[0]).max() > 0.0
    err = rel(z[0], z[1])
    print(f"  bottom={bottom} lc={lc} precision={precision} mu={mu}: folded vs separate "
          f"{err:.2e} (bitwise equal: {np.array_equal(z[0], z[1])})", flush=True)
    # the same values and sums in the same order
    assert err <= (1e-13 if precision == 0 else 1e-6)


def test_folded_fas_rhs_in_a_solve(case):
    """A full mixed W-cycle solve with the folded half-sweep converges to
    the tolerance in the iterations of the separate-kernel path."""
    from paper_2604_18886_amd import mfmg
    out = []
    for fold in ("1", "0"):
        h = _hierarchy(case, {"MFMG_FUSE_FAS": fold, "MFMG_FUSE_BOTTOM": "1"},
                       coarsest_level=2, precision=1, mu=2)
        p = case.device(np.zeros(case.T.n))
        _, st = mfmg.pcg_solve(h, case.device(case.rhs), p, rtol=1e-10)
        out.append((st["iters"], p.cpu().numpy()))
    assert out[0][0] == out[1][0]
    assert rel(out[0][1], out[1][1]) <= 1e-8
