"""The prolongation folded into the first two post-smoothing half-sweeps of
each level (k_smooth with PR = 1, 2) against the separate prolongation
kernel followed by plain half-sweeps: the same preconditioner output on
every small workload family (T-junctions, walls, cut cells with inactive
cells), both precisions, V- and W-cycles and odd smoothing counts.
MFMG_FUSE_PROLONG=0 at hierarchy build selects the separate kernel."""

import os

import numpy as np
import pytest

from gpu_fixtures import rel, small_cases

pytestmark = pytest.mark.gpu

CASES = small_cases()


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    print(f"\n[case {request.param}]", flush=True)
    return CASES[request.param]()


def _hierarchy(case, fused, bottom=True, **kw):
    saved = {k: os.environ.get(k) for k in ("MFMG_FUSE_PROLONG", "MFMG_FUSE_BOTTOM")}
    os.environ["MFMG_FUSE_PROLONG"] = "1" if fused else "0"
    os.environ["MFMG_FUSE_BOTTOM"] = "1" if bottom else "0"
    try:
        return case.gpu_hierarchy(**kw)
    finally:
        for k, v in saved.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v


def _outputs(case, seed, bottom=True, **kw):
    from paper_2604_18886_amd import mfmg
    rng = np.random.default_rng(seed)
    r = np.where(case.disc.active, rng.uniform(-1, 1, case.T.n), 0.0)
    z = []
    for fused in (True, False):
        h = _hierarchy(case, fused, bottom, **kw)
        z.append(mfmg.apply_precond(h, case.device(r)).cpu().numpy())
    return z


@pytest.mark.parametrize("precision,mu", [(0, 1), (0, 2), (1, 1), (1, 2)])
def test_fused_prolongation_matches_separate_kernel(case, precision, mu):
    z = _outputs(case, 95, precision=precision, mu=mu)
    assert np.abs(z[0]).max() > 0.0
    err = rel(z[0], z[1])
    print(f"  precision={precision} mu={mu}: fused vs separate {err:.2e} "
          f"(bitwise equal: {np.array_equal(z[0], z[1])})", flush=True)
    # every value the fused half-sweeps read is the one the separate kernel
    # stores, and every sum is taken in the same order
    assert err <= (1e-13 if precision == 0 else 1e-6)


@pytest.mark.parametrize("params", [
    dict(nu_pre=1, nu_post=1, mu=1),
    dict(nu_pre=0, nu_post=3, mu=2),
    dict(nu_pre=2, nu_post=0, mu=1),
])
def test_fused_prolongation_smoothing_counts(case, params):
    """One post-smoothing sweep (the fused pair only), three (plain sweeps
    after it), none (the separate kernel on both sides)."""
    z = _outputs(case, 96, precision=0, **params)
    assert np.abs(z[0]).max() > 0.0
    assert rel(z[0], z[1]) <= 1e-13


@pytest.mark.parametrize("precision,mu", [(0, 1), (1, 2)])
def test_fused_prolongation_without_the_fused_bottom(case, precision, mu):
    """With the bottom of the cycle in separate kernels the level above the
    coarsest also takes its prolongation in its post-smoothing."""
    z = _outputs(case, 98, bottom=False, precision=precision, mu=mu)
    assert np.abs(z[0]).max() > 0.0
    assert rel(z[0], z[1]) <= (1e-13 if precision == 0 else 1e-6)
