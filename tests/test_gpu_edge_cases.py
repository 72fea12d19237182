"""Edge cases of the GPU path against the oracle: a hierarchy whose finest
level is its coarsest (the cycle is the coarsest smoother alone), cycle
parameters other than the defaults (smoothing counts, coarsest level, the
coarse-correction factor), a zero right-hand side, a domain that is almost
all solid, a domain with no active cell, a solve stopped by its iteration
limit, and a right-hand side incompatible with a singular operator."""

import numpy as np
import pytest

import problems
from gpu_fixtures import Case, rel
from oracle import krylov as K
from oracle import multigrid as M

pytestmark = pytest.mark.gpu


def _seeded_rhs(case, seed):
    rng = np.random.default_rng(seed)
    return np.where(case.disc.active, rng.uniform(-1, 1, case.T.n), 0.0)


def _hierarchy(case, **prm):
    from paper_2604_18886_amd import mfmg
    co = mfmg.assemble_coeffs(case.tree, case.device(case.beta), case.bc, case.theta)
    return mfmg.build_hierarchy(co, **prm)


def test_single_level_hierarchy():
    """Uniform 8^3 grid at the coarsest level: the cycle is nu_coarse RBGS
    iterations in one workgroup; forward and transposed cycle and the solve
    against the oracle."""
    from paper_2604_18886_amd import mfmg
    spec = problems.uniform_spec(3)
    case = Case(1, spec, bc=(1, 0, 0, 1, 0, 0), theta=0.5, rhs=np.zeros(8 ** 3))
    case.rhs = _seeded_rhs(case, 60)
    H = M.Hierarchy(case.disc, coarsest=3)
    h = _hierarchy(case, coarsest_level=3)
    r = _seeded_rhs(case, 61)
    assert rel(mfmg.apply_precond(h, case.device(r)).cpu().numpy(), H.vcycle(r)) <= 1e-12
    assert rel(mfmg.apply_precond(h, case.device(r), transpose=True).cpu().numpy(),
               H.vcycle_T(r)) <= 1e-12
    p, st = mfmg.pcg_solve(h, case.device(case.rhs), rtol=1e-10)
    x, info = K.pcg(case.disc.A, case.rhs, H.vcycle, 1e-13, 400, active=case.disc.active)
    print(f"  single level: gpu iters={st['iters']} err={rel(p.cpu().numpy(), x):.2e}",
          flush=True)
    assert st["status"] == 0 and rel(p.cpu().numpy(), x) <= 1e-9


# (parameters, whether PCG converges with this cycle: without post-smoothing
# the cycle is far from symmetric and the oracle's PCG stalls too)
PARAMS = [
    (dict(nu_pre=1, nu_post=3, nu_coarse=4), True),
    (dict(nu_pre=0, nu_post=2, nu_coarse=10), True),
    (dict(nu_pre=3, nu_post=0, nu_coarse=6), False),
    (dict(nu_pre=2, nu_post=2, nu_coarse=10, coarsest_level=4), True),
    (dict(nu_pre=2, nu_post=2, nu_coarse=10, beta_mg=1.0), True),
]


@pytest.mark.parametrize("prm,solve", PARAMS, ids=[str(i) for i in range(len(PARAMS))])
def test_cycle_parameters_match_oracle(prm, solve):
    """One forward and one transposed cycle (FP64) and a mixed-precision
    solve with non-default cycle parameters."""
    from paper_2604_18886_amd import mfmg
    case = Case(3, problems.config_spec(3, 4, 6))
    lc = prm.get("coarsest_level", 3)
    H = M.Hierarchy(case.disc, coarsest=lc, beta_mg=prm.get("beta_mg", 2.0),
                    nu_pre=prm["nu_pre"], nu_post=prm["nu_post"], nu_coarse=prm["nu_coarse"])
    kw = dict(prm, coarsest_level=lc)
    h = _hierarchy(case, **kw)
    r = _seeded_rhs(case, 62)
    z = mfmg.apply_precond(h, case.device(r)).cpu().numpy()
    zt = mfmg.apply_precond(h, case.device(r), transpose=True).cpu().numpy()
    assert rel(z, H.vcycle(r)) <= 1e-12
    assert rel(zt, H.vcycle_T(r)) <= 1e-12
    if not solve:
        return
    hm = _hierarchy(case, precision=mfmg.MIXED, **kw)
    p, st = mfmg.pcg_solve(hm, case.device(case.rhs), rtol=1e-10, max_iter=400)
    x, info = K.pcg(case.disc.A, case.rhs, H.vcycle, 1e-13, 400, active=case.disc.active)
    print(f"  {prm}: mixed iters={st['iters']} oracle(1e-13)={info['iters']} "
          f"err={rel(p.cpu().numpy(), x):.2e}", flush=True)
    assert st["status"] == 0 and st["rel_resid_true"] <= 1e-10
    assert rel(p.cpu().numpy(), x) <= 1e-9


def test_zero_right_hand_side():
    """rhs = 0: no iteration, p = 0, status OK."""
    import torch
    from paper_2604_18886_amd import mfmg
    case = Case(3, problems.config_spec(3, 4, 6))
    for precision in (mfmg.FP64, mfmg.MIXED):
        h = _hierarchy(case, coarsest_level=3, precision=precision)
        p = torch.full((case.T.n,), 7.0, dtype=torch.float64, device="cuda")
        p, st = mfmg.pcg_solve(h, case.device(np.zeros(case.T.n)), p, rtol=1e-10)
        assert st["status"] == 0 and st["iters"] == 0
        assert st["rel_resid_true"] == 0.0
        assert torch.count_nonzero(p).item() == 0


def test_almost_all_solid():
    """beta = 0 on every face outside a small fluid block that reaches the
    Dirichlet (+y) wall: only the block's cells are active (whole bricks
    inactive, bricks partly active), and the solve matches the oracle's with
    inactive entries zero.  (A block closed off by beta = 0 on all sides
    would carry its own null space, which the automatic choice, keyed to a
    Dirichlet wall somewhere in the domain, does not remove.)"""
    from paper_2604_18886_amd import mfmg
    spec = problems.config_spec(2, 4, 6)
    base = Case(2, spec, bc=(0, 0, 0, 1, 0, 0), theta=0.5)
    d = base.disc
    lv = d.face_level
    h = np.ldexp(1.0, -lv.astype(np.int64))
    ctr = (d.face_ijk + 0.5) * h[:, None]
    inside = ((np.abs(ctr[:, 0] - 0.55) < 0.13) & (np.abs(ctr[:, 2] - 0.45) < 0.13)
              & (ctr[:, 1] > 0.55))
    beta = np.where(inside, 1.0, 0.0)
    case = Case(2, spec, bc=(0, 0, 0, 1, 0, 0), theta=0.5, beta=beta,
                rhs=np.zeros(base.T.n))
    act = case.disc.active
    case.rhs = _seeded_rhs(case, 63)
    print(f"  {int(act.sum())} active of {case.T.n} leaves", flush=True)
    assert 0 < act.sum() < case.T.n // 10
    for precision in (mfmg.FP64, mfmg.MIXED):
        hh = _hierarchy(case, coarsest_level=3, precision=precision)
        p, st = mfmg.pcg_solve(hh, case.device(case.rhs), rtol=1e-10)
        p = p.cpu().numpy()
        x, info = case.oracle_solve(1e-13)
        print(f"  precision={precision} iters={st['iters']} err={rel(p, x):.2e}", flush=True)
        assert st["status"] == 0 and rel(p, x) <= 1e-9
        assert np.all(p[~act] == 0.0)


def test_iteration_limit():
    """max_iter reached before rtol: NOT_CONVERGED with a warning, the
    iterate after exactly max_iter iterations (the oracle's)."""
    import warnings
    from paper_2604_18886_amd import mfmg
    case = Case(3, problems.config_spec(3, 4, 6))
    h = _hierarchy(case, coarsest_level=3)
    with warnings.catch_warnings(record=True) as w:
        warnings.simplefilter("always")
        p, st = mfmg.pcg_solve(h, case.device(case.rhs), rtol=1e-14, max_iter=3)
    assert any(issubclass(x.category, mfmg.NotConvergedWarning) for x in w)
    assert st["iters"] == 3 and st["status"] == mfmg.NOT_CONVERGED
    x3, info = K.pcg(case.disc.A, case.rhs, case.hier.vcycle, 1e-14, 3,
                     active=case.disc.active)
    assert info["iters"] == 3
    assert rel(p.cpu().numpy(), x3) <= 1e-10


def test_incompatible_right_hand_side():
    """No Dirichlet face and the null-space shift off: a right-hand side
    (or dL/dp) that does not sum to zero over the active cells has no
    solution and is rejected before any iteration; a zero-sum one is
    accepted."""
    from paper_2604_18886_amd import mfmg
    case = Case(3, problems.config_spec(3, 4, 6), bc=(0,) * 6, theta=0.5)
    act = case.disc.active
    h = _hierarchy(case, coarsest_level=3)
    rhs = _seeded_rhs(case, 64)
    rhs[act] -= rhs[act].mean()
    bad = np.where(act, rhs + 1e-3, 0.0)
    with pytest.raises(mfmg.MFMGError) as e:
        mfmg.pcg_solve(h, case.device(bad), rtol=1e-10, null_space=0)
    assert e.value.status == mfmg.INCOMPATIBLE_RHS
    p, st = mfmg.pcg_solve(h, case.device(rhs), rtol=1e-10)  # automatic shift
    assert st["status"] == 0
    with pytest.raises(mfmg.MFMGError) as e:
        mfmg.pcg_solve_adjoint(h, p, case.device(bad), rtol=1e-10, null_space=0)
    assert e.value.status == mfmg.INCOMPATIBLE_RHS


@pytest.mark.parametrize("bc", [(0, 0, 0, 1, 0, 0), (0,) * 6])
def test_no_active_cell(bc):
    """beta = 0 on every face: no leaf is a degree of freedom.  The forward
    and adjoint solves return zeros with status OK (with and without a
    Dirichlet wall, i.e. with the null-space shift on an empty active set)."""
    import torch
    from paper_2604_18886_amd import mfmg
    spec = problems.config_spec(2, 3, 5)
    base = Case(2, spec, bc=bc, theta=0.5)
    case = Case(2, spec, bc=bc, theta=0.5, beta=np.zeros(base.disc.n_faces),
                rhs=np.zeros(base.T.n))
    assert not case.disc.active.any()
    rng = np.random.default_rng(65)
    rhs = rng.uniform(-1, 1, case.T.n)  # entries of inactive leaves are ignored
    for precision in (mfmg.FP64, mfmg.MIXED):
        h = _hierarchy(case, coarsest_level=3, precision=precision)
        p, st = mfmg.pcg_solve(h, case.device(rhs), rtol=1e-10)
        assert st["status"] == 0 and st["iters"] == 0
        assert torch.count_nonzero(p).item() == 0
        lam, g, st2 = mfmg.pcg_solve_adjoint(h, p, case.device(rhs), rtol=1e-10)
        assert st2["status"] == 0
        assert torch.count_nonzero(lam).item() == 0 and torch.count_nonzero(g).item() == 0
