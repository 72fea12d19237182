"""GPU parity: the HIP path through the C ABI against the oracle on the same
seeded inputs (small members of every workload family, element by element)."""

import numpy as np
import pytest

from gpu_fixtures import rel, small_cases

pytestmark = pytest.mark.gpu

CASES = small_cases()


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    print(f"\n[case {request.param}]", flush=True)
    return CASES[request.param]()


def test_topology_bit_exact(case):
    lev, ijk = case.tree.leaves()
    assert np.array_equal(lev, case.T.level)
    assert np.array_equal(ijk, case.T.ijk)
    owner, d, other, kind = case.tree.faces()
    assert np.array_equal(owner, case.disc.face_owner)
    assert np.array_equal(d, case.disc.face_dir)
    assert np.array_equal(other, case.disc.face_other)
    assert np.array_equal(kind, case.disc.face_kind)


def test_leaf_coefficients(case):
    from paper_2604_18886_amd import mfmg
    co = mfmg.assemble_coeffs(case.tree, case.device(case.beta), case.bc, case.theta)
    got = co.leaf_coeffs().cpu().numpy()
    want = np.stack([case.disc.c, case.disc.dirk[:, 0], case.disc.dirk[:, 2],
                     case.disc.dirk[:, 4]])
    scale = np.abs(want).max()
    assert np.abs(got - want).max() <= 1e-15 * scale


def test_level_coefficients_algorithm3(case):
    h = case.gpu_hierarchy()
    H = case.hier
    for l in range(H.L, H.lc - 1, -1):
        coords, leaf = h.level_bricks(l)
        got = h.level_coeffs(l).cpu().numpy()  # (nb, 4, 64)
        Lv = H.levels[l]
        # map oracle level cells into (brick, local morton)
        ijk = Lv.ijk
        bc = ijk // 4
        loc = ijk % 4
        m = ((loc[:, 0] & 1) | ((loc[:, 1] & 1) << 1) | ((loc[:, 2] & 1) << 2)
             | ((loc[:, 0] & 2) << 2) | ((loc[:, 1] & 2) << 3) | ((loc[:, 2] & 2) << 4))
        key = {tuple(c): i for i, c in enumerate(coords)}
        bidx = np.array([key[tuple(c)] for c in bc])
        want = np.stack([Lv.c, Lv.kx, Lv.ky, Lv.kz], axis=1)
        g = got[bidx, :, m]
        scale = np.abs(want).max()
        assert np.abs(g - want).max() <= 1e-14 * scale, l


def test_operator_and_transpose(case):
    from paper_2604_18886_amd import mfmg
    h = case.gpu_hierarchy()
    rng = np.random.default_rng(7)
    x = np.where(case.disc.active, rng.uniform(-1, 1, case.T.n), 0.0)
    y = mfmg.apply_operator(h, case.device(x)).cpu().numpy()
    want = case.disc.A @ x
    assert np.abs(y - want).max() <= 1e-13 * np.abs(want).max()
    yt = mfmg.apply_operator(h, case.device(x), transpose=True).cpu().numpy()
    wt = case.disc.A.T @ x
    assert np.abs(yt - wt).max() <= 1e-13 * np.abs(wt).max()


def test_one_cycle_fp64(case):
    from paper_2604_18886_amd import mfmg
    h = case.gpu_hierarchy()
    rng = np.random.default_rng(8)
    r = np.where(case.disc.active, rng.uniform(-1, 1, case.T.n), 0.0)
    z = mfmg.apply_precond(h, case.device(r)).cpu().numpy()
    want = case.hier.vcycle(r)
    assert rel(z, want) <= 1e-12


def test_one_cycle_mixed_against_stored_precision_oracle(case):
    """The mixed cycle (FP32 values, FP32 leaf / FP16 inner coefficients)
    against the oracle's FP64 cycle on the coefficients that store keeps
    (Hierarchy.stored_precision): what is left is FP32 arithmetic (and the
    FP32 rounding of the input), measured 6e-8 to 7e-7 relative.  The
    coefficient rounding alone moves the cycle by 6e-7 (cut sphere) to
    1.4e-5 (cut box) on the jittered families, and by nothing where beta = 1
    (dyadic coefficients are stored exactly)."""
    from paper_2604_18886_amd import mfmg
    h = case.gpu_hierarchy(precision=mfmg.MIXED)
    rng = np.random.default_rng(9)
    r = np.where(case.disc.active, rng.uniform(-1, 1, case.T.n), 0.0)
    z = mfmg.apply_precond(h, case.device(r)).cpu().numpy()
    want = case.hier.stored_precision().vcycle(r)
    err = rel(z, want)
    moved = rel(case.hier.vcycle(r), want)
    print(f"  mixed cycle vs stored-precision oracle {err:.2e} (rounding of the "
          f"coefficients alone: {moved:.2e})", flush=True)
    assert err <= 1e-5


@pytest.mark.parametrize("precision", [0, 1])
def test_solve_matches_oracle(case, precision):
    from paper_2604_18886_amd import mfmg
    h = case.gpu_hierarchy(precision=precision)
    p, st, hist = mfmg.pcg_solve(h, case.device(case.rhs), rtol=1e-10, history=True)
    p = p.cpu().numpy()
    x, info = case.oracle_solve(1e-13)
    print(f"  precision={precision} gpu iters={st['iters']} oracle(1e-13) iters={info['iters']}"
          f" true={st['rel_resid_true']:.2e} err={rel(p, x):.2e}", flush=True)
    assert st["status"] == 0
    assert st["rel_resid_true"] <= 1e-10  # the true residual meets rtol
    assert rel(p, x) <= 1e-9
    # iteration count of the FP64 path equals the oracle's at the same rtol
    if precision == 0:
        _, info10 = case.oracle_solve(1e-10)
        assert abs(st["iters"] - info10["iters"]) <= 1
        assert np.allclose(hist[: len(info10["hist"])], info10["hist"][: len(hist)],
                           rtol=1e-6, atol=1e-14)
    # inactive leaves are zero on output
    assert np.all(p[~case.disc.active] == 0.0)


def test_null_space_all_neumann():
    """All walls Neumann and no solid: the residual is shifted to zero mean
    (Section 2.2); the zero-mean solution matches the oracle's."""
    import problems
    from gpu_fixtures import Case
    from oracle import krylov as K
    from paper_2604_18886_amd import mfmg
    spec = problems.config_spec(2, 3, 5)
    rng = np.random.default_rng(12)
    case = Case(2, spec, bc=(0,) * 6, theta=0.5)
    act = case.disc.active
    rhs = np.where(act, rng.uniform(-1, 1, case.T.n), 0.0)
    rhs[act] -= rhs[act].mean()
    h = case.gpu_hierarchy()
    p, st = mfmg.pcg_solve(h, case.device(rhs), rtol=1e-10)
    p = p.cpu().numpy()
    x, info = K.pcg(case.disc.A, rhs, case.hier.vcycle, 1e-13, 400, null_space=True,
                    active=act)
    print(f"  null space: gpu iters={st['iters']} oracle iters={info['iters']} "
          f"err={rel(p, x):.2e}", flush=True)
    assert st["status"] == 0
    assert abs(p[act].mean()) <= 1e-12 * np.abs(p).max()
    assert rel(p, x) <= 1e-9


def test_mixed_w_cycle_against_stored_precision_oracle():
    """The mixed-precision W-cycle (mu = 2) against the oracle's W-cycle on
    the coefficients the mixed store keeps, and its solve against the FP64
    oracle's solution."""
    import problems
    from gpu_fixtures import Case
    from oracle import krylov as K
    from oracle import multigrid as M
    from paper_2604_18886_amd import mfmg
    case = Case(3, problems.config_spec(3, 5, 7))
    H = M.Hierarchy(case.disc, coarsest=3, mu=2)
    h = case.gpu_hierarchy(mu=2, precision=mfmg.MIXED)
    rng = np.random.default_rng(11)
    r = np.where(case.disc.active, rng.uniform(-1, 1, case.T.n), 0.0)
    z = mfmg.apply_precond(h, case.device(r)).cpu().numpy()
    err = rel(z, H.stored_precision().vcycle(r))
    p, st = mfmg.pcg_solve(h, case.device(case.rhs), rtol=1e-10)
    x, _ = K.pcg(case.disc.A, case.rhs, H.vcycle, 1e-13, 400, active=case.disc.active)
    print(f"  mixed W-cycle vs stored-precision oracle {err:.2e}; solve iters {st['iters']} "
          f"err {rel(p.cpu().numpy(), x):.2e}", flush=True)
    assert err <= 1e-5
    assert st["status"] == 0 and rel(p.cpu().numpy(), x) <= 1e-9


@pytest.mark.parametrize("mu", [2])
def test_w_cycle_matches_oracle(mu):
    """The mu-cycle (Algorithm 4 with mu recursive coarse solves; mu = 2 is
    the W-cycle the paper uses on cut-cell grids): one cycle and a full
    solve against the oracle's."""
    import problems
    from gpu_fixtures import Case
    from oracle import krylov as K
    from oracle import multigrid as M
    from paper_2604_18886_amd import mfmg
    case = Case(3, problems.config_spec(3, 5, 7))
    H = M.Hierarchy(case.disc, coarsest=3, mu=mu)
    h = case.gpu_hierarchy(mu=mu)
    rng = np.random.default_rng(10)
    r = np.where(case.disc.active, rng.uniform(-1, 1, case.T.n), 0.0)
    z = mfmg.apply_precond(h, case.device(r)).cpu().numpy()
    assert rel(z, H.vcycle(r)) <= 1e-12
    p, st = mfmg.pcg_solve(h, case.device(case.rhs), rtol=1e-10)
    x, info = K.pcg(case.disc.A, case.rhs, H.vcycle, 1e-13, 400, active=case.disc.active)
    _, info10 = K.pcg(case.disc.A, case.rhs, H.vcycle, 1e-10, 400, active=case.disc.active)
    print(f"  mu={mu}: gpu iters={st['iters']} oracle(1e-10)={info10['iters']} "
          f"err={rel(p.cpu().numpy(), x):.2e}", flush=True)
    assert st["status"] == 0
    assert abs(st["iters"] - info10["iters"]) <= 1
    assert rel(p.cpu().numpy(), x) <= 1e-9


@pytest.mark.parametrize("precision", [0, 1])
def test_warm_start_matches_oracle(precision):
    """Algorithm 1 from an initial guess (the previous solution perturbed):
    same stop test relative to ||rhs||, same iterations as the oracle's
    warm start, and a guess that already meets the tolerance takes none."""
    import problems
    from gpu_fixtures import Case
    from oracle import krylov as K
    from paper_2604_18886_amd import mfmg
    case = Case(3, problems.config_spec(3, 5, 7))
    act = case.disc.active
    xs, _ = case.oracle_solve(1e-13)
    rng = np.random.default_rng(45)
    x0 = np.where(act, xs * (1 + 1e-3 * rng.standard_normal(case.T.n)), 0.0)
    h = case.gpu_hierarchy(precision=precision)
    p, st, hist = mfmg.pcg_solve(h, case.device(case.rhs), rtol=1e-10, history=True,
                                 x0=case.device(x0))
    xw, iw = K.pcg(case.disc.A, case.rhs, case.hier.vcycle, 1e-10, 400, active=act, x0=x0)
    p = p.cpu().numpy()
    print(f"  precision={precision} warm: gpu iters={st['iters']} oracle={iw['iters']} "
          f"true={st['rel_resid_true']:.2e} err={rel(p, xs):.2e}", flush=True)
    assert st["status"] == 0 and st["rel_resid_true"] <= 1e-10
    assert rel(p, xs) <= 1e-9
    if precision == 0:
        assert abs(st["iters"] - iw["iters"]) <= 1
        assert np.allclose(hist[: len(iw["hist"])], iw["hist"][: len(hist)], rtol=1e-6,
                           atol=1e-14)
    _, st0 = mfmg.pcg_solve(h, case.device(case.rhs), rtol=1e-10, x0=case.device(xs))
    assert st0["iters"] == 0 and st0["status"] == 0
