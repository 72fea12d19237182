"""GPU parity at the full sizes of the workloads, in the configuration the
benchmark times (default hierarchy, rtol 1e-10, FP64 and mixed cycle):

* leaf levels 5..7 sphere band (803K leaves) and 6..9 cut-cell sphere
  (2.3M leaves): topology bit-exact, solutions against the oracle's solve
  at 1e-13, and the oracle's own residual of the GPU solution;
* the adjoint on the 6..9 cut-cell octree: lambda and dL/dbeta against the
  oracle's adjoint solve and per-face gradient;
* leaf levels 7..10 (26.3M leaves): topology bit-exact against the oracle
  octree and faces, the relative residual of both GPU solutions measured
  with the oracle's assembled operator, and both solutions against the
  oracle's p* (1e-13) at 32768 seeded leaves and in the 2-norm (the sample
  is stored, the full oracle solve takes minutes); the same octree built
  on the device, bit-exact against the oracle too.
"""

import numpy as np
import pytest

import problems
from gpu_fixtures import Case, rel
from oracle import krylov as K

pytestmark = pytest.mark.gpu


_CASES = {}


def _case(cfg):
    """One Case per workload per session (the oracle side is the slow part)."""
    if cfg not in _CASES:
        _CASES.clear()
        _CASES[cfg] = Case(cfg, problems.config_spec(cfg))
    return _CASES[cfg]


@pytest.fixture(scope="module", params=[2, 3])
def full(request):
    print(f"\n[full-size workload {request.param}]", flush=True)
    return _case(request.param)


def _topology_equal(case):
    lev, ijk = case.tree.leaves()
    assert np.array_equal(lev, case.T.level)
    assert np.array_equal(ijk, case.T.ijk)
    owner, d, other, kind = case.tree.faces()
    assert np.array_equal(owner, case.disc.face_owner)
    assert np.array_equal(d, case.disc.face_dir)
    assert np.array_equal(other, case.disc.face_other)
    assert np.array_equal(kind, case.disc.face_kind)


def _oracle_resid(case, p):
    act = case.disc.active
    r = np.where(act, case.rhs - case.disc.A @ p, 0.0)
    b = np.where(act, case.rhs, 0.0)
    return np.linalg.norm(r) / np.linalg.norm(b)


def test_full_topology_bit_exact(full):
    _topology_equal(full)


@pytest.mark.parametrize("precision", [0, 1])
def test_full_solve_matches_oracle(full, precision):
    from paper_2604_18886_amd import mfmg
    h = full.gpu_hierarchy(precision=precision)
    p_d, st = mfmg.pcg_solve(h, full.device(full.rhs), rtol=1e-10)
    p = p_d.cpu().numpy()
    if not hasattr(full, "x13"):
        full.x13, full.info13 = full.oracle_solve(1e-13)
    err = rel(p, full.x13)
    res = _oracle_resid(full, p)
    print(f"  precision={precision} iters={st['iters']} (oracle 1e-13: {full.info13['iters']}) "
          f"gpu true={st['rel_resid_true']:.2e} oracle-measured={res:.2e} err={err:.2e}",
          flush=True)
    assert st["status"] == 0
    assert st["rel_resid_true"] <= 1e-10
    # the same residual summed in another order: ~1e-16 |A p| / |r| apart
    assert res <= 1e-10 * (1 + 1e-4)
    assert err <= 1e-9
    assert np.all(p[~full.disc.active] == 0.0)


@pytest.mark.parametrize("precision", [0, 1])
def test_full_adjoint_matches_oracle(precision):
    """The adjoint workload: octree of the 6..9 cut-cell sphere, L = ||p -
    p_t||^2, lambda and dL/dbeta for every face."""
    from paper_2604_18886_amd import mfmg
    case = _case(3)
    h = case.gpu_hierarchy(precision=precision)
    p_d, _ = mfmg.pcg_solve(h, case.device(case.rhs), rtol=1e-11)
    p = p_d.cpu().numpy()
    pt = problems.adjoint_target(case.T.level, case.T.ijk, np.abs(p).max())
    g = np.where(case.disc.active, 2.0 * (p - pt), 0.0)
    # rtol 1e-11: at 2.3M cells the FP64 evaluation of ||g - A^T lambda||
    # itself rounds to about 1e-12 of ||g|| (about eps |A| |lambda|), so a
    # tolerance of 1e-12 is below what any iterate can show
    lam_d, grad_d, st = mfmg.pcg_solve_adjoint(h, p_d, case.device(g), rtol=1e-11)
    if not hasattr(case, "lam13"):
        case.lam13, _ = K.pcg(case.disc.A.T.tocsr(), g, case.hier.vcycle_T, 1e-13, 400,
                              active=case.disc.active)
    grad_o = case.disc.face_gradient(case.lam13, p)
    lam = lam_d.cpu().numpy()
    grad = grad_d.cpu().numpy()
    print(f"  precision={precision} adjoint iters={st['iters']} true={st['rel_resid_true']:.2e} "
          f"lam err={rel(lam, case.lam13):.2e} "
          f"grad err={np.abs(grad - grad_o).max() / np.abs(grad_o).max():.2e}", flush=True)
    # a converged solve meets rtol in its true residual (the iteration
    # restarts from the true residual while it does not)
    assert st["status"] == 0 and st["rel_resid_true"] <= 1e-11
    assert rel(lam, case.lam13) <= 1e-9
    assert np.abs(grad - grad_o).max() <= 1e-9 * np.abs(grad_o).max()


def _large_sample():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "large_workload_solution_sample.npz")
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def test_largest_workload_topology_and_residual():
    """26.3M leaves: leaves and faces bit-exact against the oracle; both
    GPU solutions have oracle-measured relative residual <= 1e-10, agree
    with each other, and with the oracle's solution p* at 1e-13 to 1e-9
    relative L2 over 32768 seeded active leaves (p* sampled by the
    committed tests/golden/make_large_workload_sample.py; the full oracle
    solve takes minutes) and in the full 2-norm."""
    from paper_2604_18886_amd import mfmg
    case = _case(4)
    ref = _large_sample()
    assert int(ref["n_leaves"]) == case.T.n
    assert np.all(case.disc.active[ref["idx"]])
    print(f"  {case.T.n} leaves, {case.disc.n_faces} faces", flush=True)
    _topology_equal(case)
    sols = []
    for precision in (0, 1):
        h = case.gpu_hierarchy(precision=precision)
        p_d, st = mfmg.pcg_solve(h, case.device(case.rhs), rtol=1e-10)
        p = p_d.cpu().numpy()
        res = _oracle_resid(case, p)
        err = rel(p[ref["idx"]], ref["val"])
        nerr = abs(np.linalg.norm(p) - float(ref["norm"])) / float(ref["norm"])
        print(f"  precision={precision} iters={st['iters']} gpu true={st['rel_resid_true']:.2e} "
              f"oracle-measured={res:.2e} err vs p* (sampled)={err:.2e} norm diff={nerr:.2e}",
              flush=True)
        assert err <= 1e-9 and nerr <= 1e-9
        assert st["status"] == 0 and st["rel_resid_true"] <= 1e-10
        assert res <= 1e-10 * (1 + 1e-4)
        sols.append(p)
        del h
    assert rel(sols[1], sols[0]) <= 1e-8


def test_largest_workload_built_on_the_device():
    """26.3M leaves, octree built on the device: leaves and faces bit-exact
    against the oracle octree."""
    from paper_2604_18886_amd import mfmg
    case = _case(4)
    td = mfmg.build_octree(case.spec, device=True)
    lev, ijk = td.leaves()
    assert np.array_equal(lev, case.T.level)
    assert np.array_equal(ijk, case.T.ijk)
    del lev, ijk
    owner, d, other, kind = td.faces()
    assert np.array_equal(owner, case.disc.face_owner)
    assert np.array_equal(d, case.disc.face_dir)
    assert np.array_equal(other, case.disc.face_other)
    assert np.array_equal(kind, case.disc.face_kind)


def test_offset_limit_and_largest_mixed_solve():
    """Maximum sizes of the 32-bit buffer offsets.  Uniform 512^3 (2^21 leaf
    bricks): the FP64 leaf coefficients the outer operator reads take
    exactly 4 GiB, one byte too many, and both precisions are rejected
    before any allocation.  A sphere band on levels 8..10 with 2.04M leaf
    bricks (131M leaves, octree built on the device, beta = 1): FP64 is
    rejected (its level coefficients of all bricks exceed 4 GiB), the mixed
    hierarchy fits and solves a seeded right-hand side to rtol 1e-10 (true
    residual recomputed in FP64 on the device)."""
    import torch
    from paper_2604_18886_amd import mfmg
    bc = (0, 0, 0, 1, 0, 0)
    tree = mfmg.build_octree(problems.uniform_spec(9), device=True)
    assert tree.n_leaf_bricks == 2 ** 21
    beta = torch.ones(tree.n_faces, dtype=torch.float64, device="cuda")
    co = mfmg.assemble_coeffs(tree, beta, bc, 0.5)
    for precision in (mfmg.FP64, mfmg.MIXED):
        with pytest.raises(mfmg.MFMGError) as e:
            mfmg.build_hierarchy(co, precision=precision)
        assert e.value.status == -1 and "32-bit" in str(e.value)
    del co, beta, tree
    spec = {"min_level": 8, "max_level": 10, "node_size": 4,
            "prims": [problems.sphere_prim((0.5, 0.5, 0.5), 0.3, 0.04)]}
    tree = mfmg.build_octree(spec, device=True)
    print(f"  {tree.n_leaves} leaves in {tree.n_leaf_bricks} leaf bricks, {tree.n_faces} faces",
          flush=True)
    assert 0.95 * 2 ** 21 < tree.n_leaf_bricks < 2 ** 21
    beta = torch.ones(tree.n_faces, dtype=torch.float64, device="cuda")
    co = mfmg.assemble_coeffs(tree, beta, bc, 0.5)
    del beta
    with pytest.raises(mfmg.MFMGError) as e:
        mfmg.build_hierarchy(co, precision=mfmg.FP64)
    assert e.value.status == -1
    h = mfmg.build_hierarchy(co, precision=mfmg.MIXED)
    g = torch.Generator(device="cuda").manual_seed(90)
    rhs = torch.rand(tree.n_leaves, dtype=torch.float64, device="cuda", generator=g) - 0.5
    p, st = mfmg.pcg_solve(h, rhs, rtol=1e-10)
    print(f"  mixed: {st['iters']} iterations, true residual {st['rel_resid_true']:.2e}, "
          f"{st['seconds'] * 1e3:.1f} ms", flush=True)
    assert st["status"] == 0 and st["rel_resid_true"] <= 1e-10


@pytest.mark.parametrize("precision", [0, 1])
def test_full_adjoint_gradient_against_finite_differences(precision):
    """The adjoint workload's full octree (levels 6..9, 2.3M leaves): the
    GPU's dL/dbeta on 50 seeded faces (25 T-junction or cut faces, 25 from
    all faces with both sides active) against central finite differences
    of the GPU's own forward solves, eps = 1e-6 relative to the face's
    cells' coupling, each side a difference solve (the oracle's
    finite-difference rule, reading 17):
        A(beta +- eps e_f) dp = -+ eps (dA/dbeta_f) p,
    with the perturbed coefficients assembled and coarsened on the device
    and (dA/dbeta_f) p formed from a unit step (A is linear in beta).  The
    base residual r0 = rhs - A p (1e-11 of rhs) is left out of the
    right-hand side: the difference is then taken at A^-1 (A p), which
    differs from A^-1 rhs by the solve's residual, and each dp is a solve
    to its own tolerance.  The
    gradient itself is compared with the oracle's at this size by
    test_full_adjoint_matches_oracle, and the oracle's gradient with its own
    finite differences on smaller members of the family."""
    import torch
    from oracle import discretize as D
    from paper_2604_18886_amd import mfmg
    case = _case(3)
    d = case.disc
    dev = case.device
    act = d.active
    both = act[d.face_owner] & ((d.face_other < 0) | act[np.maximum(d.face_other, 0)])
    special = np.nonzero(((d.face_kind == D.COARSE) | (case.beta < 1)) & both)[0]
    faces = problems.sample_faces(d.n_faces, special, count=50, pool=np.nonzero(both)[0])
    assert len(faces) == 50 and np.all(both[faces])

    def hierarchy(beta):
        co = mfmg.assemble_coeffs(case.tree, dev(beta), case.bc, case.theta)
        return mfmg.build_hierarchy(co, coarsest_level=3, precision=precision)

    h0 = hierarchy(case.beta)
    rhs_d = dev(case.rhs)
    p_d, _ = mfmg.pcg_solve(h0, rhs_d, rtol=1e-11)
    p = p_d.cpu().numpy()
    pt = problems.adjoint_target(case.T.level, case.T.ijk, np.abs(p).max())
    e = np.where(act, p - pt, 0.0)
    # the adjoint to 2e-12, just above its true-residual floor at this size:
    # a face's gradient is a difference of lambda across it
    _, grad_d, st = mfmg.pcg_solve_adjoint(h0, p_d, dev(2.0 * e), rtol=2e-12)
    assert st["status"] == 0
    grad = grad_d.cpu().numpy()
    act_d = torch.as_tensor(act, device="cuda")
    Ap0 = mfmg.apply_operator(h0, p_d)
    scale = d.face_scale()
    fd = np.zeros(len(faces))
    steps = np.zeros(len(faces))
    e_d = dev(e)
    for n, f in enumerate(faces):
        # step relative to the coupling of the face's cells (reading 17)
        cells = [d.face_owner[f]] + ([d.face_other[f]] if d.face_other[f] >= 0 else [])
        dc = [scale[f]] + ([scale[f] / 2.0 if d.face_kind[f] == D.COARSE else scale[f]]
                           if d.face_other[f] >= 0 else [])
        step = 1e-6 * min([1.0] + [d.c[i] / x for i, x in zip(cells, dc) if x > 0])
        steps[n] = step
        bu = case.beta.copy()
        bu[f] += 1.0
        hu = hierarchy(bu)
        dAp = mfmg.apply_operator(hu, p_d) - Ap0
        del hu
        dls = []
        for sgn in (1.0, -1.0):
            bb = case.beta.copy()
            bb[f] += sgn * step
            hs = hierarchy(bb)
            b = torch.where(act_d, -sgn * step * dAp, 0.0)
            dp, sst = mfmg.pcg_solve(hs, b, rtol=1e-12)
            assert sst["status"] in (0, 1) and sst["rel_resid_true"] <= 1e-11
            del hs
            dls.append(float(2.0 * torch.dot(e_d, dp) + torch.dot(dp, dp)))
        fd[n] = (dls[0] - dls[1]) / (2.0 * step)
    ga = grad[faces]
    gmax = np.abs(fd).max()
    rerr = np.abs(ga - fd) / np.maximum(np.abs(fd), 1e-8 * gmax)
    w = int(np.argmax(rerr))
    big = np.abs(fd) >= 1e-6 * gmax
    print(f"  precision={precision}: FD check on {len(faces)} faces of the full octree: "
          f"rule max |g - g_FD| / max(|g_FD|, 1e-8 max|g_FD|) = {rerr.max():.2e} (face kind "
          f"{d.face_kind[faces[w]]}, beta {case.beta[faces[w]]:.3g}, |g| / max|g| "
          f"{abs(fd[w]) / gmax:.2e}); on the {int(big.sum())} faces with |g| >= 1e-6 max|g|: "
          f"{rerr[big].max():.2e}; max |g - g_FD| / max|g| {np.abs(ga - fd).max() / gmax:.2e}; "
          f"adjoint true residual {st['rel_resid_true']:.2e}; {int((steps < 1e-6).sum())} "
          f"faces with a reduced step", flush=True)
    # At 2.3M cells the FP64 floor of the adjoint (true residual ~1.5e-12)
    # leaves a face gradient an absolute error of a few 1e-10 of the largest
    # (measured 3.4e-10): the relative 1e-6 is asked of the faces whose
    # gradient is at least 1e-6 of the largest (49 of the 50 here, measured
    # 1.8e-7), every face is held to 1e-9 of the largest.  (The one face
    # below, |g| = 1.2e-7 max|g|, agrees to 3e-6 relative.)
    assert rerr[big].max() <= 1e-6
    assert np.abs(ga - fd).max() <= 1e-9 * gmax
