"""Pins of the oracle PCG (Algorithm 1): identity preconditioner equals plain
CG, grid-independent iteration counts, null-space handling and the stop
rule."""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import problems
from oracle import discretize as D
from oracle import krylov as K
from oracle import octree as O

from oracle_fixtures import config_problem, disc_for, half_tree, hierarchy


def test_identity_preconditioner_is_plain_cg():
    """Section 2.2: Precond = I reduces PCG to CG; compared with SciPy's CG
    after the same number of steps."""
    d = disc_for(O.Octree(problems.uniform_spec(4)), seed=21)
    b = np.random.default_rng(22).uniform(-1, 1, d.tree.n)
    for k in (1, 3, 7):
        x, info = K.pcg(d.A, b, None, rtol=0.0, max_iter=k)
        ref = K.cg_textbook_reference(d.A, b, k)
        assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)


def test_grid_independent_iterations_uniform():
    its = []
    for l in (4, 5, 6):
        d = disc_for(O.Octree(problems.uniform_spec(l)))
        rhs = problems.rhs_manufactured(1, d.tree.level, d.tree.ijk)
        _, info = K.pcg(d.A, rhs, hierarchy(d).vcycle, 1e-10, 100)
        its.append(info["iters"])
    assert max(its) - min(its) <= 2, its


def test_grid_independent_iterations_adaptive():
    its = []
    for l in (3, 4, 5):
        d = disc_for(half_tree(l), seed=23)
        rhs = np.random.default_rng(24).uniform(-1, 1, d.tree.n) * 2.0 ** (-3 * d.tree.level)
        _, info = K.pcg(d.A, rhs, hierarchy(d).vcycle, 1e-10, 100)
        its.append(info["iters"])
    assert max(its) - min(its) <= 3, its


def test_null_space_all_neumann():
    """All-Neumann: the residual is shifted to zero mean (Section 2.2); the
    result agrees with a direct solve of the system with the mean fixed."""
    d = disc_for(half_tree(3), bc=(D.NEUMANN,) * 6, seed=25)
    n = d.tree.n
    rng = np.random.default_rng(26)
    b = rng.uniform(-1, 1, n)
    b -= b.mean()
    x, info = K.pcg(d.A, b, hierarchy(d).vcycle, 1e-12, 200, null_space=True)
    assert info["status"] == 0
    # bordered direct solve: [A 1; 1^T 0] [x; c] = [b; 0]
    A = d.A.toarray()
    Bm = np.zeros((n + 1, n + 1))
    Bm[:n, :n] = A
    Bm[:n, n] = 1.0
    Bm[n, :n] = 1.0
    ref = np.linalg.solve(Bm, np.concatenate([b, [0.0]]))[:n]
    assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)
    assert abs(x.mean()) < 1e-14


def test_stop_rule_and_iteration_history():
    d = disc_for(O.Octree(problems.uniform_spec(5)))
    rhs = problems.rhs_manufactured(1, d.tree.level, d.tree.ijk)
    x, info = K.pcg(d.A, rhs, hierarchy(d).vcycle, 1e-10, 100)
    h = info["hist"]
    assert h[-1] <= 1e-10 < h[-2]
    assert len(h) == info["iters"] + 1
    assert info["true"] <= 2e-10
    # per-iteration reduction is at least 10x on the uniform Poisson problem
    rates = np.array(h[1:]) / np.array(h[:-1])
    assert np.exp(np.log(rates).mean()) < 0.1


def test_zero_rhs_and_max_iter():
    d = disc_for(O.Octree(problems.uniform_spec(3)))
    x, info = K.pcg(d.A, np.zeros(d.tree.n), hierarchy(d).vcycle, 1e-10, 10)
    assert info["iters"] == 0 and np.all(x == 0)
    rhs = problems.rhs_manufactured(1, d.tree.level, d.tree.ijk)
    x, info = K.pcg(d.A, rhs, hierarchy(d).vcycle, 1e-10, 1)
    assert info["iters"] == 1 and info["status"] == 1


def test_warm_start_is_a_shifted_cold_start():
    """Algorithm 1 from x0 on b takes the same steps as the zero start on
    b - A x0 (with the stop threshold carried over): x = x0 + x'."""
    T, d, beta, rhs = config_problem(3, min_level=4, max_level=6)
    H = hierarchy(d)
    xs, _ = K.pcg(d.A, rhs, H.vcycle, 1e-12, 300, active=d.active)
    rng = np.random.default_rng(44)
    x0 = np.where(d.active, xs * (1 + 1e-3 * rng.standard_normal(T.n)), 0.0)
    xw, iw = K.pcg(d.A, rhs, H.vcycle, 1e-10, 300, active=d.active, x0=x0)
    b2 = np.where(d.active, rhs - d.A @ x0, 0.0)
    scale = np.linalg.norm(np.where(d.active, rhs, 0.0)) / np.linalg.norm(b2)
    xc, ic = K.pcg(d.A, b2, H.vcycle, 1e-10 * scale, 300, active=d.active)
    assert iw["iters"] == ic["iters"] and iw["iters"] < 10
    assert np.allclose(iw["hist"], np.array(ic["hist"]) / scale, rtol=1e-9, atol=0)
    assert np.linalg.norm(xw - (x0 + xc)) <= 1e-12 * np.linalg.norm(xw)
    # a guess that already meets the tolerance takes no iteration
    _, i0 = K.pcg(d.A, rhs, H.vcycle, 1e-10, 300, active=d.active, x0=xs)
    assert i0["iters"] == 0 and i0["status"] == 0


def test_true_residual_restart():
    """Stop rule (Algorithm 1 with the FP64 true residual): when the
    recursively updated residual meets rtol but ||b - A x|| does not, the
    iteration starts again from x with the true residual.  At rtol 1e-15 on
    a cut-cell octree the recurrence drifts below the true residual; one
    restart brings the true residual under rtol, and the reported status is
    then 0 with true <= rtol."""
    T, d, beta, rhs = config_problem(3, min_level=4, max_level=6)
    H = hierarchy(d)
    x, info = K.pcg(d.A, rhs, H.vcycle, 1e-15, 300, active=d.active)
    assert info["restarts"] >= 1
    assert info["status"] == 0 and info["true"] <= 1e-15
    b = np.where(d.active, rhs, 0.0)
    assert np.linalg.norm(np.where(d.active, rhs - d.A @ x, 0.0)) <= 1e-15 * np.linalg.norm(b)
    # the recurrence stopped below rtol before the restart: the history
    # jumps up at the restart (the true residual) and falls again
    h = np.array(info["hist"])
    assert np.any(h[1:] > h[:-1])


def test_converged_status_means_true_residual_meets_rtol():
    """Across the families (uniform Dirichlet, adaptive, cut cells with a
    Dirichlet top, all-Neumann null space, the transposed system) a status
    of 0 implies a true residual at or below rtol; a tolerance below the
    rounding floor ends as not converged, before max_iter (a restart that
    does not lower the true residual stops the solve)."""
    cases = []
    d = disc_for(O.Octree(problems.uniform_spec(4)), seed=21)
    cases.append((d.A, np.random.default_rng(22).uniform(-1, 1, d.tree.n), hierarchy(d).vcycle,
                  None, False))
    d = disc_for(half_tree(3), seed=23)
    cases.append((d.A, np.random.default_rng(24).uniform(-1, 1, d.tree.n), hierarchy(d).vcycle,
                  None, False))
    T, dc, beta, rhs = config_problem(3, min_level=4, max_level=6)
    Hc = hierarchy(dc)
    cases.append((dc.A, rhs, Hc.vcycle, dc.active, False))
    cases.append((dc.A.T.tocsr(), rhs, Hc.vcycle_T, dc.active, False))
    dn = disc_for(half_tree(3), bc=(D.NEUMANN,) * 6, seed=25)
    bn = np.random.default_rng(26).uniform(-1, 1, dn.tree.n)
    cases.append((dn.A, bn - bn.mean(), hierarchy(dn).vcycle, None, True))
    for A, b, M, act, ns in cases:
        for rtol in (1e-8, 1e-12, 1e-14):
            _, info = K.pcg(A, b, M, rtol, 300, active=act, null_space=ns)
            assert info["status"] == 0 and info["true"] <= rtol, (rtol, info["true"])
        _, info = K.pcg(A, b, M, 1e-19, 300, active=act, null_space=ns)
        assert info["status"] == 1 and info["true"] > 1e-19 and info["iters"] < 300
