"""Pins of the oracle multigrid: Algorithm 3 against explicit Galerkin R A P,
the paper's worked coarse values, FAS flux conservation (Eq. 11), the
equivalence of beta at restriction and at prolongation (Section 3.3), and the
symmetry of the preconditioner (Section 2.3)."""

import numpy as np
import pytest
import scipy.sparse as sp

import problems
from oracle import discretize as D
from oracle import octree as O

from oracle_fixtures import disc_for, half_tree, hierarchy, read_golden


def _rap_level(H, l):
    """Explicit R A^l P for level l -> l-1 with R = P^T / alpha over all
    children (Galerkin, Eq. 12)."""
    F = H.levels[l]
    C = H.levels[l - 1]
    rows, cols = [], []
    for q in range(8):
        inner = np.nonzero(~C.leaf)[0]
        rows.append(C.ch[inner, q])
        cols.append(inner)
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    P = sp.coo_matrix((np.ones(len(r)), (r, c)), shape=(F.n, C.n)).tocsr()
    return (P.T @ F.A @ P) / H.alpha


def _coef_matrix(H, l):
    """Level-(l-1) matrix from the stored Algorithm 3 coefficients (7-point,
    no T-faces)."""
    C = H.levels[l - 1]
    act = C.active
    rows, cols, vals = [np.arange(C.n)], [np.arange(C.n)], [np.where(act, C.c, 0.0)]
    for d in range(6):
        k = H.face_coef(l - 1, d)
        m = act & (C.nkind[:, d] == 1)
        rows.append(np.nonzero(m)[0])
        cols.append(C.nidx[m, d])
        vals.append(-k[m])
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(C.n, C.n)).tocsr()


@pytest.mark.parametrize("kind", ["fluid", "jitter", "cut"])
def test_algorithm3_equals_galerkin_on_uniform_grids(kind):
    if kind == "fluid":
        d = disc_for(O.Octree(problems.uniform_spec(4)))
    elif kind == "jitter":
        d = disc_for(O.Octree(problems.uniform_spec(4)), bc=(0, 1, 0, 1, 1, 0), seed=12)
    else:
        T = O.Octree(problems.uniform_spec(5))
        d = D.Discretization(T, None, problems.config_bc(3)[0], 0.5)
        d.set_beta(problems.face_beta(3, d.face_level, d.face_ijk, d.face_dir))
        assert (~d.active).any()
    H = hierarchy(d)
    for l in range(H.L, H.lc, -1):
        G = _rap_level(H, l)
        Cm = _coef_matrix(H, l)
        act = H.levels[l - 1].active
        diff = (G - Cm)[act][:, act]
        scale = abs(G).max()
        assert abs(diff).max() <= 1e-14 * scale
        # rows of inactive coarse cells are empty in both
        assert abs(G[~act]).max() == 0.0 if (~act).any() else True


def test_galerkin_pure_fluid_values_from_paper():
    g = read_golden("coefficients_closed_form.txt")
    d = disc_for(O.Octree(problems.uniform_spec(5)))
    H = hierarchy(d, alpha=g["alpha"])
    C = H.levels[4]
    h = 2.0 ** -5
    # interior coarse cells (no wall face)
    interior = np.all((C.ijk > 0) & (C.ijk < 15), axis=1)
    assert np.allclose(C.c[interior], g["galerkin_diag_over_h_at_alpha2"] * h, rtol=1e-15)
    assert np.allclose(-C.kx[interior], g["galerkin_offdiag_over_h_at_alpha2"] * h, rtol=1e-15)
    # alpha = 4 (the graphics convention): -4h/alpha and 24h/alpha
    H4 = hierarchy(d, alpha=4.0)
    C4 = H4.levels[4]
    assert np.allclose(C4.c[interior], g["galerkin_diag_over_h_times_alpha"] * h / 4.0)
    assert np.allclose(-C4.kx[interior], g["galerkin_offdiag_over_h_times_alpha"] * h / 4.0)
    assert np.allclose(H.levels[5].R.data, g["restriction_entry"])


def test_algorithm3_galerkin_away_from_tjunctions_on_adaptive_grid():
    d = disc_for(half_tree(4), seed=13)
    H = hierarchy(d)
    l = H.L
    G = _rap_level(H, l)
    Cm = _coef_matrix(H, l)
    C = H.levels[l - 1]
    F = H.levels[l]
    # parents whose children and their neighbours see no T-face
    tchild = np.zeros(F.n, dtype=bool)
    tchild[np.nonzero((F.nkind == 2).any(axis=1))[0]] = True
    bad = np.zeros(C.n, dtype=bool)
    inner = np.nonzero(~C.leaf)[0]
    for q in range(8):
        bad[inner] |= tchild[C.ch[inner, q]]
    ok = ~C.leaf & C.active & ~bad
    # also exclude parents next to such cells (their off-diagonals involve them)
    for dd in range(6):
        nb = C.nidx[:, dd]
        m = C.nkind[:, dd] == 1
        ok[m] &= ~bad[nb[m]] & ~C.leaf[nb[m]]
    assert ok.sum() > 10
    diff = (G - Cm)[ok][:, ok]
    assert abs(diff).max() <= 1e-14 * abs(G).max()


def test_fas_prolongation_restores_coarse_means():
    """Eq. (11): after the prolongation of Algorithm 4, the mean of the active
    children equals the coarse value, on every inner cell, also at
    T-junctions.  The paper's 2-D numbers are checked with the level
    transfer operators."""
    g = read_golden("fas_2d_example.txt")
    d = disc_for(half_tree(4), seed=14)
    H = hierarchy(d)
    trace = []
    rng = np.random.default_rng(15)
    H.vcycle(rng.uniform(-1, 1, d.tree.n), trace=trace)
    assert len(trace) == H.L - H.lc
    for (l, ul, uc) in trace:
        F = H.levels[l]
        C = H.levels[l - 1]
        m = ~C.leaf & C.active
        assert np.allclose((F.Avg @ ul)[m], uc[m], rtol=1e-13, atol=1e-15)
    # the printed 2-D example: u_i + (p5 - u5) has mean p5
    u = np.array([g["u0"], g["u1"], g["u2"], g["u3"]])
    assert np.isclose(u.mean(), g["u5"])
    assert np.isclose((u + (g["p5"] - u.mean())).mean(), g["mean_p"])


@pytest.mark.parametrize("seed", [16, 17])
def test_beta_at_restriction_equals_beta_at_prolongation(seed):
    """Section 3.3: on grids without T-junctions Algorithm 4 (beta in the
    restriction) gives the same preconditioner as Algorithm 2 (beta in the
    prolongation)."""
    d = disc_for(O.Octree(problems.uniform_spec(5)), seed=seed)
    H = hierarchy(d)
    r = np.random.default_rng(seed).uniform(-1, 1, d.tree.n)
    z4 = H.vcycle(r)
    z2 = H.standard_cycle(r, beta=2.0)
    assert np.linalg.norm(z4 - z2) <= 1e-13 * np.linalg.norm(z2)
    Hw = hierarchy(d, mu=2)
    assert np.linalg.norm(Hw.vcycle(r) - Hw.standard_cycle(r, beta=2.0)) <= \
        1e-13 * np.linalg.norm(z2)


def test_preconditioner_symmetric_on_uniform_grid():
    """Opposite colour orders make M symmetric (Section 2.3)."""
    d = disc_for(O.Octree(problems.uniform_spec(4)), seed=18)
    H = hierarchy(d)
    rng = np.random.default_rng(19)
    for _ in range(3):
        x = rng.uniform(-1, 1, d.tree.n)
        y = rng.uniform(-1, 1, d.tree.n)
        a = x @ H.vcycle(y)
        b = y @ H.vcycle(x)
        assert abs(a - b) <= 1e-12 * abs(a)


def test_preconditioned_spectrum_real_positive_tiny():
    d = disc_for(O.Octree(problems.uniform_spec(3)), seed=20)
    H = hierarchy(d, coarsest=2)
    n = d.tree.n
    Mm = np.stack([H.vcycle(e) for e in np.eye(n)], axis=1)
    ev = np.linalg.eigvals(Mm @ d.A.toarray())
    assert np.abs(ev.imag).max() < 1e-8 * np.abs(ev).max()
    assert ev.real.min() > 0


@pytest.mark.parametrize("maker", ["half", "cut"])
def test_cycle_transpose_is_exact_adjoint(maker):
    """x . M y == y . M^T x for the cycle and its transpose (T-junctions and
    cut cells included), and the dense transpose on a tiny grid."""
    if maker == "half":
        d = disc_for(half_tree(3), seed=40)
    else:
        import problems as P
        T = O.Octree(P.config_spec(3, min_level=3, max_level=5))
        d = D.Discretization(T, None, P.config_bc(3)[0], 0.5)
        d.set_beta(P.face_beta(3, d.face_level, d.face_ijk, d.face_dir))
    H = hierarchy(d)
    rng = np.random.default_rng(41)
    act = d.active
    for _ in range(3):
        x = np.where(act, rng.uniform(-1, 1, d.tree.n), 0.0)
        y = np.where(act, rng.uniform(-1, 1, d.tree.n), 0.0)
        a = x @ H.vcycle(y)
        b = y @ H.vcycle_T(x)
        assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))
    if maker == "half":
        n = d.tree.n
        Mm = np.stack([H.vcycle(e) for e in np.eye(n)[:200]], axis=1)
        Mt = np.stack([H.vcycle_T(e) for e in np.eye(n)], axis=1)
        assert np.allclose(Mt[:200, :].T, Mm, rtol=0, atol=1e-13 * np.abs(Mm).max())


def _level_values(H, u):
    """Level vectors of a leaf vector: leaves hold their own value, inner
    cells the mean of their active children (recursively), i.e. the value
    the composite operator uses for an inner neighbour (Section 3.1)."""
    vals = {}
    for l in range(H.L, H.lc - 1, -1):
        Lv = H.levels[l]
        v = np.zeros(Lv.n)
        v[Lv.leaf] = u[Lv.leaf_idx[Lv.leaf]]
        if l < H.L:
            v[~Lv.leaf] = (H.levels[l + 1].Avg @ vals[l + 1])[~Lv.leaf]
        vals[l] = v
    return vals


@pytest.mark.parametrize("maker", ["three", "cut", "half_y"])
def test_level_tjunction_rows_equal_composite_rows(maker):
    """Pin of the level operators' leaf rows, T-junction coupling B^l
    included (Section 3.1, Eqs. (7)-(10); Algorithm 3 coarse coefficients):
    with inner cells holding the mean of their active children, the row
    (A^l u_l + B^l u_{l-1})_i of every active leaf i of every level is the
    composite operator's row (A u)_i, which is assembled independently and
    pinned by conservation, the direct solves and second-order convergence.
    A wrong ghost weight (the 1/2 on u_J, the 1/(2 n) on the siblings) or a
    coarse coefficient other than the sum of the sub-faces over 2 fails it."""
    from oracle_fixtures import config_problem, three_level_nodes
    if maker == "three":
        T = O.Octree({"min_level": 3, "max_level": 5, "node_size": 4, "prims": []},
                     three_level_nodes(3))
        d = disc_for(T, seed=41)
    elif maker == "half_y":
        d = disc_for(half_tree(3, axis=1), seed=42)
    else:
        _, d, _, _ = config_problem(3, min_level=4, max_level=6)
    H = hierarchy(d)
    rng = np.random.default_rng(43)
    u = np.where(d.active, rng.uniform(-1.0, 1.0, d.tree.n), 0.0)
    Au = d.A @ u
    vals = _level_values(H, u)
    n_t = 0
    for l in range(H.L, H.lc - 1, -1):
        Lv = H.levels[l]
        y = Lv.A @ vals[l]
        if Lv.B is not None:
            y = y + Lv.B @ vals[l - 1]
        rows = np.nonzero(Lv.leaf & Lv.active)[0]
        ref = Au[Lv.leaf_idx[rows]]
        assert np.allclose(y[rows], ref, rtol=0.0, atol=1e-13 * max(np.abs(Au).max(), 1e-300))
        n_t += int((Lv.nkind[rows] == 2).any(axis=1).sum())
    assert n_t > 0
    # the check is sensitive: a ghost weight of 1/4 instead of 1/2 on u_J
    # changes the T rows
    L = H.L
    Lv = H.levels[L]
    if Lv.B is not None and Lv.B.nnz:
        y_bad = Lv.A @ vals[L] + 0.5 * (Lv.B @ vals[L - 1])
        rows = np.nonzero(Lv.leaf & Lv.active)[0]
        assert not np.allclose(y_bad[rows], Au[Lv.leaf_idx[rows]], rtol=0.0,
                               atol=1e-13 * np.abs(Au).max())
