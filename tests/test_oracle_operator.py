"""Pins of the oracle discretisation: closed-form coefficients, the T-junction
ghost rule on the paper's worked example, conservation, symmetry structure,
definiteness, direct solves and second-order accuracy."""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import problems
from oracle import discretize as D
from oracle import krylov as K
from oracle import octree as O

from oracle_fixtures import (config_problem, disc_for, half_tree, hierarchy,
                             read_golden, three_level_nodes)


def uniform_tree(l):
    return O.Octree(problems.uniform_spec(l))


def test_fluid_cell_coefficients_closed_form():
    g = read_golden("coefficients_closed_form.txt")
    T = uniform_tree(4)
    h = 2.0 ** -4
    # theta = 1 is the paper's Dirichlet-cell rule: the wall face keeps -h
    d = disc_for(T, theta=1.0)
    assert np.allclose(d.dirk, -g["fluid_offdiag_over_h"] * h, rtol=0, atol=1e-18)
    assert np.allclose(d.c, g["fluid_diag_over_h"] * h, rtol=0, atol=1e-18)
    # theta = 1/2: the wall at the face doubles the wall coefficient
    d = disc_for(T, theta=0.5)
    nwall = (d.kind == D.WALL).sum(axis=1)
    assert np.allclose(d.c, (6 + nwall) * h, rtol=0, atol=1e-18)


def test_neumann_and_inactive_cells():
    T = uniform_tree(3)
    d = disc_for(T, bc=(D.NEUMANN,) * 6)
    nwall = (d.kind == D.WALL).sum(axis=1)
    h = 2.0 ** -3
    assert np.allclose(d.c, (6 - nwall) * h)
    # a cell with all faces of zero fluid area is not a degree of freedom
    beta = np.ones(d.n_faces)
    i = 200
    for dd in range(6):
        f = d.face_id[i, dd]
        if f >= 0:
            beta[f] = 0.0
        else:
            j = d.nidx[i, dd]
            beta[d.face_id[j, dd ^ 1]] = 0.0
    d.set_beta(beta)
    assert d.c[i] == 0.0 and not d.active[i]
    assert d.A[i].nnz == 0 or np.all(d.A[i].data == 0)
    assert np.all(d.A[:, i].data == 0)


def test_tjunction_ghost_on_paper_example():
    """Figure 4 values extruded along z: (A u)_i of the fine cell next to the
    coarse leaf equals the plain flux sum with the ghost value printed by the
    worked example, and the coarse leaf's face flux equals f1 + f3 scaled."""
    g = read_golden("tjunction_2d_example.txt")
    T = half_tree(3)  # x < 1/2 at level 4, rest at level 3
    d = disc_for(T)
    # parent cell (level 3) at x-index 3 (last inside the fine half),
    # coarse leaf J at x-index 4
    P = np.array([3, 2, 2])
    J = T.find(3, 4, 2, 2)
    assert J >= 0
    u = np.zeros(T.n)
    vals = {(0, 1): g["p0"], (1, 1): g["p1"], (0, 0): g["p2"], (1, 0): g["p3"]}
    for (dx, dy), v in vals.items():
        for dz in (0, 1):
            c = 2 * P + np.array([dx, dy, dz])
            u[T.find(4, *c)] = v
    u[J] = g["p4"]
    Au = d.A @ u
    for (dx, dy), ghost in (((1, 1), g["g6"]), ((1, 0), g["g7"])):
        c = 2 * P + np.array([dx, dy, 0])
        i = T.find(4, *c)
        want = 0.0
        for dd in range(6):
            k = d.dirk[i, dd]
            kind = d.kind[i, dd]
            if kind == D.COARSE:
                assert dd == 1
                want += k * (u[i] - ghost)
            elif kind == D.SAME:
                want += k * (u[i] - u[d.nidx[i, dd]])
            else:
                want += k * u[i]
        assert np.isclose(Au[i], want, rtol=1e-14, atol=1e-14)
    # flux identity f1 + f3 = f4 on each of the two z layers: the coarse leaf's
    # -x face sees K_F (u_J - mean) with K_F the sum of its sub-face k / 2
    h = 2.0 ** -4
    KF = d.dirk[J, 0]
    assert np.isclose(KF, 4 * h / 2)
    f_fine = sum(d.dirk[T.find(4, *(2 * P + np.array([1, dy, dz]))), 1]
                 * ((g["g6"] if dy else g["g7"]) - (g["p1"] if dy else g["p3"]))
                 for dy in (0, 1) for dz in (0, 1))
    f_coarse = KF * (g["p4"] - (g["p0"] + g["p1"] + g["p2"] + g["p3"]) / 4)
    assert np.isclose(f_fine, f_coarse, rtol=1e-14)
    assert np.isclose(g["f1"] + g["f3"], g["f4"], rtol=1e-14)


@pytest.mark.parametrize("maker", ["half", "three", "cut"])
def test_conservation_all_neumann(maker):
    """A 1 = 0 and 1^T A = 0 when every wall is Neumann (Eq. 8 flux
    conservation makes the column sums vanish at T-junctions)."""
    if maker == "half":
        T = half_tree(3)
        d = disc_for(T, bc=(D.NEUMANN,) * 6, seed=3)
    elif maker == "three":
        spec = {"min_level": 3, "max_level": 5, "node_size": 4, "prims": []}
        T = O.Octree(spec, three_level_nodes(3))
        d = disc_for(T, bc=(D.NEUMANN,) * 6, seed=4)
    else:
        T = O.Octree(problems.config_spec(3, min_level=3, max_level=6))
        d = D.Discretization(T, None, (D.NEUMANN,) * 6)
        d.set_beta(problems.face_beta(3, d.face_level, d.face_ijk, d.face_dir))
    one = d.active.astype(np.float64)
    scale = np.abs(d.A).sum()
    assert np.abs(d.A @ one).max() <= 1e-15 * scale
    assert np.abs(d.A.T @ one).max() <= 1e-15 * scale


def test_symmetric_without_tjunctions():
    T = uniform_tree(4)
    d = disc_for(T, seed=5)
    assert abs(d.A - d.A.T).max() == 0.0


def test_nonsymmetry_confined_to_tjunction_blocks():
    T = half_tree(3)
    d = disc_for(T, seed=6)
    S = (d.A - d.A.T).tocoo()
    rows = set(S.row[S.data != 0]) | set(S.col[S.data != 0])
    # cells that are T-face cells, coarse T cells or siblings of T-face cells
    tcells = set(np.nonzero((d.kind == D.COARSE).any(axis=1))[0])
    tcells |= set(np.nonzero((d.kind == D.FINER).any(axis=1))[0])
    sib = set()
    for i in np.nonzero((d.kind == D.COARSE).any(axis=1))[0]:
        ch, _, _ = d.parent_children(i)
        sib |= set(ch.ravel())
    assert rows <= (tcells | sib)
    assert len(rows) > 0


@pytest.mark.parametrize("seed", [7, 8])
def test_definiteness_on_tiny_adaptive_grid(seed):
    T = half_tree(3)
    d = disc_for(T, seed=seed)
    A = d.A.toarray()
    sym = 0.5 * (A + A.T)
    assert np.linalg.eigvalsh(sym).min() > 0
    ev = np.linalg.eigvals(A)
    assert ev.real.min() > 0


def test_pcg_matches_direct_solve_on_small_grids():
    for T, bc in ((half_tree(3), (D.DIRICHLET,) * 6),
                  (O.Octree({"min_level": 3, "max_level": 5, "node_size": 4, "prims": []},
                            three_level_nodes(3)), (D.NEUMANN,) * 3 + (D.DIRICHLET,) + (D.NEUMANN,) * 2)):
        d = disc_for(T, bc=bc, seed=9)
        rng = np.random.default_rng(10)
        b = rng.uniform(-1, 1, T.n)
        x_direct = spla.splu(d.A.tocsc()).solve(b)
        H = hierarchy(d)
        x, info = K.pcg(d.A, b, H.vcycle, 1e-13, 200)
        assert info["status"] == 0
        assert np.linalg.norm(x - x_direct) <= 1e-11 * np.linalg.norm(x_direct)


def _error(T, d, cfg, x):
    p, _ = problems.manufactured(cfg)
    xc, h = problems.cell_centers(T.level, T.ijk)
    e = x - p(xc[:, 0], xc[:, 1], xc[:, 2])
    return np.sqrt(np.sum(h ** 3 * e ** 2))


@pytest.mark.parametrize("cfg", [1, 2])
def test_second_order_on_self_similar_adaptive_family(cfg):
    """Manufactured solutions of workloads 1 and 2 on grids with half the
    domain one level finer (T-junctions on a fixed plane): fitted order of
    the volume-weighted RMS error is >= 1.8."""
    errs = []
    for l in (3, 4, 5):
        T = half_tree(l)
        bc, th = problems.config_bc(cfg)
        d = disc_for(T, bc=bc, theta=th)
        rhs = problems.rhs_manufactured(cfg, T.level, T.ijk, d.face_owner, d.face_level,
                                        d.face_ijk, d.face_dir, d.face_other,
                                        np.ones(d.n_faces), bc, th)
        x, info = K.pcg(d.A, rhs, hierarchy(d).vcycle, 1e-12, 200)
        errs.append(_error(T, d, cfg, x))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders >= 1.8), orders


def test_second_order_uniform_and_paper_dirichlet_rule_first_order():
    errs, errs1 = [], []
    for l in (3, 4, 5):
        T = uniform_tree(l)
        for th, out in ((0.5, errs), (1.0, errs1)):
            d = disc_for(T, theta=th)
            rhs = problems.rhs_manufactured(1, T.level, T.ijk)
            x, _ = K.pcg(d.A, rhs, hierarchy(d).vcycle, 1e-12, 200)
            out.append(_error(T, d, 1, x))
    o = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    o1 = np.log2(np.array(errs1[:-1]) / np.array(errs1[1:]))
    assert np.all(o >= 1.9), o
    # the Dirichlet-cell rule (wall value at the outside cell centre) is
    # first order for walls on cube faces
    assert np.all(o1 < 1.3), o1


def test_face_fraction_triangle_rule_against_sampling():
    rng = np.random.default_rng(11)
    for _ in range(20):
        v = rng.uniform(-1, 1, 3)
        got = problems._triangle_positive_fraction(v[:1], v[1:2], v[2:])[0]
        # dense barycentric sampling of the linear interpolant
        m = 400
        a, b = np.meshgrid(np.arange(m) + 1 / 3, np.arange(m) + 1 / 3, indexing="ij")
        a, b = a.ravel() / m, b.ravel() / m
        keep = a + b < 1
        a, b = a[keep], b[keep]
        phi = v[0] * (1 - a - b) + v[1] * a + v[2] * b
        assert abs(got - (phi > 0).mean()) < 5e-3


def test_face_fraction_planar_interface():
    # phi = x - 0.3: a face of the unit cell normal to y spanning x in [0, 1]
    def phi(x, y, z):
        return x - 0.3
    f = problems.face_fractions(np.array([0]), np.array([[0, 0, 0]]), np.array([2]), phi)
    assert np.isclose(f[0], 0.7, rtol=1e-14)
    f = problems.face_fractions(np.array([0]), np.array([[0, 0, 0]]), np.array([0]), phi)
    assert f[0] == 0.0
    f = problems.face_fractions(np.array([0]), np.array([[0, 0, 0]]), np.array([1]), phi)
    assert f[0] == 1.0


def test_cut_cell_workload_structure():
    T, d, beta, rhs = config_problem(3, min_level=4, max_level=6)
    assert np.all((beta >= 0) & (beta <= 1))
    assert (~d.active).sum() > 0  # solid cells are not unknowns
    # Dirichlet only on the top wall: the operator is definite
    H = hierarchy(d)
    x, info = K.pcg(d.A, rhs, H.vcycle, 1e-10, 200, active=d.active)
    assert info["status"] == 0 and info["true"] < 1e-9
