"""Pins of the oracle's mixed-precision store (``Hierarchy.stored_precision``),
the input transformation the GPU's mixed cycle is compared against: its
FP64 cycle runs on the coefficients an FP32-leaf / FP16-inner store keeps.
"""

import numpy as np

import problems
from oracle import multigrid as M
from oracle import octree as O

from oracle_fixtures import config_problem, disc_for, half_tree, hierarchy, three_level_nodes


def _levels_equal(H, R):
    for l in H.levels:
        A, B = H.levels[l], R.levels[l]
        assert (A.A != B.A).nnz == 0, l
        if A.B is not None:
            assert (A.B != B.B).nnz == 0, l
        assert np.array_equal(A.c, B.c), l


def test_dyadic_coefficients_are_stored_exactly():
    """With beta = 1 every coefficient of Eq. (3) and of Algorithm 3 is a
    dyadic number with a few significant bits (k = h at a face, h / theta at
    a Dirichlet wall, k / h_l small integers or halves on coarse levels,
    T-face sums over 2), so FP32 and FP16 keep them exactly: the stored
    hierarchy equals the FP64 one operator for operator -- in particular
    the diagonal rebuilt from the face coefficients, wall parts included,
    is the diagonal of Eq. (3) and Algorithm 3 -- and the cycles agree bit
    for bit."""
    trees = [O.Octree(problems.uniform_spec(5)), half_tree(4),
             O.Octree({"min_level": 4, "max_level": 6, "node_size": 4, "prims": []},
                      three_level_nodes(4))]
    rng = np.random.default_rng(71)
    for T in trees:
        d = disc_for(T)  # Dirichlet on every wall, theta = 1/2
        H = hierarchy(d)
        R = H.stored_precision()
        _levels_equal(H, R)
        r = rng.uniform(-1, 1, T.n)
        assert np.array_equal(R.vcycle(r), H.vcycle(r))


def test_rounding_bounds_and_conservation():
    """Jittered cut-cell coefficients (the cut-sphere family, levels 4..6):
    each stored face coefficient is within FP32 (leaf) or FP16 (inner)
    rounding of the FP64 one; the rebuilt diagonal is within the rounding
    of the six faces of the FP64 diagonal (a plus/minus or neighbour mix-up
    would move it by the 1% jitter); and every row of a stored level
    operator without a Dirichlet face still sums to zero (conservation)."""
    T, d, beta, rhs = config_problem(3, min_level=4, max_level=6)
    H = hierarchy(d)
    R = H.stored_precision()
    for l, Lv in H.levels.items():
        Rv = R.levels[l]
        h = 2.0 ** -l
        for a, b in ((Lv.kx, Rv.kx), (Lv.ky, Rv.ky), (Lv.kz, Rv.kz)):
            tol = np.where(Lv.leaf, 2.0 ** -24 * np.abs(a), 2.0 ** -11 * np.abs(a) + 2.0 ** -14 * h)
            assert np.all(np.abs(a - b) <= tol), l
        act = Lv.active
        # a leaf cell's plus face toward an inner cell is stored as that
        # cell stores it (FP16)
        half_nbr = np.zeros(Lv.n, dtype=bool)
        for a in range(3):
            kind, idx = Lv.nkind[:, 2 * a + 1], Lv.nidx[:, 2 * a + 1]
            same = kind == M.SAME
            half_nbr[same] |= ~Lv.leaf[idx[same]]
        tol = np.where(Lv.leaf & ~half_nbr, 6 * 2.0 ** -24 * Lv.c,
                       2.0 ** -11 * Lv.c + 6 * 2.0 ** -14 * h)
        assert np.all(np.abs(Rv.c - Lv.c)[act] <= tol[act] + 1e-15 * Lv.c[act]), l
        assert np.all(Rv.c[act] > 0.0), l
        # rows with no Dirichlet face: the level operator (ghost coupling to
        # the coarser leaves included) has zero row sums
        rows = np.asarray(Rv.A.sum(axis=1)).ravel()
        if Rv.B is not None:
            rows = rows + np.asarray(Rv.B.sum(axis=1)).ravel()
        dir_faces = np.zeros(Lv.n, dtype=bool)
        for a in range(3):
            for s in (0, 1):
                dd = 2 * a + s
                edge = (Lv.ijk[:, a] == 0) if s == 0 else (Lv.ijk[:, a] == (1 << l) - 1)
                if d.bc[dd] == 1:
                    dir_faces |= edge
        free = act & ~dir_faces
        assert np.abs(rows[free]).max() <= 1e-13 * Rv.c[free].max(), l


def test_sliver_coefficients_are_raised_to_the_fp16_normal_range():
    """A sibling group of cells whose faces all carry beta = 1e-9: on the
    coarse level their parent's coefficients (about 1e-9 h) are below
    FP16's range; stored, they become 2^-14 h_l, so the coarse cell keeps a
    positive diagonal where the FP64 one is positive and the cycle stays
    finite; zero coefficients stay zero."""
    T = O.Octree(problems.uniform_spec(4))
    d = disc_for(T)
    beta = np.ones(d.n_faces)
    # the 8 cells of the first parent (level-4 cells 0..1 in each axis)
    corner = np.all(T.ijk < 2, axis=1)
    cells = np.nonzero(corner)[0]
    touch = np.isin(d.face_owner, cells) | np.isin(d.face_other, cells)
    beta[touch] = 1e-9
    d.set_beta(beta)
    H = hierarchy(d)
    R = H.stored_precision()
    Lv, Rv = H.levels[3], R.levels[3]
    parent = Lv.find(np.array([[0, 0, 0]]))[0]
    assert 0.0 < Lv.c[parent] < 1e-7 * 2.0 ** -3
    assert Rv.c[parent] >= 2.0 ** -14 * 2.0 ** -3
    for k0, k1 in ((Lv.kx, Rv.kx), (Lv.ky, Rv.ky), (Lv.kz, Rv.kz)):
        assert np.all((k1 == 0.0) == (k0 == 0.0))
    z = R.vcycle(np.random.default_rng(72).uniform(-1, 1, T.n))
    assert np.all(np.isfinite(z))
    # without the floor the parent's FP16 coefficients would all be zero
    q = (Lv.c[parent] * 2.0 ** 3).astype(np.float32).astype(np.float16)
    assert q == 0.0
    assert M.stored_value(np.array([Lv.c[parent]]), np.array([False]), 3)[0] == 2.0 ** -17
