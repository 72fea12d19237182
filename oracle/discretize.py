"""Faces, coefficients and the composite leaf operator (test infrastructure).

Paper passages restated here
  * Section 2.1, Eq. (2) (flux form) and Eq. (3) (four-coefficient form):
    sum over faces of (p_i - p_j) S_ij / h; a cell stores its diagonal and
    the coefficients of its three negative faces.
  * Section 2.1, cell types: a fluid face has coefficient h (area h^2 over
    spacing h), a Neumann face 0, a Dirichlet face keeps its coefficient with
    the outside value 0; non-DOF cells have diagonal 0 ("active" <=> c != 0,
    Section 2.5).
  * Section 3.1, Eqs. (5)-(10): at a T-junction the fine cell i sees the
    ghost value g = u_i + (u_J - mean(children of parent(i)))/2, and the coarse
    cell J sees the face with coefficient (sum of fine face areas)/(2h).

Conventions and readings
  * Coefficients are stored as magnitudes k >= 0; the operator is
    (A u)_i = sum_faces k_f (u_i - u_nbr), i.e. the volume-integrated
    -div(beta grad u) with a positive diagonal.
  * Directions 0..5 are -x, +x, -y, +y, -z, +z.
  * Walls are the faces of the unit cube.  A Dirichlet wall face has
    coefficient beta S / (theta h) (the wall at distance theta h from the
    cell centre; theta = 1 is the paper's Dirichlet-cell rule, theta = 1/2
    puts p = 0 on the face itself).  A Neumann wall face has coefficient 0.
  * Face ownership: a face between leaves of different levels belongs to the
    finer leaf; between equal levels to the leaf on its + side; a wall face
    to its leaf.  Canonical face order is (owner, direction).
  * The mean over the children of a T-junction parent is taken over its
    *active* children.  In a balanced octree of B^3 nodes (B even), the
    children of such a parent are leaves; this is asserted.
"""

import numpy as np
import scipy.sparse as sp

from .octree import Octree

WALL, SAME, COARSE, FINER = 0, 1, 2, 3
NEUMANN, DIRICHLET = 0, 1

DIRV = np.array([(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)],
                dtype=np.int64)


def neighbours(tree: Octree):
    """Per leaf and direction: kind (WALL/SAME/COARSE/FINER) and index of the
    same-level or coarser neighbour leaf (-1 otherwise)."""
    N = tree.n
    kind = np.zeros((N, 6), dtype=np.int64)
    idx = np.full((N, 6), -1, dtype=np.int64)
    lev = tree.level
    for d in range(6):
        nb = tree.ijk + DIRV[d]
        n = np.left_shift(1, lev)
        inside = np.all((nb >= 0) & (nb < n[:, None]), axis=1)
        same = tree.find(lev, nb[:, 0], nb[:, 1], nb[:, 2])
        same = np.where(inside, same, -1)
        co = tree.find(lev - 1, nb[:, 0] >> 1, nb[:, 1] >> 1, nb[:, 2] >> 1)
        co = np.where(inside & (same < 0) & (lev - 1 >= tree.lmin), co, -1)
        k = np.full(N, FINER)
        k[~inside] = WALL
        k[same >= 0] = SAME
        k[co >= 0] = COARSE
        kind[:, d] = k
        idx[:, d] = np.where(same >= 0, same, co)
        fin = np.nonzero(k == FINER)[0]
        for l in np.unique(lev[fin]):
            f = fin[lev[fin] == l]
            assert np.all(tree.is_inner(l, nb[f, 0], nb[f, 1], nb[f, 2]))
    return kind, idx


class Discretization:
    """Faces, per-face coefficients, stored cell coefficients and the
    composite leaf operator of one octree."""

    def __init__(self, tree: Octree, face_beta=None, bc=(DIRICHLET,) * 6,
                 theta=0.5):
        self.tree = tree
        self.bc = np.asarray(bc, dtype=np.int64)
        self.theta = float(theta)
        self.kind, self.nidx = neighbours(tree)
        self._build_faces()
        if face_beta is not None:
            self.set_beta(face_beta)

    # ----------------------------------------------------------- faces
    def _build_faces(self):
        T = self.tree
        own = np.zeros((T.n, 6), dtype=bool)
        for d in range(6):
            k = self.kind[:, d]
            own[:, d] = (k == WALL) | (k == COARSE) | ((k == SAME) & (d % 2 == 0))
        owner, direc = np.nonzero(own)  # row-major: (owner, dir) order
        self.face_owner = owner.astype(np.int64)
        self.face_dir = direc.astype(np.int64)
        self.face_kind = self.kind[owner, direc]
        self.face_other = np.where(self.face_kind == WALL, -1, self.nidx[owner, direc])
        self.face_level = T.level[owner]
        self.face_ijk = T.ijk[owner]
        h = np.ldexp(1.0, -self.face_level)
        self.face_area = h * h
        self.n_faces = len(owner)
        fid = np.full((T.n, 6), -1, dtype=np.int64)
        fid[owner, direc] = np.arange(self.n_faces)
        self.face_id = fid

    def face_scale(self):
        """dk_f / dbeta_f: S/h, S/(theta h) at Dirichlet walls, 0 at Neumann."""
        h = np.ldexp(1.0, -self.face_level)
        s = self.face_area / h
        wall = self.face_kind == WALL
        dir_bc = self.bc[self.face_dir]
        s = np.where(wall & (dir_bc == DIRICHLET), self.face_area / (self.theta * h), s)
        s = np.where(wall & (dir_bc == NEUMANN), 0.0, s)
        return s

    def set_beta(self, face_beta):
        beta = np.asarray(face_beta, dtype=np.float64)
        assert beta.shape == (self.n_faces,)
        self.beta = beta
        self.kf = beta * self.face_scale()
        self._cell_coefficients()
        self.A = self.composite_operator()

    # ------------------------------------------------------ coefficients
    def subfaces(self, i, d):
        """Face ids (len(i), 4) of the finer leaves across direction d of
        leaves ``i`` (whose same-level neighbour is an inner cell)."""
        T = self.tree
        i = np.atleast_1d(i)
        l = T.level[i]
        nb = T.ijk[i] + DIRV[d]
        a, s = d // 2, d % 2
        others = [x for x in range(3) if x != a]
        out = np.empty((len(i), 4), dtype=np.int64)
        for n, (u, v) in enumerate(((0, 0), (1, 0), (0, 1), (1, 1))):
            delta = np.zeros(3, dtype=np.int64)
            delta[a] = 1 - s
            delta[others[0]] = u
            delta[others[1]] = v
            ch = 2 * nb + delta
            f = T.find(l + 1, ch[:, 0], ch[:, 1], ch[:, 2])
            assert np.all(f >= 0), "finer neighbour must be a leaf (2:1 balance)"
            out[:, n] = self.face_id[f, d ^ 1]
        assert np.all(out >= 0)
        return out

    def children_of(self, level, cell):
        """Leaf indices (len, 8) of the children at level+1 of cells ``cell``
        (len, 3) at ``level``; asserts they are leaves."""
        T = self.tree
        cell = np.atleast_2d(cell)
        level = np.broadcast_to(np.asarray(level), (len(cell),))
        out = np.empty((len(cell), 8), dtype=np.int64)
        n = 0
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    q = 2 * cell + np.array([dx, dy, dz])
                    out[:, n] = T.find(level + 1, q[:, 0], q[:, 1], q[:, 2])
                    n += 1
        assert np.all(out >= 0), "T-junction parent has non-leaf children"
        return out

    def _cell_coefficients(self):
        """dirk[i, d]: coefficient of leaf i across direction d (the face's k;
        for a finer neighbour, the sum of the 4 fine sub-face k / 2).
        c_i = sum_d dirk[i, d] (Eq. 3 diagonal).  cx, cy, cz = dirk at
        -x, -y, -z (Eq. 3 off-diagonals, stored as magnitudes)."""
        T = self.tree
        dirk = np.zeros((T.n, 6))
        for d in range(6):
            k = self.kind[:, d]
            own = self.face_id[:, d] >= 0
            dirk[own, d] = self.kf[self.face_id[own, d]]
            plus_same = (k == SAME) & (d % 2 == 1)
            j = self.nidx[plus_same, d]
            dirk[plus_same, d] = self.kf[self.face_id[j, d - 1]]
            fin = np.nonzero(k == FINER)[0]
            if len(fin):
                sub = self.subfaces(fin, d)
                acc = np.zeros(len(fin))
                for n in range(4):
                    acc = acc + self.kf[sub[:, n]] / 2.0
                dirk[fin, d] = acc
        self.dirk = dirk
        self.c = dirk.sum(axis=1)
        self.active = self.c > 0
        # a face with k > 0 never touches an inactive cell (all faces of an
        # inactive cell have k = 0); the coarsening guard relies on this
        assert np.all(self.c >= 0)

    # ------------------------------------------------- composite operator
    def parent_children(self, i):
        """Siblings (len, 8) of leaves ``i`` (children of their parents),
        with the active mask and active count."""
        T = self.tree
        i = np.atleast_1d(i)
        ch = self.children_of(T.level[i] - 1, T.ijk[i] >> 1)
        act = self.active[ch]
        return ch, act, act.sum(axis=1)

    def composite_operator(self):
        """Explicit CSR of the composite leaf operator (rows and columns of
        inactive leaves are zero)."""
        T = self.tree
        rows, cols, vals = [], [], []
        act = self.active

        def add(r, c, v):
            rows.append(np.atleast_1d(r))
            cols.append(np.atleast_1d(c))
            vals.append(np.atleast_1d(v).astype(np.float64))

        for d in range(6):
            k = self.kind[:, d]
            kd = self.dirk[:, d]
            # walls: the outside value is 0 (Dirichlet) or the face is absent
            m = (k == WALL) & act
            add(np.nonzero(m)[0], np.nonzero(m)[0], kd[m])
            # same-level faces
            m = (k == SAME) & act
            i = np.nonzero(m)[0]
            j = self.nidx[m, d]
            add(i, i, kd[m])
            add(i, j, -kd[m])
            # fine side of a T-face: (k/2) (mean_P - u_J)
            i = np.nonzero((k == COARSE) & act)[0]
            if len(i):
                J = self.nidx[i, d]
                ch, cact, cnt = self.parent_children(i)
                w = kd[i] / 2.0
                for n in range(8):
                    m = cact[:, n]
                    add(i[m], ch[m, n], w[m] / cnt[m])
                add(i, J, -w)
            # coarse side of a T-face: sum over sub-faces (k_f/2)(u_i - mean_P)
            i = np.nonzero((k == FINER) & act)[0]
            if len(i):
                cell = T.ijk[i] + DIRV[d]
                ch = self.children_of(T.level[i], cell)
                cact = self.active[ch]
                cnt = cact.sum(axis=1)
                sub = self.subfaces(i, d)
                for n in range(4):
                    w = self.kf[sub[:, n]] / 2.0
                    ok = w != 0.0
                    add(i[ok], i[ok], w[ok])
                    for q in range(8):
                        m = ok & cact[:, q]
                        add(i[m], ch[m, q], -w[m] / cnt[m])
        r = np.concatenate(rows)
        c = np.concatenate(cols)
        v = np.concatenate(vals)
        A = sp.coo_matrix((v, (r, c)), shape=(T.n, T.n)).tocsr()
        A.sum_duplicates()
        return A

    # --------------------------------------------------- per-face gradient
    def face_gradient(self, lam, p):
        """dL/dbeta_f = -lam^T (dA/dbeta_f) p for every face (0 where a side of
        the face is inactive or the face is a Neumann wall)."""
        T = self.tree
        lam = np.asarray(lam)
        p = np.asarray(p)
        s = self.face_scale()
        o = self.face_owner
        oth = self.face_other
        g = np.zeros(self.n_faces)
        kind = self.face_kind
        act = self.active
        m = (kind == WALL) & act[o]
        g[m] = -s[m] * lam[o[m]] * p[o[m]]
        m = (kind == SAME) & act[o] & act[np.maximum(oth, 0)]
        g[m] = -s[m] * (lam[o[m]] - lam[oth[m]]) * (p[o[m]] - p[oth[m]])
        f = np.nonzero((kind == COARSE) & act[o] & act[np.maximum(oth, 0)])[0]
        if len(f):
            i, J = o[f], oth[f]
            ch, cact, cnt = self.parent_children(i)
            pbar = (p[ch] * cact).sum(axis=1) / cnt
            g[f] = -(s[f] / 2.0) * (lam[i] - lam[J]) * (pbar - p[J])
        return g


def face_geometry(tree: Octree, bc=(DIRICHLET,) * 6, theta=0.5):
    """Face list without coefficients (for building problem inputs)."""
    return Discretization(tree, None, bc, theta)
