"""Multigrid hierarchy and cycles of the oracle (test infrastructure).

Paper passages restated here
  * Section 2.3: constant prolongation P (copy parent to children), restriction
    R = P^T / alpha, RBGS smoothing with nu_l = 2 pre and post in opposite
    colour orders and nu_b = 10 on the coarsest level split into two phases
    of opposite order.
  * Section 2.4, Eq. (12): Galerkin entries A^{l-1}_IJ = (1/alpha) sum of
    A^l_ij over children pairs.
  * Section 2.5, Algorithm 3: matrix-free coarsening of the four coefficients.
  * Section 3.1, Eq. (10): ghost value at a T-junction.
  * Section 3.2, Algorithm 4: FAS-style cycle; Algorithm 2: standard cycle.

Readings (the paper is silent or ambiguous)
  * Level l holds every cell of level l that is a leaf or an inner cell.  A
    level-l leaf next to a region covered by a level-(l-1) leaf J sees the
    ghost u_i + (u_J - mean_active_siblings(u))/2 with u_J read from level
    l-1 (coupling matrix B^l); the coarse side of that face is an ordinary
    same-level face at level l-1 (Algorithm 3 gives the coarse coefficient as
    the sum of fine sub-face coefficients over alpha).
  * One colour half-sweep is a Jacobi step over that colour from a snapshot
    (ghosts included), dividing by the stored diagonal c_i.  Red is even
    i+j+k at the cell's level.  Pre-smoothing (R,B)^nu, post-smoothing
    (B,R)^nu, coarsest (R,B)^(nu_b/2) then (B,R)^(nu_b/2).
  * Avg and the T-junction mean run over active children; prolongation
    updates active children only.
  * The FAS right-hand side beta R r + A^{l-1} u* replaces b on inner cells
    only; leaves of level l-1 keep their own right-hand side (the PCG
    residual), their initial guess u* is their current value.
  * Algorithm 3 is applied as printed; its off-diagonal branch needs no
    activity guard here because a face with non-zero coefficient never
    touches an inactive cell (asserted by the discretisation).
  * Mixed-precision storage (``stored_precision``): the cycle's arithmetic
    is unchanged (FP64 here); only its coefficients are replaced by the
    values a mixed-precision store keeps -- leaf cells in FP32, inner cells
    as FP16 copies of c/h_l (through FP32, round to nearest even; non-zero
    values below FP16's normal range raised to 2^-14) -- and the diagonal
    of every cell by the sum of the six face coefficients it then sees, so
    each row of a level operator stays conservative.
  * The adjoint solve uses the exact transpose M^T of the cycle M (the
    operator is non-symmetric at T-junctions, so M is not symmetric; PCG on
    A^T needs an approximation of A^-T).  M^T is the cycle's linear steps
    transposed and taken in reverse order; written out, it is a cycle for
    A^T in residual form: rho (the adjoint of u) is a residual and y (the
    adjoint of b) accumulates the solution.
"""

import copy

import numpy as np
import scipy.sparse as sp

from .discretize import DIRV, COARSE as D_COARSE
from .octree import cell_key

WALL, SAME, COARSE = 0, 1, 2


def f32(x):
    """FP64 -> FP32 (round to nearest even) -> FP64."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def stored_value(k, leaf, l):
    """Coefficients of level-l cells as a mixed-precision store keeps them:
    FP32 on leaf cells; on inner cells k = h_l * FP16(FP32(k / h_l)), a
    non-zero value below FP16's normal range (2^-14) raised to 2^-14."""
    k = np.asarray(k, dtype=np.float64)
    q = (k * 2.0 ** l).astype(np.float32).astype(np.float16).astype(np.float64)
    tiny = (k != 0.0) & (np.abs(q) < 2.0 ** -14)
    q = np.where(tiny, np.copysign(2.0 ** -14, k), q)
    return np.where(leaf, f32(k), q * 2.0 ** -l)


class Level:
    def __init__(self, l, ijk, leaf_idx):
        order = np.argsort(cell_key(np.full(len(ijk), l), ijk[:, 0], ijk[:, 1], ijk[:, 2]))
        self.l = l
        self.ijk = ijk[order]
        self.leaf_idx = leaf_idx[order]
        self.leaf = self.leaf_idx >= 0
        self.n = len(self.ijk)
        self.keys = cell_key(np.full(self.n, l), self.ijk[:, 0], self.ijk[:, 1], self.ijk[:, 2])
        self.colour = (self.ijk.sum(axis=1) % 2).astype(np.int64)
        self.h = 2.0 ** (-l)

    def find(self, ijk):
        ijk = np.atleast_2d(ijk)
        n = 1 << self.l
        ok = np.all((ijk >= 0) & (ijk < n), axis=1)
        key = cell_key(np.full(len(ijk), self.l), np.where(ok, ijk[:, 0], 0),
                       np.where(ok, ijk[:, 1], 0), np.where(ok, ijk[:, 2], 0))
        pos = np.minimum(np.searchsorted(self.keys, key), self.n - 1)
        return np.where(ok & (self.keys[pos] == key), pos, -1)


class Hierarchy:
    """Levels finest .. coarsest with Algorithm 3 coefficients and the
    explicit level operators, transfer operators and FAS/standard cycles."""

    def __init__(self, disc, coarsest=3, alpha=2.0, beta_mg=2.0, nu_pre=2,
                 nu_post=2, nu_coarse=10, mu=1):
        self.disc = disc
        T = disc.tree
        self.alpha = float(alpha)
        self.beta_mg = float(beta_mg)
        self.nu_pre, self.nu_post, self.nu_coarse, self.mu = nu_pre, nu_post, nu_coarse, mu
        self.L = int(T.level.max())
        self.lc = int(coarsest)
        assert self.lc <= T.lmin
        self.levels = {}
        for l in range(self.L, self.lc - 1, -1):
            m = T.level == l
            leaf_ijk = T.ijk[m]
            leaf_idx = np.nonzero(m)[0]
            inner = T.inner_keys(l)
            km = (1 << 13) - 1
            in_ijk = np.stack([(inner >> 26) & km, (inner >> 13) & km, inner & km], axis=1)
            ijk = np.concatenate([leaf_ijk, in_ijk]).astype(np.int64)
            idx = np.concatenate([leaf_idx, np.full(len(in_ijk), -1)])
            self.levels[l] = Level(l, ijk, idx)
        self._coefficients()
        for l in range(self.L, self.lc - 1, -1):
            self._neighbours(l)
            self._operators(l)
        for l in range(self.L, self.lc, -1):
            self._transfers(l)

    # ------------------------------------------------------- coefficients
    def children(self, l):
        """(n_{l}, 8) indices at level l+1 of the children of level-l cells
        (-1 for leaves), in Morton order dx + 2 dy + 4 dz."""
        Lv = self.levels[l]
        F = self.levels[l + 1]
        out = np.full((Lv.n, 8), -1, dtype=np.int64)
        inner = ~Lv.leaf
        n = 0
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    q = 2 * Lv.ijk[inner] + np.array([dx, dy, dz])
                    out[inner, n] = F.find(q)
                    n += 1
        assert np.all(out[inner] >= 0)
        return out

    def _coefficients(self):
        d = self.disc
        a = self.alpha
        for l in range(self.L, self.lc - 1, -1):
            Lv = self.levels[l]
            Lv.c = np.zeros(Lv.n)
            Lv.kx = np.zeros(Lv.n)
            Lv.ky = np.zeros(Lv.n)
            Lv.kz = np.zeros(Lv.n)
            Lv.kplus = np.zeros((Lv.n, 3))
            lf = Lv.leaf
            li = Lv.leaf_idx[lf]
            Lv.c[lf] = d.c[li]
            Lv.kx[lf] = d.dirk[li, 0]
            Lv.ky[lf] = d.dirk[li, 2]
            Lv.kz[lf] = d.dirk[li, 4]
            for ax in range(3):
                Lv.kplus[lf, ax] = d.dirk[li, 2 * ax + 1]
            if l < self.L:
                self._coarsen(l)
            Lv.active = Lv.c != 0.0

    def _coarsen(self, l):
        """Algorithm 3 for every inner cell of level l from level l+1."""
        Lv = self.levels[l]
        F = self.levels[l + 1]
        ch = self.children(l)
        Lv.ch = ch
        a = self.alpha
        inner = np.nonzero(~Lv.leaf)[0]
        c = np.zeros(len(inner))
        cx = np.zeros(len(inner))
        cy = np.zeros(len(inner))
        cz = np.zeros(len(inner))
        cnt = np.zeros(len(inner), dtype=np.int64)
        kk = (F.kx, F.ky, F.kz)
        acc = (cx, cy, cz)
        n = 0
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    i = ch[inner, n]
                    ci = F.c[i]
                    on = ci != 0.0
                    cnt += on
                    c = c + np.where(on, ci / a, 0.0)
                    for ax, dd in enumerate((dx, dy, dz)):
                        if dd == 1:
                            sib = ch[inner, n - (1 << ax)]
                            both = on & (F.c[sib] != 0.0)
                            c = c + np.where(both, 2.0 / a * (-kk[ax][i]), 0.0)
                        else:
                            acc[ax][:] = acc[ax] + kk[ax][i] / a
                    n += 1
        c = np.where(cnt == 0, 0.0, c)
        Lv.c[inner] = c
        Lv.kx[inner] = cx
        Lv.ky[inner] = cy
        Lv.kz[inner] = cz

    # ------------------------------------------------- stored precision
    def stored_precision(self):
        """A copy of the hierarchy whose level coefficients are those of a
        mixed-precision store (FP32 leaf cells, FP16 c/h_l inner cells; see
        the module readings), with the operators rebuilt from them.  The
        input transformation of the mixed-precision cycle: its FP64 cycle
        is the mixed cycle's arithmetic done exactly."""
        H = copy.copy(self)
        H.levels = {}
        for l, Lv0 in self.levels.items():
            Lv = copy.copy(Lv0)
            own = [Lv0.kx, Lv0.ky, Lv0.kz]
            rown = [stored_value(k, Lv0.leaf, l) for k in own]
            plus64 = [self.face_coef(l, 2 * a + 1) for a in range(3)]
            rplus = []
            for a in range(3):
                kind = Lv0.nkind[:, 2 * a + 1]
                idx = Lv0.nidx[:, 2 * a + 1]
                v = np.zeros(Lv0.n)
                same = kind == SAME
                v[same] = rown[a][idx[same]]
                co = kind == COARSE
                v[co] = f32(Lv0.kplus[co, a])
                rplus.append(v)
            # the wall part of the FP64 diagonal (its plus-wall faces), in
            # FP32 on the first plus wall of the cell
            wall = np.stack([Lv0.nkind[:, 2 * a + 1] == WALL for a in range(3)], axis=1)
            wpart = Lv0.c - (own[0] + own[1] + own[2]) - (plus64[0] + plus64[1] + plus64[2])
            first = np.argmax(wall, axis=1)
            anyw = wall.any(axis=1)
            for a in range(3):
                m = anyw & (first == a)
                rplus[a][m] = f32(wpart[m])
            Lv.kx, Lv.ky, Lv.kz = rown
            Lv.kplus = np.stack([np.where(Lv0.nkind[:, 2 * a + 1] == COARSE, rplus[a],
                                          Lv0.kplus[:, a]) for a in range(3)], axis=1)
            Lv.kplus[Lv0.leaf] = f32(Lv.kplus[Lv0.leaf])
            c = ((rown[0] + rplus[0]) + (rown[1] + rplus[1])) + (rown[2] + rplus[2])
            Lv.c = np.where(Lv0.active, c, 0.0)
            H.levels[l] = Lv
        for l in range(H.L, H.lc - 1, -1):
            H._operators(l)
        return H

    # ---------------------------------------------------------- operators
    def _neighbours(self, l):
        Lv = self.levels[l]
        Lv.nkind = np.zeros((Lv.n, 6), dtype=np.int64)
        Lv.nidx = np.full((Lv.n, 6), -1, dtype=np.int64)
        for d in range(6):
            nb = Lv.ijk + DIRV[d]
            n = 1 << l
            inside = np.all((nb >= 0) & (nb < n), axis=1)
            same = Lv.find(nb)
            kind = np.full(Lv.n, WALL)
            kind[same >= 0] = SAME
            idx = same.copy()
            miss = inside & (same < 0)
            if np.any(miss):
                assert l > self.lc
                C = self.levels[l - 1]
                J = C.find(nb[miss] >> 1)
                assert np.all(J >= 0) and np.all(C.leaf[J]), "T-face must meet a coarser leaf"
                assert np.all(Lv.leaf[miss]), "only leaves have T-faces"
                kind[miss] = COARSE
                idx[miss] = J
            Lv.nkind[:, d] = kind
            Lv.nidx[:, d] = idx

    def face_coef(self, l, d):
        """Coefficient across direction d of every level-l cell."""
        Lv = self.levels[l]
        ax = d // 2
        own = (Lv.kx, Lv.ky, Lv.kz)[ax]
        if d % 2 == 0:
            return own.copy()
        out = np.zeros(Lv.n)
        same = Lv.nkind[:, d] == SAME
        out[same] = own[Lv.nidx[same, d]]
        co = Lv.nkind[:, d] == COARSE
        out[co] = Lv.kplus[co, ax]
        wall = Lv.nkind[:, d] == WALL
        # a + wall face: its coefficient only enters the stored diagonal
        out[wall] = 0.0
        return out

    def siblings(self, l, cells):
        """(len, 8) level-l indices of the siblings of ``cells``."""
        Lv = self.levels[l]
        base = (Lv.ijk[cells] >> 1) << 1
        out = np.empty((len(cells), 8), dtype=np.int64)
        n = 0
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    out[:, n] = Lv.find(base + np.array([dx, dy, dz]))
                    n += 1
        assert np.all(out >= 0)
        return out

    def _operators(self, l):
        """A^l (level-l square part) and B^l (coupling to level-(l-1) leaves)
        of the stencil c_i u_i - sum k v_nbr with T-junction ghosts."""
        Lv = self.levels[l]
        act = Lv.active
        rows, cols, vals = [np.nonzero(act)[0]], [np.nonzero(act)[0]], [Lv.c[act]]
        brow, bcol, bval = [], [], []
        for d in range(6):
            k = self.face_coef(l, d)
            kind = Lv.nkind[:, d]
            m = act & (kind == SAME)
            j = Lv.nidx[m, d]
            assert np.all(Lv.active[j] | (k[m] == 0.0))
            rows.append(np.nonzero(m)[0])
            cols.append(j)
            vals.append(-k[m])
            m = act & (kind == COARSE)
            i = np.nonzero(m)[0]
            if len(i):
                J = Lv.nidx[i, d]
                ki = k[i]
                sib = self.siblings(l, i)
                sact = Lv.active[sib]
                cnt = sact.sum(axis=1)
                rows.append(i)
                cols.append(i)
                vals.append(-ki)
                for q in range(8):
                    mm = sact[:, q]
                    rows.append(i[mm])
                    cols.append(sib[mm, q])
                    vals.append(ki[mm] / 2.0 / cnt[mm])
                brow.append(i)
                bcol.append(J)
                bval.append(-ki / 2.0)
        r = np.concatenate(rows)
        c = np.concatenate(cols)
        v = np.concatenate(vals)
        Lv.A = sp.coo_matrix((v, (r, c)), shape=(Lv.n, Lv.n)).tocsr()
        if l > self.lc:
            nc = self.levels[l - 1].n
            if brow:
                Lv.B = sp.coo_matrix((np.concatenate(bval), (np.concatenate(brow),
                                      np.concatenate(bcol))), shape=(Lv.n, nc)).tocsr()
            else:
                Lv.B = sp.csr_matrix((Lv.n, nc))
        else:
            Lv.B = None

    def _transfers(self, l):
        """R (restriction, 1/alpha per child), Avg (mean over active children)
        and P (copy to active children) between level l and level l-1."""
        F = self.levels[l]
        C = self.levels[l - 1]
        ch = C.ch
        inner = np.nonzero(~C.leaf)[0]
        rr, cc = [], []
        for q in range(8):
            rr.append(inner)
            cc.append(ch[inner, q])
        r = np.concatenate(rr)
        c = np.concatenate(cc)
        F.R = sp.coo_matrix((np.full(len(r), 1.0 / self.alpha), (r, c)),
                            shape=(C.n, F.n)).tocsr()
        act = F.active[c]
        cnt = np.zeros(C.n)
        np.add.at(cnt, r[act], 1.0)
        w = np.where(act, 1.0 / np.maximum(cnt[r], 1.0), 0.0)
        F.Avg = sp.coo_matrix((w, (r, c)), shape=(C.n, F.n)).tocsr()
        F.P = sp.coo_matrix((act.astype(np.float64), (c, r)), shape=(F.n, C.n)).tocsr()
        F.parent = np.full(F.n, -1, dtype=np.int64)
        F.parent[c] = r

    # -------------------------------------------------------------- cycles
    def residual(self, l, u, b):
        Lv = self.levels[l]
        r = b[l] - Lv.A @ u[l]
        if Lv.B is not None:
            r = r - Lv.B @ u[l - 1]
        return np.where(Lv.active, r, 0.0)

    def half_sweep(self, l, u, b, colour):
        Lv = self.levels[l]
        r = self.residual(l, u, b)
        m = Lv.active & (Lv.colour == colour)
        u[l] = u[l] + np.where(m, r / np.where(m, Lv.c, 1.0), 0.0)

    def smooth(self, l, u, b, order, nu):
        for _ in range(nu):
            for colour in order:
                self.half_sweep(l, u, b, colour)

    def coarsest(self, u, b):
        half = self.nu_coarse // 2
        self.smooth(self.lc, u, b, (0, 1), half)
        self.smooth(self.lc, u, b, (1, 0), self.nu_coarse - half)

    def fas(self, l, u, b, trace=None):
        """Algorithm 4 (FAS-style mu-cycle) on level l, in place."""
        if l == self.lc:
            self.coarsest(u, b)
            return
        F = self.levels[l]
        C = self.levels[l - 1]
        self.smooth(l, u, b, (0, 1), self.nu_pre)
        r = self.residual(l, u, b)
        ustar = np.where(C.leaf, u[l - 1], F.Avg @ u[l])
        bc = self.beta_mg * (F.R @ r) + C.A @ ustar
        b[l - 1] = np.where(C.leaf, b[l - 1], np.where(C.active, bc, 0.0))
        u[l - 1] = np.where(C.leaf, u[l - 1], ustar)
        for _ in range(self.mu):
            self.fas(l - 1, u, b, trace)
        u[l] = u[l] + F.P @ (np.where(C.leaf, 0.0, u[l - 1] - ustar))
        if trace is not None:
            trace.append((l, u[l].copy(), u[l - 1].copy()))
        self.smooth(l, u, b, (1, 0), self.nu_post)

    def standard(self, l, u, b, beta):
        """Algorithm 2 (residual-equation mu-cycle; grids without leaves on
        coarse levels)."""
        if l == self.lc:
            self.coarsest(u, b)
            return
        F = self.levels[l]
        C = self.levels[l - 1]
        assert not np.any(C.leaf)
        self.smooth(l, u, b, (0, 1), self.nu_pre)
        r = self.residual(l, u, b)
        b[l - 1] = F.R @ r
        u[l - 1] = np.zeros(C.n)
        for _ in range(self.mu):
            self.standard(l - 1, u, b, beta)
        u[l] = u[l] + beta * (F.P @ u[l - 1])
        self.smooth(l, u, b, (1, 0), self.nu_post)

    def _init(self, r_leaf):
        u = {l: np.zeros(Lv.n) for l, Lv in self.levels.items()}
        b = {}
        for l, Lv in self.levels.items():
            bl = np.zeros(Lv.n)
            m = Lv.leaf & Lv.active
            bl[m] = r_leaf[Lv.leaf_idx[m]]
            b[l] = bl
        return u, b

    def _gather(self, u):
        z = np.zeros(self.disc.tree.n)
        for l, Lv in self.levels.items():
            m = Lv.leaf
            z[Lv.leaf_idx[m]] = np.where(Lv.active[m], u[l][m], 0.0)
        return z

    def vcycle(self, r_leaf, trace=None):
        """The preconditioner z = M r: one FAS-style cycle from u = 0 with the
        leaf right-hand sides r."""
        u, b = self._init(np.asarray(r_leaf, dtype=np.float64))
        self.fas(self.L, u, b, trace)
        return self._gather(u)

    # ------------------------------------------------ transpose of the cycle
    def half_sweep_T(self, l, rho, y, colour):
        """Transpose of one half-sweep u += D_c (b - A u - B u_c):
        w = D_c rho; y += w; rho -= A^T w; rho_c -= B^T w."""
        Lv = self.levels[l]
        m = Lv.active & (Lv.colour == colour)
        w = np.where(m, rho[l] / np.where(m, Lv.c, 1.0), 0.0)
        y[l] = y[l] + w
        rho[l] = rho[l] - Lv.A.T @ w
        if Lv.B is not None:
            rho[l - 1] = rho[l - 1] - Lv.B.T @ w

    def smooth_T(self, l, rho, y, order, nu):
        """Transpose of smooth(l, order, nu): the half-sweeps reversed."""
        seq = [c for _ in range(nu) for c in order]
        for colour in reversed(seq):
            self.half_sweep_T(l, rho, y, colour)

    def fas_T(self, l, rho, y):
        """Transpose of fas(l): the steps of Algorithm 4 in reverse order,
        each transposed."""
        if l == self.lc:
            half = self.nu_coarse // 2
            self.smooth_T(self.lc, rho, y, (1, 0), self.nu_coarse - half)
            self.smooth_T(self.lc, rho, y, (0, 1), half)
            return
        F = self.levels[l]
        C = self.levels[l - 1]
        inner = ~C.leaf
        self.smooth_T(l, rho, y, (1, 0), self.nu_post)
        # u^l += P (u^{l-1} - u*) on inner parents
        pt = F.P.T @ rho[l]
        rho[l - 1] = rho[l - 1] + np.where(inner, pt, 0.0)
        sbar = np.where(inner, -pt, 0.0)
        for _ in range(self.mu):
            self.fas_T(l - 1, rho, y)
        # u^{l-1} = u* on inner cells
        sbar = sbar + np.where(inner, rho[l - 1], 0.0)
        rho[l - 1] = np.where(inner, 0.0, rho[l - 1])
        # b^{l-1} = beta R r + A^{l-1} u* on active inner cells
        yb = np.where(inner & C.active, y[l - 1], 0.0)
        tbar = self.beta_mg * (F.R.T @ yb)
        ust = C.A.T @ yb
        sbar = sbar + np.where(inner, ust, 0.0)
        rho[l - 1] = rho[l - 1] + np.where(C.leaf, ust, 0.0)
        y[l - 1] = np.where(inner, 0.0, y[l - 1])
        # u* = Avg u^l on inner cells
        rho[l] = rho[l] + F.Avg.T @ sbar
        # r = b - A u - B u_c
        tbar = np.where(F.active, tbar, 0.0)
        y[l] = y[l] + tbar
        rho[l] = rho[l] - F.A.T @ tbar
        if F.B is not None:
            rho[l - 1] = rho[l - 1] - F.B.T @ tbar
        self.smooth_T(l, rho, y, (0, 1), self.nu_pre)

    def vcycle_T(self, zbar):
        """M^T zbar: the exact transpose of ``vcycle``."""
        zbar = np.asarray(zbar, dtype=np.float64)
        rho = {}
        y = {l: np.zeros(Lv.n) for l, Lv in self.levels.items()}
        for l, Lv in self.levels.items():
            v = np.zeros(Lv.n)
            m = Lv.leaf & Lv.active
            v[m] = zbar[Lv.leaf_idx[m]]
            rho[l] = v
        self.fas_T(self.L, rho, y)
        out = np.zeros(self.disc.tree.n)
        for l, Lv in self.levels.items():
            m = Lv.leaf & Lv.active
            out[Lv.leaf_idx[m]] = y[l][m]
        return out

    def standard_cycle(self, r_leaf, beta=None):
        u, b = self._init(np.asarray(r_leaf, dtype=np.float64))
        self.standard(self.L, u, b, self.beta_mg if beta is None else beta)
        return self._gather(u)
