"""Adaptive octree of the oracle (test infrastructure only).

Section 3 of the paper: leaf cells carry unknowns, inner cells are parents of
8 finer cells, and face-neighbouring leaves differ by at most one level.
Section 4.1: a tile that meets the surface is refined to the finest level.

Readings
  * The refinement unit is a node of B^3 cells (B = 4).  A node at cell
    level l covers an aligned cube of side B 2^-l.  For l = min .. max-1,
    every leaf node at level l whose closed box meets the predicate of some
    primitive is split into 8 children.
  * 2:1 face balance is then enforced by splitting coarse leaves to the least
    fixed point, which is unique and order independent.
  * Leaves are cells (l, i, j, k).  Canonical order is ascending Morton key
    of the cell's min corner on the 2^max grid, with x in the least
    significant interleaved bit.
"""

import numpy as np

SPHERE = 0
BOX = 1

KEY_BITS = 13  # cells per axis < 2^13


def node_box(level, a, b, c, B):
    s = B * 2.0 ** (-level)
    return (a * s, b * s, c * s), ((a + 1) * s, (b + 1) * s, (c + 1) * s)


def sphere_meets(prim, lo, hi):
    """Closed box meets the shell r - d <= |x - c| <= r + d.

    The distances from c to points of a closed box fill [dmin, dmax]; both
    are compared squared so that no square root enters the decision."""
    c = prim["center"]
    r = prim["radius"]
    d = prim["band"]
    dmin2 = 0.0
    dmax2 = 0.0
    for ax in range(3):
        t = max(lo[ax] - c[ax], 0.0, c[ax] - hi[ax])
        dmin2 = dmin2 + t * t
        u = max(abs(lo[ax] - c[ax]), abs(hi[ax] - c[ax]))
        dmax2 = dmax2 + u * u
    ro = r + d
    ri = r - d
    if dmin2 > ro * ro:
        return False
    if ri > 0.0 and dmax2 < ri * ri:
        return False
    return True


def box_meets_surface(prim, lo, hi):
    """Closed box meets the boundary of the closed obstacle box."""
    olo = prim["lo"]
    ohi = prim["hi"]
    inter = all(lo[ax] <= ohi[ax] and olo[ax] <= hi[ax] for ax in range(3))
    inside = all(olo[ax] < lo[ax] and hi[ax] < ohi[ax] for ax in range(3))
    return inter and not inside


def meets(prim, lo, hi):
    if prim["kind"] == SPHERE:
        return sphere_meets(prim, lo, hi)
    if prim["kind"] == BOX:
        return box_meets_surface(prim, lo, hi)
    raise ValueError(prim["kind"])


def morton3(x, y, z, bits):
    """Interleave the low ``bits`` bits of x, y, z (x least significant)."""
    x = np.asarray(x, dtype=np.uint64)
    y = np.asarray(y, dtype=np.uint64)
    z = np.asarray(z, dtype=np.uint64)
    key = np.zeros(np.broadcast(x, y, z).shape, dtype=np.uint64)
    one = np.uint64(1)
    for b in range(bits):
        bb = np.uint64(b)
        key |= ((x >> bb) & one) << np.uint64(3 * b)
        key |= ((y >> bb) & one) << np.uint64(3 * b + 1)
        key |= ((z >> bb) & one) << np.uint64(3 * b + 2)
    return key


def cell_key(level, i, j, k):
    """Unique integer key of a cell (level, i, j, k)."""
    level = np.asarray(level, dtype=np.int64)
    return (((level << KEY_BITS | np.asarray(i, dtype=np.int64)) << KEY_BITS
             | np.asarray(j, dtype=np.int64)) << KEY_BITS) | np.asarray(k, dtype=np.int64)


def refine_nodes(spec):
    """Leaf nodes {(level, a, b, c)} after predicate refinement and balance."""
    B = spec["node_size"]
    lmin = spec["min_level"]
    lmax = spec["max_level"]
    if (1 << lmin) % B:
        raise ValueError("min_level too small for the node size")
    n0 = (1 << lmin) // B
    leaves = {(lmin, a, b, c) for a in range(n0) for b in range(n0) for c in range(n0)}
    prims = spec["prims"]
    for lev in range(lmin, lmax):
        for node in sorted(n for n in leaves if n[0] == lev):
            lo, hi = node_box(*node, B)
            if any(meets(p, lo, hi) for p in prims):
                leaves.remove(node)
                leaves.update(children(node))
    return balance(leaves, lmin, B)


def children(node):
    lev, a, b, c = node
    return [(lev + 1, 2 * a + dx, 2 * b + dy, 2 * c + dz)
            for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)]


DIRS = ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1))


def covering_leaf(leaves, lmin, lev, a, b, c):
    """Leaf node containing node position (lev, a, b, c), or None when that
    region is refined beyond ``lev``."""
    for q in range(lev, lmin - 1, -1):
        s = lev - q
        cand = (q, a >> s, b >> s, c >> s)
        if cand in leaves:
            return cand
    return None


def balance(leaves, lmin, B, order=None):
    """Split coarse leaves until face-neighbouring leaves differ by at most
    one level.  ``order`` (a permutation seed) only changes the processing
    order; the result is the same least fixed point."""
    leaves = set(leaves)
    rng = np.random.default_rng(order) if order is not None else None
    while True:
        todo = set()
        cur = sorted(leaves)
        if rng is not None:
            rng.shuffle(cur)
        for (lev, a, b, c) in cur:
            n = (1 << lev) // B  # node positions per axis at this level
            for dx, dy, dz in DIRS:
                na, nb, nc = a + dx, b + dy, c + dz
                if min(na, nb, nc) < 0 or max(na, nb, nc) >= n:
                    continue
                cov = covering_leaf(leaves, lmin, lev, na, nb, nc)
                if cov is not None and cov[0] <= lev - 2:
                    todo.add(cov)
        if not todo:
            return leaves
        for node in todo:
            if node in leaves:
                leaves.remove(node)
                leaves.update(children(node))


class Octree:
    """Leaf cells of a balanced node octree in canonical order."""

    def __init__(self, spec, nodes=None):
        self.spec = spec
        self.B = spec["node_size"]
        self.lmin = spec["min_level"]
        self.lmax = spec["max_level"]
        if nodes is None:
            nodes = refine_nodes(spec)
        self.nodes = nodes
        B = self.B
        lv, ii, jj, kk = [], [], [], []
        loc = np.arange(B)
        lx, ly, lz = np.meshgrid(loc, loc, loc, indexing="ij")
        lx, ly, lz = lx.ravel(), ly.ravel(), lz.ravel()
        for (lev, a, b, c) in nodes:
            lv.append(np.full(B ** 3, lev))
            ii.append(a * B + lx)
            jj.append(b * B + ly)
            kk.append(c * B + lz)
        lev = np.concatenate(lv).astype(np.int64)
        ijk = np.stack([np.concatenate(ii), np.concatenate(jj),
                        np.concatenate(kk)], axis=1).astype(np.int64)
        sh = self.lmax - lev
        mk = morton3(ijk[:, 0] << sh, ijk[:, 1] << sh, ijk[:, 2] << sh, self.lmax)
        order = np.argsort(mk, kind="stable")
        self.morton = mk[order]
        self.level = lev[order]
        self.ijk = ijk[order]
        self.n = len(self.level)
        keys = cell_key(self.level, self.ijk[:, 0], self.ijk[:, 1], self.ijk[:, 2])
        self._korder = np.argsort(keys)
        self._ksorted = keys[self._korder]
        self._inner = None

    # ---------------------------------------------------------------- lookup
    def find(self, level, i, j, k):
        """Leaf index of cells (level, i, j, k), -1 where not a leaf."""
        level = np.asarray(level, dtype=np.int64)
        i = np.asarray(i, dtype=np.int64)
        j = np.asarray(j, dtype=np.int64)
        k = np.asarray(k, dtype=np.int64)
        n = np.left_shift(1, np.maximum(level, 0))
        ok = (level >= 0) & (i >= 0) & (j >= 0) & (k >= 0) & (i < n) & (j < n) & (k < n)
        key = cell_key(np.where(ok, level, 0), np.where(ok, i, 0),
                       np.where(ok, j, 0), np.where(ok, k, 0))
        pos = np.searchsorted(self._ksorted, key)
        pos = np.minimum(pos, len(self._ksorted) - 1)
        hit = ok & (self._ksorted[pos] == key)
        return np.where(hit, self._korder[pos], -1)

    def inner_keys(self, level):
        """Sorted keys of inner cells at ``level`` (ancestors of finer leaves)."""
        if self._inner is None:
            self._inner = {}
        if level not in self._inner:
            m = self.level > level
            s = self.level[m] - level
            ijk = self.ijk[m] >> s[:, None]
            keys = np.unique(cell_key(np.full(len(ijk), level), ijk[:, 0],
                                      ijk[:, 1], ijk[:, 2]))
            self._inner[level] = keys
        return self._inner[level]

    def is_inner(self, level, i, j, k):
        """Whether cells (level, i, j, k) (scalar level) are inner cells."""
        level = int(level)
        keys = self.inner_keys(level)
        key = cell_key(np.full(np.shape(i), level), i, j, k)
        if len(keys) == 0:
            return np.zeros(np.shape(key), dtype=bool)
        pos = np.minimum(np.searchsorted(keys, key), len(keys) - 1)
        return keys[pos] == key

    def volumes(self):
        return np.ldexp(1.0, -3 * self.level)
