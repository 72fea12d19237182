"""Pins of the oracle octree: exact tiling, 2:1 face balance, canonical order,
and the least balanced refinement checked against an independent dense
brute force on tiny inputs."""

import itertools

import numpy as np
import pytest

import problems
from oracle import octree as O

from oracle_fixtures import half_nodes, three_level_nodes


def dense_levels(spec):
    """Independent brute force: a dense array over the finest node grid holds
    the level of the covering leaf; refinement and balance act on it."""
    B = spec["node_size"]
    lmin, lmax = spec["min_level"], spec["max_level"]
    n = (1 << lmax) // B
    lev = np.full((n, n, n), lmin, dtype=np.int64)
    for l in range(lmin, lmax):
        s = 1 << (lmax - l)  # finest nodes per level-l node
        for a, b, c in itertools.product(range(n // s), repeat=3):
            blk = lev[a * s:(a + 1) * s, b * s:(b + 1) * s, c * s:(c + 1) * s]
            if blk[0, 0, 0] != l:
                continue
            lo, hi = O.node_box(l, a, b, c, B)
            if any(O.meets(p, lo, hi) for p in spec["prims"]):
                blk[...] = l + 1
    changed = True
    while changed:
        changed = False
        for ax in range(3):
            step = [0, 0, 0]
            step[ax] = 1
            for p in itertools.product(range(n), repeat=3):
                q = (p[0] + step[0], p[1] + step[1], p[2] + step[2])
                if q[ax] >= n:
                    continue
                # re-read the current levels: earlier splits may have acted
                for a, b in ((p, q), (q, p)):
                    if lev[b] - lev[a] >= 2:
                        l = lev[a]
                        s = 1 << (lmax - l)
                        c0 = [(x // s) * s for x in a]
                        lev[c0[0]:c0[0] + s, c0[1]:c0[1] + s, c0[2]:c0[2] + s] = l + 1
                        changed = True
    return lev


def node_set_to_dense(nodes, lmax, B):
    n = (1 << lmax) // B
    lev = np.zeros((n, n, n), dtype=np.int64)
    for (l, a, b, c) in nodes:
        s = 1 << (lmax - l)
        lev[a * s:(a + 1) * s, b * s:(b + 1) * s, c * s:(c + 1) * s] = l
    return lev


TINY_SPECS = [
    {"min_level": 3, "max_level": 6, "node_size": 4,
     "prims": [problems.sphere_prim((0.31, 0.52, 0.47), 0.2, 0.0)]},
    {"min_level": 2, "max_level": 6, "node_size": 4,
     "prims": [problems.sphere_prim((0.1, 0.1, 0.1), 0.05, 0.0)]},
    {"min_level": 3, "max_level": 6, "node_size": 4,
     "prims": [problems.box_prim((0.3, 0.2, 0.26), (0.61, 0.44, 0.9))]},
    {"min_level": 2, "max_level": 5, "node_size": 4,
     "prims": [problems.sphere_prim((0.5, 0.5, 0.5), 0.3, 0.1)]},
]


@pytest.mark.parametrize("spec", TINY_SPECS)
def test_least_balanced_refinement_matches_dense_brute_force(spec):
    nodes = O.refine_nodes(spec)
    got = node_set_to_dense(nodes, spec["max_level"], spec["node_size"])
    want = dense_levels(spec)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("spec", TINY_SPECS)
def test_balance_is_order_independent(spec):
    base = O.refine_nodes(spec)
    # undo balance: predicate refinement only, then balance in shuffled orders
    B = spec["node_size"]
    lmin, lmax = spec["min_level"], spec["max_level"]
    n0 = (1 << lmin) // B
    leaves = {(lmin, a, b, c) for a in range(n0) for b in range(n0) for c in range(n0)}
    for lev in range(lmin, lmax):
        for node in sorted(x for x in leaves if x[0] == lev):
            lo, hi = O.node_box(*node, B)
            if any(O.meets(p, lo, hi) for p in spec["prims"]):
                leaves.remove(node)
                leaves.update(O.children(node))
    for seed in (1, 2, 3):
        assert O.balance(leaves, lmin, B, order=seed) == base


def _check_tree(T):
    # exact tiling of the unit cube
    vol = np.ldexp(1.0, -3 * T.level)
    assert vol.sum() == 1.0
    # canonical order: strictly increasing Morton keys of the min corners
    assert np.all(np.diff(T.morton.astype(np.float64)) > 0)
    # 2:1 face balance over every face-neighbour pair (brute force lookup)
    for d in range(6):
        dv = np.array(O.DIRS[d])
        nb = T.ijk + dv
        n = np.left_shift(1, T.level)
        inside = np.all((nb >= 0) & (nb < n[:, None]), axis=1)
        found = np.zeros(T.n, dtype=bool)
        for dl in (-1, 0):
            l2 = T.level + dl
            j = T.find(l2, nb[:, 0] >> -dl, nb[:, 1] >> -dl, nb[:, 2] >> -dl)
            found |= j >= 0
        # otherwise the neighbour region is covered by level+1 leaves
        fine = T.find(T.level + 1, 2 * nb[:, 0], 2 * nb[:, 1], 2 * nb[:, 2])
        found |= fine >= 0
        assert np.all(found | ~inside)


@pytest.mark.parametrize("cfg", [1, 2])
def test_config_trees_tile_and_balance(cfg):
    T = O.Octree(problems.config_spec(cfg))
    _check_tree(T)


def test_small_cut_cell_family_tree():
    T = O.Octree(problems.config_spec(3, min_level=4, max_level=7))
    _check_tree(T)


def test_three_level_tree_and_half_tree():
    spec = {"min_level": 3, "max_level": 5, "node_size": 4, "prims": []}
    T = O.Octree(spec, three_level_nodes(3))
    _check_tree(T)
    assert set(np.unique(T.level)) == {3, 4, 5}
    spec = {"min_level": 3, "max_level": 4, "node_size": 4, "prims": []}
    _check_tree(O.Octree(spec, half_nodes(3)))


def test_morton_key_definition():
    # x in the least significant interleaved bit: (1,0,0)->1, (0,1,0)->2,
    # (0,0,1)->4, (2,0,0)->8
    got = O.morton3(np.array([1, 0, 0, 2, 3]), np.array([0, 1, 0, 0, 3]),
                    np.array([0, 0, 1, 0, 3]), 4)
    assert list(got) == [1, 2, 4, 8, 63]


def test_sphere_predicate_special_cases():
    p = problems.sphere_prim((0.5, 0.5, 0.5), 0.25, 0.0)
    # box containing the sphere entirely: meets the surface
    assert O.sphere_meets(p, (0, 0, 0), (1, 1, 1))
    # box strictly inside the sphere: does not meet the surface
    assert not O.sphere_meets(p, (0.45, 0.45, 0.45), (0.55, 0.55, 0.55))
    # box touching the surface at a single point (closed-box rule)
    assert O.sphere_meets(p, (0.75, 0.4, 0.4), (0.8, 0.6, 0.6))
    assert not O.sphere_meets(p, (0.7500001, 0.4, 0.4), (0.8, 0.6, 0.6))
    b = problems.box_prim((0.25, 0.25, 0.25), (0.5, 0.5, 0.5))
    assert O.box_meets_surface(b, (0.5, 0.3, 0.3), (0.6, 0.4, 0.4))  # touches face
    assert not O.box_meets_surface(b, (0.3, 0.3, 0.3), (0.4, 0.4, 0.4))  # inside
    assert not O.box_meets_surface(b, (0.6, 0.3, 0.3), (0.7, 0.4, 0.4))  # outside
