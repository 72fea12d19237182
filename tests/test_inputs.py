"""The seeded input generators (problems/) give the same inputs whatever the
integer type of the level and index arrays: the library's leaf and face
arrays are uint8 / int8 / uint32, the oracle's int64."""

import numpy as np

import problems
from oracle import discretize as D
from oracle import octree as O


def test_manufactured_rhs_independent_of_index_dtypes():
    """Config 1 (all-Dirichlet walls, wall values folded into the RHS) from
    uint8 levels, int8 directions and uint32 indices equals the int64 one."""
    spec = problems.config_spec(1)
    bc, theta = problems.config_bc(1)
    T = O.Octree(spec)
    d = D.Discretization(T, None, bc, theta)
    beta = problems.face_beta(1, d.face_level, d.face_ijk, d.face_dir)
    ref = problems.rhs_manufactured(1, T.level, T.ijk, d.face_owner, d.face_level, d.face_ijk,
                                    d.face_dir, d.face_other, beta, bc, theta)
    small = problems.rhs_manufactured(
        1, np.asarray(T.level, np.uint8), np.asarray(T.ijk, np.uint32), d.face_owner,
        np.asarray(d.face_level, np.uint8), np.asarray(d.face_ijk, np.uint32),
        np.asarray(d.face_dir, np.int8), d.face_other, beta, bc, theta)
    assert np.array_equal(small, ref)
    # the integrated RHS of a unit-scale solution is O(h^3) (h = 1/32) plus
    # the O(h^2) wall terms
    assert np.abs(ref).max() < 1e-2


def test_random_rhs_and_beta_independent_of_index_dtypes():
    spec = problems.config_spec(3, 3, 5)
    T = O.Octree(spec)
    d = D.Discretization(T, None, (0, 0, 0, 1, 0, 0), 0.5)
    r64 = problems.rhs_random(3, T.level, T.ijk)
    r8 = problems.rhs_random(3, np.asarray(T.level, np.uint8), np.asarray(T.ijk, np.uint32))
    assert np.array_equal(r8, r64)
    b64 = problems.face_beta(3, d.face_level, d.face_ijk, d.face_dir)
    b8 = problems.face_beta(3, np.asarray(d.face_level, np.uint8),
                            np.asarray(d.face_ijk, np.uint32), np.asarray(d.face_dir, np.int8))
    assert np.array_equal(b8, b64)
