"""Pins of the oracle adjoint: A^T = A without T-junctions, the per-face
gradient against dense dA/dbeta, and central finite differences computed as
difference solves."""

import numpy as np
import pytest

import problems
from oracle import discretize as D
from oracle import krylov as K
from oracle import octree as O

from oracle_fixtures import config_problem, disc_for, half_tree, hierarchy


def test_adjoint_equals_forward_without_tjunctions():
    d = disc_for(O.Octree(problems.uniform_spec(4)), seed=30)
    H = hierarchy(d)
    g = np.random.default_rng(31).uniform(-1, 1, d.tree.n)
    lam, _ = K.pcg(d.A.T.tocsr(), g, H.vcycle, 1e-13, 100)
    p, _ = K.pcg(d.A, g, H.vcycle, 1e-13, 100)
    assert np.linalg.norm(lam - p) <= 1e-11 * np.linalg.norm(p)


def test_face_gradient_against_dense_dA():
    """A is linear in beta: A(beta + e_f) - A(beta) is dA/dbeta_f exactly (no
    activity change), so -lam^T (dA/dbeta_f) p checks every face formula
    (same level, T sub-face, Dirichlet and Neumann walls)."""
    bc = (D.NEUMANN, D.DIRICHLET, D.NEUMANN, D.DIRICHLET, D.NEUMANN, D.NEUMANN)
    d = disc_for(half_tree(3), bc=bc, seed=32)
    rng = np.random.default_rng(33)
    lam = rng.uniform(-1, 1, d.tree.n)
    p = rng.uniform(-1, 1, d.tree.n)
    g = d.face_gradient(lam, p)
    base = d.A.copy()
    beta = d.beta.copy()
    for f in range(d.n_faces):
        bb = beta.copy()
        bb[f] += 1.0
        d2 = D.Discretization(d.tree, bb, bc, d.theta)
        dA = d2.A - base
        want = -lam @ (dA @ p)
        assert abs(g[f] - want) <= 1e-12 * (1 + abs(want)), (f, d.face_kind[f])
    assert (d.face_kind == D.COARSE).sum() > 0


def test_adjoint_gradient_matches_difference_solve_fd():
    """Central FD (eps = 1e-6) of L = ||p - p_t||^2 on 20 seeded faces of a
    small member of the cut-cell family, as difference solves."""
    T, d, beta, rhs = config_problem(3, min_level=3, max_level=5)
    bc, th = problems.config_bc(3)
    H = hierarchy(d)
    p, info = K.pcg(d.A, rhs, H.vcycle, 1e-13, 300, active=d.active)
    pt = problems.adjoint_target(T.level, T.ijk, np.abs(p).max())

    def lgrad(x):
        return np.where(d.active, 2.0 * (x - pt), 0.0)
    _, lam, g, _, ainfo = K.solve_and_grad(d, H, rhs, lgrad, rtol=1e-13, max_iter=300)
    assert ainfo["status"] == 0
    special = np.nonzero((d.face_kind == D.COARSE) | (beta < 1))[0]
    both = d.active[d.face_owner] & ((d.face_other < 0) | d.active[np.maximum(d.face_other, 0)])
    special = np.intersect1d(special, np.nonzero(both)[0])
    faces = problems.sample_faces(d.n_faces, special, count=20, pool=np.nonzero(both)[0])
    assert len(faces) == 20 and np.all(both[faces])

    def factory(bb):
        dd = D.Discretization(T, None, bc, th)
        dd.set_beta(bb)
        return dd
    fd, steps = K.fd_gradient(factory, beta, p, pt, faces, eps=1e-6, rtol=1e-13,
                              precond_factory=lambda dd: hierarchy(dd).vcycle, rhs=rhs,
                              return_steps=True)
    ga = g[faces]
    denom = np.maximum(np.abs(fd), 1e-8 * np.abs(fd).max())
    err = np.max(np.abs(ga - fd) / denom)
    reduced = int((steps < 1e-6).sum())
    print(f"  FD on {len(faces)} faces: max rel err {err:.2e}; {reduced} faces took a step "
          f"below 1e-6 (smallest {steps.min():.2e})")
    assert err <= 1e-6
