"""Pins of the oracle's projection wrapper (oracle/projection.py) against the
oracle's independently assembled operator, conservation, and closed forms."""

import numpy as np
import pytest

import problems
from oracle import discretize as D
from oracle import octree as O
from oracle import projection as PJ


def _adaptive_cut(bc=(0, 0, 0, 1, 0, 0)):
    """Cut-cell sphere on a 3..5 octree (T-junctions, partial faces)."""
    spec = problems.config_spec(3, 3, 5)
    T = O.Octree(spec)
    disc = D.Discretization(T, None, bc, 0.5)
    beta = problems.face_beta(3, disc.face_level, disc.face_ijk, disc.face_dir)
    disc.set_beta(beta)
    return disc, beta


def test_update_removes_exactly_the_operator():
    """div(u - s F / (beta S)) = div(u) - A p for arbitrary u and p, with A
    the composite CSR (T-junction rows included): the face fluxes are the
    operator's."""
    disc, beta = _adaptive_cut()
    assert (disc.face_kind == D.COARSE).any()
    rng = np.random.default_rng(70)
    u = rng.uniform(-1, 1, disc.n_faces)
    p = np.where(disc.active, rng.uniform(-1, 1, disc.tree.n), 0.0)
    lhs = PJ.divergence(disc, beta, PJ.project(disc, beta, u, p))
    rhs = PJ.divergence(disc, beta, u) - disc.A @ p
    act = disc.active
    scale = np.abs(disc.A @ p).max()
    assert np.abs(lhs[act] - rhs[act]).max() <= 1e-12 * scale


def test_divergence_conserves():
    """Interior fluxes cancel: the leaf divergences add up to the net flux
    through the domain walls."""
    disc, beta = _adaptive_cut()
    rng = np.random.default_rng(71)
    u = rng.uniform(-1, 1, disc.n_faces)
    div = PJ.divergence(disc, beta, u)
    wall = disc.face_kind == D.WALL
    s = np.where(disc.face_dir & 1, 1.0, -1.0)
    net = (s * beta * PJ.face_area(disc) * u)[wall].sum()
    assert abs(div.sum() - net) <= 1e-12 * np.abs(div).sum()


def test_uniform_tank_closed_form():
    """Uniform 16^3 tank, solid bottom and sides, open top, u = (0, -1, 0):
    only the bottom layer has divergence, -h^2 per leaf (inflow from above,
    none through the floor)."""
    T = O.Octree(problems.uniform_spec(4))
    bc = (0, 0, 0, 1, 0, 0)
    disc = D.Discretization(T, None, bc, 0.5)
    beta = np.ones(disc.n_faces)
    disc.set_beta(beta)
    u = PJ.tank_velocity(disc)
    div = PJ.divergence(disc, beta, u)
    h = 1.0 / 16
    bottom = T.ijk[:, 1] == 0
    assert np.all(div[bottom] == -h * h)
    assert np.all(div[~bottom] == 0.0)


@pytest.mark.parametrize("cut", [False, True])
def test_projection_with_an_exact_solve(cut):
    """Solve A p = div(u) directly: the projected field is divergence free
    to rounding; in the uniform tank it is exactly at rest (the pressure
    gradient cancels the downward flow everywhere)."""
    import scipy.sparse.linalg as sla
    bc = (0, 0, 0, 1, 0, 0)
    if cut:
        disc, beta = _adaptive_cut(bc)
    else:
        T = O.Octree(problems.uniform_spec(4))
        disc = D.Discretization(T, None, bc, 0.5)
        beta = np.ones(disc.n_faces)
        disc.set_beta(beta)
    u = PJ.tank_velocity(disc)
    div = PJ.divergence(disc, beta, u)
    act = disc.active
    A = disc.A[act][:, act].tocsc()
    p = np.zeros(disc.tree.n)
    p[act] = sla.spsolve(A, div[act])
    un = PJ.project(disc, beta, u, p)
    dn = PJ.divergence(disc, beta, un)
    assert np.abs(dn[act]).max() <= 1e-12 * np.abs(div).max()
    assert PJ.rms_divergence(disc, dn) <= 1e-11 * PJ.rms_divergence(disc, div)
    if not cut:
        assert np.abs(un).max() <= 1e-12


def test_rms_divergence_closed_form():
    """RMS_V of div_i = c V_i is |c| on any grid."""
    disc, beta = _adaptive_cut()
    V = np.ldexp(1.0, -3 * disc.tree.level.astype(np.int64))
    assert PJ.rms_divergence(disc, -2.5 * V) == pytest.approx(2.5, rel=1e-14)


@pytest.mark.parametrize("obstacle", ["sphere", "star"])
def test_static_tank_with_obstacle_is_hydrostatic(obstacle):
    """The static projection test (Section 4.4) on a small adaptive grid:
    tank with solid floor and sides, open top, a solid sphere or star at the
    centre, u = (0, -1, 0).  The continuum solution is hydrostatic: p linear
    in y with p = 0 at the top, and the projected fluid at rest.  Linear
    fields are reproduced exactly by the discretisation (Eq. 3 on cut faces,
    whatever their fractions; the Eq. (10) ghost at T-junctions; the wall at
    the face for the Dirichlet top), so the direct solve of A p = div(u)
    gives p_i = y_i - 1 at every active cell centre and the projected face
    velocities vanish on every fluid face: the divergence left after an
    exact projection is zero at any resolution."""
    import scipy.sparse.linalg as sla
    spec = problems.tank_spec(3, obstacle)
    T = O.Octree(spec)
    bc, theta = problems.tank_bc()
    disc = D.Discretization(T, None, bc, theta)
    beta = problems.tank_beta(obstacle, disc.face_level, disc.face_ijk, disc.face_dir)
    disc.set_beta(beta)
    act = disc.active
    assert (disc.face_kind == D.COARSE).any() and ((beta > 0) & (beta < 1)).any()
    assert (~act).any()
    u = problems.tank_velocity(disc.face_dir, disc.face_kind, bc)
    assert np.array_equal(u, PJ.tank_velocity(disc))
    div = PJ.divergence(disc, beta, u)
    A = disc.A[act][:, act].tocsc()
    p = np.zeros(T.n)
    p[act] = sla.spsolve(A, div[act])
    y = (T.ijk[:, 1] + 0.5) * np.ldexp(1.0, -T.level.astype(np.int64))
    assert np.abs(p[act] - (y[act] - 1.0)).max() <= 1e-12
    un = PJ.project(disc, beta, u, p)
    assert np.abs(un[beta > 0]).max() <= 1e-11
