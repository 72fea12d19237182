"""Pressure projection around the solve (test infrastructure).

Paper passages restated here
  * Section 2.1: the pressure equation -lap p = b with b = div u; integrated
    over a leaf cell both sides become sums of face fluxes (Eq. 2), each
    weighted by the fluid area of its face; the pressure gradient is taken
    at face centres.
  * Section 4.4 (static projection test): a velocity field is made
    divergence free by solving for p and applying the pressure gradient to
    the face velocities; the quality measure is the volume-weighted RMS of
    the divergence of the result (RMS_V, Section 4.2).

Readings (the paper states no formulas for these steps)
  * Velocities are MAC normal components u_f on the canonical faces, along
    the + axis of the face's axis.  A face's fluid area is beta_f S_f: the
    same beta_f that weights its operator coefficient, S_f = h^2 of the
    face's owner (the finer side).
  * div_i = sum over the faces of leaf i of s beta_f S_f u_f, s = +1 where
    the + axis points out of leaf i: the integrated divergence (net outflow).
  * The pressure flux through a face is the operator's own: with
    (A p)_i = sum over the faces of i of (+F_f for the owner, -F_f for the
    other side),
      F_f = k_f (p_o - p_t)                 same level,
      F_f = k_f (mean_P(p) - p_t) / 2       T-junction (o the fine owner,
                                            mean over o's active siblings),
      F_f = k_f p_o                         Dirichlet wall,
      F_f = 0                               Neumann wall,
    k_f = beta_f S_f / h (S_f / (theta h) at a Dirichlet wall), F_f = 0 when
    a side is inactive.  The update u_f <- u_f - s_o F_f / (beta_f S_f)
    (faces with beta_f = 0 keep u_f) then gives div(u_new) = div(u) - A p,
    so the solution of A p = div(u) leaves exactly the solver's residual as
    the divergence.
  * RMS_V(d) = sqrt(sum_i V_i d_i^2 / sum_i V_i) over the active leaves with
    d_i = div_i / V_i and V_i = h_i^3.
"""

import numpy as np

from .discretize import COARSE, DIRICHLET, NEUMANN, SAME, WALL


def _outward(face_dir):
    """s of the owner: +1 where the face's + axis points out of the owner."""
    return np.where(np.asarray(face_dir) & 1, 1.0, -1.0)


def face_area(disc):
    """Full face area S_f = h^2 of the owner."""
    h = np.ldexp(1.0, -disc.face_level.astype(np.int64))
    return h * h


def divergence(disc, beta, u):
    """Integrated divergence of the face velocities u (canonical face order)
    for every leaf: the fluxes s beta_f S_f u_f summed over its faces."""
    beta = np.asarray(beta, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    flux = beta * face_area(disc) * u
    s = _outward(disc.face_dir)
    div = np.zeros(disc.tree.n)
    for f in range(disc.n_faces):
        div[disc.face_owner[f]] += s[f] * flux[f]
        if disc.face_kind[f] != WALL:
            div[disc.face_other[f]] -= s[f] * flux[f]
    return div


def pressure_flux(disc, p):
    """F_f of the operator A (with its current beta) applied to p, per face."""
    p = np.asarray(p, dtype=np.float64)
    T = disc.tree
    act = disc.active
    k = disc.kf
    F = np.zeros(disc.n_faces)
    for f in range(disc.n_faces):
        o, t, kind, d = disc.face_owner[f], disc.face_other[f], disc.face_kind[f], disc.face_dir[f]
        if not act[o]:
            continue
        if kind == WALL:
            if disc.bc[d] == DIRICHLET:
                F[f] = k[f] * p[o]
            continue
        if not act[t]:
            continue
        if kind == SAME:
            F[f] = k[f] * (p[o] - p[t])
        elif kind == COARSE:
            ch = disc.children_of(T.level[o] - 1, T.ijk[o] >> 1)[0]
            a = act[ch]
            pbar = p[ch][a].sum() / a.sum()
            F[f] = k[f] * (pbar - p[t]) / 2.0
    return F


def project(disc, beta, u, p):
    """u_f - s_o F_f / (beta_f S_f) on faces with beta_f > 0."""
    beta = np.asarray(beta, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64).copy()
    F = pressure_flux(disc, p)
    s = _outward(disc.face_dir)
    w = beta * face_area(disc)
    on = w > 0.0
    u[on] -= s[on] * F[on] / w[on]
    return u


def rms_divergence(disc, div):
    """Volume-weighted RMS over the active leaves of div_i / V_i."""
    T = disc.tree
    V = np.ldexp(1.0, -3 * T.level.astype(np.int64))
    act = disc.active
    d = np.asarray(div)[act] / V[act]
    return float(np.sqrt((V[act] * d * d).sum() / V[act].sum()))


def tank_velocity(disc, value=-1.0, axis=1):
    """The static test's initial field: u = value along ``axis`` on every
    face of that axis, zero on the others; zero on Neumann wall faces (solid
    walls), left as is on Dirichlet (open) wall faces."""
    d = disc.face_dir
    u = np.where((d >> 1) == axis, float(value), 0.0)
    wall = disc.face_kind == WALL
    u[wall & (disc.bc[d] == NEUMANN)] = 0.0
    return u
