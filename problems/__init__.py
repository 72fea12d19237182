"""Seeded synthetic problem generators for the octree Poisson solver.

This module defines *problem inputs* only: refinement specifications, solid
geometry (signed distance functions), face fluid fractions, per-face
coefficients beta, boundary-condition flags and right-hand sides.  It holds
none of the solver's arithmetic (no coefficients, operators, cycles or
Krylov steps) and it is shared by the CPU oracle and by the GPU library's
callers, which is the only code the two sides share.

Workloads (all on the unit cube, cell level l means 2^l cells per axis):

  1  uniform 32^3 (level 5), beta = 1, Dirichlet p = 0 on every wall,
     manufactured p = sin(pi x) sin(pi y) sin(pi z).
  2  adaptive levels 5..7, refined within 0.1 of the sphere |x-c| = 0.3,
     c = (1/2,1/2,1/2); beta = 1; Dirichlet walls carrying the exact
     p = exp(-20 |x-c|^2).
  3  cut-cell adaptive levels 6..9 refined where a node touches the solid
     sphere |x-c| = 0.2; beta = fluid face fraction with 1% seeded jitter;
     Neumann walls and solid, Dirichlet on the top wall y = 1; seeded
     uniform random divergence made volume-mean free.
  4  large adaptive levels 7..10 refined where a node touches one of 8
     seeded spheres (r in [0.05, 0.15]) or the surface of a solid box;
     beta, boundary conditions and RHS as in 3.
  5  adjoint on the octree of 3: loss ||p - p_t||^2 with p_t a seeded sum
     of 4 Gaussians; 50 seeded faces for finite-difference checks.

The refinement rule follows the paper's grid generator (a tile meeting the
surface takes the finest level, Section 4.1) at the granularity of 4^3-cell
nodes.  Face fractions reconstruct the interface from the signed distance at
face corners (cut-cell method, Section 4.4).
"""

import math

import numpy as np

SPHERE = 0
BOX = 1

NEUMANN = 0
DIRICHLET = 1

NODE_SIZE = 4


# --------------------------------------------------------------------------
# refinement specifications


def sphere_prim(center, radius, band=0.0):
    return {"kind": SPHERE, "center": tuple(float(v) for v in center),
            "radius": float(radius), "band": float(band),
            "lo": (0.0, 0.0, 0.0), "hi": (0.0, 0.0, 0.0)}


def box_prim(lo, hi):
    return {"kind": BOX, "center": (0.0, 0.0, 0.0), "radius": 0.0,
            "band": 0.0, "lo": tuple(float(v) for v in lo),
            "hi": tuple(float(v) for v in hi)}


def uniform_spec(level):
    return {"min_level": level, "max_level": level, "node_size": NODE_SIZE,
            "prims": []}


def config4_geometry(seed=1004):
    """Eight refinement spheres and the solid box of workload 4."""
    rng = np.random.default_rng(seed)
    centers = rng.uniform(0.15, 0.85, size=(8, 3))
    radii = rng.uniform(0.05, 0.15, size=8)
    shift = 1.0 / 3072.0
    lo = (0.35 + shift, 0.10 + shift, 0.35 + shift)
    hi = (0.65 + shift, 0.35 + shift, 0.65 + shift)
    return centers, radii, lo, hi


def config_spec(cfg, min_level=None, max_level=None):
    """Refinement specification of workload ``cfg`` (1..5).

    ``min_level``/``max_level`` override the level range to build smaller
    members of the same family (same geometry, coarser levels).
    """
    if cfg == 1:
        lo, hi, prims = 5, 5, []
    elif cfg == 2:
        lo, hi = 5, 7
        prims = [sphere_prim((0.5, 0.5, 0.5), 0.3, 0.1)]
    elif cfg in (3, 5):
        lo, hi = 6, 9
        prims = [sphere_prim((0.5, 0.5, 0.5), 0.2, 0.0)]
    elif cfg == 4:
        lo, hi = 7, 10
        centers, radii, blo, bhi = config4_geometry()
        prims = [sphere_prim(c, r, 0.0) for c, r in zip(centers, radii)]
        prims.append(box_prim(blo, bhi))
    else:
        raise ValueError(f"unknown workload {cfg}")
    if min_level is not None:
        lo = min_level
    if max_level is not None:
        hi = max_level
    return {"min_level": lo, "max_level": hi, "node_size": NODE_SIZE,
            "prims": prims}


# --------------------------------------------------------------------------
# solid geometry: signed distance, positive in the fluid


def solid_sdf(cfg):
    """Signed distance function of the solid of workload ``cfg`` or None."""
    if cfg in (3, 5):
        def phi(x, y, z):
            return np.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2) - 0.2
        return phi
    if cfg == 4:
        _, _, lo, hi = config4_geometry()
        c = [(lo[a] + hi[a]) * 0.5 for a in range(3)]
        h = [(hi[a] - lo[a]) * 0.5 for a in range(3)]

        def phi(x, y, z):
            qx = np.abs(x - c[0]) - h[0]
            qy = np.abs(y - c[1]) - h[1]
            qz = np.abs(z - c[2]) - h[2]
            outside = np.sqrt(np.maximum(qx, 0.0) ** 2 + np.maximum(qy, 0.0) ** 2
                              + np.maximum(qz, 0.0) ** 2)
            inside = np.minimum(np.maximum(qx, np.maximum(qy, qz)), 0.0)
            return outside + inside
        return phi
    return None


# --------------------------------------------------------------------------
# static projection test (tank with an obstacle, Section 4.4)


def obstacle_level_set(name):
    """Level set of the obstacle of the static projection test, positive in
    the fluid: the sphere |x - c| - 0.25 or the star
    r - (0.237 + 0.079 cos(6 theta) cos(6 phi)) about c = (1/2, 1/2, 1/2)
    (Section 4.1), theta the polar angle from +z and phi the azimuth in the
    x-y plane.  The sphere's is a signed distance; the star's is not."""
    if name == "sphere":
        def phi(x, y, z):
            return np.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2) - 0.25
        return phi, True
    if name == "star":
        def phi(x, y, z):
            dx, dy, dz = x - 0.5, y - 0.5, z - 0.5
            r = np.sqrt(dx * dx + dy * dy + dz * dz)
            theta = np.arccos(np.clip(dz / np.maximum(r, 1e-300), -1.0, 1.0))
            az = np.arctan2(dy, dx)
            return r - (0.237 + 0.079 * np.cos(6.0 * theta) * np.cos(6.0 * az))
        return phi, False
    raise ValueError(name)


def tank_spec(root_level, obstacle):
    """Octree of the static projection test: root cells of level root_level,
    two levels finer where a 4^3 node meets the obstacle's surface (the
    sphere of radius 1/4), or, for the star, the spherical shell
    0.158 <= |x - c| <= 0.316 that contains its surface (the refinement
    predicates are closed-form tests on node boxes)."""
    if obstacle == "sphere":
        prim = sphere_prim((0.5, 0.5, 0.5), 0.25, 0.0)
    elif obstacle == "star":
        prim = sphere_prim((0.5, 0.5, 0.5), 0.237, 0.079)
    else:
        raise ValueError(obstacle)
    return {"min_level": root_level, "max_level": root_level + 2, "node_size": NODE_SIZE,
            "prims": [prim]}


def tank_bc():
    """Solid floor and sides (Neumann), open top y = 1 (Dirichlet p = 0 on
    the face)."""
    return [NEUMANN, NEUMANN, NEUMANN, DIRICHLET, NEUMANN, NEUMANN], 0.5


def tank_beta(obstacle, face_level, face_ijk, face_dir):
    """Fluid face fractions of the obstacle (no jitter)."""
    phi, is_sdf = obstacle_level_set(obstacle)
    return face_fractions(face_level, face_ijk, face_dir, phi, lipschitz=is_sdf)


def tank_velocity(face_dir, face_kind, bc):
    """MAC face velocities of the uniform downward flow (0, -1, 0): -1 on
    faces normal to y, 0 on the others and on solid (Neumann) walls."""
    d = np.asarray(face_dir)
    u = np.where((d >> 1) == 1, -1.0, 0.0)
    u[(np.asarray(face_kind) == 0) & (np.asarray(bc)[d] == NEUMANN)] = 0.0
    return u


def _triangle_positive_fraction(a, b, c):
    """Fraction of a triangle on which the linear interpolant of the vertex
    values (a, b, c) is strictly positive (vectorised, exact)."""
    v = np.stack([a, b, c], axis=-1)
    npos = (v > 0).sum(axis=-1)
    out = np.zeros(v.shape[:-1])
    out[npos == 3] = 1.0
    s = np.sort(v, axis=-1)  # ascending
    # one positive vertex p, two non-positive q, r: (p^2)/((p-q)(p-r))
    one = npos == 1
    if np.any(one):
        p, q, r = s[one, 2], s[one, 0], s[one, 1]
        out[one] = p * p / ((p - q) * (p - r))
    # two positive: 1 - n^2 / ((n-p)(n-q)) with n the non-positive vertex
    two = npos == 2
    if np.any(two):
        n, p, q = s[two, 0], s[two, 1], s[two, 2]
        out[two] = 1.0 - n * n / ((n - p) * (n - q))
    return out


def face_corners(level, ijk, direction):
    """Corner coordinates (4, F, 3) of leaf faces in the order
    (lo,lo), (hi,lo), (hi,hi), (lo,hi) of the two in-plane axes."""
    level = np.asarray(level, dtype=np.int64)
    ijk = np.asarray(ijk, dtype=np.int64).reshape(-1, 3)
    direction = np.asarray(direction, dtype=np.int64)
    h = np.ldexp(1.0, -level)
    axis = direction // 2
    side = direction % 2
    F = len(level)
    base = ijk.astype(np.float64) * h[:, None]
    corners = np.empty((4, F, 3))
    ax_u = np.where(axis == 0, 1, 0)
    ax_v = np.where(axis == 2, 1, 2)
    rows = np.arange(F)
    for n, (du, dv) in enumerate(((0, 0), (1, 0), (1, 1), (0, 1))):
        p = base.copy()
        p[rows, axis] = base[rows, axis] + side * h
        p[rows, ax_u] = base[rows, ax_u] + du * h
        p[rows, ax_v] = base[rows, ax_v] + dv * h
        corners[n] = p
    return corners


def face_fractions(level, ijk, direction, sdf, chunk=1 << 21, lipschitz=True):
    """Fluid fraction of each face: the face square is split along its
    (lo,lo)-(hi,hi) diagonal into two triangles; on each, the signed
    distance is interpolated linearly from its corners and the area where
    it is positive is measured exactly.

    A signed distance is 1-Lipschitz, so a face whose centre lies farther
    than its half-diagonal (h / sqrt 2) from the interface has four corners
    of one sign: its fraction is exactly 1 or 0 and its corners are not
    evaluated.  For a level set that is not a distance (lipschitz=False)
    every face's corners are evaluated."""
    level = np.asarray(level)
    F = len(level)
    out = np.ones(F)
    if sdf is None or F == 0:
        return out
    ijk = np.asarray(ijk).reshape(-1, 3)
    direction = np.asarray(direction)
    for s in range(0, F, chunk):
        e = min(F, s + chunk)
        lv = np.asarray(level[s:e], dtype=np.int64)
        h = np.ldexp(1.0, -lv)
        d = np.asarray(direction[s:e], dtype=np.int64)
        ctr = (np.asarray(ijk[s:e], dtype=np.float64) + 0.5) * h[:, None]
        rows = np.arange(e - s)
        ctr[rows, d // 2] += (d % 2 - 0.5) * h
        pc = sdf(ctr[:, 0], ctr[:, 1], ctr[:, 2])
        far = (np.abs(pc) > 0.7072 * h) if lipschitz else np.zeros(len(pc), dtype=bool)
        res = np.where(pc > 0, 1.0, 0.0)
        near = np.nonzero(~far)[0]
        if len(near):
            cs = face_corners(lv[near], np.asarray(ijk[s:e])[near], d[near])
            ph = [sdf(cs[n, :, 0], cs[n, :, 1], cs[n, :, 2]) for n in range(4)]
            t1 = _triangle_positive_fraction(ph[0], ph[1], ph[2])
            t2 = _triangle_positive_fraction(ph[0], ph[2], ph[3])
            res[near] = 0.5 * (t1 + t2)
        out[s:e] = res
    return out


def jittered_beta(frac, seed, amplitude=0.01):
    """beta_f = min(1, frac_f (1 + amplitude u_f)), u_f ~ U[-1, 1] drawn in
    canonical face order; faces with zero fraction stay zero."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.0, 1.0, size=len(frac))
    return np.minimum(1.0, frac * (1.0 + amplitude * u))


def config_bc(cfg):
    """(bc[6], theta): per domain wall -x,+x,-y,+y,-z,+z."""
    if cfg in (1, 2):
        return [DIRICHLET] * 6, 0.5
    if cfg in (3, 4, 5):
        return [NEUMANN, NEUMANN, NEUMANN, DIRICHLET, NEUMANN, NEUMANN], 0.5
    raise ValueError(cfg)


def config_seed(cfg):
    return 1000 + cfg


# --------------------------------------------------------------------------
# face coefficients and right-hand sides


def face_beta(cfg, face_level, face_ijk, face_dir):
    """Per-face beta in canonical face order for workload ``cfg``."""
    sdf = solid_sdf(cfg)
    if sdf is None:
        return np.ones(len(face_level))
    frac = face_fractions(face_level, face_ijk, face_dir, sdf)
    return jittered_beta(frac, config_seed(cfg))


def manufactured(cfg):
    """(p, laplacian p) of the manufactured solution of workload 1 or 2."""
    if cfg == 1:
        def p(x, y, z):
            return np.sin(math.pi * x) * np.sin(math.pi * y) * np.sin(math.pi * z)

        def lap(x, y, z):
            return -3.0 * math.pi ** 2 * p(x, y, z)
        return p, lap
    if cfg == 2:
        def p(x, y, z):
            r2 = (x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2
            return np.exp(-20.0 * r2)

        def lap(x, y, z):
            r2 = (x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2
            return (1600.0 * r2 - 120.0) * np.exp(-20.0 * r2)
        return p, lap
    raise ValueError(cfg)


def cell_centers(level, ijk):
    h = np.ldexp(1.0, -np.asarray(level, dtype=np.int64))
    ijk = np.asarray(ijk, dtype=np.float64).reshape(-1, 3)
    return (ijk + 0.5) * h[:, None], h


def rhs_manufactured(cfg, leaf_level, leaf_ijk, face_owner=None,
                     face_level=None, face_ijk=None, face_dir=None,
                     face_other=None, face_beta_=None, bc=None, theta=0.5):
    """Integrated RHS rhs_i = -lap p(x_i) h_i^3 for the PDE
    div(grad p) = lap p, plus, for inhomogeneous Dirichlet walls, the wall
    value folded in with the ghost-fluid wall coefficient beta S / (theta h)
    (wall at the face, p given at the face centre)."""
    p, lap = manufactured(cfg)
    x, h = cell_centers(leaf_level, leaf_ijk)
    rhs = -lap(x[:, 0], x[:, 1], x[:, 2]) * h ** 3
    if face_owner is not None and bc is not None:
        face_dir = np.asarray(face_dir)
        wall = np.asarray(face_other) < 0
        dirich = wall & (np.asarray(bc)[face_dir] == DIRICHLET)
        if np.any(dirich):
            corners = face_corners(np.asarray(face_level)[dirich],
                                   np.asarray(face_ijk).reshape(-1, 3)[dirich],
                                   face_dir[dirich])
            fc = corners.mean(axis=0)
            hw = np.ldexp(1.0, -np.asarray(face_level, dtype=np.int64)[dirich])
            kw = np.asarray(face_beta_)[dirich] * hw * hw / (theta * hw)
            np.add.at(rhs, np.asarray(face_owner)[dirich],
                      kw * p(fc[:, 0], fc[:, 1], fc[:, 2]))
    return rhs


def rhs_random(cfg, leaf_level, leaf_ijk):
    """rhs_i = -b_i h_i^3 with b_i ~ U[-1, 1] in canonical leaf order, made
    volume-mean free over all leaves."""
    rng = np.random.default_rng(config_seed(cfg) + 17)
    n = len(leaf_level)
    b = rng.uniform(-1.0, 1.0, size=n)
    h3 = np.ldexp(1.0, -3 * np.asarray(leaf_level, dtype=np.int64))
    b = b - np.dot(b, h3) / h3.sum()
    return -b * h3


def adjoint_target(leaf_level, leaf_ijk, pmax, seed=1005 + 29):
    """Smooth target field: a seeded sum of 4 Gaussians."""
    rng = np.random.default_rng(seed)
    cs = rng.uniform(0.2, 0.8, size=(4, 3))
    sig = rng.uniform(0.05, 0.2, size=4)
    amp = rng.uniform(-1.0, 1.0, size=4) * pmax
    x, _ = cell_centers(leaf_level, leaf_ijk)
    out = np.zeros(len(x))
    for c, s, a in zip(cs, sig, amp):
        r2 = ((x - c) ** 2).sum(axis=1)
        out += a * np.exp(-r2 / (2.0 * s * s))
    return out


def sample_faces(n_faces, special, count=50, seed=1005 + 31, pool=None):
    """Half of ``count`` faces drawn from ``special`` (indices where the
    operator is non-symmetric or beta < 1), half uniformly from ``pool``
    (default: all faces)."""
    rng = np.random.default_rng(seed)
    special = np.asarray(special)
    k = min(count // 2, len(special))
    a = rng.choice(special, size=k, replace=False) if k else np.zeros(0, int)
    rest = np.setdiff1d(np.arange(n_faces) if pool is None else np.asarray(pool), a)
    b = rng.choice(rest, size=count - k, replace=False)
    return np.sort(np.concatenate([a, b]).astype(np.int64))
