"""Shared helpers for the oracle tests: small octrees and problem setup."""

import numpy as np

import problems
from oracle import discretize as D
from oracle import multigrid as M
from oracle import octree as O


def read_golden(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    out = {}
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        k, v = line.split("=")
        out[k.strip()] = float(v)
    return out


def half_nodes(l, B=4, axis=0):
    """Nodes of a grid whose lower half (along ``axis``) is one level finer."""
    n = (1 << l) // B
    nodes = set()
    for a in range(n):
        for b in range(n):
            for c in range(n):
                if (a, b, c)[axis] < n // 2:
                    nodes.update(O.children((l, a, b, c)))
                else:
                    nodes.add((l, a, b, c))
    return nodes


def half_tree(l, axis=0):
    spec = {"min_level": l, "max_level": l + 1, "node_size": 4, "prims": []}
    return O.Octree(spec, half_nodes(l, axis=axis))


def three_level_nodes(l):
    """Corner node refined twice, its neighbours once: three leaf levels."""
    nodes = half_nodes(l)
    fine = [n for n in nodes if n[0] == l + 1 and n[1] == 0 and n[2] == 0 and n[3] == 0]
    for f in fine:
        nodes.remove(f)
        nodes.update(O.children(f))
    return O.balance(nodes, l, 4)


def disc_for(tree, beta=None, bc=(D.DIRICHLET,) * 6, theta=0.5, seed=None):
    d = D.Discretization(tree, None, bc, theta)
    if beta is None:
        if seed is None:
            beta = np.ones(d.n_faces)
        else:
            rng = np.random.default_rng(seed)
            beta = rng.uniform(0.5, 1.0, size=d.n_faces)
    d.set_beta(beta)
    return d


def config_problem(cfg, **levels):
    T = O.Octree(problems.config_spec(cfg, **levels))
    bc, th = problems.config_bc(cfg)
    d = D.Discretization(T, None, bc, th)
    beta = problems.face_beta(cfg, d.face_level, d.face_ijk, d.face_dir)
    d.set_beta(beta)
    if cfg in (1, 2):
        rhs = problems.rhs_manufactured(cfg, T.level, T.ijk, d.face_owner, d.face_level,
                                        d.face_ijk, d.face_dir, d.face_other, beta, bc, th)
    else:
        rhs = problems.rhs_random(cfg, T.level, T.ijk)
    return T, d, beta, rhs


def hierarchy(d, **kw):
    return M.Hierarchy(d, coarsest=kw.pop("coarsest", min(3, d.tree.lmin)), **kw)
