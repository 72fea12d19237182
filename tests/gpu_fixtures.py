"""Helpers for the GPU parity tests: build the same problem on the library
(through the C ABI) and on the oracle, from the shared seeded inputs."""

import functools

import numpy as np

import problems
from oracle import discretize as D
from oracle import krylov as K
from oracle import multigrid as M
from oracle import octree as O


def torch_cuda():
    import torch
    return torch


class Case:
    """A workload built on both sides.  ``spec``/``cfg`` select geometry and
    inputs; ``beta``/``rhs`` are numpy arrays in canonical order."""

    def __init__(self, cfg, spec, bc=None, theta=None, beta=None, rhs=None, nodes=None):
        from paper_2604_18886_amd import mfmg
        self.cfg = cfg
        self.spec = spec
        bc0, th0 = problems.config_bc(cfg)
        self.bc = tuple(bc if bc is not None else bc0)
        self.theta = th0 if theta is None else theta
        self.T = O.Octree(spec, nodes)
        self.tree = mfmg.build_octree(spec) if nodes is None else None
        self.disc = D.Discretization(self.T, None, self.bc, self.theta)
        if beta is None:
            beta = problems.face_beta(cfg, self.disc.face_level, self.disc.face_ijk,
                                      self.disc.face_dir)
        self.beta = np.asarray(beta, dtype=np.float64)
        self.disc.set_beta(self.beta)
        if rhs is None:
            if cfg in (1, 2):
                rhs = problems.rhs_manufactured(
                    cfg, self.T.level, self.T.ijk, self.disc.face_owner, self.disc.face_level,
                    self.disc.face_ijk, self.disc.face_dir, self.disc.face_other, self.beta,
                    self.bc, self.theta)
            else:
                rhs = problems.rhs_random(cfg, self.T.level, self.T.ijk)
        self.rhs = np.asarray(rhs, dtype=np.float64)

    @functools.cached_property
    def hier(self):
        return M.Hierarchy(self.disc, coarsest=min(3, self.T.lmin))

    def device(self, x):
        torch = torch_cuda()
        return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")

    def gpu_hierarchy(self, precision=0, **kw):
        from paper_2604_18886_amd import mfmg
        co = mfmg.assemble_coeffs(self.tree, self.device(self.beta), self.bc, self.theta)
        return mfmg.build_hierarchy(co, coarsest_level=min(3, self.T.lmin),
                                    precision=precision, **kw)

    def oracle_solve(self, rtol=1e-13):
        x, info = K.pcg(self.disc.A, self.rhs, self.hier.vcycle, rtol, 400,
                        active=self.disc.active)
        return x, info


def small_cases():
    """Workload-family members small enough for per-element oracle parity:
    several bricks, three leaf levels, T-junctions and cut cells."""
    return {
        "uniform32": lambda: Case(1, problems.config_spec(1)),
        "sphere_band_4_6": lambda: Case(2, problems.config_spec(2, 4, 6)),
        "cut_sphere_5_7": lambda: Case(3, problems.config_spec(3, 5, 7)),
        "cut_box_4_6": lambda: Case(4, problems.config_spec(4, 4, 6)),
    }


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
