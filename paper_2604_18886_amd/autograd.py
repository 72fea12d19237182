"""torch.autograd.Function around the solver: p = A(beta)^-1 rhs forward,
and the hand-written adjoint backward.

backward(dL/dp) solves A^T lambda = dL/dp (PCG with the transposed cycle)
and returns dL/dbeta_f = -lambda^T (dA/dbeta_f) p per face and
dL/drhs = lambda.  Every step runs in the library's kernels.
"""

import torch

from . import mfmg


class MFMGSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, face_beta, rhs, tree, bc, theta, rtol, hierarchy_kw):
        co = mfmg.assemble_coeffs(tree, face_beta.detach().contiguous(), bc, theta)
        h = mfmg.build_hierarchy(co, **(hierarchy_kw or {}))
        p, stats = mfmg.pcg_solve(h, rhs.detach().contiguous(), rtol=rtol)
        ctx.h = h
        ctx.rtol = rtol
        ctx.stats = stats
        ctx.save_for_backward(p)
        return p

    @staticmethod
    def backward(ctx, dL_dp):
        (p,) = ctx.saved_tensors
        lam, g, _ = mfmg.pcg_solve_adjoint(ctx.h, p, dL_dp.contiguous(), rtol=ctx.rtol)
        return g, lam, None, None, None, None, None


def solve(face_beta, rhs, tree, bc=(mfmg.DIRICHLET,) * 6, theta=0.5, rtol=1e-10,
          **hierarchy_kw):
    """p with A(face_beta) p = rhs, differentiable in face_beta and rhs."""
    return MFMGSolve.apply(face_beta, rhs, tree, tuple(bc), float(theta), float(rtol),
                           hierarchy_kw)
