"""PCG, adjoint solve and finite-difference gradient reference (test
infrastructure).

Paper passages restated here
  * Section 2.2, Algorithm 1: PCG from x0 = 0 with alpha_k = (r,z)/(Ap,p) and
    beta_k = (r_{k+1}, z_{k+1}) / (r_k, z_k); the preconditioner is one
    multigrid cycle.
  * Section 2.2: with a null space (no Dirichlet face), the residual is shifted
    to zero mean after it is formed (initial residual and every update).

Readings
  * Stop when ||r_k||_2 <= rtol ||r_0||_2 (r_0 after the null-space shift);
    the preconditioner is not applied to a residual that already meets the
    tolerance (the iterate does not depend on it).  Then the FP64 true
    residual ||b - A x|| / ||r_0|| is formed; while it exceeds rtol and
    iterations are left, Algorithm 1 starts again from the current iterate
    with r = b - A x (same tolerance, same iteration budget), so a solve
    reported as converged meets rtol in its true residual.  A restart that
    does not lower the true residual (the rounding floor of the problem is
    above rtol) ends the solve as not converged.
  * The null-space shift subtracts the unweighted mean over active cells; the
    returned solution is then shifted to zero mean as well.
  * The adjoint solves A^T lambda = dL/dp preconditioned by the transpose
    M^T of the same cycle (so that M^T A^T = (A M)^T has the spectrum of the
    forward preconditioned operator); the per-face gradient is
    -lambda^T (dA/dbeta_f) p (the operator is linear in beta).
"""

import numpy as np


class BreakdownError(RuntimeError):
    pass


def pcg(A, b, precond=None, rtol=1e-10, max_iter=200, null_space=False,
        active=None, x_out=None, x0=None):
    """Returns (x, info) with info = dict(iters, hist, true, status).

    x0 (optional) is an initial guess: the iteration starts from the residual
    b - A x0, and the stop test and the history are taken relative to
    ||b|| (which is ||r_0|| for the zero start), so a good guess stops
    earlier at the same accuracy."""
    b = np.asarray(b, dtype=np.float64)
    n = len(b)
    if active is None:
        active = np.ones(n, dtype=bool)
    b = np.where(active, b, 0.0)
    nact = active.sum()

    def project(v):
        if not null_space:
            return v
        return np.where(active, v - v[active].sum() / nact, 0.0)

    M = precond if precond is not None else (lambda r: r.copy())
    if x0 is None:
        x = np.zeros(n)
        r = project(b.copy())
        r0 = np.linalg.norm(r)
        hist = [1.0 if r0 > 0 else 0.0]
    else:
        x = np.where(active, np.asarray(x0, dtype=np.float64), 0.0)
        r = project(np.where(active, b - A @ x, 0.0))
        r0 = np.linalg.norm(project(b.copy()))
        hist = [np.linalg.norm(r) / r0 if r0 > 0 else 0.0]
    info = {"iters": 0, "hist": hist, "true": 0.0, "status": 0, "restarts": 0}
    if r0 == 0.0:
        return x, info
    if x0 is not None and np.linalg.norm(r) <= rtol * r0:
        info["true"] = hist[0]
        return x, info
    k = 0
    restarts = 0
    true = np.inf
    while True:
        z = np.where(active, M(r), 0.0)
        p = z.copy()
        rz = r @ z
        status = 1
        while k < max_iter:
            if not (rz > 0.0) or not np.isfinite(rz):
                raise BreakdownError("(r, z) <= 0")
            Ap = A @ p
            pAp = p @ Ap
            if not (pAp > 0.0) or not np.isfinite(pAp):
                raise BreakdownError("(p, Ap) <= 0")
            alpha = rz / pAp
            x = x + alpha * p
            r = project(r - alpha * Ap)
            k += 1
            rn = np.linalg.norm(r)
            hist.append(rn / r0)
            if rn <= rtol * r0:
                status = 0
                break
            z = np.where(active, M(r), 0.0)
            rz_new = r @ z
            beta = rz_new / rz
            rz = rz_new
            p = z + beta * p
        if null_space:
            x = np.where(active, x - x[active].sum() / nact, 0.0)
        r = project(np.where(active, b - A @ x, 0.0))
        prev, true = (true if restarts else np.inf), float(np.linalg.norm(r) / r0)
        if status != 0 or true <= rtol or k >= max_iter or not true < prev:
            break
        # the recurrence met the tolerance but the true residual does not:
        # start again from x with the true residual
        restarts += 1
    if status == 0 and true > rtol:
        status = 1
    info["iters"] = k
    info["status"] = status
    info["true"] = true
    info["restarts"] = restarts
    return x, info


def cg_textbook_reference(A, b, iters):
    """Unpreconditioned CG iterates via SciPy (an independent implementation)
    for the identity-preconditioner pin."""
    import scipy.sparse.linalg as spla
    x, _ = spla.cg(A, b, rtol=0.0, atol=0.0, maxiter=iters)
    return x


def solve_and_grad(disc, hier, rhs, loss_grad, rtol=1e-10, max_iter=200):
    """Forward solve, adjoint solve and per-face gradient."""
    act = disc.active
    p, info = pcg(disc.A, rhs, hier.vcycle, rtol, max_iter, active=act)
    g = loss_grad(p)
    At = disc.A.T.tocsr()
    lam, ainfo = pcg(At, g, hier.vcycle_T, rtol, max_iter, active=act)
    return p, lam, disc.face_gradient(lam, p), info, ainfo


def fd_gradient(disc_factory, beta, p, p_target, faces, eps=1e-6, rtol=1e-13,
                precond_factory=None, max_iter=400, rhs=None, return_steps=False):
    """Central finite differences of L = sum_active (p - p_t)^2 with respect to
    beta_f, computed as difference solves so that cancellation does not
    destroy the O(eps) change of L:

      A(beta +- eps e_f) dp_pm = r0 -+ eps (dA/dbeta_f) p,   r0 = rhs - A(beta) p
      dL_pm = 2 (p - p_t) . dp_pm + ||dp_pm||^2

    where p is the base solution; then g_f = (dL_+ - dL_-) / (2 eps).
    ``disc_factory(beta)`` returns a Discretization for coefficients beta.
    Every face coefficient of Eq. (3) is proportional to beta (and the
    coarse side of a T-face is a sum of such), so A is linear in beta and
    (dA/dbeta_f) p = (A(beta + e_f) - A(beta)) p exactly; forming it with a
    unit step keeps the cancellation of the two products at the level of
    the operator, not of eps.  ``rhs`` (optional) gives r0; without it r0
    is taken as 0 (p solved to tight tolerance).

    The step is relative to the coupling of the face's cells: eps_f = eps *
    min(1, c_i / (dc_i/dbeta_f)) over the face's cells i.  At a nearly solid
    cell (all face fractions ~1e-4) a fixed step of 1e-6 would change its
    operator by ~1% and the O(eps^2) error of the central difference would
    dominate; elsewhere c_i / (dc_i/dbeta_f) is the sum of the cell's face
    betas (about 6) and eps_f = eps.  Returns g_f (and the steps eps_f with
    return_steps)."""
    out = np.zeros(len(faces))
    steps = np.zeros(len(faces))
    base = disc_factory(beta)
    base_Ap = base.A @ p
    r0 = np.zeros_like(p) if rhs is None else np.where(base.active, rhs - base_Ap, 0.0)
    for n, f in enumerate(faces):
        bu = beta.copy()
        bu[f] = bu[f] + 1.0
        du = disc_factory(bu)
        dA_p = du.A @ p - base_Ap
        cells = [base.face_owner[f]] + ([base.face_other[f]] if base.face_other[f] >= 0 else [])
        ratio = [base.c[i] / (du.c[i] - base.c[i]) for i in cells if du.c[i] != base.c[i]]
        step = eps * min([1.0] + ratio)
        steps[n] = step
        dls = []
        for sgn in (+1.0, -1.0):
            bb = beta.copy()
            bb[f] = bb[f] + sgn * step
            dpert = disc_factory(bb)
            act = dpert.active
            b = np.where(act, r0 - sgn * step * dA_p, 0.0)
            M = precond_factory(dpert) if precond_factory else None
            # the difference solve is a forward solve with A(beta +- eps e_f)
            dp, _ = pcg(dpert.A, b, M, rtol, max_iter, active=act)
            e = np.where(act, p - p_target, 0.0)
            dls.append(2.0 * e @ dp + dp @ dp)
        out[n] = (dls[0] - dls[1]) / (2.0 * step)
    return (out, steps) if return_steps else out
