"""Thin ctypes binding of libmfmg.so (the solver's C ABI, include/mfmg.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  Device buffers are torch tensors on the current HIP device and the
library runs on torch's current stream.  The library is loaded from this
package directory; when it is missing, importing the solver fails loudly.
"""

import ctypes
import os
import warnings

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmfmg.so")

OK = 0
NOT_CONVERGED = 1
INCOMPATIBLE_RHS = -6
SPHERE, BOX = 0, 1
NEUMANN, DIRICHLET = 0, 1
FP64, MIXED = 0, 1


class MFMGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"mfmg status {status}: {msg}")
        self.status = status


class NotConvergedWarning(RuntimeWarning):
    pass


class _Prim(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("center", ctypes.c_double * 3),
                ("radius", ctypes.c_double), ("band", ctypes.c_double),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3)]


class _Spec(ctypes.Structure):
    _fields_ = [("min_level", ctypes.c_int), ("max_level", ctypes.c_int),
                ("node_size", ctypes.c_int), ("n_prims", ctypes.c_int),
                ("prims", ctypes.POINTER(_Prim))]


class _BC(ctypes.Structure):
    _fields_ = [("bc", ctypes.c_int * 6), ("theta", ctypes.c_double)]


class _MGParams(ctypes.Structure):
    _fields_ = [("nu_pre", ctypes.c_int), ("nu_post", ctypes.c_int),
                ("nu_coarse", ctypes.c_int), ("mu", ctypes.c_int),
                ("coarsest_level", ctypes.c_int), ("alpha", ctypes.c_double),
                ("beta_mg", ctypes.c_double), ("precision", ctypes.c_int)]


class _SolveParams(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("null_space", ctypes.c_int), ("warm_start", ctypes.c_int)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("status", ctypes.c_int),
                ("rel_resid_recur", ctypes.c_double),
                ("rel_resid_true", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_VP = ctypes.c_void_p
_I64P = ctypes.POINTER(ctypes.c_int64)

# exported symbol -> (restype, argtypes); every symbol of include/mfmg.h
SIGNATURES = {
    "mfmg_last_error": (ctypes.c_char_p, []),
    "mfmg_build_octree": (ctypes.c_int, [ctypes.POINTER(_Spec), ctypes.POINTER(_VP)]),
    "mfmg_build_octree_device": (ctypes.c_int, [ctypes.POINTER(_Spec), _VP,
                                                ctypes.POINTER(_VP)]),
    "mfmg_octree_info": (ctypes.c_int, [_VP, _I64P, _I64P, _I64P]),
    "mfmg_octree_leaves": (ctypes.c_int, [_VP, _VP, _VP]),
    "mfmg_octree_faces": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "mfmg_octree_leaves_device": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "mfmg_octree_faces_device": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    "mfmg_destroy_octree": (None, [_VP]),
    "mfmg_assemble_coeffs": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(_BC), _VP,
                                            ctypes.POINTER(_VP)]),
    "mfmg_coeffs_leaf": (ctypes.c_int, [_VP, _VP, _VP]),
    "mfmg_destroy_coeffs": (None, [_VP]),
    "mfmg_build_hierarchy": (ctypes.c_int, [_VP, ctypes.POINTER(_MGParams), _VP,
                                            ctypes.POINTER(_VP)]),
    "mfmg_hierarchy_level_coeffs": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _VP]),
    "mfmg_hierarchy_level_bricks": (ctypes.c_int, [_VP, ctypes.c_int, _I64P, _VP, _VP]),
    "mfmg_destroy_hierarchy": (None, [_VP]),
    "mfmg_pcg_solve": (ctypes.c_int, [_VP, _VP, _VP, ctypes.POINTER(_SolveParams), _VP,
                                      ctypes.POINTER(SolveStats), _VP]),
    "mfmg_pcg_solve_adjoint": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP,
                                              ctypes.POINTER(_SolveParams), _VP,
                                              ctypes.POINTER(SolveStats)]),
    "mfmg_divergence": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "mfmg_project_velocity": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "mfmg_divergence_rms": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(ctypes.c_double), _VP]),
    "mfmg_divergence_rms_noalloc": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "mfmg_apply_operator": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int, _VP]),
    "mfmg_apply_precond": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int, _VP]),
    "mfmg_profile": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP,
                                    ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]),
}

_lib = None


def load_library(path=LIB_PATH):
    """Load libmfmg.so and declare its C signatures (no device call)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python -m paper_2604_18886_amd.build`")
    # torch ships its own HIP runtime (soname libamdhip64.so.7); loading it
    # first makes the dynamic linker bind this library to that same runtime
    # instead of mapping a second copy from /opt/rocm
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status, allow_not_converged=False):
    if status == OK:
        return
    msg = _lib.mfmg_last_error().decode()
    if status == NOT_CONVERGED and allow_not_converged:
        warnings.warn(msg, NotConvergedWarning)
        return
    raise MFMGError(status, msg)


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    torch = _torch()
    assert isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous(), \
        "device buffers must be contiguous HIP tensors"
    return ctypes.c_void_p(t.data_ptr())


def _vec(t, n, what):
    """Pointer to a float64 device vector of exactly n entries (the C ABI
    cannot check the length of a device buffer, so the binding does)."""
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.dtype == torch.float64 and t.numel() == n):
        raise ValueError(f"{what}: expected a float64 device tensor of {n} entries")
    return _ptr(t)


# --------------------------------------------------------------------- octree
class Octree:
    def __init__(self, handle):
        self._h = handle
        lib = load_library()
        nl, nf, nb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib.mfmg_octree_info(self._h, ctypes.byref(nl), ctypes.byref(nf),
                                    ctypes.byref(nb)))
        self.n_leaves = nl.value
        self.n_faces = nf.value
        self.n_leaf_bricks = nb.value

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mfmg_destroy_octree(self._h)
            self._h = None

    def leaves(self):
        """(level uint8[n], ijk int32[n, 3]) in canonical order."""
        lev = np.empty(self.n_leaves, dtype=np.uint8)
        ijk = np.empty((self.n_leaves, 3), dtype=np.int32)
        _check(_lib.mfmg_octree_leaves(self._h, lev.ctypes.data_as(_VP),
                                       ijk.ctypes.data_as(_VP)))
        return lev, ijk

    def faces(self):
        """(owner int64, dir int8, other int64, kind int8) in canonical order."""
        n = self.n_faces
        owner = np.empty(n, dtype=np.int64)
        d = np.empty(n, dtype=np.int8)
        other = np.empty(n, dtype=np.int64)
        kind = np.empty(n, dtype=np.int8)
        _check(_lib.mfmg_octree_faces(self._h, owner.ctypes.data_as(_VP),
                                      d.ctypes.data_as(_VP), other.ctypes.data_as(_VP),
                                      kind.ctypes.data_as(_VP)))
        return owner, d, other, kind

    def leaves_device(self):
        """leaves() as device tensors, written on the current stream."""
        torch = _torch()
        lev = torch.empty(max(1, self.n_leaves), dtype=torch.uint8, device="cuda")
        ijk = torch.empty((max(1, self.n_leaves), 3), dtype=torch.int32, device="cuda")
        _check(_lib.mfmg_octree_leaves_device(self._h, _ptr(lev), _ptr(ijk), _stream()))
        return lev[:self.n_leaves], ijk[:self.n_leaves]

    def faces_device(self):
        """faces() as device tensors, written on the current stream."""
        torch = _torch()
        n = max(1, self.n_faces)
        owner = torch.empty(n, dtype=torch.int64, device="cuda")
        d = torch.empty(n, dtype=torch.int8, device="cuda")
        other = torch.empty(n, dtype=torch.int64, device="cuda")
        kind = torch.empty(n, dtype=torch.int8, device="cuda")
        _check(_lib.mfmg_octree_faces_device(self._h, _ptr(owner), _ptr(d), _ptr(other),
                                             _ptr(kind), _stream()))
        k = self.n_faces
        return owner[:k], d[:k], other[:k], kind[:k]


def build_octree(spec, device=False):
    """Octree from a spec dict {min_level, max_level, node_size, prims}
    (prims: dicts with kind, center, radius, band, lo, hi), built on the
    host, or with device=True on the device (current stream)."""
    lib = load_library()
    prims = spec.get("prims", [])
    arr = (_Prim * max(1, len(prims)))()
    for i, p in enumerate(prims):
        arr[i].kind = int(p["kind"])
        for a in range(3):
            arr[i].center[a] = float(p.get("center", (0, 0, 0))[a])
            arr[i].lo[a] = float(p.get("lo", (0, 0, 0))[a])
            arr[i].hi[a] = float(p.get("hi", (0, 0, 0))[a])
        arr[i].radius = float(p.get("radius", 0.0))
        arr[i].band = float(p.get("band", 0.0))
    s = _Spec(int(spec["min_level"]), int(spec["max_level"]),
              int(spec.get("node_size", 4)), len(prims), arr)
    h = _VP()
    if device:
        _check(lib.mfmg_build_octree_device(ctypes.byref(s), _stream(), ctypes.byref(h)))
    else:
        _check(lib.mfmg_build_octree(ctypes.byref(s), ctypes.byref(h)))
    return Octree(h)


# ---------------------------------------------------------------- coefficients
class Coeffs:
    def __init__(self, handle, tree, bc, theta):
        self._h = handle
        self.tree = tree  # keeps the octree alive
        self.bc = tuple(bc)
        self.theta = theta

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mfmg_destroy_coeffs(self._h)
            self._h = None

    def leaf_coeffs(self):
        """Device tensor (4, n_leaves): c, kx, ky, kz."""
        torch = _torch()
        out = torch.empty((4, self.tree.n_leaves), dtype=torch.float64, device="cuda")
        _check(_lib.mfmg_coeffs_leaf(self._h, _ptr(out), _stream()))
        return out


def assemble_coeffs(tree, face_beta, bc=(DIRICHLET,) * 6, theta=0.5):
    """Leaf coefficients from per-face beta (device float64 tensor)."""
    torch = _torch()
    lib = load_library()
    b = _BC((ctypes.c_int * 6)(*[int(x) for x in bc]), float(theta))
    h = _VP()
    _check(lib.mfmg_assemble_coeffs(tree._h, _vec(face_beta, tree.n_faces, "face_beta"),
                                    ctypes.byref(b), _stream(), ctypes.byref(h)))
    return Coeffs(h, tree, bc, theta)


# ------------------------------------------------------------------- hierarchy
class Hierarchy:
    def __init__(self, handle, coeffs, params):
        self._h = handle
        self.coeffs = coeffs
        self.params = params

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mfmg_destroy_hierarchy(self._h)
            self._h = None

    @property
    def n_leaves(self):
        return self.coeffs.tree.n_leaves

    def level_bricks(self, level):
        n = ctypes.c_int64()
        _check(_lib.mfmg_hierarchy_level_bricks(self._h, level, ctypes.byref(n), None, None))
        coords = np.empty((n.value, 3), dtype=np.int32)
        leaf = np.empty(n.value, dtype=np.uint8)
        _check(_lib.mfmg_hierarchy_level_bricks(self._h, level, ctypes.byref(n),
                                                coords.ctypes.data_as(_VP),
                                                leaf.ctypes.data_as(_VP)))
        return coords, leaf.astype(bool)

    def level_coeffs(self, level):
        """Device tensor (n_bricks, 4, 64) of FP64 level coefficients."""
        torch = _torch()
        coords, _ = self.level_bricks(level)
        out = torch.empty((len(coords), 4, 64), dtype=torch.float64, device="cuda")
        _check(_lib.mfmg_hierarchy_level_coeffs(self._h, level, _ptr(out), _stream()))
        return out


def build_hierarchy(coeffs, nu_pre=2, nu_post=2, nu_coarse=10, mu=1, coarsest_level=3,
                    alpha=2.0, beta_mg=2.0, precision=FP64):
    lib = load_library()
    p = _MGParams(nu_pre, nu_post, nu_coarse, mu, coarsest_level, alpha, beta_mg, precision)
    h = _VP()
    _check(lib.mfmg_build_hierarchy(coeffs._h, ctypes.byref(p), _stream(), ctypes.byref(h)))
    return Hierarchy(h, coeffs, dict(nu_pre=nu_pre, nu_post=nu_post, nu_coarse=nu_coarse,
                                     mu=mu, coarsest_level=coarsest_level, alpha=alpha,
                                     beta_mg=beta_mg, precision=precision))


# ----------------------------------------------------------------------- solve
def pcg_solve(h, rhs, p=None, rtol=1e-10, max_iter=200, null_space=-1, history=False,
              x0=None):
    """Solve A p = rhs; returns (p, stats dict[, residual history]).  With x0
    (device tensor) the iteration starts from that guess and stops at
    ||r|| <= rtol ||rhs||."""
    torch = _torch()
    n = h.n_leaves
    if p is None:
        p = torch.empty_like(rhs)
    if x0 is not None:
        p.copy_(x0)
    sp = _SolveParams(float(rtol), int(max_iter), int(null_space), int(x0 is not None))
    st = SolveStats()
    hist = np.zeros(max_iter + 1) if history else None
    status = _lib.mfmg_pcg_solve(h._h, _vec(rhs, n, "rhs"), _vec(p, n, "p"),
                                 ctypes.byref(sp), _stream(),
                                 ctypes.byref(st),
                                 hist.ctypes.data_as(_VP) if history else None)
    _check(status, allow_not_converged=True)
    out = st.as_dict()
    if history:
        return p, out, hist[: st.iters + 1]
    return p, out


def pcg_solve_adjoint(h, p, dL_dp, rtol=1e-10, max_iter=200, null_space=-1):
    """lambda with A^T lambda = dL/dp and dL/dbeta per face."""
    torch = _torch()
    lam = torch.empty_like(dL_dp)
    g = torch.empty(h.coeffs.tree.n_faces, dtype=torch.float64, device=dL_dp.device)
    sp = _SolveParams(float(rtol), int(max_iter), int(null_space), 0)
    st = SolveStats()
    n = h.n_leaves
    status = _lib.mfmg_pcg_solve_adjoint(h._h, _vec(p, n, "p"), _vec(dL_dp, n, "dL_dp"),
                                         _ptr(lam), _ptr(g), ctypes.byref(sp), _stream(),
                                         ctypes.byref(st))
    _check(status, allow_not_converged=True)
    return lam, g, st.as_dict()


# ------------------------------------------------------------------ projection
def divergence(h, beta, u):
    """Integrated divergence (canonical leaf order) of face velocities u
    with face fluid fractions beta (device tensors, canonical face order)."""
    torch = _torch()
    nf = h.coeffs.tree.n_faces
    pb, pu = _vec(beta, nf, "beta"), _vec(u, nf, "u")
    div = torch.empty(h.n_leaves, dtype=torch.float64, device="cuda")
    _check(_lib.mfmg_divergence(h._h, pb, pu, _ptr(div), _stream()))
    return div


def project_velocity(h, beta, p, u):
    """u -= s F(p) / (beta h^2) in place (see mfmg_project_velocity)."""
    nf = h.coeffs.tree.n_faces
    _check(_lib.mfmg_project_velocity(h._h, _vec(beta, nf, "beta"), _vec(p, h.n_leaves, "p"),
                                      _vec(u, nf, "u"), _stream()))
    return u


def divergence_rms(h, div):
    """Volume-weighted RMS of div_i / V_i over the active leaves."""
    r = ctypes.c_double()
    _check(_lib.mfmg_divergence_rms(h._h, _vec(div, h.n_leaves, "div"), ctypes.byref(r),
                                    _stream()))
    return r.value


def divergence_rms_noalloc(h, div, out=None):
    """mfmg_divergence_rms_noalloc: the RMS into a device tensor of one
    double (out, allocated here when None), queued on the current stream."""
    torch = _torch()
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=div.device)
    _check(_lib.mfmg_divergence_rms_noalloc(h._h, _vec(div, h.n_leaves, "div"),
                                            _vec(out, 1, "out"), _stream()))
    return out


def project(h, beta, u, rtol=1e-10, max_iter=200):
    """One pressure projection of the face velocities u (in place):
    rhs = div(u), solve A p = rhs, update u.  Returns (p, solve stats,
    RMS of the divergence before, after)."""
    div = divergence(h, beta, u)
    rms0 = divergence_rms(h, div)
    p, st = pcg_solve(h, div, rtol=rtol, max_iter=max_iter)
    project_velocity(h, beta, p, u)
    rms1 = divergence_rms(h, divergence(h, beta, u))
    return p, st, rms0, rms1


def apply_operator(h, x, transpose=False):
    torch = _torch()
    y = torch.empty_like(x)
    _check(_lib.mfmg_apply_operator(h._h, _vec(x, h.n_leaves, "x"), _ptr(y), int(transpose),
                                    _stream()))
    return y


def apply_precond(h, r, transpose=False):
    torch = _torch()
    z = torch.empty_like(r)
    _check(_lib.mfmg_apply_precond(h._h, _vec(r, h.n_leaves, "r"), _ptr(z), int(transpose),
                                   _stream()))
    return z


PROFILE_SMOOTH, PROFILE_CYCLE, PROFILE_COPY = 0, 1, 2


def profile(h, what, level=0, reps=20):
    """(ms per launch, algorithmic bytes per launch) of a hot-path step,
    measured with HIP events on the current stream."""
    ms = ctypes.c_double()
    by = ctypes.c_double()
    _check(_lib.mfmg_profile(h._h, int(what), int(level), int(reps), _stream(),
                             ctypes.byref(ms), ctypes.byref(by)))
    return ms.value, by.value
