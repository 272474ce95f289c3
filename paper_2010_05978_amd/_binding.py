"""ctypes binding of libfresnel_hip.so (argument marshalling only).

Every function here has the name of the C entry point it calls and does no
arithmetic of the method: all steps run in the library's HIP kernels.  Arrays
may be torch tensors (device or host) or numpy arrays (host); the memory space
argument of the C call follows from where the array lives.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfresnel_hip.so")

FH_OK = 0
FH_ERR_INVALID_ARG = 1
FH_ERR_ODD_GRID = 2
FH_ERR_NONPOSITIVE_LZ = 3
FH_ERR_NONFINITE = 4
FH_ERR_ALLOC = 5
FH_ERR_HIP = 6
FH_ERR_FFT = 7
FH_ERR_UNSUPPORTED = 8

FH_FP64 = 0
FH_MIXED = 1
FH_MEM_HOST = 0
FH_MEM_DEVICE = 1

EXPORTED = [
    "fh_create", "fh_destroy", "fh_set_stream", "fh_synchronize", "fh_order_after", "fh_set_options", "fh_query_params",
    "fh_status_string", "fh_last_error", "fh_quad_from_boundary", "fh_quad_radial", "fh_quad_polygon",
    "fh_quad_starshade", "fh_quad_from_nodes", "fh_quad_size", "fh_quad_export", "fh_quad_device_ptrs",
    "fh_quad_destroy", "fh_targets_create", "fh_targets_size", "fh_targets_box", "fh_targets_destroy",
    "fh_field_grid", "fh_field_points", "fh_field_targets", "fh_field_grid_batch", "fh_field_grid_vjp",
    "fh_starshade_vjp", "fh_autotune_grid", "fh_set_timing", "fh_last_timing", "fh_timing_totals",
    "fh_boundary_radial", "fh_boundary_polygon", "fh_boundary_starshade", "fh_field_nsli",
    "fh_quad_fourier", "fh_boundary_fourier", "fh_quad_koch", "fh_quad_starshade_rigid",
    "fh_quad_starshade_tab", "fh_targets_sort", "fh_probe_ceilings", "fh_quad_set_illumination",
    "fh_field_nsli_noalloc", "fh_quad_starshade_ribbon", "fh_autotune_batch", "fh_field_grid_batch_rebuild",
    "fh_field_grid_vjp_sum",
]


class FresnelError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{_status_name(status)}: {message}")


class fh_options(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("kernel_width", ctypes.c_int32), ("beta", ctypes.c_double),
                ("tile", ctypes.c_int32), ("max_subproblem", ctypes.c_int32), ("spread_method", ctypes.c_int32),
                ("deterministic", ctypes.c_int32)]


_lib = None


def lib():
    """Load the shared library; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2010_05978_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        pvp = ctypes.POINTER(ctypes.c_void_p)
        sig = {
            "fh_create": [pvp, ctypes.c_int, ctypes.c_int, d, ctypes.POINTER(fh_options)],
            "fh_destroy": [vp],
            "fh_set_stream": [vp, vp],
            "fh_synchronize": [vp],
            "fh_order_after": [vp, vp],
            "fh_set_options": [vp, ctypes.POINTER(fh_options)],
            "fh_query_params": [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(d), ctypes.POINTER(d),
                                ctypes.POINTER(i32)],
            "fh_quad_from_boundary": [vp, vp, vp, vp, vp, i64, i32, ctypes.c_int, pvp],
            "fh_quad_radial": [vp, d, vp, vp, i32, i32, i32, i32, pvp],
            "fh_quad_polygon": [vp, vp, vp, i32, i32, i32, pvp],
            "fh_quad_starshade": [vp, i32, d, d, d, d, i32, i32, i32, i32, vp, i32, ctypes.c_int, pvp],
            "fh_quad_from_nodes": [vp, vp, vp, vp, i64, ctypes.c_int, pvp],
            "fh_quad_size": [vp, ctypes.POINTER(i64)],
            "fh_quad_export": [vp, vp, vp, vp, ctypes.c_int],
            "fh_quad_device_ptrs": [vp, pvp, pvp, pvp],
            "fh_quad_destroy": [vp],
            "fh_field_grid": [vp, vp, d, d, i32, i32, d, d, d, d, i32, vp, ctypes.c_int],
            "fh_field_points": [vp, vp, d, d, i64, vp, vp, i32, vp, ctypes.c_int],
            "fh_targets_create": [vp, i64, vp, vp, ctypes.POINTER(d), ctypes.c_int, pvp],
            "fh_targets_size": [vp, ctypes.POINTER(i64)],
            "fh_targets_sort": [vp],
            "fh_targets_box": [vp, ctypes.POINTER(d)],
            "fh_targets_destroy": [vp],
            "fh_field_targets": [vp, vp, d, d, vp, i32, vp, ctypes.c_int],
            "fh_field_grid_batch": [vp, i32, vp, vp, vp, i32, i32, d, d, d, d, vp, vp],
            "fh_field_grid_vjp": [vp, vp, d, d, i32, i32, d, d, d, d, i32, vp, vp, vp, vp],
            "fh_starshade_vjp": [vp, i32, d, d, d, d, i32, i32, i32, i32, vp, i32, vp, vp, vp, vp],
            "fh_autotune_grid": [vp, vp, d, d, i32, i32, d, d, ctypes.c_char_p, ctypes.POINTER(fh_options)],
            "fh_autotune_batch": [vp, i32, vp, vp, vp, i32, i32, d, d, ctypes.c_char_p, ctypes.POINTER(fh_options)],
            "fh_field_grid_batch_rebuild": [vp, i32, vp, vp, vp, i32, i32, d, d, d, d, vp, vp],
            "fh_field_grid_vjp_sum": [vp, vp, i32, vp, vp, i32, i32, d, d, d, d, i32, vp, vp, vp, vp],
            "fh_set_timing": [vp, i32],
            "fh_last_timing": [vp, ctypes.POINTER(d)],
            "fh_timing_totals": [vp, i32, ctypes.POINTER(d), ctypes.POINTER(i64), i32],
            "fh_boundary_radial": [vp, d, vp, vp, i32, i32, i32, vp, vp, vp, vp, ctypes.c_int],
            "fh_boundary_polygon": [vp, vp, vp, i32, i32, vp, vp, vp, vp, ctypes.c_int],
            "fh_boundary_starshade": [vp, i32, d, d, d, d, i32, i32, i32, vp, vp, vp, vp, ctypes.c_int],
            "fh_field_nsli": [vp, vp, vp, vp, vp, i64, d, d, i64, vp, vp, d, i32, vp, ctypes.c_int],
            "fh_quad_fourier": [vp, i32, vp, vp, vp, vp, i32, i32, i32, pvp],
            "fh_quad_koch": [vp, i32, vp, pvp],
            "fh_quad_starshade_rigid": [vp, i32, d, d, d, d, i32, i32, i32, i32, vp, i32, i32, pvp],
            "fh_quad_starshade_tab": [vp, i32, d, d, vp, i32, i32, i32, i32, vp, i32, ctypes.c_int, pvp],
            "fh_quad_starshade_ribbon": [vp, i32, d, d, d, d, i32, i32, i32, i32, vp, i32, ctypes.c_int, i32, pvp],
            "fh_boundary_fourier": [vp, i32, vp, vp, vp, vp, i32, i32, vp, vp, vp, vp, ctypes.c_int],
            "fh_probe_ceilings": [vp, ctypes.POINTER(d)],
            "fh_quad_set_illumination": [vp, vp, vp, d, ctypes.c_int],
            "fh_field_nsli_noalloc": [vp, vp, vp, vp, vp, i64, d, d, i64, vp, vp, d, i32, vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.fh_status_string.argtypes = [ctypes.c_int]
        L.fh_status_string.restype = ctypes.c_char_p
        L.fh_last_error.argtypes = []
        L.fh_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _status_name(s: int) -> str:
    try:
        return lib().fh_status_string(s).decode()
    except Exception:  # pragma: no cover
        return f"status {s}"


def _check(status: int):
    if status != FH_OK:
        raise FresnelError(status, lib().fh_last_error().decode())


# ------------------------------------------------------------ marshalling
def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _ptr_mem(a):
    """(pointer, memspace) of a torch tensor or numpy array (or None)."""
    if a is None:
        return None, FH_MEM_HOST
    if _is_torch(a):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ctypes.c_void_p(a.data_ptr()), (FH_MEM_DEVICE if a.is_cuda else FH_MEM_HOST)
    if isinstance(a, np.ndarray):
        if not a.flags.c_contiguous:
            raise ValueError("array must be C-contiguous")
        return ctypes.c_void_p(a.ctypes.data), FH_MEM_HOST
    raise TypeError(f"unsupported array type {type(a)}")


def _same_mem(*arrays):
    mems = {_ptr_mem(a)[1] for a in arrays if a is not None}
    if len(mems) > 1:
        raise ValueError("arrays must all be on the host or all on the device")
    return mems.pop() if mems else FH_MEM_HOST


# ----------------------------------------------------------------- calls
def fh_create(device: int = 0, precision: int = FH_FP64, tol: float = 1e-9, options: fh_options | None = None):
    h = ctypes.c_void_p()
    _check(lib().fh_create(ctypes.byref(h), device, precision, tol,
                           ctypes.byref(options) if options is not None else None))
    return h


def fh_destroy(ctx):
    _check(lib().fh_destroy(ctx))


def fh_set_stream(ctx, stream):
    """stream: a torch.cuda.Stream, an int handle, or None for the null stream."""
    if stream is not None and hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    _check(lib().fh_set_stream(ctx, ctypes.c_void_p(stream or 0)))


def fh_synchronize(ctx):
    _check(lib().fh_synchronize(ctx))


def fh_order_after(after, before):
    _check(lib().fh_order_after(after, before))


def fh_set_options(ctx, options: fh_options | None):
    _check(lib().fh_set_options(ctx, ctypes.byref(options) if options is not None else None))


def fh_query_params(ctx, n: int):
    w, beta, sigma, nf = ctypes.c_int32(), ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
    _check(lib().fh_query_params(ctx, n, ctypes.byref(w), ctypes.byref(beta), ctypes.byref(sigma),
                                 ctypes.byref(nf)))
    return {"width": w.value, "beta": beta.value, "sigma": sigma.value, "nf": nf.value}


def fh_status_string(s: int) -> str:
    return lib().fh_status_string(s).decode()


def fh_last_error() -> str:
    return lib().fh_last_error().decode()


def _new_quad():
    return ctypes.c_void_p()


def fh_quad_from_boundary(ctx, X, Y, W, V, m: int):
    mem = _same_mem(X, Y, W, V)
    q = _new_quad()
    _check(lib().fh_quad_from_boundary(ctx, _ptr_mem(X)[0], _ptr_mem(Y)[0], _ptr_mem(W)[0], _ptr_mem(V)[0],
                                       len(X), m, mem, ctypes.byref(q)))
    return q


def fh_quad_radial(ctx, r0: float, a=None, b=None, panels: int = 1, q: int = 20, m: int = 10):
    K = 0 if a is None else len(a)
    a = None if a is None else np.ascontiguousarray(a, dtype=np.float64)
    b = None if b is None else np.ascontiguousarray(b, dtype=np.float64)
    if b is not None and len(b) != K:
        raise ValueError("a and b must have the same length")
    h = _new_quad()
    _check(lib().fh_quad_radial(ctx, r0, _ptr_mem(a)[0], _ptr_mem(b)[0], K, panels, q, m, ctypes.byref(h)))
    return h


def fh_quad_polygon(ctx, vx, vy, q: int, m: int):
    vx = np.ascontiguousarray(vx, dtype=np.float64)
    vy = np.ascontiguousarray(vy, dtype=np.float64)
    h = _new_quad()
    _check(lib().fh_quad_polygon(ctx, _ptr_mem(vx)[0], _ptr_mem(vy)[0], len(vx), q, m, ctypes.byref(h)))
    return h


def fh_quad_starshade(ctx, Np, a, R, b, p, m, np_, nd, md, coef=None, K=0):
    if coef is not None and not _is_torch(coef):
        coef = np.ascontiguousarray(coef, dtype=np.float64)
    ptr, mem = _ptr_mem(coef)
    h = _new_quad()
    _check(lib().fh_quad_starshade(ctx, Np, a, R, b, p, m, np_, nd, md, ptr, K if coef is not None else 0,
                                   mem, ctypes.byref(h)))
    return h


def fh_quad_from_nodes(ctx, x, y, w):
    mem = _same_mem(x, y, w)
    h = _new_quad()
    _check(lib().fh_quad_from_nodes(ctx, _ptr_mem(x)[0], _ptr_mem(y)[0], _ptr_mem(w)[0], len(x), mem,
                                    ctypes.byref(h)))
    return h


def fh_quad_size(q) -> int:
    n = ctypes.c_int64()
    _check(lib().fh_quad_size(q, ctypes.byref(n)))
    return n.value


def fh_quad_export(q, x=None, y=None, w=None):
    mem = _same_mem(x, y, w)
    _check(lib().fh_quad_export(q, _ptr_mem(x)[0], _ptr_mem(y)[0], _ptr_mem(w)[0], mem))


def fh_quad_device_ptrs(q):
    x, y, w = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
    _check(lib().fh_quad_device_ptrs(q, ctypes.byref(x), ctypes.byref(y), ctypes.byref(w)))
    return x.value, y.value, w.value


def fh_quad_set_illumination(ctx, q, src=None, D=0.0):
    """src: None, or N complex128 values (numpy array or torch tensor); D: point-source distance (0: plane)."""
    if src is None:
        _check(lib().fh_quad_set_illumination(ctx, q, None, float(D), FH_MEM_HOST))
        return
    if _is_torch(src):
        import torch
        t = src.detach().to(torch.complex128).contiguous()
        ptr, mem = _ptr_mem(torch.view_as_real(t))
        _check(lib().fh_quad_set_illumination(ctx, q, ptr, float(D), mem))
        return
    a = np.ascontiguousarray(np.asarray(src, dtype=np.complex128))
    _check(lib().fh_quad_set_illumination(ctx, q, a.ctypes.data_as(ctypes.c_void_p), float(D), FH_MEM_HOST))


def fh_quad_destroy(q):
    _check(lib().fh_quad_destroy(q))


def fh_field_grid(ctx, q, lam, z, n1, n2, h1, h2, xc, yc, occulter, u):
    ptr, mem = _ptr_mem(u)
    _check(lib().fh_field_grid(ctx, q, lam, z, n1, n2, h1, h2, xc, yc, int(bool(occulter)), ptr, mem))


def fh_field_points(ctx, q, lam, z, xi, eta, occulter, u):
    mem = _same_mem(xi, eta, u)
    _check(lib().fh_field_points(ctx, q, lam, z, len(xi), _ptr_mem(xi)[0], _ptr_mem(eta)[0],
                                 int(bool(occulter)), _ptr_mem(u)[0], mem))


def _rows4(B):
    """The four rows (X, Y, W, V) of a boundary rule: a (4, n) array or tensor."""
    if B.shape[0] != 4:
        raise ValueError("a boundary rule is a (4, n) array: X, Y, W, V")
    return B[0], B[1], B[2], B[3]


def fh_boundary_radial(ctx, r0, a, b, panels, q, B):
    """Fill B (4 x n doubles, n = panels q or q) with the curve's boundary rule."""
    K = 0 if a is None else len(a)
    a = None if a is None else np.ascontiguousarray(a, dtype=np.float64)
    b = None if b is None else np.ascontiguousarray(b, dtype=np.float64)
    X, Y, W, V = _rows4(B)
    mem = _same_mem(X, Y, W, V)
    _check(lib().fh_boundary_radial(ctx, r0, _ptr_mem(a)[0], _ptr_mem(b)[0], K, panels, q, _ptr_mem(X)[0],
                                    _ptr_mem(Y)[0], _ptr_mem(W)[0], _ptr_mem(V)[0], mem))


def _fourier_coefs(ax, bx, ay, by):
    ax = np.ascontiguousarray(ax, dtype=np.float64)
    K = len(ax) - 1
    out = [ax]
    for a in (bx, ay, by):
        a = np.zeros(K + 1) if a is None else np.ascontiguousarray(a, dtype=np.float64)
        if len(a) != K + 1:
            raise ValueError("Fourier coefficient arrays must all have length K + 1")
        out.append(a)
    return K, out


def fh_quad_fourier(ctx, ax, bx, ay, by, panels, q, m):
    K, cs = _fourier_coefs(ax, bx, ay, by)
    h = _new_quad()
    _check(lib().fh_quad_fourier(ctx, K, *[_ptr_mem(a)[0] for a in cs], panels, q, m, ctypes.byref(h)))
    return h


def fh_quad_starshade_ribbon(ctx, Np, a, R, b, p, m, np_, nd, md, coef, K, mr):
    if not _is_torch(coef):
        coef = np.ascontiguousarray(coef, dtype=np.float64)  # kept alive through the call
    ptr, mem = _ptr_mem(coef)
    h = _new_quad()
    _check(lib().fh_quad_starshade_ribbon(ctx, Np, a, R, b, p, m, np_, nd, md, ptr, K, mem, mr, ctypes.byref(h)))
    return h


def fh_quad_starshade_tab(ctx, Np, a, R, A, m, np_, nd, md, coef=None, K=0):
    A = np.ascontiguousarray(A, dtype=np.float64)
    if A.size != m:
        raise ValueError("A needs one value per radial node")
    cptr, cmem = (None, FH_MEM_HOST)
    if coef is not None:
        if not _is_torch(coef):
            coef = np.ascontiguousarray(coef, dtype=np.float64)
        cptr, cmem = _ptr_mem(coef)
    h = _new_quad()
    _check(lib().fh_quad_starshade_tab(ctx, Np, a, R, ctypes.c_void_p(A.ctypes.data), m, np_, nd, md, cptr,
                                       K if coef is not None else 0, cmem, ctypes.byref(h)))
    return h


def fh_quad_starshade_rigid(ctx, Np, a, R, b, p, m, np_, nd, md, motion, nb, mb):
    motion = np.ascontiguousarray(motion, dtype=np.float64).reshape(-1)
    if motion.size != 3 * Np:
        raise ValueError("motion needs 3 values per petal")
    h = _new_quad()
    _check(lib().fh_quad_starshade_rigid(ctx, Np, a, R, b, p, m, np_, nd, md, ctypes.c_void_p(motion.ctypes.data),
                                         nb, mb, ctypes.byref(h)))
    return h


def fh_quad_koch(ctx, L: int, p):
    p = np.ascontiguousarray(p, dtype=np.int32)
    if len(p) != L + 1:
        raise ValueError("p needs L + 1 entries")
    h = _new_quad()
    _check(lib().fh_quad_koch(ctx, L, ctypes.c_void_p(p.ctypes.data), ctypes.byref(h)))
    return h


def fh_boundary_fourier(ctx, ax, bx, ay, by, panels, q, B):
    K, cs = _fourier_coefs(ax, bx, ay, by)
    X, Y, W, V = _rows4(B)
    mem = _same_mem(X, Y, W, V)
    _check(lib().fh_boundary_fourier(ctx, K, *[_ptr_mem(a)[0] for a in cs], panels, q, _ptr_mem(X)[0],
                                     _ptr_mem(Y)[0], _ptr_mem(W)[0], _ptr_mem(V)[0], mem))


def fh_boundary_polygon(ctx, vx, vy, q, B):
    vx = np.ascontiguousarray(vx, dtype=np.float64)
    vy = np.ascontiguousarray(vy, dtype=np.float64)
    X, Y, W, V = _rows4(B)
    mem = _same_mem(X, Y, W, V)
    _check(lib().fh_boundary_polygon(ctx, _ptr_mem(vx)[0], _ptr_mem(vy)[0], len(vx), q, _ptr_mem(X)[0],
                                     _ptr_mem(Y)[0], _ptr_mem(W)[0], _ptr_mem(V)[0], mem))


def fh_boundary_starshade(ctx, Np, a, R, b, p, m, ntip, ngap, B):
    X, Y, W, V = _rows4(B)
    mem = _same_mem(X, Y, W, V)
    _check(lib().fh_boundary_starshade(ctx, Np, a, R, b, p, m, ntip, ngap, _ptr_mem(X)[0], _ptr_mem(Y)[0],
                                       _ptr_mem(W)[0], _ptr_mem(V)[0], mem))


def fh_field_nsli(ctx, B, lam, z, xi, eta, far, occulter, u):
    X, Y, W, V = _rows4(B)
    if len(xi) != len(eta):
        raise ValueError("xi and eta must have the same length")
    mem = _same_mem(X, Y, W, V, xi, eta, u)
    _check(lib().fh_field_nsli(ctx, _ptr_mem(X)[0], _ptr_mem(Y)[0], _ptr_mem(W)[0], _ptr_mem(V)[0], X.shape[0],
                               lam, z, len(xi), _ptr_mem(xi)[0], _ptr_mem(eta)[0], float(far),
                               int(bool(occulter)), _ptr_mem(u)[0], mem))


def fh_field_nsli_noalloc(ctx, B, lam, z, xi, eta, far, occulter, u):
    """As fh_field_nsli, device arrays only; the library allocates nothing."""
    X, Y, W, V = _rows4(B)
    if len(xi) != len(eta):
        raise ValueError("xi and eta must have the same length")
    if _same_mem(X, Y, W, V, xi, eta, u) != FH_MEM_DEVICE:
        raise ValueError("fh_field_nsli_noalloc takes device arrays only")
    _check(lib().fh_field_nsli_noalloc(ctx, _ptr_mem(X)[0], _ptr_mem(Y)[0], _ptr_mem(W)[0], _ptr_mem(V)[0],
                                       X.shape[0], lam, z, len(xi), _ptr_mem(xi)[0], _ptr_mem(eta)[0],
                                       float(far), int(bool(occulter)), _ptr_mem(u)[0]))


def fh_targets_create(ctx, xi, eta, box=None):
    """box: None (bounding box computed) or (xmin, xmax, ymin, ymax)."""
    mem = _same_mem(xi, eta)
    if len(xi) != len(eta):
        raise ValueError("xi and eta must have the same length")
    bx = None if box is None else (ctypes.c_double * 4)(*[float(v) for v in box])
    h = ctypes.c_void_p()
    _check(lib().fh_targets_create(ctx, len(xi), _ptr_mem(xi)[0], _ptr_mem(eta)[0], bx, mem, ctypes.byref(h)))
    return h


def fh_targets_sort(t):
    _check(lib().fh_targets_sort(t))


def fh_targets_size(t) -> int:
    n = ctypes.c_int64()
    _check(lib().fh_targets_size(t, ctypes.byref(n)))
    return n.value


def fh_targets_box(t):
    arr = (ctypes.c_double * 4)()
    _check(lib().fh_targets_box(t, arr))
    return tuple(arr)


def fh_targets_destroy(t):
    _check(lib().fh_targets_destroy(t))


def fh_field_targets(ctx, q, lam, z, t, occulter, u):
    ptr, mem = _ptr_mem(u)
    _check(lib().fh_field_targets(ctx, q, lam, z, t, int(bool(occulter)), ptr, mem))


def fh_field_grid_batch(ctx, quads, lams, zs, n1, n2, h1, h2, xc, yc, occulter, u):
    B = len(quads)
    qarr = (ctypes.c_void_p * B)(*[q.value if isinstance(q, ctypes.c_void_p) else q for q in quads])
    la = np.ascontiguousarray(lams, dtype=np.float64)
    za = np.ascontiguousarray(zs, dtype=np.float64)
    oc = np.ascontiguousarray(np.broadcast_to(np.asarray(occulter, dtype=np.int32), (B,)))
    ptr, mem = _ptr_mem(u)
    if mem != FH_MEM_DEVICE:
        raise ValueError("fh_field_grid_batch writes device memory only")
    _check(lib().fh_field_grid_batch(ctx, B, ctypes.cast(qarr, ctypes.c_void_p), _ptr_mem(la)[0],
                                     _ptr_mem(za)[0], n1, n2, h1, h2, xc, yc, _ptr_mem(oc)[0], ptr))


def fh_field_grid_vjp(ctx, q, lam, z, n1, n2, h1, h2, xc, yc, occulter, g_u, g_x, g_y, g_w):
    for a in (g_u, g_x, g_y, g_w):
        if _ptr_mem(a)[1] != FH_MEM_DEVICE:
            raise ValueError("fh_field_grid_vjp takes device arrays")
    _check(lib().fh_field_grid_vjp(ctx, q, lam, z, n1, n2, h1, h2, xc, yc, int(bool(occulter)),
                                   _ptr_mem(g_u)[0], _ptr_mem(g_x)[0], _ptr_mem(g_y)[0], _ptr_mem(g_w)[0]))


def fh_field_grid_vjp_sum(ctx, q, lams, zs, n1, n2, h1, h2, xc, yc, occulter, g_u, g_x, g_y, g_w):
    for a in (g_u, g_x, g_y, g_w):
        if _ptr_mem(a)[1] != FH_MEM_DEVICE:
            raise ValueError("fh_field_grid_vjp_sum takes device arrays")
    la = np.ascontiguousarray(lams, dtype=np.float64)
    za = np.ascontiguousarray(zs, dtype=np.float64)
    if la.shape != za.shape or la.ndim != 1:
        raise ValueError("lams and zs must be 1-D arrays of one length")
    _check(lib().fh_field_grid_vjp_sum(ctx, q, len(la), _ptr_mem(la)[0], _ptr_mem(za)[0], n1, n2, h1, h2, xc, yc,
                                       int(bool(occulter)), _ptr_mem(g_u)[0], _ptr_mem(g_x)[0], _ptr_mem(g_y)[0],
                                       _ptr_mem(g_w)[0]))


def fh_starshade_vjp(ctx, Np, a, R, b, p, m, np_, nd, md, coef, K, g_x, g_y, g_w, g_coef):
    for t in (coef, g_x, g_y, g_w, g_coef):
        if _ptr_mem(t)[1] != FH_MEM_DEVICE:
            raise ValueError("fh_starshade_vjp takes device arrays")
    _check(lib().fh_starshade_vjp(ctx, Np, a, R, b, p, m, np_, nd, md, _ptr_mem(coef)[0], K,
                                  _ptr_mem(g_x)[0], _ptr_mem(g_y)[0], _ptr_mem(g_w)[0], _ptr_mem(g_coef)[0]))


def fh_autotune_grid(ctx, q, lam, z, n1, n2, h1, h2, cache_path=None):
    best = fh_options()
    cp = cache_path.encode() if cache_path else None
    _check(lib().fh_autotune_grid(ctx, q, lam, z, n1, n2, h1, h2, cp, ctypes.byref(best)))
    return best


def fh_field_grid_batch_rebuild(ctx, quads, lams, zs, n1, n2, h1, h2, xc, yc, occulter, u):
    B = len(quads)
    qarr = (ctypes.c_void_p * B)(*[q.value if isinstance(q, ctypes.c_void_p) else q for q in quads])
    la = np.ascontiguousarray(lams, dtype=np.float64)
    za = np.ascontiguousarray(zs, dtype=np.float64)
    oc = np.ascontiguousarray(np.broadcast_to(np.asarray(occulter, dtype=np.int32), (B,)))
    ptr, mem = _ptr_mem(u)
    if mem != FH_MEM_DEVICE:
        raise ValueError("fh_field_grid_batch_rebuild writes device memory only")
    _check(lib().fh_field_grid_batch_rebuild(ctx, B, ctypes.cast(qarr, ctypes.c_void_p), _ptr_mem(la)[0],
                                             _ptr_mem(za)[0], n1, n2, h1, h2, xc, yc, _ptr_mem(oc)[0], ptr))


def fh_autotune_batch(ctx, quads, lams, zs, n1, n2, h1, h2, cache_path=None):
    B = len(quads)
    qarr = (ctypes.c_void_p * B)(*[q.value if isinstance(q, ctypes.c_void_p) else q for q in quads])
    la = np.ascontiguousarray(lams, dtype=np.float64)
    za = np.ascontiguousarray(zs, dtype=np.float64)
    best = fh_options()
    cp = cache_path.encode() if cache_path else None
    _check(lib().fh_autotune_batch(ctx, B, ctypes.cast(qarr, ctypes.c_void_p), _ptr_mem(la)[0], _ptr_mem(za)[0],
                                   n1, n2, h1, h2, cp, ctypes.byref(best)))
    return best


def fh_set_timing(ctx, enable: bool):
    _check(lib().fh_set_timing(ctx, int(bool(enable))))


def fh_last_timing(ctx):
    arr = (ctypes.c_double * 5)()
    _check(lib().fh_last_timing(ctx, arr))
    return list(arr)


TIMING_GRID, TIMING_POINTS, TIMING_VJP, TIMING_BATCH = 0, 1, 2, 3


def fh_timing_totals(ctx, kind: int, reset: bool = False):
    """(per-stage millisecond sums, number of timed calls) for one call kind."""
    arr = (ctypes.c_double * 5)()
    n = ctypes.c_int64()
    _check(lib().fh_timing_totals(ctx, kind, arr, ctypes.byref(n), int(bool(reset))))
    return list(arr), n.value


def fh_probe_ceilings(ctx):
    """Measured ceilings: {'hbm_copy_gbs', 'lds_add_f32_gbs', 'lds_add_f64_gbs', 'lds_rmw_c128_gbs',
    'lds_rmw_c64_gbs', 'mfma_f64_tflops', 'mfma_f32_tflops'}."""
    arr = (ctypes.c_double * 7)()
    _check(lib().fh_probe_ceilings(ctx, arr))
    return {"hbm_copy_gbs": arr[0], "lds_add_f32_gbs": arr[1], "lds_add_f64_gbs": arr[2],
            "lds_rmw_c128_gbs": arr[3], "lds_rmw_c64_gbs": arr[4], "mfma_f64_tflops": arr[5],
            "mfma_f32_tflops": arr[6]}
