"""CPU FP64 oracle for areal-quadrature Fresnel diffraction (test infrastructure).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  It wraps ``fresnel_oracle.c`` (plain C, FP64, OpenMP
over targets) through ctypes and shares no source with the GPU library.

What it computes (Barnett, arXiv:2010.05978):
  * Gauss-Legendre rules and the boundary vector line-integral rules (eq. vliq:
    Gauss-Legendre panels in angle, the periodic trapezoid rule of eq. ptr,
    for radial curves and general Fourier curves such as the kite of sec. 3.1;
    polygons with Gauss-Legendre nodes per edge);
  * the dilation areal rule (eqs. aqnod/aqwei, sec. 3.1) and the starshade
    disc + petal rule (sec. 3.2), optionally with lateral edge perturbations,
    either deforming the petals or as the ideal rule plus signed ribbons
    along the edges (sec. 5);
  * the direct quadrature sum (eq. faq) with the Babinet complement (eq. bab),
    also with a source term per node and a spherical incident wave;
  * the exact gradient of that sum with respect to nodes and weights, and its
    chain rule through the perturbed starshade construction;
  * the non-singular line integral over a boundary rule (appendix, eq. nsli),
    with the deep-shadow option of eq. li, and the starshade outline rule.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fresnel_oracle.c")
_LIB = os.path.join(_HERE, "libfresnel_oracle.so")

_dp = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile the oracle shared library in place (gcc -O3, OpenMP).  The
    in-tree library targets x86-64-v3 (AVX2), so that a copy built on one
    host runs on another; the benchmark's CPU baseline builds its own copy
    with -march=native on the host it runs on (build_native)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        _compile(_LIB, "x86-64-v3")
    return _LIB


def _compile(path: str, march: str) -> None:
    tmp = path + ".tmp"
    cmd = ["gcc", "-O3", f"-march={march}", "-fopenmp", "-fPIC", "-shared",
           "-std=c99", "-D_GNU_SOURCE", _SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, path)


def build_native(directory: str) -> str:
    """Compile a -O3 -march=native copy of the oracle into `directory` and use
    it for every later call of this module (the CPU-baseline timing)."""
    global _lib, _LIB
    os.makedirs(directory, exist_ok=True)
    path = os.path.join(directory, "libfresnel_oracle_native.so")
    _compile(path, "native")
    _LIB = path
    _lib = None
    return path


def build_sanitized(directory: str) -> str:
    """Compile an AddressSanitizer + UndefinedBehaviorSanitizer copy of the
    oracle (gcc -O1 -g, no OpenMP, any report aborts) into `directory` and
    use it for every later call of this module.  A process that loads it
    needs the ASan runtime preloaded (its path: gcc -print-file-name=libasan.so)."""
    global _lib, _LIB
    os.makedirs(directory, exist_ok=True)
    path = os.path.join(directory, "libfresnel_oracle_san.so")
    tmp = path + ".tmp"
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fPIC", "-shared", "-std=c99", "-D_GNU_SOURCE", _SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
    os.replace(tmp, path)
    _LIB = path
    _lib = None
    return path


_lib = None


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        i64, i32, d = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        lib.orc_gauss_legendre.argtypes = [i32, _dp, _dp]
        lib.orc_bdry_radial_gl.argtypes = [d, _dp, _dp, i32, i32, i32, _dp, _dp, _dp, _dp]
        lib.orc_bdry_radial_ptr.argtypes = [d, _dp, _dp, i32, i32, _dp, _dp, _dp, _dp]
        lib.orc_bdry_polygon.argtypes = [_dp, _dp, i32, i32, _dp, _dp, _dp, _dp]
        lib.orc_dilation.argtypes = [_dp, _dp, _dp, _dp, i64, i32, _dp, _dp, _dp]
        lib.orc_starshade_size.argtypes = [i32, i32, i32, i32, i32]
        lib.orc_starshade_size.restype = i64
        lib.orc_starshade.argtypes = [i32, d, d, d, d, i32, i32, i32, i32, _dp, i32, _dp, _dp, _dp]
        lib.orc_fresnel_direct.argtypes = [_dp, _dp, _dp, i64, d, d, _dp, _dp, i64, i32, _dp]
        lib.orc_starshade_tab.argtypes = [i32, d, d, _dp, i32, i32, i32, i32, _dp, i32, _dp, _dp, _dp]
        lib.orc_starshade_ribbon_size.argtypes = [i32, i32, i32, i32, i32, i32]
        lib.orc_starshade_ribbon_size.restype = i64
        lib.orc_starshade_ribbon.argtypes = [i32, d, d, d, d, i32, i32, i32, i32, _dp, i32, i32, _dp, _dp, _dp]
        lib.orc_starshade_rigid.argtypes = [i32, d, d, d, d, i32, i32, i32, i32, _dp, i32, i32, _dp, _dp, _dp]
        lib.orc_fresnel_direct_src.argtypes = [_dp, _dp, _dp, _dp, i64, d, d, d, _dp, _dp, i64, i32, _dp]
        lib.orc_fresnel_direct_vjp.argtypes = [_dp, _dp, _dp, i64, d, d, _dp, _dp, i64, i32,
                                               _dp, _dp, _dp, _dp]
        lib.orc_starshade_vjp.argtypes = [i32, d, d, d, d, i32, i32, i32, i32, _dp, i32,
                                          _dp, _dp, _dp, _dp]
        ip = ctypes.POINTER(ctypes.c_int)
        lib.orc_koch_size.argtypes = [i32, ip]
        lib.orc_koch_size.restype = i64
        lib.orc_koch.argtypes = [i32, ip, _dp, _dp, _dp]
        lib.orc_koch_outline.argtypes = [i32, _dp, _dp]
        lib.orc_bdry_fourier.argtypes = [_dp, _dp, _dp, _dp, i32, i32, i32, _dp, _dp, _dp, _dp]
        lib.orc_bdry_starshade.argtypes = [i32, d, d, d, d, i32, i32, i32, _dp, _dp, _dp, _dp]
        lib.orc_nsli.argtypes = [_dp, _dp, _dp, _dp, i64, d, d, _dp, _dp, i64, d, i32, _dp]
        lib.orc_num_threads.restype = i32
        lib.orc_set_threads.argtypes = [i32]
        lib.orc_set_threads.restype = i32
        for name in ("orc_gauss_legendre", "orc_bdry_radial_gl", "orc_bdry_radial_ptr",
                     "orc_bdry_polygon", "orc_dilation", "orc_starshade",
                     "orc_fresnel_direct", "orc_fresnel_direct_vjp", "orc_starshade_vjp",
                     "orc_bdry_starshade", "orc_nsli", "orc_bdry_fourier", "orc_koch", "orc_fresnel_direct_src", "orc_starshade_rigid", "orc_starshade_tab",
                     "orc_koch_outline", "orc_starshade_ribbon"):
            getattr(lib, name).restype = i32
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(n: int) -> None:
    """Run the OpenMP loops on n threads from now on."""
    _load().orc_set_threads(int(n))


# ---------------------------------------------------------------- 1D rules
def gauss_legendre(q: int):
    """q-node Gauss-Legendre rule on [-1, 1] (ascending nodes, weights)."""
    x = np.empty(q)
    w = np.empty(q)
    _check(_load().orc_gauss_legendre(q, _p(x), _p(w)), "gauss_legendre")
    return x, w


# ---------------------------------------------------------- boundary rules
def boundary_radial_gl(r0, a=None, b=None, panels=1, q=20):
    """Vector line rule (eq. vliq) for x(t) = r(t)(cos t, sin t),
    r = r0 + sum_k a_k cos kt + b_k sin kt, GL panels in t.  Returns X, Y, W, V."""
    K = 0 if a is None else len(a)
    a = None if a is None else _f64(a)
    b = None if b is None else _f64(b)
    if a is not None and b is None:
        b = np.zeros(K)
    n = panels * q
    out = np.empty((4, n))
    _check(_load().orc_bdry_radial_gl(r0, _p(a), _p(b), K, panels, q,
                                       _p(out[0]), _p(out[1]), _p(out[2]), _p(out[3])),
           "boundary_radial_gl")
    return out[0], out[1], out[2], out[3]


def boundary_radial_ptr(r0, a=None, b=None, n=100):
    """Periodic trapezoid vector line rule, eq. ptr."""
    K = 0 if a is None else len(a)
    a = None if a is None else _f64(a)
    b = None if b is None else _f64(b)
    if a is not None and b is None:
        b = np.zeros(K)
    out = np.empty((4, n))
    _check(_load().orc_bdry_radial_ptr(r0, _p(a), _p(b), K, n,
                                        _p(out[0]), _p(out[1]), _p(out[2]), _p(out[3])),
           "boundary_radial_ptr")
    return out[0], out[1], out[2], out[3]


def boundary_polygon(vx, vy, q):
    """GL nodes on each straight edge of a CCW polygon."""
    vx, vy = _f64(vx), _f64(vy)
    n = len(vx) * q
    out = np.empty((4, n))
    _check(_load().orc_bdry_polygon(_p(vx), _p(vy), len(vx), q,
                                     _p(out[0]), _p(out[1]), _p(out[2]), _p(out[3])),
           "boundary_polygon")
    return out[0], out[1], out[2], out[3]


def boundary_fourier(ax, bx, ay, by, panels=0, q=100):
    """Vector line rule (eq. vliq1) for the closed curve X(t) = sum_k ax_k cos kt
    + bx_k sin kt, Y(t) likewise, k = 0..K (arrays of length K+1): panels = 0
    is the periodic trapezoid rule of eq. ptr with q nodes, else GL panels."""
    ax, bx, ay, by = (_f64(t) for t in (ax, bx, ay, by))
    K = len(ax) - 1
    if not (len(bx) == len(ay) == len(by) == K + 1):
        raise ValueError("coefficient arrays must have the same length K+1")
    n = panels * q if panels > 0 else q
    out = np.empty((4, n))
    _check(_load().orc_bdry_fourier(_p(ax), _p(bx), _p(ay), _p(by), K, panels, q,
                                     _p(out[0]), _p(out[1]), _p(out[2]), _p(out[3])),
           "boundary_fourier")
    return out[0], out[1], out[2], out[3]


def boundary_starshade(Np, a, R, b, p, m, ntip=4, ngap=0):
    """Outline rule of the starshade (sec. 3.2's petal shape, HG apodisation):
    per petal the lower edge (m GL radii, outward), the tip arc (ntip GL
    angles), the upper edge (inward) and the gap arc at r = a (ngap).
    Returns X, Y, W, V with n = Np (2 m + ntip + ngap)."""
    n = Np * (2 * m + ntip + ngap)
    out = np.empty((4, n))
    _check(_load().orc_bdry_starshade(Np, a, R, b, p, m, ntip, ngap,
                                       _p(out[0]), _p(out[1]), _p(out[2]), _p(out[3])),
           "boundary_starshade")
    return out[0], out[1], out[2], out[3]


def _ints(p):
    a = np.ascontiguousarray(np.asarray(p, dtype=np.intc))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def koch_size(L, p):
    a, pa = _ints(p)
    if len(a) != L + 1:
        raise ValueError("p needs L + 1 entries")
    return int(_load().orc_koch_size(L, pa))


def quad_koch(L, p):
    """Koch snowflake rule of sec. 4.4: level-L construction, the p[k] x p[k]
    dilation rule from a vertex on every level-k triangle; returns x, y, w."""
    a, pa = _ints(p)
    N = koch_size(L, a)
    out = np.empty((3, N))
    _check(_load().orc_koch(L, pa, _p(out[0]), _p(out[1]), _p(out[2])), "koch")
    return out[0], out[1], out[2]


def koch_outline(L):
    """CCW vertices of the level-L snowflake's outline (3 4^L of them)."""
    n = 3 * 4 ** L
    vx, vy = np.empty(n), np.empty(n)
    _check(_load().orc_koch_outline(L, _p(vx), _p(vy)), "koch_outline")
    return vx, vy


def dilation(X, Y, W, V, m):
    """Areal rule of eqs. aqnod/aqwei from a boundary rule; returns x, y, w."""
    X, Y, W, V = (_f64(t) for t in (X, Y, W, V))
    n = len(X)
    out = np.empty((3, n * m))
    _check(_load().orc_dilation(_p(X), _p(Y), _p(W), _p(V), n, m,
                                 _p(out[0]), _p(out[1]), _p(out[2])), "dilation")
    return out[0], out[1], out[2]


def quad_radial(r0, a=None, b=None, panels=1, q=20, m=10):
    return dilation(*boundary_radial_gl(r0, a, b, panels, q), m)


def quad_polygon(vx, vy, q, m):
    return dilation(*boundary_polygon(vx, vy, q), m)


def starshade_size(Np, m, np_, nd, md):
    return int(_load().orc_starshade_size(Np, m, np_, nd, md))


def quad_starshade(Np, a, R, b, p, m, np_, nd, md, coef=None, K=0):
    """Starshade disc + petal rule (sec. 3.2) with HG apodisation
    A(r) = exp(-((r-a)/b)^p) on (a, R); optional edge perturbation coef
    (2*Np*K values, see fresnel_oracle.c)."""
    N = starshade_size(Np, m, np_, nd, md)
    coef = None if coef is None else _f64(coef)
    if coef is not None and coef.size != 2 * Np * K:
        raise ValueError("coef must have 2*Np*K entries")
    out = np.empty((3, N))
    _check(_load().orc_starshade(Np, a, R, b, p, m, np_, nd, md, _p(coef),
                                  K if coef is not None else 0,
                                  _p(out[0]), _p(out[1]), _p(out[2])), "starshade")
    return out[0], out[1], out[2]


def quad_starshade_tab(Np, a, R, A, m, np_, nd, md, coef=None, K=0):
    """Starshade rule with a tabulated apodisation: A[l] = A(r_l) at the m
    Gauss-Legendre radii r_l on (a, R)."""
    A = _f64(A)
    if A.size != m:
        raise ValueError("A needs one value per radial node")
    N = starshade_size(Np, m, np_, nd, md)
    coef = None if coef is None else _f64(coef)
    out = np.empty((3, N))
    _check(_load().orc_starshade_tab(Np, a, R, _p(A), m, np_, nd, md, _p(coef), K if coef is not None else 0,
                                      _p(out[0]), _p(out[1]), _p(out[2])), "starshade_tab")
    return out[0], out[1], out[2]


def quad_starshade_ribbon(Np, a, R, b, p, m, np_, nd, md, coef, K, mr):
    """Ideal starshade plus the signed ribbons between each petal's ideal
    edges and its laterally displaced edges (sec. 5's ribbon construction);
    mr Gauss-Legendre nodes across each ribbon, or mr = 0 for the line
    integral on the ideal edge."""
    coef = _f64(coef)
    N = _load().orc_starshade_ribbon_size(Np, m, np_, nd, md, mr)
    out = np.empty((3, N))
    _check(_load().orc_starshade_ribbon(Np, a, R, b, p, m, np_, nd, md, _p(coef), K, mr,
                                        _p(out[0]), _p(out[1]), _p(out[2])), "starshade_ribbon")
    return out[0], out[1], out[2]


def quad_starshade_rigid(Np, a, R, b, p, m, np_, nd, md, motion, nb, mb):
    """Starshade rule with misaligned rigid petals (sec. 5): motion = Np rows of
    (rotation angle about the origin, tx, ty); the signed bridges between each
    petal's root arc and its moved image get nb x mb GL nodes."""
    motion = _f64(motion).reshape(-1)
    if motion.size != 3 * Np:
        raise ValueError("motion needs 3 values per petal")
    N = starshade_size(Np, m, np_, nd, md) + Np * nb * mb
    out = np.empty((3, N))
    _check(_load().orc_starshade_rigid(Np, a, R, b, p, m, np_, nd, md, _p(motion), nb, mb,
                                        _p(out[0]), _p(out[1]), _p(out[2])), "starshade_rigid")
    return out[0], out[1], out[2]


# --------------------------------------------------------------- the sum
def grid_targets(n1, n2, h1, h2, xc=0.0, yc=0.0):
    """Grid targets (xc + h1 k1, yc + h2 k2), -n/2 <= k < n/2, k1 fastest
    (the uniform target grid of sec. 2.2)."""
    k1 = np.arange(-(n1 // 2), n1 - n1 // 2)
    k2 = np.arange(-(n2 // 2), n2 - n2 // 2)
    XI, ETA = np.meshgrid(xc + h1 * k1, yc + h2 * k2, indexing="xy")
    return XI.ravel().copy(), ETA.ravel().copy()


def fresnel_direct(x, y, w, lam, z, xi, eta, occulter=False):
    """Direct sum (eq. faq), Babinet (eq. bab) if occulter; complex128 array."""
    x, y, w, xi, eta = (_f64(t) for t in (x, y, w, xi, eta))
    M = len(xi)
    u = np.empty(2 * M)
    _check(_load().orc_fresnel_direct(_p(x), _p(y), _p(w), len(x), lam, z,
                                       _p(xi), _p(eta), M, int(bool(occulter)), _p(u)),
           "fresnel_direct")
    return u.view(np.complex128)


def fresnel_direct_src(x, y, w, lam, z, xi, eta, src=None, D=0.0, occulter=False):
    """Direct sum with a complex source term s_j per node (None: 1) and a
    spherical incident wave exp(i pi |x|^2/(lam D)) (D <= 0: plane wave)."""
    x, y, w, xi, eta = (_f64(t) for t in (x, y, w, xi, eta))
    sp = None
    if src is not None:
        sp = np.ascontiguousarray(np.asarray(src, dtype=np.complex128)).view(np.float64)
        if sp.size != 2 * len(x):
            raise ValueError("src needs one complex value per node")
    M = len(xi)
    u = np.empty(2 * M)
    _check(_load().orc_fresnel_direct_src(_p(x), _p(y), _p(w), _p(sp), len(x), lam, z, float(D),
                                           _p(xi), _p(eta), M, int(bool(occulter)), _p(u)),
           "fresnel_direct_src")
    return u.view(np.complex128)


def fresnel_direct_vjp(x, y, w, lam, z, xi, eta, g, occulter=False):
    """Gradient (dL/dx, dL/dy, dL/dw) of a real loss through the direct sum,
    given g = dL/dRe(u) + i dL/dIm(u) at the targets."""
    x, y, w, xi, eta = (_f64(t) for t in (x, y, w, xi, eta))
    g = np.ascontiguousarray(np.asarray(g, dtype=np.complex128)).view(np.float64)
    N = len(x)
    gx, gy, gw = np.empty(N), np.empty(N), np.empty(N)
    _check(_load().orc_fresnel_direct_vjp(_p(x), _p(y), _p(w), N, lam, z, _p(xi), _p(eta),
                                           len(xi), int(bool(occulter)), _p(g),
                                           _p(gx), _p(gy), _p(gw)), "fresnel_direct_vjp")
    return gx, gy, gw


def starshade_vjp(Np, a, R, b, p, m, np_, nd, md, coef, K, gx, gy, gw):
    """Chain (dL/dx, dL/dy, dL/dw) through the perturbed starshade rule to the
    2*Np*K edge coefficients."""
    coef = _f64(coef)
    gx, gy, gw = _f64(gx), _f64(gy), _f64(gw)
    out = np.empty(2 * Np * K)
    _check(_load().orc_starshade_vjp(Np, a, R, b, p, m, np_, nd, md, _p(coef), K,
                                      _p(gx), _p(gy), _p(gw), _p(out)), "starshade_vjp")
    return out


def nsli(X, Y, W, V, lam, z, xi, eta, far=0.0, occulter=False):
    """Non-singular line integral (appendix, eq. nsli) at targets (xi, eta)
    from a CCW vector line rule (X, Y, W, V); with far > 0, targets at least
    that far from every node use eq. li with the integer winding number
    (the deep-shadow remark).  Babinet if occulter; complex128 array."""
    X, Y, W, V, xi, eta = (_f64(t) for t in (X, Y, W, V, xi, eta))
    M = len(xi)
    u = np.empty(2 * M)
    _check(_load().orc_nsli(_p(X), _p(Y), _p(W), _p(V), len(X), lam, z, _p(xi), _p(eta), M,
                            float(far), int(bool(occulter)), _p(u)), "nsli")
    return u.view(np.complex128)
