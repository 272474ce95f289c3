"""MI355X-native fast Fresnel diffraction (Barnett, arXiv:2010.05978).

The compute path lives in ``libfresnel_hip.so`` (HIP kernels for gfx950 plus
rocFFT) behind the C ABI of ``include/fresnel_hip.h``.  This package is the
Python binding: ``_binding`` mirrors the C entry points one to one, and
``Context``/``Quad`` below only allocate torch tensors for outputs and pass
pointers and the current torch stream through.  There is no fallback: if the
library is missing, using the package raises.
"""
from __future__ import annotations

from ._binding import (  # noqa: F401
    EXPORTED, FH_ERR_ALLOC, FH_ERR_FFT, FH_ERR_HIP, FH_ERR_INVALID_ARG, FH_ERR_NONFINITE,
    FH_ERR_NONPOSITIVE_LZ, FH_ERR_ODD_GRID, FH_ERR_UNSUPPORTED, FH_FP64, FH_MEM_DEVICE, FH_MEM_HOST,
    FH_MIXED, FH_OK, LIB_PATH, FresnelError, fh_options, lib,
)
from . import _binding as abi  # noqa: F401

__all__ = ["Context", "Quad", "Targets", "FresnelError", "fh_options", "abi", "lib", "LIB_PATH"]


class Quad:
    """A device-resident areal quadrature rule owned by the library."""

    def __init__(self, ctx: "Context", handle):
        self.ctx = ctx
        self.handle = handle

    @property
    def N(self) -> int:
        return abi.fh_quad_size(self.handle)

    def set_illumination(self, src=None, D: float = 0.0):
        """Source term per node (N complex, or None) and point-source distance D (0: plane wave)."""
        if src is not None and len(src) != self.N:
            raise ValueError(f"src needs {self.N} values")
        abi.fh_quad_set_illumination(self.ctx.handle, self.handle, src, D)
        return self

    def export(self):
        """(x, y, w) as float64 device tensors (copies)."""
        import torch
        n = self.N
        out = [torch.empty(n, dtype=torch.float64, device=self.ctx.device) for _ in range(3)]
        abi.fh_quad_export(self.handle, *out)
        return tuple(out)

    def close(self):
        # a rule's device memory belongs to its context; once the context is
        # gone there is nothing left to release
        if self.handle is not None and self.ctx.handle is not None:
            abi.fh_quad_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Targets:
    """Scattered targets and their planning box for repeated type-3 calls
    (device arrays are referenced: keep them alive and unchanged)."""

    def __init__(self, ctx: "Context", handle):
        self.ctx = ctx
        self.handle = handle

    @property
    def M(self) -> int:
        return abi.fh_targets_size(self.handle)

    @property
    def box(self):
        return abi.fh_targets_box(self.handle)

    def sort(self):
        """Evaluate in spatial order from now on (results keep the given order)."""
        abi.fh_targets_sort(self.handle)
        return self

    def close(self):
        if self.handle is not None and self.ctx.handle is not None:
            abi.fh_targets_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """A library context bound to the current torch stream of one GPU."""

    def __init__(self, precision: str = "fp64", tol: float | None = None, device: int = 0,
                 options: fh_options | None = None):
        import torch
        if precision not in ("fp64", "mixed"):
            raise ValueError("precision must be 'fp64' or 'mixed'")
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible to torch")
        self.precision = precision
        self.tol = tol if tol is not None else (1e-9 if precision == "fp64" else 1e-5)
        self.device = torch.device("cuda", device)
        self.cdtype = torch.complex128 if precision == "fp64" else torch.complex64
        self.handle = abi.fh_create(device, FH_FP64 if precision == "fp64" else FH_MIXED, self.tol, options)
        abi.fh_set_stream(self.handle, torch.cuda.current_stream(self.device))

    # ------------------------------------------------------- quadrature
    def quad_radial(self, r0, a=None, b=None, panels=1, q=20, m=10) -> Quad:
        return Quad(self, abi.fh_quad_radial(self.handle, r0, a, b, panels, q, m))

    def quad_fourier(self, ax, bx, ay, by, panels=0, q=100, m=10) -> Quad:
        """Rule for the closed curve X = sum ax_k cos kt + bx_k sin kt, Y likewise."""
        return Quad(self, abi.fh_quad_fourier(self.handle, ax, bx, ay, by, panels, q, m))

    def quad_starshade_tab(self, Np, a, R, A, m, np_, nd, md, coef=None, K=0) -> Quad:
        """Starshade with a tabulated apodisation A[l] = A(r_l) at the m radial Gauss nodes."""
        return Quad(self, abi.fh_quad_starshade_tab(self.handle, Np, a, R, A, m, np_, nd, md, coef, K))

    def quad_starshade_ribbon(self, Np, a, R, b, p, m, np_, nd, md, coef, K, mr=2) -> Quad:
        """Ideal starshade plus signed ribbons along the displaced petal edges (sec. 5);
        mr nodes across each ribbon, or mr = 0 for the line integral on the ideal edge."""
        return Quad(self, abi.fh_quad_starshade_ribbon(self.handle, Np, a, R, b, p, m, np_, nd, md, coef, K, mr))

    def quad_starshade_rigid(self, Np, a, R, b, p, m, np_, nd, md, motion, nb=16, mb=4) -> Quad:
        """Starshade whose petals moved rigidly (motion: Np rows of angle, tx, ty)."""
        return Quad(self, abi.fh_quad_starshade_rigid(self.handle, Np, a, R, b, p, m, np_, nd, md, motion, nb, mb))

    def quad_koch(self, L, p) -> Quad:
        """Koch snowflake rule (level L, p[k] x p[k] nodes per level-k triangle)."""
        return Quad(self, abi.fh_quad_koch(self.handle, L, p))

    def quad_polygon(self, vx, vy, q, m) -> Quad:
        return Quad(self, abi.fh_quad_polygon(self.handle, vx, vy, q, m))

    def quad_starshade(self, Np, a, R, b, p, m, np_, nd, md, coef=None, K=0) -> Quad:
        return Quad(self, abi.fh_quad_starshade(self.handle, Np, a, R, b, p, m, np_, nd, md, coef, K))

    def quad_from_boundary(self, X, Y, W, V, m) -> Quad:
        return Quad(self, abi.fh_quad_from_boundary(self.handle, X, Y, W, V, m))

    def quad_from_nodes(self, x, y, w) -> Quad:
        return Quad(self, abi.fh_quad_from_nodes(self.handle, x, y, w))

    def quad_for(self, shape) -> Quad:
        """Rule for a shape description with the attributes of workloads.py's
        RadialCurve / Polygon / Starshade."""
        kind = type(shape).__name__
        if kind == "RadialCurve":
            a = shape.a if len(shape.a) else None
            b = shape.b if len(shape.b) else None
            return self.quad_radial(shape.r0, a, b, shape.panels, shape.q, shape.m)
        if kind == "Polygon":
            return self.quad_polygon(shape.vx, shape.vy, shape.q, shape.m)
        if kind == "Starshade":
            return self.quad_starshade(shape.Np, shape.a, shape.R, shape.b, shape.p, shape.m, shape.np_,
                                       shape.nd, shape.md, shape.coef, shape.K)
        raise TypeError(f"unknown shape {kind}")

    # ------------------------------------------------- boundary rules
    # A boundary rule is a (4, n) float64 device tensor: rows X, Y, W, V.
    def _bdry(self, n):
        import torch
        return torch.empty((4, n), dtype=torch.float64, device=self.device)

    def boundary_radial(self, r0, a=None, b=None, panels=1, q=20):
        B = self._bdry(panels * q if panels > 0 else q)
        abi.fh_boundary_radial(self.handle, r0, a, b, panels, q, B)
        return B

    def boundary_fourier(self, ax, bx, ay, by, panels=0, q=100):
        B = self._bdry(panels * q if panels > 0 else q)
        abi.fh_boundary_fourier(self.handle, ax, bx, ay, by, panels, q, B)
        return B

    def boundary_polygon(self, vx, vy, q):
        B = self._bdry(len(vx) * q)
        abi.fh_boundary_polygon(self.handle, vx, vy, q, B)
        return B

    def boundary_starshade(self, Np, a, R, b, p, m, ntip=4, ngap=0):
        B = self._bdry(Np * (2 * m + ntip + ngap))
        abi.fh_boundary_starshade(self.handle, Np, a, R, b, p, m, ntip, ngap, B)
        return B

    def targets(self, xi, eta, box=None) -> Targets:
        """Target set for repeated type-3 calls; box = (xmin, xmax, ymin, ymax)
        declares the region (no readback), None computes it."""
        t = Targets(self, abi.fh_targets_create(self.handle, xi, eta, box))
        t._keep = (xi, eta)  # device arrays are used in place
        return t

    # ------------------------------------------------------------ fields
    def field_grid(self, quad: Quad, lam, z, n1, n2, h1, h2, xc=0.0, yc=0.0, occulter=False, out=None):
        import torch
        if out is None:
            out = torch.empty((n2, n1), dtype=self.cdtype, device=self.device)
        abi.fh_field_grid(self.handle, quad.handle, lam, z, n1, n2, h1, h2, xc, yc, occulter, out)
        return out

    def field_points(self, quad: Quad, lam, z, xi, eta, occulter=False, out=None):
        import torch
        if out is None:
            dev = xi.device if hasattr(xi, "device") else self.device
            out = torch.empty(len(xi), dtype=self.cdtype, device=dev)
        abi.fh_field_points(self.handle, quad.handle, lam, z, xi, eta, occulter, out)
        return out

    def field_targets(self, quad: Quad, lam, z, targets: Targets, occulter=False, out=None):
        import torch
        if out is None:
            out = torch.empty(targets.M, dtype=self.cdtype, device=self.device)
        abi.fh_field_targets(self.handle, quad.handle, lam, z, targets.handle, occulter, out)
        return out

    def field_nsli(self, B, lam, z, xi, eta, far=0.0, occulter=False, out=None):
        """Edge-integral field (eq. nsli) from a boundary rule B (4 x n)."""
        import torch
        if out is None:
            dev = xi.device if hasattr(xi, "device") else self.device
            out = torch.empty(len(xi), dtype=self.cdtype, device=dev)
        abi.fh_field_nsli(self.handle, B, lam, z, xi, eta, far, occulter, out)
        return out

    def field_grid_batch(self, quads, lams, zs, n1, n2, h1, h2, xc=0.0, yc=0.0, occulter=False, out=None):
        import torch
        if out is None:
            out = torch.empty((len(quads), n2, n1), dtype=self.cdtype, device=self.device)
        abi.fh_field_grid_batch(self.handle, [q.handle for q in quads], lams, zs, n1, n2, h1, h2, xc, yc,
                                occulter, out)
        return out

    def field_grid_batch_rebuild(self, quads, lams, zs, n1, n2, h1, h2, xc=0.0, yc=0.0, occulter=False, out=None):
        """field_grid_batch with every rule rebuilt on the device first, inside
        the same captured graph (radial and polygon rules only)."""
        import torch
        if out is None:
            out = torch.empty((len(quads), n2, n1), dtype=self.cdtype, device=self.device)
        abi.fh_field_grid_batch_rebuild(self.handle, [q.handle for q in quads], lams, zs, n1, n2, h1, h2, xc, yc,
                                        occulter, out)
        return out

    def field_grid_vjp(self, quad: Quad, lam, z, n1, n2, h1, h2, g_u, xc=0.0, yc=0.0, occulter=False):
        import torch
        n = quad.N
        gx, gy, gw = (torch.empty(n, dtype=torch.float64, device=self.device) for _ in range(3))
        abi.fh_field_grid_vjp(self.handle, quad.handle, lam, z, n1, n2, h1, h2, xc, yc, occulter,
                              g_u.contiguous(), gx, gy, gw)
        return gx, gy, gw

    def field_grid_vjp_sum(self, quad: Quad, lams, zs, n1, n2, h1, h2, g_u, xc=0.0, yc=0.0, occulter=False):
        """Node gradients summed over wavelengths; g_u holds one cotangent plane per wavelength."""
        import torch
        n = quad.N
        gx, gy, gw = (torch.empty(n, dtype=torch.float64, device=self.device) for _ in range(3))
        abi.fh_field_grid_vjp_sum(self.handle, quad.handle, lams, zs, n1, n2, h1, h2, xc, yc, occulter,
                                  g_u.contiguous(), gx, gy, gw)
        return gx, gy, gw

    def autotune_grid(self, quad: Quad, lam, z, n1, n2, h1, h2, cache_path=None) -> fh_options:
        """Time the grid field over the tuning space and keep the fastest options."""
        return abi.fh_autotune_grid(self.handle, quad.handle, lam, z, n1, n2, h1, h2, cache_path)

    def autotune_batch(self, quads, lams, zs, n1, n2, h1, h2, cache_path=None) -> fh_options:
        """Time the batched call (graph capture and replay) over the tuning
        space and keep the fastest options; keyed by the batch's signature."""
        return abi.fh_autotune_batch(self.handle, [q.handle for q in quads], lams, zs, n1, n2, h1, h2, cache_path)

    def query_params(self, n):
        return abi.fh_query_params(self.handle, n)

    def set_options(self, options: fh_options | None):
        abi.fh_set_options(self.handle, options)

    def synchronize(self):
        abi.fh_synchronize(self.handle)

    def order_after(self, other: "Context"):
        """Work enqueued later here waits for the work enqueued so far on other."""
        abi.fh_order_after(self.handle, other.handle)

    def last_timing(self):
        return abi.fh_last_timing(self.handle)

    def set_timing(self, enable: bool):
        abi.fh_set_timing(self.handle, enable)

    def timing_totals(self, kind: int, reset: bool = False):
        return abi.fh_timing_totals(self.handle, kind, reset)

    def probe_ceilings(self):
        """Measured HBM copy and LDS rates of this device (roofline denominators)."""
        return abi.fh_probe_ceilings(self.handle)

    def close(self):
        if self.handle is not None:
            abi.fh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
