"""torch.autograd.Function wrappers over the library's hand-written adjoint.

Both functions only marshal arguments: the forward field, the type-2 adjoint
and the starshade chain rule all run in libfresnel_hip's HIP kernels.
PyTorch's convention for a real loss L and complex output u is
grad_u = dL/dRe(u) + i dL/dIm(u), which is the cotangent the library takes.
"""
from __future__ import annotations

import torch

from . import _binding as abi


class NodeGridField(torch.autograd.Function):
    """u = field_grid(rule (x, y, w)); gradients with respect to x, y, w."""

    @staticmethod
    def forward(ctx, x, y, w, fctx, lam, z, grid, occulter):
        q = fctx.quad_from_nodes(x.detach().contiguous(), y.detach().contiguous(), w.detach().contiguous())
        u = fctx.field_grid(q, lam, z, grid.n1, grid.n2, grid.h1, grid.h2, grid.xc, grid.yc, occulter)
        ctx.fctx, ctx.q, ctx.args = fctx, q, (lam, z, grid, occulter)
        return u

    @staticmethod
    def backward(ctx, gu):
        lam, z, grid, occulter = ctx.args
        gx, gy, gw = ctx.fctx.field_grid_vjp(ctx.q, lam, z, grid.n1, grid.n2, grid.h1, grid.h2,
                                             gu.contiguous(), grid.xc, grid.yc, occulter)
        return gx, gy, gw, None, None, None, None, None


class StarshadeGridField(torch.autograd.Function):
    """u = field_grid(perturbed starshade rule(coef)); gradient with respect to
    the 2 Np K edge coefficients."""

    @staticmethod
    def forward(ctx, coef, fctx, shape, lam, z, grid, occulter):
        c = coef.detach().contiguous()
        q = fctx.quad_starshade(shape.Np, shape.a, shape.R, shape.b, shape.p, shape.m, shape.np_, shape.nd,
                                shape.md, c, shape.K)
        u = fctx.field_grid(q, lam, z, grid.n1, grid.n2, grid.h1, grid.h2, grid.xc, grid.yc, occulter)
        ctx.fctx, ctx.q, ctx.args = fctx, q, (shape, lam, z, grid, occulter)
        ctx.save_for_backward(c)
        return u

    @staticmethod
    def backward(ctx, gu):
        (c,) = ctx.saved_tensors
        shape, lam, z, grid, occulter = ctx.args
        f = ctx.fctx
        gx, gy, gw = f.field_grid_vjp(ctx.q, lam, z, grid.n1, grid.n2, grid.h1, grid.h2, gu.contiguous(),
                                      grid.xc, grid.yc, occulter)
        gcoef = torch.empty_like(c)
        abi.fh_starshade_vjp(f.handle, shape.Np, shape.a, shape.R, shape.b, shape.p, shape.m, shape.np_, shape.nd,
                             shape.md, c, shape.K, gx, gy, gw, gcoef)
        return gcoef, None, None, None, None, None, None


class StarshadeGridSweep(torch.autograd.Function):
    """u[l] = field_grid(perturbed starshade rule(coef), lams[l], zs[l]) for L
    wavelengths (sec. 4.3's sweep of one rule): the rule is built once and
    the L fields computed in one batched call; the backward pass sums the L
    node gradients in one library call and chains them to the 2 Np K edge
    coefficients once."""

    @staticmethod
    def forward(ctx, coef, fctx, shape, lams, zs, grid, occulter):
        import numpy as np
        c = coef.detach().contiguous()
        q = fctx.quad_starshade(shape.Np, shape.a, shape.R, shape.b, shape.p, shape.m, shape.np_, shape.nd,
                                shape.md, c, shape.K)
        lams = np.asarray(lams, dtype=np.float64)
        zs = np.broadcast_to(np.asarray(zs, dtype=np.float64), lams.shape).copy()
        u = fctx.field_grid_batch([q] * len(lams), lams, zs, grid.n1, grid.n2, grid.h1, grid.h2, grid.xc, grid.yc,
                                  occulter)
        ctx.fctx, ctx.q, ctx.args = fctx, q, (shape, lams, zs, grid, occulter)
        ctx.save_for_backward(c)
        return u

    @staticmethod
    def backward(ctx, gu):
        (c,) = ctx.saved_tensors
        shape, lams, zs, grid, occulter = ctx.args
        f = ctx.fctx
        gx, gy, gw = f.field_grid_vjp_sum(ctx.q, lams, zs, grid.n1, grid.n2, grid.h1, grid.h2, gu.contiguous(),
                                          grid.xc, grid.yc, occulter)
        gcoef = torch.empty_like(c)
        abi.fh_starshade_vjp(f.handle, shape.Np, shape.a, shape.R, shape.b, shape.p, shape.m, shape.np_, shape.nd,
                             shape.md, c, shape.K, gx, gy, gw, gcoef)
        return gcoef, None, None, None, None, None, None


def starshade_sweep(coef, fctx, shape, lams, zs, grid, occulter=True):
    """Fields of one perturbed starshade at several wavelengths (L x n2 x n1)."""
    return StarshadeGridSweep.apply(coef, fctx, shape, lams, zs, grid, occulter)


def starshade_field(coef, fctx, shape, lam, z, grid, occulter=True):
    return StarshadeGridField.apply(coef, fctx, shape, lam, z, grid, occulter)


def node_field(x, y, w, fctx, lam, z, grid, occulter=False):
    return NodeGridField.apply(x, y, w, fctx, lam, z, grid, occulter)
