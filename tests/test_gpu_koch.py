"""Koch snowflake (sec. 4.4) on the GPU vs the CPU FP64 oracle.

The device rule (fh_quad_koch) node by node against the oracle's
construction, fields of a small snowflake element by element, and the
paper-scale case -- level 13, about 68 million nodes, the type-1 field at
lambda z = 0.01 on a 1000^2 grid at tolerance 1e-6, in the launch shape the
benchmark times -- on sampled targets against the oracle's direct sum over
its own level-13 rule.
"""
import math

import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def koch_orders(L):
    """Rule orders per level for the paper-scale snowflake: 217 on the first
    triangle, halving per level with a floor of 2, and 1 from level 10 on."""
    return [max(2, math.ceil(217 / 2 ** k)) if k <= 9 else 1 for k in range(L + 1)]


def relL2(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def cpu(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def fh():
    import paper_2010_05978_amd as fh
    return fh


def test_koch_rule_matches_oracle(fh):
    print("koch rule", flush=True)
    ctx = fh.Context("fp64")
    for L, p in ((0, [5]), (2, [4, 3, 2]), (5, [6, 5, 4, 3, 2, 1])):
        q = ctx.quad_koch(L, p)
        x, y, w = (cpu(t) for t in q.export())
        rx, ry, rw = oracle.quad_koch(L, p)
        assert len(x) == len(rx)
        assert max(np.abs(x - rx).max(), np.abs(y - ry).max(), np.abs(w - rw).max()) < 1e-14, (L, p)
        q.close()
    with pytest.raises(fh.FresnelError, match="FH_ERR_INVALID_ARG"):
        ctx.quad_koch(2, [3, 0, 1])
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_koch_fields_level4(fh, prec):
    print(f"koch fields level 4 {prec}", flush=True)
    ctx = fh.Context(prec)
    L, p, lz = 4, [80, 40, 24, 14, 8], 0.1
    q = ctx.quad_koch(L, p)
    x, y, w = oracle.quad_koch(L, p)
    n, h = 128, 0.02
    u = cpu(ctx.field_grid(q, 1.0, lz, n, n, h, h, occulter=True)).ravel()
    xi, eta = oracle.grid_targets(n, n, h, h)
    ref = oracle.fresnel_direct(x, y, w, 1.0, lz, xi, eta, occulter=True)
    tol = 1e-9 if prec == "fp64" else 1e-5
    assert relL2(1 - u, 1 - ref) < tol
    g = np.random.Generator(np.random.PCG64(4))
    xr, er = g.uniform(-1.4, 1.4, 3000), g.uniform(-1.4, 1.4, 3000)
    v = cpu(ctx.field_points(q, 1.0, lz, torch.tensor(xr, device="cuda"), torch.tensor(er, device="cuda")))
    refv = oracle.fresnel_direct(x, y, w, 1.0, lz, xr, er)
    assert relL2(v, refv) < tol
    ctx.close()


def test_koch_level13_grid_sampled(fh):
    L, lz, n, h = 13, 0.01, 1000, 0.003
    p = koch_orders(L)
    ctx = fh.Context("fp64", tol=1e-6)
    q = ctx.quad_koch(L, p)
    print(f"koch level 13: {q.N} nodes, type-1 field on {n}^2", flush=True)
    assert q.N == oracle.koch_size(L, p)
    u = cpu(ctx.field_grid(q, 1.0, lz, n, n, h, h)).ravel()
    q.close()
    ctx.close()
    assert np.isfinite(u).all()
    print("koch level 13: oracle rule and direct sum at 16 targets", flush=True)
    x, y, w = oracle.quad_koch(L, p)
    xi, eta = oracle.grid_targets(n, n, h, h)
    idx = np.random.Generator(np.random.PCG64(13)).choice(len(xi), 16, replace=False)
    ref = oracle.fresnel_direct(x, y, w, 1.0, lz, xi[idx], eta[idx])
    assert relL2(u[idx], ref) < 1e-6
