"""Target sets (fh_targets_create / fh_field_targets) vs the CPU FP64 oracle.

A target set holds scattered targets (device arrays in place, or a copy of
host arrays) with a planning box that is either declared (no device work and
no host synchronisation) or computed.  Every comparison is element by
element.  Bars as in test_gpu_parity.py.
"""
import math

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-9, "mixed": 1e-5}


def relL2(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def cpu(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def fh():
    import paper_2010_05978_amd as fh
    return fh


@pytest.fixture(scope="module", params=["fp64", "mixed"])
def ctx(request, fh):
    c = fh.Context(request.param)
    yield c
    c.close()


def rule(shape):
    return oracle.quad_radial(shape.r0, shape.a if len(shape.a) else None, shape.b if len(shape.b) else None,
                              shape.panels, shape.q, shape.m)


def test_workload2_declared_box_sampled(ctx):
    wl = workloads.workload(2)
    xi, eta = wl.points
    print(f"target set workload 2 {ctx.precision}", flush=True)
    q = ctx.quad_for(wl.shape)
    dxi, deta = torch.tensor(xi, device="cuda"), torch.tensor(eta, device="cuda")
    tg = ctx.targets(dxi, deta, box=(-1.5, 1.5, -1.5, 1.5))
    assert tg.M == len(xi) and tg.box == (-1.5, 1.5, -1.5, 1.5)
    u = cpu(ctx.field_targets(q, wl.lam, wl.z, tg))
    rng = np.random.Generator(np.random.PCG64(198))
    idx = rng.choice(len(xi), 3000, replace=False)
    x, y, w = rule(wl.shape)
    ref = oracle.fresnel_direct(x, y, w, wl.lam, wl.z, xi[idx], eta[idx])
    err = relL2(u[idx], ref)
    print(f"  rel L2 (3000 samples) = {err:.3e}", flush=True)
    assert err <= TOL[ctx.precision]
    # the one-shot call (computed box) gives the same field
    up = cpu(ctx.field_points(q, wl.lam, wl.z, dxi, deta))
    assert relL2(u, up) <= 2 * TOL[ctx.precision]
    tg.close()


@pytest.mark.parametrize("M", [1, 63, 64, 65, 777, 4099])
def test_small_sets_full(ctx, M):
    # ragged sizes around the 64-target wavefront chunk, whole output compared
    wl = workloads.workload(1)
    g = np.random.Generator(np.random.PCG64(1000 + M))
    xi = g.uniform(-1.7, 0.9, M)
    eta = g.uniform(-0.4, 1.3, M)
    q = ctx.quad_for(wl.shape)
    x, y, w = rule(wl.shape)
    ref = oracle.fresnel_direct(x, y, w, wl.lam, wl.z, xi, eta)
    for box in (None, (-1.7, 0.9, -0.4, 1.3)):
        tg = ctx.targets(torch.tensor(xi, device="cuda"), torch.tensor(eta, device="cuda"), box=box)
        u = cpu(ctx.field_targets(q, wl.lam, wl.z, tg))
        if M == 1:
            assert abs(u[0] - ref[0]) <= 10 * TOL[ctx.precision] * max(1.0, abs(ref[0]))
        else:
            assert relL2(u, ref) <= TOL[ctx.precision], (M, box)
        tg.close()


def test_host_arrays_and_host_output(fh, ctx):
    wl = workloads.workload(1)
    g = np.random.Generator(np.random.PCG64(7))
    M = 1500
    xi = g.uniform(-1.2, 1.2, M)
    eta = g.uniform(-1.2, 1.2, M)
    q = ctx.quad_for(wl.shape)
    x, y, w = rule(wl.shape)
    ref = oracle.fresnel_direct(x, y, w, wl.lam, wl.z, xi, eta)
    tg = ctx.targets(xi, eta)  # host arrays, computed box
    b = tg.box
    assert b[0] == xi.min() and b[1] == xi.max() and b[2] == eta.min() and b[3] == eta.max()
    uh = np.empty(M, dtype=np.complex128 if ctx.precision == "fp64" else np.complex64)
    fh.abi.fh_field_targets(ctx.handle, q.handle, wl.lam, wl.z, tg.handle, True, uh)
    assert relL2(1 - uh, ref) <= TOL[ctx.precision]
    tg.close()


def test_one_set_many_wavelengths_and_shapes(ctx):
    # the sweep pattern: one target set, several wavelengths and rules
    wl = workloads.workload(2)
    M = 2000
    xi, eta = wl.points[0][:M], wl.points[1][:M]
    tg = ctx.targets(torch.tensor(xi, device="cuda"), torch.tensor(eta, device="cuda"),
                     box=(-1.5, 1.5, -1.5, 1.5))
    shapes = [workloads.RadialCurve(1.0, wl.shape.a, wl.shape.b, panels=10, q=16, m=50),
              workloads.RadialCurve(0.8, np.zeros(0), np.zeros(0), panels=6, q=20, m=40)]
    for s in shapes:
        q = ctx.quad_for(s)
        x, y, w = rule(s)
        for lz in (0.05, 0.0845, 0.2):
            lam = 6e-7
            u = cpu(ctx.field_targets(q, lam, lz / lam, tg))
            ref = oracle.fresnel_direct(x, y, w, lam, lz / lam, xi, eta)
            assert relL2(u, ref) <= TOL[ctx.precision], (s.r0, lz)
        q.close()
    tg.close()


def test_outside_box_and_nonfinite_give_nan(fh, ctx):
    wl = workloads.workload(1)
    xi = np.array([0.1, 2.0, -0.3, float("nan"), 0.5])
    eta = np.array([0.2, 0.0, 0.4, 0.1, float("inf")])
    q = ctx.quad_for(wl.shape)
    tg = ctx.targets(torch.tensor(xi, device="cuda"), torch.tensor(eta, device="cuda"), box=(-1, 1, -1, 1))
    u = cpu(ctx.field_targets(q, wl.lam, wl.z, tg))
    bad = np.array([False, True, False, True, True])
    assert np.all(np.isnan(u[bad]))
    x, y, w = rule(wl.shape)
    ref = oracle.fresnel_direct(x, y, w, wl.lam, wl.z, xi[~bad], eta[~bad])
    assert relL2(u[~bad], ref) <= TOL[ctx.precision]
    tg.close()
    # without a declared box a non-finite target is an error
    with pytest.raises(fh.FresnelError) as e:
        ctx.targets(torch.tensor(xi, device="cuda"), torch.tensor(eta, device="cuda"))
    assert e.value.status == fh.FH_ERR_NONFINITE


def test_empty_set_and_empty_rule(fh, ctx):
    wl = workloads.workload(1)
    q = ctx.quad_for(wl.shape)
    z0 = torch.zeros(0, dtype=torch.float64, device="cuda")
    tg = ctx.targets(z0, z0, box=(0, 0, 0, 0))
    assert tg.M == 0
    u = ctx.field_targets(q, wl.lam, wl.z, tg)
    assert u.numel() == 0
    tg.close()
    e = ctx.quad_from_nodes(np.zeros(0), np.zeros(0), np.zeros(0))
    xi = torch.linspace(-1, 1, 9, dtype=torch.float64, device="cuda")
    tg = ctx.targets(xi, xi)
    assert np.all(cpu(ctx.field_targets(e, 1.0, 1.0, tg, occulter=True)) == 1)
    assert np.all(cpu(ctx.field_targets(e, 1.0, 1.0, tg)) == 0)
    tg.close()


def test_bad_boxes(fh, ctx):
    xi = torch.zeros(3, dtype=torch.float64, device="cuda")
    with pytest.raises(fh.FresnelError) as e:
        ctx.targets(xi, xi, box=(1.0, -1.0, 0.0, 1.0))
    assert e.value.status == fh.FH_ERR_INVALID_ARG
    with pytest.raises(fh.FresnelError) as e:
        ctx.targets(xi, xi, box=(0.0, math.inf, 0.0, 1.0))
    assert e.value.status == fh.FH_ERR_NONFINITE


def test_pipelined_contexts_with_order_after(fh, ctx):
    # the bench step's pattern: a target set and its field on one context's
    # stream, the rule and the grid field on another, ordered by
    # fh_order_after in both directions, repeated so that pooled memory is
    # reused across steps
    wl = workloads.workload(2)
    g = wl.grid
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        other = fh.Context(ctx.precision)
    try:
        M = 4000
        xi = torch.tensor(wl.points[0][:M], device="cuda")
        eta = torch.tensor(wl.points[1][:M], device="cuda")
        up = torch.empty(M, dtype=ctx.cdtype, device="cuda")
        ug = torch.empty((160, 160), dtype=ctx.cdtype, device="cuda")
        for _ in range(4):
            tg = other.targets(xi, eta, box=(-1.5, 1.5, -1.5, 1.5))
            q = ctx.quad_for(wl.shape)
            other.order_after(ctx)
            ctx.field_grid(q, wl.lam, wl.z, 160, 160, g.h1, g.h2, out=ug)
            other.field_targets(q, wl.lam, wl.z, tg, out=up)
            ctx.order_after(other)
            q.close()
            tg.close()
        torch.cuda.synchronize()
        x, y, w = rule(wl.shape)
        ref = oracle.fresnel_direct(x, y, w, wl.lam, wl.z, wl.points[0][:M], wl.points[1][:M])
        assert relL2(cpu(up), ref) <= TOL[ctx.precision]
        xs, ys = oracle.grid_targets(160, 160, g.h1, g.h2)
        rng = np.random.Generator(np.random.PCG64(11))
        idx = rng.choice(len(xs), 400, replace=False)
        refg = oracle.fresnel_direct(x, y, w, wl.lam, wl.z, xs[idx], ys[idx])
        assert relL2(cpu(ug).ravel()[idx], refg) <= TOL[ctx.precision]
    finally:
        other.close()


def test_sorted_target_sets(ctx):
    # fh_targets_sort: evaluation in spatial order, results in the caller's order
    print(f"sorted target sets {ctx.precision}", flush=True)
    wl = workloads.workload(2)
    q = ctx.quad_for(wl.shape)
    g = np.random.Generator(np.random.PCG64(321))
    M = 20011
    xi, eta = g.uniform(-1.5, 1.5, M), g.uniform(-1.5, 1.5, M)
    xi[7], eta[7] = 2.5, 0.0        # outside the declared box: NaN
    xi[8] = np.nan                  # non-finite: NaN
    dxi, deta = torch.tensor(xi, device="cuda"), torch.tensor(eta, device="cuda")
    box = (-1.5, 1.5, -1.5, 1.5)
    plain = cpu(ctx.field_targets(q, wl.lam, wl.z, ctx.targets(dxi, deta, box=box)))
    tg = ctx.targets(dxi, deta, box=box).sort()
    tg.sort()  # a second sort is a no-op
    u = cpu(ctx.field_targets(q, wl.lam, wl.z, tg))
    ok = np.ones(M, bool)
    ok[[7, 8]] = False
    assert np.isnan(u[~ok]).all() and np.isfinite(u[ok]).all()
    assert relL2(u[ok], plain[ok]) < (1e-14 if ctx.precision == "fp64" else 1e-6)
    idx = np.random.Generator(np.random.PCG64(5)).choice(np.flatnonzero(ok), 1500, replace=False)
    x, y, w = rule(wl.shape)
    ref = oracle.fresnel_direct(x, y, w, wl.lam, wl.z, xi[idx], eta[idx])
    assert relL2(u[idx], ref) < TOL[ctx.precision]
    # the sorted set keeps its own copy: the caller's arrays may change
    dxi.fill_(0.0)
    u2 = cpu(ctx.field_targets(q, wl.lam, wl.z, tg, occulter=True))
    assert relL2(1 - u2[ok], u[ok]) < (1e-14 if ctx.precision == "fp64" else 1e-6)
    tg.close()
    # host arrays, and tiny sets
    th = ctx.targets(xi[:1000].copy(), eta[:1000].copy(), box=box).sort()
    uh = cpu(ctx.field_targets(q, wl.lam, wl.z, th))
    fin = np.isfinite(plain[:1000])
    assert relL2(uh[fin], plain[:1000][fin]) < (1e-14 if ctx.precision == "fp64" else 1e-6)
    th.close()
    t1 = ctx.targets(dxi[:1], deta[:1], box=box).sort()
    assert t1.M == 1
    t1.close()
    q.close()
