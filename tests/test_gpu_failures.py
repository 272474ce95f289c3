"""Failure paths forced from the host: a device-memory cap (FH_ERR_ALLOC),
a refused rocFFT plan (FH_ERR_FFT) and a refused graph capture (the batched
call must then run eagerly).  After each failure the same context must keep
working and match the oracle."""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def relL2(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def cpu(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def fh():
    import paper_2010_05978_amd as fh
    return fh


def disk():
    wl = workloads.workload(1)
    s, g = wl.shape, wl.grid
    x, y, w = oracle.quad_radial(s.r0, None, None, s.panels, s.q, s.m)
    xi, eta = oracle.grid_targets(g.n1, g.n2, g.h1, g.h2)
    return wl, oracle.fresnel_direct(x, y, w, wl.lam, wl.z, xi, eta)


def test_allocation_cap(fh, monkeypatch):
    monkeypatch.setenv("FH_ALLOC_CAP_BYTES", str(48 << 20))
    ctx = fh.Context("fp64")
    monkeypatch.delenv("FH_ALLOC_CAP_BYTES")
    wl, ref = disk()
    q = ctx.quad_for(wl.shape)
    g = wl.grid
    # a 4096^2 grid needs far more than 48 MiB of workspace
    big = torch.empty((4096, 4096), dtype=torch.complex128, device="cuda")
    with pytest.raises(fh.FresnelError) as e:
        ctx.field_grid(q, wl.lam, wl.z, 4096, 4096, 0.001, 0.001, out=big)
    assert e.value.status == fh.FH_ERR_ALLOC
    print(f"  capped context: {e.value}", flush=True)
    del big
    u = cpu(ctx.field_grid(q, wl.lam, wl.z, g.n1, g.n2, g.h1, g.h2))
    assert relL2(u, ref) <= 1e-9
    q.close()
    ctx.close()


def test_refused_fft_plan(fh, monkeypatch):
    # a 2048^2 grid in FP64 needs rocFFT (a 4096-point row of complex doubles
    # does not fit in LDS)
    monkeypatch.setenv("FH_INJECT_FAULT", "fft_plan")
    ctx = fh.Context("fp64")
    monkeypatch.delenv("FH_INJECT_FAULT")
    wl = workloads.workload(1)
    q = ctx.quad_for(wl.shape)
    n, h = 2048, 3.0 / 2048
    with pytest.raises(fh.FresnelError) as e:
        ctx.field_grid(q, wl.lam, wl.z, n, n, h, h)
    assert e.value.status == fh.FH_ERR_FFT
    # the context still serves what needs no rocFFT plan: type 3 on small
    # grids runs its transforms in LDS
    rng = np.random.Generator(np.random.PCG64(5))
    xi, eta = rng.uniform(-1.2, 1.2, 500), rng.uniform(-1.2, 1.2, 500)
    v = cpu(ctx.field_points(q, wl.lam, wl.z, torch.tensor(xi, device="cuda"), torch.tensor(eta, device="cuda")))
    x, y, w = oracle.quad_radial(wl.shape.r0, None, None, wl.shape.panels, wl.shape.q, wl.shape.m)
    assert relL2(v, oracle.fresnel_direct(x, y, w, wl.lam, wl.z, xi, eta)) <= 1e-9
    q.close()
    ctx.close()
    # a context made without the fault plans normally
    ok = fh.Context("fp64")
    q = ok.quad_for(wl.shape)
    u = cpu(ok.field_grid(q, wl.lam, wl.z, n, n, h, h)).ravel()
    gx, gy = oracle.grid_targets(n, n, h, h)
    idx = np.random.Generator(np.random.PCG64(6)).choice(n * n, 300, replace=False)
    assert relL2(u[idx], oracle.fresnel_direct(x, y, w, wl.lam, wl.z, gx[idx], gy[idx])) <= 1e-9
    q.close()
    ok.close()


def test_refused_graph_capture_runs_eagerly(fh, monkeypatch):
    shapes = workloads.batch_shapes(count=4, nmin=3000, nmax=8000)
    lams = workloads.batch_lambdas(64)[:4] * 1.0
    zs = np.full(4, workloads.BATCH_Z)
    n = 96
    g = workloads.Grid(n, n, 3.0 / n, 3.0 / n)
    monkeypatch.setenv("FH_INJECT_FAULT", "graph_capture")
    ctx = fh.Context("fp64")
    monkeypatch.delenv("FH_INJECT_FAULT")
    quads = [ctx.quad_for(s) for s in shapes]
    xi, eta = oracle.grid_targets(n, n, g.h1, g.h2)
    for rep in range(2):
        u = cpu(ctx.field_grid_batch(quads, lams, zs, n, n, g.h1, g.h2))
        for b, s in enumerate(shapes):
            if type(s).__name__ == "RadialCurve":
                x, y, w = oracle.quad_radial(s.r0, s.a, s.b, s.panels, s.q, s.m)
            else:
                x, y, w = oracle.quad_polygon(s.vx, s.vy, s.q, s.m)
            idx = np.random.Generator(np.random.PCG64(60 + b)).choice(g.M, 200, replace=False)
            ref = oracle.fresnel_direct(x, y, w, lams[b], zs[b], xi[idx], eta[idx])
            assert relL2(u[b].ravel()[idx], ref) <= 1e-9, (rep, b)
    for q in quads:
        q.close()
    ctx.close()
