"""The hand-written adjoint (type-2 NUFFT back to the nodes + starshade chain
rule) against the CPU oracle's exact direct-sum gradient, finite differences
and torch's autograd plumbing."""
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


@pytest.fixture(scope="module")
def fh():
    import paper_2010_05978_amd as fh
    return fh


@pytest.fixture(scope="module", params=["fp64", "mixed"])
def ctx(request, fh):
    c = fh.Context(request.param)
    yield c
    c.close()


def cpu(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("occ,xc,yc,n1,n2,h", [
    (False, 0.0, 0.0, 64, 48, 0.05),
    (True, 0.21, -0.33, 40, 56, 0.045),
    (False, 0.0, 0.0, 16, 16, 0.4),     # folded: rows cover the whole period
])
def test_grid_vjp_matches_oracle(ctx, occ, xc, yc, n1, n2, h):
    a = np.zeros(5)
    a[4] = 0.3
    shape = workloads.RadialCurve(1.0, a, np.zeros(5), panels=10, q=16, m=30)
    lam, z = 1.0, 0.12
    q = ctx.quad_for(shape)
    g = np.random.Generator(np.random.PCG64(21))
    gu = (g.normal(size=(n2, n1)) + 1j * g.normal(size=(n2, n1)))
    gu_t = torch.tensor(gu, dtype=ctx.cdtype, device="cuda")
    gx, gy, gw = (cpu(t) for t in ctx.field_grid_vjp(q, lam, z, n1, n2, h, h, gu_t, xc, yc, occ))
    x, y, w = oracle.quad_radial(shape.r0, shape.a, shape.b, shape.panels, shape.q, shape.m)
    xi, eta = oracle.grid_targets(n1, n2, h, h, xc, yc)
    gref = cpu(gu_t).astype(np.complex128).ravel()
    rx, ry, rw = oracle.fresnel_direct_vjp(x, y, w, lam, z, xi, eta, gref, occ)
    for got, ref, name in ((gx, rx, "x"), (gy, ry, "y"), (gw, rw, "w")):
        err = relL2(got, ref)
        print(f"  d/d{name}: rel L2 {err:.2e}", flush=True)
        assert err <= TOL[ctx.precision], name


def test_starshade_vjp_matches_oracle(fh):
    c = fh.Context("fp64")
    s = workloads.workload(5, reduced=True).shape
    N = s.n_nodes
    g = np.random.Generator(np.random.PCG64(22))
    gx, gy, gw = g.normal(size=(3, N))
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    out = torch.empty(2 * s.Np * s.K, dtype=torch.float64, device="cuda")
    from paper_2010_05978_amd import abi
    abi.fh_starshade_vjp(c.handle, s.Np, s.a, s.R, s.b, s.p, s.m, s.np_, s.nd, s.md, dev(s.coef), s.K,
                         dev(gx), dev(gy), dev(gw), out)
    ref = oracle.starshade_vjp(s.Np, s.a, s.R, s.b, s.p, s.m, s.np_, s.nd, s.md, s.coef, s.K, gx, gy, gw)
    assert relL2(cpu(out), ref) <= 1e-12
    c.close()


def _oracle_loss_and_grad(wl, mask):
    s, gd = wl.shape, wl.grid
    x, y, w = oracle.quad_starshade(s.Np, s.a, s.R, s.b, s.p, s.m, s.np_, s.nd, s.md, s.coef, s.K)
    xi, eta = oracle.grid_targets(gd.n1, gd.n2, gd.h1, gd.h2)
    xi, eta = xi[mask], eta[mask]
    Min = int(mask.sum())
    L = 0.0
    gx = np.zeros_like(x); gy = np.zeros_like(x); gw = np.zeros_like(x)
    uap_n, uoc_n = 0.0, 0.0
    for lam in wl.lams:
        u = oracle.fresnel_direct(x, y, w, lam, wl.z, xi, eta, occulter=True)
        L += float((np.abs(u) ** 2).sum()) / (len(wl.lams) * Min)
        g = 2.0 * u / (len(wl.lams) * Min)
        a, b, cc = oracle.fresnel_direct_vjp(x, y, w, lam, wl.z, xi, eta, g, occulter=True)
        gx += a; gy += b; gw += cc
        uoc_n += float((np.abs(u) ** 2).sum())
        uap_n += float((np.abs(1 - u) ** 2).sum())
    gc = oracle.starshade_vjp(s.Np, s.a, s.R, s.b, s.p, s.m, s.np_, s.nd, s.md, s.coef, s.K, gx, gy, gw)
    # errors in u_ap carry over to u_oc = 1 - u_ap absolutely: relative to the
    # shadow field they are amplified by |u_ap|/|u_oc|
    kappa = math.sqrt(uap_n / uoc_n)
    return L, gc, kappa


def _gpu_loss(fh_ctx, wl, coef, mask_t):
    from paper_2010_05978_amd.autograd import starshade_field
    gd = wl.grid
    Min = int(mask_t.sum())
    L = 0.0
    for lam in wl.lams:
        u = starshade_field(coef, fh_ctx, wl.shape, lam, wl.z, gd, occulter=True)
        L = L + ((u.abs() ** 2).reshape(-1) * mask_t).sum() / (len(wl.lams) * Min)
    return L


def test_autograd_starshade_gradient_vs_direct_sum(ctx):
    wl = workloads.workload(5, reduced=True)
    mask = workloads.pupil_mask(wl.grid.n1)
    mask_t = torch.tensor(mask, dtype=torch.float64 if ctx.precision == "fp64" else torch.float32, device="cuda")
    coef = torch.tensor(wl.shape.coef, dtype=torch.float64, device="cuda", requires_grad=True)
    print(f"autograd starshade {ctx.precision}", flush=True)
    L = _gpu_loss(ctx, wl, coef, mask_t)
    L.backward()
    Lref, gref, kappa = _oracle_loss_and_grad(wl, mask)
    errL = abs(float(L) - Lref) / Lref
    errg = relL2(cpu(coef.grad), gref)
    print(f"  loss {float(L):.6e} (oracle {Lref:.6e}, rel {errL:.2e}); grad rel L2 {errg:.2e}; "
          f"shadow amplification {kappa:.1f}", flush=True)
    # the bar is the stated tolerance itself; kappa (how much the u_ap
    # tolerance could be amplified in the shadow) is reported beside it
    assert errL <= TOL[ctx.precision]
    assert errg <= TOL[ctx.precision]


def test_wavelength_sweep_gradient(ctx):
    """The sweep form (rule built once, one batched forward over the three
    wavelengths, node gradients summed over them in one call and chained
    once) against the oracle's direct-sum gradient and against the
    per-wavelength form."""
    from paper_2010_05978_amd.autograd import starshade_sweep
    wl = workloads.workload(5, reduced=True)
    mask = workloads.pupil_mask(wl.grid.n1)
    rdt = torch.float64 if ctx.precision == "fp64" else torch.float32
    mask_t = torch.tensor(mask, dtype=rdt, device="cuda")
    Min = int(mask_t.sum())
    nl = len(wl.lams)
    coef = torch.tensor(wl.shape.coef, dtype=torch.float64, device="cuda", requires_grad=True)
    u = starshade_sweep(coef, ctx, wl.shape, wl.lams, wl.z, wl.grid, occulter=True)
    assert u.shape == (nl, wl.grid.n2, wl.grid.n1)
    L = ((u.abs() ** 2).reshape(nl, -1) * mask_t.reshape(1, -1)).sum() / (nl * Min)
    L.backward()
    g_sweep = cpu(coef.grad)
    Lref, gref, kappa = _oracle_loss_and_grad(wl, mask)
    errL = abs(float(L) - Lref) / Lref
    errg = relL2(g_sweep, gref)
    print(f"sweep {ctx.precision}: loss rel {errL:.2e}, grad rel L2 {errg:.2e} (kappa {kappa:.1f})", flush=True)
    assert errL <= TOL[ctx.precision]
    assert errg <= TOL[ctx.precision]
    coef2 = torch.tensor(wl.shape.coef, dtype=torch.float64, device="cuda", requires_grad=True)
    _gpu_loss(ctx, wl, coef2, mask_t).backward()
    d = relL2(g_sweep, cpu(coef2.grad))
    print(f"  sweep vs per-wavelength form: {d:.2e}", flush=True)
    assert d <= (1e-12 if ctx.precision == "fp64" else 1e-6)


def test_vjp_sum_is_the_sum_of_vjps(ctx):
    wl = workloads.workload(5, reduced=True)
    s = wl.shape
    q = ctx.quad_starshade(s.Np, s.a, s.R, s.b, s.p, s.m, s.np_, s.nd, s.md, s.coef, s.K)
    g = wl.grid
    rng = np.random.Generator(np.random.PCG64(23))
    nl = len(wl.lams)
    gu_np = rng.standard_normal((nl, g.n2, g.n1)) + 1j * rng.standard_normal((nl, g.n2, g.n1))
    gu = torch.tensor(gu_np, dtype=ctx.cdtype, device="cuda")
    zs = np.full(nl, wl.z)
    sx, sy, sw = ctx.field_grid_vjp_sum(q, wl.lams, zs, g.n1, g.n2, g.h1, g.h2, gu, occulter=True)
    acc = [np.zeros(q.N) for _ in range(3)]
    for l in range(nl):
        parts = ctx.field_grid_vjp(q, wl.lams[l], wl.z, g.n1, g.n2, g.h1, g.h2, gu[l].contiguous(), occulter=True)
        for a, p in zip(acc, parts):
            a += cpu(p)
    for got, ref in zip((sx, sy, sw), acc):
        e = relL2(cpu(got), ref)
        assert e <= 1e-14 if ctx.precision == "fp64" else e <= 1e-6, e
    with pytest.raises(Exception):
        ctx.field_grid_vjp_sum(q, wl.lams, zs[:1], g.n1, g.n2, g.h1, g.h2, gu)
    q.close()


def test_finite_differences(fh):
    """Central differences of the FP64 GPU loss against the adjoint, on 32
    seeded coefficients and one seeded random direction of all 384.  The bar
    follows from the step: the truncation error of the h-difference is
    estimated from the 2h-difference (their gap is 3/4 of the h^2 term's
    growth), and the rounding noise of the loss, measured from two
    evaluations at the same point (floored at 1e-15 |L|), enters as 2 e_L/h;
    the adjoint's own error enters as the FP64 tolerance times the larger of
    |g| and the gradient's rms component."""
    c = fh.Context("fp64")
    wl = workloads.workload(5, reduced=True)
    mask_t = torch.tensor(workloads.pupil_mask(wl.grid.n1), dtype=torch.float64, device="cuda")
    coef = torch.tensor(wl.shape.coef, dtype=torch.float64, device="cuda", requires_grad=True)
    L = _gpu_loss(c, wl, coef, mask_t)
    L.backward()
    grad = cpu(coef.grad)
    base = coef.detach().clone()
    with torch.no_grad():
        L0 = float(L)
        L1 = float(_gpu_loss(c, wl, base, mask_t))
        noise = max(abs(L1 - L0), 1e-15 * abs(L0))
        h = 1e-7

        def fd(d, step):
            return (float(_gpu_loss(c, wl, base + step * d, mask_t)) -
                    float(_gpu_loss(c, wl, base - step * d, mask_t))) / (2 * step)

        rng = np.random.Generator(np.random.PCG64(23))
        idx = rng.choice(len(grad), 32, replace=False)
        dirs = []
        for i in idx:
            d = torch.zeros_like(base)
            d[i] = 1.0
            dirs.append((f"coef {i}", d, grad[i]))
        v = rng.normal(size=len(grad))
        v /= np.linalg.norm(v)
        dirs.append(("random direction", torch.tensor(v, device="cuda"), float(grad @ v)))
        # the adjoint's own error: the FP64 tolerance relative to the
        # gradient's rms component (the bar of the parity test is relative L2)
        g_rms = float(np.sqrt(np.mean(grad ** 2)))
        worst = 0.0
        for name, d, g in dirs:
            f1, f2 = fd(d, h), fd(d, 2 * h)
            bar = abs(f2 - f1) + 2 * noise / h + 1e-9 * max(abs(g), g_rms)
            worst = max(worst, abs(f1 - g) / bar)
            print(f"  {name}: adjoint {g:.10e} fd {f1:.10e} |diff| {abs(f1 - g):.2e} bar {bar:.2e}", flush=True)
            assert abs(f1 - g) <= bar, name
        print(f"  worst |diff|/bar {worst:.2f}", flush=True)
    c.close()


def test_node_autograd_matches_torch_direct(fh):
    # gradients through NodeGridField vs torch autograd of the plain sum
    from paper_2010_05978_amd.autograd import node_field
    c = fh.Context("fp64")
    g = np.random.Generator(np.random.PCG64(24))
    N = 300
    x = g.uniform(-0.8, 0.8, N); y = g.uniform(-0.8, 0.8, N); w = g.uniform(0.0, 0.01, N)
    grid = workloads.Grid(24, 20, 0.07, 0.08, 0.1, -0.05)
    lam, z = 1.0, 0.3
    tx, ty, tw = (torch.tensor(v, device="cuda", requires_grad=True) for v in (x, y, w))
    u = node_field(tx, ty, tw, c, lam, z, grid, occulter=True)
    wt = torch.tensor(g.uniform(0.5, 1.5, (grid.n2, grid.n1)), device="cuda")
    (wt * u.abs() ** 2).sum().backward()
    # reference: torch autograd of the plain sum on the CPU in float64
    cx, cy, cw = (torch.tensor(v, requires_grad=True) for v in (x, y, w))
    xi, eta = oracle.grid_targets(grid.n1, grid.n2, grid.h1, grid.h2, grid.xc, grid.yc)
    xi, eta = torch.tensor(xi), torch.tensor(eta)
    ph = math.pi * ((xi[:, None] - cx[None]) ** 2 + (eta[:, None] - cy[None]) ** 2) / (lam * z)
    E = torch.polar(torch.ones_like(ph), ph)
    ur = 1 - (E * cw[None].to(E.dtype)).sum(1) / (1j * lam * z)
    (wt.cpu().reshape(-1) * ur.abs() ** 2).sum().backward()
    for got, ref in ((tx.grad, cx.grad), (ty.grad, cy.grad), (tw.grad, cw.grad)):
        assert relL2(cpu(got), ref.numpy()) <= 1e-9
    c.close()
