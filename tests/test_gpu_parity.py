"""GPU path vs the CPU FP64 oracle, through the C ABI.

Bars (relative L2 over the compared targets, on u_ap: the context's tolerance):
  FP64 context, tol 1e-9   ->  <= 1e-9
  mixed context, tol 1e-5  ->  <= 1e-5
Full-size workloads compare a seeded sample of targets that the oracle sums
one by one.
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


@pytest.fixture(scope="module")
def fh():
    import paper_2010_05978_amd as fh
    print("libfresnel_hip:", fh.LIB_PATH, flush=True)
    return fh


@pytest.fixture(scope="module", params=["fp64", "mixed"])
def ctx(request, fh):
    c = fh.Context(request.param)
    yield c
    c.close()


def oracle_quad(shape):
    k = type(shape).__name__
    if k == "RadialCurve":
        return oracle.quad_radial(shape.r0, shape.a if len(shape.a) else None,
                                  shape.b if len(shape.b) else None, shape.panels, shape.q, shape.m)
    if k == "Polygon":
        return oracle.quad_polygon(shape.vx, shape.vy, shape.q, shape.m)
    return oracle.quad_starshade(shape.Np, shape.a, shape.R, shape.b, shape.p, shape.m, shape.np_,
                                 shape.nd, shape.md, shape.coef, shape.K)


def cpu(t):
    return t.detach().cpu().numpy()


# ------------------------------------------------------------- quadrature
@pytest.mark.parametrize("wid", [1, 2, 3])
def test_quadrature_matches_oracle(fh, wid):
    c = fh.Context("fp64")
    shape = workloads.workload(wid).shape
    print(f"quadrature workload {wid}", flush=True)
    q = c.quad_for(shape)
    x, y, w = (cpu(t) for t in q.export())
    xo, yo, wo = oracle_quad(shape)
    assert len(x) == len(xo) == shape.n_nodes
    sc = np.abs(xo).max()
    assert np.abs(x - xo).max() <= 1e-14 * sc
    assert np.abs(y - yo).max() <= 1e-14 * sc
    assert np.abs(w - wo).max() <= 1e-14 * np.abs(wo).max()
    c.close()


def test_quadrature_polygon_perturbed_starshade_and_boundary(fh):
    c = fh.Context("fp64")
    shapes = workloads.batch_shapes(count=4, nmin=2000, nmax=5000)
    for s in shapes:
        q = c.quad_for(s)
        x, y, w = (cpu(t) for t in q.export())
        xo, yo, wo = oracle_quad(s)
        assert np.abs(x - xo).max() <= 1e-14 * np.abs(xo).max()
        assert np.abs(w - wo).max() <= 1e-14 * np.abs(wo).max()
    s = workloads.workload(5, reduced=True).shape
    for coef_on_device in (False, True):
        coef = torch.tensor(s.coef, device="cuda") if coef_on_device else s.coef
        q = c.quad_starshade(s.Np, s.a, s.R, s.b, s.p, s.m, s.np_, s.nd, s.md, coef, s.K)
        x, y, w = (cpu(t) for t in q.export())
        xo, yo, wo = oracle_quad(s)
        assert np.abs(x - xo).max() <= 1e-14 * 12
        assert np.abs(w - wo).max() <= 1e-14 * np.abs(wo).max()
    # user-supplied boundary rule -> dilation
    X, Y, W, V = oracle.boundary_radial_ptr(1.3, n=50)
    q = c.quad_from_boundary(X, Y, W, V, 7)
    x, y, w = (cpu(t) for t in q.export())
    xo, yo, wo = oracle.dilation(X, Y, W, V, 7)
    assert np.abs(w - wo).max() <= 1e-14 * np.abs(wo).max()
    c.close()


@pytest.mark.parametrize("nv", [3, 128, 129, 300])
def test_quadrature_polygon_vertex_counts(fh, nv):
    # up to 128 vertices travel in the kernel arguments, more go through
    # device memory: both give the oracle's rule
    c = fh.Context("fp64")
    g = np.random.Generator(np.random.PCG64(300 + nv))
    t = np.sort(g.uniform(0, 2 * math.pi, nv))
    r = 1.0 + 0.2 * g.uniform(-1, 1, nv)
    vx, vy = r * np.cos(t), r * np.sin(t)
    q = c.quad_polygon(vx, vy, 5, 7)
    x, y, w = (cpu(a) for a in q.export())
    xo, yo, wo = oracle.quad_polygon(vx, vy, 5, 7)
    assert len(x) == nv * 35
    assert np.abs(x - xo).max() <= 1e-14 and np.abs(y - yo).max() <= 1e-14
    assert np.abs(w - wo).max() <= 1e-14 * np.abs(wo).max()
    c.close()


# --------------------------------------------------------------- type 1
def test_grid_workload1_full(ctx):
    wl = workloads.workload(1)
    g = wl.grid
    print(f"type-1 workload 1 {ctx.precision}", flush=True)
    q = ctx.quad_for(wl.shape)
    u = cpu(ctx.field_grid(q, wl.lam, wl.z, g.n1, g.n2, g.h1, g.h2))
    x, y, w = oracle_quad(wl.shape)
    xi, eta = oracle.grid_targets(g.n1, g.n2, g.h1, g.h2)
    ref = oracle.fresnel_direct(x, y, w, wl.lam, wl.z, xi, eta)
    err = relL2(u, ref)
    print(f"  rel L2 = {err:.3e}", flush=True)
    assert err <= TOL[ctx.precision]
    # occulter output is the Babinet complement of the same sum
    uo = cpu(ctx.field_grid(q, wl.lam, wl.z, g.n1, g.n2, g.h1, g.h2, occulter=True))
    assert relL2(1 - uo, ref) <= TOL[ctx.precision]


@pytest.mark.parametrize("n1,n2,h1,h2,xc,yc", [
    (34, 18, 0.07, 0.11, 0.0, 0.0),        # rectangular, ragged tile tail
    (64, 64, 0.05, 0.05, 0.31, -0.47),     # translated grid (pre-phasing)
    (2, 2, 0.5, 0.5, 0.0, 0.0),            # smallest grid
    (256, 130, 0.012, 0.02, -0.2, 0.1),
])
def test_grid_shapes_and_translation(ctx, n1, n2, h1, h2, xc, yc):
    a = np.zeros(5)
    a[4] = 0.3
    shape = workloads.RadialCurve(1.0, a, np.zeros(5), panels=10, q=16, m=40)
    lam, z = 5e-7, 0.2 / 5e-7
    q = ctx.quad_for(shape)
    u = cpu(ctx.field_grid(q, lam, z, n1, n2, h1, h2, xc, yc))
    x, y, w = oracle_quad(shape)
    xi, eta = oracle.grid_targets(n1, n2, h1, h2, xc, yc)
    ref = oracle.fresnel_direct(x, y, w, lam, z, xi, eta)
    assert u.shape == (n2, n1)
    assert relL2(u, ref) <= TOL[ctx.precision]


@pytest.mark.parametrize("method,tile,P,sigma", [
    (1, 16, 64, 0.0), (2, 16, 64, 0.0), (1, 32, 1024, 0.0), (2, 32, 4096, 0.0), (2, 8, 256, 0.0),
    (2, 32, 256, 1.25), (1, 16, 512, 1.25), (3, 16, 64, 0.0), (3, 32, 16, 1.25), (0, 0, 0, 0.0),
    (4, 16, 64, 0.0), (4, 8, 256, 0.0), (4, 16, 32, 1.25), (4, 32, 64, 0.0), (4, 16, 4096, 0.0),
    (4, 8, 16, 0.0), (5, 16, 64, 0.0), (5, 8, 256, 0.0), (5, 16, 4096, 1.25), (5, 8, 16, 0.0),
    (5, 32, 1024, 0.0),
])
def test_spread_variants(fh, ctx, method, tile, P, sigma):
    # every spread method / tile / work-item size / upsampling the autotuner
    # may pick meets the same bar
    wl = workloads.workload(2)
    shape = workloads.RadialCurve(1.0, wl.shape.a, wl.shape.b, panels=12, q=16, m=60)
    opt = fh.fh_options(sigma=sigma, kernel_width=0, beta=0.0, tile=tile, max_subproblem=P, spread_method=method)
    ctx.set_options(opt)
    try:
        q = ctx.quad_for(shape)
        n = 160
        u = cpu(ctx.field_grid(q, wl.lam, wl.z, n, n, 0.02, 0.02))
        xi_t = torch.tensor(wl.points[0][:3000], device="cuda")
        eta_t = torch.tensor(wl.points[1][:3000], device="cuda")
        up = cpu(ctx.field_points(q, wl.lam, wl.z, xi_t, eta_t))
    finally:
        ctx.set_options(None)
    x, y, w = oracle_quad(shape)
    xi, eta = oracle.grid_targets(n, n, 0.02, 0.02)
    ref = oracle.fresnel_direct(x, y, w, wl.lam, wl.z, xi, eta)
    assert relL2(u, ref) <= TOL[ctx.precision]
    refp = oracle.fresnel_direct(x, y, w, wl.lam, wl.z, wl.points[0][:3000], wl.points[1][:3000])
    assert relL2(up, refp) <= TOL[ctx.precision]


@pytest.mark.parametrize("tile", [4, 5])
def test_small_tiles(fh, ctx, tile):
    # the smallest tiles the options allow (16 and 25 cells) with a width-5
    # kernel: 256 consecutive cells of the list reduce then span the most
    # listed tiles a step stages in LDS (17 of 18 for 16-cell tiles)
    wl = workloads.workload(2)
    shape = workloads.RadialCurve(1.0, wl.shape.a, wl.shape.b, panels=12, q=16, m=60)
    opt = fh.fh_options(sigma=2.0, kernel_width=5, beta=0.0, tile=tile, max_subproblem=0, spread_method=2)
    ctx.set_options(opt)
    n = 160
    try:
        q = ctx.quad_for(shape)
        u = cpu(ctx.field_grid(q, wl.lam, wl.z, n, n, 0.02, 0.02))
    finally:
        ctx.set_options(None)
    x, y, w = oracle_quad(shape)
    xi, eta = oracle.grid_targets(n, n, 0.02, 0.02)
    ref = oracle.fresnel_direct(x, y, w, wl.lam, wl.z, xi, eta)
    err = relL2(u, ref)
    print(f"  {ctx.precision} tile {tile} width 5: rel L2 {err:.2e}", flush=True)
    # a width-5 kernel resolves about 1e-5 (the ES rule for sigma = 2)
    assert err <= 1e-4


def test_grid_folding_undersampled(ctx):
    # target grid coarser than the field: rescaled nodes leave [-pi, pi) and
    # must be folded (sec. 2.2)
    shape = workloads.RadialCurve(1.0, np.zeros(0), np.zeros(0), panels=6, q=20, m=40)
    lam, z, n, h = 1.0, 0.1, 16, 0.4
    q = ctx.quad_for(shape)
    u = cpu(ctx.field_grid(q, lam, z, n, n, h, h))
    x, y, w = oracle_quad(shape)
    xi, eta = oracle.grid_targets(n, n, h, h)
    ref = oracle.fresnel_direct(x, y, w, lam, z, xi, eta)
    assert 2 * math.pi * h * 1.0 / (lam * z) > math.pi
    assert relL2(u, ref) <= TOL[ctx.precision]


def test_single_node_plane_wave(ctx):
    # one node: u_k = exp(i pi |xi_k - x0|^2/lz) w0/(i lz) at every target
    x0, y0, w0 = np.array([0.123]), np.array([-0.456]), np.array([0.7])
    q = ctx.quad_from_nodes(x0, y0, w0)
    lam, z = 1.0, 0.3
    u = cpu(ctx.field_grid(q, lam, z, 40, 24, 0.05, 0.07))
    xi, eta = oracle.grid_targets(40, 24, 0.05, 0.07)
    ref = np.exp(1j * math.pi * ((xi - x0) ** 2 + (eta - y0) ** 2) / (lam * z)) * w0 / (1j * lam * z)
    assert relL2(u, ref) <= TOL[ctx.precision]


def test_empty_rule(ctx):
    q = ctx.quad_from_nodes(np.zeros(0), np.zeros(0), np.zeros(0))
    u = cpu(ctx.field_grid(q, 1.0, 1.0, 8, 6, 0.1, 0.1))
    assert np.all(u == 0)
    u = cpu(ctx.field_grid(q, 1.0, 1.0, 8, 6, 0.1, 0.1, occulter=True))
    assert np.all(u == 1)
    xi = torch.zeros(5, dtype=torch.float64, device="cuda")
    u = cpu(ctx.field_points(q, 1.0, 1.0, xi, xi, occulter=True))
    assert np.all(u == 1)


def test_grid_workload2_full_size_sampled(ctx):
    wl = workloads.workload(2)
    g = wl.grid
    print(f"type-1 workload 2 {ctx.precision}", flush=True)
    q = ctx.quad_for(wl.shape)
    u = cpu(ctx.field_grid(q, wl.lam, wl.z, g.n1, g.n2, g.h1, g.h2)).ravel()
    rng = np.random.Generator(np.random.PCG64(99))
    idx = rng.choice(g.M, 3000, replace=False)
    x, y, w = oracle_quad(wl.shape)
    xi, eta = oracle.grid_targets(g.n1, g.n2, g.h1, g.h2)
    ref = oracle.fresnel_direct(x, y, w, wl.lam, wl.z, xi[idx], eta[idx])
    err = relL2(u[idx], ref)
    print(f"  rel L2 (3000 samples) = {err:.3e}", flush=True)
    assert err <= TOL[ctx.precision]


# --------------------------------------------------------------- type 3
def test_points_workload2_sampled(ctx):
    wl = workloads.workload(2)
    xi, eta = wl.points
    print(f"type-3 workload 2 {ctx.precision}", flush=True)
    q = ctx.quad_for(wl.shape)
    dxi = torch.tensor(xi, device="cuda")
    deta = torch.tensor(eta, device="cuda")
    u = cpu(ctx.field_points(q, wl.lam, wl.z, dxi, deta))
    rng = np.random.Generator(np.random.PCG64(98))
    idx = rng.choice(len(xi), 3000, replace=False)
    x, y, w = oracle_quad(wl.shape)
    ref = oracle.fresnel_direct(x, y, w, wl.lam, wl.z, xi[idx], eta[idx])
    err = relL2(u[idx], ref)
    print(f"  rel L2 (3000 samples) = {err:.3e}", flush=True)
    assert err <= TOL[ctx.precision]
    # host arrays in, host array out: same answer
    uh = np.empty(len(xi), dtype=np.complex128 if ctx.precision == "fp64" else np.complex64)
    from paper_2010_05978_amd import abi
    abi.fh_field_points(ctx.handle, q.handle, wl.lam, wl.z, xi, eta, False, uh)
    assert relL2(uh[idx], ref) <= TOL[ctx.precision]


def test_points_small_full(ctx):
    shape = workloads.workload(1).shape
    wl = workloads.workload(1)
    g = np.random.Generator(np.random.PCG64(5))
    M = 777
    xi = g.uniform(-1.7, 0.9, M)
    eta = g.uniform(-0.4, 1.3, M)
    q = ctx.quad_for(shape)
    u = cpu(ctx.field_points(q, wl.lam, wl.z, torch.tensor(xi, device="cuda"), torch.tensor(eta, device="cuda")))
    x, y, w = oracle_quad(shape)
    ref = oracle.fresnel_direct(x, y, w, wl.lam, wl.z, xi, eta)
    assert relL2(u, ref) <= TOL[ctx.precision]
    # single target (zero target extent)
    u1 = cpu(ctx.field_points(q, wl.lam, wl.z, torch.tensor(xi[:1], device="cuda"),
                              torch.tensor(eta[:1], device="cuda")))
    assert abs(u1[0] - ref[0]) <= TOL[ctx.precision] * max(1.0, abs(ref[0])) * 10


def test_points_equal_grid_at_grid_targets(ctx):
    wl = workloads.workload(1)
    g = wl.grid
    q = ctx.quad_for(wl.shape)
    ug = cpu(ctx.field_grid(q, wl.lam, wl.z, g.n1, g.n2, g.h1, g.h2)).ravel()
    xi, eta = oracle.grid_targets(g.n1, g.n2, g.h1, g.h2)
    up = cpu(ctx.field_points(q, wl.lam, wl.z, torch.tensor(xi, device="cuda"), torch.tensor(eta, device="cuda")))
    assert relL2(up, ug) <= 2 * TOL[ctx.precision]


def test_rule_shared_by_contexts_on_two_streams(fh, ctx):
    # a rule made by one context feeds another context on another stream,
    # ordered by an event, as in a pipelined step
    wl = workloads.workload(2)
    g = wl.grid
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        other = fh.Context(ctx.precision)
    try:
        M = 5000
        xi = torch.tensor(wl.points[0][:M], device="cuda")
        eta = torch.tensor(wl.points[1][:M], device="cuda")
        ref_pts = cpu(ctx.field_points(ctx.quad_for(wl.shape), wl.lam, wl.z, xi, eta))
        ev_rule, ev_done = torch.cuda.Event(), torch.cuda.Event()
        main = torch.cuda.current_stream()
        up = torch.empty(M, dtype=ctx.cdtype, device="cuda")
        for _ in range(3):
            q = ctx.quad_for(wl.shape)
            ev_rule.record(main)
            ug = ctx.field_grid(q, wl.lam, wl.z, 200, 200, g.h1, g.h2)
            side.wait_event(ev_rule)
            other.field_points(q, wl.lam, wl.z, xi, eta, out=up)
            ev_done.record(side)
            main.wait_event(ev_done)
            q.close()
        torch.cuda.synchronize()
        # same rule and targets: equal to the rounding of the summation order
        assert relL2(cpu(up), ref_pts) <= (1e-12 if ctx.precision == "fp64" else 1e-6)
        x, y, w = oracle_quad(wl.shape)
        xs, ys = oracle.grid_targets(200, 200, g.h1, g.h2)
        rng = np.random.Generator(np.random.PCG64(8))
        idx = rng.choice(len(xs), 300, replace=False)
        ref = oracle.fresnel_direct(x, y, w, wl.lam, wl.z, xs[idx], ys[idx])
        assert relL2(cpu(ug).ravel()[idx], ref) <= TOL[ctx.precision]
    finally:
        other.close()


@pytest.fixture(scope="module")
def starshade_refs():
    """Workload 3's oracle values, shared by both precisions: at each of the
    3 wavelengths, 3,300 grid targets (2,400 seeded, 300 on the grid's first
    row k2 = -n/2, 300 on its first column k1 = -n/2, 300 at the pupil's edge
    2.35 <= |xi| < 2.4) and 3,000 seeded pupil points."""
    wl = workloads.workload(3)
    g = wl.grid
    x, y, w = oracle_quad(wl.shape)
    xi_g, eta_g = oracle.grid_targets(g.n1, g.n2, g.h1, g.h2)
    rng = np.random.Generator(np.random.PCG64(96))
    r = np.hypot(xi_g, eta_g)
    edge = np.flatnonzero((r >= 2.35) & (r < 2.4))
    gidx = np.concatenate([rng.choice(g.M, 2400, replace=False),
                           rng.choice(g.n1, 300, replace=False),                 # k2 = -n2/2
                           rng.choice(g.n2, 300, replace=False) * g.n1,          # k1 = -n1/2
                           rng.choice(edge, 300, replace=False)])
    pidx = np.random.Generator(np.random.PCG64(97)).choice(len(wl.points[0]), 3000, replace=False)
    xi_p, eta_p = wl.points
    refs = {}
    for lam in wl.lams:
        refs[lam] = (oracle.fresnel_direct(x, y, w, lam, wl.z, xi_g[gidx], eta_g[gidx]),
                     oracle.fresnel_direct(x, y, w, lam, wl.z, xi_p[pidx], eta_p[pidx]))
    return wl, gidx, pidx, refs


def _check_u_oc(prec, got_oc, ref_ap, what):
    """Relative L2 on u_ap (the bar) and the maximum absolute error of the
    returned u_oc, which must stay within 10 tol times the rms of u_ap."""
    err = relL2(1 - got_oc, ref_ap)
    mx = float(np.abs(got_oc - (1 - ref_ap)).max())
    rms = float(np.sqrt(np.mean(np.abs(ref_ap) ** 2)))
    print(f"  {what}: rel L2 (u_ap) {err:.3e}, max abs (u_oc) {mx:.3e}", flush=True)
    assert err <= TOL[prec], what
    assert mx <= 10 * TOL[prec] * rms, what


def test_starshade_workload3_points_sampled(ctx, starshade_refs):
    wl, _, pidx, refs = starshade_refs
    xi, eta = wl.points
    print(f"type-3 workload 3 {ctx.precision}", flush=True)
    q = ctx.quad_for(wl.shape)
    txi, teta = torch.tensor(xi, device="cuda"), torch.tensor(eta, device="cuda")
    for lam in wl.lams:
        u = cpu(ctx.field_points(q, lam, wl.z, txi, teta, occulter=True))
        _check_u_oc(ctx.precision, u[pidx], refs[lam][1], f"lambda={lam:.2e}, 3000 of 1e6 points")


def test_starshade_workload3_grid_sampled(ctx, starshade_refs):
    wl, gidx, _, refs = starshade_refs
    g = wl.grid
    print(f"type-1 workload 3 {ctx.precision}", flush=True)
    q = ctx.quad_for(wl.shape)
    for lam in wl.lams:
        u = ctx.field_grid(q, lam, wl.z, g.n1, g.n2, g.h1, g.h2, occulter=True).reshape(-1)
        got = cpu(u.index_select(0, torch.as_tensor(gidx, device="cuda")))
        _check_u_oc(ctx.precision, got, refs[lam][0],
                    f"lambda={lam:.2e}, 3300 grid targets (first row, first column, pupil edge)")


# -------------------------------------------------------- error statuses
def test_error_statuses(fh):
    c = fh.Context("fp64")
    q = c.quad_radial(1.0, panels=2, q=4, m=3)
    u = torch.empty((4, 5), dtype=torch.complex128, device="cuda")
    from paper_2010_05978_amd import abi
    with pytest.raises(fh.FresnelError) as e:
        abi.fh_field_grid(c.handle, q.handle, 1.0, 1.0, 5, 4, 0.1, 0.1, 0, 0, False, u)
    assert e.value.status == fh.FH_ERR_ODD_GRID
    with pytest.raises(fh.FresnelError) as e:
        abi.fh_field_grid(c.handle, q.handle, 1.0, -1.0, 4, 4, 0.1, 0.1, 0, 0, False, u)
    assert e.value.status == fh.FH_ERR_NONPOSITIVE_LZ
    with pytest.raises(fh.FresnelError) as e:
        abi.fh_field_grid(c.handle, q.handle, float("nan"), 1.0, 4, 4, 0.1, 0.1, 0, 0, False, u)
    assert e.value.status == fh.FH_ERR_NONFINITE
    with pytest.raises(fh.FresnelError) as e:
        abi.fh_quad_radial(c.handle, 1.0, np.zeros(65), None, 1, 4, 3)
    assert e.value.status == fh.FH_ERR_INVALID_ARG
    # spread tiles of 4 to 32 cells only (the tile reduce covers at most
    # 1024 cells per tile)
    for bad in (3, 64):
        with pytest.raises(fh.FresnelError) as e:
            c.set_options(fh.fh_options(sigma=0, kernel_width=0, beta=0.0, tile=bad, max_subproblem=0,
                                        spread_method=0))
        assert e.value.status == fh.FH_ERR_INVALID_ARG
    c.set_options(None)
    # the context stays usable after errors
    v = c.field_grid(q, 1.0, 1.0, 4, 4, 0.1, 0.1)
    assert torch.isfinite(torch.view_as_real(v)).all()
    c.close()


# ------------------------------------------------- transform length sweep
def test_many_transform_lengths(fh, ctx):
    # grids and target extents chosen so that the fine grids and upsampled
    # grids take many 2-3-5-7-smooth lengths (LDS FFT radix passes 16, 8, 4,
    # 2, 3, 5, 7 in many combinations), each against the oracle
    shape = workloads.RadialCurve(0.7, np.array([0.0, 0.1]), np.array([0.05, 0.0]), panels=4, q=12, m=10)
    x, y, w = oracle_quad(shape)
    lam, z = 1.0, 0.05
    seen = set()
    for n in (6, 10, 22, 30, 46, 62, 98, 126, 190, 250, 334):
        h = 1.2 / n
        u = cpu(ctx.field_grid(ctx.quad_for(shape), lam, z, n, n + 4, h, 0.9 * h))
        xi, eta = oracle.grid_targets(n, n + 4, h, 0.9 * h)
        ref = oracle.fresnel_direct(x, y, w, lam, z, xi, eta)
        assert relL2(u, ref) <= TOL[ctx.precision], n
        seen.add(ctx.query_params(n)["nf"])
    assert len(seen) >= 8
    g = np.random.Generator(np.random.PCG64(31))
    q = ctx.quad_for(shape)
    for ext in (0.05, 0.2, 0.45, 0.8, 1.3, 2.1):
        M = 300
        xi = g.uniform(-ext, ext, M)
        eta = g.uniform(-0.6 * ext, ext, M)
        up = cpu(ctx.field_points(q, lam, z, torch.tensor(xi, device="cuda"), torch.tensor(eta, device="cuda")))
        ref = oracle.fresnel_direct(x, y, w, lam, z, xi, eta)
        assert relL2(up, ref) <= TOL[ctx.precision], ext


@pytest.mark.parametrize("method,tile", [(5, 0), (5, 6), (5, 10), (2, 6), (2, 10)])
@pytest.mark.parametrize("h", [0.006, 0.05])
def test_tiles_that_do_not_divide_the_grid(fh, ctx, method, tile, h):
    # tiles of 6 or 10 cells on fine grids of 1024 x 768 cells: the last
    # tile of each row (and, for 10, of each column) is partial and the
    # padded tiles that wrap around the period land closer; h = 0.006 holds a
    # window of rows, h = 0.05 the whole period (folded nodes, wrap in y)
    wl = workloads.workload(2)
    shape = workloads.RadialCurve(1.0, wl.shape.a, wl.shape.b, panels=12, q=16, m=60)
    opt = fh.fh_options(sigma=2.0, kernel_width=0, beta=0.0, tile=tile, max_subproblem=0, spread_method=method)
    ctx.set_options(opt)
    n1, n2 = 512, 384
    try:
        q = ctx.quad_for(shape)
        u = cpu(ctx.field_grid(q, wl.lam, wl.z, n1, n2, h, 0.9 * h, xc=0.02, yc=-0.03)).ravel()
        assert ctx.query_params(n1)["nf"] == 1024
    finally:
        ctx.set_options(None)
    x, y, w = oracle_quad(shape)
    xi, eta = oracle.grid_targets(n1, n2, h, 0.9 * h, 0.02, -0.03)
    idx = np.random.Generator(np.random.PCG64(41)).choice(n1 * n2, 4000, replace=False)
    # every target of the first and last rows and columns as well
    k = np.arange(n1 * n2).reshape(n2, n1)
    idx = np.unique(np.concatenate([idx, k[0], k[-1], k[:, 0], k[:, -1]]))
    ref = oracle.fresnel_direct(x, y, w, wl.lam, wl.z, xi[idx], eta[idx])
    err = relL2(u[idx], ref)
    print(f"  {ctx.precision} method {method} tile {tile} h {h}: rel L2 {err:.2e}", flush=True)
    assert err <= TOL[ctx.precision]
