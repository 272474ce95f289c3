"""Edge integral (eq. nsli) and boundary rules on the GPU vs the CPU FP64 oracle.

The library's boundary rules (fh_boundary_radial / _polygon / _starshade) are
compared with the oracle's node by node, and fh_field_nsli with the oracle's
edge integral element by element on the same boundary rule: at sizes the
oracle finishes in seconds (several workgroups and node groups, ragged
tails), on the workload-2 starfish outline at its full 1000 x 1000 target
grid (sampled), for targets on and next to nodes, with the deep-shadow
option, and for empty inputs.  The arithmetic is FP64 in both precisions,
so the bar is 1e-12 relative L2 (fp64 output) and the complex64 rounding
(mixed output).
"""
import math

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-6}


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


@pytest.fixture(scope="module")
def ctx64(fh):
    c = fh.Context("fp64")
    yield c
    c.close()


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def test_boundary_rules_match_oracle(ctx64):
    print("boundary rules", flush=True)
    s = workloads.workload(2).shape
    B = cpu(ctx64.boundary_radial(s.r0, s.a, s.b, s.panels, s.q))
    ref = np.array(oracle.boundary_radial_gl(s.r0, s.a, s.b, s.panels, s.q))
    assert np.abs(B - ref).max() < 1e-14
    B = cpu(ctx64.boundary_radial(1.3, None, None, 0, 77))
    ref = np.array(oracle.boundary_radial_ptr(1.3, n=77))
    assert np.abs(B - ref).max() < 1e-14
    vx = np.array([-1.0, 1.0, 1.0, 0.2, 0.0, -0.2, -1.0])
    vy = np.array([-1.0, -1.0, 1.0, 1.0, 0.1, 1.0, 1.0])
    B = cpu(ctx64.boundary_polygon(vx, vy, 13))
    ref = np.array(oracle.boundary_polygon(vx, vy, 13))
    assert np.abs(B - ref).max() < 1e-15
    for args in ((16, 12.5, 31.0, 12.5, 6.0, 60, 4, 4), (24, 6.0, 12.0, 6.0, 6.0, 37, 3, 0),
                 (5, 1.0, 2.0, 0.7, 4.0, 9, 0, 2)):
        B = cpu(ctx64.boundary_starshade(*args))
        ref = np.array(oracle.boundary_starshade(*args))
        scale = np.abs(ref).max()
        assert np.abs(B - ref).max() < 1e-14 * scale, args
    # host output path
    import paper_2010_05978_amd._binding as abi
    Bh = np.empty((4, 40))
    abi.fh_boundary_radial(ctx64.handle, 1.0, [0.1], [0.2], 2, 20, Bh)
    ref = np.array(oracle.boundary_radial_gl(1.0, [0.1], [0.2], 2, 20))
    assert np.abs(Bh - ref).max() < 1e-14


def _targets(n, seed, rmax=1.5):
    g = np.random.Generator(np.random.PCG64(seed))
    r = rmax * np.sqrt(g.uniform(size=n)); t = g.uniform(0, 2 * np.pi, n)
    return r * np.cos(t), r * np.sin(t)


@pytest.mark.parametrize("M,panels", [(1, 20), (257, 20), (5000, 20), (4099, 3), (20000, 60)])
def test_nsli_starfish_random(ctx, M, panels):
    print(f"nsli starfish M={M} panels={panels} {ctx.precision}", flush=True)
    s = workloads.workload(2).shape
    wl = workloads.workload(2)
    X, Y, W, V = oracle.boundary_radial_gl(s.r0, s.a, s.b, panels, s.q)
    xi, eta = _targets(M, 1000 + M)
    # targets on nodes, and next to them
    k = min(M, 6)
    xi[:k] = X[:k]; eta[:k] = Y[:k]
    if M > 12:
        xi[6:12] = X[10:16] + 1e-9; eta[6:12] = Y[10:16] - 1e-12
    ref = oracle.nsli(X, Y, W, V, wl.lam, wl.z, xi, eta)
    B = ctx.boundary_radial(s.r0, s.a, s.b, panels, s.q)
    u = cpu(ctx.field_nsli(B, wl.lam, wl.z, dev(xi), dev(eta)))
    assert relL2(u, ref) < TOL[ctx.precision]
    assert np.abs(u - ref).max() < (1e-13 if ctx.precision == "fp64" else 1e-6)


def test_nsli_workload2_grid_sampled(ctx):
    # full 1000 x 1000 target grid of workload 2 on the 400-node outline,
    # in the launch shape the benchmark times; sampled against the oracle
    print(f"nsli workload 2 grid {ctx.precision}", flush=True)
    wl = workloads.workload(2)
    s = wl.shape
    g = wl.grid
    xi, eta = oracle.grid_targets(g.n1, g.n2, g.h1, g.h2)
    B = ctx.boundary_radial(s.r0, s.a, s.b, s.panels, s.q)
    u = cpu(ctx.field_nsli(B, wl.lam, wl.z, dev(xi), dev(eta), occulter=True))
    rng = np.random.Generator(np.random.PCG64(77))
    idx = np.concatenate([rng.choice(len(xi), 3000, replace=False), [0, len(xi) - 1]])
    X, Y, W, V = oracle.boundary_radial_gl(s.r0, s.a, s.b, s.panels, s.q)
    ref = oracle.nsli(X, Y, W, V, wl.lam, wl.z, xi[idx], eta[idx], occulter=True)
    assert relL2(1 - u[idx], 1 - ref) < TOL[ctx.precision]
    assert np.isfinite(u).all()


def test_nsli_shadow_option_starshade(ctx):
    # HG outline (sec. 4.2 design) with the eq. li form away from the edge
    print(f"nsli starshade shadow {ctx.precision}", flush=True)
    Np, a, R, b, p = 16, 12.5, 31.0, 12.5, 6.0
    lam, z = 5e-7, 8e7
    xi, eta = _targets(3000, 5, rmax=40.0)
    args = (Np, a, R, b, p, 60, 4, 4)
    X, Y, W, V = oracle.boundary_starshade(*args)
    B = ctx.boundary_starshade(*args)
    for far in (0.0, 0.5):
        ref = oracle.nsli(X, Y, W, V, lam, z, xi, eta, far=far, occulter=True)
        u = cpu(ctx.field_nsli(B, lam, z, dev(xi), dev(eta), far=far, occulter=True))
        assert relL2(u, ref) < TOL[ctx.precision], far
    # midpoint polygon rule: the two forms differ; each matches its oracle
    vx, vy = X[::2].copy(), Y[::2].copy()
    Bp = oracle.boundary_polygon(vx, vy, 1)
    Bd = dev(np.array(Bp))
    for far in (0.0, 1.0):
        ref = oracle.nsli(*Bp, lam, z, xi, eta, far=far, occulter=True)
        u = cpu(ctx.field_nsli(Bd, lam, z, dev(xi), dev(eta), far=far, occulter=True))
        assert np.abs(u - ref).max() < (1e-12 if ctx.precision == "fp64" else 1e-6), far


def test_nsli_node_groups_and_tails(ctx64):
    # few targets and many nodes: the node range is split over workgroups and
    # the partial sums added in a second pass
    print("nsli node groups", flush=True)
    s = workloads.workload(2).shape
    for M, panels in ((3, 400), (700, 100), (2 * 256 * 8 + 1, 33)):
        X, Y, W, V = oracle.boundary_radial_gl(s.r0, s.a, s.b, panels, s.q)
        xi, eta = _targets(M, M)
        ref = oracle.nsli(X, Y, W, V, 1.0, 0.0845, xi, eta, far=0.01)
        u = cpu(ctx64.field_nsli(dev(np.array([X, Y, W, V])), 1.0, 0.0845, dev(xi), dev(eta), far=0.01))
        assert relL2(u, ref) < 1e-12, (M, panels)


def test_nsli_host_memory_and_edge_cases(ctx64, fh):
    print("nsli host memory and edge cases", flush=True)
    import paper_2010_05978_amd._binding as abi
    X, Y, W, V = oracle.boundary_radial_gl(1.0, panels=8, q=20)
    Bh = np.ascontiguousarray(np.array([X, Y, W, V]))
    xi, eta = _targets(100, 3)
    u = np.empty(100, dtype=np.complex128)
    abi.fh_field_nsli(ctx64.handle, Bh, 1.0, 0.1, xi, eta, 0.0, False, u)
    ref = oracle.nsli(X, Y, W, V, 1.0, 0.1, xi, eta)
    assert relL2(u, ref) < 1e-12
    # a single target (one tail lane of one workgroup) gives the same value
    u_one = np.empty(1, dtype=np.complex128)
    abi.fh_field_nsli(ctx64.handle, Bh, 1.0, 0.1, xi[:1].copy(), eta[:1].copy(), 0.0, False, u_one)
    assert abs(u_one[0] - u[0]) < 1e-15
    # empty rule: u_ap = 0, u_oc = 1
    E = torch.empty((4, 0), dtype=torch.float64, device="cuda")
    u0 = cpu(ctx64.field_nsli(E, 1.0, 1.0, dev(xi), dev(eta)))
    assert np.all(u0 == 0)
    u1 = cpu(ctx64.field_nsli(E, 1.0, 1.0, dev(xi), dev(eta), occulter=True))
    assert np.all(u1 == 1)
    # no targets: no-op
    B = dev(Bh)
    out = ctx64.field_nsli(B, 1.0, 1.0, dev(np.empty(0)), dev(np.empty(0)))
    assert out.numel() == 0
    # argument errors
    with pytest.raises(fh.FresnelError, match="FH_ERR_NONPOSITIVE_LZ"):
        ctx64.field_nsli(B, 1.0, -1.0, dev(xi), dev(eta))
    with pytest.raises(fh.FresnelError, match="FH_ERR_NONFINITE"):
        ctx64.field_nsli(B, float("nan"), 1.0, dev(xi), dev(eta))
    with pytest.raises(fh.FresnelError, match="FH_ERR_INVALID_ARG"):
        ctx64.field_nsli(B, 1.0, 1.0, dev(xi), dev(eta), far=-1.0)
    with pytest.raises(fh.FresnelError, match="FH_ERR_INVALID_ARG"):
        ctx64.boundary_starshade(16, 12.5, 10.0, 12.5, 6.0, 60)
    torch.cuda.synchronize()


def test_nsli_agrees_with_type3_field(ctx64):
    # two methods of the library on the same shape: the edge integral over
    # the 60-panel boundary rule and the type-3 field of its dilation rule
    print("nsli vs type 3", flush=True)
    s = workloads.workload(2).shape
    wl = workloads.workload(2)
    xi, eta = _targets(20000, 8)
    B = ctx64.boundary_radial(s.r0, s.a, s.b, 60, s.q)
    q = ctx64.quad_from_boundary(B[0].contiguous(), B[1].contiguous(), B[2].contiguous(), B[3].contiguous(), 200)
    ue = cpu(ctx64.field_nsli(B, wl.lam, wl.z, dev(xi), dev(eta)))
    ua = cpu(ctx64.field_points(q, wl.lam, wl.z, dev(xi), dev(eta)))
    assert relL2(ue, ua) < 1e-9
