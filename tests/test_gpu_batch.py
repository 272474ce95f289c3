"""Batched grid fields (one persistent spread over every instance's work
items, one batched FFT, hipGraph capture and replay), the rule rebuild inside
the graph, and the autotuner (single rule and batch)."""
import os

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


def oracle_quad(s):
    if type(s).__name__ == "RadialCurve":
        return oracle.quad_radial(s.r0, s.a, s.b, s.panels, s.q, s.m)
    return oracle.quad_polygon(s.vx, s.vy, s.q, s.m)


def _batch_inputs(count=6):
    shapes = workloads.batch_shapes(count=count, nmin=3000, nmax=12000)
    lams = workloads.batch_lambdas(64)[:count] * 1.0
    zs = np.full(count, workloads.BATCH_Z)
    occ = np.array([0, 1, 0, 1, 1, 0][:count], dtype=np.int32)
    n = 128
    grid = workloads.Grid(n, n, 3.0 / n, 3.0 / n)
    return shapes, lams, zs, occ, grid


def test_batch_matches_single_and_oracle(ctx):
    shapes, lams, zs, occ, g = _batch_inputs()
    quads = [ctx.quad_for(s) for s in shapes]
    print(f"batch {ctx.precision}: N = {[q.N for q in quads]}", flush=True)
    ub = cpu(ctx.field_grid_batch(quads, lams, zs, g.n1, g.n2, g.h1, g.h2, occulter=occ))
    xi, eta = oracle.grid_targets(g.n1, g.n2, g.h1, g.h2)
    rng = np.random.Generator(np.random.PCG64(31))
    for b, (s, q) in enumerate(zip(shapes, quads)):
        us = cpu(ctx.field_grid(q, lams[b], zs[b], g.n1, g.n2, g.h1, g.h2, occulter=bool(occ[b])))
        ap_b = 1 - ub[b] if occ[b] else ub[b]
        ap_s = 1 - us if occ[b] else us
        assert relL2(ap_b, ap_s) <= TOL[ctx.precision]
        idx = rng.choice(g.M, 400, replace=False)
        x, y, w = oracle_quad(s)
        ref = oracle.fresnel_direct(x, y, w, lams[b], zs[b], xi[idx], eta[idx])
        err = relL2(ap_b.ravel()[idx], ref)
        print(f"  instance {b}: rel L2 vs oracle (400 samples) {err:.2e}", flush=True)
        assert err <= TOL[ctx.precision]


def test_batch_graph_replays(ctx, monkeypatch):
    shapes, lams, zs, occ, g = _batch_inputs(4)
    quads = [ctx.quad_for(s) for s in shapes]
    out = torch.empty((len(quads), g.n2, g.n1), dtype=ctx.cdtype, device="cuda")
    monkeypatch.setenv("FH_NO_GRAPH", "1")
    eager = cpu(ctx.field_grid_batch(quads, lams, zs, g.n1, g.n2, g.h1, g.h2, occulter=occ, out=out)).copy()
    monkeypatch.delenv("FH_NO_GRAPH")
    scratch = torch.randn(1 << 20, device="cuda")
    # LDS atomics of several wavefronts land in any order: replays agree with
    # the eager run to the rounding of the working precision
    rounding = 1e-12 if ctx.precision == "fp64" else 1e-6
    for rep in range(4):
        got = cpu(ctx.field_grid_batch(quads, lams, zs, g.n1, g.n2, g.h1, g.h2, occulter=occ, out=out))
        assert relL2(got, eager) <= rounding, rep
        # the program's own eager work between replays
        scratch.mul_(1.0001)
        ctx.field_grid(quads[0], lams[0], zs[0], g.n1, g.n2, g.h1, g.h2)
        torch.cuda.synchronize()
    # same node counts, different rules: the replay must read the new nodes
    shapes2 = []
    for s in shapes:
        if type(s).__name__ == "RadialCurve":
            shapes2.append(workloads.RadialCurve(0.9 * s.r0, 0.9 * s.a, 0.9 * s.b, s.panels, s.q, s.m))
        else:
            shapes2.append(workloads.Polygon(0.9 * s.vx, 0.9 * s.vy, s.q, s.m))
    quads2 = [ctx.quad_for(s) for s in shapes2]
    got = cpu(ctx.field_grid_batch(quads2, lams, zs, g.n1, g.n2, g.h1, g.h2, occulter=occ, out=out))
    for b, q in enumerate(quads2):
        us = cpu(ctx.field_grid(q, lams[b], zs[b], g.n1, g.n2, g.h1, g.h2, occulter=bool(occ[b])))
        assert relL2(got[b] - (1 if occ[b] else 0), us - (1 if occ[b] else 0)) <= TOL[ctx.precision]


def test_autotune_keeps_accuracy_and_caches(ctx, tmp_path):
    wl = workloads.workload(2)
    s = workloads.RadialCurve(1.0, wl.shape.a, wl.shape.b, panels=12, q=16, m=50)
    q = ctx.quad_for(s)
    n = 200
    h = 0.015
    path = str(tmp_path / "tune.jsonl")
    best = ctx.autotune_grid(q, wl.lam, wl.z, n, n, h, h, cache_path=path)
    print(f"  tuned {ctx.precision}: sigma {best.sigma} tile {best.tile} P {best.max_subproblem} "
          f"method {best.spread_method}", flush=True)
    assert best.spread_method in (1, 2, 3, 4, 5) and best.sigma in (1.25, 2.0)
    assert os.path.exists(path)
    again = ctx.autotune_grid(q, wl.lam, wl.z, n, n, h, h, cache_path=path)
    assert (again.sigma, again.tile, again.max_subproblem, again.spread_method) == \
        (best.sigma, best.tile, best.max_subproblem, best.spread_method)
    u = cpu(ctx.field_grid(q, wl.lam, wl.z, n, n, h, h))
    x, y, w = oracle_quad(s)
    xi, eta = oracle.grid_targets(n, n, h, h)
    ref = oracle.fresnel_direct(x, y, w, wl.lam, wl.z, xi, eta)
    assert relL2(u, ref) <= TOL[ctx.precision]
    ctx.set_options(None)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_single_instance_batches_use_each_calls_parameters(fh, prec):
    """Batched calls with one instance run eagerly: each call must use its
    own rule and wavelength, not those of an earlier call with the same
    shape of arguments (a captured graph would have baked them in)."""
    ctx = fh.Context(prec)
    s = workloads.workload(2).shape
    n, h = 64, 0.03
    xi, eta = oracle.grid_targets(n, n, h, h)
    qa = ctx.quad_radial(s.r0, s.a, s.b, 8, 20, 40)
    qb = ctx.quad_radial(0.8 * s.r0, 0.8 * s.a, 0.8 * s.b, 8, 20, 40)
    xa, ya, wa = oracle.quad_radial(s.r0, s.a, s.b, 8, 20, 40)
    xb, yb, wb = oracle.quad_radial(0.8 * s.r0, 0.8 * s.a, 0.8 * s.b, 8, 20, 40)
    rules = {id(qa): (xa, ya, wa), id(qb): (xb, yb, wb)}
    for q, lam, occ in ((qa, 1.0, 0), (qb, 0.7, 1), (qa, 0.9, 0), (qb, 1.1, 0)):
        u = cpu(ctx.field_grid_batch([q], np.array([lam]), np.array([0.2]), n, n, h, h,
                                     occulter=np.array([occ], dtype=np.int32)))
        x, y, w = rules[id(q)]
        ref = oracle.fresnel_direct(x, y, w, lam, 0.2, xi, eta)
        got = 1 - u[0].ravel() if occ else u[0].ravel()
        assert relL2(got, ref) <= TOL[prec], lam
    qa.close()
    qb.close()
    ctx.close()


class _DeviceArray:
    """A raw device pointer seen by torch (no copy)."""

    def __init__(self, ptr, n):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": "<f8", "data": (ptr, False), "version": 3}


def _wipe_weights(fh, q):
    _, _, wp = fh._binding.fh_quad_device_ptrs(q.handle)
    torch.as_tensor(_DeviceArray(wp, q.N), device="cuda").zero_()


def test_rebuild_batch_recomputes_rules_in_the_graph(ctx, fh):
    shapes, lams, zs, occ, g = _batch_inputs()
    quads = [ctx.quad_for(s) for s in shapes]
    ref = cpu(ctx.field_grid_batch(quads, lams, zs, g.n1, g.n2, g.h1, g.h2, occulter=occ))
    out = torch.empty((len(quads), g.n2, g.n1), dtype=ctx.cdtype, device="cuda")
    for rep in range(3):  # capture, then replays
        # zero every rule's weights: only the rebuild inside the call brings
        # them back
        ctx.synchronize()
        for q in quads:
            _wipe_weights(fh, q)
        torch.cuda.synchronize()
        got = cpu(ctx.field_grid_batch_rebuild(quads, lams, zs, g.n1, g.n2, g.h1, g.h2, occulter=occ, out=out))
        for b in range(len(quads)):
            e = relL2(got[b] - occ[b], ref[b] - occ[b])
            assert e <= TOL[ctx.precision], (rep, b, e)
    print(f"  rebuild {ctx.precision}: three calls match the plain batch", flush=True)
    # the rules hold their constructors' nodes and weights again
    for q, s in zip(quads[:2], shapes[:2]):
        x, y, w = (cpu(t) for t in q.export())
        xo, yo, wo = oracle_quad(s)
        assert np.abs(x - xo).max() <= 1e-14 and np.abs(w - wo).max() <= 1e-14 * np.abs(wo).max()
    # a starshade rule cannot be rebuilt: refused before anything runs
    st = ctx.quad_for(workloads.workload(5, reduced=True).shape)
    with pytest.raises(fh.FresnelError, match="FH_ERR_UNSUPPORTED"):
        ctx.field_grid_batch_rebuild(quads[:2] + [st], lams[:3], zs[:3], g.n1, g.n2, g.h1, g.h2)
    st.close()
    for q in quads:
        q.close()


def test_autotune_batch_keeps_accuracy_flags_and_caches(ctx, fh, tmp_path):
    shapes, lams, zs, occ, g = _batch_inputs()
    quads = [ctx.quad_for(s) for s in shapes]
    path = str(tmp_path / "tune_batch.jsonl")
    ctx.set_options(fh.fh_options(deterministic=1))
    best = ctx.autotune_batch(quads, lams, zs, g.n1, g.n2, g.h1, g.h2, cache_path=path)
    print(f"  batch tuned {ctx.precision}: sigma {best.sigma} tile {best.tile} P {best.max_subproblem} "
          f"method {best.spread_method} deterministic {best.deterministic}", flush=True)
    assert best.spread_method in (2, 4, 5) and best.sigma in (1.25, 2.0)
    assert best.deterministic == 1
    with open(path) as f:
        assert '"key": "batch|' in f.read()
    ctx.set_options(None)
    again = ctx.autotune_batch(quads, lams, zs, g.n1, g.n2, g.h1, g.h2, cache_path=path)
    assert (again.sigma, again.tile, again.max_subproblem, again.spread_method) == \
        (best.sigma, best.tile, best.max_subproblem, best.spread_method)
    assert again.deterministic == 0
    u = cpu(ctx.field_grid_batch(quads, lams, zs, g.n1, g.n2, g.h1, g.h2, occulter=occ))
    xi, eta = oracle.grid_targets(g.n1, g.n2, g.h1, g.h2)
    for b, s in enumerate(shapes):
        x, y, w = oracle_quad(s)
        idx = np.random.Generator(np.random.PCG64(40 + b)).choice(g.M, 200, replace=False)
        ref = oracle.fresnel_direct(x, y, w, lams[b], zs[b], xi[idx], eta[idx])
        got = u[b].ravel()[idx]
        got = 1 - got if occ[b] else got
        assert relL2(got, ref) <= TOL[ctx.precision], b
    ctx.set_options(None)
    for q in quads:
        q.close()


def test_batch_with_empty_and_single_node_instances(ctx):
    """Ragged batches: an instance with no nodes (u_ap = 0, u_oc = 1) and one
    with a single node (a closed form) between ordinary ones, captured and
    replayed."""
    shapes, lams, zs, occ, g = _batch_inputs(count=2)
    quads = [ctx.quad_for(s) for s in shapes]
    empty = ctx.quad_from_nodes(np.zeros(0), np.zeros(0), np.zeros(0))
    x0, y0, w0 = 0.013, -0.021, 0.7
    one = ctx.quad_from_nodes(np.array([x0]), np.array([y0]), np.array([w0]))
    qs = [quads[0], empty, one, quads[1], empty]
    la = np.array([lams[0], lams[1], 0.9e-6, lams[1], 0.7e-6])
    za = np.full(5, workloads.BATCH_Z)
    oc = np.array([0, 1, 0, 1, 0], dtype=np.int32)
    xi, eta = oracle.grid_targets(g.n1, g.n2, g.h1, g.h2)
    out = torch.empty((5, g.n2, g.n1), dtype=ctx.cdtype, device="cuda")
    for rep in range(3):
        u = cpu(ctx.field_grid_batch(qs, la, za, g.n1, g.n2, g.h1, g.h2, occulter=oc, out=out))
        assert np.all(u[1] == 1) and np.all(u[4] == 0), rep
        lz = la[2] * za[2]
        ref1 = np.exp(1j * np.pi * ((xi - x0) ** 2 + (eta - y0) ** 2) / lz) * w0 / (1j * lz)
        assert relL2(u[2].ravel(), ref1) <= TOL[ctx.precision], rep
        for b, s in ((0, shapes[0]), (3, shapes[1])):
            x, y, w = oracle_quad(s)
            idx = np.random.Generator(np.random.PCG64(70 + b)).choice(g.M, 200, replace=False)
            ref = oracle.fresnel_direct(x, y, w, la[b], za[b], xi[idx], eta[idx])
            got = u[b].ravel()[idx]
            got = 1 - got if oc[b] else got
            assert relL2(got, ref) <= TOL[ctx.precision], (rep, b)
    for q in quads + [empty, one]:
        q.close()
