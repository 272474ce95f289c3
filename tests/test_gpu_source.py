"""Source-plane amplitude/phase terms (sec. 5) and a spherical incident wave
(sec. 1) on the GPU against the CPU FP64 oracle.

A rule's illumination (fh_quad_set_illumination) multiplies each areal weight
by its node's source term and, for a point source at distance D, adds
pi |x|^2/(lambda D) to the source chirp.  Every field path (type 1 on a
translated grid, type 3 at points and at a target set, batched type 1
captured and replayed) is compared element by element with the oracle's
direct sum with the same terms; the adjoint refuses both.
"""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-9, "mixed": 1e-5}


def relL2(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


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


def starfish_rule():
    s = workloads.workload(2).shape
    return s, oracle.quad_radial(s.r0, s.a, s.b, 8, 20, 40)


def source_terms(x, y, lz):
    # a tilted wave with a smooth amplitude taper
    return (1.0 + 0.3 * np.cos(2 * x) * np.sin(y)) * np.exp(2j * np.pi * (0.11 * x - 0.05 * y) / lz)


@pytest.mark.parametrize("D", [0.0, 0.7])
def test_source_and_incidence_grid_and_points(ctx, D):
    print(f"source terms, D={D}, {ctx.precision}", flush=True)
    s, (x, y, w) = starfish_rule()
    lam, z = 1.0, 0.2
    q = ctx.quad_radial(s.r0, s.a, s.b, 8, 20, 40)
    src = source_terms(x, y, lam * z)
    q.set_illumination(src, D)
    n, h = 96, 0.02
    u = cpu(ctx.field_grid(q, lam, z, n, n, h, h, xc=0.05, yc=-0.1)).ravel()
    xi, eta = oracle.grid_targets(n, n, h, h, 0.05, -0.1)
    ref = oracle.fresnel_direct_src(x, y, w, lam, z, xi, eta, src=src, D=D)
    err = relL2(u, ref)
    print(f"  grid: rel L2 {err:.2e}", flush=True)
    assert err <= TOL[ctx.precision]
    g = np.random.Generator(np.random.PCG64(77))
    xr, er = g.uniform(-1.2, 1.2, 2000), g.uniform(-1.2, 1.2, 2000)
    dxr, der = torch.tensor(xr, device="cuda"), torch.tensor(er, device="cuda")
    refp = oracle.fresnel_direct_src(x, y, w, lam, z, xr, er, src=src, D=D, occulter=True)
    v = cpu(ctx.field_points(q, lam, z, dxr, der, occulter=True))
    assert relL2(1 - v, 1 - refp) <= TOL[ctx.precision]
    tg = ctx.targets(dxr, der, box=(-1.2, 1.2, -1.2, 1.2))
    v2 = cpu(ctx.field_targets(q, lam, z, tg, occulter=True))
    assert relL2(1 - v2, 1 - refp) <= TOL[ctx.precision]
    tg.close()
    # source terms from a device array, then back to plain illumination
    q.set_illumination(torch.tensor(src, device="cuda"), D)
    u2 = cpu(ctx.field_grid(q, lam, z, n, n, h, h, xc=0.05, yc=-0.1)).ravel()
    assert relL2(u2, ref) <= TOL[ctx.precision]
    q.set_illumination(None, 0.0)
    u0 = cpu(ctx.field_grid(q, lam, z, n, n, h, h, xc=0.05, yc=-0.1)).ravel()
    assert relL2(u0, oracle.fresnel_direct(x, y, w, lam, z, xi, eta)) <= TOL[ctx.precision]
    q.close()


def test_source_terms_in_batches(fh):
    print("source terms in batches", flush=True)
    ctx = fh.Context("fp64")
    s, (x, y, w) = starfish_rule()
    n, h = 64, 0.03
    xi, eta = oracle.grid_targets(n, n, h, h)
    qa = ctx.quad_radial(s.r0, s.a, s.b, 8, 20, 40).set_illumination(None, 2.5)
    qb = ctx.quad_radial(s.r0, s.a, s.b, 8, 20, 40)
    src = source_terms(x, y, 0.2)
    qb.set_illumination(src, 2.5)
    lams, zs = np.array([1.0, 0.8]), np.array([0.2, 0.2])
    ra = oracle.fresnel_direct_src(x, y, w, 1.0, 0.2, xi, eta, D=2.5)
    rb = oracle.fresnel_direct_src(x, y, w, 0.8, 0.2, xi, eta, src=src, D=2.5)
    out = torch.empty((2, n, n), dtype=torch.complex128, device="cuda")
    for rep in range(3):  # capture, then replays
        u = cpu(ctx.field_grid_batch([qa, qb], lams, zs, n, n, h, h, out=out))
        assert relL2(u[0].ravel(), ra) <= 1e-9, rep
        assert relL2(u[1].ravel(), rb) <= 1e-9, rep
    # single-instance batches with and without the terms
    for q, lam, sr in ((qa, 1.0, None), (qb, 0.7, src), (qa, 0.9, None)):
        u = cpu(ctx.field_grid_batch([q], np.array([lam]), np.array([0.2]), n, n, h, h))
        ref = oracle.fresnel_direct_src(x, y, w, lam, 0.2, xi, eta, src=sr, D=2.5)
        assert relL2(u[0].ravel(), ref) <= 1e-9, lam
    # the adjoint refuses source terms and a spherical wave
    gz = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
    with pytest.raises(fh.FresnelError, match="FH_ERR_UNSUPPORTED"):
        ctx.field_grid_vjp(qb, 1.0, 0.2, n, n, h, h, gz)
    with pytest.raises(fh.FresnelError, match="FH_ERR_UNSUPPORTED"):
        ctx.field_grid_vjp(qa, 1.0, 0.2, n, n, h, h, gz)
    with pytest.raises(fh.FresnelError, match="FH_ERR_INVALID_ARG"):
        qa.set_illumination(None, -1.0)
    bad = src.copy()
    bad[3] = np.nan
    with pytest.raises(fh.FresnelError, match="FH_ERR_NONFINITE"):
        qb.set_illumination(bad, 0.0)
    qa.close()
    qb.close()
    ctx.close()
