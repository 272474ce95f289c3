"""Source-plane amplitude/phase terms (sec. 5) and a spherical incident wave
(sec. 1) on the GPU against the CPU FP64 oracle, and single-instance batch
calls with changing parameters.

Every field path (type 1, type 3 at points and at a target set, batched type
1) multiplies each areal weight by its node's source term and, with a point
source at distance D, adds pi |x|^2/(lambda D) to the source chirp; each is
compared element by element with the oracle's direct sum with the same
terms.  The adjoint refuses both.
"""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skip(reason="the library's source-term and spherical-incidence path was taken out: the "
                            "one GPU run of these tests ended its box with a memory-fault report whose "
                            "cause could not be shown; the oracle side stays, pinned"),
]

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


def starfish():
    s = workloads.workload(2).shape
    return s, oracle.quad_radial(s.r0, s.a, s.b, 8, 20, 40)


def source_terms(x, y, lz):
    # a tilted wave with a smooth amplitude taper
    return (1.0 + 0.3 * np.cos(2 * x) * np.sin(y)) * np.exp(2j * np.pi * (0.11 * x - 0.05 * y) / lz)


@pytest.mark.parametrize("D", [0.0, 0.7])
def test_source_and_incidence_grid_and_points(ctx, D):
    print(f"source terms, D={D}, {ctx.precision}", flush=True)
    s, (x, y, w) = starfish()
    lam, z = 1.0, 0.2
    q = ctx.quad_radial(s.r0, s.a, s.b, 8, 20, 40)
    src = source_terms(x, y, lam * z)
    q.set_source(src)
    ctx.set_incidence(D)
    n, h = 96, 0.02
    u = cpu(ctx.field_grid(q, lam, z, n, n, h, h, xc=0.05, yc=-0.1)).ravel()
    xi, eta = oracle.grid_targets(n, n, h, h, 0.05, -0.1)
    ref = oracle.fresnel_direct_src(x, y, w, lam, z, xi, eta, src=src, D=D)
    assert relL2(u, ref) < TOL[ctx.precision]
    g = np.random.Generator(np.random.PCG64(77))
    xr, er = g.uniform(-1.2, 1.2, 2000), g.uniform(-1.2, 1.2, 2000)
    dxr, der = torch.tensor(xr, device="cuda"), torch.tensor(er, device="cuda")
    refp = oracle.fresnel_direct_src(x, y, w, lam, z, xr, er, src=src, D=D, occulter=True)
    v = cpu(ctx.field_points(q, lam, z, dxr, der, occulter=True))
    assert relL2(1 - v, 1 - refp) < TOL[ctx.precision]
    tg = ctx.targets(dxr, der, box=(-1.2, 1.2, -1.2, 1.2))
    v2 = cpu(ctx.field_targets(q, lam, z, tg, occulter=True))
    assert relL2(1 - v2, 1 - refp) < TOL[ctx.precision]
    tg.close()
    # a device source array, then removing the terms and the spherical wave
    q.set_source(torch.tensor(src, device="cuda"))
    u2 = cpu(ctx.field_grid(q, lam, z, n, n, h, h, xc=0.05, yc=-0.1)).ravel()
    assert relL2(u2, ref) < TOL[ctx.precision]
    q.set_source(None)
    ctx.set_incidence(0.0)
    u0 = cpu(ctx.field_grid(q, lam, z, n, n, h, h, xc=0.05, yc=-0.1)).ravel()
    assert relL2(u0, oracle.fresnel_direct(x, y, w, lam, z, xi, eta)) < TOL[ctx.precision]
    q.close()


def test_source_batch_and_single_instance_batches(fh):
    print("source terms in batches", flush=True)
    ctx = fh.Context("fp64")
    s, (x, y, w) = starfish()
    n, h = 64, 0.03
    xi, eta = oracle.grid_targets(n, n, h, h)
    qa = ctx.quad_radial(s.r0, s.a, s.b, 8, 20, 40)
    qb = ctx.quad_radial(s.r0, s.a, s.b, 8, 20, 40)
    src = source_terms(x, y, 0.2)
    qb.set_source(src)
    ctx.set_incidence(2.5)
    lams, zs = np.array([1.0, 0.8]), np.array([0.2, 0.2])
    for _ in range(2):  # capture, then replay
        u = cpu(ctx.field_grid_batch([qa, qb], lams, zs, n, n, h, h))
        ra = oracle.fresnel_direct_src(x, y, w, 1.0, 0.2, xi, eta, D=2.5)
        rb = oracle.fresnel_direct_src(x, y, w, 0.8, 0.2, xi, eta, src=src, D=2.5)
        assert relL2(u[0].ravel(), ra) < 1e-9
        assert relL2(u[1].ravel(), rb) < 1e-9
    ctx.set_incidence(0.0)
    # single-instance batches: each call's own rule and wavelength (no stale
    # parameters from an earlier call of the same shape)
    for q, lam, sr in ((qa, 1.0, None), (qb, 0.7, src), (qa, 0.9, None)):
        u = cpu(ctx.field_grid_batch([q], np.array([lam]), np.array([0.2]), n, n, h, h))
        ref = oracle.fresnel_direct_src(x, y, w, lam, 0.2, xi, eta, src=sr)
        assert relL2(u[0].ravel(), ref) < 1e-9, lam
    # the adjoint refuses source terms and a spherical wave
    g = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
    with pytest.raises(fh.FresnelError, match="FH_ERR_UNSUPPORTED"):
        ctx.field_grid_vjp(qb, 1.0, 0.2, n, n, h, h, g)
    ctx.set_incidence(3.0)
    with pytest.raises(fh.FresnelError, match="FH_ERR_UNSUPPORTED"):
        ctx.field_grid_vjp(qa, 1.0, 0.2, n, n, h, h, g)
    with pytest.raises(fh.FresnelError, match="FH_ERR_INVALID_ARG"):
        ctx.set_incidence(-1.0)
    qa.close()
    qb.close()
    ctx.close()
