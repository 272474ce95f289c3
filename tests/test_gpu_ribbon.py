"""The ribbon form of the perturbed starshade (sec. 5) on the GPU: the
device rule node by node against the oracle's, and its field against the
oracle's direct sum, in both precisions, with Gauss-Legendre nodes across
the ribbons and with the line integral on the ideal edge (mr = 0)."""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-9, "mixed": 1e-5}


def relL2(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


@pytest.fixture(scope="module")
def fh():
    import paper_2010_05978_amd as fh
    return fh


@pytest.mark.parametrize("mr", [0, 3])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_ribbon_rule_and_field(fh, prec, mr):
    ctx = fh.Context(prec)
    wl = workloads.workload(5, reduced=True)
    s, g = wl.shape, wl.grid
    q = ctx.quad_starshade_ribbon(s.Np, s.a, s.R, s.b, s.p, s.m, s.np_, s.nd, s.md, s.coef, s.K, mr)
    x, y, w = oracle.quad_starshade_ribbon(s.Np, s.a, s.R, s.b, s.p, s.m, s.np_, s.nd, s.md, s.coef, s.K, mr)
    assert q.N == len(x)
    gx, gy, gw = (t.cpu().numpy() for t in q.export())
    scale = np.abs(w).max()
    print(f"  {prec} mr={mr}: N = {q.N}, max node diff {max(np.abs(gx - x).max(), np.abs(gy - y).max()):.1e}, "
          f"max weight diff {np.abs(gw - w).max() / scale:.1e}", flush=True)
    assert np.abs(gx - x).max() <= 1e-13 * s.R and np.abs(gy - y).max() <= 1e-13 * s.R
    assert np.abs(gw - w).max() <= 1e-13 * scale
    u = ctx.field_grid(q, wl.lam, wl.z, g.n1, g.n2, g.h1, g.h2, occulter=True).cpu().numpy().ravel()
    xi, eta = oracle.grid_targets(g.n1, g.n2, g.h1, g.h2)
    idx = np.random.Generator(np.random.PCG64(71)).choice(g.M, 600, replace=False)
    ref = oracle.fresnel_direct(x, y, w, wl.lam, wl.z, xi[idx], eta[idx], occulter=True)
    err = relL2(1 - u[idx], 1 - ref)
    print(f"    field: rel L2 (u_ap) {err:.2e}", flush=True)
    assert err <= TOL[prec]
    q.close()
    ctx.close()
