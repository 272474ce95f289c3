"""The allocation-free edge integral (fh_field_nsli_noalloc) against the
allocating call (fh_field_nsli), through the C ABI, in both precisions: two
calls in a row, the second with fewer nodes and targets, each small enough
that the nodes are split into groups whose partial sums live in the device
scratch (so the second call runs over what the first left there)."""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-9, "mixed": 1e-5}


def relL2(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_edge_integral_matches_allocating_call(prec):
    import paper_2010_05978_amd as fh
    from paper_2010_05978_amd import abi
    ctx = fh.Context(prec)
    wl = workloads.workload(2)
    s = wl.shape
    # (panels, q, targets, far): 400 nodes and 3000 targets (6 node groups),
    # then 192 nodes and 700 targets (3 node groups), the second with the
    # deep-shadow form
    for panels, q, M, far in ((20, 20, 3000, 0.0), (12, 16, 700, 0.3)):
        B = ctx.boundary_radial(s.r0, s.a, s.b, panels, q)
        g = np.random.Generator(np.random.PCG64(900 + M))
        xh, eh = g.uniform(-1.5, 1.5, M), g.uniform(-1.5, 1.5, M)
        xi, eta = torch.tensor(xh, device="cuda"), torch.tensor(eh, device="cuda")
        ref = torch.empty(M, dtype=ctx.cdtype, device="cuda")
        got = torch.full((M,), float("nan"), dtype=ctx.cdtype, device="cuda")
        abi.fh_field_nsli(ctx.handle, B, wl.lam, wl.z, xi, eta, far, True, ref)
        abi.fh_field_nsli_noalloc(ctx.handle, B, wl.lam, wl.z, xi, eta, far, True, got)
        r, v = ref.cpu().numpy(), got.cpu().numpy()
        err = relL2(1 - v, 1 - r)
        print(f"  {prec}: n = {B.shape[1]}, M = {M}: rel L2 (u_ap) against fh_field_nsli {err:.2e}, "
              f"max |diff| {np.abs(v - r).max():.2e}", flush=True)
        assert np.isfinite(v).all()
        assert err <= TOL[prec]
        # and the oracle's edge integral on a sample
        X, Y, W, V = oracle.boundary_radial_gl(s.r0, s.a, s.b, panels, q)
        idx = g.choice(M, 200, replace=False)
        o = oracle.nsli(X, Y, W, V, wl.lam, wl.z, xh[idx], eh[idx], far=far, occulter=True)
        assert relL2(1 - v[idx], 1 - o) <= TOL[prec]
    ctx.close()
