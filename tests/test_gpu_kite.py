"""The kite of sec. 3.1 and Table t:kite on the GPU.

The kite X(t) = 0.5 cos t + 0.5 cos 2t, Y(t) = sin t with the periodic
trapezoid boundary rule (eq. ptr) and the dilation rule: the library's rules
node by node against the oracle's, and the paper's accuracy experiment at its
converged parameters -- the type-3 field at 1e6 random targets in
[-3/2, 3/2]^2 and the type-1 field on the 1000^2 grid with nh = 3, at NUFFT
tolerances 1e-6 and 1e-12, against the oracle's edge integral (eq. nsli) at
every target.  The absolute errors in u_oc must stay within a factor of 2 of
the median and maximum errors the paper prints in Table t:kite (fixture
tests/golden/kite_table.json): the paper's tolerance is its NUFFT library's,
this library's is a relative L2 target on u_ap, and the two choose different
kernels, so the error levels agree in size, not digit for digit.
"""
import json
import os

import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(HERE, "golden", "kite_table.json")) as f:
    KITE = json.load(f)
K = KITE["kite"]


def cpu(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def fh():
    import paper_2010_05978_amd as fh
    return fh


def test_kite_rules_match_oracle(fh):
    print("kite rules", flush=True)
    ctx = fh.Context("fp64")
    for panels, q in ((0, 320), (0, 77), (12, 20)):
        B = cpu(ctx.boundary_fourier(K["ax"], K["bx"], K["ay"], K["by"], panels, q))
        ref = np.array(oracle.boundary_fourier(K["ax"], K["bx"], K["ay"], K["by"], panels, q))
        assert np.abs(B - ref).max() < 1e-14, (panels, q)
    q = ctx.quad_fourier(K["ax"], K["bx"], K["ay"], K["by"], 0, 320, 80)
    x, y, w = (cpu(t) for t in q.export())
    rx, ry, rw = oracle.dilation(*oracle.boundary_fourier(K["ax"], K["bx"], K["ay"], K["by"], 0, 320), 80)
    assert max(np.abs(x - rx).max(), np.abs(y - ry).max(), np.abs(w - rw).max()) < 1e-14
    # the edge integral over the kite outline
    xi = np.linspace(-1.5, 1.5, 301)
    eta = np.sin(7 * xi)
    Bd = ctx.boundary_fourier(K["ax"], K["bx"], K["ay"], K["by"], 0, 320)
    u = cpu(ctx.field_nsli(Bd, 1.0, 0.1, torch.tensor(xi, device="cuda"), torch.tensor(eta, device="cuda")))
    ref = oracle.nsli(*oracle.boundary_fourier(K["ax"], K["bx"], K["ay"], K["by"], 0, 320), 1.0, 0.1, xi, eta)
    assert np.abs(u - ref).max() < 1e-13
    ctx.close()


@pytest.mark.parametrize("row", [0, 1])
def test_table_kite_errors(fh, row):
    r = KITE["rows"][row]
    lz, n, m = r["lambda_z"], r["n"], r["m"]
    b = KITE["targets_box"]
    g = np.random.Generator(np.random.PCG64(31 + row))
    M = r["t3"]["M"]
    xi_r, eta_r = g.uniform(-b, b, M), g.uniform(-b, b, M)
    G = KITE["grid"]
    xi_g, eta_g = oracle.grid_targets(G["n"], G["n"], G["h"], G["h"])
    Bh = oracle.boundary_fourier(K["ax"], K["bx"], K["ay"], K["by"], 0, n)
    print(f"kite table row {row}: oracle edge integral at {M} + {xi_g.size} targets", flush=True)
    ref_r = oracle.nsli(*Bh, 1.0, lz, xi_r, eta_r, occulter=True)
    ref_g = oracle.nsli(*Bh, 1.0, lz, xi_g, eta_g, occulter=True)
    dxi, deta = torch.tensor(xi_r, device="cuda"), torch.tensor(eta_r, device="cuda")
    got = []
    for k, eps in enumerate(r["t3"]["eps"]):
        print(f"kite table row {row}: eps {eps}", flush=True)
        ctx = fh.Context("fp64", tol=eps)
        q = ctx.quad_fourier(K["ax"], K["bx"], K["ay"], K["by"], 0, n, m)
        u3 = cpu(ctx.field_points(q, 1.0, lz, dxi, deta, occulter=True))
        e3 = np.abs(u3 - ref_r)
        u1 = cpu(ctx.field_grid(q, 1.0, lz, G["n"], G["n"], G["h"], G["h"], occulter=True)).ravel()
        e1 = np.abs(u1 - ref_g)
        for kind, e in (("t3", e3), ("t1", e1)):
            med, mx = float(np.median(e)), float(e.max())
            pm, px = r[kind]["median_err"][k], r[kind]["max_err"][k]
            print(f"  {kind} eps {eps}: median {med:.2e} (paper {pm:.1e}), max {mx:.2e} (paper {px:.1e})",
                  flush=True)
            got.append((kind, eps, med, mx, pm, px))
        q.close()
        ctx.close()
    for kind, eps, med, mx, pm, px in got:
        assert med <= 2 * pm and mx <= 2 * px, (kind, eps, med, mx, pm, px)
