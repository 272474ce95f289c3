"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

Every oracle entry point the other tests use runs once, on small inputs, in a
child process that loads a sanitized build of fresnel_oracle.c with the ASan
runtime preloaded; any out-of-bounds access, use after free, signed overflow,
misaligned or null dereference aborts the child.  The results are also
compared with the regular build's, to 1e-12 (the sanitized build is compiled
at -O1 without OpenMP, so sums may round differently)."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = textwrap.dedent('''
    import sys, json
    sys.path.insert(0, {root!r})
    import numpy as np
    import oracle, workloads
    if sys.argv[1] == "san":
        oracle.build_sanitized(sys.argv[2])
    out = {{}}
    xg, wg = oracle.gauss_legendre(9)
    out["gl"] = float(np.sum(wg * xg ** 2))
    s2 = workloads.workload(2).shape
    x, y, w = oracle.quad_radial(s2.r0, s2.a, s2.b, 4, 8, 6)
    out["radial"] = float(np.sum(w))
    xp, yp, wp = oracle.quad_polygon(np.array([1.0, -0.4, -0.6, 0.5]), np.array([0.1, 0.9, -0.7, -0.8]), 5, 4)
    out["polygon"] = float(np.sum(wp))
    X, Y, W, V = oracle.boundary_fourier(np.array([0.0, 1.0, 0.2]), np.array([0.0, 0.0, 0.0]),
                                         np.array([0.0, 0.0, 0.0]), np.array([0.0, 0.8, 0.1]), 3, 6)
    xd, yd, wd = oracle.dilation(X, Y, W, V, 5)
    out["dilation"] = float(np.sum(wd))
    st = workloads.workload(5, reduced=True).shape
    args = (st.Np, st.a, st.R, st.b, st.p, 6, 5, 7, 4)
    xs, ys, ws = oracle.quad_starshade(*args, st.coef, st.K)
    out["starshade"] = float(np.sum(ws))
    xr, yr, wr = oracle.quad_starshade_ribbon(*args, st.coef, st.K, 2)
    out["ribbon"] = float(np.sum(wr))
    xk, yk, wk = oracle.quad_koch(2, [3, 2, 2])
    out["koch"] = float(np.sum(wk))
    xi, eta = oracle.grid_targets(6, 4, 0.2, 0.3)
    u = oracle.fresnel_direct(x, y, w, 1.0, 0.2, xi, eta, occulter=True)
    out["direct"] = [float(np.real(u).sum()), float(np.imag(u).sum())]
    us = oracle.fresnel_direct_src(x, y, w, 1.0, 0.2, xi, eta, src=np.exp(1j * x), D=0.7)
    out["direct_src"] = [float(np.real(us).sum()), float(np.imag(us).sum())]
    g = np.exp(1j * np.arange(len(xi)))
    gx, gy, gw = oracle.fresnel_direct_vjp(xs, ys, ws, 1e-6, 3.7e7, xi, eta, g, occulter=True)
    gc = oracle.starshade_vjp(*args, st.coef, st.K, gx, gy, gw)
    out["vjp"] = float(np.sum(gc))
    Xb, Yb, Wb, Vb = oracle.boundary_radial_gl(s2.r0, s2.a, s2.b, 4, 8)
    un = oracle.nsli(Xb, Yb, Wb, Vb, 1.0, 0.2, xi, eta, far=0.5)
    out["nsli"] = [float(np.real(un).sum()), float(np.imag(un).sum())]
    Xs, Ys, Ws, Vs = oracle.boundary_starshade(st.Np, st.a, st.R, st.b, st.p, 6)
    out["outline"] = float(np.sum(Ws))
    print(json.dumps(out))
''')


def _asan_runtime():
    try:
        p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True, timeout=30)
    except (OSError, subprocess.TimeoutExpired):
        return None
    path = p.stdout.strip()
    return path if path and os.path.isabs(path) and os.path.exists(path) else None


def _run(mode, tmp_path, env=None):
    script = tmp_path / "run_oracle.py"
    script.write_text(SCRIPT.format(root=ROOT))
    p = subprocess.run([sys.executable, str(script), mode, str(tmp_path / "san")], capture_output=True, text=True,
                       env=env, timeout=600)
    return p


def test_oracle_under_sanitizers(tmp_path):
    import json
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no ASan runtime for gcc on this host")
    env = dict(os.environ)
    env["LD_PRELOAD"] = rt
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    san = _run("san", tmp_path, env)
    assert san.returncode == 0, san.stderr[-4000:]
    assert "runtime error" not in san.stderr and "AddressSanitizer" not in san.stderr, san.stderr[-4000:]
    plain = _run("plain", tmp_path)
    assert plain.returncode == 0, plain.stderr[-2000:]
    a = json.loads(san.stdout.strip().splitlines()[-1])
    b = json.loads(plain.stdout.strip().splitlines()[-1])
    assert a.keys() == b.keys()
    for k in a:
        va = a[k] if isinstance(a[k], list) else [a[k]]
        vb = b[k] if isinstance(b[k], list) else [b[k]]
        for p, q in zip(va, vb):
            assert abs(p - q) <= 1e-12 * max(1.0, abs(q)), (k, p, q)
