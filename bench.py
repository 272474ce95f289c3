#!/usr/bin/env python3
"""Throughput of the fast Fresnel-diffraction path on one MI355X.

A step is one pass of the whole hot path over the starfish workload (Fresnel
number 20; workload 2 of workloads.py): device quadrature generation (20 GL
panels x 20 nodes on the boundary, dilation with 100 radial nodes: 40,000
nodes), the type-1 field on the 1000 x 1000 target grid, and the type-3 field
at 1e5 scattered targets in the disk |x| < 1.5.  Shape parameters and target
coordinates are resident on the device before the timed region starts.

value = targets per second of the FP64 path (tolerance 1e-9, relative L2
against the exact quadrature sum); the mixed-precision path (tolerance 1e-5)
is timed in the same run and reported beside it.  The roofline entry is for
the kernel with the largest device time per step, timed live with HIP events
on the library's streams over a second timed pass of the same steps (the
events cost host time, so the throughput pass runs without them).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# LDS: 256 CUs x 128 bytes per clock x 2.4 GHz ("Rooflines")
LDS_PEAK_GBS = 256 * 128 * 2.4
# HBM traffic of the step's candidate dominant kernels (rocprofv3 FETCH_SIZE and
# WRITE_SIZE, copy-calibrated), each tied to the kernel sources it was taken on
TRAFFIC_FILES = [os.path.join(ROOT, "profiles", f)
                 for f in ("traffic_starfish_F20.json", "traffic_starfish_F20_t1cols.json")]
METRIC = "target pts/s at 1e-9 (FP64) vs 1e-5 (mixed); backward/forward time ratio"
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2010_05978_amd", "csrc", f)
                  for f in ("fh_kernels.hpp", "fh_fft.hpp", "fh_field.hip", "fh_common.hpp")]


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    ap.add_argument("--only", choices=["fp64", "mixed"], default=None, help="time one precision only")
    ap.add_argument("--pmc-calib", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration for rocprofv3 --pmc)")
    ap.add_argument("--no-grad", action="store_true", help="skip the backward/forward ratio (workload 5)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workload 4")
    ap.add_argument("--parts", default="step,grad,batch,nsli,kite,koch,hg",
                    help="comma list of step, grad, batch, nsli, kite, koch, hg to run (profiling one part "
                         "alone; without step the line carries no value)")
    return ap.parse_args()


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


class Step:
    """One pass of the hot path for one precision: the quadrature rule, its
    field on the grid (type 1) and at the scattered targets (type 3).  The two
    field calls are independent and run on two streams, each context building
    its own copy of the rule (one kernel, a few microseconds) so that nothing
    orders one stream after the other: a cross-stream wait costs more than the
    rule.  The scattered targets become a target set every step, planned on the
    pupil's box |x|, |y| <= 1.5 that the workload draws them in, so no call
    reads anything back to the host."""

    def __init__(self, fh, precision, wl, dev):
        import torch
        self.sA = torch.cuda.current_stream(dev)
        self.sB = torch.cuda.Stream(device=dev)
        self.ctx = fh.Context(precision)
        with torch.cuda.stream(self.sB):
            self.ctx_pts = fh.Context(precision)
        self.wl = wl
        self.shape = wl.shape
        g = wl.grid
        self.g = g
        self.xi = torch.tensor(wl.points[0], device=dev)
        self.eta = torch.tensor(wl.points[1], device=dev)
        self.ugrid = torch.empty((g.n2, g.n1), dtype=self.ctx.cdtype, device=dev)
        self.upts = torch.empty(len(wl.points[0]), dtype=self.ctx.cdtype, device=dev)
        self.box = (-wl.pupil, wl.pupil, -wl.pupil, wl.pupil)
        self.M = g.M + len(wl.points[0])

    def __call__(self):
        wl, g = self.wl, self.g
        # type 3 on stream B (enqueued first: its chain is the longer one)
        qb = self.ctx_pts.quad_for(self.shape)
        tg = self.ctx_pts.targets(self.xi, self.eta, box=self.box)
        self.ctx_pts.field_targets(qb, wl.lam, wl.z, tg, out=self.upts)
        # each rule's memory goes back to its own context's pool, reused on
        # the same stream
        qb.close()
        tg.close()
        # type 1 on stream A
        qa = self.ctx.quad_for(self.shape)
        self.ctx.field_grid(qa, wl.lam, wl.z, g.n1, g.n2, g.h1, g.h2, out=self.ugrid)
        qa.close()

    def set_timing(self, on):
        self.ctx.set_timing(on)
        self.ctx_pts.set_timing(on)

    def close(self):
        self.ctx.close()
        self.ctx_pts.close()


def time_steps(step, steps, warmup):
    """Wall time of `steps` steps, then the per-stage device times of another
    `steps` steps timed with HIP events on the library's streams.  Recording
    the events costs host time on every call, so the throughput pass runs
    without them."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    step.set_timing(True)
    step.ctx.timing_totals(0, reset=True)
    step.ctx_pts.timing_totals(1, reset=True)
    torch.cuda.synchronize()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    grid_ms, ngrid = step.ctx.timing_totals(0)
    pts_ms, npts = step.ctx_pts.timing_totals(1)
    step.set_timing(False)
    return dt, [v / max(ngrid, 1) for v in grid_ms], [v / max(npts, 1) for v in pts_ms]


def spread_waves(W, rs, T=16):
    """Wavefronts per spread work item at tile T: two when their two tiles
    (one spare cell each), the staging of 64 points and two wavefronts'
    kernel arguments fit in 64 KiB of LDS."""
    L = T + W - 1
    tile = 2 * rs * (L * L + 1)
    staging = rs * (64 * (2 * W + 2) + 128)
    return 2 if 2 * tile + staging <= 64 * 1024 else 1


def roofline(res, prec, wl):
    """Roofline of the kernel with the most device time per step.

    Candidates are the stages that bracket one kernel: the spread of each
    call, the type-1 epilogue and the type-3 interpolation."""
    r = res[prec]
    p = r["params"]
    W = p["width"]
    rs = 8 if prec == "fp64" else 4
    N = wl.shape.n_nodes
    n1, n2 = wl.grid.n1, wl.grid.n2
    M3 = len(wl.points[0])
    g, pt = r["grid_stage_ms"], r["points_stage_ms"]
    cands = {
        # spread: 2 W^2 LDS atomic adds of one real each per node
        "spread": {"kernel": f"k_spread_wave<{'double' if rs == 8 else 'float'}, {W}, false, {spread_waves(W, rs)}>",
                   "ms": (g[1] + pt[1]) / 2,
                   "launches": 2, "bound": "alu", "unit": "GB/s", "peak": LDS_PEAK_GBS,
                   "bytes": N * W * W * 2 * rs},
        # type-1 column pass + epilogue: at least one complex output written per
        # target (the band it reads is not counted)
        "t1_cols": {"kernel": f"k_t1_cols<{'double' if rs == 8 else 'float'}>", "ms": g[3], "launches": 1,
                    "bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS, "bytes": n1 * n2 * 2 * rs},
        # interpolation: target coordinates and index in, one output out
        "interp": {"kernel": f"k_t3_interp<{'double' if rs == 8 else 'float'}, {W}>", "ms": pt[3], "launches": 1,
                   "bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS, "bytes": M3 * (16 + 4 + 2 * rs)},
    }
    name, c = max(cands.items(), key=lambda kv: kv[1]["ms"] * kv[1]["launches"])
    achieved = c["bytes"] / (c["ms"] * 1e-3) / 1e9
    out = {"bound": c["bound"], "achieved": achieved, "peak": c["peak"], "unit": c["unit"],
           "frac": achieved / c["peak"], "traffic": None, "kernel": c["kernel"],
           "avg_launch_ms": c["ms"], "algorithmic_bytes_per_launch": c["bytes"],
           "per_step_ms": {k: v["ms"] * v["launches"] for k, v in cands.items()}}
    for path in TRAFFIC_FILES:
        if not os.path.exists(path):
            continue
        t = json.load(open(path))
        if t.get("kernel") == c["kernel"] and t.get("source_hash") == kernel_source_hash():
            out["traffic"] = t.get("bytes_per_launch")
    return out


def grad_ratio(fh, precision, steps, warmup):
    """Backward/forward device time of the starshade shape-gradient problem
    (workload 5: 998,400 nodes, 384 edge coefficients, 512^2 pupil grid with
    the k1^2 + k2^2 < 256^2 mask, 3 wavelengths, loss = mean |u_oc|^2)."""
    import torch
    import workloads
    from paper_2010_05978_amd.autograd import starshade_field
    wl = workloads.workload(5)
    ctx = fh.Context(precision)
    rdt = torch.float64 if precision == "fp64" else torch.float32
    mask = torch.tensor(workloads.pupil_mask(wl.grid.n1), dtype=rdt, device="cuda")
    Min = float(mask.sum())
    coef = torch.tensor(wl.shape.coef, dtype=torch.float64, device="cuda", requires_grad=True)

    def forward():
        L = 0.0
        for lam in wl.lams:
            u = starshade_field(coef, ctx, wl.shape, lam, wl.z, wl.grid, occulter=True)
            L = L + ((u.abs() ** 2).reshape(-1) * mask).sum() / (len(wl.lams) * Min)
        return L

    for _ in range(warmup):
        forward().backward()
    fwd = bwd = 0.0
    for _ in range(steps):
        coef.grad = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L = forward()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        fwd += t1 - t0
        bwd += t2 - t1
    ctx.close()
    return {"fwd_ms": 1e3 * fwd / steps, "bwd_ms": 1e3 * bwd / steps, "ratio": bwd / fwd,
            "workload": "24-petal starshade, 998400 nodes, 384 edge coefficients, 512^2 masked pupil, "
                        "3 wavelengths; forward includes quadrature generation"}


def batch_throughput(fh, steps, warmup):
    """Workload 4: 256 random shapes (node counts uniform in [1e4, 4e5]), one
    wavelength each from 64 log-spaced in [0.5, 1.0] um, 512^2 grids, mixed
    precision; one batched call replayed from a hipGraph."""
    import numpy as np
    import torch
    import workloads
    ctx = fh.Context("mixed")
    shapes = workloads.batch_shapes()
    lams = workloads.batch_lambdas(64)
    quads = [ctx.quad_for(s) for s in shapes]
    B = len(quads)
    lam = np.array([lams[i % 64] for i in range(B)])
    zs = np.full(B, workloads.BATCH_Z)
    g = workloads.BATCH_GRID
    out = torch.empty((B, g.n2, g.n1), dtype=ctx.cdtype, device="cuda")
    for _ in range(warmup):
        ctx.field_grid_batch(quads, lam, zs, g.n1, g.n2, g.h1, g.h2, occulter=False, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.field_grid_batch(quads, lam, zs, g.n1, g.n2, g.h1, g.h2, occulter=False, out=out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    N = sum(q.N for q in quads)
    ctx.close()
    return {"value": B * g.M / dt, "unit": "targets/s", "ms_per_call": 1e3 * dt, "nodes_per_s": N / dt,
            "instances": B, "nodes": N, "dtype": "c64-f64phase", "tolerance": 1e-5}


# FP64 flops per node-target pair of the edge-integral kernel (an FMA counts
# 2): the inner loop of k_nsli as built, per pair 31 FMAs and 9 adds or
# multiplies (displacement, r^2, cross product, turns and their reduction,
# the two Taylor series of sin/cos(pi f), the refined reciprocal of r^2 and
# the three accumulations).
NSLI_FLOPS_PER_PAIR = 71
FP64_PEAK_TFLOPS = 78.6


def nsli_throughput(fh, wl, steps, warmup, cpu_seconds):
    """Edge integral (eq. nsli) over the starfish outline (20 GL panels x 20 =
    400 boundary nodes) at the step's 1.1e6 targets (the 1000^2 grid and the
    1e5 scattered points), FP64; one kernel launch per call, timed with HIP
    events on the context's stream.  The oracle's edge integral is timed on a
    seeded sample of the same targets."""
    import numpy as np
    import torch
    import oracle
    ctx = fh.Context("fp64")
    s = wl.shape
    B = ctx.boundary_radial(s.r0, s.a, s.b, s.panels, s.q)
    g = wl.grid
    k1 = torch.arange(-(g.n1 // 2), g.n1 - g.n1 // 2, dtype=torch.float64, device="cuda") * g.h1
    k2 = torch.arange(-(g.n2 // 2), g.n2 - g.n2 // 2, dtype=torch.float64, device="cuda") * g.h2
    XI, ETA = torch.meshgrid(k1, k2, indexing="xy")
    xi = torch.cat([XI.reshape(-1), torch.tensor(wl.points[0], device="cuda")]).contiguous()
    eta = torch.cat([ETA.reshape(-1), torch.tensor(wl.points[1], device="cuda")]).contiguous()
    M, n = xi.numel(), B.shape[1]
    u = torch.empty(M, dtype=torch.complex128, device="cuda")
    for _ in range(warmup):
        ctx.field_nsli(B, wl.lam, wl.z, xi, eta, occulter=True, out=u)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for k in range(steps):
        ctx.field_nsli(B, wl.lam, wl.z, xi, eta, occulter=True, out=u)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    per = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
    ms = sum(per) / steps
    ctx.close()
    achieved = NSLI_FLOPS_PER_PAIR * M * n / (ms * 1e-3) / 1e12
    out = {"value": M / (ms * 1e-3), "unit": "targets/s", "ms_per_call": ms, "pairs_per_s": M * n / (ms * 1e-3),
           "nodes": n, "targets": M, "dtype": "f64",
           "workload": "starfish outline, 20 GL panels x 20 nodes; the step's 1000x1000 grid + 1e5 random targets",
           "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None, "kernel": "k_nsli<2, double>",
                        "flops_per_pair": NSLI_FLOPS_PER_PAIR, "avg_launch_ms": ms}}
    if cpu_seconds > 0:
        X, Y, W, V = oracle.boundary_radial_gl(s.r0, s.a, s.b, s.panels, s.q)
        xh, eh = xi.cpu().numpy(), eta.cpu().numpy()
        rng = np.random.Generator(np.random.PCG64(4343))
        probe = rng.choice(M, 2048, replace=False)
        t0 = time.perf_counter()
        oracle.nsli(X, Y, W, V, wl.lam, wl.z, xh[probe], eh[probe], occulter=True)
        per_t = (time.perf_counter() - t0) / 2048
        m = int(min(M, max(2048, cpu_seconds / max(per_t, 1e-9))))
        idx = rng.choice(M, m, replace=False)
        t0 = time.perf_counter()
        oracle.nsli(X, Y, W, V, wl.lam, wl.z, xh[idx], eh[idx], occulter=True)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": m / dt, "unit": "targets/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "sample": f"{m} of the {M} targets, oracle edge integral "
                                                           f"over all {n} nodes, {dt:.1f} s"}
    return out


def kite_table(fh, steps, warmup):
    """Table t:kite's timing tasks (sec. 3.1) at the paper's converged
    parameters: the kite with the n-node trapezoid boundary rule and m radial
    nodes, the type-3 field at 1e6 random targets in [-3/2, 3/2]^2 (a target
    set with that declared box), the type-1 field on the 1000^2 grid with
    h = 0.003, FP64 contexts at NUFFT tolerances 1e-6 and 1e-12, and the edge
    integral at the same 1e6 random targets.  As in the paper, the quadrature
    is built before the timed calls; the target set is built and sorted into
    spatial order (once) before them too.  The paper's CPU seconds (4-core laptop)
    are reported beside each time as context."""
    import numpy as np
    import torch
    with open(os.path.join(ROOT, "tests", "golden", "kite_table.json")) as f:
        kt = json.load(f)
    k = kt["kite"]
    b = kt["targets_box"]
    G = kt["grid"]
    rows = []
    for ri, r in enumerate(kt["rows"]):
        g = np.random.Generator(np.random.PCG64(31 + ri))
        M = r["t3"]["M"]
        xi = torch.tensor(g.uniform(-b, b, M), device="cuda")
        eta = torch.tensor(g.uniform(-b, b, M), device="cuda")
        stream = torch.cuda.current_stream()

        def timed(fn):
            for _ in range(warmup):
                fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(steps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / steps

        entry = {"lambda_z": r["lambda_z"], "fresnel": r["fresnel"], "n": r["n"], "m": r["m"],
                 "N": r["n"] * r["m"], "M": M, "by_eps": []}
        for ke, eps in enumerate(r["t3"]["eps"]):
            ctx = fh.Context("fp64", tol=eps)
            q = ctx.quad_fourier(k["ax"], k["bx"], k["ay"], k["by"], 0, r["n"], r["m"])
            # the set is evaluated many times: sorted once into spatial order
            tg = ctx.targets(xi, eta, box=(-b, b, -b, b)).sort()
            u3 = torch.empty(M, dtype=torch.complex128, device="cuda")
            u1 = torch.empty((G["n"], G["n"]), dtype=torch.complex128, device="cuda")
            t3 = timed(lambda: ctx.field_targets(q, 1.0, r["lambda_z"], tg, occulter=True, out=u3))
            t1 = timed(lambda: ctx.field_grid(q, 1.0, r["lambda_z"], G["n"], G["n"], G["h"], G["h"],
                                              occulter=True, out=u1))
            entry["by_eps"].append({"eps": eps, "t3_ms": t3, "t1_ms": t1,
                                    "paper_t3_s": r["t3"]["cpu_s"][ke], "paper_t1_s": r["t1"]["cpu_s"][ke]})
            tg.close()
            q.close()
            ctx.close()
        ctx = fh.Context("fp64")
        B = ctx.boundary_fourier(k["ax"], k["bx"], k["ay"], k["by"], 0, r["n"])
        un = torch.empty(M, dtype=torch.complex128, device="cuda")
        entry["nsli_ms"] = timed(lambda: ctx.field_nsli(B, 1.0, r["lambda_z"], xi, eta, occulter=True, out=un))
        entry["paper_nsli_s"] = r["nsli_cpu_s"]
        ctx.close()
        rows.append(entry)
    return {"workload": "kite of sec. 3.1, Table t:kite tasks (quadrature built before timing, as in the paper)",
            "rows": rows}


def koch_orders(L):
    """Rule orders per level of the paper-scale snowflake: 217 on the first
    triangle, halving per level with a floor of 2, and 1 from level 10 on
    (sec. 4.4 gives the two ends of the range)."""
    import math
    return [max(2, math.ceil(217 / 2 ** k)) if k <= 9 else 1 for k in range(L + 1)]


def koch_snowflake(fh, steps, warmup):
    """Sec. 4.4's fractal aperture: the level-13 Koch snowflake (about 68
    million areal nodes, built on the device each call) and its type-1 field
    at lambda z = 0.01 on a 1000^2 grid of spacing 0.003, FP64 at NUFFT
    tolerance 1e-6 as in the paper.  Build and field are timed separately
    with HIP events; the paper's laptop took about 4 minutes to build the
    rule and 4.6 s per field."""
    import torch
    L, lz, n, h = 13, 0.01, 1000, 0.003
    p = koch_orders(L)
    ctx = fh.Context("fp64", tol=1e-6)
    u = torch.empty((n, n), dtype=torch.complex128, device="cuda")
    stream = torch.cuda.current_stream()
    build_ms, field_ms = [], []
    N = 0
    for it in range(warmup + steps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record(stream)
        q = ctx.quad_koch(L, p)
        e[1].record(stream)
        ctx.field_grid(q, 1.0, lz, n, n, h, h, out=u)
        e[2].record(stream)
        torch.cuda.synchronize()
        N = q.N
        q.close()
        if it >= warmup:
            build_ms.append(e[0].elapsed_time(e[1]))
            field_ms.append(e[1].elapsed_time(e[2]))
    ctx.close()
    b, f = sum(build_ms) / steps, sum(field_ms) / steps
    return {"workload": "Koch snowflake level 13 (sec. 4.4), lambda z = 0.01, 1000^2 grid, h = 0.003, "
                        "FP64 at tolerance 1e-6", "levels": L, "orders": p, "nodes": N,
            "build_ms": b, "field_ms": f, "nodes_per_s_field": N / (f * 1e-3),
            "paper_build_s": 240, "paper_field_s": 4.6}


def hg_starshade(fh, steps, warmup):
    """The HG starshade of sec. 4.2 (16 petals, 37,440 nodes): Table t:star's
    type-1 task at tolerance 1e-8 on a 1000^2 grid over [-16, 16)^2 m, and
    the sec. 4.3 wavelength sweep -- 50 wavelengths in [0.4, 1.0] um, at each
    the type-3 field at 200 radii x 300 angles (60,000 targets, one target
    set; the circles are already in spatial order) and the maximum intensity
    over the angles at each radius.  The sweep is timed whole, including
    building the quadrature and the target set once.  The
    paper's laptop took 0.042 s for the grid task and 6 s for the sweeps of
    two starshades."""
    import numpy as np
    import torch
    with open(os.path.join(ROOT, "tests", "golden", "hg_starshade.json")) as f:
        hg = json.load(f)
    half = 16.0
    stream = torch.cuda.current_stream()
    args = (hg["Np"], hg["a"], hg["R"], hg["b"], hg["p"], hg["m"], hg["np"], hg["nd"], hg["md"])
    ctx = fh.Context("fp64", tol=hg["table_t_star"]["t1_eps"])
    q = ctx.quad_starshade(*args)
    n = 1000
    h = 2 * half / n
    u = torch.empty((n, n), dtype=torch.complex128, device="cuda")
    for _ in range(warmup):
        ctx.field_grid(q, hg["lambda"], hg["z"], n, n, h, h, occulter=True, out=u)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        ctx.field_grid(q, hg["lambda"], hg["z"], n, n, h, h, occulter=True, out=u)
    e1.record(stream)
    torch.cuda.synchronize()
    t1_ms = e0.elapsed_time(e1) / steps
    q.close()
    ctx.close()
    sw = hg["sweep"]
    rho = half * np.arange(1, sw["n_radii"] + 1) / sw["n_radii"]
    th = 2 * np.pi * np.arange(sw["n_angles"]) / sw["n_angles"]
    R, T = np.meshgrid(rho, th, indexing="ij")
    xi = torch.tensor((R * np.cos(T)).ravel(), device="cuda")
    eta = torch.tensor((R * np.sin(T)).ravel(), device="cuda")
    lams = np.linspace(0.4e-6, 1.0e-6, sw["n_lambda"])
    ctx = fh.Context("fp64", tol=1e-9)
    M = xi.numel()
    uo = torch.empty(M, dtype=torch.complex128, device="cuda")
    peak = torch.empty((len(lams), sw["n_radii"]), dtype=torch.float64, device="cuda")

    def sweep():
        qq = ctx.quad_starshade(*args)
        tg = ctx.targets(xi, eta, box=(-half, half, -half, half))
        for i, lam in enumerate(lams):
            ctx.field_targets(qq, float(lam), hg["z"], tg, occulter=True, out=uo)
            peak[i] = uo.abs().square().view(sw["n_radii"], sw["n_angles"]).amax(dim=1)
        tg.close()
        qq.close()

    sweep()
    torch.cuda.synchronize()
    e0.record(stream)
    sweep()
    e1.record(stream)
    torch.cuda.synchronize()
    sweep_ms = e0.elapsed_time(e1)
    ctx.close()
    return {"workload": "HG starshade (sec. 4.2), 37440 nodes, z = 8e7 m", "grid_t1": {
                "lambda": hg["lambda"], "n": n, "extent_m": [-half, half], "tol": hg["table_t_star"]["t1_eps"],
                "ms": t1_ms, "paper_s": hg["table_t_star"]["t1_cpu_s"]},
            "sweep_t3": {"wavelengths": len(lams), "lambda_range_m": [lams[0], lams[-1]], "targets": M,
                         "tol": 1e-9, "ms_total": sweep_ms, "ms_per_wavelength": sweep_ms / len(lams),
                         "paper_s_two_starshades": sw["cpu_s_both_starshades"],
                         "max_intensity_in_shadow": float(peak[:, : int(0.6 * sw["n_radii"])].max())}}


def cpu_baseline(wl, seconds):
    """The oracle (direct FP64 sum) on a seeded sample of the step's targets."""
    import numpy as np
    import oracle
    s = wl.shape
    x, y, w = oracle.quad_radial(s.r0, s.a, s.b, s.panels, s.q, s.m)
    xi_g, eta_g = oracle.grid_targets(wl.grid.n1, wl.grid.n2, wl.grid.h1, wl.grid.h2)
    xi = np.concatenate([xi_g, wl.points[0]])
    eta = np.concatenate([eta_g, wl.points[1]])
    rng = np.random.Generator(np.random.PCG64(4242))
    probe = rng.choice(len(xi), 1024, replace=False)
    t0 = time.perf_counter()
    oracle.fresnel_direct(x, y, w, wl.lam, wl.z, xi[probe], eta[probe])
    per = (time.perf_counter() - t0) / 1024
    n = int(min(len(xi), max(1024, seconds / max(per, 1e-9))))
    idx = rng.choice(len(xi), n, replace=False)
    t0 = time.perf_counter()
    oracle.fresnel_direct(x, y, w, wl.lam, wl.z, xi[idx], eta[idx])
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "targets/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{n} of the step's {len(xi)} targets (grid and scattered, seeded), "
                      f"direct FP64 sum over all {len(x)} nodes, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported by this build "
              "(the path shards by instance or by node; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2010_05978_amd as fh
    import workloads

    dev = torch.device("cuda", 0)
    wl = workloads.workload(2)
    precs = [args.only] if args.only else ["fp64", "mixed"]
    parts = set(args.parts.split(","))
    if "step" not in parts:
        out = {"metric": METRIC, "value": None, "unit": "targets/s", "n_gpus": 1, "parts": sorted(parts)}
        if "grad" in parts and not args.no_grad:
            out["backward_forward"] = {p: grad_ratio(fh, p, 3, 1) for p in precs}
        if "batch" in parts and not args.no_batch:
            out["batch"] = batch_throughput(fh, 5, 2)
        if "nsli" in parts:
            out["nsli"] = nsli_throughput(fh, wl, args.steps, args.warmup,
                                          0.0 if args.no_cpu_baseline else 3.0)
        if "kite" in parts:
            out["kite_table"] = kite_table(fh, 5, 2)
        if "koch" in parts:
            out["koch"] = koch_snowflake(fh, 3, 1)
        if "hg" in parts:
            out["hg"] = hg_starshade(fh, 5, 2)
        print(json.dumps(out))
        return
    res = {}
    for p in precs:
        st = Step(fh, p, wl, dev)
        dt, gstage, pstage = time_steps(st, args.steps, args.warmup)
        res[p] = {"ms_per_step": 1e3 * dt / args.steps, "value": st.M * args.steps / dt,
                  "grid_stage_ms": gstage, "points_stage_ms": pstage,
                  "params": st.ctx.query_params(wl.grid.n1)}
        st.close()
    if args.pmc_calib:
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
    main_p = precs[0]
    r = res[main_p]
    out = {
        "metric": METRIC,
        "value": r["value"], "unit": "targets/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if main_p == "fp64" else "c64-f64phase", "data": "synthetic",
        "config": {"workload": "starfish r=1+0.3cos5t, Fresnel number 20, 40000 nodes; 1000x1000 grid "
                               "(type 1) + 1e5 random targets (type 3) on two streams; quadrature generated each "
                               "step (once per stream)",
                   "tolerance": 1e-9 if main_p == "fp64" else 1e-5, "targets_per_step": 1_100_000},
        "roofline": roofline(res, main_p, wl),
        "stages_ms": {p: {"grid": res[p]["grid_stage_ms"], "points": res[p]["points_stage_ms"]} for p in precs},
    }
    if "mixed" in res and main_p != "mixed":
        out["mixed"] = {"value": res["mixed"]["value"], "ms_per_step": res["mixed"]["ms_per_step"],
                        "dtype": "c64-f64phase", "tolerance": 1e-5, "roofline": roofline(res, "mixed", wl)}
    if not args.no_grad and "grad" in parts:
        out["backward_forward"] = {p: grad_ratio(fh, p, 3, 1) for p in precs}
    if not args.no_batch and "batch" in parts:
        out["batch"] = batch_throughput(fh, 5, 2)
    if "nsli" in parts:
        out["nsli"] = nsli_throughput(fh, wl, args.steps, args.warmup, 0.0 if args.no_cpu_baseline else 3.0)
    if "kite" in parts:
        out["kite_table"] = kite_table(fh, 5, 2)
    if "koch" in parts:
        out["koch"] = koch_snowflake(fh, 3, 1)
    if "hg" in parts:
        out["hg"] = hg_starshade(fh, 5, 2)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
