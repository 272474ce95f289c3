#!/usr/bin/env python3
"""Throughput of the fast Fresnel-diffraction path on one MI355X.

Headline step: the batched workload (workload 4 of workloads.py) -- 256
random shapes (smooth radial Fourier curves and polygons, node counts uniform
in [1e4, 4e5], 51.7 million nodes in all), one wavelength each from 64
log-spaced in [0.5, 1.0] um, z = 1e5 m, every shape's field on a 512 x 512
grid over [-1.5, 1.5)^2 (67.1 million targets), as one batched call: strengths
and binning, the spread over every instance's work items, the row FFTs, the
column FFTs with the deconvolving epilogue, replayed from a hipGraph, with the
options the batch autotuner picks for this batch (tuned before the timed
region).  As in the paper's timings, the rules are built before the timed
region; a second figure (with_rules) regenerates all 256 rules on the device
inside the same captured graph in every step.

value = targets/s of the FP64 path (tolerance 1e-9, relative L2 against the
exact quadrature sum); beside it the mixed-precision path (tolerance 1e-5) and
the plain FP64 single-instance form (256 separate calls).  Shape parameters
and rules are resident on the device before the timed region starts.

The roofline entry is for the kernel with the most device time in the
headline step (the spread), from its average launch time measured live with
HIP events on the library's stream over a second pass of the same steps,
against MI355X's published peak for the unit that bounds it (the matrix
cores for the matrix-core spread), with the measured ceilings beside it
(fh_probe_ceilings).  Further legs: the
starshade of workload 3 (2048^2 grid and 1e6 pupil points at 3 wavelengths),
the starfish of workload 2, the shape gradient of workload 5, the edge
integral and the paper's own tasks (kite, HG starshade, Koch snowflake).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "target pts/s at 1e-9 (FP64) vs 1e-5 (mixed); backward/forward time ratio"
# HBM traffic of the headline's spread (rocprofv3 FETCH_SIZE and WRITE_SIZE,
# copy-calibrated), tied to the kernel sources it was taken on
TRAFFIC_FILES = [os.path.join(ROOT, "profiles", f)
                 for f in ("traffic_batch256_spread_fp64.json", "traffic_batch256_spread_mixed.json")]
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2010_05978_amd", "csrc", f)
                  for f in ("fh_kernels.hpp", "fh_fft.hpp", "fh_field.hip", "fh_common.hpp")]
ALL_PARTS = "batch,single,starshade,starfish,grad,nsli,kite,koch,hg"


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the headline oracle sample")
    ap.add_argument("--only", choices=["fp64", "mixed"], default=None, help="time one precision only")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON-lines cache of the batch autotuner (a later run with the same file skips the tuning)")
    ap.add_argument("--pmc-calib", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration for rocprofv3 --pmc)")
    ap.add_argument("--parts", default=ALL_PARTS,
                    help="comma list of " + ALL_PARTS + " (profiling one part alone; without batch the line "
                         "carries no value)")
    return ap.parse_args()


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def cuda_ms(fn, steps, warmup):
    """Average milliseconds of fn() over `steps` calls after `warmup`, by host
    wall clock with a device synchronisation on both sides."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / steps


# ------------------------------------------------------------ headline leg
class Batch:
    """Workload 4: 256 rules resident on the device, one batched grid call."""

    def __init__(self, fh, precision):
        import numpy as np
        import torch
        import workloads
        self.ctx = fh.Context(precision)
        self.shapes = workloads.batch_shapes()
        self.B = len(self.shapes)
        lam64 = workloads.batch_lambdas(64)
        self.lams = np.array([lam64[i % 64] for i in range(self.B)])
        self.zs = np.full(self.B, workloads.BATCH_Z)
        self.g = workloads.BATCH_GRID
        self.quads = [self.ctx.quad_for(s) for s in self.shapes]
        self.N = sum(q.N for q in self.quads)
        self.M = self.B * self.g.M
        self.out = torch.empty((self.B, self.g.n2, self.g.n1), dtype=self.ctx.cdtype, device="cuda")
        self.tuned = None

    def tune(self, cache=None):
        """Options of the batched call from the batch autotuner (graph replays
        of this batch over methods, tiles, item sizes and sigma), or from its
        cache file when that holds this batch's signature."""
        g = self.g
        t0 = time.perf_counter()
        o = self.ctx.autotune_batch(self.quads, self.lams, self.zs, g.n1, g.n2, g.h1, g.h2, cache_path=cache)
        self.tuned = {"sigma": o.sigma, "tile": o.tile, "max_subproblem": o.max_subproblem,
                      "spread_method": o.spread_method, "tuning_s": time.perf_counter() - t0}
        return self.tuned

    def field(self, quads=None):
        g = self.g
        self.ctx.field_grid_batch(quads or self.quads, self.lams, self.zs, g.n1, g.n2, g.h1, g.h2, out=self.out)

    def field_rebuild(self):
        """The batched field with all 256 rules generated again on the device
        inside the same captured graph."""
        g = self.g
        self.ctx.field_grid_batch_rebuild(self.quads, self.lams, self.zs, g.n1, g.n2, g.h1, g.h2, out=self.out)

    def with_rules_api(self):
        """Build all 256 rules through the API (one call each), then the
        batched field."""
        quads = [self.ctx.quad_for(s) for s in self.shapes]
        self.field(quads)
        for q in quads:
            q.close()

    def close(self):
        for q in self.quads:
            q.close()
        self.ctx.close()


# MI355X published dense peaks (matrix cores, vector FP64) and HBM bandwidth
MFMA_PEAK_TFLOPS = {"fp64": 78.6, "mixed": 157.3}
FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


def spread_name(prec, W, method=5, tile=0):
    """Kernel name of the spread for width W, method and tile option (0:
    the method's own tile): the matrix-core spread holds a 16-cell padded
    tile (tile 17 - W) in one 16 x 16 block, a larger one in 2 x 2 blocks, and
    stages 16 points at a time; the wavefront spread takes two wavefronts per
    work item when their two tiles and the staging fit 64 KiB."""
    rs = 8 if prec == "fp64" else 4
    real = "double" if rs == 8 else "float"
    if method == 5 and W <= 11:
        T = tile if tile else 17 - W
        return f"k_spread_mfma<{real}, {W}, {1 if T + W - 1 <= 16 else 2}, 16>"
    T = tile if tile else 16
    L = T + W - 1
    if method == 4:
        return f"k_spread_reg<{real}, {W}, {T}>"
    tile_b = 2 * rs * (L * L + 1)
    staging = rs * (64 * (2 * W + 2) + 128)
    nv = 2 if 2 * tile_b + staging <= 64 * 1024 else 1
    return f"k_spread_wave<{real}, {W}, {'true' if method == 3 else 'false'}, {nv}>"


def batch_leg(fh, prec, steps, warmup, ceilings, tune_cache=None):
    """Throughput of the batched call, the same steps with the rules built in
    each, and the spread's average launch time from HIP events on the
    library's stream (timing on: the batch then runs eagerly, stage [1]
    brackets the spread kernel alone)."""
    b = Batch(fh, prec)
    tuned = b.tune(tune_cache)
    ms = cuda_ms(b.field, steps, warmup)
    ms_rules = cuda_ms(b.field_rebuild, steps, warmup)
    ms_api = cuda_ms(b.with_rules_api, max(3, steps // 4), 1)
    b.ctx.set_timing(True)
    b.ctx.timing_totals(3, reset=True)
    for _ in range(steps):
        b.field()
    tot, n = b.ctx.timing_totals(3)
    b.ctx.set_timing(False)
    stages = [v / max(n, 1) for v in tot]
    p = b.ctx.query_params(b.g.n1)
    rs = 8 if prec == "fp64" else 4
    W = p["width"]
    t_spread = stages[1] * 1e-3
    # the method's spreading work: per node and stencil cell a complex
    # strength times two real kernel values, added to the cell (w^2 * 8 flops);
    # the matrix cores issue 16 * 16 * 4 * 2 * 2 / 4 = 1024 flops per node on
    # one 16 x 16 block (real and imaginary parts, four nodes per product)
    flops = b.N * W * W * 8
    hbm_bytes = b.N * (4 + 4 * rs)             # packed cell, offsets and strength per node
    kern = spread_name(prec, W, tuned["spread_method"], tuned["tile"])
    hbm = {"achieved": hbm_bytes / t_spread / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": hbm_bytes / t_spread / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": hbm_bytes,
           "measured_copy_gbs": ceilings["hbm_copy_gbs"]}
    if kern.startswith("k_spread_mfma"):
        # the matrix cores issue 16 * 16 * 4 * 2 * 2 / 4 flops per node and
        # 16 x 16 block (real and imaginary parts, four nodes per product)
        issued = b.N * 1024 * (1 if ", 1, 16>" in kern else 4)
        peak = MFMA_PEAK_TFLOPS[prec]
        roof = {"bound": "mfma", "achieved": flops / t_spread / 1e12, "peak": peak, "unit": "TFLOP/s",
                "frac": flops / t_spread / 1e12 / peak, "traffic": None, "kernel": kern,
                "avg_launch_ms": stages[1], "algorithmic_flops_per_launch": flops,
                "peak_source": "MI355X published dense " + ("FP64" if rs == 8 else "FP32") + " matrix-core peak",
                "issued_mfma_tflops": issued / t_spread / 1e12,
                "measured_mfma_peak_tflops": ceilings["mfma_f64_tflops" if rs == 8 else "mfma_f32_tflops"],
                "hbm": hbm}
    else:
        # one complex read-modify-write of an LDS cell per stencil cell and node
        lds_bytes = b.N * W * W * 4 * rs
        lds_peak = ceilings["lds_rmw_c128_gbs" if prec == "fp64" else "lds_rmw_c64_gbs"]
        roof = {"bound": "lds", "achieved": lds_bytes / t_spread / 1e9, "peak": lds_peak, "unit": "GB/s",
                "frac": lds_bytes / t_spread / 1e9 / lds_peak, "traffic": None, "kernel": kern,
                "avg_launch_ms": stages[1], "algorithmic_bytes_per_launch": lds_bytes,
                "peak_source": "fh_probe_ceilings: LDS read-modify-write of complex cells", "hbm": hbm}
    for path in TRAFFIC_FILES:
        if os.path.exists(path):
            t = json.load(open(path))
            if t.get("kernel") == kern and t.get("source_hash") == kernel_source_hash():
                roof["traffic"] = t.get("bytes_per_launch")
    out = {"value": b.M / (ms * 1e-3), "unit": "targets/s", "ms_per_call": ms, "nodes_per_s": b.N / (ms * 1e-3),
           "instances": b.B, "nodes": b.N, "targets": b.M, "tolerance": b.ctx.tol,
           "dtype": "f64" if prec == "fp64" else "c64-f64phase", "params": p,
           "stages_ms": {"strengths_and_binning": stages[0], "spread": stages[1],
                         "slot_merge_reduce_row_fft": stages[2], "column_fft_epilogue": stages[3],
                         "whole_call_eager": stages[4]},
           "with_rules": {"ms_per_step": ms_rules, "value": b.M / (ms_rules * 1e-3),
                          "note": "the 256 rule kernels and the batched call in one captured graph per step "
                                  "(fh_field_grid_batch_rebuild)"},
           "rules_through_api": {"ms_per_step": ms_api,
                                 "note": "256 fh_quad_* calls (allocation and one launch each), then the "
                                         "batched call"},
           "tuned_options": tuned,
           "roofline": roof}
    b.close()
    return out


def single_leg(fh, steps, warmup):
    """The plain FP64 single-instance form of workload 4: the same 256 rules
    and grids, one fh_field_grid call each."""
    b = Batch(fh, "fp64")
    g = b.g
    u = b.out

    def step():
        for i, q in enumerate(b.quads):
            b.ctx.field_grid(q, b.lams[i], b.zs[i], g.n1, g.n2, g.h1, g.h2, out=u[i])

    ms = cuda_ms(step, steps, warmup)
    out = {"value": b.M / (ms * 1e-3), "unit": "targets/s", "ms_per_step": ms, "calls_per_step": b.B,
           "dtype": "f64", "tolerance": 1e-9}
    b.close()
    return out


# --------------------------------------------------------- CPU baselines
def oracle_rules(shape):
    import oracle
    if type(shape).__name__ == "RadialCurve":
        return oracle.quad_radial(shape.r0, shape.a, shape.b, shape.panels, shape.q, shape.m)
    if type(shape).__name__ == "Polygon":
        return oracle.quad_polygon(shape.vx, shape.vy, shape.q, shape.m)
    s = shape
    return oracle.quad_starshade(s.Np, s.a, s.R, s.b, s.p, s.m, s.np_, s.nd, s.md, s.coef, s.K)


def oracle_sample(cases, seconds, seed):
    """Time the oracle's direct sum over cases [(rule, lam, z, xi, eta)] on
    seeded target samples, case by case, until about `seconds` of CPU time;
    returns (targets, node-target pairs, seconds)."""
    import numpy as np
    import oracle
    rng = np.random.Generator(np.random.PCG64(seed))
    done_t = done_p = 0
    spent = 0.0
    order = rng.permutation(len(cases))
    k = 0
    while spent < seconds:
        (x, y, w), lam, z, xi, eta = cases[order[k % len(cases)]]
        # about 0.5 s per case at ~1e9 pairs/s
        m = int(max(64, min(len(xi), 5e8 / max(len(x), 1))))
        idx = rng.choice(len(xi), m, replace=False)
        t0 = time.perf_counter()
        oracle.fresnel_direct(x, y, w, lam, z, xi[idx], eta[idx])
        spent += time.perf_counter() - t0
        done_t += m
        done_p += m * len(x)
        k += 1
    return done_t, done_p, spent


def cpu_baseline_batch(seconds):
    """The oracle (direct FP64 sum, -O3 -march=native, every host core) on a
    seeded sample of workload 4's targets; the full workload's time is
    extrapolated from the measured node-target pair rate.  A 1-core figure
    comes from a shorter run of the same sample kind."""
    import oracle
    import workloads
    shapes = workloads.batch_shapes()
    lam64 = workloads.batch_lambdas(64)
    g = workloads.BATCH_GRID
    xi, eta = oracle.grid_targets(g.n1, g.n2, g.h1, g.h2)
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(4242))
    pick = rng.choice(len(shapes), 24, replace=False)
    cases = [(oracle_rules(shapes[i]), lam64[i % 64], workloads.BATCH_Z, xi, eta) for i in pick]
    total_pairs = sum(s.n_nodes for s in shapes) * g.M
    cores = oracle.num_threads()
    t, pairs, dt = oracle_sample(cases, seconds, 7)
    rate = pairs / dt
    oracle.set_threads(1)
    t1, pairs1, dt1 = oracle_sample(cases, max(1.0, seconds / 4), 8)
    oracle.set_threads(cores)
    return {"value": t / dt, "unit": "targets/s", "cores": cores, "kind": "oracle",
            "sample": f"{t} grid targets of 24 of the 256 instances (seeded), direct FP64 sum over each "
                      f"instance's nodes, {dt:.1f} s; -O3 -march=native",
            "pairs_per_s": rate, "extrapolated_full_workload_s": total_pairs / rate,
            "extrapolated_targets_per_s": len(shapes) * g.M / (total_pairs / rate),
            "one_core": {"value": t1 / dt1, "unit": "targets/s", "pairs_per_s": pairs1 / dt1,
                         "sample": f"{t1} targets, {dt1:.1f} s"}}


# -------------------------------------------------------- starshade leg
def starshade_leg(fh, prec, steps, warmup, cpu_seconds):
    """Workload 3: the 24-petal starshade (998,400 nodes, z = 3.7e7 m) at
    lambda = 0.5, 0.75 and 1.0 um; per wavelength the type-1 field on the
    2048^2 grid over [-2.4, 2.4)^2 and the type-3 field at 1e6 uniform points
    in the 2.4 m pupil (a target set planned on the pupil box).  The rule is
    built once before the timed region (reused across wavelengths, sec.
    4.3)."""
    import torch
    import workloads
    wl = workloads.workload(3)
    ctx = fh.Context(prec)
    q = ctx.quad_for(wl.shape)
    g = wl.grid
    xi = torch.tensor(wl.points[0], device="cuda")
    eta = torch.tensor(wl.points[1], device="cuda")
    P = wl.pupil
    tg = ctx.targets(xi, eta, box=(-P, P, -P, P))
    ug = torch.empty((g.n2, g.n1), dtype=ctx.cdtype, device="cuda")
    up = torch.empty(xi.numel(), dtype=ctx.cdtype, device="cuda")

    def grid_only():
        for lam in wl.lams:
            ctx.field_grid(q, lam, wl.z, g.n1, g.n2, g.h1, g.h2, occulter=True, out=ug)

    def pts_only():
        for lam in wl.lams:
            ctx.field_targets(q, lam, wl.z, tg, occulter=True, out=up)

    ms_g = cuda_ms(grid_only, steps, warmup)
    ms_p = cuda_ms(pts_only, steps, warmup)
    nl = len(wl.lams)
    out = {"workload": "24-petal starshade, 998400 nodes, 3 wavelengths; 2048^2 grid (type 1) and 1e6 pupil "
                       "points (type 3), rule built once",
           "dtype": "f64" if prec == "fp64" else "c64-f64phase", "tolerance": ctx.tol,
           "grid": {"ms_per_step": ms_g, "value": nl * g.M / (ms_g * 1e-3), "unit": "targets/s"},
           "points": {"ms_per_step": ms_p, "value": nl * xi.numel() / (ms_p * 1e-3), "unit": "targets/s"},
           "value": nl * (g.M + xi.numel()) / ((ms_g + ms_p) * 1e-3), "unit": "targets/s"}
    tg.close()
    q.close()
    ctx.close()
    if cpu_seconds > 0:
        import oracle
        rule = oracle_rules(wl.shape)
        xg, eg = oracle.grid_targets(g.n1, g.n2, g.h1, g.h2)
        cases = [(rule, lam, wl.z, xg, eg) for lam in wl.lams] + \
                [(rule, lam, wl.z, wl.points[0], wl.points[1]) for lam in wl.lams]
        t, pairs, dt = oracle_sample(cases, cpu_seconds, 11)
        full = nl * (g.M + xi.numel()) * wl.shape.n_nodes / (pairs / dt)
        out["cpu_baseline"] = {"value": t / dt, "unit": "targets/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "sample": f"{t} grid and pupil targets (seeded), direct FP64 "
                                                           f"sum over all 998400 nodes, {dt:.1f} s",
                               "extrapolated_full_workload_s": full}
    return out


# --------------------------------------------------------- starfish leg
class Step:
    """Workload 2, one pass: the quadrature rule, its field on the grid (type
    1) and at the scattered targets (type 3).  The two field calls are
    independent and run on two streams, each context building its own copy of
    the rule (one kernel, a few microseconds) so that nothing orders one
    stream after the other: a cross-stream wait costs more than the rule.  The
    scattered targets become a target set every step, planned on the pupil's
    box |x|, |y| <= 1.5 that the workload draws them in, so no call reads
    anything back to the host."""

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
        qb = self.ctx_pts.quad_for(self.shape)
        tg = self.ctx_pts.targets(self.xi, self.eta, box=self.box)
        self.ctx_pts.field_targets(qb, wl.lam, wl.z, tg, out=self.upts)
        qb.close()
        tg.close()
        qa = self.ctx.quad_for(self.shape)
        self.ctx.field_grid(qa, wl.lam, wl.z, g.n1, g.n2, g.h1, g.h2, out=self.ugrid)
        qa.close()

    def close(self):
        self.ctx.close()
        self.ctx_pts.close()


def starfish_leg(fh, prec, steps, warmup, cpu_seconds):
    """Workload 2 (starfish, Fresnel number 20, 40,000 nodes): the rule built
    each step on each of two streams, the 1000^2 grid (type 1) and 1e5
    random points (type 3)."""
    import torch
    import workloads
    wl = workloads.workload(2)
    st = Step(fh, prec, wl, torch.device("cuda", 0))
    ms = cuda_ms(st, steps, warmup)
    out = {"workload": "starfish r = 1 + 0.3 cos 5t, Fresnel number 20, 40000 nodes; 1000^2 grid + 1e5 random "
                       "targets on two streams; rule built each step",
           "dtype": "f64" if prec == "fp64" else "c64-f64phase", "tolerance": st.ctx.tol,
           "ms_per_step": ms, "value": st.M / (ms * 1e-3), "unit": "targets/s"}
    st.close()
    if cpu_seconds > 0:
        import oracle
        import numpy as np
        rule = oracle_rules(wl.shape)
        xg, eg = oracle.grid_targets(wl.grid.n1, wl.grid.n2, wl.grid.h1, wl.grid.h2)
        cases = [(rule, wl.lam, wl.z, np.concatenate([xg, wl.points[0]]), np.concatenate([eg, wl.points[1]]))]
        t, pairs, dt = oracle_sample(cases, cpu_seconds, 13)
        out["cpu_baseline"] = {"value": t / dt, "unit": "targets/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "sample": f"{t} of the step's targets (seeded), direct FP64 sum "
                                                           f"over all 40000 nodes, {dt:.1f} s"}
    return out


def grad_ratio(fh, precision, steps, warmup):
    """Backward/forward device time of the starshade shape-gradient problem
    (workload 5: 998,400 nodes, 384 edge coefficients, 512^2 pupil grid with
    the k1^2 + k2^2 < 256^2 mask, 3 wavelengths, loss = mean |u_oc|^2): the
    sweep form (the rule built once per forward, one batched call for the
    three fields; the backward sums the node gradients over the wavelengths
    in one call and chains them to the coefficients once), and beside it the
    per-wavelength form (a rule, a field and a chain rule per wavelength)."""
    import torch
    import workloads
    from paper_2010_05978_amd.autograd import starshade_field, starshade_sweep
    wl = workloads.workload(5)
    ctx = fh.Context(precision)
    rdt = torch.float64 if precision == "fp64" else torch.float32
    mask = torch.tensor(workloads.pupil_mask(wl.grid.n1), dtype=rdt, device="cuda")
    Min = float(mask.sum())
    nl = len(wl.lams)
    coef = torch.tensor(wl.shape.coef, dtype=torch.float64, device="cuda", requires_grad=True)

    def sweep():
        u = starshade_sweep(coef, ctx, wl.shape, wl.lams, wl.z, wl.grid, occulter=True)
        return ((u.abs() ** 2).reshape(nl, -1) * mask.reshape(1, -1)).sum() / (nl * Min)

    def per_wavelength():
        L = 0.0
        for lam in wl.lams:
            u = starshade_field(coef, ctx, wl.shape, lam, wl.z, wl.grid, occulter=True)
            L = L + ((u.abs() ** 2).reshape(-1) * mask).sum() / (nl * Min)
        return L

    def timed(forward):
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
        return 1e3 * fwd / steps, 1e3 * bwd / steps

    f1, b1 = timed(sweep)
    f0, b0 = timed(per_wavelength)
    ctx.close()
    return {"fwd_ms": f1, "bwd_ms": b1, "ratio": b1 / f1,
            "per_wavelength": {"fwd_ms": f0, "bwd_ms": b0, "ratio": b0 / f0},
            "workload": "24-petal starshade, 998400 nodes, 384 edge coefficients, 512^2 masked pupil, "
                        "3 wavelengths; forward includes quadrature generation (once per forward)"}


# FP64 flops per node-target pair of the edge-integral kernel (an FMA counts
# 2): the inner loop of k_nsli as built, per pair 31 FMAs and 9 adds or
# multiplies (displacement, r^2, cross product, turns and their reduction,
# the two Taylor series of sin/cos(pi f), the refined reciprocal of r^2 and
# the three accumulations).
NSLI_FLOPS_PER_PAIR = 71


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


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(batches would shard by whole instances and a single large rule by its nodes, "
              "with one reduction of the partial fields; only one GPU is driven here)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2010_05978_amd as fh

    precs = [args.only] if args.only else ["fp64", "mixed"]
    parts = set(args.parts.split(","))
    cpu = not args.no_cpu_baseline
    if cpu:
        import oracle
        oracle.build_native(os.path.join(tempfile.gettempdir(), "fh_oracle_native"))
    pc = fh.Context("fp64")
    ceilings = pc.probe_ceilings()
    pc.close()
    out = {"metric": METRIC, "value": None, "unit": "targets/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64" if precs[0] == "fp64" else "c64-f64phase", "data": "synthetic"}
    if "batch" in parts:
        res = {p: batch_leg(fh, p, args.steps, args.warmup, ceilings, args.tune_cache) for p in precs}
        r = res[precs[0]]
        out.update({
            "value": r["value"], "ms_per_step": r["ms_per_call"],
            "config": {"workload": "256 random shapes (smooth radial Fourier curves and polygons, 8-32 modes), "
                                   "node counts uniform in [1e4, 4e5], one wavelength each from 64 log-spaced in "
                                   "[0.5, 1.0] um, z = 1e5 m; 512x512 grid on [-1.5, 1.5)^2 per shape; one "
                                   "batched call replayed from a hipGraph with autotuned options; rules built "
                                   "before the timed region (with_rules: inside it)",
                       "instances": r["instances"], "nodes": r["nodes"], "targets_per_step": r["targets"],
                       "tolerance": r["tolerance"]},
            "roofline": r["roofline"],
        })
        out["batch"] = res
        if len(precs) > 1:
            out["mixed"] = {"value": res["mixed"]["value"], "ms_per_step": res["mixed"]["ms_per_call"],
                            "dtype": "c64-f64phase", "tolerance": res["mixed"]["tolerance"],
                            "roofline": res["mixed"]["roofline"]}
    out["ceilings"] = ceilings
    if args.pmc_calib:
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
    if "single" in parts and "fp64" in precs:
        out["fp64_single_instance"] = single_leg(fh, 3, 1)
    if "starshade" in parts:
        out["starshade"] = {p: starshade_leg(fh, p, args.steps, args.warmup, 6.0 if cpu and p == precs[0] else 0.0)
                            for p in precs}
    if "starfish" in parts:
        out["starfish"] = {p: starfish_leg(fh, p, args.steps, args.warmup, 4.0 if cpu and p == precs[0] else 0.0)
                           for p in precs}
    if "grad" in parts:
        out["backward_forward"] = {p: grad_ratio(fh, p, 3, 1) for p in precs}
    if "nsli" in parts:
        import workloads
        out["nsli"] = nsli_throughput(fh, workloads.workload(2), args.steps, args.warmup, 3.0 if cpu else 0.0)
    if "kite" in parts:
        out["kite_table"] = kite_table(fh, 5, 2)
    if "koch" in parts:
        out["koch"] = koch_snowflake(fh, 3, 1)
    if "hg" in parts:
        out["hg"] = hg_starshade(fh, 5, 2)
    if cpu and "batch" in parts:
        out["cpu_baseline"] = cpu_baseline_batch(args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
