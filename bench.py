"""Benchmark: multigrid time-to-solution and smoother throughput on one MI355X.

Workload (one "step"): reset an 8193 x 8193 unit-square grid (h = 1/8192,
beta = 1, Dirichlet values U[0,1) from seed 2, zero interior, f = 0) and solve
it to ||r||_2/||r_0||_2 < 1e-10 with FP64 V(2,2) multigrid (red-black
Gauss-Seidel smoother, full weighting, bilinear interpolation, 12 levels down
to 5 x 5 solved directly).  `value` is the smoother throughput of the step in
GLUP/s: interior nodes updated by all smoothing sweeps on all levels, per
second of whole-step wall time (inputs resident in HBM).

Also measured in the same run, each leg on its own grids (setup untimed):
  * mixed precision (FP32 V-cycles inside FP64 defect correction) vs FP64
    multigrid on the 8193^2 and 4097^2 grids with a 32-bump source: time to
    1e-10 (graph replay, the third solve of each precision), speedup,
    difference between the two results;
  * red-black SOR with w = 2/(1+sin(pi h)) to 1e-10 on 4097^2 and 8193^2;
    FP64 multigrid on 4097^2;
  * the paper's 25 x 17 chamber on the GPU: red-black SOR for w = 1.00 ..
    1.95, zebra ADI, the 3-level V(2,2) cycle, to max|r| < 1e-6;
  * a ragged batch of 512 grids (mixed multigrid, zebra ADI) and the serving
    loop (Poisson arrivals, 2000 requests per rate after 200 warm-up);
  * the roofline of the dominant kernel (the finest-level kernel class with
    the most device time) from HIP events around each of its launches;
  * the CPU oracle on the host (one FP64 V-cycle of the 8193^2 solve,
    extrapolated to the solve's cycle count), and in the same leg the error
    of the large GPU results against the oracle's exact spectral solution.

stdout: ONE compact JSON line (the headline, `roofline`, `cpu_baseline` and
short per-leg figures in `legs`).  The full record of every leg goes to
stderr as one JSON line, and to --detail-out if given.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--size N] [--no-cpu] [--quick]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

METRIC = "GLUP/s + time to 1e-10 residual (FP32+FP64 refine vs FP64); p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# Relaxation of the red-black multigrid smoother in the "relaxed" leg: the
# legs above keep the paper's Gauss-Seidel smoother (omega 1); over-relaxed
# red-black Gauss-Seidel cuts the V(2,2) cycles to 1e-10 on the unit square
# from 7 to 5 (oracle, 513^2 and 1025^2, with and without a source;
# anisotropic grids 13 -> 9).
MG_OMEGA = 1.15
# FP32 V-cycles per FP64 defect correction timed in the mixed-precision leg
# (the fastest is reported as "mixed")
MIXED_INNERS = (1, 2, 3, 4)
BATCH_INNERS = (1, 2, 3, 4)
BATCH_INNER_MARGIN = 0.03
# HBM bytes per launch of the finest-level kernels (8193^2, f = 0) measured
# with rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE, scaled by the counts of a
# 1 GiB stream copy (summaries under profiles/); keyed by kernel class and the
# tiling (V, ty, target waves) they were taken with, for this kernel version.
FINE_TRAFFIC = {("pre", 2, 0, 32768): 1.2863e9, ("two", 2, 0, 3072): 1.2285e9}

# kernel classes timed on the finest level (numbering of lap.h)
FINE_CLASSES = {"sweep": 0, "sweep_prolong": 1, "restrict": 2, "pre": 10, "two": 11}
FINE_LABELS = {
    "sweep": "k_sweep<double,V,0>: one red-black sweep (finest level, f = 0)",
    "sweep_prolong": "k_sweep<double,V,4>: bilinear correction + one red-black sweep",
    "restrict": "k_restrict<double,V>: residual + full weighting",
    "pre": "k_fused<double,2,56> pre pass: input norms, 2 RB sweeps, residual, full weighting",
    "two": "k_fused<double,V,36> post pass: bilinear correction, 2 RB sweeps",
}
ALL_CLASSES = range(15)
KC_RESIDUAL = 8


def lup_per_cycle(levels, nu1=2, nu2=2):
    """Interior nodes updated by the smoother in one V(nu1,nu2) cycle."""
    return sum((nu1 + nu2) * (m - 2) * (n - 2) for (m, n) in levels[:-1])


def sync():
    import torch
    torch.cuda.synchronize()


def say(*a):
    """Progress line on stderr (one per leg)."""
    print("[bench]", time.strftime("%H:%M:%S"), *a, file=sys.stderr, flush=True)


def sig(x, d=4):
    """Round to d significant digits (compact output)."""
    if x is None or not isinstance(x, (int, float)) or x == 0 or not math.isfinite(x):
        return x
    return float(f"{x:.{d}g}")


def timed_solves(g, reset, reps, **kw):
    """`reps` timed solves after the grid's graph exists (two untimed solves
    first: the graph is captured on the second solve with the same options);
    returns (median seconds, info of the last solve)."""
    for _ in range(2):
        reset()
        g.solve(**kw)
    ts, info = [], None
    for _ in range(reps):
        reset()
        sync()
        t0 = time.perf_counter()
        info = g.solve(**kw)
        sync()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)), info


# ------------------------------------------------------------------ headline
def run_headline(args, ctx, torch, lap, dev, keep):
    N = args.size
    out = {}
    p = W.square_problem(N, seed=2)
    psi0 = torch.as_tensor(p.psi0, device=dev)
    g = ctx.grid(psi0, None, p.dx, p.dy, alloc=lap.LAP_ALLOC_FP64)
    levels = g.levels()
    lpc = lup_per_cycle(levels)

    def one_solve():
        g.write(psi0)
        return g.solve("mg", precision="fp64", tol=1e-10, max_iter=60)

    for _ in range(args.warmup):
        one_solve()
    # timed region: kernel timing on (HIP events around every finest-level
    # launch on the library's stream; coarser launches are counted untimed)
    ctx.set_timing(2)
    ctx.reset_stats()
    sync()
    t0 = time.perf_counter()
    infos = [one_solve() for _ in range(args.steps)]
    sync()
    dt = time.perf_counter() - t0
    fine = {k: ctx.kernel_stats(c, fine_only=True) for k, c in FINE_CLASSES.items()}
    every = [ctx.kernel_stats(c) for c in ALL_CLASSES]
    ctx.set_timing(False)
    assert all(i["status"] == 0 for i in infos), infos
    total_lup = sum(i["iterations"] for i in infos) * lpc
    out["value"] = total_lup / dt / 1e9
    out["ms_per_step"] = dt / args.steps * 1e3
    out["cycles"] = infos[-1]["iterations"]
    out["levels"] = len(levels)
    out["rel_res"] = infos[-1]["rel_res_l2"]
    # graph replay (no per-launch events) for the same solve
    out["time_to_tol_graph_s"] = None
    if not args.measure_only:
        tg, _ = timed_solves(g, lambda: g.write(psi0), 3, method="mg", precision="fp64", tol=1e-10, max_iter=60)
        out["time_to_tol_graph_s"] = tg
        # the same solve started by one full multigrid pass (counted as the first iteration)
        tf, fi = timed_solves(g, lambda: g.write(psi0), 3, method="mg", precision="fp64", tol=1e-10, max_iter=60,
                              fmg=True)
        out["fmg"] = {"time_to_tol_s": tf, "iterations": fi["iterations"], "rel_res": fi["rel_res_l2"],
                      "status": fi["status"]}

    # roofline of the dominant kernel: the finest-level kernel class with the
    # most device time (HIP events around each launch on the library's stream)
    dom = max(fine, key=lambda k: fine[k]["device_ms"])
    st = fine[dom]
    ach = st["alg_bytes"] / (st["device_ms"] / 1e3) / 1e9 if st["device_ms"] > 0 else 0.0
    if dom == "pre":
        tiling = (2, 0, 32768)          # the canonical norm tiling (the pass carries the stopping test)
    else:
        tiling = tuple(ctx.get_tiling(FINE_CLASSES[dom], 0, lap.size_class(N, N)))
    out["roofline"] = {
        "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(ach / HBM_PEAK_GBS, 4),
        "traffic": FINE_TRAFFIC.get((dom,) + tiling) if N == 8193 else None,
        "kernel": FINE_LABELS[dom],
        "tiling": {"V": tiling[0], "ty": tiling[1], "target_waves": tiling[2]},
        "alg_bytes_per_launch": st["alg_bytes"] / max(1, st["launches"]),
        "avg_launch_ms": st["device_ms"] / max(1, st["launches"]),
        "launches": st["launches"],
    }
    out["kernels_fine"] = fine
    # whole solve: algorithmic bytes of every launch over the step time
    alg = sum(e["alg_bytes"] for e in every)
    out["solve_hbm"] = {"alg_bytes_per_step": alg / args.steps, "GB/s_over_step_time": alg / dt / 1e9}
    l2, linf = g.residual()
    out["final_res_l2"] = l2
    out["residual_kernel"] = run_residual_leg(ctx, g)
    if keep is not None:
        keep["mg"] = (p, g.read().cpu().numpy())
    g.destroy()
    return out


def run_residual_leg(ctx, g, reps=20):
    """The FP64 residual-norm kernel alone (lap_residual: r = f - L_h u and its
    norms, u and f read once): HIP events around each launch on the
    library's stream."""
    g.residual()
    ctx.set_timing(True)
    ctx.reset_stats()
    for _ in range(reps):
        g.residual()
    st = ctx.kernel_stats(KC_RESIDUAL)
    ctx.set_timing(False)
    ms = st["device_ms"] / max(1, st["launches"])
    gbs = st["alg_bytes"] / max(1, st["launches"]) / (ms / 1e3) / 1e9 if ms > 0 else 0.0
    return {"launches": st["launches"], "avg_launch_ms": ms,
            "alg_bytes_per_launch": st["alg_bytes"] / max(1, st["launches"]),
            "achieved_GB/s": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS}


def run_mixed_leg(N, ctx, torch, lap, dev, keep=None, reps=3, inners=MIXED_INNERS, omega=1.0):
    """Mixed precision vs FP64 multigrid on the N x N grid with the 32-bump
    source: time to a 1e-10 relative residual (median of `reps` graph-replay
    solves per configuration, each grid holding one configuration's graph),
    outer steps / cycles, and the largest difference of the two results.
    Each count of FP32 cycles per defect correction in `inners` is timed
    ("mixed_inner<k>"); "mixed" is the fastest of them (its count in
    "inner_fp32_cycles").  `omega`: the smoother's relaxation."""
    pb = W.square_problem(N, seed=2, bumps=True, bump_seed=3)
    psib = torch.as_tensor(pb.psi0, device=dev)
    fb = torch.as_tensor(pb.f, device=dev)
    res = {}
    u64 = umx = None
    best = None
    for key, prec, inner, alloc in (("fp64", "fp64", 1, lap.LAP_ALLOC_FP64),
                                    *[(f"mixed_inner{k}", "mixed", k, lap.LAP_ALLOC_MIXED) for k in inners]):
        g = ctx.grid(psib, fb, pb.dx, pb.dy, alloc=alloc)
        t, info = timed_solves(g, lambda: g.write(psib), reps, method="mg", precision=prec, inner=inner,
                               omega=omega, tol=1e-10, max_iter=60)
        res[key] = {"time_to_tol_s": t, "iterations": info["iterations"], "rel_res": info["rel_res_l2"],
                    "status": info["status"], "graph_replay": True}
        if prec == "fp64":
            u64 = g.read()
            if omega == 1.0:
                res["residual_kernel_with_f"] = run_residual_leg(ctx, g)
        else:
            res[key]["inner_fp32_cycles"] = inner
            res[key]["speedup_over_fp64"] = res["fp64"]["time_to_tol_s"] / t
            if best is None or t < res[best]["time_to_tol_s"]:
                best = key
                umx = g.read()
        g.destroy()
    res["mixed"] = dict(res[best])
    res["max_abs_mixed_vs_fp64"] = float((umx - u64).abs().max().item())
    res["speedup_mixed_over_fp64"] = res["fp64"]["time_to_tol_s"] / res["mixed"]["time_to_tol_s"]
    if keep is not None:
        keep["bumps"] = (pb, u64.cpu().numpy(), umx.cpu().numpy())
    del u64, umx
    return res


def run_sor_leg(ctx, torch, lap, dev, sizes):
    """Red-black SOR at w = 2/(1+sin(pi h)) to a 1e-10 relative residual
    (stopping test every 50 sweeps)."""
    sor = {}
    for Ns in sizes:
        ps = W.square_problem(Ns, seed=2)
        h = 1.0 / (Ns - 1)
        w = 2.0 / (1.0 + math.sin(math.pi * h))
        gs = ctx.grid(torch.as_tensor(ps.psi0, device=dev), None, ps.dx, ps.dy, alloc=lap.LAP_ALLOC_ADI)
        sync()
        t0 = time.perf_counter()
        info = gs.solve("sor", omega=w, tol=1e-10, max_iter=80000, check_every=50)
        sync()
        t = time.perf_counter() - t0
        lups = info["iterations"] * (Ns - 2) ** 2
        sor[str(Ns)] = {"omega": w, "sweeps": info["iterations"], "seconds": t, "GLUP/s": lups / t / 1e9,
                        "rel_res": info["rel_res_l2"], "status": info["status"]}
        gs.destroy()
    return sor


def run_mg4097_leg(ctx, torch, lap, dev):
    p4 = W.square_problem(4097, seed=2)
    psi = torch.as_tensor(p4.psi0, device=dev)
    g4 = ctx.grid(psi, None, p4.dx, p4.dy, alloc=lap.LAP_ALLOC_FP64)
    t4, i4 = timed_solves(g4, lambda: g4.write(psi), 3, method="mg", tol=1e-10, max_iter=60)
    out = {"time_to_tol_s": t4, "cycles": i4["iterations"],
           "GLUP/s": i4["iterations"] * lup_per_cycle(g4.levels()) / t4 / 1e9}
    g4.destroy()
    return out


def run_relaxed_leg(args, ctx, torch, lap, dev, N):
    """The large-grid multigrid solves with the over-relaxed red-black
    smoother (omega MG_OMEGA) beside the Gauss-Seidel one: FP64 to 1e-10 on
    the N x N headline grid (graph replay, median of 3 per smoother), FP64 vs
    mixed on the 32-bump problem, and the ragged batch (mixed)."""
    p = W.square_problem(N, seed=2)
    psi = torch.as_tensor(p.psi0, device=dev)
    g = ctx.grid(psi, None, p.dx, p.dy, alloc=lap.LAP_ALLOC_FP64)
    out = {"omega": MG_OMEGA}
    for w in (1.0, MG_OMEGA):
        t, info = timed_solves(g, lambda: g.write(psi), 3, method="mg", precision="fp64", omega=w, tol=1e-10,
                               max_iter=60)
        out[f"fp64_w{w:g}"] = {"time_to_tol_s": t, "cycles": info["iterations"], "rel_res": info["rel_res_l2"],
                               "status": info["status"]}
    g.destroy()
    del psi
    out["mixed"] = run_mixed_leg(N, ctx, torch, lap, dev, inners=args.mixed_inner, omega=MG_OMEGA)
    if args.batch:
        probs = W.ragged_batch(count=args.batch_count, lo=33, hi=1025, seed=4)
        grids = [ctx.grid(torch.as_tensor(q.psi0, device=dev), None, q.dx, q.dy, alloc=lap.LAP_ALLOC_MIXED)
                 for q in probs]
        def reset():
            for gg, q in zip(grids, probs):
                gg.write(torch.as_tensor(q.psi0, device=dev))

        for inner in args.batch_inner:
            t, infos = time_batch(ctx, grids, reset, method="mg", precision="mixed", inner=inner, omega=MG_OMEGA,
                                  tol=1e-10, max_iter=200)
            its = [i["iterations"] for i in infos]
            r = {"seconds": t, "inner_fp32_cycles": inner, "steps_min": min(its), "steps_max": max(its),
                 "all_converged": all(i["status"] == 0 for i in infos)}
            b = out.get("batch_mixed")
            if b is None or t < b["seconds"] * (1.0 if b["inner_fp32_cycles"] != 1 else 1.0 - BATCH_INNER_MARGIN):
                out["batch_mixed"] = r
            out[f"batch_mixed_inner{inner}"] = r
        for gg in grids:
            gg.destroy()
    if args.serve:
        out["serving"] = run_serving_leg(args, ctx, torch, lap, dev, omega=MG_OMEGA, rates=[1000, 3000],
                                         baseline_rates=[1000])
    return out


def run_chamber_leg(ctx, torch, lap, dev, reps=5):
    """The paper's 25 x 17 chamber (psi_AB = 100) on the GPU, to max|r| < 1e-6
    (physical units): red-black SOR for w = 1.00 .. 1.95, zebra ADI
    (relaxation after the line solve, w = 1; inside, w = 1.3) and the 3-level
    V(2,2) multigrid cycle (25x17 -> 13x9 -> 7x5, the last solved exactly);
    iterations and microseconds per solve (median of `reps`)."""
    p = W.chamber(psi_ab=100.0)
    psi = torch.as_tensor(p.psi0, device=dev)
    g = ctx.grid(psi, None, p.dx, p.dy)

    def run(method, **kw):
        ts, info = [], None
        for _ in range(reps):
            g.write(psi)
            sync()
            t0 = time.perf_counter()
            info = g.solve(method, tol=1e-6, stop="res_inf", max_iter=20000, **kw)
            sync()
            ts.append(time.perf_counter() - t0)
        assert info["status"] == 0, (method, kw, info)
        return info["iterations"], float(np.median(ts)) * 1e6

    sor = {}
    for k in range(20):
        w = round(1.0 + 0.05 * k, 2)
        sor[f"{w:.2f}"] = run("sor", omega=w)
    best = min(sor, key=lambda w: (sor[w][0], float(w)))
    # the paper's own orderings (one workgroup, the grid in LDS, whole solve in one launch)
    lex = {}
    for k in range(20):
        w = round(1.0 + 0.05 * k, 2)
        lex[f"{w:.2f}"] = run("sor_lex", omega=w)
    lbest = min(lex, key=lambda w: (lex[w][0], float(w)))
    out = {"levels": g.levels(), "sor_iters_us": sor, "sor_best_omega": float(best),
           "adi_after_w1": run("adi", omega=1.0, adi_form="after"),
           "adi_inside_w1.3": run("adi", omega=1.3, adi_form="inside"),
           "mg_v22": run("mg"),
           "paper_order": {"jacobi": run("jacobi"), "sor_lex": lex, "sor_lex_best_omega": float(lbest),
                           "slora_w1": run("slor_lex", omega=1.0, adi_form="after"),
                           "slorb_w1.25": run("slor_lex", omega=1.25, adi_form="inside"),
                           "adi_lex_w1.3": run("adi_lex", omega=1.3, adi_form="inside")}}
    g.destroy()
    return out


def device_request(torch, req, dev):
    """A serving request's inputs generated on the device (U[0,1) boundary
    and 32 Gaussian bumps drawn from the request's seed, the bumps evaluated
    with torch; the same draws as workloads.request_problem)."""
    rng = np.random.default_rng(req.seed)
    m, n = req.m, req.n
    h = 1.0 / (max(m, n) - 1)
    psi0 = W.random_boundary(m, n, rng)
    lx, ly = h * (m - 1), h * (n - 1)
    amp = rng.standard_normal(32)
    cx = rng.random(32) * lx
    cy = rng.random(32) * ly
    sig_ = rng.uniform(0.01, 0.1, 32) * max(lx, ly)
    x = torch.arange(m, device=dev, dtype=torch.float64) * h
    y = torch.arange(n, device=dev, dtype=torch.float64) * h
    f = torch.zeros((n, m), device=dev, dtype=torch.float64)
    for k in range(32):
        gx = torch.exp(-((x - cx[k]) ** 2) / (2.0 * sig_[k] ** 2))
        gy = torch.exp(-((y - cy[k]) ** 2) / (2.0 * sig_[k] ** 2))
        f += amp[k] * torch.outer(gy, gx)
    return torch.as_tensor(psi0, device=dev), f, h, h


def run_copy_probe(torch, lap, dev):
    """Achievable HBM bandwidth: plain copy of 1 GiB (also the calibration
    kernel of the byte counters), timed two ways: ten launches back to back
    (wall clock; each launch starts with the last one's written lines dirty in
    the caches) and single launches after a 1 GiB read of another buffer has
    flushed the caches (HIP events); plus a 1 GiB read-only reduction."""
    src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    other = torch.ones((1 << 30) // 8, dtype=torch.float64, device=dev)
    b2b, single = {}, {}
    for blocks in (1024, 2048, 4096, 8192, 32768):
        lap.op_stream_copy(src, dst, blocks=blocks)
        sync()
        t0 = time.perf_counter()
        for _ in range(10):
            lap.op_stream_copy(src, dst, blocks=blocks)
        sync()
        t = (time.perf_counter() - t0) / 10
        b2b[blocks] = 2 * (1 << 30) / t / 1e9
        ts = []
        for _ in range(5):
            other.sum()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            lap.op_stream_copy(src, dst, blocks=blocks)
            e1.record()
            sync()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        ts.sort()
        single[blocks] = [2 * (1 << 30) / ts[len(ts) // 2] / 1e9, 2 * (1 << 30) / ts[0] / 1e9]
    rd = []
    for _ in range(5):
        src.view(torch.float64).sum()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        other.sum()
        e1.record()
        sync()
        rd.append((1 << 30) / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del src, dst, other
    return {"bytes_per_launch": 2 * (1 << 30), "GB/s_by_blocks": b2b, "best_GB/s": max(b2b.values()),
            "single_after_flush_GB/s_median_best": single, "read_only_GB/s_best": max(rd)}


def time_batch(ctx, grids, reset, **kw):
    """Warm-up solve (plans, graphs), then one timed solve of the batch."""
    reset()
    ctx.solve_batch(grids, **kw)
    reset()
    sync()
    t0 = time.perf_counter()
    infos = ctx.solve_batch(grids, **kw)
    sync()
    return time.perf_counter() - t0, infos


def run_batch_leg(args, ctx, torch, lap, dev):
    """Ragged batch: 512 grids, m, n log-uniform in [33, 1025] (snapped to
    c*2^k+1), aspect <= 3, beta in [0.5, 2], U[0,1) boundary, f = 0.  The
    mixed solve is timed for each count of FP32 cycles per defect correction
    in args.batch_inner ("mg_mixed_inner<k>"); "mg_mixed" is the fastest, one
    cycle per correction unless another count is faster by BATCH_INNER_MARGIN
    (batch times vary by ~2% between runs)."""
    count = args.batch_count
    probs = W.ragged_batch(count=count, lo=33, hi=1025, seed=4)
    grids = [ctx.grid(torch.as_tensor(p.psi0, device=dev), None, p.dx, p.dy,
                      alloc=lap.LAP_ALLOC_MIXED | lap.LAP_ALLOC_ADI | lap.LAP_ALLOC_FP64) for p in probs]
    nodes = sum((p.m - 2) * (p.n - 2) for p in probs)
    lpc = [lup_per_cycle(g.levels()) for g in grids]
    out = {"grids": count, "interior_nodes": nodes}

    def reset():
        for g, p in zip(grids, probs):
            g.write(torch.as_tensor(p.psi0, device=dev))

    # batched mixed-precision multigrid, one to several FP32 cycles per correction
    best = None
    for inner in args.batch_inner:
        mkw = dict(method="mg", precision="mixed", inner=inner, tol=1e-10, max_iter=200)
        t, infos = time_batch(ctx, grids, reset, **mkw)
        its = [i["iterations"] for i in infos]
        r = {"seconds": t, "inner_fp32_cycles": inner, "steps_min": min(its), "steps_max": max(its),
             "all_converged": all(i["status"] == 0 for i in infos), "solves_per_s": count / t}
        if inner == 1:
            # one cycle per step: the lattice updates of every cycle are known
            r["GLUP/s"] = sum(k * l for k, l in zip(its, lpc)) / t / 1e9
            r["cycles_min"], r["cycles_max"] = min(its), max(its)
        out[f"mg_mixed_inner{inner}"] = r
        if best is None or t < best[0] * (1.0 if best[1] != 1 else 1.0 - BATCH_INNER_MARGIN):
            best = (t, inner, its, mkw)
    t, best_inner, its, mkw = best
    out["mg_mixed"] = dict(out[f"mg_mixed_inner{best_inner}"])
    # the same batch with zebra line smoothing (V(1,1): robust for beta != 1)
    zkw = dict(method="mg", precision="mixed", smoother="zebra", nu1=1, nu2=1, tol=1e-10, max_iter=200)
    tz, zinf = time_batch(ctx, grids, reset, **zkw)
    zits = [i["iterations"] for i in zinf]
    out["mg_mixed_zebra"] = {"seconds": tz, "GLUP/s": sum(k * l for k, l in zip(zits, lpc)) / tz / 1e9,
                             "cycles_min": min(zits), "cycles_max": max(zits),
                             "all_converged": all(i["status"] == 0 for i in zinf), "solves_per_s": count / tz}
    # error against FP64: sampled grids solved alone with FP64 multigrid
    sample = list(range(0, count, max(1, count // 8)))
    reset()
    ctx.solve_batch(grids, **mkw)
    mixed_u = {k: grids[k].read() for k in sample}
    errs = []
    for k in sample:
        g = grids[k]
        g.write(torch.as_tensor(probs[k].psi0, device=dev))
        g.solve("mg", precision="fp64", tol=1e-10, max_iter=200)
        errs.append(float((g.read() - mixed_u[k]).abs().max().item()))
    out["mg_mixed"]["max_abs_vs_fp64_sampled"] = max(errs)
    out["mg_mixed"]["sampled_grids"] = len(sample)
    # the same grids one at a time
    reset()
    sync()
    t0 = time.perf_counter()
    seq = [g.solve(**mkw) for g in grids]
    sync()
    ts = time.perf_counter() - t0
    out["mg_mixed_one_at_a_time"] = {"seconds": ts, "speedup_of_batch": ts / t,
                                     "same_iterations": [i["iterations"] for i in seq] == its}
    # batched zebra ADI: fixed number of iterations (every interior node is
    # updated twice per iteration: once by its row, once by its column)
    nit = args.adi_iters
    reset()
    # warm-up builds the merged-launch plan of the timed step (same check block)
    ctx.solve_batch(grids, method="adi", omega=1.0, tol=0.0, max_iter=nit, check_every=nit)
    reset()
    sync()
    t0 = time.perf_counter()
    ctx.solve_batch(grids, method="adi", omega=1.0, tol=0.0, max_iter=nit, check_every=nit)
    sync()
    ta = time.perf_counter() - t0
    # algorithmic bytes: each of the four line launches of an iteration (rows,
    # columns; two parities each) reads its lines' old values and the other
    # parity's lines once and writes its lines (f = 0): 12 B per grid node and
    # launch, 48 B per node and iteration
    out["adi"] = {"iterations": nit, "seconds": ta, "line_updates_G/s": 2 * nit * nodes / ta / 1e9,
                  "alg_GB/s": 48.0 * nit * nodes / ta / 1e9}
    for g in grids:
        g.destroy()
    return out


def run_serving_leg(args, ctx, torch, lap, dev, omega=1.0, rates=None, baseline_rates=None):
    """Poisson arrivals; m, n log-uniform in [17, 4097] snapped, beta = 1,
    32-bump source, tol 1e-8 or 1e-10; continuous batching (mixed) vs
    one-at-a-time FP64 solves.  Every rate serves warm-up + count requests
    (the request sizes, seeds and tolerances are the same at every rate, only
    the arrival times scale); latency percentiles, solves/s and GLUP/s cover
    the `count` requests after the warm-up, over the span from the first of
    them arriving to the last finishing.  `omega`: the multigrid smoother's
    relaxation (served and one-at-a-time solves alike)."""
    rates = args.rates if rates is None else rates
    baseline_rates = args.baseline_rates if baseline_rates is None else baseline_rates
    from paper_2208_02427_amd.serving import Job, Server, DeviceBackend, serve_sequential
    warm, count = args.serve_warmup, args.serve_count
    total = warm + count
    base = W.poisson_requests(1.0, total, seed=5, lo=17, hi=4097)
    payload = {r.rid: device_request(torch, r, dev) for r in base}
    sync()
    lpc = {}

    def lpc_of(m, n):          # smoother updates per cycle, from the hierarchy of an admitted grid
        return lpc[(m, n)]

    # requests whose result is compared with an FP64 solve of the same input
    sample = {r.rid for r in base[warm:] if r.m * r.n <= 1025 * 1025}
    sample = set(sorted(sample)[:: max(1, len(sample) // 6)])

    class Backend(DeviceBackend):
        def admit(self, job):
            g = super().admit(job)
            lpc[(job.m, job.n)] = lup_per_cycle(g.levels())
            g._rid = job.rid
            return g

        def retire(self, g):
            job_rid = getattr(g, "_rid", None)
            out = g.read() if job_rid in sample else None
            g.destroy()
            return out

    def stats_of(jobs):
        meas = [j for j in jobs if j.rid >= warm and j.finished is not None]
        lat = np.array([j.finished - j.arrival for j in meas])
        span = max(j.finished for j in meas) - min(j.arrival for j in meas)
        lups = sum(j.iterations * lpc_of(j.m, j.n) for j in meas)
        return {"requests": len(meas), "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "solves_per_s": len(meas) / span,
                "GLUP/s": lups / span / 1e9,
                "failed": sum(1 for j in jobs if j.status not in (None, 0))}

    res = {"warmup_requests": warm, "measured_requests": count}
    errs = []
    for rate in rates:
        say("serving", rate, "requests/s", "omega", omega)
        jobs = [Job(r.rid, r.arrival / rate, r.m, r.n, r.tol, payload=payload[r.rid]) for r in base]
        sync()
        server = Server(Backend(ctx, precision="mixed", omega=omega), max_active=256, burst=args.burst,
                        solo_max_nodes=args.solo_max_nodes)
        stats = server.run(jobs)
        sm = stats_of(jobs)
        sm["max_active"] = stats.max_active
        sm["solo"] = stats.solo
        res[str(int(rate))] = {"batched_mixed": sm}
        if not errs:
            # error against FP64 of sampled served results (first rate only)
            for j in jobs:
                if j.rid in sample and j.result is not None:
                    psi0, f, dx, dy = j.payload
                    g = ctx.grid(psi0, f, dx, dy, alloc=lap.LAP_ALLOC_FP64)
                    g.solve("mg", precision="fp64", omega=omega, tol=j.tol, max_iter=100)
                    errs.append(float((g.read() - j.result).abs().max().item()))
                    g.destroy()
            res["max_abs_served_vs_fp64_sampled"] = max(errs) if errs else None
            res["sampled_requests"] = len(errs)
        for j in jobs:
            j.result = None
        if rate in baseline_rates:
            def solve_one(job):
                psi0, f, dx, dy = job.payload
                g = ctx.grid(psi0, f, dx, dy, alloc=lap.LAP_ALLOC_FP64)
                info = g.solve("mg", precision="fp64", omega=omega, tol=job.tol, max_iter=100)
                lpc[(job.m, job.n)] = lup_per_cycle(g.levels())
                g.destroy()
                return info
            jobs2 = [Job(r.rid, r.arrival / rate, r.m, r.n, r.tol, payload=payload[r.rid]) for r in base]
            say("serving one at a time (FP64)", rate, "requests/s")
            sync()
            serve_sequential(solve_one, jobs2)
            res[str(int(rate))]["one_at_a_time_fp64"] = stats_of(jobs2)
        torch.cuda.empty_cache()
    del payload
    return res


def cpu_baseline_leg(headline, keep, N):
    """The oracle as it stands, on this host: one FP64 V(2,2) cycle of the
    N x N headline solve (numpy; its elementwise operations run on one core),
    extrapolated to the solve's cycle count.  The oracle is loaded here, so
    this leg also checks the large GPU results against the oracle's exact
    spectral solution of the same discrete problem (DST-I in x and y)."""
    from oracle import multigrid as omg, direct
    p = W.square_problem(N, seed=2)
    lv = omg.hierarchy(N, N, p.dx, p.dy)
    u = p.psi0.copy()
    t0 = time.perf_counter()
    omg.vcycle(lv, 0, u, None)
    t = time.perf_counter() - t0
    lups = lup_per_cycle([(a, b) for a, b, _, _ in lv])
    cycles = headline["cycles"]
    base = {"value": lups / t / 1e9, "unit": "GLUP/s", "cores": 1, "kind": "oracle",
            "sample": f"1 of {cycles} FP64 V(2,2) cycles of the {N}^2 solve (numpy, {t:.1f} s, 1 core of "
                      f"{len(os.sched_getaffinity(0))}); solve x{cycles} = {cycles * t:.0f} s extrapolated"}
    errors = {}
    t0 = time.perf_counter()
    if "mg" in keep:
        pp, ug = keep["mg"]
        ex = direct.dst_solve(pp.m, pp.n, pp.dx, pp.dy, pp.psi0, pp.f)
        errors["fp64_mg_vs_exact"] = float(np.max(np.abs(ug - ex)))
        del ex
    if "bumps" in keep:
        pb, u64, umx = keep["bumps"]
        ex = direct.dst_solve(pb.m, pb.n, pb.dx, pb.dy, pb.psi0, pb.f)
        errors["bumps_fp64_vs_exact"] = float(np.max(np.abs(u64 - ex)))
        errors["bumps_mixed_vs_exact"] = float(np.max(np.abs(umx - ex)))
        errors["bumps_exact_max_abs"] = float(np.max(np.abs(ex)))
        del ex
    errors["dst_seconds"] = time.perf_counter() - t0
    return base, errors


def serve_rows(s):
    """The serving record as one row per rate."""
    sv = {}
    for rate, v in s.items():
        if not isinstance(v, dict) or "batched_mixed" not in v:
            continue
        bm = v["batched_mixed"]
        row = [sig(bm["p50_ms"], 3), sig(bm["p99_ms"], 3), sig(bm["solves_per_s"], 4), sig(bm["GLUP/s"], 3)]
        if "one_at_a_time_fp64" in v:
            o = v["one_at_a_time_fp64"]
            row += [sig(o["p50_ms"], 3), sig(o["p99_ms"], 3), sig(o["solves_per_s"], 4)]
        sv[rate] = row
    sv["cols"] = "p50,p99 ms,solves/s,GLUP/s[,FP64 1-by-1 p50,p99,solves/s]"
    return sv


def compact(line_full, d):
    """The per-leg figures that go on the stdout line."""
    legs = {}
    if d.get("time_to_tol_graph_s"):
        legs["mg_graph_ms"] = sig(d["time_to_tol_graph_s"] * 1e3)
    if "fmg" in d:
        legs["fmg_ms_it"] = [sig(d["fmg"]["time_to_tol_s"] * 1e3), d["fmg"]["iterations"]]
    legs["residual_kernel_frac"] = sig(d["residual_kernel"]["frac_of_peak"], 3)
    legs["solve_alg_GB/s"] = sig(d["solve_hbm"]["GB/s_over_step_time"])
    for key in ("mixed", "mixed_4097"):
        if key in d:
            x = d[key]
            legs[key] = {"fp64_ms": sig(x["fp64"]["time_to_tol_s"] * 1e3),
                         "mixed_ms": sig(x["mixed"]["time_to_tol_s"] * 1e3),
                         "speedup": sig(x["speedup_mixed_over_fp64"], 3),
                         "steps": [x["fp64"]["iterations"], x["mixed"]["iterations"]],
                         "inner": x["mixed"].get("inner_fp32_cycles", 1),
                         "err": sig(x["max_abs_mixed_vs_fp64"], 2)}
            legs[key]["ms_by_inner"] = {k[len("mixed_inner"):]: sig(v["time_to_tol_s"] * 1e3)
                                        for k, v in x.items() if k.startswith("mixed_inner")}
    if "sor" in d:
        legs["sor"] = {k: [v["sweeps"], sig(v["seconds"], 3), sig(v["GLUP/s"])] for k, v in d["sor"].items()}
        legs["sor"]["cols"] = "sweeps,s,GLUP/s"
    if "mg_4097" in d:
        legs["mg_4097_ms"] = sig(d["mg_4097"]["time_to_tol_s"] * 1e3)
    if "relaxed" in d:
        r = d["relaxed"]
        w1, w2 = r["fp64_w1"], r[f"fp64_w{r['omega']:g}"]
        m = r["mixed"]
        legs["relaxed_w" + f"{r['omega']:g}"] = {
            "mg_ms": [sig(w1["time_to_tol_s"] * 1e3), sig(w2["time_to_tol_s"] * 1e3)],
            "cycles": [w1["cycles"], w2["cycles"]],
            "mixed": {"fp64_ms": sig(m["fp64"]["time_to_tol_s"] * 1e3), "mixed_ms": sig(m["mixed"]["time_to_tol_s"] * 1e3),
                      "speedup": sig(m["speedup_mixed_over_fp64"], 3), "inner": m["mixed"]["inner_fp32_cycles"],
                      "steps": [m["fp64"]["iterations"], m["mixed"]["iterations"]],
                      "err": sig(m["max_abs_mixed_vs_fp64"], 2)}}
        if "batch_mixed" in r:
            b = r["batch_mixed"]
            legs["relaxed_w" + f"{r['omega']:g}"]["batch512"] = {
                "ms": sig(b["seconds"] * 1e3), "inner": b["inner_fp32_cycles"], "steps": [b["steps_min"], b["steps_max"]],
                "ms_by_inner": {k[len("batch_mixed_inner"):]: sig(v["seconds"] * 1e3)
                                for k, v in r.items() if k.startswith("batch_mixed_inner")}}
        if "serving" in r:
            legs["relaxed_w" + f"{r['omega']:g}"]["serve"] = serve_rows(r["serving"])
    if "chamber" in d:
        c = d["chamber"]
        wb = f"{c['sor_best_omega']:.2f}"
        legs["chamber"] = {"cols": "iterations,us", "sor1": [c["sor_iters_us"]["1.00"][0], sig(c["sor_iters_us"]["1.00"][1], 3)],
                           "sor" + wb: [c["sor_iters_us"][wb][0], sig(c["sor_iters_us"][wb][1], 3)],
                           "adi1": [c["adi_after_w1"][0], sig(c["adi_after_w1"][1], 3)],
                           "mg": [c["mg_v22"][0], sig(c["mg_v22"][1], 3)]}
        po = c["paper_order"]
        lb = f"{po['sor_lex_best_omega']:.2f}"
        legs["chamber_lex"] = {"jacobi": [po["jacobi"][0], sig(po["jacobi"][1], 3)],
                               "gs": [po["sor_lex"]["1.00"][0], sig(po["sor_lex"]["1.00"][1], 3)],
                               "sor" + lb: [po["sor_lex"][lb][0], sig(po["sor_lex"][lb][1], 3)],
                               "slorb1.25": [po["slorb_w1.25"][0], sig(po["slorb_w1.25"][1], 3)],
                               "adi1.3": [po["adi_lex_w1.3"][0], sig(po["adi_lex_w1.3"][1], 3)]}
    if "ragged_batch" in d:
        b = d["ragged_batch"]
        b1 = b.get("mg_mixed_inner1", {})
        legs["batch512"] = {"mg_ms": sig(b["mg_mixed"]["seconds"] * 1e3),
                            "inner": b["mg_mixed"]["inner_fp32_cycles"],
                            "steps": [b["mg_mixed"]["steps_min"], b["mg_mixed"]["steps_max"]],
                            "ms_by_inner": {k[len("mg_mixed_inner"):]: sig(v["seconds"] * 1e3)
                                            for k, v in b.items() if k.startswith("mg_mixed_inner")},
                            "cycles_inner1": [b1.get("cycles_min"), b1.get("cycles_max")],
                            "GLUP/s_inner1": sig(b1.get("GLUP/s")),
                            "vs_one_at_a_time": sig(b["mg_mixed_one_at_a_time"]["speedup_of_batch"], 3),
                            "err": sig(b["mg_mixed"]["max_abs_vs_fp64_sampled"], 2),
                            "zebra_ms": sig(b["mg_mixed_zebra"]["seconds"] * 1e3),
                            "zebra_cycles": [b["mg_mixed_zebra"]["cycles_min"], b["mg_mixed_zebra"]["cycles_max"]],
                            "adi20_ms": sig(b["adi"]["seconds"] * 1e3), "adi_GB/s": sig(b["adi"]["alg_GB/s"])}
    if "serving" in d:
        sv = serve_rows(d["serving"])
        sv["err"] = sig(d["serving"].get("max_abs_served_vs_fp64_sampled"), 2)
        legs["serve"] = sv
    if "errors_vs_exact" in d:
        short = {"fp64_mg_vs_exact": "mg", "bumps_fp64_vs_exact": "bumps_fp64", "bumps_mixed_vs_exact": "bumps_mixed",
                 "bumps_exact_max_abs": "bumps_max|u|"}
        legs["err_vs_exact"] = {short[k]: sig(v, 2) for k, v in d["errors_vs_exact"].items() if k in short}
    line_full["legs"] = legs
    return line_full


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--size", type=int, default=8193)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="headline only")
    ap.add_argument("--no-tune", action="store_true", help="keep the shipped tiling table, no autotuning")
    ap.add_argument("--tuning-out", default=None,
                    help="write the autotune reports as a tiling table (the format of the shipped "
                         "paper_2208_02427_amd/tuning_gfx950.json)")
    ap.add_argument("--detail-out", default=None, help="also write the full record of every leg here (JSON)")
    ap.add_argument("--copy-probe", action="store_true", help="also time a plain 1 GiB device copy")
    ap.add_argument("--measure-only", action="store_true",
                    help="only measured-mode solves (for profiler runs: no graph replay leg)")
    ap.add_argument("--no-batch", dest="batch", action="store_false", help="skip the ragged-batch leg")
    ap.add_argument("--mixed-inner", type=int, nargs="+", default=list(MIXED_INNERS),
                    help="FP32 cycles per correction timed in the mixed leg (the fastest is reported)")
    ap.add_argument("--mixed-only", action="store_true",
                    help="run only the mixed-vs-FP64 leg and print its JSON (profiling aid; not the benchmark line)")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the ragged-batch leg and print its JSON (profiling aid; not the benchmark line)")
    ap.add_argument("--no-serve", dest="serve", action="store_false", help="skip the serving leg")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--batch-inner", type=int, nargs="+", default=list(BATCH_INNERS),
                    help="FP32 cycles per defect correction timed in the ragged-batch legs")
    ap.add_argument("--adi-iters", type=int, default=20)
    ap.add_argument("--serve-count", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--burst", type=int, default=4, help="outer steps per serving tick when no request waits")
    ap.add_argument("--solo-max-nodes", type=int, default=4097 * 4097,
                    help="largest request (m*n) solved alone when it finds the device idle (0: never)")
    ap.add_argument("--rates", type=float, nargs="*", default=[100, 300, 1000, 3000, 10000])
    ap.add_argument("--baseline-rates", type=float, nargs="*", default=[100, 1000])
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library runs each grid on a single MI355X "
              "(sharding across GPUs is not implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2208_02427_amd as lap
    dev = "cuda:0"
    if args.mixed_only or args.batch_only:
        ctx = lap.Context(arena_bytes=16 << 30, device=dev)
        res = {"mixed": run_mixed_leg(args.size, ctx, torch, lap, dev, inners=args.mixed_inner)} if args.mixed_only else \
              {"ragged_batch": run_batch_leg(args, ctx, torch, lap, dev)}
        if args.copy_probe:
            res["copy_probe"] = run_copy_probe(torch, lap, dev)
        print(json.dumps(res), flush=True)
        return

    N = args.size
    ctx = lap.Context(arena_bytes=(16 << 30) if N > 4097 else (4 << 30), device=dev)
    d = {}
    # autotune the tilings of every level size the hierarchy visits down to
    # the small-level subtree (setup, untimed); without it the Context keeps
    # the shipped MI355X table
    if not args.no_tune:
        say("autotune")
        sizes = [N]
        while sizes[-1] > 65 and (sizes[-1] - 1) % 2 == 0:
            sizes.append((sizes[-1] - 1) // 2 + 1)
        t0 = time.perf_counter()
        tune = [ctx.autotune(tn, tn, reps=3) for tn in sizes]
        d["autotune"] = {"sizes": sizes, "seconds": time.perf_counter() - t0}
        if args.tuning_out:
            with open(args.tuning_out, "w") as fh:
                json.dump({"device": "gfx950 (MI355X, 256 CUs)",
                           "source": "lap_autotune on one MI355X, reps=3, sizes " + "/".join(map(str, sizes))
                                     + " (python bench.py --tuning-out ...)",
                           "reports": tune}, fh, indent=1)
    if args.copy_probe:
        d["copy_probe"] = run_copy_probe(torch, lap, dev)
    keep = {} if not args.no_cpu else None
    say("headline", N)
    d.update(run_headline(args, ctx, torch, lap, dev, keep))
    if not args.quick:
        say("mixed", N)
        d["mixed"] = run_mixed_leg(N, ctx, torch, lap, dev, keep, inners=args.mixed_inner)
        if N > 4097:
            say("mixed", 4097)
            d["mixed_4097"] = run_mixed_leg(4097, ctx, torch, lap, dev, inners=args.mixed_inner)
        say("sor")
        d["sor"] = run_sor_leg(ctx, torch, lap, dev, sorted({4097, N}))
        d["mg_4097"] = run_mg4097_leg(ctx, torch, lap, dev)
        say("relaxed smoother")
        d["relaxed"] = run_relaxed_leg(args, ctx, torch, lap, dev, N)
        say("chamber")
        d["chamber"] = run_chamber_leg(ctx, torch, lap, dev)
        if args.batch:
            say("ragged batch")
            d["ragged_batch"] = run_batch_leg(args, ctx, torch, lap, dev)
        if args.serve:
            d["serving"] = run_serving_leg(args, ctx, torch, lap, dev)
    ctx.close()
    line = {
        "metric": METRIC,
        "value": round(d["value"], 3),
        "unit": "GLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(d["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{N}^2 unit square, U[0,1) boundary (seed 2), f=0, FP64 V(2,2) MG to rel.res 1e-10",
            "levels": d["levels"], "cycles": d["cycles"],
        },
        "roofline": {k: d["roofline"][k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic", "kernel")},
    }
    if not args.no_cpu:
        say("cpu baseline (oracle) and errors against the exact solution")
        base, errors = cpu_baseline_leg(d, keep, N)
        line["cpu_baseline"] = base
        d["cpu_baseline"] = base
        d["errors_vs_exact"] = errors
    d["roofline_full"] = d["roofline"]
    print(json.dumps(d, default=float), file=sys.stderr, flush=True)
    if args.detail_out:
        with open(args.detail_out, "w") as fh:
            json.dump(d, fh, indent=1, default=float)
    print(json.dumps(compact(line, d)), flush=True)


if __name__ == "__main__":
    main()
