"""Benchmark: multigrid time-to-solution and smoother throughput on one MI355X.

Workload (one "step"): reset an 8193 x 8193 unit-square grid (h = 1/8192,
beta = 1, Dirichlet values U[0,1) from seed 2, zero interior, f = 0) and solve
it to ||r||_2/||r_0||_2 < 1e-10 with FP64 V(2,2) multigrid (red-black
Gauss-Seidel smoother, full weighting, bilinear interpolation, 12 levels down
to 5 x 5 solved directly).  `value` is the smoother throughput of the step in
GLUP/s: interior nodes updated by all smoothing sweeps on all levels, per
second of whole-step wall time (inputs resident in HBM).

Also measured in the same run (reported beside the headline):
  * mixed precision on the same grid with a 32-bump source: FP32 V-cycles
    inside FP64 defect correction vs FP64 multigrid, time to 1e-10 and speedup;
  * red-black SOR with w = 2/(1+sin(pi h)): sweeps/s and GLUP/s, and time to
    1e-10 on 4097 x 4097;
  * the roofline of the dominant kernel (the finest-level kernel class with
    the most device time: the fused pre- or post-smoothing pass) from HIP
    events around each of its launches;
  * the CPU oracle on the host cores (one V-cycle of the 4097 x 4097 solve).

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
# HBM bytes per launch of the finest-level kernels (8193^2, f = 0) measured
# with rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE, scaled by the counts of a
# 1 GiB stream copy (summaries under profiles/); keyed by kernel class and the
# tiling (V, ty, target waves) they were taken with, for this kernel version.
FINE_TRAFFIC = {("pre", 2, 0, 32768): 1.2917e9, ("two", 2, 64, 0): 1.2517e9, ("two", 4, 0, 6144): 1.3161e9}

# kernel classes timed on the finest level (numbering of lap.h)
FINE_CLASSES = {"sweep": 0, "sweep_prolong": 1, "restrict": 2, "pre": 10, "two": 11}
FINE_LABELS = {
    "sweep": "k_sweep<double,V,0>: one red-black sweep (finest level, f = 0)",
    "sweep_prolong": "k_sweep<double,V,4>: bilinear correction + one red-black sweep",
    "restrict": "k_restrict<double,V>: residual + full weighting",
    "pre": "k_fused<double,2,56>: residual norms of the iterate + two red-black sweeps + residual + full "
           "weighting (finest level, f = 0, canonical norm tiling)",
    "two": "k_fused<double,V,36>: bilinear correction + two red-black sweeps (finest level, f = 0)",
}
ALL_CLASSES = range(13)


def lup_per_cycle(levels, nu1=2, nu2=2):
    """Interior nodes updated by the smoother in one V(nu1,nu2) cycle."""
    return sum((nu1 + nu2) * (m - 2) * (n - 2) for (m, n) in levels[:-1])


def sync():
    import torch
    torch.cuda.synchronize()


def run_gpu(args):
    import torch
    import paper_2208_02427_amd as lap

    N = args.size
    dev = "cuda:0"
    arena = 12 << 30 if N > 4097 else 4 << 30
    ctx = lap.Context(arena_bytes=arena, device=dev)
    out = {}
    # autotune the tilings of every level size the hierarchy visits down to
    # the small-level subtree (setup, untimed); without it the Context keeps
    # the shipped MI355X table
    tune = []
    if not args.no_tune:
        sizes = [N]
        while sizes[-1] > 65 and (sizes[-1] - 1) % 2 == 0:
            sizes.append((sizes[-1] - 1) // 2 + 1)
        for tn in sizes:
            tune.append(ctx.autotune(tn, tn, reps=3))
        if args.tuning_out:
            with open(args.tuning_out, "w") as fh:
                json.dump({"device": "gfx950 (MI355X, 256 CUs)",
                           "source": "lap_autotune on one MI355X, reps=3, sizes " + "/".join(map(str, sizes))
                                     + " (python bench.py --tuning-out ...)",
                           "reports": tune}, fh, indent=1)
    out["autotune"] = tune

    if args.copy_probe:
        out["copy_probe"] = run_copy_probe(torch, lap, dev)

    # ---------------------------------------------------------------- headline
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
    cycles = infos[-1]["iterations"]
    assert all(i["status"] == 0 for i in infos), infos
    total_lup = sum(i["iterations"] for i in infos) * lpc
    out["value"] = total_lup / dt / 1e9
    out["ms_per_step"] = dt / args.steps * 1e3
    out["cycles"] = cycles
    out["rel_res"] = infos[-1]["rel_res_l2"]
    # graph replay (no per-launch events) for the same solve
    out["time_to_tol_graph_s"] = None
    if not args.measure_only:
        sync()
        t0 = time.perf_counter()
        one_solve()
        sync()
        out["time_to_tol_graph_s"] = time.perf_counter() - t0
    out["time_to_tol_s"] = out["ms_per_step"] / 1e3

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
        "tiling": {"V": tiling[0], "ty": tiling[1], "target_waves": tiling[2]},
        "kernel": FINE_LABELS[dom],
        "alg_bytes_per_launch": st["alg_bytes"] / max(1, st["launches"]),
        "avg_launch_ms": st["device_ms"] / max(1, st["launches"]),
        "launches": st["launches"],
    }
    out["kernels_fine"] = fine
    # whole solve: algorithmic bytes of every launch over the step time
    alg = sum(e["alg_bytes"] for e in every)
    out["solve_hbm"] = {"alg_bytes_per_step": alg / args.steps, "GB/s_over_step_time": alg / dt / 1e9}
    # correctness of the timed result: oracle-side residual at sampled rows is
    # checked in the GPU tests; here record the library's own FP64 residual
    l2, linf = g.residual()
    out["final_res_l2"] = l2
    out["residual_kernel"] = run_residual_leg(ctx, g, lap)
    g.destroy()

    if args.quick:
        args.batch = args.serve = False
    if not args.quick:
        out["mixed"] = run_mixed_leg(N, ctx, torch, lap, dev)

        # ---------------------------------------------- red-black SOR
        sor = {}
        for Ns, full in ((4097, True), (N, False)):
            ps = W.square_problem(Ns, seed=2)
            h = 1.0 / (Ns - 1)
            w = 2.0 / (1.0 + math.sin(math.pi * h))
            gs = ctx.grid(torch.as_tensor(ps.psi0, device=dev), None, ps.dx, ps.dy, alloc=lap.LAP_ALLOC_ADI)
            nsw = 40000 if full else 2000
            sync()
            t0 = time.perf_counter()
            info = gs.solve("sor", omega=w, tol=1e-10 if full else 0.0, max_iter=nsw, check_every=50)
            sync()
            t = time.perf_counter() - t0
            lups = info["iterations"] * (Ns - 2) ** 2
            sor[str(Ns)] = {"omega": w, "sweeps": info["iterations"], "seconds": t, "GLUP/s": lups / t / 1e9,
                            "to_tol": full, "rel_res": info["rel_res_l2"], "status": info["status"]}
            gs.destroy()
        out["sor"] = sor
        # ---------------------------------------------- MG at 4097
        p4 = W.square_problem(4097, seed=2)
        g4 = ctx.grid(torch.as_tensor(p4.psi0, device=dev), None, p4.dx, p4.dy, alloc=lap.LAP_ALLOC_FP64)
        g4.solve("mg", tol=1e-10, max_iter=60)
        g4.write(torch.as_tensor(p4.psi0, device=dev))
        sync()
        t0 = time.perf_counter()
        i4 = g4.solve("mg", tol=1e-10, max_iter=60)
        sync()
        t4 = time.perf_counter() - t0
        out["mg_4097"] = {"time_to_tol_s": t4, "cycles": i4["iterations"],
                          "GLUP/s": i4["iterations"] * lup_per_cycle(g4.levels()) / t4 / 1e9}
        g4.destroy()
    if args.batch:
        out["ragged_batch"] = run_batch_leg(args, ctx, torch, lap, dev)
    if args.serve:
        out["serving"] = run_serving_leg(args, ctx, torch, lap, dev)
    ctx.close()
    return out, levels


def run_residual_leg(ctx, g, lap, reps=20):
    """The FP64 residual-norm kernel alone (lap_residual: r = f - L_h u and its
    norms, u and f read once): HIP events around each launch on the
    library's stream."""
    KC_RESIDUAL = 8
    g.residual()
    ctx.set_timing(True)
    ctx.reset_stats()
    for _ in range(reps):
        g.residual()
    st = ctx.kernel_stats(KC_RESIDUAL)
    ctx.set_timing(False)
    ms = st["device_ms"] / max(1, st["launches"])
    gbs = st["alg_bytes"] / max(1, st["launches"]) / (ms / 1e3) / 1e9 if ms > 0 else 0.0
    return {"launches": st["launches"], "avg_launch_ms": ms, "alg_bytes_per_launch": st["alg_bytes"] / max(1, st["launches"]),
            "achieved_GB/s": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS}


def run_mixed_leg(N, ctx, torch, lap, dev):
    """Mixed precision vs FP64 multigrid on the N x N grid with the 32-bump
    source: time to a 1e-10 relative residual (the second of two solves of
    each), cycles / outer steps, and the largest difference of the results."""
    sync = torch.cuda.synchronize
    pb = W.square_problem(N, seed=2, bumps=True, bump_seed=3)
    psib = torch.as_tensor(pb.psi0, device=dev)
    fb = torch.as_tensor(pb.f, device=dev)
    gb = ctx.grid(psib, fb, pb.dx, pb.dy, alloc=lap.LAP_ALLOC_FP64 | lap.LAP_ALLOC_MIXED)
    res = {}
    for prec in ("fp64", "mixed", "fp64", "mixed"):
        gb.write(psib)
        sync()
        t0 = time.perf_counter()
        info = gb.solve("mg", precision=prec, tol=1e-10, max_iter=60)
        sync()
        t = time.perf_counter() - t0
        res[prec] = {"time_to_tol_s": t, "iterations": info["iterations"], "rel_res": info["rel_res_l2"],
                     "status": info["status"]}
    gb.write(psib)
    gb.solve("mg", precision="fp64", tol=1e-10, max_iter=60)
    u64 = gb.read()
    gb.write(psib)
    gb.solve("mg", precision="mixed", tol=1e-10, max_iter=60)
    um = gb.read()
    res["max_abs_mixed_vs_fp64"] = float((um - u64).abs().max().item())
    res["speedup_mixed_over_fp64"] = res["fp64"]["time_to_tol_s"] / res["mixed"]["time_to_tol_s"]
    res["residual_kernel_with_f"] = run_residual_leg(ctx, gb, lap)
    gb.destroy()
    return res


def device_request(torch, req, dev):
    """A serving request's inputs generated on the device (same recipe as
    workloads.request_problem: U[0,1) boundary and 32 Gaussian bumps drawn
    from the request's seed; the bumps are evaluated with torch)."""
    rng = np.random.default_rng(req.seed)
    m, n = req.m, req.n
    h = 1.0 / (max(m, n) - 1)
    psi0 = W.random_boundary(m, n, rng)
    lx, ly = h * (m - 1), h * (n - 1)
    amp = rng.standard_normal(32)
    cx = rng.random(32) * lx
    cy = rng.random(32) * ly
    sig = rng.uniform(0.01, 0.1, 32) * max(lx, ly)
    x = torch.arange(m, device=dev, dtype=torch.float64) * h
    y = torch.arange(n, device=dev, dtype=torch.float64) * h
    f = torch.zeros((n, m), device=dev, dtype=torch.float64)
    for k in range(32):
        gx = torch.exp(-((x - cx[k]) ** 2) / (2.0 * sig[k] ** 2))
        gy = torch.exp(-((y - cy[k]) ** 2) / (2.0 * sig[k] ** 2))
        f += amp[k] * torch.outer(gy, gx)
    return torch.as_tensor(psi0, device=dev), f, h, h


def run_copy_probe(torch, lap, dev):
    """Achievable HBM bandwidth: plain copy of 1 GiB with several grid sizes
    (also the calibration kernel of the byte counters)."""
    src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    best = {}
    for blocks in (1024, 2048, 4096, 8192):
        lap.op_stream_copy(src, dst, blocks=blocks)
        sync()
        t0 = time.perf_counter()
        for _ in range(10):
            lap.op_stream_copy(src, dst, blocks=blocks)
        sync()
        t = (time.perf_counter() - t0) / 10
        best[blocks] = 2 * (1 << 30) / t / 1e9
    del src, dst
    return {"bytes_per_launch": 2 * (1 << 30), "GB/s_by_blocks": best, "best_GB/s": max(best.values())}


def run_batch_leg(args, ctx, torch, lap, dev):
    """Ragged batch: 512 grids, m, n log-uniform in [33, 1025] (snapped to
    c*2^k+1), aspect <= 3, beta in [0.5, 2], U[0,1) boundary, f = 0."""
    count = args.batch_count
    probs = W.ragged_batch(count=count, lo=33, hi=1025, seed=4)
    grids = [ctx.grid(torch.as_tensor(p.psi0, device=dev), None, p.dx, p.dy,
                      alloc=lap.LAP_ALLOC_MIXED | lap.LAP_ALLOC_ADI) for p in probs]
    nodes = sum((p.m - 2) * (p.n - 2) for p in probs)
    lpc = [lup_per_cycle(g.levels()) for g in grids]
    out = {"grids": count, "interior_nodes": nodes}
    # warm-up (plans, graphs), then timed batched mixed-precision multigrid
    ctx.solve_batch(grids, method="mg", precision="mixed", tol=1e-10, max_iter=200)
    for g, p in zip(grids, probs):
        g.write(torch.as_tensor(p.psi0, device=dev))
    sync()
    t0 = time.perf_counter()
    infos = ctx.solve_batch(grids, method="mg", precision="mixed", tol=1e-10, max_iter=200)
    sync()
    t = time.perf_counter() - t0
    its = [i["iterations"] for i in infos]
    out["mg_mixed"] = {"seconds": t, "GLUP/s": sum(k * l for k, l in zip(its, lpc)) / t / 1e9,
                       "cycles_min": min(its), "cycles_max": max(its),
                       "all_converged": all(i["status"] == 0 for i in infos),
                       "solves_per_s": count / t}
    # the same grids one at a time
    for g, p in zip(grids, probs):
        g.write(torch.as_tensor(p.psi0, device=dev))
    sync()
    t0 = time.perf_counter()
    seq = [g.solve("mg", precision="mixed", tol=1e-10, max_iter=200) for g in grids]
    sync()
    ts = time.perf_counter() - t0
    out["mg_mixed_one_at_a_time"] = {"seconds": ts, "speedup_of_batch": ts / t,
                                     "same_iterations": [i["iterations"] for i in seq] == its}
    # batched zebra ADI: fixed number of iterations (every interior node is
    # updated twice per iteration: once by its row, once by its column)
    for g, p in zip(grids, probs):
        g.write(torch.as_tensor(p.psi0, device=dev))
    nit = args.adi_iters
    # warm-up builds the merged-launch plan of the timed step (same check block)
    ctx.solve_batch(grids, method="adi", omega=1.0, tol=0.0, max_iter=nit, check_every=nit)
    for g, p in zip(grids, probs):
        g.write(torch.as_tensor(p.psi0, device=dev))
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


def run_serving_leg(args, ctx, torch, lap, dev):
    """Poisson arrivals; m, n log-uniform in [17, 4097] snapped, beta = 1,
    32-bump source, tol 1e-8 or 1e-10; continuous batching (mixed) vs
    one-at-a-time FP64 solves."""
    from paper_2208_02427_amd.serving import Job, Server, DeviceBackend, serve_sequential
    res = {}
    for rate in args.rates:
        reqs = W.poisson_requests(rate, args.serve_count, seed=5, lo=17, hi=4097)
        jobs = [Job(r.rid, r.arrival, r.m, r.n, r.tol, payload=device_request(torch, r, dev)) for r in reqs]
        nodes = {j.rid: (j.m - 2) * (j.n - 2) for j in jobs}
        sync()
        stats = Server(DeviceBackend(ctx, precision="mixed"), max_active=256, burst=args.burst,
                       solo_max_nodes=args.solo_max_nodes).run(jobs)
        sm = stats.summary()
        sm["GLUP/s"] = None
        sm["burst"] = args.burst
        sm["solo_max_nodes"] = args.solo_max_nodes
        res[str(int(rate))] = {"batched_mixed": sm}
        if rate in args.baseline_rates:
            def solve_one(job):
                psi0, f, dx, dy = job.payload
                g = ctx.grid(psi0, f, dx, dy, alloc=lap.LAP_ALLOC_FP64)
                info = g.solve("mg", precision="fp64", tol=job.tol, max_iter=100)
                g.destroy()
                return info
            jobs2 = [Job(j.rid, r.arrival, j.m, j.n, j.tol, payload=j.payload) for j, r in zip(jobs, reqs)]
            sync()
            res[str(int(rate))]["one_at_a_time_fp64"] = serve_sequential(solve_one, jobs2).summary()
        del jobs
        torch.cuda.empty_cache()
    return res


def cpu_baseline():
    """The oracle as it stands: one FP64 V(2,2) cycle of the 4097 x 4097 solve."""
    from oracle import multigrid as omg
    N = 4097
    p = W.square_problem(N, seed=2)
    lv = omg.hierarchy(N, N, p.dx, p.dy)
    u = p.psi0.copy()
    t0 = time.perf_counter()
    omg.vcycle(lv, 0, u, None)
    t = time.perf_counter() - t0
    lups = lup_per_cycle([(a, b) for a, b, _, _ in lv])
    return {"value": lups / t / 1e9, "unit": "GLUP/s", "cores": 1, "kind": "oracle",
            "sample": f"one FP64 V(2,2) cycle of the 4097x4097 solve (11 levels), numpy oracle, {t:.1f} s; "
                      f"host has {len(os.sched_getaffinity(0))} cores, numpy elementwise runs on 1"}


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
    ap.add_argument("--copy-probe", action="store_true", help="also time a plain 1 GiB device copy")
    ap.add_argument("--measure-only", action="store_true",
                    help="only measured-mode solves (for profiler runs: no graph replay leg)")
    ap.add_argument("--no-batch", dest="batch", action="store_false", help="skip the ragged-batch leg")
    ap.add_argument("--mixed-only", action="store_true",
                    help="run only the mixed-vs-FP64 leg and print its JSON (profiling aid; not the benchmark line)")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the ragged-batch leg and print its JSON (profiling aid; not the benchmark line)")
    ap.add_argument("--no-serve", dest="serve", action="store_false", help="skip the serving leg")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--adi-iters", type=int, default=20)
    ap.add_argument("--serve-count", type=int, default=300)
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
    if args.mixed_only:
        import torch
        import paper_2208_02427_amd as lap
        ctx = lap.Context(arena_bytes=16 << 30, device="cuda:0")
        res = {"mixed": run_mixed_leg(args.size, ctx, torch, lap, "cuda:0")}
        if args.copy_probe:
            res["copy_probe"] = run_copy_probe(torch, lap, "cuda:0")
        print(json.dumps(res), flush=True)
        return
    if args.batch_only:
        import torch
        import paper_2208_02427_amd as lap
        ctx = lap.Context(arena_bytes=16 << 30, device="cuda:0")
        res = {"ragged_batch": run_batch_leg(args, ctx, torch, lap, "cuda:0")}
        if args.copy_probe:
            res["copy_probe"] = run_copy_probe(torch, lap, "cuda:0")
        print(json.dumps(res), flush=True)
        return
    out, levels = run_gpu(args)
    line = {
        "metric": METRIC,
        "value": round(out["value"], 3),
        "unit": "GLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(out["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.size}x{args.size} Laplace, unit square, U[0,1) Dirichlet (seed 2), f=0, "
                        f"FP64 V(2,2) multigrid to rel. residual 1e-10",
            "levels": len(levels), "cycles": out["cycles"], "parallelism": "single GPU",
        },
        "time_to_tol_s": round(out["time_to_tol_s"], 5),
        "time_to_tol_graph_s": None if out["time_to_tol_graph_s"] is None else round(out["time_to_tol_graph_s"], 5),
        "rel_res": out["rel_res"],
        "roofline": out["roofline"],
    }
    for k in ("solve_hbm", "residual_kernel", "copy_probe", "mixed", "sor", "mg_4097", "ragged_batch", "serving",
              "kernels_fine", "autotune"):
        if k in out:
            line[k] = out[k]
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
