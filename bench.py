"""Benchmark: one Newton-CG step of the 32-disk workload per timed step.

Workload (256x256 RGB, 32 disks with (cx, cy, r) = 96 parameters, sigma 0.02,
aggregate-importance-sampled HVPs with N = 65536 draws, 10 CG products per
Newton step).  A step = hr_newton_cg_step_dev on device-resident theta:
  1 gradient estimate (2N renders) + up to 10 HVP estimates (4N renders each)
  + the FP64 CG solve, every step of the path (draws, perturbed records,
  fused raster + MSE, weights, lobe sums, finalisation, solve) in the
  library's kernels.  Inputs (scene, target, theta, v) are resident in HBM
  before the timed region.

metric: perturbed Mpix/s = (renders actually made) * 65536 pixels / time.
Also reported: p50/p99 latency of single HVP queries, the roofline of the
dominant kernel (raster + MSE) from HIP events on its stream, and the CPU
oracle on a bounded sample of the same workload; then, on the same line,
`other_workloads` (one-disk gradient + Hessian, path-traced 6x6 Hessian),
`extensions` (limit HVP, grey-box, comparators, optimiser loop),
`uneven_batch` (64 uneven instances: plain calls vs one batch) and `serving`
(Poisson-arriving Newton optimisations: server vs plain calls).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--sections ...]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Hessian-estimator throughput (perturbed Mpix/s) + p50/p99 HVP-query latency"
PEAK_FP32_TFLOPS = 157.3          # MI355X fp32 vector (published)
PEAK_HBM_GBS = 8000.0             # MI355X HBM3E (published)
# path tracer, FP32 arithmetic per path of one render (FMA = 2 FLOP): the
# FMA/ADD/MUL instruction counters of the Hessian launch per path at full
# lanes when every render traced its camera ray alone (the kernel now finds a
# draw's shared camera-ray hits once, and executes 401 per path).  A path
# that takes every branch (two closest-hit searches over 4 spheres, plane and
# light, two light samples with shadow tests, frames, bounce, throughput) is
# ~550 by hand; rays that leave the scene and shadow tests that stop at their
# first blocker make the average path cheaper.  Square roots, reciprocals and
# sines (one instruction each) are not counted.
PT_FLOP_PER_PATH = 434.0
# the a-priori count of a path (4 rays x (4 spheres at ~17 FLOP + plane +
# light quad) + shading), reported beside the counter figure
PT_FLOP_PER_PATH_ESTIMATE = 520.0
# algorithmic work per perturbed pixel of the bbox-culled rasteriser + loss:
# 9 FLOP for the 3-channel squared error, 5 FLOP per disk test times the
# 0.593 disks whose bounding box holds an average pixel (32 disks, E[r^2]).
FLOP_PER_PIXEL = 12.0
# HBM bytes per k_raster_dloss launch (an HVP's render pairs) from rocprofv3
# FETCH_SIZE / WRITE_SIZE runs scaled by a 256 MiB copy, valid for the kernel
# source with this code digest (code_digest: comments and blank lines left
# out); reported as null once the code has changed (or before it is measured).
TRAFFIC_BYTES_PER_LAUNCH = 56815075
TRAFFIC_SOURCE_DIGEST = "9e16c4411464b8edfbc5c75948d831571bb90950294de1965e129fce815d7944"
# SQ counters of the same kernel source (rocprofv3 --pmc, mean of the step's
# 10 launches): VALU instructions per launch (131072 pairs), VALU
# instructions per CU and GRBM_GUI_ACTIVE cycle, and lane activity
# (SQ_THREAD_CYCLES_VALU / (64 SQ_ACTIVE_INST_VALU)); null once the code changes
COUNTERS_PER_LAUNCH = {"valu_insts": 626283457, "valu_per_cu_cycle": 1.229,
                       "lane_activity": 0.650}
# the same counters of the gradient's per-render kernel (k_raster_loss, 131072
# renders per launch), valid for the rasteriser source with this digest
GRADIENT_COUNTERS_PER_LAUNCH = {"valu_insts": 1574085178, "valu_per_cu_cycle": 0.997,
                                "lane_activity": 0.978}
GRADIENT_SOURCE_DIGEST = "3dab424d78be75391800e75b8beae93e6966f334696d37011efe1eb4c360ea6e"


def code_digest(path):
    """SHA-256 of a C++ source without its // comments and blank lines, so that
    an edit of comments alone keeps the measured traffic valid."""
    import hashlib
    import re
    lines = []
    for line in open(path, encoding="utf-8").read().splitlines():
        line = re.sub(r"//.*$", "", line).rstrip()
        if line:
            lines.append(line)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()


def raster_traffic():
    src = os.path.join(ROOT, "paper_2412_03489_amd", "csrc", "hr_edges.hip")
    return TRAFFIC_BYTES_PER_LAUNCH if code_digest(src) == TRAFFIC_SOURCE_DIGEST else None


def raster_counters():
    return dict(COUNTERS_PER_LAUNCH) if raster_traffic() is not None else None


def gradient_counters():
    src = os.path.join(ROOT, "paper_2412_03489_amd", "csrc", "hr_raster.hip")
    ok = code_digest(src) == GRADIENT_SOURCE_DIGEST
    return dict(GRADIENT_COUNTERS_PER_LAUNCH) if ok else None


def golden(name):
    """Expected values written by tests/golden/make_golden.py with the CPU FP64
    oracle alone (None if the file is absent)."""
    path = os.path.join(ROOT, "tests", "golden", f"full_{name}.npz")
    return np.load(path) if os.path.exists(path) else None


def cpu_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "affinity": avail, "model": model}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def render_target_on_gpu(P, ctx, w):
    """The benchmark's target is the library's own render at theta* (the GPU
    leg never runs the oracle)."""
    blank = np.zeros((w.H, w.W, w.C), np.float32)
    s0 = P.Scene.disks(ctx, w.W, w.H, w.C, w.colors, blank, radius=w.radius, ppd=w.ppd)
    tgt = s0.render(w.theta_star)
    s0.close()
    return tgt


def cpu_baseline(w, draws, single_draws, reps, gpu_hvp):
    """The oracle, untuned, on the first `draws` draws of the same HVP query:
    the median of `reps` runs on the host threads a GPU's share allows, one
    run on a single thread (first `single_draws` draws), and the GPU's result
    on the same draws against it."""
    import oracle as O
    O.build(force=False)
    blank = np.zeros((w.H, w.W, w.C), np.float32)
    sc0 = O.Scene.disks(w.W, w.H, w.C, w.colors, blank, radius=w.radius, ppd=w.ppd)
    tgt = O.render(sc0, w.theta_star, w.H, w.W, w.C).astype(np.float32)
    osc = O.Scene.disks(w.W, w.H, w.C, w.colors, tgt, radius=w.radius, ppd=w.ppd)
    info = cpu_info()
    # one GPU's share of a box's host is 16 threads (the worker-pool size the
    # boxes set); the oracle uses all of them when the host has that many
    share = int(os.environ.get("OMP_NUM_THREADS", "16") or 16)
    cores = max(1, min(info["affinity"], share))
    times = []
    ref = None
    for _ in range(reps):
        t0 = time.perf_counter()
        ref = O.estimate("hvp", osc, w.theta0, w.sigma, draws, w.seed, v=w.v, nthreads=cores)
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    t0 = time.perf_counter()
    O.estimate("hvp", osc, w.theta0, w.sigma, single_draws, w.seed, v=w.v, nthreads=1)
    dt1 = time.perf_counter() - t0
    renders = 4 * draws
    out = {"value": renders * w.pixels / dt / 1e6, "unit": "Mpix/s", "cores": cores,
           "kind": "oracle",
           "sample": f"one AIS HVP query of the same workload at N={draws} draws "
                     f"({renders} renders of 256x256x3), median of {reps} runs "
                     f"({', '.join(f'{t:.2f}' for t in times)} s)",
           "single_core_Mpix_per_s": 4 * single_draws * w.pixels / dt1 / 1e6,
           "single_core_sample": f"N={single_draws} draws on 1 thread, {dt1:.2f} s",
           "host": info}
    if gpu_hvp is not None:
        out["gpu_vs_oracle_rel_inf"] = rel_inf(gpu_hvp, ref)
    return out


def rel_inf(x, ref):
    x = np.ravel(np.asarray(x, float))
    ref = np.ravel(np.asarray(ref, float))
    return float(np.abs(x - ref).max() / max(np.abs(ref).max(), 1e-300))


def uneven_section(P, ctx, reps):
    """64 uneven disk instances at their full sample budgets: plain per-query
    calls one after another vs one batch (persistent launches, graph replay,
    autotuned raster configuration)."""
    import workloads as WL
    ws = WL.uneven(64)
    scenes, qs = [], []
    renders = pixels = 0
    for w in ws:
        sc = P.Scene.disks(ctx, w.W, w.H, w.C, w.colors, render_target_on_gpu(P, ctx, w),
                           radius=w.radius, ppd=w.ppd)
        scenes.append(sc)
        kind = w.kinds[0]
        q = dict(scene=sc, kind=kind, theta=w.theta0, sigma=w.sigma, N=w.N, seed=w.seed)
        if kind == "hvp":
            q["v"] = w.v
        qs.append(q)
        R = P.n_renders(kind, w.n, w.N)
        renders += R
        pixels += R * w.pixels

    def plain():
        return [P.estimate(q["kind"], q["scene"], q["theta"], q["sigma"], q["N"], q["seed"],
                           v=q.get("v")) for q in qs]

    log("bench: uneven batch, plain per-query calls")
    ref = plain()
    t0 = time.perf_counter()
    for _ in range(reps):
        plain()
    t_plain = (time.perf_counter() - t0) / reps
    log("bench: uneven batch, batched with the default raster configuration")
    b0 = P.Batch(ctx, use_graph=True, autotune=False)
    b0.run(qs)
    t0 = time.perf_counter()
    for _ in range(reps):
        b0.run(qs)
    t_default = (time.perf_counter() - t0) / reps
    b0.close()
    log("bench: uneven batch, batched (autotune on the first run)")
    b = P.Batch(ctx, use_graph=True, autotune=True)
    got = b.run(qs)
    t0 = time.perf_counter()
    for _ in range(reps):
        got = b.run(qs)
    t_batch = (time.perf_counter() - t0) / reps
    rep = b.report()
    picks = {}
    for sc in scenes:
        spb, tile = P.tuned(ctx, sc)
        key = f"S={spb},tile={('32x32', '32x32', '64x16', '16x64')[tile]}"
        picks[key] = picks.get(key, 0) + 1
    identical = all(np.array_equal(x, y) for x, y in zip(got, ref))
    # precision plan: compensated-FP32 lobe sums against FP64 accumulation
    fp64 = P.Batch(ctx, use_graph=False).run([dict(q, accum_fp64=True) for q in qs])
    err = max(rel_inf(x, y) for x, y in zip(got, fp64))
    b.close()
    for sc in scenes:
        sc.close()
    return {"instances": len(qs), "renders": renders, "perturbed_Mpix": round(pixels / 1e6, 1),
            "plain": {"ms": round(t_plain * 1e3, 3), "queries_per_s": round(len(qs) / t_plain, 1),
                      "Mpix_per_s": round(pixels / t_plain / 1e6, 1)},
            "batched": {"ms": round(t_batch * 1e3, 3),
                        "queries_per_s": round(len(qs) / t_batch, 1),
                        "Mpix_per_s": round(pixels / t_batch / 1e6, 1),
                        "graph": bool(rep["graph"]), "raster_items": rep["raster_items"],
                        "raster_blocks": rep["raster_blocks"]},
            "batched_default_config_ms": round(t_default * 1e3, 3),
            "autotuned_instances_by_choice": picks,
            "speedup": round(t_plain / t_batch, 3), "identical_to_plain": identical,
            "comp_fp32_vs_fp64_accum_max_rel": err, "reps": reps}


def serving_section(P, ctx, args):
    """Newton optimisations over the raster and path-traced scenes:
    continuous-batching server vs plain per-query calls served one at a time
    in the order queries become ready.  Two regimes:
      * the workloads' own sample budgets (raster HVPs and gradients at
        N = 65536, path-traced gradients and 6x6 Hessians at N = 8192): an
        open-loop saturating run (Poisson arrivals of optimisations of one
        step each), then closed-loop clients with no think time (the plain
        capacity of their query mix) and with think times offering 0.5, 0.8,
        1.0 and 1.5 x that capacity;
      * the paper's per-iteration budgets (appendix "Hyperparameters": a few
        antithetic draws per estimate; here 6), where a query is a few
        microseconds of GPU work: closed-loop clients with no think time and
        an open-loop Poisson stream."""
    import workloads as WL
    import bench_serving as SV
    wr = WL.disks32()
    wp = WL.pt_spheres()
    sr = P.Scene.disks(ctx, wr.W, wr.H, wr.C, wr.colors, render_target_on_gpu(P, ctx, wr),
                       radius=wr.radius, ppd=wr.ppd)
    s0 = P.Scene.pt(ctx, wp.W, wp.H, wp.spp, wp.desc, np.zeros((wp.H, wp.W, 3), np.float32))
    tp = s0.render(wp.theta_star, seed=wp.target_seed, s=0, spp=wp.target_spp)
    s0.close()
    sp = P.Scene.pt(ctx, wp.W, wp.H, wp.spp, wp.desc, tp)
    scenes = {"raster": sr, "pt": sp}
    sigma = {"raster": wr.sigma, "pt": wp.sigma}
    cg = args.serving_cg
    rnd = lambda d: {k: (round(v, 3) if isinstance(v, float) else v) for k, v in d.items()}
    keep = ("queries", "queries_per_s", "p50_ms", "p99_ms", "by_kind")
    keep_srv = keep + ("batches", "mean_batch")

    def clients(specs, N, steps=1):
        return SV.make_clients(specs, scenes, sigma, N, cg, steps=steps, full_cg=True)

    def regime(N, open_clients, rate, sweep):
        # warm both paths
        warm = WL.serving_clients(4, rate=1e6, base_seed=99)
        SV.run_plain(ctx, clients(warm, N))
        SV.run_served(ctx, clients(warm, N))
        out = {"client": f"raster: 1 gradient + {cg} HVPs (N={N['raster']}); "
                         f"path-traced: gradient + 6x6 Hessian (N={N['pt']})"}
        specs = WL.serving_clients(open_clients, rate=rate)
        log(f"bench: serving N={N}, {len(specs)} optimisations arriving at {rate}/s, plain")
        plain = SV.run_plain(ctx, clients(specs, N))
        log(f"bench: serving N={N}, {len(specs)} optimisations arriving at {rate}/s, served")
        served = SV.run_served(ctx, clients(specs, N))
        out["open_loop"] = {"optimisations": len(specs), "arrival_rate_per_s": rate,
                            "plain": rnd(plain), "served": rnd(served),
                            "qps_ratio": round(served["queries_per_s"] / plain["queries_per_s"], 3)}
        # closed loop: the clients all start together and keep taking Newton
        # steps, thinking an exponential time before each query; no query
        # becomes ready after the window.  The plain capacity of the mix is
        # measured first (no think time) and the offered loads are scaled
        # from it (think mean = clients / (load x capacity)).
        win = args.serving_window
        nc = args.serving_sweep_clients
        specs = WL.serving_clients(nc, rate=1e6, base_seed=3000)
        log(f"bench: serving N={N}, closed loop, {nc} clients, no think time")
        pl = SV.run_plain(ctx, clients(specs, N, 10 ** 6), think_ms=0.0, window_s=win)
        sv = SV.run_served(ctx, clients(specs, N, 10 ** 6), think_ms=0.0, window_s=win)
        cap = pl["queries_per_s"]
        out["closed_loop_saturated"] = {"clients": nc, "window_s": win,
                                        "plain": rnd({k: pl[k] for k in keep}),
                                        "served": rnd({k: sv[k] for k in keep_srv}),
                                        "qps_ratio": round(sv["queries_per_s"] / cap, 3)}
        out["closed_loop_plain_capacity_qps"] = round(cap, 2)
        rows = []
        for rho in sweep:
            think_ms = 1e3 * nc / (rho * cap)
            log(f"bench: serving N={N}, closed loop, load {rho} x plain capacity "
                f"(think {think_ms:.1f} ms)")
            pl = SV.run_plain(ctx, clients(specs, N, 10 ** 6), think_ms=think_ms, window_s=win)
            sv = SV.run_served(ctx, clients(specs, N, 10 ** 6), think_ms=think_ms, window_s=win)
            rows.append({"load": rho, "think_ms": round(think_ms, 2), "window_s": win,
                         "plain": rnd({k: pl[k] for k in keep}),
                         "served": rnd({k: sv[k] for k in keep_srv})})
        if rows:
            out["closed_loop_sweep"] = rows
        return out

    out = {"clients": args.serving_clients}
    out["workload_budgets"] = regime({"raster": args.serving_n_raster, "pt": args.serving_n_pt},
                                     args.serving_clients, args.serving_rate,
                                     (0.5, 0.8, 1.0, 1.5))
    out["paper_budgets"] = regime({"raster": args.serving_small_n, "pt": args.serving_small_n},
                                  args.serving_small_clients, args.serving_small_rate,
                                  (0.5, 1.0))
    sr.close()
    sp.close()
    return out


def main_section(P, ctx, args):
    """The headline workload: Newton-CG steps of the 32-disk scene, single-HVP
    latency and the raster kernel's roofline."""
    import workloads as WL
    w = WL.disks32()
    tgt = render_target_on_gpu(P, ctx, w)
    sc = P.Scene.disks(ctx, w.W, w.H, w.C, w.colors, tgt, radius=w.radius, ppd=w.ppd)
    th0 = ctx.alloc(8 * w.n)
    th = ctx.alloc(8 * w.n)
    v = ctx.alloc(8 * w.n)
    out = ctx.alloc(8 * w.n)
    th0.upload(w.theta0)
    v.upload(w.v)
    # Hessian modification inside CG (curvature |v^T H v|, steps truncated to
    # Delta = 0.05, the scale of the disks' offsets): every step makes its 10
    # HVP products
    kw = dict(cg_iters=w.cg_iters, trust_radius=0.05, modified=True,
              samples_per_block=args.samples_per_block)

    def step():
        th.copy_from(th0)
        return P.newton_cg_step_dev(sc, th.ptr, w.sigma, w.N, w.seed, **kw)

    log(f"bench: workload {w.name}, N={w.N}, warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    ctx.synchronize()
    ctx.reset_stats()
    ctx.enable_timing(True)
    log(f"bench: timing {args.steps} steps")
    renders = 0
    t0 = time.perf_counter()
    for k in range(args.steps):
        rep = step()
        renders += 2 * w.N + rep["iters_done"] * 4 * w.N
    ctx.synchronize()
    dt = time.perf_counter() - t0
    # the HVPs' render pairs (k_raster_dloss) and the gradient's renders
    # (k_raster_loss), each timed by HIP events on the launch stream
    launches, raster_ms = ctx.kernel_stats("raster_dloss")
    g_launches, g_raster_ms = ctx.kernel_stats("raster_loss")
    red_launches, red_ms = ctx.kernel_stats("tile_reduce")
    ctx.enable_timing(False)
    log(f"bench: {args.steps} steps in {dt:.3f} s, pair raster launches {launches}, "
        f"gradient raster launches {g_launches}")
    theta_step = th.download(w.n)

    # single-HVP query latency (host wall clock, call to completion)
    lat = []
    for q in range(args.hvp_queries):
        t1 = time.perf_counter()
        P.estimate_dev("hvp", sc, th0.ptr, w.sigma, w.N, w.seed + 1 + q, out.ptr, d_v=v.ptr)
        ctx.synchronize()
        lat.append((time.perf_counter() - t1) * 1e3)
    lat = np.array(lat) if lat else np.array([float("nan")])
    if args.calibrate_copy_mb > 0:
        nb = args.calibrate_copy_mb << 20
        src, dst = ctx.alloc(nb), ctx.alloc(nb)
        dst.copy_from(src)
        ctx.synchronize()
        src.free()
        dst.free()
        log(f"bench: calibration copy of {nb} bytes done")

    # the error of the benchmarked results against FP64: the timed step, a
    # full-size HVP and gradient, against the oracle's expected values
    errors = {}
    ref = golden("disks32_newton")
    if ref is not None:
        errors["newton_step_rel_inf"] = rel_inf(theta_step - w.theta0, ref["theta"] - w.theta0)
    ref = golden("disks32_hvp")
    if ref is not None:
        errors["hvp_rel_inf"] = rel_inf(P.estimate("hvp", sc, w.theta0, w.sigma, w.N, w.seed,
                                                   v=ref["v"]), ref["out"])
    ref = golden("disks32_grad")
    if ref is not None:
        errors["gradient_rel_inf"] = rel_inf(P.estimate("grad", sc, w.theta0, w.sigma, w.N,
                                                        w.seed), ref["out"])
    gpu_hvp_sample = P.estimate("hvp", sc, w.theta0, w.sigma, args.cpu_draws, w.seed, v=w.v)

    pix_total = renders * w.pixels
    value = pix_total / dt / 1e6
    # dominant kernel: the HVPs' render pairs (4N renders per launch); the
    # gradient's launch (2N renders) is reported beside it
    steps = args.steps
    hvps = (renders - 2 * w.N * steps) // (4 * w.N)
    avg_ms = raster_ms / max(launches, 1)
    flop_per_launch = FLOP_PER_PIXEL * 4 * w.N * w.pixels
    achieved = flop_per_launch / (avg_ms * 1e-3) / 1e12
    g_avg_ms = g_raster_ms / max(g_launches, 1)
    g_achieved = FLOP_PER_PIXEL * 2 * w.N * w.pixels / (g_avg_ms * 1e-3) / 1e12
    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "disks32_256x256_rgb: one Newton-CG step = 1 gradient + "
                               "10 aggregate-sampled HVPs (CG with Hessian modification), "
                               "N=65536 draws, antithetic",
                   "pixels_per_render": w.pixels, "params": w.n, "sigma": w.sigma,
                   "draws": w.N, "renders_per_step": renders // steps,
                   "hvps_per_step": hvps / steps},
        "hvp_latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                           "p99": round(float(np.percentile(lat, 99)), 3),
                           "queries": int(args.hvp_queries)},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                     "traffic": raster_traffic(), "kernel": "k_raster_dloss",
                     "avg_launch_ms": round(avg_ms, 4), "launches": int(launches),
                     "flop_per_pixel": FLOP_PER_PIXEL,
                     "renders_per_launch": 4 * w.N,
                     # the kernel decides only the pixels along the disks'
                     # edges, so the rate per perturbed pixel can exceed the
                     # FP32 peak; VALU issue is its bound
                     "per_pixel_equivalent": True,
                     "counters": raster_counters()},
        "roofline_gradient": {"bound": "alu", "kernel": "k_raster_loss",
                              "achieved": round(g_achieved, 3), "peak": PEAK_FP32_TFLOPS,
                              "unit": "TFLOP/s", "frac": round(g_achieved / PEAK_FP32_TFLOPS, 4),
                              "avg_launch_ms": round(g_avg_ms, 4), "launches": int(g_launches),
                              "renders_per_launch": 2 * w.N,
                              # at the VALU issue limit (one non-packed
                              # instruction per CU-cycle)
                              "counters": gradient_counters()},
        "error_vs_fp64": errors,
        "cpu_baseline": None,
    }
    # the loss pass of the gradient's renders (an HVP's render pairs write
    # their loss differences directly): per render its wave-tile partials are
    # read (4 B each) and one FP64 value written; HBM-bound, against the
    # 8 TB/s peak
    subs = ((w.W + 15) // 16) * ((w.H + 15) // 16)
    outputs = 2 * w.N * red_launches
    red_bytes = outputs * (subs * 4 + 8)
    red_gbs = red_bytes / (red_ms * 1e-3) / 1e9 if red_ms > 0 else None
    line["loss_pass"] = {"bound": "hbm", "kernel": "k_tile_reduce",
                         "achieved": round(red_gbs, 1) if red_gbs else None,
                         "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": round(red_gbs / PEAK_HBM_GBS, 4) if red_gbs else None,
                         "avg_launch_ms": round(red_ms / max(red_launches, 1), 4),
                         "launches": int(red_launches),
                         "bytes_per_output": subs * 4 + 8,
                         "outputs": int(outputs)}
    for b in (th0, th, v, out):
        b.free()
    sc.close()
    return line, gpu_hvp_sample


def configs_section(P, ctx, reps):
    """The other workloads of the estimator: the one-disk gradient + Hessian
    (64x64, N = 4096; mean per pair and p50/p99 latency per call) and the
    path-traced full 6x6 Hessian (128x128, 4 spp, N = 8192), each timed as
    host call to result."""
    import workloads as WL
    out = {}
    w = WL.one_disk()
    sc = P.Scene.disks(ctx, w.W, w.H, w.C, w.colors, render_target_on_gpu(P, ctx, w),
                       radius=w.radius, ppd=w.ppd)

    def one_disk():
        P.estimate("grad", sc, w.theta0, w.sigma, w.N, w.seed)
        P.estimate("hess", sc, w.theta0, w.sigma, w.N, w.seed)

    one_disk()
    t0 = time.perf_counter()
    for _ in range(reps):
        one_disk()
    dt = (time.perf_counter() - t0) / reps
    renders = 2 * P.n_renders("grad", w.n, w.N)
    # latency of single calls (host pointer in, result on the host), 200 each
    lat = {}
    for kind in ("grad", "hess"):
        xs = []
        for i in range(200):
            t1 = time.perf_counter()
            P.estimate(kind, sc, w.theta0, w.sigma, w.N, w.seed + i)
            xs.append((time.perf_counter() - t1) * 1e3)
        lat[kind] = {"p50_ms": round(float(np.percentile(xs, 50)), 4),
                     "p99_ms": round(float(np.percentile(xs, 99)), 4)}
    out["one_disk_grad_hess"] = {"ms": round(dt * 1e3, 3), "renders": renders,
                                 "Mpix_per_s": round(renders * w.pixels / dt / 1e6, 1),
                                 "latency": lat}
    sc.close()
    wp = WL.pt_spheres()
    s0 = P.Scene.pt(ctx, wp.W, wp.H, wp.spp, wp.desc, np.zeros((wp.H, wp.W, 3), np.float32))
    tp = s0.render(wp.theta_star, seed=wp.target_seed, s=0, spp=wp.target_spp)
    s0.close()
    sp = P.Scene.pt(ctx, wp.W, wp.H, wp.spp, wp.desc, tp)
    P.estimate("hess", sp, wp.theta0, wp.sigma, wp.N, wp.seed)
    t0 = time.perf_counter()
    for _ in range(reps):
        P.estimate("hess", sp, wp.theta0, wp.sigma, wp.N, wp.seed)
    dt = (time.perf_counter() - t0) / reps
    renders = P.n_renders("hess", wp.n, wp.N)
    paths = renders * wp.pixels * wp.spp
    tflops = PT_FLOP_PER_PATH * paths / dt / 1e12
    tflops_est = PT_FLOP_PER_PATH_ESTIMATE * paths / dt / 1e12
    out["pt_spheres_hessian"] = {"ms": round(dt * 1e3, 3), "renders": renders,
                                 "Mpix_per_s": round(renders * wp.pixels / dt / 1e6, 1),
                                 "Mpaths_per_s": round(paths / dt / 1e6, 1),
                                 "roofline": {"bound": "alu", "flop_per_path": PT_FLOP_PER_PATH,
                                              "achieved": round(tflops, 3),
                                              "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                                              "frac": round(tflops / PEAK_FP32_TFLOPS, 4),
                                              "flop_per_path_estimate": PT_FLOP_PER_PATH_ESTIMATE,
                                              "achieved_at_estimate": round(tflops_est, 3),
                                              "frac_at_estimate": round(tflops_est / PEAK_FP32_TFLOPS, 4)}}
    sp.close()
    return out


def extensions_section(P, ctx, reps):
    """The estimator's extensions on the 96-parameter raster scene, each timed
    as host call to result: the limit-kernel HVP against the central
    difference, the grey-box composition against the plain estimates, the
    plain-Gaussian and FR22 comparators against the aggregate gradient, and
    the optimiser loop (Newton-CG iterations with sigma annealing and a line
    search on the smoothed loss)."""
    import workloads as WL
    w = WL.disks32()
    sc = P.Scene.disks(ctx, w.W, w.H, w.C, w.colors, render_target_on_gpu(P, ctx, w),
                       radius=w.radius, ppd=w.ppd)

    def timed(fn):
        fn()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        return (time.perf_counter() - t0) / reps * 1e3

    N = w.N
    out = {"workload": "disks32_256x256_rgb", "draws": N}
    hvp = timed(lambda: P.estimate("hvp", sc, w.theta0, w.sigma, N, w.seed, v=w.v))
    lim = timed(lambda: P.estimate("hvp_limit", sc, w.theta0, w.sigma, N, w.seed, v=w.v))
    out["hvp_central_ms"] = round(hvp, 3)
    out["hvp_limit_ms"] = round(lim, 3)
    # grey-box: 32 inner parameters (one scale per disk) mapped linearly onto
    # the 96 scene parameters
    J = np.zeros((w.n, 32))
    for k in range(32):
        J[3 * k:3 * k + 3, k] = w.theta0[3 * k:3 * k + 3]
    y = w.theta0
    out["greybox_grad_ms"] = round(timed(lambda: P.estimate_greybox("grad", sc, y, J, w.sigma, N,
                                                                     w.seed)), 3)
    out["plain_grad_ms"] = round(timed(lambda: P.estimate("grad", sc, y, w.sigma, N, w.seed)), 3)
    out["greybox_hess_ms"] = round(timed(lambda: P.estimate_greybox("hess", sc, y, J, w.sigma,
                                                                     4096, w.seed)), 3)
    out["plain_hess_N4096_ms"] = round(timed(lambda: P.estimate("hess", sc, y, w.sigma, 4096,
                                                                w.seed)), 3)
    out["gauss_grad_ms"] = round(timed(lambda: P.estimate("grad", sc, y, w.sigma, N, w.seed,
                                                          sampler=P.GAUSS)), 3)
    out["fr22_grad_N1024_ms"] = round(timed(lambda: P.estimate("grad", sc, y, w.sigma, 1024,
                                                               w.seed, sampler=P.FR22)), 3)
    t0 = time.perf_counter()
    P.optimize(sc, w.theta0, 16384, w.seed, 4, 0.04, 0.02, method="newton_cg", ls_iters=3,
               N_loss=4096, cg_iters=4, trust_radius=0.05, modified=True)
    out["optimiser_newton_cg_ms_per_iter"] = round((time.perf_counter() - t0) / 4 * 1e3, 3)
    out["optimiser_setup"] = "N=16384, 4 CG products, 3 line-search halvings, N_loss=4096"
    sc.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--hvp-queries", type=int, default=30)
    ap.add_argument("--cpu-draws", type=int, default=4096,
                    help="draws of the oracle's timed HVP (median of --cpu-reps runs)")
    ap.add_argument("--cpu-reps", type=int, default=5)
    ap.add_argument("--cpu-single-draws", type=int, default=256,
                    help="draws of the oracle's single-thread run")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--samples-per-block", type=int, default=0)
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="after the run, one device-to-device copy of this many MiB "
                         "(a kernel of known traffic for scaling memory counters)")
    ap.add_argument("--sections", default="main,configs,extensions,uneven,serving",
                    help="comma list of main, configs, extensions, uneven, serving "
                         "(default: all)")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven-batch section")
    ap.add_argument("--uneven-reps", type=int, default=3)
    ap.add_argument("--no-serving", action="store_true", help="skip the serving section")
    ap.add_argument("--serving-clients", type=int, default=128)
    ap.add_argument("--serving-rate", type=float, default=256.0)
    ap.add_argument("--serving-sweep-clients", type=int, default=256)
    ap.add_argument("--serving-window", type=float, default=4.0,
                    help="seconds of closed-loop traffic per offered load")
    ap.add_argument("--serving-n-raster", type=int, default=65536)
    ap.add_argument("--serving-n-pt", type=int, default=8192)
    ap.add_argument("--serving-small-n", type=int, default=6,
                    help="draws per estimate of the paper-budget serving regime")
    ap.add_argument("--serving-small-clients", type=int, default=512)
    ap.add_argument("--serving-small-rate", type=float, default=8192.0)
    ap.add_argument("--serving-cg", type=int, default=10)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import paper_2412_03489_amd as P
    import workloads as WL

    sections = set(args.sections.split(","))
    if args.no_uneven:
        sections.discard("uneven")
    if args.no_serving:
        sections.discard("serving")
    ctx = P.Context(0)
    gpu_hvp_sample = None
    if "main" in sections:
        line, gpu_hvp_sample = main_section(P, ctx, args)
    else:   # a diagnostic run of the other sections only (for profiling)
        line = {"metric": METRIC, "value": None, "unit": "Mpix/s", "n_gpus": 1,
                "note": "headline section skipped (--sections)"}
    if "configs" in sections:
        line["other_workloads"] = configs_section(P, ctx, 5)
    if "extensions" in sections:
        line["extensions"] = extensions_section(P, ctx, 3)
    if "uneven" in sections:
        line["uneven_batch"] = uneven_section(P, ctx, args.uneven_reps)
    if "serving" in sections:
        line["serving"] = serving_section(P, ctx, args)
    ctx.close()
    if not args.no_cpu and "main" in sections:
        log(f"bench: CPU oracle baseline at N={args.cpu_draws}")
        line["cpu_baseline"] = cpu_baseline(WL.disks32(), args.cpu_draws, args.cpu_single_draws,
                                            args.cpu_reps, gpu_hvp_sample)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
