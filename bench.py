"""Benchmark of the SEPSO planner hot path on one MI355X.

A step is one planning frame of every instance of the batched workload:
1024 independent dynamic instances of uneven size (8-32 waypoints, 4-100
rectangles, 32-256 particles per group over 8 groups, maps 128-512 cells),
each frame (100 timed by default) = device obstacle motion + Priori Initialization + up to 50 fused
iterations with Auto Truncation and online self-evolution, all in one
captured HIP graph.  Inputs are resident in HBM before timing starts.

Printed: one JSON line with plans/s (value), segment x edge tests/s, the
roofline of the dominant kernel (the fused iteration, FP32 VALU bound), the
FP64 oracle timed on host cores, and the paper-shaped single instance.
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

METRIC = "plans/sec at oracle-matched cost; seg×edge tests/s vs FP32 VALU peak"
PEAK_FP32 = 157.3e12   # MI355X FP32 vector, published (packed FP32)
PEAK_HBM = 8.0e12      # MI355X HBM3E, published
F_TEST = 10.0          # algorithmic FLOP per segment x edge test
BYTES_PER_ELEM = 20.0  # algorithmic HBM bytes per swarm element and iteration
COUNTERS = os.path.join(ROOT, "profiles", "iter_kernel_batch1024_counters.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2308_10169_amd", "csrc", "kernels.hip")


def counter_record(kernel, tune):
    """HBM traffic and VALU instruction count per launch of the fused
    iteration for this tile shape, from the committed rocprofv3 counter
    summary -- only while it describes this kernel source (else None)."""
    import hashlib
    try:
        sha, rec = None, None
        with open(COUNTERS) as f:
            for line in f:
                line = line.strip()
                if line.startswith("source_sha256: "):
                    sha = line.split(": ", 1)[1]
                elif line.startswith(f"tile {tune[0]},{tune[1]}: "):
                    rec = dict(kv.split("=", 1) for kv in line.split(": ", 1)[1].split())
        with open(KERNEL_SRC, "rb") as f:
            cur = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    if rec is None or sha != cur or rec.get("kernel") != kernel:
        return None
    out = dict(hbm_bytes=float(rec["hbm_bytes_per_launch"]),
               valu_insts=float(rec["valu_insts_per_launch"]))
    if "valu_busy" in rec:
        out["valu_issue_ratio"] = float(rec["valu_busy"])
    if "fp32_flop_per_launch" in rec:
        out["fp32_flop"] = float(rec["fp32_flop_per_launch"])
    return out


def executed_fraction(bp, specs, sws, tile_of, sample):
    """Share of the segment x edge tests the fused iteration actually runs:
    a wave skips a rectangle outside the bounding box of its points, and of a
    rectangle it keeps, every edge whose line does not pass strictly through
    that box.  The
    kernel's mapping (blocks of an even number of whole particles, thread t
    on chunk t // ppb of K segments of particle t % ppb, 64 threads per wave)
    is replayed on the swarm state left by the timed launches of sampled
    instances."""
    run = tot = 0.0
    for i in sample:
        K, B = tile_of(i)
        spec, sw = specs[i], sws[i]
        W, S = sw.waypoints, sw.waypoints + 2
        X = bp.get_state(i)["X"].reshape(-1, 2 * W).astype(np.float64)
        P = len(X)
        px = np.empty((P, S))
        py = np.empty((P, S))
        px[:, 0], py[:, 0] = spec.start
        px[:, -1], py[:, -1] = spec.target
        px[:, 1:-1], py[:, 1:-1] = X[:, :W], X[:, W:]
        rects = np.array([[v[:, 0].min(), v[:, 1].min(), v[:, 0].max(), v[:, 1].max()]
                          for v in (spec.verts[spec.poly_ptr[q]:spec.poly_ptr[q + 1]]
                                    for q in range(spec.n_polys))]).reshape(-1, 4)
        C = (W + K) // K
        ppb = max(2, (B // C) & ~1)
        t = np.arange(B)
        c, jt = t // ppb, t % ppb
        for p0 in range(0, P, ppb):
            np_ = min(ppb, P - p0)
            for w0 in range(0, B, 64):
                lanes = slice(w0, w0 + 64)
                ok = (c[lanes] < C) & (jt[lanes] < np_)
                if not ok.any():
                    continue
                cc, jj = c[lanes][ok], jt[lanes][ok]
                idx = np.minimum(cc[:, None] * K + np.arange(K + 1)[None, :], S - 1)
                wx, wy = px[p0 + jj[:, None], idx], py[p0 + jj[:, None], idx]
                segs = np.count_nonzero(cc[:, None] * K + np.arange(K)[None, :] < S - 1)
                x0, x1, y0, y1 = wx.min(), wx.max(), wy.min(), wy.max()
                keep = ~((rects[:, 2] <= x0) | (rects[:, 0] >= x1) |
                         (rects[:, 3] <= y0) | (rects[:, 1] >= y1))
                r = rects[keep]
                edges = (((r[:, 1] > y0) & (r[:, 1] < y1)).sum() + ((r[:, 3] > y0) & (r[:, 3] < y1)).sum()
                         + ((r[:, 0] > x0) & (r[:, 0] < x1)).sum() + ((r[:, 2] > x0) & (r[:, 2] < x1)).sum())
                run += float(segs) * edges
                tot += 4.0 * segs * len(rects)
    return run / tot if tot else 1.0


def batch_workload(n_inst, seed_base=0):
    from paper_2308_10169_amd import inputs as I
    specs, sws = [], []
    for i in range(n_inst):
        m, shape = I.batch_instance(i, seed_base)
        sws.append(I.dynamic_swarm(m.scale, seed=seed_base, instance=i, **shape))
        specs.append(m)
    return specs, sws


def cost_parity(gpu_cost, orc_cost):
    """Plans at oracle-matched cost: frame 0 of the instances the oracle
    planned, GPU (FP32) against oracle (FP64) on the same instances and
    random streams.  Matched when the median over instances of the cost
    ratio GPU / oracle is within 1% of 1.  The instances differ in map size
    (128-512) and obstacle count, so their costs spread over a wide range;
    the gap between the two sides' medians over instances is reported too,
    but it moves by whole spacings between neighbouring instances whenever
    one instance near the middle lands on the other side of it."""
    ids = sorted(orc_cost)
    g = np.array([gpu_cost[i] for i in ids], dtype=np.float64)
    o = np.array([orc_cost[i] for i in ids], dtype=np.float64)
    med_g, med_o = float(np.median(g)), float(np.median(o))
    ratio = g / o
    med_ratio = float(np.median(ratio))
    return dict(instances=len(ids), median_cost_ratio=med_ratio,
                geomean_cost_ratio=float(np.exp(np.mean(np.log(ratio)))),
                instances_within_1pct=int(np.sum(np.abs(ratio - 1.0) <= 0.01)),
                median_cost_gpu=med_g, median_cost_oracle=med_o,
                median_gap=abs(med_g - med_o) / abs(med_o),
                matched=bool(abs(med_ratio - 1.0) <= 0.01))


_CPU_WORK = None  # (specs, swarms) shared with the forked oracle processes


def _oracle_process(job):
    """One host process: the FP64 oracle (single-threaded) plans the first
    frame of its share of the batch instances until the budget is spent."""
    share, budget_s = job
    from oracle import pyorc as orc
    specs, sws = _CPU_WORK
    t0 = time.perf_counter()
    done, tests, costs = 0, 0.0, {}
    for i in share:
        s = orc.Swarm(sws[i], specs[i].width, specs[i].height)
        r = s.plan_frame(orc.Map(specs[i]), 0)
        done += 1
        costs[i] = r["cost"]
        tests += sws[i].groups * sws[i].particles * (sws[i].waypoints + 1) * specs[i].n_edges * r["iters"]
        if time.perf_counter() - t0 > budget_s:
            break
    return done, tests, time.perf_counter() - t0, costs


def cpu_baseline(specs, sws, budget_s):
    """Oracle throughput on the host: one process per core (at most 16, the
    host share of one GPU), each planning first frames of its own instances
    (instance i goes to process i mod P).  Runs before the GPU is touched,
    so the processes are plain forks."""
    global _CPU_WORK
    import multiprocessing
    procs = max(1, min(16, len(os.sched_getaffinity(0))))
    _CPU_WORK = (specs, sws)
    jobs = [(list(range(w, len(specs), procs)), budget_s) for w in range(procs)]
    with multiprocessing.get_context("fork").Pool(procs) as pool:
        res = pool.map(_oracle_process, jobs)
    _CPU_WORK = None
    done = sum(r[0] for r in res)
    tests = sum(r[1] for r in res)
    wall = max(r[2] for r in res)
    costs = {}
    for r in res:
        costs.update(r[3])
    return dict(value=done / wall, unit="plans/s", cores=procs, kind="oracle",
                sample=f"first frames (frame 0: uniform start, up to 50 iterations with AT and "
                       f"online HSEF) of {done} batch instances (FP64 oracle, {procs} "
                       f"single-threaded processes, one per core), {wall:.1f} s; "
                       f"{tests / wall:.3g} tests/s"), costs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--instances", type=int, default=1024)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="library default tile instead of the autotuner")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: every box here has a single MI355X; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    t_gen = time.perf_counter()
    specs, sws = batch_workload(args.instances)
    print(f"# generated {args.instances} instances in {time.perf_counter() - t_gen:.1f}s",
          file=sys.stderr, flush=True)
    # the oracle baseline first: its host processes are forked before any GPU use
    cpu, orc_cost = (None, None) if args.no_cpu else cpu_baseline(specs, sws, args.cpu_budget)

    import torch
    from paper_2308_10169_amd import inputs as I
    from paper_2308_10169_amd import sepso

    sepso.lib()
    bp = sepso.BatchPlanner(specs, sws)
    tune, tiling = None, None
    if not args.no_tune:
        # tiles per bucket of instances (split by waypoint count), or one tile
        # for all when that plans a frame faster -- the autotuner decides
        tiles, bucket_of, fms = bp.autotune_buckets(4, frame_ms=True)
        tune = tiles[0] if len(tiles) == 1 else None
        tiling = dict(tiles=tiles, bucket_sizes=np.bincount(bucket_of).tolist(),
                      frame0_ms_buckets=fms[0], frame0_ms_one_tile=fms[1],
                      frame0_plans_per_s_buckets=args.instances / (fms[0] * 1e-3),
                      frame0_plans_per_s_one_tile=args.instances / (fms[1] * 1e-3))
    tests_iter, elems_iter = bp.work()
    print(f"# tiling {tiling}, tests/iteration {tests_iter:.4g}", file=sys.stderr, flush=True)

    # frame 0 of every instance from the fresh batch (the autotuner leaves it
    # as new): the cost the oracle reached on the same instances and streams
    torch.cuda.synchronize()
    tf0 = time.perf_counter()
    res0 = bp.plan(1)
    torch.cuda.synchronize()
    frame0_s = time.perf_counter() - tf0
    parity = cost_parity(res0["cost"][0], orc_cost) if orc_cost else None
    if parity:
        print(f"# frame-0 cost parity: {parity}", file=sys.stderr, flush=True)

    # dominant kernel: fused iteration over all instances (HIP events, library stream)
    bp.profile_step(20)  # warm-up: clocks settle
    kern_ms = bp.profile_step(20)

    bp.plan(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = bp.plan(args.steps, want_paths=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    plans = args.instances * args.steps
    iters = res["iters"].astype(np.float64)
    tests_run = 0.0
    for i in range(args.instances):
        per = sws[i].groups * sws[i].particles * (sws[i].waypoints + 1) * specs[i].n_edges
        tests_run += per * iters[:, i].sum()
    print(f"# {plans} plans in {dt:.3f}s, mean iters {iters.mean():.1f}", file=sys.stderr, flush=True)

    # Roofline of the fused iteration.  At this state (a frame planned, the
    # swarms converged) its time is set by its memory phase -- streaming every
    # swarm element once (read X, V, P; write X, V: 20 B) -- and not by its
    # crossing tests: a build without the crossing tests takes as long.  So
    # the bound is HBM, at the algorithmic 20 B per element; the ALU side (the
    # tests the wave culling leaves, replayed on the host from sampled
    # instances' swarm state, 10 FLOP each) is reported beside it.
    tile_of = ((lambda i: tune) if tune else
               (lambda i: tiling["tiles"][bucket_of[i]]) if tiling else (lambda i: (8, 128)))
    executed = executed_fraction(bp, specs, sws, tile_of,
                                 range(0, args.instances, max(1, args.instances // 64)))
    alg_bytes = BYTES_PER_ELEM * elems_iter
    all_pairs = F_TEST * tests_iter / (kern_ms * 1e-3)
    alu = executed * all_pairs
    kname = f"iter_kernel<{tune[0]}>" if tune else "iter_kernel (one launch per bucket)"
    rec = counter_record(kname, tune) if tune else None
    roof = dict(bound="hbm", achieved=alg_bytes / (kern_ms * 1e-3) / 1e9, peak=PEAK_HBM / 1e9,
                unit="GB/s", frac=alg_bytes / (kern_ms * 1e-3) / PEAK_HBM,
                traffic=rec["hbm_bytes"] if rec else None,
                kernel=f"{kname} (fused iteration, tile {tune or tiling})", ms_per_launch=kern_ms,
                elements_per_launch=elems_iter, bytes_per_element=BYTES_PER_ELEM,
                alu=dict(bound="alu", achieved=alu / 1e12, peak=PEAK_FP32 / 1e12, unit="TFLOP/s",
                         frac=alu / PEAK_FP32, tests_per_launch_executed=executed * tests_iter,
                         flop_per_test=F_TEST, tests_per_launch_all_pairs=tests_iter,
                         tests_executed_frac=executed,
                         # the planner's effective rate over every segment x edge
                         # pair of Eq.(13), culled ones included: not a utilisation
                         all_pairs_effective_tflops=all_pairs / 1e12,
                         all_pairs_effective_frac=all_pairs / PEAK_FP32))
    if rec:
        roof["traffic_tb_per_s"] = rec["hbm_bytes"] / (kern_ms * 1e-3) / 1e12
        # VALU issue: wave instructions x 64 lanes against the lane rate behind
        # the FP32 peak (157.3 TFLOP/s / 2 FLOP per FMA lane)
        lanes = rec["valu_insts"] * 64 / (kern_ms * 1e-3)
        roof["alu"]["valu_lane_ops_per_s"] = lanes
        roof["alu"]["valu_util"] = lanes / (PEAK_FP32 / 2)
        # VALU issue against one wave64 instruction per SIMD every 4 cycles
        # (the ceiling without packed FP32), from the counter run's own cycles
        if "valu_issue_ratio" in rec:
            roof["alu"]["valu_issue_ratio"] = rec["valu_issue_ratio"]
        # FP32 FLOP the counters saw (64 per ADD/MUL, 128 per FMA wave instruction)
        if "fp32_flop" in rec:
            roof["alu"]["counter_tflops"] = rec["fp32_flop"] / (kern_ms * 1e-3) / 1e12
            roof["alu"]["counter_frac"] = rec["fp32_flop"] / (kern_ms * 1e-3) / PEAK_FP32

    # paper-shaped single instance (366 map, 30 rectangles, 8 x 170, W = 20)
    spec2 = I.dynamic_map(0)
    sw2 = I.dynamic_swarm(spec2.scale, seed=0)
    pl = sepso.Planner(spec2, sw2)
    tune2 = pl.autotune()
    for _ in range(3):
        pl.plan_frame()
    t1 = time.perf_counter()
    its = []
    nf = 100
    for _ in range(nf):
        its.append(pl.plan_frame()["iters"])
    t2 = time.perf_counter() - t1
    paper = dict(workload="366x366 map, 10 static + 20 moving rectangles, 8 groups x 170 "
                          "particles, 20 waypoints, AT + PI + online HSEF, 50 iterations max",
                 plans_per_s=nf / t2, mean_iters=float(np.mean(its)), frames=nf,
                 paper_context_plans_per_s=67, tune=tune2)
    pl.close()

    out = dict(metric=METRIC, value=plans / dt, unit="plans/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=1e3 * dt / args.steps, higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload=f"batched frame loop: {args.instances} independent dynamic "
                                    "instances (W 8-32, 4-100 rectangles, 32-256 particles/group "
                                    "x 8 groups, maps 128-512), AT + PI + online HSEF, <=50 "
                                    "iterations/frame, one hipGraph per frame",
                           instances=args.instances, tune=tune, tiling=tiling,
                           oracle_matched=parity["matched"] if parity else None),
               cost_parity=parity,
               gpu_frame0=dict(plans_per_s=args.instances / frame0_s,
                               mean_iters=float(np.mean(res0["iters"]))),
               all_pairs_tests_per_s=tests_run / dt, roofline=roof, paper_shaped=paper)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    bp.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
