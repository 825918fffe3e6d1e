"""Benchmark-function runs in the setups of Sec. "Standard benchmark
functions" (80 particles in 8 groups, D = 30, 1400 iterations, Table hyper8)
and Sec. "Large-scale benchmark functions" (16K particles, D = 1K, 1400
iterations; the paper's Table large_bf reports 23.8 / 30.3 / 29.6 / 30.2 s for
its PyTorch GPU version).  Prints one JSON line per case: wall and device
time of the whole run, the final total best, and the move+evaluate kernel's
HBM bandwidth (20 bytes per swarm element per iteration).

  python -m paper_2308_10169_amd.bf --case large

With --evolve: the evolution phase of Sec. "Evolution Phase on Benchmark
Functions" (H-SEPSO with Table hyper8 over the lower level's (8, 6) hyper
matrix, each H particle's fitness the LFV of a fresh 80-particle, 30-dimension,
1400-iteration run), then the application phase: the best matrix found
against Table hyper8 over independent 1400-iteration trials.

  python -m paper_2308_10169_amd.bf --evolve --evolutions 500
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2308_10169_amd import inputs as I  # noqa: E402

PAPER_LARGE_GPU_S = {"sphere": 23.8, "rosenbrock": 30.3, "rastrigin": 29.6, "griewank": 30.2}
CASES = {"standard": (8, 10, 30), "large": (8, 2048, 1000)}
BYTES_PER_ELEM = 20  # X, V, P read; X, V written


def run(case="large", funcs=("sphere", "rosenbrock", "rastrigin", "griewank"), iters=1400,
        seed=0):
    from paper_2308_10169_amd import sepso
    import torch
    G, N, D = CASES[case]
    out = []
    for name in funcs:
        sw = sepso.BFSwarm(name, G, N, D, iters, I.HYPER8, seed=seed)
        sw.profile(5)  # warm-up (clocks, code load); state re-created below
        sw.close()
        sw = sepso.BFSwarm(name, G, N, D, iters, I.HYPER8, seed=seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ms_it = sw.profile(iters)
        wall = time.perf_counter() - t0
        st = sw.get_state(rows=False)
        sw.close()
        elems = G * N * D
        row = dict(case=case, func=name, particles=G * N, dims=D, iters=iters, wall_s=wall,
                   device_s=ms_it * iters / 1e3, ms_per_iter=ms_it, best=float(st["tbest"][2]),
                   hbm_gbs=BYTES_PER_ELEM * elems / (ms_it * 1e-3) / 1e9)
        if case == "large":
            row["paper_gpu_s"] = PAPER_LARGE_GPU_S[name]
            row["speedup_vs_paper"] = PAPER_LARGE_GPU_S[name] / wall
        out.append(row)
    return out


def evolve(funcs=("sphere", "rosenbrock", "rastrigin", "griewank"), evolutions=500, iters=1400,
           h_groups=8, h_particles=4, trials=50, seed=0):
    """Evolution then application phase per function; one JSON row each."""
    from paper_2308_10169_amd import sepso
    import torch
    G, N, D = CASES["standard"]
    out = []
    for name in funcs:
        ev = sepso.BFEvolver(name, G, N, D, iters, h_groups=h_groups, h_particles=h_particles,
                             evolutions=evolutions, seed=seed, h_seed=seed + 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        curve = ev.run(evolutions)
        secs = time.perf_counter() - t0
        hyper, lfv = ev.best()
        ev.close()
        # application phase: independent trials (swarms with their own random
        # streams, a seed apart from the evolution's) of the best matrix and of
        # Table hyper8
        finals = {}
        for tag, h in (("evolved", hyper), ("hyper8", I.HYPER8)):
            sw = sepso.BFSwarm(name, G, N, D, iters, np.tile(np.asarray(h, np.float32), (trials, 1)),
                               seed=seed + 1000, swarms=trials)
            sw.step(iters)
            finals[tag] = sw.swarm_best().astype(np.float64)
            sw.close()
        pick = np.unique(np.round(np.geomspace(1, evolutions, 12)).astype(int)) - 1
        e, h = finals["evolved"], finals["hyper8"]
        # probability that a trial of the evolved matrix ends below one of
        # Table hyper8 (ties count half): the comparison stays meaningful when
        # trials reach the FP32 floor (exactly 0)
        p_lower = float(np.mean((e[:, None] < h[None, :]) + 0.5 * (e[:, None] == h[None, :])))
        out.append(dict(func=name, particles=G * N, dims=D, iters=iters,
                        h_particles=h_groups * h_particles, evolutions=evolutions,
                        evolution_s=secs, ms_per_evolution=1e3 * secs / evolutions,
                        lfv_curve={int(k + 1): float(curve[k]) for k in pick},
                        best_lfv=float(lfv), best_hyper=np.round(hyper, 4).tolist(),
                        trials=trials,
                        median_final_evolved=float(np.median(e)),
                        median_final_hyper8=float(np.median(h)),
                        mean_final_evolved=float(np.mean(e)), mean_final_hyper8=float(np.mean(h)),
                        frac_zero_evolved=float(np.mean(e == 0)),
                        frac_zero_hyper8=float(np.mean(h == 0)),
                        p_evolved_lower=p_lower))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--case", choices=sorted(CASES), default="large")
    ap.add_argument("--iters", type=int, default=1400)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--evolve", action="store_true", help="evolution + application phase")
    ap.add_argument("--evolutions", type=int, default=500)
    ap.add_argument("--funcs", default="sphere,rosenbrock,rastrigin,griewank")
    ap.add_argument("--seeds", type=int, default=1, help="--evolve: independent evolutions per function")
    args = ap.parse_args()
    funcs = tuple(args.funcs.split(","))
    if not args.evolve:
        for row in run(args.case, funcs, iters=args.iters, seed=args.seed):
            print(json.dumps(row), flush=True)
        return
    per = {f: [] for f in funcs}
    for sd in range(args.seed, args.seed + args.seeds):
        for row in evolve(funcs, args.evolutions, args.iters, seed=sd):
            row["seed"] = sd
            per[row["func"]].append(row)
            print(json.dumps(row), flush=True)
    if args.seeds > 1:
        for f, rows in per.items():
            p = [r["p_evolved_lower"] for r in rows]
            print(json.dumps(dict(func=f, seeds=len(rows), p_evolved_lower_per_seed=p,
                                  median_p_evolved_lower=float(np.median(p)),
                                  seeds_evolved_better=int(sum(v > 0.5 for v in p)),
                                  median_final_evolved_per_seed=[r["median_final_evolved"] for r in rows],
                                  median_final_hyper8_per_seed=[r["median_final_hyper8"] for r in rows])),
                  flush=True)


if __name__ == "__main__":
    main()
