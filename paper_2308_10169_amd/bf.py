"""Benchmark-function runs in the setups of Sec. "Standard benchmark
functions" (80 particles in 8 groups, D = 30, 1400 iterations, Table hyper8)
and Sec. "Large-scale benchmark functions" (16K particles, D = 1K, 1400
iterations; the paper's Table large_bf reports 23.8 / 30.3 / 29.6 / 30.2 s for
its PyTorch GPU version).  Prints one JSON line per case: wall and device
time of the whole run, the final total best, and the move+evaluate kernel's
HBM bandwidth (20 bytes per swarm element per iteration).

  python -m paper_2308_10169_amd.bf --case large
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--case", choices=sorted(CASES), default="large")
    ap.add_argument("--iters", type=int, default=1400)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    for row in run(args.case, iters=args.iters, seed=args.seed):
        print(json.dumps(row), flush=True)


if __name__ == "__main__":
    main()
