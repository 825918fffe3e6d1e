"""Learned initializer workflow on the GPU: the planner generates its own
training set (converged group bests on random single-plan maps), the MLP is
trained by the library's BF16 MFMA kernels, and the trained network is
compared with the plain planner on held-out maps.

  python -m paper_2308_10169_amd.learned --samples 32768 --steps 2000

Every step runs in libsepso; this module only drives it.
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
from paper_2308_10169_amd import sepso  # noqa: E402


def plan_set(maps, seed_base, lin=None, iters=50, tune=(12, 256)):
    """Plan one frame of every map (optionally with learned proposals);
    returns (costs, Tbest history (n, iters), batch planner)."""
    sws = [I.learned_swarm(seed=seed_base, instance=i, iters=iters) for i in range(len(maps))]
    bp = sepso.BatchPlanner(maps, sws, tune=tune)
    if lin is not None:
        bp.attach(lin)
    r = bp.plan(1)
    return r["cost"][0], bp.history()[:, :iters], bp


def generate(lin, n_samples, seed=1, chunk=4096):
    """Fill lin's training set with n_samples planner results."""
    done = 0
    while done < n_samples:
        n = min(chunk, n_samples - done)
        maps = I.random_static_maps(n, seed=seed * 1000003 + done)
        _, _, bp = plan_set(maps, seed_base=seed + done)
        lin.collect(bp)
        bp.close()
        done += n
    return lin.samples()


def iters_to_reach(hist, target):
    """First iteration (1-based) whose Tbest fitness is <= target, or
    len+1 when never reached."""
    hit = hist <= target[:, None] * (1 + 1e-6)
    first = np.where(hit.any(axis=1), hit.argmax(axis=1) + 1, hist.shape[1] + 1)
    return first


def evaluate(lin, n_maps=512, seed=2_000_000, iters=50):
    """Held-out comparison: iterations the learned start needs to reach the
    plain planner's final cost, against the plain planner's own."""
    maps = I.random_static_maps(n_maps, seed=seed)
    c_plain, h_plain, bp = plan_set(maps, seed_base=seed, iters=iters)
    bp.close()
    c_lin, h_lin, bp = plan_set(maps, seed_base=seed, lin=lin, iters=iters)
    bp.close()
    it_plain = iters_to_reach(h_plain, c_plain)
    it_lin = iters_to_reach(h_lin, c_plain)
    return dict(maps=n_maps, median_iters_plain=float(np.median(it_plain)),
                median_iters_learned=float(np.median(it_lin)),
                mean_iters_plain=float(np.mean(it_plain)), mean_iters_learned=float(np.mean(it_lin)),
                frac_learned_faster=float(np.mean(it_lin < it_plain)),
                median_cost_plain=float(np.median(c_plain)),
                median_cost_learned=float(np.median(c_lin)),
                first_iter_cost_plain=float(np.median(h_plain[:, 0])),
                first_iter_cost_learned=float(np.median(h_lin[:, 0])))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=32768)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--heldout", type=int, default=512)
    ap.add_argument("--out", default=None, help="write trained weights (.npy) here")
    args = ap.parse_args()
    lin = sepso.LearnedInit(max_rows=4096, max_samples=args.samples, seed=0)
    t0 = time.perf_counter()
    n = generate(lin, args.samples)
    t1 = time.perf_counter()
    loss = lin.train(args.steps, args.batch, args.lr)
    t2 = time.perf_counter()
    ev = evaluate(lin, n_maps=args.heldout)
    if args.out:
        np.save(args.out, lin.get_weights())
    print(json.dumps(dict(samples=n, gen_s=t1 - t0, train_s=t2 - t1, steps=args.steps,
                          loss_first=float(loss[:10].mean()), loss_last=float(loss[-10:].mean()),
                          **ev)), flush=True)


if __name__ == "__main__":
    main()
