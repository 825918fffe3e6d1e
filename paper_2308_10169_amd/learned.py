"""Learned initializer workflow on the GPU: the planner generates its own
training set (converged group bests on random single-plan maps), the MLP is
trained by the library's BF16 MFMA kernels, and the trained network is
compared with the plain planner on held-out maps (a uniform first frame) and
on held-out dynamic sequences (plain Priori Initialization from the previous
frame's plan).

  python -m paper_2308_10169_amd.learned --samples 32768 --steps 2000
  python -m paper_2308_10169_amd.learned --samples 16384 --train-only 5 --steps 20 --batch 8192

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


def dynamic_maps(n, seed, vmax=1.0):
    """Held-out dynamic sequences on the training generator's maps: every
    rectangle moves by a constant velocity uniform in +-vmax cells per frame
    (bouncing off the walls), start and target move vertically by half a
    cell per frame; all on the 1/256 grid."""
    maps = I.random_static_maps(n, seed=seed)
    rng = np.random.default_rng(seed + 1)
    for m in maps:
        m.poly_vel = I.snap(rng.uniform(-vmax, vmax, size=(m.n_polys, 2)))
        m.endpoint_vel = I.snap(np.array([0.0, rng.choice([-0.5, 0.5]), 0.0, rng.choice([-0.5, 0.5])]))
    return maps


def evaluate_dynamic(lin, n_maps=256, frames=6, seed=3_000_000, iters=50, tune=(12, 256)):
    """Learned start against plain Priori Initialization on dynamic
    sequences: both planners run every frame to the iteration cap (no Auto
    Truncation); the plain one seeds frames after the first from its
    previous plan, the learned one from the network's proposals for the
    moved map.  Per frame after the first: iterations each needs to reach
    the plain planner's final cost of that frame, and the time to get there
    -- iterations x the measured time per iteration, plus the network's
    inference per frame for the learned start (the difference of the two
    planners' measured frame times)."""
    import torch
    maps = dynamic_maps(n_maps, seed)
    runs = {}
    for tag, use in (("plain", None), ("learned", lin)):
        sws = [I.learned_swarm(seed=seed, instance=i, iters=iters) for i in range(n_maps)]
        for sw in sws:
            sw.use_pi = 1
        bp = sepso.BatchPlanner(maps, sws, tune=tune)
        bp.attach(use)
        bp.plan(1)  # warm-up frame: captures the frame graphs
        bp.close()
        bp = sepso.BatchPlanner(maps, sws, tune=tune)
        bp.attach(use)
        cost, hist, secs = [], [], []
        for _ in range(frames):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = bp.plan(1)
            torch.cuda.synchronize()
            secs.append(time.perf_counter() - t0)
            cost.append(r["cost"][0])
            hist.append(bp.history()[:, :iters])
        bp.close()
        runs[tag] = (np.array(cost), np.array(hist), np.array(secs))
    c_p, h_p, t_p = runs["plain"]
    c_l, h_l, t_l = runs["learned"]
    it_p = np.stack([iters_to_reach(h_p[f], c_p[f]) for f in range(1, frames)])
    it_l = np.stack([iters_to_reach(h_l[f], c_p[f]) for f in range(1, frames)])
    t_iter = float(np.median(t_p[1:])) / iters          # both run `iters` iterations per frame
    t_infer = max(0.0, float(np.median(t_l[1:]) - np.median(t_p[1:])))
    ms_p = 1e3 * t_iter * it_p
    ms_l = 1e3 * (t_infer + t_iter * it_l)
    return dict(maps=n_maps, frames=frames,
                median_iters_plain_pi=float(np.median(it_p)),
                median_iters_learned=float(np.median(it_l)),
                mean_iters_plain_pi=float(np.mean(it_p)), mean_iters_learned=float(np.mean(it_l)),
                frac_learned_fewer_iters=float(np.mean(it_l < it_p)),
                frac_learned_reaches=float(np.mean(it_l <= iters)),
                frame_ms_plain=1e3 * float(np.median(t_p[1:])),
                frame_ms_learned=1e3 * float(np.median(t_l[1:])),
                batch_ms_per_iter=1e3 * t_iter, inference_ms_per_frame=1e3 * t_infer,
                median_ms_to_reach_plain_pi=float(np.median(ms_p)),
                median_ms_to_reach_learned=float(np.median(ms_l)),
                median_cost_plain_pi=float(np.median(c_p[1:])),
                median_cost_learned=float(np.median(c_l[1:])),
                frame0_median_iters_uniform=float(np.median(iters_to_reach(h_p[0], c_p[0]))),
                frame0_median_iters_learned=float(np.median(iters_to_reach(h_l[0], c_p[0]))))


def train_only(args):
    """Training steps alone (the MLP kernels' workload for profiling): fill the
    training set, take warm-up steps, then time `args.steps` steps."""
    import torch
    lin = sepso.LearnedInit(max_rows=max(4096, args.batch), max_samples=args.samples, seed=0)
    n = generate(lin, args.samples, seed=7)
    lin.train(args.train_only, args.batch, args.lr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = lin.train(args.steps, args.batch, args.lr)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(json.dumps(dict(samples=n, batch=args.batch, steps=args.steps, ms_per_step=1e3 * dt / args.steps,
                          loss_last=float(loss[-1]))), flush=True)
    lin.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=32768)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--heldout", type=int, default=512)
    ap.add_argument("--dynamic", type=int, default=256, help="held-out dynamic sequences")
    ap.add_argument("--out", default=None, help="write trained weights (.npy) here")
    ap.add_argument("--train-only", type=int, default=0, metavar="W",
                    help="generate, take W warm-up steps, then time --steps training steps only")
    args = ap.parse_args()
    if args.train_only:
        train_only(args)
        return
    lin = sepso.LearnedInit(max_rows=4096, max_samples=args.samples, seed=0)
    t0 = time.perf_counter()
    n = generate(lin, args.samples)
    t1 = time.perf_counter()
    loss = lin.train(args.steps, args.batch, args.lr)
    t2 = time.perf_counter()
    ev = evaluate(lin, n_maps=args.heldout)
    if args.dynamic > 0:
        ev["dynamic"] = evaluate_dynamic(lin, n_maps=args.dynamic)
    if args.out:
        np.save(args.out, lin.get_weights())
    print(json.dumps(dict(samples=n, gen_s=t1 - t0, train_s=t2 - t1, steps=args.steps,
                          loss_first=float(loss[:10].mean()), loss_last=float(loss[-10:].mean()),
                          **ev)), flush=True)


if __name__ == "__main__":
    main()
