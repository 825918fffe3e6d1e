"""Ablation of the application-phase mechanisms in the shape of Table ppresult:
SEPSO (evolved hyper-parameters + Priori Initialization + Auto Truncation),
SEPSO without AT, SEPSO without PI, and DTPSO (unevolved hyper-parameters),
on a paper-shaped dynamic scene (366 x 366, 2 static + 6 moving obstacles,
8 groups x 170 particles, 8 waypoints, alpha = 30, beta = 4, gamma = 0.25,
delta = 10, TW = 20, a 30-iteration cap), once with the truncation window
taken literally and once with a window that grows from two values.  The paper's own layout is not
available, so the numbers are not comparable with its table -- only the
direction of each mechanism's effect is.

  python -m paper_2308_10169_amd.ablation --frames 100
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

CAP = 30  # iteration cap of the variants without truncation (Sec. Experiments)


def scene(seed=0):
    return I.dynamic_map(seed, S=366.0, n_static=2, n_moving=6, side=(20.0, 60.0), vmax=2.0)


def variant_swarm(name, S, seed=0, particles=170, waypoints=8, at_mode=1):
    """at_mode 1 is the paper's window rule taken literally (std over the last
    TW values once TW exist); 3 lets the window grow from two values."""
    pp = I.PARAMS_PATH
    evolved = I.HYPER8PATH
    base = dict(alpha=pp["alpha"], beta=pp["beta"], seed=seed, pi_gamma=pp["gamma"],
                pi_radius=0.05 * S, at_window=pp["tw"], at_delta=pp["delta"])
    online = dict(hsef_every=10, hsef_hyper=I.HYPER8)
    if name == "SEPSO":
        return I.SwarmSpec(8, particles, waypoints, CAP, evolved, use_pi=1, at_mode=at_mode, **online, **base)
    if name == "SEPSO(NoAT)":
        return I.SwarmSpec(8, particles, waypoints, CAP, evolved, use_pi=1, at_mode=0, **online, **base)
    if name == "SEPSO(NoPI)":
        return I.SwarmSpec(8, particles, waypoints, CAP, evolved, use_pi=0, at_mode=at_mode, **online, **base)
    if name == "DTPSO":
        return I.SwarmSpec(8, particles, waypoints, CAP, I.HYPER8, use_pi=0, at_mode=0, **base)
    raise ValueError(name)


VARIANTS = ("SEPSO", "SEPSO(NoAT)", "SEPSO(NoPI)", "DTPSO")


def run_variant(name, frames=100, seed=0, particles=170, waypoints=8, tune=(4, 64), at_mode=1):
    """Per-frame results of one variant on the scene of `seed`."""
    from paper_2308_10169_amd import sepso
    spec = scene(seed)
    sw = variant_swarm(name, spec.scale, seed, particles, waypoints, at_mode)
    pl = sepso.Planner(spec, sw)
    if tune is not None:
        pl.set_tune(*tune)
    out = dict(length=[], iters=[], device_ms=[], crossings=[])
    t0 = time.perf_counter()
    for _ in range(frames):
        r = pl.plan_frame()
        for k in out:
            out[k].append(r[k])
    out["wall_s"] = time.perf_counter() - t0
    pl.close()
    return out


def run(frames=100, seed=0, particles=170, waypoints=8, tune=(4, 64), at_mode=1):
    """Table ppresult rows: means over `frames` consecutive frames."""
    rows = {}
    for name in VARIANTS:
        r = run_variant(name, frames, seed, particles, waypoints, tune, at_mode)
        rows[name] = dict(path_length=float(np.mean(r["length"])),
                          iters_per_frame=float(np.mean(r["iters"])),
                          device_ms_per_frame=float(np.mean(r["device_ms"])),
                          plans_per_s=frames / r["wall_s"],
                          collision_free_frames=float(np.mean(np.asarray(r["crossings"]) == 0)))
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--frames", type=int, default=100)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    for mode in (1, 3):
        print(json.dumps(dict(at_mode=mode, rows=run(args.frames, args.seed, at_mode=mode))),
              flush=True)


if __name__ == "__main__":
    main()
