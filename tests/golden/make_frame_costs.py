"""Writes frame_costs_dynamic366.txt: the FP64 oracle's frame loop on the
paper-shaped dynamic run (366 x 366 map, 10 static + 20 moving rectangles,
8 groups x 170 particles, 20 waypoints, Priori Initialization, Auto
Truncation mode 2, online self-evolution every 10 iterations, at most 50
iterations per frame), seeds 0-99, frames 0-2 (obstacles and endpoints moved
by the oracle's own motion model between frames).  Calls only the oracle and
the seeded input generators.  Run: python tests/golden/make_frame_costs.py"""
import multiprocessing
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "frame_costs_dynamic366.txt")
SEEDS, FRAMES = 100, 3


def plan(seed):
    from oracle import pyorc as orc
    from paper_2308_10169_amd import inputs as I
    spec = I.dynamic_map(seed)
    sw = I.dynamic_swarm(spec.scale, seed=seed)
    o = orc.Swarm(sw, spec.width, spec.height)
    ref = spec.copy()
    rows = []
    for f in range(FRAMES):
        if f > 0:
            orc.sim_step(ref)
        r = o.plan_frame(orc.Map(ref), f)
        rows.append((seed, f, r["cost"], r["iters"], r["crossings"]))
    return rows


def main():
    procs = max(1, min(16, len(os.sched_getaffinity(0))))
    with multiprocessing.get_context("spawn").Pool(procs) as pool:
        res = pool.map(plan, range(SEEDS))
    with open(OUT, "w") as f:
        f.write("# FP64 oracle frame loop, paper-shaped dynamic run (366 map, 30 rectangles, 8 x 170,\n"
                "# W = 20, PI + AT mode 2 + online HSEF every 10, <= 50 iterations); written by\n"
                "# make_frame_costs.py.  columns: seed frame cost iterations crossings\n")
        for rows in res:
            for s, fr, c, it, q in rows:
                f.write(f"{s} {fr} {c!r} {it} {q}\n")


if __name__ == "__main__":
    main()
