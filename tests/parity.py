"""Helpers shared by the GPU parity tests: inject the HIP path's state into
the FP64 oracle, run the oracle's version of the same iteration and compare.

Tolerances (stated once, used everywhere):
  * crossing counts: bit-exact when the oracle flags no degenerate test for
    the path (|orientation| < 1e-6 * S^2); otherwise Q_gpu lies in
    [q_yes, q_yes + n_deg];
  * fitness / length: |d| <= 1e-5 * max(|ref|, 1) where Q agrees;
  * positions and velocities: |d| <= 1e-5 * max(|ref|, S).
"""
import numpy as np

from oracle import pyorc as orc

REL = 1e-5


def load_oracle(o, st):
    """Copy a GPU state dict (FP32) into oracle swarm `o` (FP64, exact)."""
    for k in ("X", "V", "P", "f", "L", "Pf", "PL"):
        getattr(o, k)[...] = st[k].astype(np.float64)
    o.Q[...] = st["Q"]
    o.PQ[...] = st["PQ"]
    o.gbest_n[...] = st["gbest_n"]
    o.gbest_f[...] = st["gbest_f"].astype(np.float64)
    o.hyper[...] = st["hyper"].astype(np.float64)
    o.set_scalars(k=st["k"], ctr=st["ctr"], tbest=st["tbest"])


def check_fitness(m, st_before, st_after, W, alpha, beta, stats=None):
    """f/L/Q of the GPU (st_after) against the oracle on st_before's X."""
    G, N, D = st_before["X"].shape
    r = orc.fitness(m, st_before["X"].reshape(-1, D).astype(np.float64), W, alpha, beta)
    qg = st_after["Q"].reshape(-1)
    lo, hi = r["q_yes"], r["q_yes"] + r["n_deg"]
    assert np.all(qg >= lo) and np.all(qg <= hi), "crossing count outside the oracle's bracket"
    clean = r["n_deg"] == 0
    assert np.array_equal(qg[clean], r["Q"][clean]), "crossing count differs on robust paths"
    agree = qg == r["Q"]
    Lg = st_after["L"].reshape(-1).astype(np.float64)
    assert np.all(np.abs(Lg - r["L"]) <= REL * np.maximum(np.abs(r["L"]), 1.0))
    fg = st_after["f"].reshape(-1).astype(np.float64)
    assert np.all(np.abs(fg[agree] - r["f"][agree]) <= REL * np.maximum(np.abs(r["f"][agree]), 1.0))
    if stats is not None:
        stats["paths"] = stats.get("paths", 0) + len(qg)
        stats["degenerate_paths"] = stats.get("degenerate_paths", 0) + int((~clean).sum())
        stats["q_differs"] = stats.get("q_differs", 0) + int((~agree).sum())
    return r


def check_step(o, m, st0, st1, S, stats=None):
    """One full iteration: GPU st0 -> st1 versus oracle from st0.

    The oracle evaluates the fitness itself (checked against the GPU's), then
    takes the GPU's FP32 fitness values for the best-tracking so that both
    sides make the same comparisons on the same numbers, and finally applies
    its own FP64 velocity/position update."""
    W = o.W
    check_fitness(m, st0, st1, W, o.sw.alpha, o.sw.beta, stats)
    load_oracle(o, st0)
    o.s.k = st0["k"] + 1
    o.f[...] = st1["f"].astype(np.float64)
    o.L[...] = st1["L"].astype(np.float64)
    o.Q[...] = st1["Q"]
    o.bests()
    assert np.array_equal(o.Pf.astype(np.float32), st1["Pf"]), "Pbest fitness"
    assert np.array_equal(o.PQ, st1["PQ"])
    assert np.array_equal(o.gbest_n, st1["gbest_n"]), "group best index"
    assert np.array_equal(o.gbest_f.astype(np.float32), st1["gbest_f"])
    assert (o.s.tbest_g, o.s.tbest_n) == tuple(st1["tbest"][:2]), "total best index"
    o.update()
    o.s.ctr += 1
    tolX = REL * np.maximum(np.abs(o.X), S)
    tolV = REL * np.maximum(np.abs(o.V), S)
    dX = np.abs(st1["X"] - o.X)
    dV = np.abs(st1["V"] - o.V)
    assert np.all(dX <= tolX), f"positions differ: max {dX.max()}"
    assert np.all(dV <= tolV), f"velocities differ: max {dV.max()}"
    # Pbest positions: those that improved this iteration equal st0's X
    assert np.array_equal(st1["P"], o.P.astype(np.float32)), "Pbest positions"
    assert st1["k"] == o.s.k and st1["ctr"] == o.s.ctr


def check_frame_step(o, m, st0, st1, out0, out1, S, sample, hsef):
    """One iteration of a frame (sepso_step_frame) of a large swarm, from the
    GPU state st0 (outer-swarm state out0) to st1 / out1: the fitness of the
    sampled particles against the oracle's; then, for every particle, the
    oracle's bests on the GPU's FP32 fitness values, its online outer step
    when one is due (Sec. HSEF: after the bests, before the update) and its
    FP64 update."""
    W, D = o.W, o.D
    sub = lambda st: dict(X=st["X"].reshape(-1, D)[sample][None], Q=st["Q"].reshape(-1)[sample][None],
                          L=st["L"].reshape(-1)[sample][None], f=st["f"].reshape(-1)[sample][None])
    check_fitness(m, sub(st0), sub(st1), W, o.sw.alpha, o.sw.beta)
    load_oracle(o, st0)
    o.s.k = st0["k"] + 1
    o.f[...] = st1["f"].astype(np.float64)
    o.L[...] = st1["L"].astype(np.float64)
    o.Q[...] = st1["Q"]
    o.bests()
    assert np.array_equal(o.Pf.astype(np.float32), st1["Pf"]), "Pbest fitness"
    assert np.array_equal(o.gbest_n, st1["gbest_n"]), "group best index"
    assert (o.s.tbest_g, o.s.tbest_n) == tuple(st1["tbest"][:2]), "total best index"
    if hsef:
        o.ov[...] = out0["ov"].astype(np.float64)
        o.op[...] = out0["op"].astype(np.float64)
        o.opf[...] = out0["opf"].astype(np.float64)
        o.h.otb, o.h.epoch_in_frame, o.h.epoch_ctr = out0["otb"], out0["epoch_in_frame"], out0["epoch_ctr"]
        o.hsef_step()
        assert o.h.otb == out1["otb"] and o.h.epoch_in_frame == out1["epoch_in_frame"]
        assert o.h.epoch_ctr == out1["epoch_ctr"]
        assert np.array_equal(o.opf.astype(np.float32), out1["opf"]), "outer Pbest fitness"
        assert np.array_equal(o.op.astype(np.float32), out1["op"]), "outer Pbest positions"
        assert np.allclose(out1["ov"], o.ov, rtol=0, atol=1e-5), "outer velocities"
        assert np.allclose(st1["hyper"], o.hyper, rtol=0, atol=1e-5), "evolved hyper-parameters"
        assert not np.array_equal(st1["hyper"], st0["hyper"]), "the outer step moved nothing"
    else:
        assert np.array_equal(st1["hyper"], st0["hyper"])
    o.update()
    o.s.ctr += 1
    dX = np.abs(st1["X"] - o.X)
    dV = np.abs(st1["V"] - o.V)
    assert np.all(dX <= REL * np.maximum(np.abs(o.X), S)), f"positions differ: max {dX.max()}"
    assert np.all(dV <= REL * np.maximum(np.abs(o.V), S)), f"velocities differ: max {dV.max()}"
    assert np.array_equal(st1["P"], o.P.astype(np.float32)), "Pbest positions"
    assert st1["k"] == o.s.k and st1["ctr"] == o.s.ctr
