"""Benchmark-function workload on the GPU (sepso_bf) against the oracle:
initial swarm, one injected iteration per function (fitness, bests, move) at
ragged and multi-chunk row lengths and at the paper's large shape, and the
descent over many iterations."""
import numpy as np
import pytest

from oracle import pyorc as orc
from paper_2308_10169_amd import inputs as I

pytestmark = pytest.mark.gpu
FUNCS = (1, 2, 3, 4)


@pytest.fixture(scope="module")
def sp():
    from paper_2308_10169_amd import sepso
    sepso.lib()
    return sepso


def _hyper(G):
    return I.HYPER8[np.arange(G) % 8]


def test_init_matches_oracle(sp):
    g = sp.BFSwarm(1, 3, 7, 30, 100, _hyper(3), seed=5)
    o = orc.BFSwarm(1, 3, 7, 30, 100, _hyper(3), seed=5)
    st = g.get_state()
    assert np.max(np.abs(st["X"] - o.X)) <= 1200 * 2 ** -23
    assert np.max(np.abs(st["V"] - o.V)) <= 1200 * 2 ** -23
    assert np.array_equal(st["X"], st["P"]) and st["k"] == 0 and st["pending"] == 0
    g.close()


def _inject_step(sp, func, G, N, D, warm, seed=1, tol=1e-5):
    g = sp.BFSwarm(func, G, N, D, 50, _hyper(G), seed=seed)
    g.step(warm)
    st0 = g.get_state()
    g.step(1)
    st1 = g.get_state()
    o = orc.BFSwarm(func, G, N, D, 50, _hyper(G), seed=seed)
    for k in ("X", "V", "P", "Pf", "gbest_f"):
        getattr(o, k)[...] = st0[k].astype(np.float64)
    o.gbest_n[...] = st0["gbest_n"]
    o.set_scalars(k=st0["k"] + 1, ctr=st0["ctr"])
    o.eval()
    f_ref = o.f.copy()
    fg = st1["f"].astype(np.float64)
    scale = np.maximum(np.abs(f_ref), 1.0) + 1e-6 * D
    assert np.all(np.abs(fg - f_ref) <= tol * scale), np.max(np.abs(fg - f_ref) / scale)
    o.f[...] = fg  # same comparisons on the same numbers
    o.advance()
    assert np.array_equal(st1["Pf"], o.Pf.astype(np.float32))
    assert np.array_equal(st1["gbest_n"], o.gbest_n)
    assert st1["tbest"][:2] == o.tbest[:2]
    assert st1["k"] == o.k and st1["ctr"] == o.ctr
    for k in ("X", "V", "P"):
        d = np.abs(st1[k] - getattr(o, k))
        assert np.max(d) <= 2e-4, (k, np.max(d))   # 1.7e-7 of the 1200-wide box
    g.close()


@pytest.mark.parametrize("func", FUNCS)
@pytest.mark.parametrize("D", [30, 300])
def test_injected_step(sp, func, D):
    # D = 30: one partial chunk (padded to 32); D = 300: a full 256-element
    # chunk plus a ragged one (Rosenbrock's pair across the chunk seam)
    _inject_step(sp, func, 3, 9, D, warm=3)


@pytest.mark.parametrize("func", [1, 3])
def test_injected_step_large_shape(sp, func):
    # the paper's large case: 16K particles (8 x 2048) x 1K dimensions
    _inject_step(sp, func, 8, 2048, 1000, warm=2)


@pytest.mark.parametrize("func", FUNCS)
def test_descent_matches_oracle(sp, func):
    # 80 particles x 30 dims for 300 iterations, 4 seeds: the total best
    # falls like the oracle's (chaotic runs, so medians in log space)
    lg, lo = [], []
    for seed in range(4):
        g = sp.BFSwarm(func, 8, 10, 30, 300, I.HYPER8, seed=seed)
        g.step(300)
        lg.append(np.log10(max(g.get_state(rows=False)["tbest"][2], 1e-30)))
        g.close()
        o = orc.BFSwarm(func, 8, 10, 30, 300, I.HYPER8, seed=seed)
        o.step(300)
        lo.append(np.log10(max(o.tbest[2], 1e-30)))
        f0 = orc.BFSwarm(func, 8, 10, 30, 300, I.HYPER8, seed=seed)
        f0.step(1)
        assert o.tbest[2] < f0.tbest[2]
    print(func, np.median(lg), np.median(lo))
    assert abs(np.median(lg) - np.median(lo)) <= 0.5


def test_multi_swarm_init_matches_oracle(sp):
    # S independent swarms side by side: swarm s draws as the oracle's
    # instance s
    S, G, N, D = 3, 2, 5, 30
    hy = np.tile(_hyper(G), (S, 1))
    g = sp.BFSwarm(4, G, N, D, 50, hy, seed=8, swarms=S)
    st = g.get_state()
    for s in range(S):
        o = orc.BFSwarm(4, G, N, D, 50, _hyper(G), seed=8, instance=s)
        sl = slice(s * G, (s + 1) * G)
        assert np.max(np.abs(st["X"][sl] - o.X)) <= 1200 * 2 ** -23
        assert np.max(np.abs(st["V"][sl] - o.V)) <= 1200 * 2 ** -23
    g.close()


@pytest.mark.parametrize("func", [2, 3])
def test_multi_swarm_injected_step(sp, func):
    # one iteration of every swarm from the GPU's state: fitness, bests, and
    # each swarm's move toward its own Tbest
    S, G, N, D = 4, 3, 6, 40
    hy = np.concatenate([_hyper(8)[(np.arange(G) + s) % 8] for s in range(S)])
    g = sp.BFSwarm(func, G, N, D, 50, hy, seed=2, swarms=S)
    g.step(3)
    st0 = g.get_state()
    g.step(1)
    st1 = g.get_state()
    for s in range(S):
        sl = slice(s * G, (s + 1) * G)
        o = orc.BFSwarm(func, G, N, D, 50, hy[sl], seed=2, instance=s)
        for k in ("X", "V", "P", "Pf", "gbest_f"):
            getattr(o, k)[...] = st0[k][sl].astype(np.float64)
        o.gbest_n[...] = st0["gbest_n"][sl]
        o.set_scalars(k=st0["k"] + 1, ctr=st0["ctr"])
        o.eval()
        fg = st1["f"][sl].astype(np.float64)
        scale = np.maximum(np.abs(o.f), 1.0) + 1e-6 * D
        assert np.all(np.abs(fg - o.f) <= 1e-5 * scale)
        o.f[...] = fg
        o.advance()
        assert np.array_equal(st1["Pf"][sl], o.Pf.astype(np.float32))
        assert np.array_equal(st1["gbest_n"][sl], o.gbest_n)
        for k in ("X", "V", "P"):
            assert np.max(np.abs(st1[k][sl] - getattr(o, k))) <= 2e-4, (s, k)
    assert np.array_equal(g.swarm_best(st1), st1["gbest_f"].reshape(S, G).min(1))
    g.close()


def _same_state(a, b):
    for k in ("X", "V", "P", "f", "Pf", "gbest_n", "gbest_f"):
        assert np.array_equal(a[k], b[k]), k
    assert a["tbest"] == b["tbest"] and a["k"] == b["k"] and a["ctr"] == b["ctr"]
    assert a["pending"] == b["pending"]


@pytest.mark.parametrize("func", FUNCS)
@pytest.mark.parametrize("shape", [(8, 10, 30), (3, 7, 37), (2, 5, 1), (2, 3, 256), (5, 25, 40)])
def test_whole_run_equals_stepwise(sp, func, shape):
    # one workgroup per swarm for a whole call against two launches per
    # iteration: bit-identical state after calls of 60, 1 and 39 iterations
    # (ragged rows: 37 -> 10 float4 groups on 16 lanes; 1; the 256-float row
    # limit; 125 particles of 40 floats: 64 500 bytes of LDS, just under the
    # 64 KiB limit)
    G, N, D = shape
    S = 3
    hy = np.concatenate([_hyper(8)[(np.arange(G) + s) % 8] for s in range(S)])
    a = sp.BFSwarm(func, G, N, D, 100, hy, seed=4, swarms=S)
    b = sp.BFSwarm(func, G, N, D, 100, hy, seed=4, swarms=S, stepwise=True)
    for n in (60, 1, 39):
        a.step(n)
        b.step(n)
        _same_state(a.get_state(), b.get_state())
    a.close()
    b.close()


def test_whole_run_evolution_equals_stepwise(sp):
    ea = sp.BFEvolver(2, 8, 10, 30, 50, h_groups=2, h_particles=3, evolutions=4, seed=1, h_seed=3)
    eb = sp.BFEvolver(2, 8, 10, 30, 50, h_groups=2, h_particles=3, evolutions=4, seed=1, h_seed=3,
                      stepwise=True)
    ca, cb = ea.run(3), eb.run(3)
    assert np.array_equal(ca, cb)
    sa, sb = ea.get_state(), eb.get_state()
    for k in ("X", "V", "P", "Pf", "lfv"):
        assert np.array_equal(sa[k], sb[k]), k
    _same_state(ea.lower.get_state(), eb.lower.get_state())
    ea.close()
    eb.close()
