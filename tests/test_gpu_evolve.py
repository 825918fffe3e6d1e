"""Evolution phase on the GPU (sepso_evolve) against the oracle: the higher
level bit-for-bit in its decisions and to FP32 rounding in its positions, the
lower-level runs in distribution, plus the wiring between the two levels."""
import numpy as np
import pytest

from oracle import pyorc as orc
from paper_2308_10169_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    from paper_2308_10169_amd import sepso
    sepso.lib()
    return sepso


def _case(Gl=4, N=24, W=6, T=15):
    spec = I.dynamic_map(4, S=200.0, n_static=3, n_moving=0, side=(15.0, 40.0))
    lsw = I.SwarmSpec(Gl, N, W, T, I.HYPER8[:Gl], alpha=30.0, beta=4, seed=11)
    return spec, lsw


def _pair(sp, Gh=3, Nh=5, E=6, seed=9, **kw):
    spec, lsw = _case(**kw)
    g = sp.Evolver(spec, lsw, Gh, Nh, E, seed=seed)
    o = orc.Evolve(spec, lsw, Gh, Nh, E, seed=seed)
    return g, o


def _close(a, b, span, tol=2e-6):
    assert np.max(np.abs(a - b) / span) <= tol, np.max(np.abs(a - b) / span)


def test_init_matches_oracle(sp):
    g, o = _pair(sp)
    st = g.get_state()
    span = np.tile(o.hi - o.lo, o.Dh // 6)
    _close(st["X"], o.X, span)
    _close(st["V"], o.V, span)
    assert np.array_equal(st["X"], st["P"]) and np.all(np.isinf(st["Pf"])) and st["k"] == 0
    # the lower level starts from the H positions
    for i in range(g.n):
        assert np.array_equal(g.lower_state(i)["hyper"].reshape(-1), st["X"][i])
    g.close()


def test_injected_steps_match_oracle(sp):
    g, o = _pair(sp, Gh=4, Nh=6, E=5)
    rng = np.random.default_rng(3)
    span = np.tile(o.hi - o.lo, o.Dh // 6)
    for step in range(7):
        lfv = rng.uniform(100, 200, g.n).astype(np.float32)
        lfv[rng.integers(0, g.n, 2)] = np.float32(rng.choice([np.nan, np.inf]))
        if step == 3:
            lfv[:] = np.float32(150.0)  # all tied: nothing improves, lowest indices win
        g.inject(lfv)
        o.step(lfv.astype(np.float64))
        st = g.get_state()
        assert np.array_equal(st["Pf"], o.Pf.astype(np.float32))
        assert np.array_equal(st["gbest_n"], o.gbest_n)
        assert st["tbest"][:2] == o.tbest[:2] and st["tbest"][2] == np.float32(o.tbest[2])
        assert st["k"] == o.k and st["ctr"] == o.ctr
        tol = 2e-6 * (step + 1)
        _close(st["X"], o.X, span, tol)
        _close(st["V"], o.V, span, tol)
        _close(st["P"], o.P, span, tol)
    g.close()


def test_levels_are_wired(sp):
    spec, lsw = _case()
    g = sp.Evolver(spec, lsw, 2, 4, 4, seed=1)
    curve = g.run(2)
    st = g.get_state()
    assert st["k"] == 2 and np.all(np.diff(curve) <= 0)
    for i in range(g.n):
        ls = g.lower_state(i)
        assert ls["frame"] == 2 and ls["k"] == lsw.max_iters
        assert ls["tbest"][2] == st["lfv"][i]          # fitness = the lower run's LFV
        assert np.array_equal(ls["hyper"].reshape(-1), st["X"][i])  # next run's hyper
    hyper, f = g.best()
    tg, tn, tf = st["tbest"]
    assert f == tf == curve[-1] and np.array_equal(hyper.reshape(-1), st["P"][tg * 4 + tn])
    # a new tile plan re-captures the evolution graph
    g.set_tune(8, 64)
    g.run(1)
    assert g.get_state()["k"] == 3
    g.close()


def test_evolution_distribution_matches_oracle(sp):
    g, o = _pair(sp, Gh=4, Nh=4, E=4)
    gl, ol = [], []
    for _ in range(4):
        g.run(1)
        gl.append(g.get_state()["lfv"].copy())
        o.evolve(1, hyper_cast=lambda x: x.astype(np.float32).astype(np.float64))
        ol.append(np.array([sw.s.tbest_f for sw in o.lower]))
    gl, ol = np.array(gl), np.array(ol)
    print("median LFV", np.median(gl), np.median(ol), "best", gl.min(), ol.min())
    assert np.all(np.isfinite(gl))
    assert abs(np.median(gl) - np.median(ol)) <= 0.02 * np.median(ol)
    assert abs(gl.min() - ol.min()) <= 0.02 * ol.min()


def test_bad_config_rejected(sp):
    spec, lsw = _case()
    with pytest.raises(sp.SepsoError):
        sp.Evolver(spec, lsw, 65, 1, 4)
    with pytest.raises(sp.SepsoError):
        sp.Evolver(spec, lsw, 8, 129, 4)   # 1032 H particles > 1024
    with pytest.raises(sp.SepsoError):
        sp.Evolver(spec, lsw, 2, 2, 4, lo=np.ones(6), hi=np.ones(6))
