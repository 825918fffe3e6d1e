"""Pins of the oracle's evolution phase (H-SEPSO over lower-level hyper
matrices, Sec. "Hierarchical Self-evolving Framework", Eq.(9), with the
move of Eq.(6)-(8)) -- CPU only, closed forms of special hyper-parameters."""
import numpy as np
import pytest

from paper_2308_10169_amd import inputs as I


def _evolve(orc, Gh=2, Nh=3, E=4, seed=5, h_hyper=None):
    spec = I.dynamic_map(0, S=128.0, n_static=2, n_moving=2, side=(10.0, 30.0))
    lsw = I.SwarmSpec(2, 8, 4, 6, I.HYPER8[:2], alpha=30.0, beta=4)
    return orc.Evolve(spec, lsw, Gh, Nh, E, seed=seed, h_hyper=h_hyper)


def _row(C1, C2, C3, wi, we, vl):
    return [C1, C2, C3, wi, we, vl]


def test_init_in_box(orc):
    e = _evolve(orc, Gh=8, Nh=16)
    lo, hi = np.tile(e.lo, e.Dh // 6), np.tile(e.hi, e.Dh // 6)
    assert np.all(e.X >= lo) and np.all(e.X <= hi)
    assert np.array_equal(e.X, e.P) and np.all(np.isinf(e.Pf))
    vl = e.h_hyper[np.repeat(np.arange(8), 16), 5][:, None]
    assert np.all(np.abs(e.V) <= vl * (hi - lo) / 2 + 1e-12)
    # uniform in the box: column means near the centre (n = 128 * 8 per column)
    cols = e.X.reshape(-1, 6)
    assert np.allclose(cols.mean(0), (e.lo + e.hi) / 2, atol=0.08 * (e.hi - e.lo))


def test_pure_inertia_closed_form(orc):
    # C = 0, w = 1: X_k = clamp(X_0 + k V_0) (V never clipped: |V_0| <= vmax)
    e = _evolve(orc, h_hyper=np.array([_row(0, 0, 0, 1, 1, 1)] * 2))
    X0, V0 = e.X.copy(), e.V.copy()
    lo, hi = np.tile(e.lo, e.Dh // 6), np.tile(e.hi, e.Dh // 6)
    rng = np.random.default_rng(0)
    for k in range(1, 7):
        e.step(rng.uniform(100, 200, len(X0)))
        assert np.allclose(e.X, np.clip(X0 + k * V0, lo, hi), atol=1e-12)
        assert np.array_equal(e.V, V0)


def test_inertia_schedule(orc):
    # C = 0, w_init = 1, w_end = 0 over E = 4: V_k = (1 - k/4) V_{k-1}; w stays 0 past E
    e = _evolve(orc, E=4, h_hyper=np.array([_row(0, 0, 0, 1, 0, 1)] * 2))
    V = e.V.copy()
    for k in range(1, 7):
        e.step(np.full(6, 1.0))
        V = V * max(0.0, 1 - k / 4)
        assert np.allclose(e.V, V, atol=1e-15)


def _attractor_case(orc, which):
    # step 1 (pure inertia) moves X off P = X_0; step 2 with one attractor,
    # w = 0 and no Pbest change: X_2 - X_1 = r (A - X_1) with one r per particle
    inert, pull = _row(0, 0, 0, 1, 1, 1), [0.0] * 6
    pull[which], pull[5] = 1.0, 1.0
    e = _evolve(orc, Gh=2, Nh=3, h_hyper=np.array([inert] * 2))
    lfv = np.array([5.0, 3.0, 4.0, 2.0, 6.0, 7.0])  # group bests: n=1 (3.0), n=0 (2.0)
    e.step(lfv)
    assert np.array_equal(e.Pf, lfv) and list(e.gbest_n) == [1, 0]
    assert e.tbest[:2] == (1, 0) and e.tbest[2] == 2.0
    P, X1 = e.P.copy(), e.X.copy()
    e.h_hyper[:] = np.array([pull] * 2)
    e.step(np.full(6, np.inf))  # nothing improves
    assert np.array_equal(e.P, P)
    lo, hi = np.tile(e.lo, e.Dh // 6), np.tile(e.hi, e.Dh // 6)
    ratios = []
    for i in range(6):
        g = i // 3
        A = {0: P[i], 1: P[3 * g + e.gbest_n[g]], 2: P[3 * 1 + 0]}[which]
        d = A - X1[i]
        # velocity and box clips aside
        m = (np.abs(d) > 1e-9) & (e.X[i] > lo) & (e.X[i] < hi) & (np.abs(e.V[i]) < (hi - lo) / 2)
        r = (e.X[i] - X1[i])[m] / d[m]
        assert np.allclose(r, r[0], atol=1e-9) and 0.0 <= r[0] < 1.0
        ratios.append(r[0])
    return np.array(ratios)


@pytest.mark.parametrize("which", [0, 1, 2])
def test_single_attractor(orc, which):
    r = _attractor_case(orc, which)
    assert len(set(np.round(r, 12))) == len(r)  # independent factor per particle


def test_attractors_use_distinct_random_factors(orc):
    a, b, c = (_attractor_case(orc, w) for w in range(3))
    assert not np.allclose(a, b) and not np.allclose(b, c)


def test_velocity_clip(orc):
    e = _evolve(orc, h_hyper=np.array([_row(3, 3, 3, 1, 1, 0.01)] * 2))
    e.step(np.arange(6, dtype=float))
    e.step(np.arange(6, dtype=float)[::-1])
    lim = np.tile(0.01 * (e.hi - e.lo) / 2, e.Dh // 6)
    assert np.all(np.abs(e.V) <= lim * (1 + 1e-12))
    assert np.any(np.isclose(np.abs(e.V), lim))


def test_bests_running_min_and_ties(orc):
    e = _evolve(orc, Gh=2, Nh=3)
    rng = np.random.default_rng(1)
    best = np.full(6, np.inf)
    for _ in range(5):
        lfv = rng.integers(0, 4, 6).astype(float)  # many ties
        lfv[rng.integers(0, 6)] = np.nan           # non-finite counts as +inf
        e.step(lfv)
        best = np.minimum(best, np.where(np.isfinite(lfv), lfv, np.inf))
        assert np.array_equal(e.Pf, best)
        for g in range(2):
            grp = best[3 * g:3 * g + 3]
            assert e.gbest_n[g] == int(np.argmin(grp)) and e.gbest_f[g] == grp.min()
        tg = int(np.argmin(e.gbest_f))
        assert e.tbest == (tg, e.gbest_n[tg], e.gbest_f[tg])


def test_evolution_curve_and_lower_level(orc):
    e = _evolve(orc, Gh=2, Nh=2, E=3)
    spec = I.dynamic_map(0, S=128.0, n_static=2, n_moving=2, side=(10.0, 30.0))
    straight = np.hypot(*(spec.target - spec.start))
    curve = e.evolve(3)
    assert np.all(np.diff(curve) <= 0)          # total best never worsens
    assert np.all(curve >= straight - 1e-9)     # no path is shorter than the chord
    assert e.k == 3 and e.ctr == 3
    # every lower-level run used the H particle's values as its hyper matrix
    for i, sw in enumerate(e.lower):
        assert sw.s.k > 0
