"""Pins of the oracle's benchmark-function workload (Table BFs with DTPSO,
Algorithm 1 / Eq.(6)-(8)) -- CPU only: textbook values of the four
functions and closed forms of the swarm under special hyper-parameters."""
import numpy as np
import pytest

from paper_2308_10169_amd import inputs as I


def test_function_values(orc):
    D = 30
    z, one = np.zeros(D), np.ones(D)
    assert orc.bf_value(orc.BF_SPHERE, z) == 0.0
    assert orc.bf_value(orc.BF_SPHERE, 3 * one) == 9.0 * D
    assert orc.bf_value(orc.BF_ROSENBROCK, one) == 0.0
    assert orc.bf_value(orc.BF_ROSENBROCK, z) == D - 1          # (1 - 0)^2 per term
    assert orc.bf_value(orc.BF_ROSENBROCK, np.array([2.0, 4.0])) == 1.0
    assert orc.bf_value(orc.BF_ROSENBROCK, np.array([0.0, 1.0])) == 101.0
    assert abs(orc.bf_value(orc.BF_RASTRIGIN, z)) < 1e-12
    ints = np.arange(-3, 3, dtype=float)
    assert abs(orc.bf_value(orc.BF_RASTRIGIN, ints) - np.sum(ints ** 2)) < 1e-9
    assert abs(orc.bf_value(orc.BF_RASTRIGIN, 0.5 * one) - D * 20.25) < 1e-9
    assert abs(orc.bf_value(orc.BF_GRIEWANK, z)) < 1e-15
    assert abs(orc.bf_value(orc.BF_GRIEWANK, np.array([np.pi])) - (2 + np.pi ** 2 / 4000)) < 1e-15
    # second coordinate scaled by 1/sqrt(2): cos(pi*sqrt(2)/sqrt(2)) = -1
    x = np.array([0.0, np.pi * np.sqrt(2)])
    assert abs(orc.bf_value(orc.BF_GRIEWANK, x) - (1 + 2 * np.pi ** 2 / 4000 + 1)) < 1e-12


def _swarm(orc, func=1, G=2, N=3, D=5, T=4, hyper=None, seed=3):
    h = I.HYPER8[:G] if hyper is None else np.asarray(hyper, float)
    return orc.BFSwarm(func, G, N, D, T, h, seed=seed)


def test_init_in_box(orc):
    s = _swarm(orc, G=8, N=20, D=30)
    assert np.all(np.abs(s.X) <= 600) and np.array_equal(s.X, s.P)
    vmax = s.hyper[:, 5] * 600
    assert np.all(np.abs(s.V) <= vmax[:, None, None])
    assert abs(s.X.mean()) < 20 and s.X.std() > 300   # U(-600, 600): std 346


def test_pure_inertia_and_fitness(orc):
    s = _swarm(orc, hyper=[[0, 0, 0, 1, 1, 1]] * 2)
    X0, V0 = s.X.copy(), s.V.copy()
    for k in range(1, 5):
        Xk = s.X.copy()
        s.step()
        f = np.array([[orc.bf_value(1, Xk[g, n]) for n in range(3)] for g in range(2)])
        assert np.allclose(s.f, f, rtol=1e-15)              # f is the value of the evaluated X
        assert np.allclose(s.X, np.clip(X0 + k * V0, -600, 600), atol=1e-9)


def test_gbest_attractor_ratio(orc):
    # w = 0, only C2: X_new - X = r (Gbest - X), one r per particle
    s = _swarm(orc, hyper=[[0, 1, 0, 0, 0, 1]] * 2, D=8)
    X = s.X.copy()
    s.step()
    for g in range(2):
        gb = s.P[g, s.gbest_n[g]]
        for n in range(3):
            d = gb - X[g, n]
            m = np.abs(d) > 1e-9
            r = (s.X[g, n] - X[g, n])[m] / d[m]
            if m.any():
                assert np.allclose(r, r[0]) and 0 <= r[0] < 1


def test_bests_and_ranking(orc):
    s = _swarm(orc, func=3, G=3, N=4, D=6)
    best = np.full((3, 4), np.inf)
    for _ in range(6):
        Xk = s.X.copy()
        s.step()
        f = np.array([[orc.bf_value(3, Xk[g, n]) for n in range(4)] for g in range(3)])
        best = np.minimum(best, f)
        assert np.allclose(s.Pf, best, rtol=1e-15)
        assert np.array_equal(s.gbest_n, best.argmin(1))
        tg = int(best.min(1).argmin())
        assert s.tbest[0] == tg and s.tbest[2] == best.min()


@pytest.mark.parametrize("func", [1, 2, 3, 4])
def test_swarm_descends(orc, func):
    s = _swarm(orc, func=func, G=8, N=10, D=30, T=300, hyper=I.HYPER8)
    s.step(1)
    f1 = s.tbest[2]
    s.step(299)
    assert s.tbest[2] < 0.2 * f1
