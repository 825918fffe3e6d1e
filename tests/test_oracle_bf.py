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


def test_instance_and_run_streams(orc):
    # swarm instance s, run r: initial draws at counter (block, r, s, tag), the
    # move at (particle, ctr, s, tag); instance 0, run 0 is the default stream
    G, N, D, lo, hi = 2, 3, 7, -600.0, 600.0
    base = _swarm(orc, G=G, N=N, D=D)
    same = orc.BFSwarm(1, G, N, D, 4, I.HYPER8[:G], seed=3, instance=0, run=0)
    assert np.array_equal(base.X, same.X) and np.array_equal(base.V, same.V)
    s = orc.BFSwarm(1, G, N, D, 4, I.HYPER8[:G], seed=3, instance=5, run=2)
    nb = (D + 3) // 4
    for i in (0, G * N - 1):
        for d in range(D):
            w = orc.philox([i * nb + d // 4, 2, 5, 10], [3, 0])
            assert s.X.reshape(-1, D)[i, d] == lo + orc.u01(int(w[d % 4])) * (hi - lo)
    assert not np.array_equal(s.X, base.X)
    r = orc.BFSwarm(1, G, N, D, 4, I.HYPER8[:G], seed=3, instance=0, run=1)
    assert not np.array_equal(r.X, base.X)
    # the move of instance 5 draws (r1, r2, r3) from (particle, ctr, 5, 9): with
    # only C1 and w = 0 the first move is X + r1 (P - X) = X (P = X after the
    # first evaluation), so compare the second move against the drawn r1
    h = np.array([[1.0, 0, 0, 0, 0, 1]] * G)
    t = orc.BFSwarm(1, G, N, D, 4, h, seed=3, instance=5)
    t.step(1)
    X1 = t.X.copy()
    ctr = t.ctr
    t.step(1)
    X1, P2, X2 = X1.reshape(-1, D), t.P.reshape(-1, D), t.X.reshape(-1, D)
    for i in range(G * N):
        r1 = orc.u01(int(orc.philox([i, ctr, 5, 9], [3, 0])[0]))
        exp = np.clip(X1[i] + np.clip(r1 * (P2[i] - X1[i]), -600, 600), lo, hi)
        assert np.allclose(X2[i], exp, rtol=0, atol=1e-9)


def test_bf_evolve_one_iteration_lfv(orc):
    # with one evaluated iteration a lower-level run's LFV is the lowest
    # function value over its initial swarm, whatever the hyper-parameters
    ev = orc.BFEvolve(3, 2, 4, 6, 1, h_groups=2, h_particles=3, evolutions=5, seed=7, h_seed=1)
    for e in range(2):
        lfv = ev.lfv()
        for i in range(6):
            init = orc.BFSwarm(3, 2, 4, 6, 1, I.HYPER8[:2], seed=7, instance=i, run=e)
            vals = [orc.bf_value(3, x) for x in init.X.reshape(-1, 6)]
            assert lfv[i] == min(vals)
        ev.step(lfv)
        ev.evolution += 1
    assert ev.k == 2


def test_bf_evolve_curve(orc):
    # the total best LFV never rises, and the H particles move inside the box
    ev = orc.BFEvolve(1, 2, 5, 10, 30, h_groups=2, h_particles=3, evolutions=6, seed=2, h_seed=4)
    curve = ev.evolve(6)
    assert np.all(np.diff(curve) <= 0) and curve[-1] < np.inf
    lo, hi = np.tile(ev.lo, 2), np.tile(ev.hi, 2)
    assert np.all(ev.X >= lo) and np.all(ev.X <= hi)
    # the reported best is the LFV of the total-best H Pbest's own run
    tg, tn, tf = ev.tbest
    assert tf == ev.Pf[tg * ev.Nh + tn] == curve[-1]
