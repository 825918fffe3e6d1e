"""Pins of the oracle's application-phase pieces: Auto Truncation, online
self-evolution, obstacle motion and the frame loop -- CPU only."""
import numpy as np

from paper_2308_10169_amd import inputs as I


def test_at_mode1_std_window(orc):
    # Sec. "Auto Truncation": std of the last TW values below delta AND the
    # best path collision-free.
    hist = np.r_[np.linspace(500, 420, 10), np.full(20, 400.0) + np.arange(20) * 0.1]
    assert orc.at_check(hist, 30, 1, 20, 10.0, 0) == 1
    assert orc.at_check(hist, 30, 1, 20, 10.0, 2) == 0  # collides -> keep going
    assert orc.at_check(hist, 19, 1, 20, 10.0, 0) == 0  # window not filled
    wide = np.r_[np.full(10, 400.0), np.full(10, 440.0)]  # std = 20
    assert orc.at_check(wide, 20, 1, 20, 10.0, 0) == 0
    assert orc.at_check(wide, 20, 1, 20, 20.5, 0) == 1


def test_at_mode2_relative_improvement(orc):
    hist = np.array([900.0, 800.0, 700.0, 600.0, 500.0, 499.9, 499.8])
    # k = 6: 800 - 499.9 = 300 > 0.5 -> no; k = 7 vs k = 2: 800 - 499.8 no
    assert orc.at_check(hist, 6, 2, 5, 1e-3, 0) == 0
    flat = np.array([900.0, 500.0, 499.9, 499.85, 499.8, 499.75, 499.7])
    # k = 7: hist[1] - hist[6] = 0.3 < 1e-3 * 499.7 = 0.4997 -> stop
    assert orc.at_check(flat, 7, 2, 5, 1e-3, 0) == 1
    assert orc.at_check(flat, 5, 2, 5, 1e-3, 0) == 0  # needs k > window


def test_at_mode3_growing_window(orc):
    # std over the last min(k, TW) values once two exist
    hist = np.array([430.0, 424.0, 421.0, 420.5, 420.4] + [420.4] * 30)
    # k = 2: std(430, 424) = 3 < 10 -> stop;  k = 1: never
    assert orc.at_check(hist, 1, 3, 20, 10.0, 0) == 0
    assert orc.at_check(hist, 2, 3, 20, 10.0, 0) == 1
    assert orc.at_check(hist, 2, 3, 20, 2.9, 0) == 0
    assert orc.at_check(hist, 2, 3, 20, 10.0, 1) == 0  # collision -> keep going
    # beyond TW values the window is capped: k = 30 sees only the flat tail
    assert orc.at_check(hist, 30, 3, 20, 1e-9, 0) == 1
    wide = np.r_[np.full(10, 400.0), np.full(10, 440.0)]  # std 20 over 20 values
    assert orc.at_check(wide, 20, 3, 20, 20.5, 0) == 1 and orc.at_check(wide, 20, 3, 20, 19.5, 0) == 0


def _dyn_swarm(orc, spec, **kw):
    sw = I.dynamic_swarm(spec.scale, seed=2, particles=24, waypoints=6, **kw)
    return orc.Swarm(sw, spec.width, spec.height)


def test_hsef_bounds_and_outer_memory(orc):
    spec = I.dynamic_map(1)
    m = orc.Map(spec)
    s = _dyn_swarm(orc, spec)
    s.init(0)
    s.hsef_reset_frame()
    h0 = s.hyper.copy()
    best = np.full(8, np.inf)
    for epoch in range(6):
        for _ in range(10):
            s.step(m)
        s.hsef_step()
        best = np.minimum(best, s.gbest_f)
        assert np.all(s.opf == best)  # outer Pbest fitness = running minimum
        assert np.all(s.hyper[:, 3] >= s.hyper[:, 4] - 1e-15) and np.all(s.hyper[:, 3] <= 1.0)
        assert np.all((s.hyper[:, :2] >= 0) & (s.hyper[:, :2] <= 3))
        # only w_init, C1, C2 move; C3, w_end, V_limit stay
        assert np.array_equal(s.hyper[:, [2, 4, 5]], h0[:, [2, 4, 5]])
    assert not np.array_equal(s.hyper, h0)


def test_sim_bounce_closed_form(orc):
    # A 10-wide box moving +3/frame in x on a 40-wide map: x_min follows a
    # reflected walk that stays in [0, 30]; velocity flips at each wall.
    spec = I.make_map(40.0, 40.0, [[[20, 5], [30, 5], [30, 15], [20, 15]]], (1, 20), (39, 20),
                      poly_vel=[[3.0, 0.0]], endpoint_vel=[0, 1.5, 0, -2.0])
    xs, vs = [], []
    for _ in range(40):
        orc.sim_step(spec)
        xs.append(spec.verts[:, 0].min())
        vs.append(spec.poly_vel[0, 0])
        assert spec.verts.min() >= 0 and spec.verts[:, 0].max() <= 40
        assert 0 <= spec.start[1] <= 40 and 0 <= spec.target[1] <= 40
    # unfolded coordinate of a reflected walk: period 2*(40-10) = 60 cells
    for k, x in enumerate(xs, start=1):
        u = (20 + 3 * k) % 60
        assert x == (u if u <= 30 else 60 - u)
    assert set(vs) == {3.0, -3.0}
    assert spec.verts[:, 1].min() == 5.0  # no vertical motion


def test_frame_loop_truncation_and_pi(orc):
    spec = I.dynamic_map(3)
    m = orc.Map(spec)
    s_at = _dyn_swarm(orc, spec)
    s_no = _dyn_swarm(orc, spec, at_mode=0)
    it_at, it_no = [], []
    for f in range(6):
        r = s_at.plan_frame(m, f)
        r2 = s_no.plan_frame(m, f)
        it_at.append(r["iters"])
        it_no.append(r2["iters"])
        assert r2["iters"] == 50 and r2["truncated"] == 0
        if r["truncated"]:
            assert r["crossings"] == 0 and r["iters"] > 5
        assert r["cost"] == s_at.tbest[2]
        # frame result equals the oracle's own fitness of the returned path
        chk = orc.fitness(m, r["path"][None, :], 6, s_at.sw.alpha, s_at.sw.beta)
        assert abs(chk["f"][0] - r["cost"]) <= 1e-9 * r["cost"]
        orc.sim_step(spec)
        m = orc.Map(spec)
    assert np.mean(it_at) < np.mean(it_no)
