"""Pins of the oracle's application-phase pieces: Auto Truncation, online
self-evolution, obstacle motion and the frame loop -- CPU only."""
import numpy as np
import pytest

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


def _hsef_swarm(orc, outer_row, G=8):
    """An oracle swarm whose outer swarm uses `outer_row` for every outer
    particle (C1, C2, C3, w_init, w_end, V_limit), with its outer memory reset
    for a new frame (Pbest = current hyper, zero velocity)."""
    spec = I.dynamic_map(1)
    sw = I.dynamic_swarm(spec.scale, seed=3, groups=G, particles=8, waypoints=4)
    sw.hsef_hyper = np.tile(np.asarray(outer_row, float), (G, 1))
    s = orc.Swarm(sw, spec.width, spec.height)
    s.init(0)
    s.hsef_reset_frame()
    return s


def _outer_r(orc, s, g, word):
    """The outer step's random factor of outer particle g (Sec. HSEF: the
    grouped update of Eq.(4) with one draw per particle), from the generator."""
    sw = s.sw
    w = orc.philox([g, s.h.epoch_ctr, sw.instance, orc.TAG_HSEF],
                   [sw.seed & 0xFFFFFFFF, sw.seed >> 32])
    return (int(w[word]) >> 8) * 2.0 ** -24


COLS = [3, 0, 1]  # the outer particle's (w_init, C1, C2) columns of the hyper matrix


def test_hsef_pure_inertia(orc):
    # omega = 1 and no attractors: each outer coordinate moves by its own
    # velocity, which is kept (Eq.(4) with C = 0, Eq.(7)-(8) without clamps).
    s = _hsef_swarm(orc, [0, 0, 0, 1, 1, 1e6])
    s.hyper[:, 4] = 0.1  # w_end: w_init's lower bound
    s.hyper[:, COLS] = [0.5, 1.5, 1.2]
    rng = np.random.default_rng(0)
    s.ov[:] = rng.uniform(-0.2, 0.2, s.ov.shape)
    x0, v0 = s.hyper[:, COLS].copy(), s.ov.copy()
    s.hsef_step()
    assert np.array_equal(s.ov, v0)
    assert np.array_equal(s.hyper[:, COLS], x0 + v0)


@pytest.mark.parametrize("which", [0, 1, 2])
def test_hsef_single_attractor(orc, which):
    # omega = 0 and one attractor constant c: every coordinate of outer
    # particle g moves by the same factor c * r towards the attractor --
    # its own Pbest for C1 and C2 (each outer particle is its own group, so
    # its group best is its Pbest), the outer total best for C3 -- with r the
    # particle's draw 0, 1 or 2 of the step.
    c = 0.75
    row = [0.0, 0.0, 0.0, 0.0, 0.0, 1e6]
    row[which] = c
    s = _hsef_swarm(orc, row)
    G = s.G
    rng = np.random.default_rng(which)
    s.hyper[:, 4] = 0.05
    s.hyper[:, COLS] = np.c_[rng.uniform(0.2, 0.9, G), rng.uniform(0.2, 2.8, (G, 2))]
    s.op[:] = np.c_[rng.uniform(0.2, 0.9, G), rng.uniform(0.2, 2.8, (G, 2))]
    # the outer Pbest fitness is below any group best (no Pbest update), and
    # its argmin, the outer total best, is the last particle
    s.opf[:] = -1e6 - np.arange(G)
    s.gbest_f[:] = 100.0
    x0, op = s.hyper[:, COLS].copy(), s.op.copy()
    r = np.array([_outer_r(orc, s, g, which) for g in range(G)])
    s.hsef_step()
    target = op if which < 2 else np.tile(op[G - 1], (G, 1))
    want = x0 + (c * r)[:, None] * (target - x0)
    assert np.allclose(s.hyper[:, COLS], want, rtol=0, atol=1e-15)
    assert s.h.otb == G - 1
    assert 0 < len(set(r)) and np.all((r >= 0) & (r < 1))


def test_hsef_outer_inertia_schedule(orc):
    # Eq.(6) over the outer epochs of a frame: omega_e = w_init - (w_init -
    # w_end) * e / T_outer, e = 1, 2, ... and held at w_end once e >= T_outer
    # (T_outer = ceil(T_max / hsef_every) = 5 here).
    s = _hsef_swarm(orc, [0, 0, 0, 0.9, 0.4, 1e6])
    assert s.h.T_outer == 5
    s.hyper[:, 4] = 0.05
    for e in range(1, 9):
        s.hyper[:, COLS] = [0.5, 1.5, 1.5]
        s.ov[:] = 0.25
        s.hsef_step()
        w = 0.9 - 0.5 * min(e, 5) / 5
        assert np.allclose(s.ov, 0.25 * w, rtol=0, atol=1e-15), e
        assert s.h.epoch_in_frame == e


def test_plan_frame_order_hand_traced(orc):
    # One frame of T = 3 iterations with the outer step after every
    # iteration, against the same primitives called by hand in Algorithm 1's
    # order: evaluate, bests, (outer step), update -- and after the last
    # evaluation no outer step and no update, only the random-stream advance.
    import dataclasses
    spec = I.dynamic_map(2)
    sw = dataclasses.replace(I.dynamic_swarm(spec.scale, seed=7, particles=16, waypoints=6,
                                             iters=3, at_mode=0, hsef_every=1))
    m = orc.Map(spec)
    a = orc.Swarm(sw, spec.width, spec.height)
    ra = a.plan_frame(m, 0)
    b = orc.Swarm(sw, spec.width, spec.height)
    b.init(0)
    b.hsef_reset_frame()
    hist = []
    for k in (1, 2, 3):
        b.s.k = k
        b.eval(m)
        b.bests()
        hist.append(b.tbest[2])
        if k == 3:
            b.s.ctr += 1
            break
        b.hsef_step()
        b.update()
        b.s.ctr += 1
    for name in ("X", "V", "P", "Pf", "hyper", "ov", "op", "opf"):
        assert np.array_equal(getattr(a, name), getattr(b, name)), name
    assert (a.k, a.ctr, a.tbest) == (b.k, b.ctr, b.tbest) == (3, 3, a.tbest)
    assert np.array_equal(a.hist[:3], hist)
    assert ra["iters"] == 3 and ra["cost"] == b.tbest[2]
    # the order is observable: the update before the outer step moves the
    # swarm with the old hyper-parameters, which ends elsewhere
    c = orc.Swarm(sw, spec.width, spec.height)
    c.init(0)
    c.hsef_reset_frame()
    for k in (1, 2):
        c.s.k = k
        c.eval(m)
        c.bests()
        c.update()
        c.hsef_step()
        c.s.ctr += 1
    assert not np.array_equal(c.X, b.X)


def test_at_mode2_needs_an_earlier_best(orc):
    # "improves by < delta over w iterations" compares Tbest after iteration k
    # with Tbest after iteration k - w; before iteration w + 1 the earlier
    # value is the +inf of the empty start, so the test cannot pass -- the
    # same decisions as evaluating from k >= w with Tbest_0 = +inf.
    flat = np.full(10, 500.0)
    assert orc.at_check(flat, 5, 2, 5, 1e-3, 0) == 0
    assert orc.at_check(flat, 6, 2, 5, 1e-3, 0) == 1
    with_inf = np.r_[np.inf, flat]  # index 0 = Tbest before iteration 1
    for k in range(1, 10):
        lit = (with_inf[k - 5] - with_inf[k] < 1e-3 * 500.0) if k >= 5 else False
        assert orc.at_check(flat, k, 2, 5, 1e-3, 0) == int(lit), k
