"""GPU parity of the fused DTPSO iteration against the FP64 oracle, by state
injection at every step (tolerances in parity.py)."""
import numpy as np
import pytest

from oracle import pyorc as orc
from paper_2308_10169_amd import inputs as I

from parity import check_fitness, check_frame_step, check_step

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    from paper_2308_10169_amd import sepso
    sepso.lib()
    return sepso


def _run_injected(sp, spec, sw, steps, stats=None):
    pl = sp.Planner(spec, sw)
    o = orc.Swarm(sw, spec.width, spec.height)
    m = orc.Map(spec)
    st0 = pl.get_state()
    for _ in range(steps):
        pl.step(1)
        st1 = pl.get_state()
        check_step(o, m, st0, st1, spec.scale, stats)
        st0 = st1
    pl.close()


@pytest.mark.parametrize("waypoints", [8, 7, 9])  # D % 4 == 0, and 2: rows off 16-byte boundaries
def test_init_draws_bit_exact(sp, waypoints):
    # X0 = u * hi with u a 24-bit Philox uniform: the FP32 product is the
    # correctly rounded exact product, so it must equal the oracle's value
    # rounded to FP32 -- any differing random word would show.
    spec, sw = I.static_map(0), I.static_swarm(seed=12345, waypoints=waypoints)
    pl = sp.Planner(spec, sw)
    st = pl.get_state()
    o = orc.Swarm(sw, spec.width, spec.height)
    o.init(0)
    assert np.array_equal(st["X"], o.X.astype(np.float32))
    assert np.allclose(st["V"], o.V, rtol=0, atol=1e-5 * 100)
    assert np.all(np.isinf(st["Pf"]))
    pl.close()


@pytest.mark.parametrize("variant", ["hyper1", "hyper8"])
def test_static_plan_every_step(sp, variant):
    # Single static plan (100x100, 4 rectangles, 4x32 particles, W=8, 50
    # iterations); variant hyper8 exercises the Tbest attractor (C3 != 0).
    stats = {}
    for seed in (0, 1, 2):
        spec = I.static_map(seed)
        sw = I.static_swarm(seed=seed, variant=variant)
        _run_injected(sp, spec, sw, 50, stats)
    print("parity stats", stats)
    assert stats["paths"] == 3 * 50 * 128


@pytest.mark.parametrize("variant", ["hyper8", "dyn"])
def test_per_coordinate_factors_every_step(sp, variant):
    # Variant of the update with one (r1, r2, r3) per coordinate: every step
    # of the HIP path against the oracle's (static plan and a dynamic shape
    # with a ragged W = 13 stream).
    import dataclasses
    stats = {}
    if variant == "hyper8":
        spec = I.static_map(5)
        sw = dataclasses.replace(I.static_swarm(seed=5, variant="hyper8"), rand_per_dim=1)
        _run_injected(sp, spec, sw, 30, stats)
    else:
        spec = I.dynamic_map(6, S=200.0, n_static=6, n_moving=6, side=(8.0, 30.0))
        sw = dataclasses.replace(I.dynamic_swarm(spec.scale, seed=4, groups=3, particles=37,
                                                 waypoints=13), rand_per_dim=1)
        _run_injected(sp, spec, sw, 12, stats)
    print("parity stats", stats)


def test_nonconvex_polygons_every_step(sp):
    # Rectangles mixed with non-convex stars (10-16 vertices each): the
    # general edge path and the rectangle path in one instance, ragged W = 11.
    stats = {}
    for seed in (0, 1):
        spec = I.nonconvex_map(seed)
        sw = I.dynamic_swarm(spec.scale, seed=seed, groups=4, particles=48, waypoints=11)
        _run_injected(sp, spec, sw, 10, stats)
    print("parity stats", stats)
    assert stats["paths"] == 2 * 10 * 4 * 48


def test_convex_polygons_every_step(sp):
    # Rectangles mixed with convex polygons of 3-8 vertices listed in both
    # orientations: the convex in/out path (and any polygon that snapping left
    # not strictly convex, on the edge-by-edge path), ragged W = 11.
    stats = {}
    for seed in (0, 1, 2):
        spec = I.convex_map(seed)
        sw = I.dynamic_swarm(spec.scale, seed=seed, groups=4, particles=48, waypoints=11)
        _run_injected(sp, spec, sw, 10, stats)
    print("parity stats", stats)
    assert stats["paths"] == 3 * 10 * 4 * 48


def test_polygons_the_convex_form_must_refuse(sp):
    # Polygons whose turns all agree but that are no simple convex polygon
    # (a pentagram), with a straight angle (three collinear vertices), with
    # more than eight vertices, and a convex one among them: only the last
    # may take the convex form, and every step must match the oracle.
    import math
    S = 200.0
    star = [(100 + 40 * math.cos(math.pi / 2 + 4 * math.pi * k / 5),
             100 + 40 * math.sin(math.pi / 2 + 4 * math.pi * k / 5)) for k in range(5)]
    flat = [(20, 120), (50, 120), (80, 120), (60, 170), (30, 160)]
    ring = [(150 + 25 * math.cos(2 * math.pi * k / 12), 60 + 25 * math.sin(2 * math.pi * k / 12))
            for k in range(12)]
    tri = [(40, 40), (80, 50), (55, 85)]
    spec = I.make_map(S, S, [I.snap(p) for p in (star, flat, ring, tri)], (8.0, 12.0), (192.0, 188.0))
    sw = I.dynamic_swarm(spec.scale, seed=5, groups=4, particles=48, waypoints=11)
    stats = {}
    _run_injected(sp, spec, sw, 8, stats)
    print("parity stats", stats)
    assert stats["paths"] == 8 * 4 * 48


def test_nonconvex_edges_over_several_passes(sp):
    # 30 stars (about 400 edges): the edge records pass through LDS in more
    # than one chunk.
    stats = {}
    spec = I.nonconvex_map(4, n_stars=30)
    assert spec.poly_ptr[-1] - 4 * 6 > 256
    sw = I.dynamic_swarm(spec.scale, seed=4, groups=4, particles=48, waypoints=11)
    _run_injected(sp, spec, sw, 6, stats)
    print("parity stats", stats)
    assert stats["paths"] == 6 * 4 * 48


def test_dynamic_shape_steps(sp):
    # Paper-shaped instance: 366 map, 30 rectangles, 8 x 170 particles, W = 20.
    spec = I.dynamic_map(0)
    sw = I.dynamic_swarm(spec.scale, seed=3)
    stats = {}
    _run_injected(sp, spec, sw, 12, stats)
    print("parity stats", stats)


@pytest.mark.parametrize("K,B", [(4, 64), (8, 128), (12, 256), (16, 256), (24, 128)])
def test_tile_shapes_agree(sp, K, B):
    # Every tile configuration yields the oracle's crossings and the same
    # per-particle fitness (ragged tails: N = 37 particles, W = 13).
    spec = I.dynamic_map(2, S=200.0, n_static=6, n_moving=6, side=(8.0, 30.0))
    sw = I.dynamic_swarm(spec.scale, seed=9, groups=3, particles=37, waypoints=13)
    bp = sp.BatchPlanner([spec], [sw], tune=(K, B))
    o = orc.Swarm(sw, spec.width, spec.height)
    o.init(0)
    st = bp.get_state(0)
    assert np.array_equal(st["X"], o.X.astype(np.float32))
    bp.profile_step(1)  # one fused iteration, then the pending update
    st1 = bp.get_state(0)
    check_fitness(orc.Map(spec), st, st1, 13, sw.alpha, sw.beta)
    bp.close()


@pytest.mark.parametrize("K,B", [(4, 64), (8, 256), (16, 256)])
def test_many_groups_per_block(sp, K, B):
    # 64 groups of 3 particles at W = 64: a block spans dozens of groups, so
    # dozens of gbest rows are staged per block; every step against the oracle.
    spec = I.dynamic_map(4, S=300.0, n_static=5, n_moving=5, side=(8.0, 30.0))
    sw = I.dynamic_swarm(spec.scale, seed=21, groups=64, particles=3, waypoints=64)
    bp = sp.BatchPlanner([spec], [sw], tune=(K, B))
    o = orc.Swarm(sw, spec.width, spec.height)
    m = orc.Map(spec)
    stats = {}
    st0 = bp.get_state(0)
    for _ in range(4):
        bp.profile_step(1)
        st1 = bp.get_state(0)
        check_step(o, m, st0, st1, spec.scale, stats)
        st0 = st1
    bp.close()
    assert stats["paths"] == 4 * 64 * 3


@pytest.mark.parametrize("tune", [(8, 64), (8, 128), (4, 256)])  # 1, 2, 4 wave groups
@pytest.mark.parametrize("n_rects", [1, 3, 5, 6, 9])
def test_ragged_rectangle_quads(sp, tune, n_rects):
    # Rectangles are read four at a time from a slice padded to whole quads
    # and dealt over the wave groups quad by quad: counts that are not a
    # multiple of four, and fewer quads than wave groups, against the oracle.
    spec = I.dynamic_map(30 + n_rects, S=200.0, n_static=n_rects, n_moving=0, side=(20.0, 50.0))
    sw = I.dynamic_swarm(spec.scale, seed=n_rects, groups=4, particles=48, waypoints=12)
    bp = sp.BatchPlanner([spec], [sw], tune=tune)
    o = orc.Swarm(sw, spec.width, spec.height)
    m = orc.Map(spec)
    stats = {}
    st0 = bp.get_state(0)
    for _ in range(3):
        bp.profile_step(1)
        st1 = bp.get_state(0)
        check_step(o, m, st0, st1, spec.scale, stats)
        st0 = st1
    bp.close()
    assert stats["paths"] == 3 * 4 * 48


def test_adversarial_degenerate_paths(sp):
    # Waypoints placed exactly on obstacle vertices, on edges and along edge
    # lines: many degenerate tests; counts must stay in the oracle bracket.
    spec = I.static_map(7)
    sw = I.static_swarm(seed=1, groups=2, particles=64, waypoints=8)
    pl = sp.Planner(spec, sw)
    rng = np.random.default_rng(0)
    V = spec.verts
    X = np.zeros((2, 64, 16))
    for g in range(2):
        for n in range(64):
            for j in range(8):
                a, b = V[rng.integers(len(V))], V[rng.integers(len(V))]
                t = rng.integers(0, 5) / 4.0  # vertex, edge point or beyond
                p = a + t * (b - a)
                X[g, n, j], X[g, n, 8 + j] = np.clip(p, 0, 100)
    st = pl.get_state()
    st["X"] = X.astype(np.float32)
    st["Pf"][:] = np.inf
    pl.set_state(st)
    st0 = pl.get_state()
    pl.step(1)
    st1 = pl.get_state()
    r = check_fitness(orc.Map(spec), st0, st1, 8, sw.alpha, sw.beta)
    assert r["n_deg"].sum() > 100
    pl.close()


@pytest.mark.parametrize("tune", [(8, 256), (4, 256)])
def test_full_batch_sampled(sp, tune):
    # The benchmark workload at full size (1024 uneven dynamic instances) in the
    # launch configuration the benchmark times: its tile, after 20 iterations
    # (a converging swarm, wave culling active).  One more injected iteration is
    # checked against the oracle on 16 instances spread over the batch, every
    # particle of each: crossings, fitness, bests, update.
    specs, sws = [], []
    for i in range(1024):
        m, shape = I.batch_instance(i, 0)
        sws.append(I.dynamic_swarm(m.scale, seed=0, instance=i, **shape))
        specs.append(m)
    bp = sp.BatchPlanner(specs, sws, tune=tune)
    bp.profile_step(20)
    sample = list(range(0, 1024, 64))
    st0 = {i: bp.get_state(i) for i in sample}
    bp.profile_step(1)
    stats = {}
    for i in sample:
        o = orc.Swarm(sws[i], specs[i].width, specs[i].height)
        check_step(o, orc.Map(specs[i]), st0[i], bp.get_state(i), specs[i].scale, stats)
    bp.close()
    print("parity stats", stats)
    assert stats["paths"] == sum(sws[i].groups * sws[i].particles for i in sample)


def test_large_stress_sampled(sp):
    # Stress scene at full size (512 map, 500 rectangles + 100 quads = 2400
    # edges, 8 x 4096 particles, W = 64); fitness of a sample of particles
    # against the oracle.
    spec = I.stress_map(0)
    sw = I.SwarmSpec(8, 4096, 64, 200, I.HYPER8PATH, alpha=30.0, beta=4, seed=4)
    pl = sp.Planner(spec, sw)
    st0 = pl.get_state()
    pl.step(1)
    st1 = pl.get_state()
    idx = np.random.default_rng(1).choice(8 * 4096, 96, replace=False)
    sub = lambda st: dict(X=st["X"].reshape(-1, 128)[idx][None], Q=st["Q"].reshape(-1)[idx][None],
                          L=st["L"].reshape(-1)[idx][None], f=st["f"].reshape(-1)[idx][None])
    check_fitness(orc.Map(spec), sub(st0), sub(st1), 64, sw.alpha, sw.beta)
    pl.close()


def test_determinism(sp):
    spec, sw = I.dynamic_map(5), I.dynamic_swarm(366.0, seed=5)
    a, b = sp.Planner(spec, sw), sp.Planner(spec, sw)
    a.step(20)
    b.step(20)
    sa, sb = a.get_state(), b.get_state()
    for k in ("X", "V", "P", "Pf", "Q"):
        assert np.array_equal(sa[k], sb[k])
    a.close()
    b.close()


def test_end_to_end_median_cost(sp):
    # Static plan over 100 seeds: the median final Tbest fitness of the GPU
    # planner is within 1% of the oracle planner's.
    g, c = [], []
    for seed in range(100):
        spec, sw = I.static_map(seed), I.static_swarm(seed=seed)
        pl = sp.Planner(spec, sw)
        pl.step(sw.max_iters)
        g.append(pl.get_state()["tbest"][2])
        pl.close()
        c.append(orc.plan_static(spec, sw)[0])
    mg, mc = np.median(g), np.median(c)
    print("median cost gpu", mg, "oracle", mc)
    assert abs(mg - mc) <= 0.01 * mc


@pytest.mark.parametrize("first,c1,c2,c3,key", [
    (0, 0, 0, 0, 0),                                    # the published all-zero case and on
    (0, 7, 513, 0, 0x0123456789ABCDEF),                # an update stream: step 7, instance 513
    (0xFFC00000, 0xFFFFFFFF, 1023, 12, 2**64 - 1),     # counters that wrap the first word
])
def test_philox_stream_bit_exact(sp, first, c1, c2, c3, key):
    # 4.2 million consecutive blocks of the GPU's generator, word for word
    # against the oracle's own implementation.
    n = 1 << 22
    g = sp.philox(first, c1, c2, c3, key, n)
    ctr = np.empty((n, 4), dtype=np.uint32)
    ctr[:, 0] = (np.uint64(first) + np.arange(n, dtype=np.uint64)).astype(np.uint32)
    ctr[:, 1], ctr[:, 2], ctr[:, 3] = c1, c2, c3
    o = orc.philox_many(ctr, np.array([key & 0xFFFFFFFF, key >> 32], dtype=np.uint32))
    assert np.array_equal(g, o)


def test_stress_frame_with_self_evolution(sp):
    # Stress scene at full size (512 map, 500 rectangles + 100 quads = 2400
    # edges, 400 of them general-polygon records: two LDS passes; 8 x 4096
    # particles, W = 64) in a 200-iteration frame with the online outer step
    # every 10 iterations: iterations 1, 50 and 150 checked by state
    # injection -- fitness on 2048 sampled particles, bests, the outer step
    # (due at 50 and 150) and the update of every particle.  By iteration 150
    # the swarm has converged, so the wave culling is active.
    spec = I.stress_map(0)
    sw = I.SwarmSpec(8, 4096, 64, 200, I.HYPER8PATH, alpha=30.0, beta=4, seed=4, hsef_every=10)
    pl = sp.Planner(spec, sw)
    o = orc.Swarm(sw, spec.width, spec.height)
    m = orc.Map(spec)
    sample = np.sort(np.random.default_rng(2).choice(8 * 4096, 2048, replace=False))
    done = 0
    for it in (1, 50, 150):
        pl.step_frame(it - 1 - done)
        st0, out0 = pl.get_state(), pl.get_outer()
        assert st0["k"] == it - 1
        pl.step_frame(1)
        st1, out1 = pl.get_state(), pl.get_outer()
        print(f"stress frame iteration {it}: tbest {st1['tbest'][2]:.2f}", flush=True)
        check_frame_step(o, m, st0, st1, out0, out1, spec.scale, sample, hsef=it % 10 == 0)
        done = it
    pl.close()
