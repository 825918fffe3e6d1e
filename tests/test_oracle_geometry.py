"""Pins of the oracle's fitness (Eq.(11)-(13)) against closed forms, exact
integer/rational predicates and hand-built maps -- CPU only."""
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_2308_10169_amd import inputs as I


def _path_X(waypoints):
    w = np.asarray(waypoints, dtype=np.float64)
    return np.concatenate([w[:, 0], w[:, 1]])[None, :]


def _map(polys, start, target, S=100.0):
    return I.make_map(S, S, polys, start, target)


BOX = [[40, 40], [60, 40], [60, 60], [40, 60]]


def test_straight_line_length_is_distance(orc):
    # Ordered collinear waypoints on the start-target segment, no obstacles:
    # the polyline length equals the Euclidean distance (closed form).
    s, t = (5.0, 5.0), (95.0, 95.0)
    wp = [(5 + 10 * i, 5 + 10 * i) for i in range(1, 9)]
    m = orc.Map(_map([], s, t))
    r = orc.fitness(m, _path_X(wp), 8, alpha=1e3, beta=1)
    assert r["Q"][0] == 0
    assert abs(r["L"][0] - 90.0 * math.sqrt(2.0)) < 1e-12
    assert r["f"][0] == r["L"][0]


def test_length_right_angle_legs(orc):
    # 3-4-5 legs: (0,0)->(3,4)->(3,4)+(4,3)... each leg has length 5.
    s, t = (10.0, 10.0), (24.0, 24.0)
    wp = [(13.0, 14.0), (17.0, 17.0), (20.0, 21.0)]  # legs 5, 5, 5, sqrt(25)=5
    m = orc.Map(_map([], s, t))
    r = orc.fitness(m, _path_X(wp), 3, alpha=1.0, beta=1)
    assert r["L"][0] == 20.0


def test_length_scales_and_reverses(orc):
    rng = np.random.default_rng(1)
    wp = I.snap(rng.uniform(0, 50, size=(7, 2)))
    s, t = (1.0, 2.0), (49.0, 47.0)
    m1 = orc.Map(_map([], s, t, S=50.0))
    m2 = orc.Map(_map([], (2.0, 4.0), (98.0, 94.0), S=100.0))
    mr = orc.Map(_map([], t, s, S=50.0))
    L1 = orc.fitness(m1, _path_X(wp), 7, 1.0, 1)["L"][0]
    L2 = orc.fitness(m2, _path_X(2 * wp), 7, 1.0, 1)["L"][0]
    Lr = orc.fitness(mr, _path_X(wp[::-1]), 7, 1.0, 1)["L"][0]
    assert L2 == 2.0 * L1  # power-of-two scaling is exact
    assert abs(Lr - L1) <= 1e-12 * L1
    assert L1 >= math.dist(s, t)  # triangle inequality


def test_box_crossed_twice_and_penalty(orc):
    # Horizontal path through a box crosses its left and right edges.
    m = orc.Map(_map([BOX], (10, 50), (90, 50)))
    r = orc.fitness(m, _path_X([(30, 50), (50, 50), (70, 50)]), 3, alpha=30.0, beta=4)
    assert r["Q"][0] == 2 and r["q_yes"][0] == 2 and r["n_deg"][0] == 0
    assert r["f"][0] - r["L"][0] == 30.0 * 2 ** 4
    assert r["L"][0] == 80.0


def test_two_boxes_four_crossings(orc):
    box2 = [[70, 45], [80, 45], [80, 55], [70, 55]]
    m = orc.Map(_map([BOX, box2], (10, 50), (95, 50)))
    r = orc.fitness(m, _path_X([(30, 50), (50, 50), (75, 50)]), 3, alpha=1.0, beta=1)
    assert r["Q"][0] == 4 and r["q_yes"][0] == 4 and r["n_deg"][0] == 0


def test_path_around_box_is_free(orc):
    m = orc.Map(_map([BOX], (10, 50), (90, 50)))
    r = orc.fitness(m, _path_X([(30, 70), (50, 70), (70, 70)]), 3, alpha=1e3, beta=1)
    assert r["Q"][0] == 0 and r["n_deg"][0] == 0


def test_vertex_and_edge_contacts_are_degenerate(orc):
    # Diagonal through two opposite corners: every contact is at a vertex.
    m = orc.Map(_map([BOX], (30, 30), (70, 70)))
    r = orc.fitness(m, _path_X([(50, 50)]), 1, alpha=1.0, beta=1)
    assert r["q_yes"][0] == 0 and r["n_deg"][0] > 0 and r["Q"][0] == 0
    # Path running along the bottom edge.
    m = orc.Map(_map([BOX], (30, 40), (70, 40)))
    r = orc.fitness(m, _path_X([(50, 40)]), 1, alpha=1.0, beta=1)
    assert r["q_yes"][0] == 0 and r["n_deg"][0] > 0
    # Segment ending exactly on the left edge (touching).
    m = orc.Map(_map([BOX], (30, 50), (30, 20)))
    r = orc.fitness(m, _path_X([(40, 50)]), 1, alpha=1.0, beta=1)
    assert r["q_yes"][0] == 0 and r["n_deg"][0] > 0


def test_non_convex_u_shape(orc):
    U = [[20, 20], [80, 20], [80, 80], [60, 80], [60, 40], [40, 40], [40, 80], [20, 80]]
    m = orc.Map(_map([U], (10, 60), (90, 60)))
    r = orc.fitness(m, _path_X([(30, 60), (50, 60), (70, 60)]), 3, alpha=1.0, beta=1)
    assert r["Q"][0] == 4 and r["q_yes"][0] == 4  # both prongs
    m = orc.Map(_map([U], (10, 30), (90, 30)))
    r = orc.fitness(m, _path_X([(30, 30), (50, 30), (70, 30)]), 3, alpha=1.0, beta=1)
    assert r["Q"][0] == 2  # below the notch: outer walls only


def test_zero_length_segment_counts_nothing(orc):
    m = orc.Map(_map([BOX], (10, 50), (90, 50)))
    r = orc.fitness(m, _path_X([(50, 50), (50, 50), (50, 50)]), 3, alpha=1.0, beta=1)
    assert r["Q"][0] == 2 and r["n_deg"][0] == 0
    assert orc.classify((50, 50), (50, 50), (40, 40), (60, 40), 1e-2) == 0


def _sgn(v):
    return (v > 0) - (v < 0)


def _orient_exact(a, b, c):
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])


def _cross_exact(p, q, a, b):
    o1, o2 = _orient_exact(p, q, a), _orient_exact(p, q, b)
    o3, o4 = _orient_exact(a, b, p), _orient_exact(a, b, q)
    return int(_sgn(o1) * _sgn(o2) < 0 and _sgn(o3) * _sgn(o4) < 0)


def test_crossing_matches_exact_integer_predicate(orc):
    # Small integer coordinates: many collinear and touching cases.  The FP64
    # orientation is exact there, so the oracle must equal the integer result.
    rng = np.random.default_rng(7)
    pts = rng.integers(0, 6, size=(20000, 4, 2))
    got = [orc.crosses(*(c.astype(float) for c in case)) for case in pts]
    want = [_cross_exact(*(tuple(int(v) for v in c) for c in case)) for case in pts]
    assert got == want
    assert sum(want) > 500  # the sample does contain crossings


def test_classification_against_exact_rationals(orc):
    # Near-collinear grid points: exact rational orientations decide the
    # robust / degenerate class under tau; the oracle must agree.
    rng = np.random.default_rng(3)
    S = 64.0
    tau = 1e-6 * S * S
    n_deg = 0
    for _ in range(3000):
        # p, q on the integer grid; a, b exactly on line pq (multiples of
        # 1/16 along it) plus a jitter of -1, 0 or +1 grid cells, so that the
        # orientations straddle tau.
        p = rng.integers(0, 8, 2).astype(float)
        q = rng.integers(0, 8, 2).astype(float)
        t = rng.integers(-4, 21, 2) / 16.0
        base = p[None, :] + t[:, None] * (q - p)[None, :]
        jitter = rng.integers(-1, 2, size=(2, 2)) / 256.0
        a, b = base[0] + jitter[0], base[1] + jitter[1]
        F = [tuple(Fraction(float(v)) for v in x) for x in (p, q, a, b)]
        o = [_orient_exact(F[0], F[1], F[2]), _orient_exact(F[0], F[1], F[3]),
             _orient_exact(F[2], F[3], F[0]), _orient_exact(F[2], F[3], F[1])]
        big12 = abs(o[0]) >= tau and abs(o[1]) >= tau
        big34 = abs(o[2]) >= tau and abs(o[3]) >= tau
        if (tuple(p) == tuple(q)) or (big12 and o[0] * o[1] > 0) or (big34 and o[2] * o[3] > 0):
            want = 0
        elif big12 and big34 and o[0] * o[1] < 0 and o[2] * o[3] < 0:
            want = 1
        else:
            want = -1
        n_deg += want == -1
        assert orc.classify(p, q, a, b, tau) == want
    assert n_deg > 50


def test_degenerate_bracket_holds_for_random_maps(orc):
    # Q (strict FP64) lies within [q_yes, q_yes + n_deg] for every path.
    spec = I.static_map(5)
    m = orc.Map(spec)
    rng = np.random.default_rng(0)
    X = I.snap(rng.uniform(0, 100, size=(200, 16)))
    r = orc.fitness(m, X, 8, alpha=1.0, beta=1)
    assert np.all(r["Q"] >= r["q_yes"]) and np.all(r["Q"] <= r["q_yes"] + r["n_deg"])
    # brute force over all (segment, edge) pairs with the exact predicate
    for i in range(0, 200, 17):
        x = X[i]
        pts = [tuple(spec.start)] + [(x[j], x[8 + j]) for j in range(8)] + [tuple(spec.target)]
        q = 0
        for a in range(9):
            for poly in range(spec.n_polys):
                v0, v1 = spec.poly_ptr[poly], spec.poly_ptr[poly + 1]
                vs = [tuple(Fraction(float(c)) for c in spec.verts[j]) for j in range(v0, v1)]
                for j in range(len(vs)):
                    P = tuple(Fraction(float(c)) for c in pts[a])
                    Qp = tuple(Fraction(float(c)) for c in pts[a + 1])
                    q += _cross_exact(P, Qp, vs[j], vs[(j + 1) % len(vs)])
        assert q == r["Q"][i]


@pytest.mark.parametrize("beta", [1, 2, 4])
def test_penalty_power(orc, beta):
    m = orc.Map(_map([BOX, [[70, 45], [80, 45], [80, 55], [70, 55]]], (10, 50), (95, 50)))
    r = orc.fitness(m, _path_X([(30, 50), (50, 50), (75, 50)]), 3, alpha=2.5, beta=beta)
    assert r["f"][0] - r["L"][0] == 2.5 * 4 ** beta
