"""The crossing count can be bit-exact: a CPU emulation of the fused
iteration's FP32 orientation arithmetic (exact rational FMA, one rounding to
FP32 per operation) gives the same sign pattern as the FP64 oracle on every
segment x edge test the oracle calls robust (|orientation| >= 1e-6 * S^2,
Eq.(13)'s proper-crossing test), on random and near-collinear cases at the
largest map side, for both obstacle forms (rectangle corners and general
edges) -- CPU only."""
from fractions import Fraction as Fr

import numpy as np
import pytest


def _round32(x: Fr) -> float:
    """x rounded to the nearest FP32 value, ties to even (normal range)."""
    if x == 0:
        return 0.0
    s = -1 if x < 0 else 1
    a = abs(x)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fr(2) ** e > a:
        e -= 1
    q = a / Fr(2) ** (e - 23)  # in [2^23, 2^24)
    n = q.numerator // q.denominator
    r = q - n
    if r > Fr(1, 2) or (r == Fr(1, 2) and n % 2 == 1):
        n += 1
    v = s * n * 2.0 ** (e - 23)
    assert np.float32(v) == v
    return v


def fma32(a, b, c):
    return _round32(Fr(a) * Fr(b) + Fr(c))


def sub32(a, b):
    return _round32(Fr(a) - Fr(b))


def mul32(a, b):
    return _round32(Fr(a) * Fr(b))


def seg_line(p, q):
    """The kernel's line of segment p -> q: (dx, -dy, nc), nc = dy*px - dx*py
    by one product and one FMA."""
    dx, dy = sub32(q[0], p[0]), sub32(q[1], p[1])
    nc = fma32(dy, p[0], -mul32(dx, p[1]))
    return dx, -dy, nc


def side_seg(line, v):
    dx, ndy, nc = line
    return fma32(dx, v[1], fma32(ndy, v[0], nc))


def rect_corner_sides(line, box):
    """o00 by two FMAs, the other corners by one FMA each along the exact
    side lengths w, h (o11 from o10)."""
    dx, ndy, nc = line
    x0, y0, x1, y1 = box
    w, h = sub32(x1, x0), sub32(y1, y0)
    o00 = fma32(dx, y0, fma32(ndy, x0, nc))
    o10 = fma32(ndy, w, o00)
    o01 = fma32(dx, h, o00)
    o11 = fma32(dx, h, o10)
    return {(x0, y0): o00, (x1, y0): o10, (x0, y1): o01, (x1, y1): o11}


def edge_rec(a, b):
    """General edge record: ex, -ey exact on the grid, nce = -(ex*ay - ey*ax)
    by one product and one FMA."""
    ex, ey = sub32(b[0], a[0]), sub32(b[1], a[1])
    nce = -fma32(ex, a[1], -mul32(ey, a[0]))
    return ex, -ey, nce


def side_edge(rec, p):
    ex, ney, nce = rec
    return fma32(ex, p[1], fma32(ney, p[0], nce))


def orient64(a, b, c):
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])


def neg(x):
    return np.signbit(np.float32(x))


def _cases(rng, S, n, near):
    out = []
    for _ in range(n):
        if near:
            # a segment whose line passes within a hair of an edge end point
            a = np.round(rng.uniform(0, S, 2) * 256) / 256
            b = np.round(rng.uniform(0, S, 2) * 256) / 256
            d = rng.normal(size=2)
            d /= np.linalg.norm(d)
            t0, t1 = rng.uniform(-S, 0), rng.uniform(0, S)
            off = rng.normal() * 1e-4 * np.array([-d[1], d[0]])
            p = np.clip(a + t0 * d + off, 0, S)
            q = np.clip(a + t1 * d - off, 0, S)
        else:
            p, q = rng.uniform(0, S, 2), rng.uniform(0, S, 2)
            a = np.round(rng.uniform(0, S, 2) * 256) / 256
            b = np.round(rng.uniform(0, S, 2) * 256) / 256
        p, q = p.astype(np.float32).astype(float), q.astype(np.float32).astype(float)
        out.append((p, q, a, b))
    return out


@pytest.mark.parametrize("near", [False, True])
def test_general_edge_signs_match_when_robust(orc, near):
    S = 512.0
    tau = 1e-6 * S * S
    rng = np.random.default_rng(7 + near)
    robust = 0
    for p, q, a, b in _cases(rng, S, 1500, near):
        line, rec = seg_line(p, q), edge_rec(a, b)
        o = [orient64(p, q, a), orient64(p, q, b), orient64(a, b, p), orient64(a, b, q)]
        g = [side_seg(line, a), side_seg(line, b), side_edge(rec, p), side_edge(rec, q)]
        # the kernel's values are orient(p, q, v) and orient(a, b, p) themselves
        for o64, o32 in zip(o, g):
            if abs(o64) >= tau:
                assert neg(o32) == (o64 < 0)
        cls = orc.classify(p, q, a, b, tau)
        gpu = int(neg(g[0]) != neg(g[1]) and neg(g[2]) != neg(g[3]))
        if cls >= 0:
            robust += 1
            assert gpu == cls
    assert robust > 1000


@pytest.mark.parametrize("near", [False, True])
def test_rectangle_corner_signs_match_when_robust(orc, near):
    S = 512.0
    tau = 1e-6 * S * S
    rng = np.random.default_rng(11 + near)
    checked = 0
    for p, q, a, _ in _cases(rng, S, 1000, near):
        w, h = np.round(rng.uniform(5, 40, 2) * 256) / 256
        x0, y0 = min(a[0], S - w), min(a[1], S - h)
        box = (x0, y0, x0 + w, y0 + h)
        if near:  # pass the segment's line close by a corner
            c = np.array([box[2], box[3]])
            d = (q - p) / np.linalg.norm(q - p)
            p = np.clip(c - 40 * d + 1e-4 * np.array([-d[1], d[0]]), 0, S).astype(np.float32).astype(float)
            q = np.clip(c + 40 * d, 0, S).astype(np.float32).astype(float)
        line = seg_line(p, q)
        sides = rect_corner_sides(line, box)
        for v, o32 in sides.items():
            o64 = orient64(p, q, v)
            if abs(o64) >= tau:
                checked += 1
                assert neg(o32) == (o64 < 0), (p, q, v, o64, o32)
    assert checked > 3000


def rect_count_inout(p, q, box):
    """The fused iteration's count of proper crossings of segment p -> q
    with the four edges of an axis-aligned box, emulated in FP32: the end
    points' strict sides of the box's four lines (exact comparisons); one
    crossing when exactly one end point lies strictly inside; two when both
    lie outside, the segment's x and y ranges overlap the box's open ranges
    and the box's corners are not all on one side of the segment's line,
    tested at the box centre: |o(c)| < |dx| h/2 + |dy| w/2, by two FMAs for
    o(c) and two for the difference."""
    x0, y0, x1, y1 = box
    L = lambda v: sub32(x0, v[0]) < 0          # v.x > x0
    R = lambda v: sub32(v[0], x1) < 0          # v.x < x1
    B = lambda v: sub32(y0, v[1]) < 0
    T = lambda v: sub32(v[1], y1) < 0
    inside = lambda v: L(v) and R(v) and B(v) and T(v)
    ip, iq = inside(p), inside(q)
    if ip != iq:
        return 1
    if ip or iq:
        return 0
    ov = (L(p) or L(q)) and (R(p) or R(q)) and (B(p) or B(q)) and (T(p) or T(q))
    if not ov:
        return 0
    dx, ndy, nc = seg_line(p, q)
    xc, yc = (x0 + x1) / 2, (y0 + y1) / 2      # exact: coordinates on a 1/256 grid
    hw, hh = (x1 - x0) / 2, (y1 - y0) / 2
    oc = fma32(dx, yc, fma32(ndy, xc, nc))
    d = fma32(-abs(dx), hh, abs(oc))
    d = fma32(-abs(ndy), hw, d)
    return 2 if d < 0 else 0


def _box_cases(rng, S, n):
    """Segments against boxes on a 1/256 grid: random, through the box,
    ending inside, grazing a corner, along an edge line, on an edge,
    axis-parallel and zero-length."""
    g = lambda v: np.round(np.asarray(v, float) * 256) / 256
    f32 = lambda v: np.asarray(v, np.float64).astype(np.float32).astype(float)
    for k in range(n):
        w, h = g(rng.uniform(5, 40, 2))
        x0, y0 = g(rng.uniform(0, S - w)), g(rng.uniform(0, S - h))
        box = (x0, y0, x0 + w, y0 + h)
        c = np.array([box[(k % 2) * 2], box[1 + ((k // 2) % 2) * 2]])  # a corner
        kind = k % 8
        if kind == 0:
            p, q = rng.uniform(0, S, 2), rng.uniform(0, S, 2)
        elif kind == 1:  # through the box
            m = np.array([x0 + w / 2, y0 + h / 2]) + rng.normal(size=2) * [w / 3, h / 3]
            d = rng.normal(size=2)
            p, q = m - 60 * d, m + 60 * d
        elif kind == 2:  # one end inside
            p = np.array([rng.uniform(x0, x0 + w), rng.uniform(y0, y0 + h)])
            q = p + rng.normal(size=2) * 30
        elif kind == 3:  # line grazing a corner by ~1e-4
            d = rng.normal(size=2)
            d /= np.linalg.norm(d)
            off = rng.choice([-1, 1]) * rng.uniform(0, 2e-4) * np.array([-d[1], d[0]])
            p, q = c - rng.uniform(1, 50) * d + off, c + rng.uniform(1, 50) * d + off
        elif kind == 4:  # along an edge line
            p = np.array([box[0], rng.uniform(0, S)])
            q = np.array([box[0], rng.uniform(0, S)])
        elif kind == 5:  # end point on an edge
            p = np.array([box[2], rng.uniform(y0, y0 + h)])
            q = rng.uniform(0, S, 2)
        elif kind == 6:  # axis-parallel through or near
            y = rng.choice([y0, y0 + h, rng.uniform(y0, y0 + h), y0 + h + 1e-3])
            p, q = np.array([x0 - 20, y]), np.array([x0 + w + 20, y])
        else:  # zero length, inside or outside
            p = rng.uniform(0, S, 2) if rng.random() < 0.5 else np.array([x0 + w / 2, y0 + h / 2])
            q = p.copy()
        p, q = f32(np.clip(p, 0, S)), f32(np.clip(q, 0, S))
        yield p, q, box


def test_rectangle_inout_count_in_bracket(orc):
    # The in/out form of the rectangle count against the oracle's per-edge
    # classification: equal to the robust count when no edge test is
    # degenerate, inside [q_yes, q_yes + n_deg] always.
    S = 512.0
    tau = 1e-6 * S * S
    rng = np.random.default_rng(23)
    exact = 0
    for p, q, (x0, y0, x1, y1) in _box_cases(rng, S, 6000):
        corners = [(x0, y0), (x1, y0), (x1, y1), (x0, y1)]
        cls = [orc.classify(p, q, np.array(corners[e]), np.array(corners[(e + 1) % 4]), tau)
               for e in range(4)]
        yes, deg = sum(c == 1 for c in cls), sum(c == -1 for c in cls)
        got = rect_count_inout(p, q, (x0, y0, x1, y1))
        assert yes <= got <= yes + deg, (p, q, (x0, y0, x1, y1), cls, got)
        if deg == 0:
            exact += 1
            assert got == yes
    assert exact > 3000
