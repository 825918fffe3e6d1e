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
