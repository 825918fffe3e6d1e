"""sepso_fitness (Eq.(11)-(13)) on the GPU against the FP64 oracle's
fitness, path by path: crossing counts bit-exact where the oracle flags no
degenerate test (else inside [q_yes, q_yes + n_deg]), lengths within
1e-5 * max(L, 1), fitness within 1e-5 * max(f, 1) where the counts agree.
Sizes span several 256-thread blocks with ragged tails, several LDS passes
of edge records (the stress map's 2400 edges against 512 per pass), W = 1
and W = 64, and the empty cases."""
import numpy as np
import pytest

from oracle import pyorc as orc
from paper_2308_10169_amd import inputs as I

pytestmark = pytest.mark.gpu

REL = 1e-5


def _gpu():
    from paper_2308_10169_amd import sepso
    return sepso


def _paths(rng, spec, n, W, near=None):
    X = np.empty((n, 2 * W))
    X[:, :W] = rng.uniform(0, spec.width, (n, W))
    X[:, W:] = rng.uniform(0, spec.height, (n, W))
    if near is not None:  # waypoints on obstacle vertices and edges (degenerate contacts)
        v = np.asarray(spec.verts, dtype=np.float64).reshape(-1, 2)
        pick = rng.integers(0, len(v), (n, W))
        t = rng.choice([0.0, 0.5, 1.0], (n, W))
        nxt = np.minimum(pick + 1, len(v) - 1)
        pts = v[pick] * (1 - t[..., None]) + v[nxt] * t[..., None]
        m = rng.random((n, W)) < near
        X[:, :W][m] = pts[..., 0][m]
        X[:, W:][m] = pts[..., 1][m]
    return X.astype(np.float32)


def check(spec, X, W, alpha, beta, out):
    m = orc.Map(spec)
    r = orc.fitness(m, X.astype(np.float64), W, alpha, beta)
    q = out["Q"]
    assert np.all(q >= r["q_yes"]) and np.all(q <= r["q_yes"] + r["n_deg"]), "Q outside the bracket"
    clean = r["n_deg"] == 0
    assert np.array_equal(q[clean], r["Q"][clean]), "Q differs on robust paths"
    L = out["L"].astype(np.float64)
    assert np.all(np.abs(L - r["L"]) <= REL * np.maximum(np.abs(r["L"]), 1.0)), "length"
    agree = q == r["Q"]
    f = out["f"].astype(np.float64)
    assert np.all(np.abs(f[agree] - r["f"][agree]) <= REL * np.maximum(np.abs(r["f"][agree]), 1.0))
    return int(clean.sum())


@pytest.mark.parametrize("case", ["static", "stress", "nonconvex", "dynamic"])
def test_fitness_matches_oracle(case):
    sepso = _gpu()
    rng = np.random.default_rng(11)
    if case == "static":
        spec, W, n, a, b = I.static_map(0), 8, 1000, 1e3, 1
    elif case == "stress":
        spec, W, n, a, b = I.stress_map(0), 64, 300, 30.0, 4
    elif case == "nonconvex":
        spec, W, n, a, b = I.nonconvex_map(0), 1, 257, 30.0, 4
    else:
        spec, W, n, a, b = I.dynamic_map(0), 20, 2049, 30.0, 4
    X = _paths(rng, spec, n, W)
    print(f"fitness case={case} n={n} W={W} edges={spec.n_edges}", flush=True)
    out = sepso.fitness(spec, X, W, a, b)
    # random paths over the stress map's 2400 edges often come within the
    # degenerate band of some edge (about half of them here); the rest are
    # compared exactly
    clean = check(spec, X, W, a, b, out)
    assert clean > (0.3 if case == "stress" else 0.9) * n


def test_fitness_degenerate_contacts():
    """Waypoints on obstacle vertices and edge midpoints: every count inside
    the oracle's bracket, exact where it flags nothing."""
    sepso = _gpu()
    rng = np.random.default_rng(5)
    for spec, W in ((I.static_map(3), 8), (I.nonconvex_map(2), 12)):
        X = _paths(rng, spec, 700, W, near=0.3)
        out = sepso.fitness(spec, X, W, 30.0, 4)
        check(spec, X, W, 30.0, 4, out)


def test_fitness_empty_and_obstacle_free():
    sepso = _gpu()
    spec = I.static_map(0)
    out = sepso.fitness(spec, np.zeros((0, 16), np.float32), 8, 1e3, 1)
    assert len(out["f"]) == 0
    free = I.make_map(100.0, 100.0, [], (5.0, 5.0), (95.0, 95.0))
    # collinear waypoints on the start-target chord: L = |t - s|, Q = 0
    W = 8
    t = np.linspace(0.1, 0.9, W)
    X = np.concatenate([5 + 90 * t, 5 + 90 * t])[None, :].repeat(3, 0).astype(np.float32)
    out = sepso.fitness(free, X, W, 1e3, 1)
    assert np.all(out["Q"] == 0)
    assert np.allclose(out["L"], 90 * np.sqrt(2), rtol=1e-6)
    assert np.array_equal(out["f"], out["L"])
