"""Fixtures printed by the paper (Tables hyper8, hyper8path, params_path,
BFs) and by the published definition of the random generator (Philox4x32-10
known-answer vectors) against the oracle and the constants the inputs use."""
import os

import numpy as np

from paper_2308_10169_amd import inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    out = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                out.append(line.split())
    return out


def test_philox_known_answers(orc):
    for r in _rows("philox4x32_10_kat.txt"):
        v = [int(x, 16) for x in r]
        out = orc.philox(v[:4], v[4:6])
        assert [int(x) for x in out] == v[6:]


def test_hyper_tables_as_printed(orc):
    assert np.array_equal(I.HYPER8, np.array(_rows("table_hyper8.txt"), float))
    assert np.array_equal(orc.HYPER8, np.array(_rows("table_hyper8.txt"), float))
    assert np.array_equal(I.HYPER8PATH, np.array(_rows("table_hyper8path.txt"), float))
    a, b, g, dlt, tw = _rows("table_params_path.txt")[0]
    pp = I.PARAMS_PATH
    assert (pp["alpha"], pp["beta"], pp["gamma"], pp["delta"], pp["tw"]) == \
        (float(a), int(b), float(g), float(dlt), int(tw))


def test_benchmark_minima_as_printed(orc):
    for fid, name, D, lo, hi, fmin in _rows("table_bfs.txt"):
        fid, D = int(fid), int(D)
        xstar = np.ones(D) if name == "rosenbrock" else np.zeros(D)
        assert abs(orc.bf_value(fid, xstar) - float(fmin)) < 1e-12
        assert float(lo) <= xstar.min() and xstar.max() <= float(hi)
        # the minimum is a minimum: random points of the box score higher
        rng = np.random.default_rng(fid)
        for _ in range(20):
            assert orc.bf_value(fid, rng.uniform(float(lo), float(hi), D)) > float(fmin)
