"""sepso_fitness_noalloc (the allocation-free variant of sepso_fitness, its
scratch a fixed per-GPU device array) through the C-ABI: two calls in a row,
the second smaller, each identical to sepso_fitness on the same inputs (the
same kernels, so bit for bit) and inside the oracle's bracket; a request
beyond the array's size is refused before any device work."""
import ctypes as C

import numpy as np
import pytest

from oracle import pyorc as orc
from paper_2308_10169_amd import inputs as I

pytestmark = pytest.mark.gpu


def _paths(seed, spec, n, W):
    rng = np.random.default_rng(seed)
    X = np.empty((n, 2 * W))
    X[:, :W] = rng.uniform(0, spec.width, (n, W))
    X[:, W:] = rng.uniform(0, spec.height, (n, W))
    return X.astype(np.float32)


def test_noalloc_matches_workspace_variant():
    from paper_2308_10169_amd import sepso
    cases = [(I.stress_map(1), 64, 900, 30.0, 4), (I.static_map(2), 8, 77, 1e3, 1)]
    for k, (spec, W, n, a, b) in enumerate(cases):  # second call: fewer edges, paths, waypoints
        X = _paths(k, spec, n, W)
        print(f"noalloc call {k}: n={n} W={W} edges={spec.n_edges}", flush=True)
        got = sepso.fitness(spec, X, W, a, b, noalloc=True)
        ref = sepso.fitness(spec, X, W, a, b)
        for key in ("f", "L", "Q"):
            assert np.array_equal(got[key], ref[key]), key
        r = orc.fitness(orc.Map(spec), X.astype(np.float64), W, a, b)
        assert np.all(got["Q"] >= r["q_yes"]) and np.all(got["Q"] <= r["q_yes"] + r["n_deg"])
        clean = r["n_deg"] == 0
        assert np.array_equal(got["Q"][clean], r["Q"][clean])
        assert np.all(np.abs(got["L"] - r["L"]) <= 1e-5 * np.maximum(r["L"], 1.0))


def test_noalloc_refuses_oversized_request():
    from paper_2308_10169_amd import sepso
    L = sepso.lib()
    n = C.c_size_t()
    assert L.sepso_fitness_workspace_bytes(8, 200000, 64, C.byref(n)) == 0
    assert n.value > 8 << 20
    # arguments are checked before the device is touched: dangling device
    # pointers are never dereferenced on this path
    fake = C.c_void_p(256)
    st = L.sepso_fitness_noalloc(2, 8, fake, fake, fake, fake, 200000, 64, 1.0, 1, fake, fake,
                                 fake, None)
    assert st == sepso.E_ARG
    assert b"8388608" in L.sepso_last_error() or b"holds" in L.sepso_last_error()
