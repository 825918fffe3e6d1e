"""The C-ABI library loads, exports every function include/sepso.h declares,
and rejects bad arguments before touching a device -- CPU only."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2308_10169_amd", "libsepso.so")
HDR = os.path.join(ROOT, "include", "sepso.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2308_10169_amd import build
        build.build()
    L = C.CDLL(LIB)
    L.sepso_last_error.restype = C.c_char_p
    return L


def test_exports_every_declared_function(lib):
    names = set(re.findall(r"\b(sepso_[a-z_]+)\s*\(", open(HDR).read()))
    assert len(names) >= 20
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing


def _args(**over):
    from paper_2308_10169_amd import inputs as I
    from paper_2308_10169_amd.sepso import _MapArgs, _SwarmArgs
    spec, sw = I.static_map(0), I.static_swarm(0)
    for k, v in over.items():
        setattr(sw, k, v)
    return _MapArgs(spec), _SwarmArgs(sw)


def _ws_bytes(lib, m, s):
    n = C.c_size_t()
    st = lib.sepso_workspace_bytes(C.byref(m.c), C.byref(s.c), C.byref(n))
    return st, n.value


def test_workspace_bytes_valid(lib):
    m, s = _args()
    st, n = _ws_bytes(lib, m, s)
    assert st == 0
    # X, V, P alone need 3 * 4*32*16 floats
    assert n >= 3 * 4 * 4 * 32 * 16


@pytest.mark.parametrize("field,value", [("groups", 0), ("groups", 65), ("waypoints", 0),
                                         ("waypoints", 65), ("particles", 0), ("beta", 0),
                                         ("max_iters", 0), ("at_mode", 4), ("at_mode", -1), ("at_window", 64),
                                         ("hsef_every", -1)])
def test_bad_swarm_rejected(lib, field, value):
    m, s = _args()
    setattr(s.c, field, value)
    st, _ = _ws_bytes(lib, m, s)
    assert st == 1, lib.sepso_last_error()
    assert lib.sepso_last_error()


def test_bad_map_rejected(lib):
    m, s = _args()
    m.c.width = -1.0
    assert _ws_bytes(lib, m, s)[0] == 1
    m, s = _args()
    m.verts[0] = 1e4  # vertex outside the map
    assert _ws_bytes(lib, m, s)[0] == 1
    m, s = _args()
    m.pptr[1] = 2  # polygon with 2 vertices
    assert _ws_bytes(lib, m, s)[0] == 1
    m, s = _args()
    m.c.start[0] = float("nan")
    assert _ws_bytes(lib, m, s)[0] == 1


def test_null_handles_rejected(lib):
    assert lib.sepso_step(None, 1) == 1
    assert lib.sepso_destroy(None) == 1
    assert lib.sepso_plan_frame(None, None, None, None) == 1


def test_create_rejects_small_or_misaligned_workspace(lib):
    m, s = _args()
    h = C.c_void_p()
    st = lib.sepso_create(C.byref(m.c), C.byref(s.c), C.c_void_p(256), C.c_size_t(16), None,
                          C.byref(h))
    assert st == 2 and not h.value  # workspace too small: nothing created
    st = lib.sepso_create(C.byref(m.c), C.byref(s.c), C.c_void_p(257), C.c_size_t(1 << 30), None,
                          C.byref(h))
    assert st == 1


def test_philox_rejects_bad_arguments(lib):
    f = lib.sepso_philox
    f.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64, C.c_int64,
                  C.c_void_p, C.c_void_p]
    assert f(0, 0, 0, 0, 0, -1, C.c_void_p(256), None) == 1          # negative count
    assert f(0, 0, 0, 0, 0, (1 << 32) + 1, C.c_void_p(256), None) == 1  # beyond the counter word
    assert f(0, 0, 0, 0, 0, 8, None, None) == 1                      # no output
    assert f(0, 0, 0, 0, 0, 8, C.c_void_p(260), None) == 1           # misaligned output
    assert f(0, 0, 0, 0, 0, 0, None, None) == 0                      # nothing to do


def test_negative_vlimit_rejected(lib):
    m, s = _args()
    s.hyper[5] = -0.1  # group 0's V_limit
    assert _ws_bytes(lib, m, s)[0] == 1
    assert b"V_limit" in lib.sepso_last_error()


def test_tune_cache_and_set_tune_need_a_batch(lib):
    assert lib.sepso_autotune_cached(None, b"/tmp/x", None) == 1
    assert lib.sepso_batch_set_tune(None, None) == 1


def test_bucket_calls_reject_null_batch(lib):
    tl = (C.c_int32 * 2)(8, 256)
    bo = (C.c_int32 * 1)(0)
    assert lib.sepso_batch_set_tiles(None, 1, bo, tl) == 1
    assert lib.sepso_autotune_buckets(None, 2, None, tl, bo, None, None) == 1
