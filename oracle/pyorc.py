"""ctypes binding of the FP64 oracle (liborc.so, plain C++ built with g++).

Test infrastructure only.  Builds the library on first use if it is absent.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborc.so")
SOURCES = ["orc_core.cpp", "orc_frame.cpp", "orc_mlp.cpp", "orc_evolve.cpp", "orc_bf.cpp"]

(TAG_UPDATE, TAG_INIT_X, TAG_INIT_V, TAG_PI, TAG_HSEF, TAG_LEARNED, TAG_EVOLVE, TAG_EVOLVE_X,
 TAG_EVOLVE_V, TAG_BF_UPDATE, TAG_BF_INIT_X, TAG_BF_INIT_V, TAG_UPDATE_DIM) = range(13)
BF_SPHERE, BF_ROSENBROCK, BF_RASTRIGIN, BF_GRIEWANK = 1, 2, 3, 4


def build(force: bool = True) -> str:
    """Compile liborc.so with g++ (no GPU code involved)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    tmp = LIB_PATH + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-o", tmp] + srcs
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None

dp = C.POINTER(C.c_double)
ip = C.POINTER(C.c_int32)
up = C.POINTER(C.c_uint32)


class OrcMap(C.Structure):
    _fields_ = [("width", C.c_double), ("height", C.c_double), ("n_polys", C.c_int32),
                ("poly_ptr", ip), ("verts", dp), ("start", C.c_double * 2),
                ("target", C.c_double * 2)]


class OrcSwarm(C.Structure):
    _fields_ = [("G", C.c_int32), ("N", C.c_int32), ("W", C.c_int32), ("T", C.c_int32),
                ("width", C.c_double), ("height", C.c_double), ("hyper", dp),
                ("alpha", C.c_double), ("beta", C.c_int32), ("seed", C.c_uint64),
                ("instance", C.c_uint32), ("X", dp), ("V", dp), ("P", dp), ("f", dp),
                ("L", dp), ("Q", ip), ("Pf", dp), ("PL", dp), ("PQ", ip), ("gbest_n", ip),
                ("gbest_f", dp), ("tbest_g", C.c_int32), ("tbest_n", C.c_int32),
                ("tbest_f", C.c_double), ("k", C.c_int32), ("ctr", C.c_uint32),
                ("rand_per_dim", C.c_int32)]


class OrcHsef(C.Structure):
    _fields_ = [("outer_hyper", dp), ("ov", dp), ("op", dp), ("opf", dp), ("otb", C.c_int32),
                ("epoch_in_frame", C.c_int32), ("T_outer", C.c_int32),
                ("epoch_ctr", C.c_uint32)]


class OrcFrameCfg(C.Structure):
    _fields_ = [("use_pi", C.c_int32), ("pi_gamma", C.c_double), ("pi_radius", C.c_double),
                ("at_mode", C.c_int32), ("at_window", C.c_int32), ("at_delta", C.c_double),
                ("hsef_every", C.c_int32)]


class OrcFrameResult(C.Structure):
    _fields_ = [("cost", C.c_double), ("length", C.c_double), ("crossings", C.c_int32),
                ("iters", C.c_int32), ("truncated", C.c_int32)]


class OrcEvolve(C.Structure):
    _fields_ = [("Gh", C.c_int32), ("Nh", C.c_int32), ("Dh", C.c_int32), ("E", C.c_int32),
                ("h_hyper", dp), ("lo", dp), ("hi", dp), ("seed", C.c_uint64),
                ("X", dp), ("V", dp), ("P", dp), ("Pf", dp), ("gbest_n", ip), ("gbest_f", dp),
                ("tb_g", C.c_int32), ("tb_n", C.c_int32), ("tb_f", C.c_double),
                ("k", C.c_int32), ("ctr", C.c_uint32)]


class OrcBF(C.Structure):
    _fields_ = [("func", C.c_int32), ("G", C.c_int32), ("N", C.c_int32), ("D", C.c_int32),
                ("T", C.c_int32), ("lo", C.c_double), ("hi", C.c_double), ("hyper", dp),
                ("seed", C.c_uint64), ("X", dp), ("V", dp), ("P", dp), ("f", dp), ("Pf", dp),
                ("gbest_n", ip), ("gbest_f", dp), ("tb_g", C.c_int32), ("tb_n", C.c_int32),
                ("tb_f", C.c_double), ("k", C.c_int32), ("ctr", C.c_uint32),
                ("instance", C.c_uint32), ("run", C.c_uint32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.orc_philox4x32_10.argtypes = [up, up, up]
        L.orc_philox_many.argtypes = [C.c_int64, up, up, up]
        L.orc_u01.argtypes = [C.c_uint32]
        L.orc_u01.restype = C.c_double
        L.orc_classify.argtypes = [dp, dp, dp, dp, C.c_double]
        L.orc_classify.restype = C.c_int32
        L.orc_crosses.argtypes = [dp, dp, dp, dp]
        L.orc_crosses.restype = C.c_int32
        L.orc_fitness.argtypes = [C.POINTER(OrcMap), C.c_int32, C.c_int32, dp, C.c_double,
                                  C.c_int32, C.c_double, dp, dp, ip, ip, ip]
        for fn in ("orc_eval", "orc_step"):
            getattr(L, fn).argtypes = [C.POINTER(OrcSwarm), C.POINTER(OrcMap)]
        for fn in ("orc_bests", "orc_update"):
            getattr(L, fn).argtypes = [C.POINTER(OrcSwarm)]
        L.orc_init.argtypes = [C.POINTER(OrcSwarm), C.c_int32, dp, C.c_double, C.c_double]
        L.orc_hsef_reset_frame.argtypes = [C.POINTER(OrcSwarm), C.POINTER(OrcHsef)]
        L.orc_hsef_step.argtypes = [C.POINTER(OrcSwarm), C.POINTER(OrcHsef)]
        L.orc_at_check.argtypes = [dp, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_int32]
        L.orc_at_check.restype = C.c_int32
        L.orc_sim_step.argtypes = [C.c_double, C.c_double, C.c_int32, ip, dp, dp, dp, dp, dp]
        L.orc_plan_frame.argtypes = [C.POINTER(OrcSwarm), C.POINTER(OrcHsef), C.POINTER(OrcMap),
                                     C.POINTER(OrcFrameCfg), C.c_int32, dp, dp, dp,
                                     C.POINTER(OrcFrameResult)]
        L.orc_bf_value.argtypes = [C.c_int32, C.c_int32, dp]
        L.orc_bf_value.restype = C.c_double
        L.orc_bf_init.argtypes = [C.POINTER(OrcBF)]
        L.orc_bf_step.argtypes = [C.POINTER(OrcBF)]
        L.orc_bf_eval.argtypes = [C.POINTER(OrcBF)]
        L.orc_bf_advance.argtypes = [C.POINTER(OrcBF)]
        L.orc_evolve_init.argtypes = [C.POINTER(OrcEvolve)]
        L.orc_evolve_step.argtypes = [C.POINTER(OrcEvolve), dp]
        _lib = L
    return _lib


def _p(a, t=dp):
    return a.ctypes.data_as(t)


# ---------------------------------------------------------------------------
def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c, up), _p(k, up), _p(out, up))
    return out


def philox_many(ctrs, key):
    c = np.ascontiguousarray(ctrs, dtype=np.uint32).reshape(-1, 4)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros_like(c)
    lib().orc_philox_many(len(c), _p(c, up), _p(k, up), _p(out, up))
    return out


def u01(word) -> float:
    return lib().orc_u01(int(word))


class Map:
    """Oracle view of a map (keeps the numpy buffers alive)."""

    def __init__(self, spec):
        self.spec = spec
        self.poly_ptr = np.ascontiguousarray(spec.poly_ptr, dtype=np.int32)
        self.verts = np.ascontiguousarray(spec.verts, dtype=np.float64).reshape(-1, 2)
        self.s = OrcMap(float(spec.width), float(spec.height), len(self.poly_ptr) - 1,
                        _p(self.poly_ptr, ip), _p(self.verts),
                        (C.c_double * 2)(*map(float, spec.start)),
                        (C.c_double * 2)(*map(float, spec.target)))

    @property
    def scale(self):
        return max(self.s.width, self.s.height)


def classify(p, q, a, b, tau):
    arr = [np.ascontiguousarray(x, dtype=np.float64) for x in (p, q, a, b)]
    return lib().orc_classify(*[_p(x) for x in arr], float(tau))


def crosses(p, q, a, b):
    arr = [np.ascontiguousarray(x, dtype=np.float64) for x in (p, q, a, b)]
    return lib().orc_crosses(*[_p(x) for x in arr])


def fitness(m: Map, X, W, alpha, beta, tau=None):
    """Returns dict(f, L, Q, q_yes, n_deg) for paths X (n, 2W)."""
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 2 * W)
    n = len(X)
    if tau is None:
        tau = 1e-6 * m.scale ** 2
    f = np.zeros(n)
    Lv = np.zeros(n)
    Q = np.zeros(n, np.int32)
    yes = np.zeros(n, np.int32)
    deg = np.zeros(n, np.int32)
    lib().orc_fitness(C.byref(m.s), n, W, _p(X), float(alpha), int(beta), float(tau), _p(f),
                      _p(Lv), _p(Q, ip), _p(yes, ip), _p(deg, ip))
    return dict(f=f, L=Lv, Q=Q, q_yes=yes, n_deg=deg)


class Swarm:
    """Oracle swarm with numpy-owned state."""

    def __init__(self, sw, width, height):
        G, N, W = sw.groups, sw.particles, sw.waypoints
        D = 2 * W
        self.G, self.N, self.W, self.D = G, N, W, D
        self.sw = sw
        self.hyper = np.ascontiguousarray(sw.hyper, dtype=np.float64).reshape(G, 6).copy()
        z = lambda *sh: np.zeros(sh, np.float64)
        self.X, self.V, self.P = z(G, N, D), z(G, N, D), z(G, N, D)
        self.f, self.L, self.Pf, self.PL = z(G, N), z(G, N), z(G, N), z(G, N)
        self.Q = np.zeros((G, N), np.int32)
        self.PQ = np.zeros((G, N), np.int32)
        self.gbest_n = np.zeros(G, np.int32)
        self.gbest_f = z(G)
        self.s = OrcSwarm(G, N, W, sw.max_iters, float(width), float(height), _p(self.hyper),
                          float(sw.alpha), int(sw.beta), int(sw.seed), int(sw.instance),
                          _p(self.X), _p(self.V), _p(self.P), _p(self.f), _p(self.L),
                          _p(self.Q, ip), _p(self.Pf), _p(self.PL), _p(self.PQ, ip),
                          _p(self.gbest_n, ip), _p(self.gbest_f), 0, 0, float("inf"), 0, 0,
                          int(getattr(sw, "rand_per_dim", 0)))
        # online self-evolution state
        self.outer_hyper = np.ascontiguousarray(sw.hsef_hyper, dtype=np.float64).reshape(G, 6)
        self.ov, self.op, self.opf = z(G, 3), z(G, 3), np.full(G, np.inf)
        t_outer = -(-sw.max_iters // sw.hsef_every) if sw.hsef_every > 0 else 1
        self.h = OrcHsef(_p(self.outer_hyper), _p(self.ov), _p(self.op), _p(self.opf), 0, 0,
                         t_outer, 0)
        self.cfg = OrcFrameCfg(int(sw.use_pi), float(sw.pi_gamma), float(sw.pi_radius),
                               int(sw.at_mode), int(sw.at_window), float(sw.at_delta),
                               int(sw.hsef_every))
        self.hist = z(max(sw.max_iters, 1))
        self.prev_path = None

    # scalar state
    k = property(lambda self: self.s.k)
    ctr = property(lambda self: self.s.ctr)
    tbest = property(lambda self: (self.s.tbest_g, self.s.tbest_n, self.s.tbest_f))

    def init(self, frame=0, prev_path=None, gamma=0.25, radius=0.0):
        pp = None
        if prev_path is not None:
            self._pp = np.ascontiguousarray(prev_path, dtype=np.float64)
            pp = _p(self._pp)
        lib().orc_init(C.byref(self.s), int(frame), pp, float(gamma), float(radius))

    def eval(self, m: Map):
        lib().orc_eval(C.byref(self.s), C.byref(m.s))

    def bests(self):
        lib().orc_bests(C.byref(self.s))

    def update(self):
        lib().orc_update(C.byref(self.s))

    def step(self, m: Map, n=1):
        for _ in range(n):
            lib().orc_step(C.byref(self.s), C.byref(m.s))

    def hsef_reset_frame(self):
        lib().orc_hsef_reset_frame(C.byref(self.s), C.byref(self.h))

    def hsef_step(self):
        lib().orc_hsef_step(C.byref(self.s), C.byref(self.h))

    def plan_frame(self, m: Map, frame: int):
        D = self.D
        out = np.zeros(D)
        res = OrcFrameResult()
        pp = None
        if self.prev_path is not None:
            pp = _p(self.prev_path)
        lib().orc_plan_frame(C.byref(self.s), C.byref(self.h), C.byref(m.s), C.byref(self.cfg),
                             int(frame), pp, _p(out), _p(self.hist), C.byref(res))
        self.prev_path = out.copy()
        return dict(cost=res.cost, length=res.length, crossings=res.crossings, iters=res.iters,
                    truncated=res.truncated, path=out)

    def set_scalars(self, k=None, ctr=None, tbest=None):
        if k is not None:
            self.s.k = int(k)
        if ctr is not None:
            self.s.ctr = int(ctr)
        if tbest is not None:
            self.s.tbest_g, self.s.tbest_n, self.s.tbest_f = int(tbest[0]), int(tbest[1]), float(tbest[2])


def at_check(hist, k, mode, window, delta, q_tbest):
    h = np.ascontiguousarray(hist, dtype=np.float64)
    return lib().orc_at_check(_p(h), int(k), int(mode), int(window), float(delta), int(q_tbest))


def sim_step(spec):
    """Advance a MapSpec's obstacles and endpoints by one frame (in place)."""
    ptr = np.ascontiguousarray(spec.poly_ptr, dtype=np.int32)
    verts = np.ascontiguousarray(spec.verts, dtype=np.float64)
    vel = np.ascontiguousarray(spec.poly_vel, dtype=np.float64)
    s = np.ascontiguousarray(spec.start, dtype=np.float64)
    t = np.ascontiguousarray(spec.target, dtype=np.float64)
    ev = np.ascontiguousarray(spec.endpoint_vel, dtype=np.float64)
    lib().orc_sim_step(float(spec.width), float(spec.height), len(ptr) - 1, _p(ptr, ip),
                       _p(verts), _p(vel), _p(s), _p(t), _p(ev))
    spec.verts, spec.poly_vel, spec.start, spec.target, spec.endpoint_vel = verts, vel, s, t, ev
    return spec


def plan_static(spec, sw, iters=None):
    """Plain static plan (Algorithm 1 from a uniform swarm); returns the final
    Tbest fitness and the oracle swarm."""
    m = Map(spec)
    s = Swarm(sw, spec.width, spec.height)
    s.init(0)
    s.step(m, iters if iters is not None else sw.max_iters)
    return s.s.tbest_f, s


# ---------------------------------------------------------------------------
# learned initializer (MLP) oracle
def bf16(x):
    """Round-to-nearest-even BF16 of each value (FP64 in, FP64 out)."""
    L = lib()
    L.orc_bf16.argtypes = [C.c_double]
    L.orc_bf16.restype = C.c_double
    a = np.asarray(x, dtype=np.float64)
    return np.vectorize(L.orc_bf16, otypes=[np.float64])(a) if a.ndim else L.orc_bf16(float(a))


def mlp(sizes, W, b, x, target=None, round=True, grads=True):
    """FP64 MLP forward (+ backward when target given and grads).  W[l]:
    (sizes[l+1], sizes[l]); returns dict(y, loss, gW, gb, gWmag) -- gWmag[l]
    per weight-gradient element the same products run on magnitudes (|x|,
    |W|, |b| forward, 2 (Mag(y) + |t|) / (B n) backward through |W| with every
    unit kept), which bounds how far BF16 storage can move the element."""
    L = lib()
    nl = len(sizes) - 1
    sz = np.ascontiguousarray(sizes, dtype=np.int32)
    Wc = [np.ascontiguousarray(w, dtype=np.float64) for w in W]
    bc = [np.ascontiguousarray(v, dtype=np.float64) for v in b]
    x = np.ascontiguousarray(x, dtype=np.float64)
    B = x.shape[0]
    y = np.zeros((B, sizes[-1]))
    loss = C.c_double(0.0)
    Wp = (dp * nl)(*[_p(w) for w in Wc])
    bp = (dp * nl)(*[_p(v) for v in bc])
    tg = None
    if target is not None:
        tg = np.ascontiguousarray(target, dtype=np.float64)
    gW = [np.zeros_like(w) for w in Wc]
    gb = [np.zeros_like(v) for v in bc]
    do_g = grads and target is not None
    gWa = [np.zeros_like(w) for w in Wc]
    gWp = (dp * nl)(*[_p(w) for w in gW]) if do_g else None
    gbp = (dp * nl)(*[_p(v) for v in gb]) if do_g else None
    gWap = (dp * nl)(*[_p(w) for w in gWa]) if do_g else None
    L.orc_mlp.argtypes = [C.c_int32, ip, C.POINTER(dp), C.POINTER(dp), C.c_int32, dp, dp,
                          C.c_int32, dp, C.POINTER(C.c_double), C.POINTER(dp), C.POINTER(dp),
                          C.POINTER(dp)]
    L.orc_mlp(nl, _p(sz, ip), Wp, bp, B, _p(x), _p(tg) if tg is not None else None,
              int(bool(round)), _p(y), C.byref(loss), gWp, gbp, gWap)
    return dict(y=y, loss=loss.value if target is not None else None,
                gW=gW if do_g else None, gb=gb if do_g else None, gWmag=gWa if do_g else None)


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One FP64 Adam step (Kingma and Ba, ICLR 2015, Algorithm 1) in place on
    p, m, v (float64 arrays of one shape); t is the 1-based step index."""
    L = lib()
    L.orc_adam_step.argtypes = [C.c_int64, dp, dp, dp, dp, C.c_int32, C.c_double, C.c_double,
                                C.c_double, C.c_double]
    for a in (p, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    gc = np.ascontiguousarray(g, dtype=np.float64)
    assert gc.size == p.size == m.size == v.size
    L.orc_adam_step(p.size, _p(p), _p(gc), _p(m), _p(v), int(t), float(lr), float(b1), float(b2),
                    float(eps))


def raster(spec, n=64):
    L = lib()
    ptr = np.ascontiguousarray(spec.poly_ptr, dtype=np.int32)
    verts = np.ascontiguousarray(spec.verts, dtype=np.float64)
    out = np.zeros((n, n))
    L.orc_raster.argtypes = [C.c_double, C.c_double, C.c_int32, ip, dp, C.c_int32, dp]
    L.orc_raster(float(spec.width), float(spec.height), len(ptr) - 1, _p(ptr, ip), _p(verts),
                 int(n), _p(out))
    return out


# Table hyper8 (the paper's DTPSO / H-SEPSO defaults): rows = groups,
# columns = C1, C2, C3, w_init, w_end, V_limit.  The oracle's own copy of the
# printed table (tests check it against tests/golden/table_hyper8.txt).
HYPER8 = np.array([
    [2, 1, 1, 0.4, 0.2, 0.2],
    [1, 1, 2, 0.7, 0.3, 0.1],
    [2, 2, 1, 0.8, 0.1, 0.6],
    [2, 2, 1, 0.8, 0.6, 0.4],
    [2, 1, 2, 0.2, 0.1, 0.3],
    [2, 1, 2, 0.9, 0.5, 0.5],
    [1, 2, 2, 0.4, 0.1, 0.8],
    [1, 2, 2, 0.9, 0.3, 0.3],
], dtype=np.float64)

# Default per-column box of the evolved hyper-parameters (C1, C2, C3, w_init,
# w_end, V_limit); the paper does not state one.
EVOLVE_LO = np.array([0.0, 0.0, 0.0, 0.0, 0.0, 0.0])
EVOLVE_HI = np.array([3.0, 3.0, 3.0, 1.0, 1.0, 1.0])


class _HLevel:
    """Higher level of the evolution phase (H-SEPSO, Sec. "Hierarchical
    Self-evolving Framework", Eq.(9)), run by liborc: particle i is a whole
    (G_L, 6) lower-level hyper matrix, its fitness the LFV handed to step()."""

    def __init__(self, Gl, h_groups, h_particles, evolutions, seed, h_hyper, lo, hi):
        self.Gh, self.Nh, self.Dh = h_groups, h_particles, 6 * Gl
        n = h_groups * h_particles
        hh = HYPER8[np.arange(h_groups) % 8] if h_hyper is None else h_hyper
        self.h_hyper = np.ascontiguousarray(hh, dtype=np.float64).reshape(h_groups, 6).copy()
        self.lo = np.ascontiguousarray(EVOLVE_LO if lo is None else lo, dtype=np.float64).copy()
        self.hi = np.ascontiguousarray(EVOLVE_HI if hi is None else hi, dtype=np.float64).copy()
        z = lambda *sh: np.zeros(sh, np.float64)
        self.X, self.V, self.P = z(n, self.Dh), z(n, self.Dh), z(n, self.Dh)
        self.Pf = np.full(n, np.inf)
        self.gbest_n = np.zeros(h_groups, np.int32)
        self.gbest_f = np.full(h_groups, np.inf)
        self.h = OrcEvolve(h_groups, h_particles, self.Dh, evolutions, _p(self.h_hyper),
                           _p(self.lo), _p(self.hi), int(seed), _p(self.X), _p(self.V), _p(self.P),
                           _p(self.Pf), _p(self.gbest_n, ip), _p(self.gbest_f), 0, 0,
                           float("inf"), 0, 0)
        lib().orc_evolve_init(C.byref(self.h))
        self.evolution = 0

    k = property(lambda self: self.h.k)
    ctr = property(lambda self: self.h.ctr)
    tbest = property(lambda self: (self.h.tb_g, self.h.tb_n, self.h.tb_f))

    def step(self, lfv):
        v = np.ascontiguousarray(lfv, dtype=np.float64)
        lib().orc_evolve_step(C.byref(self.h), _p(v))

    def lfv(self, hyper_rows=None):
        raise NotImplementedError

    def evolve(self, n=1, hyper_cast=None):
        """n evolutions; hyper_cast maps the positions handed to the lower
        level (e.g. to FP32).  Returns the per-evolution total-best LFV."""
        curve = []
        for _ in range(n):
            rows = self.X if hyper_cast is None else hyper_cast(self.X)
            self.step(self.lfv(rows))
            self.evolution += 1
            curve.append(self.h.tb_f)
        return np.array(curve)


class Evolve(_HLevel):
    """Evolution phase for path planning: each H particle's fitness is the
    lowest fitness value of a full lower-level run (one oracle frame with
    truncation, priori initialisation and online evolution switched off) of
    its own persistent lower-level swarm, instance i, with the particle's
    values as the lower level's (G_L, 6) hyper matrix."""

    def __init__(self, spec, lsw, h_groups=8, h_particles=4, evolutions=500, seed=0,
                 h_hyper=None, lo=None, hi=None):
        import dataclasses
        super().__init__(lsw.groups, h_groups, h_particles, evolutions, seed, h_hyper, lo, hi)
        self.map = Map(spec)
        self.lower = []
        for i in range(h_groups * h_particles):
            sw = dataclasses.replace(lsw, instance=i, use_pi=0, at_mode=0, hsef_every=0)
            self.lower.append(Swarm(sw, spec.width, spec.height))

    def lfv(self, hyper_rows=None):
        """Lowest fitness value of every H particle's lower-level run at the
        current evolution (hyper_rows overrides the H positions)."""
        src = self.X if hyper_rows is None else hyper_rows
        out = np.empty(len(self.lower))
        for i, sw in enumerate(self.lower):
            sw.hyper[:] = src[i].reshape(sw.G, 6)
            out[i] = sw.plan_frame(self.map, self.evolution)["cost"]
        return out


class BFEvolve(_HLevel):
    """Evolution phase on a benchmark function (Sec. "Evolution Phase on
    Benchmark Functions"): H particle i's fitness is the lowest fitness value
    after `iters` evaluated iterations of a fresh DTPSO swarm (instance i,
    run = evolutions done) with the particle's values as its (G, 6) hyper
    matrix."""

    def __init__(self, func, groups, particles, dims, iters, h_groups=8, h_particles=4,
                 evolutions=500, lo=-600.0, hi=600.0, seed=0, h_seed=0, h_hyper=None, h_lo=None,
                 h_hi=None):
        super().__init__(groups, h_groups, h_particles, evolutions, h_seed, h_hyper, h_lo, h_hi)
        self.bf = (func, groups, particles, dims, iters, lo, hi, seed)

    def lower_run(self, i, hyper, run):
        func, G, N, D, T, lo, hi, seed = self.bf
        sw = BFSwarm(func, G, N, D, T, hyper, lo=lo, hi=hi, seed=seed, instance=i, run=run)
        sw.step(T)
        return sw

    def lfv(self, hyper_rows=None):
        src = self.X if hyper_rows is None else hyper_rows
        return np.array([self.lower_run(i, src[i], self.evolution).tbest[2]
                         for i in range(len(src))])


def bf_value(func, x):
    """Benchmark function `func` (1..4, Table BFs) of one point x (D,)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib().orc_bf_value(int(func), len(x), _p(x))


class BFSwarm:
    """DTPSO on a benchmark function (Table BFs) with numpy-owned state."""

    def __init__(self, func, groups, particles, dims, iters, hyper, lo=-600.0, hi=600.0, seed=0,
                 instance=0, run=0):
        G, N, D = groups, particles, dims
        self.G, self.N, self.D = G, N, D
        self.hyper = np.ascontiguousarray(hyper, dtype=np.float64).reshape(G, 6).copy()
        z = lambda *sh: np.zeros(sh, np.float64)
        self.X, self.V, self.P = z(G, N, D), z(G, N, D), z(G, N, D)
        self.f, self.Pf = z(G, N), z(G, N)
        self.gbest_n = np.zeros(G, np.int32)
        self.gbest_f = z(G)
        self.s = OrcBF(int(func), G, N, D, int(iters), float(lo), float(hi), _p(self.hyper),
                       int(seed), _p(self.X), _p(self.V), _p(self.P), _p(self.f), _p(self.Pf),
                       _p(self.gbest_n, ip), _p(self.gbest_f), 0, 0, float("inf"), 0, 0,
                       int(instance), int(run))
        lib().orc_bf_init(C.byref(self.s))

    k = property(lambda self: self.s.k)
    ctr = property(lambda self: self.s.ctr)
    tbest = property(lambda self: (self.s.tb_g, self.s.tb_n, self.s.tb_f))

    def step(self, n=1):
        for _ in range(n):
            lib().orc_bf_step(C.byref(self.s))

    def eval(self):
        lib().orc_bf_eval(C.byref(self.s))

    def advance(self):
        lib().orc_bf_advance(C.byref(self.s))

    def set_scalars(self, k=None, ctr=None, tbest=None):
        if k is not None:
            self.s.k = int(k)
        if ctr is not None:
            self.s.ctr = int(ctr)
        if tbest is not None:
            self.s.tb_g, self.s.tb_n, self.s.tb_f = int(tbest[0]), int(tbest[1]), float(tbest[2])
