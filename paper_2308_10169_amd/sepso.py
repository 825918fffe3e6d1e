"""Thin ctypes binding of libsepso (argument marshalling only).

Every step of the planner runs in the library's HIP kernels.  PyTorch is used
for the device workspace and the stream; it must own the HIP runtime in this
process, so it is imported (and initialised) before the library is loaded.
There is no CPU fallback: without the built library or a GPU this module
raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsepso.so")

OK, E_ARG, E_NOMEM, E_HIP, E_STATE, E_UNSUPPORTED = range(6)

fp = C.POINTER(C.c_float)
ip = C.POINTER(C.c_int32)


class SepsoError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libsepso status {status}: {msg}")
        self.status = status


class CMap(C.Structure):
    _fields_ = [("width", C.c_float), ("height", C.c_float), ("n_polys", C.c_int32),
                ("poly_ptr", ip), ("verts", fp), ("start", C.c_float * 2),
                ("target", C.c_float * 2), ("poly_vel", fp), ("endpoint_vel", C.c_float * 4)]


class CSwarm(C.Structure):
    _fields_ = [("groups", C.c_int32), ("particles", C.c_int32), ("waypoints", C.c_int32),
                ("max_iters", C.c_int32), ("hyper", fp), ("alpha", C.c_float),
                ("beta", C.c_int32), ("use_pi", C.c_int32), ("pi_gamma", C.c_float),
                ("pi_radius", C.c_float), ("at_mode", C.c_int32), ("at_window", C.c_int32),
                ("at_delta", C.c_float), ("hsef_every", C.c_int32), ("hsef_hyper", fp),
                ("seed", C.c_uint64), ("instance", C.c_uint32), ("rand_per_dim", C.c_int32)]


class CFrameResult(C.Structure):
    _fields_ = [("cost", C.c_float), ("length", C.c_float), ("crossings", C.c_int32),
                ("iters", C.c_int32), ("truncated", C.c_int32), ("used_learned", C.c_int32),
                ("device_ms", C.c_float)]


class CState(C.Structure):
    _fields_ = [("X", fp), ("V", fp), ("P", fp), ("f", fp), ("L", fp), ("Pf", fp), ("PL", fp),
                ("Q", ip), ("PQ", ip), ("gbest_n", ip), ("gbest_f", fp), ("hyper", fp),
                ("tbest_g", C.c_int32), ("tbest_n", C.c_int32), ("tbest_f", C.c_float),
                ("k", C.c_int32), ("ctr", C.c_uint32), ("frame", C.c_int32)]


class COuter(C.Structure):
    _fields_ = [("ov", fp), ("op", fp), ("opf", fp), ("otb", C.c_int32),
                ("epoch_in_frame", C.c_int32), ("epoch_ctr", C.c_uint32)]


class CTune(C.Structure):
    _fields_ = [("seg_per_thread", C.c_int32), ("block_threads", C.c_int32)]


class CBFCfg(C.Structure):
    _fields_ = [("func", C.c_int32), ("groups", C.c_int32), ("particles", C.c_int32),
                ("dims", C.c_int32), ("max_iters", C.c_int32), ("hyper", fp), ("lo", C.c_float),
                ("hi", C.c_float), ("seed", C.c_uint64), ("swarms", C.c_int32), ("path", C.c_int32)]


class CBFState(C.Structure):
    _fields_ = [("X", fp), ("V", fp), ("P", fp), ("f", fp), ("Pf", fp), ("gbest_n", ip),
                ("gbest_f", fp), ("tb_g", C.c_int32), ("tb_n", C.c_int32), ("tb_f", C.c_float),
                ("k", C.c_int32), ("ctr", C.c_uint32), ("pending", C.c_int32)]


class CEvolveCfg(C.Structure):
    _fields_ = [("h_groups", C.c_int32), ("h_particles", C.c_int32), ("evolutions", C.c_int32),
                ("h_hyper", fp), ("lo", fp), ("hi", fp), ("seed", C.c_uint64)]


class CEvolveState(C.Structure):
    _fields_ = [("X", fp), ("V", fp), ("P", fp), ("Pf", fp), ("lfv", fp), ("gbest_n", ip),
                ("gbest_f", fp), ("tb_g", C.c_int32), ("tb_n", C.c_int32), ("tb_f", C.c_float),
                ("k", C.c_int32), ("ctr", C.c_uint32)]


_lib = None
_torch = None


def _load():
    global _lib, _torch
    if _lib is not None:
        return _lib
    import torch  # owns the HIP runtime of this process
    if not torch.cuda.is_available():
        raise SepsoError(E_UNSUPPORTED, "no HIP device visible: libsepso needs an MI355X")
    torch.cuda.init()
    if not os.path.exists(LIB_PATH):
        raise SepsoError(E_UNSUPPORTED, f"{LIB_PATH} is not built (run __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    vp, sz = C.c_void_p, C.c_size_t
    L.sepso_last_error.restype = C.c_char_p
    L.sepso_version.restype = C.c_char_p
    L.sepso_workspace_bytes.argtypes = [C.POINTER(CMap), C.POINTER(CSwarm), C.POINTER(sz)]
    L.sepso_create.argtypes = [C.POINTER(CMap), C.POINTER(CSwarm), vp, sz, vp, C.POINTER(vp)]
    L.sepso_destroy.argtypes = [vp]
    L.sepso_step.argtypes = [vp, C.c_int32]
    L.sepso_reinit.argtypes = [vp, C.c_int32, C.c_int32]
    L.sepso_step_frame.argtypes = [vp, C.c_int32]
    L.sepso_get_outer.argtypes = [vp, C.POINTER(COuter)]
    L.sepso_set_outer.argtypes = [vp, C.POINTER(COuter)]
    L.sepso_plan_frame.argtypes = [vp, C.POINTER(CMap), C.POINTER(CFrameResult), fp]
    L.sepso_get_state.argtypes = [vp, C.POINTER(CState)]
    L.sepso_set_state.argtypes = [vp, C.POINTER(CState)]
    L.sepso_get_geometry.argtypes = [vp, fp, fp]
    L.sepso_profile_step.argtypes = [vp, C.c_int32, fp]
    L.sepso_set_tune.argtypes = [vp, C.POINTER(CTune)]
    L.sepso_autotune_ctx.argtypes = [vp, C.POINTER(CTune)]
    L.sepso_batch_workspace_bytes.argtypes = [C.POINTER(CMap), C.POINTER(CSwarm), C.c_int32,
                                              C.POINTER(sz)]
    L.sepso_batch_create.argtypes = [C.POINTER(CMap), C.POINTER(CSwarm), C.c_int32, vp, sz, vp,
                                     C.POINTER(CTune), C.POINTER(vp)]
    L.sepso_batch_destroy.argtypes = [vp]
    L.sepso_batch_path_offsets.argtypes = [vp, C.POINTER(C.c_int64)]
    L.sepso_batch_plan.argtypes = [vp, C.c_int32, C.POINTER(CFrameResult), fp]
    L.sepso_batch_get_state.argtypes = [vp, C.c_int32, C.POINTER(CState)]
    L.sepso_batch_profile_step.argtypes = [vp, C.c_int32, fp]
    L.sepso_philox.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64,
                               C.c_int64, vp, vp]
    L.sepso_autotune.argtypes = [vp, C.POINTER(CTune)]
    L.sepso_autotune_cached.argtypes = [vp, C.c_char_p, C.POINTER(CTune)]
    L.sepso_batch_work.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.sepso_batch_history.argtypes = [vp, fp]
    L.sepso_batch_set_tune.argtypes = [vp, C.POINTER(CTune)]
    L.sepso_batch_set_tiles.argtypes = [vp, C.c_int32, ip, C.POINTER(CTune)]
    L.sepso_autotune_buckets.argtypes = [vp, C.c_int32, C.c_char_p, C.POINTER(CTune), ip, ip, fp]
    L.sepso_bf_workspace_bytes.argtypes = [C.POINTER(CBFCfg), C.POINTER(sz)]
    L.sepso_bf_create.argtypes = [C.POINTER(CBFCfg), vp, sz, vp, C.POINTER(vp)]
    L.sepso_bf_destroy.argtypes = [vp]
    L.sepso_bf_step.argtypes = [vp, C.c_int32]
    L.sepso_bf_profile.argtypes = [vp, C.c_int32, fp]
    L.sepso_bf_get_state.argtypes = [vp, C.POINTER(CBFState)]
    L.sepso_bf_set_state.argtypes = [vp, C.POINTER(CBFState)]
    L.sepso_evolve_workspace_bytes.argtypes = [C.POINTER(CMap), C.POINTER(CSwarm),
                                               C.POINTER(CEvolveCfg), C.POINTER(sz)]
    L.sepso_evolve_create.argtypes = [C.POINTER(CMap), C.POINTER(CSwarm), C.POINTER(CEvolveCfg),
                                      vp, sz, vp, C.POINTER(vp)]
    L.sepso_evolve_destroy.argtypes = [vp]
    L.sepso_evolve_run.argtypes = [vp, C.c_int32, fp]
    L.sepso_evolve_inject.argtypes = [vp, fp]
    L.sepso_evolve_get_state.argtypes = [vp, C.POINTER(CEvolveState)]
    L.sepso_evolve_best.argtypes = [vp, fp, fp]
    L.sepso_evolve_lower.argtypes = [vp, C.POINTER(vp)]
    L.sepso_bf_evolve_workspace_bytes.argtypes = [C.POINTER(CBFCfg), C.POINTER(CEvolveCfg),
                                                  C.POINTER(sz)]
    L.sepso_bf_evolve_create.argtypes = [C.POINTER(CBFCfg), C.POINTER(CEvolveCfg), vp, sz, vp,
                                         C.POINTER(vp)]
    L.sepso_bf_evolve_destroy.argtypes = [vp]
    L.sepso_bf_evolve_run.argtypes = [vp, C.c_int32, fp]
    L.sepso_bf_evolve_get_state.argtypes = [vp, C.POINTER(CEvolveState)]
    L.sepso_bf_evolve_best.argtypes = [vp, fp, fp]
    L.sepso_bf_evolve_lower.argtypes = [vp, C.POINTER(vp)]
    L.sepso_lin_param_count.restype = C.c_int64
    L.sepso_lin_workspace_bytes.argtypes = [C.c_int32, C.c_int64, C.POINTER(sz)]
    L.sepso_lin_create.argtypes = [C.c_int32, C.c_int64, C.c_uint64, vp, sz, vp, C.POINTER(vp)]
    L.sepso_lin_destroy.argtypes = [vp]
    L.sepso_lin_set_weights.argtypes = [vp, fp]
    L.sepso_lin_get_weights.argtypes = [vp, fp]
    L.sepso_lin_forward.argtypes = [vp, fp, C.c_int32, fp]
    L.sepso_lin_grads.argtypes = [vp, fp, fp, C.c_int32, fp, fp]
    L.sepso_lin_collect.argtypes = [vp, vp]
    L.sepso_lin_samples.argtypes = [vp, C.POINTER(C.c_int64)]
    L.sepso_lin_train.argtypes = [vp, C.c_int32, C.c_int32, C.c_float, fp]
    L.sepso_lin_features.argtypes = [vp, vp, fp]
    L.sepso_lin_attach.argtypes = [vp, vp]
    L.sepso_lin_attach_ctx.argtypes = [vp, vp]
    L.sepso_fitness_workspace_bytes.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.POINTER(sz)]
    L.sepso_fitness.argtypes = [C.c_int32, C.c_int32, vp, vp, vp, vp, C.c_int32, C.c_int32,
                                C.c_float, C.c_int32, vp, vp, vp, vp, sz, vp]
    L.sepso_fitness_noalloc.argtypes = [C.c_int32, C.c_int32, vp, vp, vp, vp, C.c_int32,
                                        C.c_int32, C.c_float, C.c_int32, vp, vp, vp, vp]
    _lib, _torch = L, torch
    return L


def lib():
    return _load()


def philox(first, c1, c2, c3, key, n):
    """n Philox4x32-10 blocks of counters (first + i, c1, c2, c3) under the
    64-bit key, computed by the library on the GPU: (n, 4) uint32."""
    _load()
    torch = _torch
    out = torch.empty((max(int(n), 1), 4), dtype=torch.int32, device="cuda")
    st = torch.cuda.current_stream()
    _check(_lib.sepso_philox(int(first) & 0xFFFFFFFF, int(c1) & 0xFFFFFFFF, int(c2) & 0xFFFFFFFF,
                             int(c3) & 0xFFFFFFFF, int(key) & (2**64 - 1), int(n),
                             C.c_void_p(out.data_ptr()), C.c_void_p(st.cuda_stream)))
    st.synchronize()
    return out[:int(n)].cpu().numpy().view(np.uint32)


def fitness(spec, paths, waypoints, alpha, beta, noalloc=False):
    """sepso_fitness (or, with noalloc, sepso_fitness_noalloc) on device
    copies of the map's polygons and endpoints and of paths (n, 2W):
    returns dict(f, L, Q) as numpy arrays."""
    _load()
    torch = _torch
    W = int(waypoints)
    dev = "cuda"
    pp = torch.from_numpy(np.ascontiguousarray(spec.poly_ptr, dtype=np.int32)).to(dev)
    vv = torch.from_numpy(_f32(spec.verts).reshape(-1)).to(dev)
    ee = torch.from_numpy(_f32(list(spec.start) + list(spec.target))).to(dev)
    X = torch.from_numpy(_f32(paths).reshape(-1, 2 * W)).to(dev)
    n = X.shape[0]
    n_polys, n_vert = len(spec.poly_ptr) - 1, int(spec.poly_ptr[-1])
    f = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
    Lv = torch.empty_like(f)
    Q = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    st = torch.cuda.current_stream()
    ptr = lambda t: C.c_void_p(t.data_ptr())
    if noalloc:
        _check(_lib.sepso_fitness_noalloc(n_polys, n_vert, ptr(pp), ptr(vv), ptr(ee), ptr(X), n, W,
                                          float(alpha), int(beta), ptr(f), ptr(Lv), ptr(Q),
                                          C.c_void_p(st.cuda_stream)))
    else:
        nbytes = C.c_size_t()
        _check(_lib.sepso_fitness_workspace_bytes(n_vert, n, W, C.byref(nbytes)))
        ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=dev)
        _check(_lib.sepso_fitness(n_polys, n_vert, ptr(pp), ptr(vv), ptr(ee), ptr(X), n, W,
                                  float(alpha), int(beta), ptr(f), ptr(Lv), ptr(Q), ptr(ws),
                                  nbytes.value, C.c_void_p(st.cuda_stream)))
    st.synchronize()
    return dict(f=f[:n].cpu().numpy(), L=Lv[:n].cpu().numpy(), Q=Q[:n].cpu().numpy())


def _check(st):
    if st != OK:
        raise SepsoError(st, _lib.sepso_last_error().decode())


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64), dtype=np.float32)


class _MapArgs:
    """Keeps the arrays behind a CMap alive."""

    def __init__(self, spec: "I.MapSpec"):
        self.pptr = np.ascontiguousarray(spec.poly_ptr, dtype=np.int32)
        self.verts = _f32(spec.verts).reshape(-1)
        self.vel = _f32(spec.poly_vel).reshape(-1)
        n_polys = len(self.pptr) - 1
        self.c = CMap(float(spec.width), float(spec.height), n_polys,
                      self.pptr.ctypes.data_as(ip), self.verts.ctypes.data_as(fp),
                      (C.c_float * 2)(*spec.start), (C.c_float * 2)(*spec.target),
                      self.vel.ctypes.data_as(fp) if n_polys else None,
                      (C.c_float * 4)(*spec.endpoint_vel))


class _SwarmArgs:
    def __init__(self, sw: "I.SwarmSpec"):
        self.hyper = _f32(sw.hyper).reshape(-1)
        self.hsef = _f32(sw.hsef_hyper).reshape(-1)
        self.c = CSwarm(sw.groups, sw.particles, sw.waypoints, sw.max_iters,
                        self.hyper.ctypes.data_as(fp), float(sw.alpha), int(sw.beta),
                        int(sw.use_pi), float(sw.pi_gamma), float(sw.pi_radius), int(sw.at_mode),
                        int(sw.at_window), float(sw.at_delta), int(sw.hsef_every),
                        self.hsef.ctypes.data_as(fp), int(sw.seed), int(sw.instance),
                        int(getattr(sw, "rand_per_dim", 0)))


def _result(r):
    return dict(cost=r.cost, length=r.length, crossings=r.crossings, iters=r.iters,
                truncated=r.truncated, used_learned=r.used_learned, device_ms=r.device_ms)


def _state_buffers(G, N, W):
    D = 2 * W
    z = lambda *s: np.zeros(s, np.float32)
    zi = lambda *s: np.zeros(s, np.int32)
    return dict(X=z(G, N, D), V=z(G, N, D), P=z(G, N, D), f=z(G, N), L=z(G, N), Pf=z(G, N),
                PL=z(G, N), Q=zi(G, N), PQ=zi(G, N), gbest_n=zi(G), gbest_f=z(G),
                hyper=z(G, 6))


def _cstate(bufs, scal=None):
    cs = CState()
    for k, v in bufs.items():
        if v is not None:
            setattr(cs, k, v.ctypes.data_as(ip if v.dtype == np.int32 else fp))
    if scal:
        for k, v in scal.items():
            setattr(cs, k, v)
    return cs


class Planner:
    """One planner instance (sepso_ctx)."""

    def __init__(self, spec, sw, stream=None):
        L = _load()
        torch = _torch
        self.spec, self.sw = spec, sw
        self._m, self._s = _MapArgs(spec), _SwarmArgs(sw)
        nbytes = C.c_size_t()
        _check(L.sepso_workspace_bytes(C.byref(self._m.c), C.byref(self._s.c), C.byref(nbytes)))
        self.ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.Stream()
        h = C.c_void_p()
        _check(L.sepso_create(C.byref(self._m.c), C.byref(self._s.c), C.c_void_p(self.ws.data_ptr()),
                              nbytes.value, C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            _check(_lib.sepso_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        _check(_lib.sepso_step(self.h, int(n)))

    def step_frame(self, n=1):
        """n iterations of the current frame (AT and online HSEF included)."""
        _check(_lib.sepso_step_frame(self.h, int(n)))

    def get_outer(self):
        G = self.sw.groups
        o = dict(ov=np.zeros((G, 3), np.float32), op=np.zeros((G, 3), np.float32),
                 opf=np.zeros(G, np.float32))
        c = COuter(o["ov"].ctypes.data_as(fp), o["op"].ctypes.data_as(fp),
                   o["opf"].ctypes.data_as(fp), 0, 0, 0)
        _check(_lib.sepso_get_outer(self.h, C.byref(c)))
        o.update(otb=c.otb, epoch_in_frame=c.epoch_in_frame, epoch_ctr=c.epoch_ctr)
        return o

    def set_outer(self, o):
        a = {k: np.ascontiguousarray(o[k], dtype=np.float32) for k in ("ov", "op", "opf")}
        c = COuter(a["ov"].ctypes.data_as(fp), a["op"].ctypes.data_as(fp),
                   a["opf"].ctypes.data_as(fp), int(o["otb"]), int(o["epoch_in_frame"]),
                   int(o["epoch_ctr"]))
        _check(_lib.sepso_set_outer(self.h, C.byref(c)))

    def reinit(self, frame=0, use_prev=False):
        _check(_lib.sepso_reinit(self.h, int(frame), int(bool(use_prev))))

    def synchronize(self):
        self.stream.synchronize()

    def plan_frame(self, next_map=None):
        res = CFrameResult()
        path = np.zeros(2 * self.sw.waypoints, np.float32)
        m = _MapArgs(next_map) if next_map is not None else None
        _check(_lib.sepso_plan_frame(self.h, C.byref(m.c) if m else None, C.byref(res),
                                     path.ctypes.data_as(fp)))
        out = _result(res)
        out["path"] = path
        return out

    def get_state(self):
        b = _state_buffers(self.sw.groups, self.sw.particles, self.sw.waypoints)
        cs = _cstate(b)
        _check(_lib.sepso_get_state(self.h, C.byref(cs)))
        b.update(tbest=(cs.tbest_g, cs.tbest_n, cs.tbest_f), k=cs.k, ctr=cs.ctr, frame=cs.frame)
        return b

    def set_state(self, st):
        keys = ("X", "V", "P", "f", "L", "Pf", "PL", "Q", "PQ", "gbest_n", "gbest_f", "hyper")
        bufs = {}
        for k in keys:
            if k in st and st[k] is not None:
                dt = np.int32 if k in ("Q", "PQ", "gbest_n") else np.float32
                bufs[k] = np.ascontiguousarray(st[k], dtype=dt)
        tb = st.get("tbest", (0, 0, float("inf")))
        cs = _cstate(bufs, dict(tbest_g=int(tb[0]), tbest_n=int(tb[1]), tbest_f=float(tb[2]),
                                k=int(st.get("k", 0)), ctr=int(st.get("ctr", 0)),
                                frame=int(st.get("frame", 0))))
        _check(_lib.sepso_set_state(self.h, C.byref(cs)))

    def geometry(self):
        nv = int(self.spec.poly_ptr[-1])
        v = np.zeros(max(2 * nv, 1), np.float32)
        e = np.zeros(4, np.float32)
        _check(_lib.sepso_get_geometry(self.h, v.ctypes.data_as(fp), e.ctypes.data_as(fp)))
        return v[:2 * nv].reshape(-1, 2), e

    def profile_step(self, n=10):
        ms = C.c_float()
        _check(_lib.sepso_profile_step(self.h, int(n), C.byref(ms)))
        return ms.value

    def set_tune(self, K, B):
        _check(_lib.sepso_set_tune(self.h, C.byref(CTune(int(K), int(B)))))

    def autotune(self):
        t = CTune()
        _check(_lib.sepso_autotune_ctx(self.h, C.byref(t)))
        return (t.seg_per_thread, t.block_threads)


class BatchPlanner:
    """Many independent planner instances in one set of launches (sepso_batch)."""

    def __init__(self, specs, sws, tune=None, stream=None):
        L = _load()
        torch = _torch
        n = len(specs)
        self.specs, self.sws, self.n = specs, sws, n
        self._m = [_MapArgs(s) for s in specs]
        self._s = [_SwarmArgs(s) for s in sws]
        self._cm = (CMap * n)(*[m.c for m in self._m])
        self._cs = (CSwarm * n)(*[s.c for s in self._s])
        nbytes = C.c_size_t()
        _check(L.sepso_batch_workspace_bytes(self._cm, self._cs, n, C.byref(nbytes)))
        self.ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.Stream()
        t = CTune(*tune) if tune is not None else None
        h = C.c_void_p()
        _check(L.sepso_batch_create(self._cm, self._cs, n, C.c_void_p(self.ws.data_ptr()),
                                    nbytes.value, C.c_void_p(self.stream.cuda_stream),
                                    C.byref(t) if t else None, C.byref(h)))
        self.h = h
        off = (C.c_int64 * (n + 1))()
        _check(L.sepso_batch_path_offsets(h, off))
        self.path_off = np.array(off[:], dtype=np.int64)

    def close(self):
        if self.h:
            _check(_lib.sepso_batch_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def plan(self, n_frames=1, want_paths=False):
        res = (CFrameResult * (self.n * n_frames))()
        paths = np.zeros(max(int(self.path_off[-1]), 1), np.float32) if want_paths else None
        _check(_lib.sepso_batch_plan(self.h, int(n_frames), res,
                                     paths.ctypes.data_as(fp) if want_paths else None))
        cost = np.array([r.cost for r in res], np.float64).reshape(n_frames, self.n)
        iters = np.array([r.iters for r in res], np.int32).reshape(n_frames, self.n)
        q = np.array([r.crossings for r in res], np.int32).reshape(n_frames, self.n)
        trunc = np.array([r.truncated for r in res], np.int32).reshape(n_frames, self.n)
        out = dict(cost=cost, iters=iters, crossings=q, truncated=trunc)
        if want_paths:
            out["paths"] = [paths[self.path_off[i]:self.path_off[i + 1]] for i in range(self.n)]
        return out

    def get_state(self, i):
        sw = self.sws[i]
        b = _state_buffers(sw.groups, sw.particles, sw.waypoints)
        cs = _cstate(b)
        _check(_lib.sepso_batch_get_state(self.h, int(i), C.byref(cs)))
        b.update(tbest=(cs.tbest_g, cs.tbest_n, cs.tbest_f), k=cs.k, ctr=cs.ctr, frame=cs.frame)
        return b

    def profile_step(self, n=10):
        ms = C.c_float()
        _check(_lib.sepso_batch_profile_step(self.h, int(n), C.byref(ms)))
        return ms.value

    def set_tiles(self, bucket_of, tiles):
        """Tiles per bucket: bucket_of[i] is instance i's bucket, tiles[j] =
        (K, block_threads) of bucket j."""
        bo = np.ascontiguousarray(bucket_of, dtype=np.int32)
        tl = (CTune * len(tiles))(*[CTune(int(k), int(b)) for k, b in tiles])
        _check(_lib.sepso_batch_set_tiles(self.h, len(tiles), bo.ctypes.data_as(ip), tl))

    def autotune_buckets(self, max_buckets=4, cache_path=None, frame_ms=False):
        """Per-bucket tiles by the autotuner: returns (tiles, bucket_of) --
        one tile in the list when a single tile for all instances planned its
        frame faster -- and, with frame_ms, the two frames' device times
        (buckets, one tile)."""
        tl = (CTune * max_buckets)()
        bo = np.zeros(self.n, np.int32)
        nb = C.c_int32()
        ms = np.zeros(2, np.float32)
        _check(_lib.sepso_autotune_buckets(self.h, int(max_buckets),
                                           cache_path.encode() if cache_path else None, tl,
                                           bo.ctypes.data_as(ip), C.byref(nb),
                                           ms.ctypes.data_as(fp)))
        tiles = [(tl[j].seg_per_thread, tl[j].block_threads) for j in range(nb.value)]
        return (tiles, bo, tuple(float(v) for v in ms)) if frame_ms else (tiles, bo)

    def autotune(self, cache_path=None):
        """Time the tile candidates (or take this batch's entry of the tune
        cache file cache_path, appending one when it has none)."""
        t = CTune()
        if cache_path is None:
            _check(_lib.sepso_autotune(self.h, C.byref(t)))
        else:
            _check(_lib.sepso_autotune_cached(self.h, os.fsencode(cache_path), C.byref(t)))
        return (t.seg_per_thread, t.block_threads)

    def work(self):
        a, b = C.c_double(), C.c_double()
        _check(_lib.sepso_batch_work(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def history(self):
        """Tbest fitness after each iteration of the last frame (n, 64)."""
        out = np.zeros((self.n, 64), np.float32)
        _check(_lib.sepso_batch_history(self.h, out.ctypes.data_as(fp)))
        return out

    def attach(self, lin):
        _check(_lib.sepso_lin_attach(self.h, lin.h if lin is not None else None))

    def set_tune(self, K, B):
        _check(_lib.sepso_batch_set_tune(self.h, C.byref(CTune(int(K), int(B)))))


class Evolver:
    """Evolution phase (sepso_evolve): H-SEPSO over whole lower-level hyper
    matrices, each H particle's fitness the LFV of a full lower-level run of
    its own batch instance."""

    def __init__(self, spec, lower, h_groups=8, h_particles=8, evolutions=500, seed=0,
                 h_hyper=None, lo=None, hi=None, stream=None):
        L = _load()
        torch = _torch
        self.spec, self.lower = spec, lower
        self.n, self.Dh = h_groups * h_particles, 6 * lower.groups
        self.Gh, self.E = h_groups, evolutions
        self._m, self._s = _MapArgs(spec), _SwarmArgs(lower)
        self._keep = [None if a is None else _f32(a).reshape(-1) for a in (h_hyper, lo, hi)]
        ptr = lambda a: a.ctypes.data_as(fp) if a is not None else None
        self._cfg = CEvolveCfg(h_groups, h_particles, evolutions, *[ptr(a) for a in self._keep],
                               int(seed))
        nbytes = C.c_size_t()
        _check(L.sepso_evolve_workspace_bytes(C.byref(self._m.c), C.byref(self._s.c),
                                              C.byref(self._cfg), C.byref(nbytes)))
        self.ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.Stream()
        h = C.c_void_p()
        _check(L.sepso_evolve_create(C.byref(self._m.c), C.byref(self._s.c), C.byref(self._cfg),
                                     C.c_void_p(self.ws.data_ptr()), nbytes.value,
                                     C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        b = C.c_void_p()
        _check(L.sepso_evolve_lower(h, C.byref(b)))
        self._lower_h = b

    def close(self):
        if self.h:
            _check(_lib.sepso_evolve_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, n=1):
        """n evolutions; returns the total-best LFV after each."""
        out = np.zeros(max(int(n), 1), np.float32)
        done = 0
        while done < n:
            m = min(n - done, self.E)
            _check(_lib.sepso_evolve_run(self.h, int(m), out[done:].ctypes.data_as(fp)))
            done += m
        return out[:n]

    def inject(self, lfv):
        v = np.ascontiguousarray(lfv, dtype=np.float32)
        assert v.size == self.n
        _check(_lib.sepso_evolve_inject(self.h, v.ctypes.data_as(fp)))

    def get_state(self):
        z = lambda *sh: np.zeros(sh, np.float32)
        b = dict(X=z(self.n, self.Dh), V=z(self.n, self.Dh), P=z(self.n, self.Dh), Pf=z(self.n),
                 lfv=z(self.n), gbest_n=np.zeros(self.Gh, np.int32), gbest_f=z(self.Gh))
        cs = CEvolveState()
        for k, v in b.items():
            setattr(cs, k, v.ctypes.data_as(ip if v.dtype == np.int32 else fp))
        _check(_lib.sepso_evolve_get_state(self.h, C.byref(cs)))
        b.update(tbest=(cs.tb_g, cs.tb_n, cs.tb_f), k=cs.k, ctr=cs.ctr)
        return b

    def best(self):
        hyper = np.zeros(self.Dh, np.float32)
        f = C.c_float()
        _check(_lib.sepso_evolve_best(self.h, hyper.ctypes.data_as(fp), C.byref(f)))
        return hyper.reshape(-1, 6), f.value

    def lower_state(self, i):
        sw = self.lower
        b = _state_buffers(sw.groups, sw.particles, sw.waypoints)
        cs = _cstate(b)
        _check(_lib.sepso_batch_get_state(self._lower_h, int(i), C.byref(cs)))
        b.update(tbest=(cs.tbest_g, cs.tbest_n, cs.tbest_f), k=cs.k, ctr=cs.ctr, frame=cs.frame)
        return b

    def set_tune(self, K, B):
        _check(_lib.sepso_batch_set_tune(self._lower_h, C.byref(CTune(int(K), int(B)))))

    def autotune(self):
        t = CTune()
        _check(_lib.sepso_autotune(self._lower_h, C.byref(t)))
        return (t.seg_per_thread, t.block_threads)


BF_FUNCS = {"sphere": 1, "rosenbrock": 2, "rastrigin": 3, "griewank": 4}


class BFSwarm:
    """DTPSO on a benchmark function of Table BFs (sepso_bf); with swarms > 1,
    that many independent swarms of `groups` groups stepped together."""

    def __init__(self, func, groups, particles, dims, iters, hyper, lo=-600.0, hi=600.0, seed=0,
                 stream=None, swarms=1, stepwise=False):
        L = _load()
        torch = _torch
        self.S, self.Gs = swarms, groups
        self.G, self.N, self.D = swarms * groups, particles, dims
        self._hyper = _f32(hyper).reshape(-1)
        f = BF_FUNCS.get(func, func)
        self._cfg = CBFCfg(int(f), groups, particles, dims, iters,
                           self._hyper.ctypes.data_as(fp), float(lo), float(hi), int(seed),
                           int(swarms), int(bool(stepwise)))
        nbytes = C.c_size_t()
        _check(L.sepso_bf_workspace_bytes(C.byref(self._cfg), C.byref(nbytes)))
        self.ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.Stream()
        h = C.c_void_p()
        _check(L.sepso_bf_create(C.byref(self._cfg), C.c_void_p(self.ws.data_ptr()), nbytes.value,
                                 C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self._owned = True

    @classmethod
    def borrowed(cls, h, swarms, groups, particles, dims):
        """View of a handle owned elsewhere (an evolution's lower level)."""
        self = cls.__new__(cls)
        self.S, self.Gs = swarms, groups
        self.G, self.N, self.D = swarms * groups, particles, dims
        self.h, self._owned = h, False
        return self

    def close(self):
        if self.h and self._owned:
            _check(_lib.sepso_bf_destroy(self.h))
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def swarm_best(self, st=None):
        """Each swarm's lowest fitness value (from a state dict or read now)."""
        st = self.get_state(rows=False) if st is None else st
        return st["gbest_f"].reshape(self.S, self.Gs).min(axis=1)

    def step(self, n=1):
        _check(_lib.sepso_bf_step(self.h, int(n)))

    def profile(self, n):
        ms = C.c_float()
        _check(_lib.sepso_bf_profile(self.h, int(n), C.byref(ms)))
        return ms.value

    def get_state(self, rows=True):
        G, N, D = self.G, self.N, self.D
        z = lambda *sh: np.zeros(sh, np.float32)
        b = dict(f=z(G, N), Pf=z(G, N), gbest_n=np.zeros(G, np.int32), gbest_f=z(G))
        if rows:
            b.update(X=z(G, N, D), V=z(G, N, D), P=z(G, N, D))
        cs = CBFState()
        for k, v in b.items():
            setattr(cs, k, v.ctypes.data_as(ip if v.dtype == np.int32 else fp))
        _check(_lib.sepso_bf_get_state(self.h, C.byref(cs)))
        b.update(tbest=(cs.tb_g, cs.tb_n, cs.tb_f), k=cs.k, ctr=cs.ctr, pending=cs.pending)
        return b

    def set_state(self, st):
        cs = CBFState()
        keep = {}
        for k in ("X", "V", "P", "f", "Pf", "gbest_f", "gbest_n"):
            if st.get(k) is not None:
                dt = np.int32 if k == "gbest_n" else np.float32
                keep[k] = np.ascontiguousarray(st[k], dtype=dt)
                setattr(cs, k, keep[k].ctypes.data_as(ip if dt == np.int32 else fp))
        cs.k, cs.ctr, cs.pending = int(st.get("k", 0)), int(st.get("ctr", 0)), int(st.get("pending", 0))
        _check(_lib.sepso_bf_set_state(self.h, C.byref(cs)))


class BFEvolver:
    """Evolution phase on a benchmark function (sepso_bf_evolve): H-SEPSO
    over (groups, 6) hyper matrices, each H particle's fitness the LFV of a
    fresh `iters`-iteration run of its own lower-level swarm."""

    def __init__(self, func, groups, particles, dims, iters, h_groups=8, h_particles=4,
                 evolutions=500, lo=-600.0, hi=600.0, seed=0, h_seed=0, h_hyper=None, h_lo=None,
                 h_hi=None, stream=None, stepwise=False):
        L = _load()
        torch = _torch
        self.n, self.Dh, self.Gh, self.E = h_groups * h_particles, 6 * groups, h_groups, evolutions
        self.shape = (groups, particles, dims)
        f = BF_FUNCS.get(func, func)
        self._lcfg = CBFCfg(int(f), groups, particles, dims, iters, None, float(lo), float(hi),
                            int(seed), 0, int(bool(stepwise)))
        self._keep = [None if a is None else _f32(a).reshape(-1) for a in (h_hyper, h_lo, h_hi)]
        ptr = lambda a: a.ctypes.data_as(fp) if a is not None else None
        self._cfg = CEvolveCfg(h_groups, h_particles, evolutions, *[ptr(a) for a in self._keep],
                               int(h_seed))
        nbytes = C.c_size_t()
        _check(L.sepso_bf_evolve_workspace_bytes(C.byref(self._lcfg), C.byref(self._cfg),
                                                 C.byref(nbytes)))
        self.ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.Stream()
        h = C.c_void_p()
        _check(L.sepso_bf_evolve_create(C.byref(self._lcfg), C.byref(self._cfg),
                                        C.c_void_p(self.ws.data_ptr()), nbytes.value,
                                        C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        b = C.c_void_p()
        _check(L.sepso_bf_evolve_lower(h, C.byref(b)))
        self.lower = BFSwarm.borrowed(b, self.n, groups, particles, dims)

    def close(self):
        if self.h:
            self.lower.h = None
            _check(_lib.sepso_bf_evolve_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, n=1):
        """n evolutions; returns the total-best LFV after each."""
        out = np.zeros(max(int(n), 1), np.float32)
        done = 0
        while done < n:
            m = min(n - done, self.E)
            _check(_lib.sepso_bf_evolve_run(self.h, int(m), out[done:].ctypes.data_as(fp)))
            done += m
        return out[:n]

    def get_state(self):
        z = lambda *sh: np.zeros(sh, np.float32)
        b = dict(X=z(self.n, self.Dh), V=z(self.n, self.Dh), P=z(self.n, self.Dh), Pf=z(self.n),
                 lfv=z(self.n), gbest_n=np.zeros(self.Gh, np.int32), gbest_f=z(self.Gh))
        cs = CEvolveState()
        for k, v in b.items():
            setattr(cs, k, v.ctypes.data_as(ip if v.dtype == np.int32 else fp))
        _check(_lib.sepso_bf_evolve_get_state(self.h, C.byref(cs)))
        b.update(tbest=(cs.tb_g, cs.tb_n, cs.tb_f), k=cs.k, ctr=cs.ctr)
        return b

    def best(self):
        hyper = np.zeros(self.Dh, np.float32)
        f = C.c_float()
        _check(_lib.sepso_bf_evolve_best(self.h, hyper.ctypes.data_as(fp), C.byref(f)))
        return hyper.reshape(-1, 6), f.value


LIN_IN, LIN_OUT, LIN_HIDDEN = 4100, 320, 512


class LearnedInit:
    """Learned initializer (sepso_lin): BF16 MLP trained and run by the
    library's MFMA kernels."""

    def __init__(self, max_rows=1024, max_samples=0, seed=0, stream=None):
        L = _load()
        torch = _torch
        nbytes = C.c_size_t()
        _check(L.sepso_lin_workspace_bytes(int(max_rows), int(max_samples), C.byref(nbytes)))
        self.ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.Stream()
        h = C.c_void_p()
        _check(L.sepso_lin_create(int(max_rows), int(max_samples), int(seed),
                                  C.c_void_p(self.ws.data_ptr()), nbytes.value,
                                  C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self.max_rows = max_rows
        self.n_params = int(L.sepso_lin_param_count())

    def close(self):
        if self.h:
            _check(_lib.sepso_lin_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_weights(self):
        w = np.zeros(self.n_params, np.float32)
        _check(_lib.sepso_lin_get_weights(self.h, w.ctypes.data_as(fp)))
        return w

    def set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        _check(_lib.sepso_lin_set_weights(self.h, w.ctypes.data_as(fp)))

    def forward(self, x):
        x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, LIN_IN)
        y = np.zeros((len(x), LIN_OUT), np.float32)
        _check(_lib.sepso_lin_forward(self.h, x.ctypes.data_as(fp), len(x), y.ctypes.data_as(fp)))
        return y

    def grads(self, x, t):
        x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, LIN_IN)
        t = np.ascontiguousarray(t, dtype=np.float32).reshape(-1, LIN_OUT)
        g = np.zeros(self.n_params, np.float32)
        loss = C.c_float()
        _check(_lib.sepso_lin_grads(self.h, x.ctypes.data_as(fp), t.ctypes.data_as(fp), len(x),
                                    C.byref(loss), g.ctypes.data_as(fp)))
        return loss.value, g

    def collect(self, batch):
        _check(_lib.sepso_lin_collect(self.h, batch.h))

    def samples(self):
        n = C.c_int64()
        _check(_lib.sepso_lin_samples(self.h, C.byref(n)))
        return n.value

    def train(self, steps, batch=256, lr=1e-3):
        loss = np.zeros(steps, np.float32)
        _check(_lib.sepso_lin_train(self.h, int(steps), int(batch), float(lr),
                                    loss.ctypes.data_as(fp)))
        return loss

    def features(self, batch):
        out = np.zeros((batch.n, LIN_IN), np.float32)
        _check(_lib.sepso_lin_features(self.h, batch.h, out.ctypes.data_as(fp)))
        return out


def split_params(flat):
    """Flat parameter vector -> ([W1..W4], [b1..b4]) views (out, in)."""
    sizes = [LIN_IN, LIN_HIDDEN, LIN_HIDDEN, LIN_HIDDEN, LIN_OUT]
    W, b, o = [], [], 0
    for l in range(4):
        n_in, n_out = sizes[l], sizes[l + 1]
        W.append(flat[o:o + n_in * n_out].reshape(n_out, n_in))
        o += n_in * n_out
        b.append(flat[o:o + n_out])
        o += n_out
    return W, b
