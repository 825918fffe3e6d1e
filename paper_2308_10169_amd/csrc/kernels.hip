// libsepso device code (gfx950, FP32 VALU).
//
// Kernels:
//   geom_kernel  -- obstacle/endpoint motion for one frame and the derived
//                   per-edge records the fitness test reads;
//   init_kernel  -- uniform swarm and Priori Initialization;
//   step_kernel  -- one fused DTPSO iteration per launch: the previous
//                   iteration's velocity/position update (Eq.(6)-(8)), the
//                   path fitness (Eq.(11)-(13)), the Pbest update and a tile
//                   argmin; the last block of each instance to finish reduces
//                   the group and total bests and runs Auto Truncation and
//                   the online hierarchical self-evolution step.
#include "common.h"
#include "kernels.h"

namespace sepso {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// multiplies by fixed odd constants; high halves are xor-mixed with the other
// two counter words and the round key, the key advances by two Weyl constants.
// ---------------------------------------------------------------------------
struct U4 {
  uint32_t v[4];
};

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return U4{{c0, c1, c2, c3}};
}

// 24-bit uniform in [0,1), exact in FP32.
__device__ __forceinline__ float u01(uint32_t w) { return (float)(w >> 8) * 5.9604644775390625e-8f; }

__device__ __forceinline__ float clampf(float x, float lo, float hi) {
  return x < lo ? lo : (x > hi ? hi : x);
}

__device__ __forceinline__ bool better(float fa, int na, float fb, int nb) {
  return fa < fb || (fa == fb && na < nb);
}

// ---------------------------------------------------------------------------
// Geometry: obstacles translate by their per-frame velocity and bounce off
// the map border (velocity component reversed, overshoot mirrored); start
// and target move the same way.  All inputs lie on a 1/256 grid, so every
// operation here is exact in FP32.  Then the per-edge records are derived.
// ---------------------------------------------------------------------------
__device__ void bounce(float* c, int n, int stride, float* vel, float hi) {
  float mn = c[0], mx = c[0];
  for (int i = 1; i < n; ++i) {
    mn = fminf(mn, c[i * stride]);
    mx = fmaxf(mx, c[i * stride]);
  }
  float shift = 0.f;
  if (mn < 0.f)
    shift = -2.f * mn;
  else if (mx > hi)
    shift = -2.f * (mx - hi);
  if (shift != 0.f) {
    for (int i = 0; i < n; ++i) c[i * stride] += shift;
    *vel = -*vel;
  }
}

__global__ __launch_bounds__(256) void geom_kernel(Pools pl, int move) {
  const int inst = blockIdx.x;
  const InstDesc& d = pl.desc[inst];
  const int t = threadIdx.x;
  float2* verts = pl.verts + d.eo;
  const int32_t* pp = pl.poly_ptr + d.plo;
  if (move) {
    float2* pv = pl.poly_vel + d.pvo;
    for (int q = t; q < d.n_polys; q += blockDim.x) {
      float2 v = pv[q];
      if (v.x == 0.f && v.y == 0.f) continue;
      const int v0 = pp[q], nv = pp[q + 1] - v0;
      for (int j = v0; j < v0 + nv; ++j) {
        verts[j].x += v.x;
        verts[j].y += v.y;
      }
      bounce(&verts[v0].x, nv, 2, &v.x, d.width);
      bounce(&verts[v0].y, nv, 2, &v.y, d.height);
      pv[q] = v;
    }
    if (t == 0) {
      float4 e = pl.ends[inst], ev = pl.end_vel[inst];
      e.x += ev.x;
      e.y += ev.y;
      e.z += ev.z;
      e.w += ev.w;
      bounce(&e.x, 1, 1, &ev.x, d.width);
      bounce(&e.y, 1, 1, &ev.y, d.height);
      bounce(&e.z, 1, 1, &ev.z, d.width);
      bounce(&e.w, 1, 1, &ev.w, d.height);
      pl.ends[inst] = e;
      pl.end_vel[inst] = ev;
    }
    __syncthreads();
  }
  EdgeRec* er = pl.edges + d.eo;
  for (int q = t; q < d.n_polys; q += blockDim.x) {
    const int v0 = pp[q], m = pp[q + 1] - v0;
    for (int j = 0; j < m; ++j) {
      const float2 a = verts[v0 + j], b = verts[v0 + (j + 1 == m ? 0 : j + 1)];
      EdgeRec r;
      r.bx = b.x;
      r.by = b.y;
      r.ex = b.x - a.x;
      const float ey = b.y - a.y;
      r.ney = -ey;
      r.nce = -fmaf(r.ex, a.y, -(ey * a.x));
      r.ax = a.x;
      r.ay = a.y;
      r.flags = (j == 0 ? EDGE_FIRST : 0) | (j == m - 1 ? EDGE_LAST : 0);
      er[v0 + j] = r;
    }
  }
}

// ---------------------------------------------------------------------------
// Init: X ~ U(box), V ~ U(+-vmax); with a previous plan, the first n_pi
// particles of every group are drawn within +-radius of it (Priori
// Initialization).  Counter (particle*ceil(D/4) + d/4, frame, instance, tag).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void init_kernel(Pools pl, int frame_override, int use_prev) {
  const int2 bi = pl.blk_init[blockIdx.x];
  const int inst = bi.x;
  const InstDesc& d = pl.desc[inst];
  InstCtl* ctl = pl.ctl + inst;
  const int W = d.W, D = 2 * W;
  const int64_t PD = (int64_t)d.G * d.N * D;
  const int64_t e = (int64_t)bi.y + threadIdx.x;
  const int frame = frame_override >= 0 ? frame_override : ctl->frame;
  const bool learned = use_prev && ctl->use_learned;
  const bool pi = !learned && use_prev && d.use_pi && ctl->have_prev;
  if (e < PD) {
    const int i = (int)(e / D), dd = (int)(e - (int64_t)i * D);
    const int g = i / d.N, n = i - g * d.N;
    const float hi = dd < W ? d.width : d.height;
    const float vl = pl.hyper[d.go * 6 + g * 6 + 5];
    const float vmax = vl * hi * 0.5f;
    const uint32_t c0 = (uint32_t)(i * ((D + 3) / 4) + dd / 4);
    const U4 rx = philox(c0, (uint32_t)frame, d.instance, TAG_INIT_X, d.seed_lo, d.seed_hi);
    const U4 rv = philox(c0, (uint32_t)frame, d.instance, TAG_INIT_V, d.seed_lo, d.seed_hi);
    float x = u01(rx.v[dd & 3]) * hi;
    if ((pi || learned) && n < d.n_pi) {
      // Priori Initialization around the previous plan, or around this
      // group's learned proposal when the network supplied one
      const U4 rp = philox(c0, (uint32_t)frame, d.instance, TAG_PI, d.seed_lo, d.seed_hi);
      const float r = d.pi_radius;
      const float c = learned ? pl.proposal[d.gpo + g * D + dd] : pl.prev_path[d.dpo + dd];
      x = clampf(c + (-r + u01(rp.v[dd & 3]) * (2.f * r)), 0.f, hi);
    }
    const float v = -vmax + u01(rv.v[dd & 3]) * (2.f * vmax);
    const int64_t o = d.xo + e;
    pl.X[o] = x;
    pl.V[o] = v;
    pl.P[o] = x;
    if (dd == 0) {
      const int64_t po = d.po + i;
      pl.f[po] = INFINITY;
      pl.L[po] = INFINITY;
      pl.Pf[po] = INFINITY;
      pl.PL[po] = INFINITY;
      pl.Q[po] = 0;
      pl.PQ[po] = 0;
    }
  }
  if (bi.y == 0 && threadIdx.x < 64) {
    for (int g = threadIdx.x; g < d.G; g += 64) {
      const float* hy = pl.hyper + d.go * 6 + g * 6;
      pl.gbest_n[d.go + g] = 0;
      pl.gbest_f[d.go + g] = INFINITY;
      pl.opf[d.go + g] = INFINITY;
      float* op = pl.op + (d.go + g) * 3;
      float* ov = pl.ov + (d.go + g) * 3;
      op[0] = hy[3];
      op[1] = hy[0];
      op[2] = hy[1];
      ov[0] = ov[1] = ov[2] = 0.f;
    }
    if (threadIdx.x == 0) {
      ctl->k = 0;
      ctl->pending = 0;
      ctl->done = 0;
      ctl->tb_g = 0;
      ctl->tb_n = 0;
      ctl->tb_f = INFINITY;
      ctl->arrive = 0;
      ctl->epoch_in_frame = 0;
      ctl->otb = 0;
      ctl->truncated = 0;
      if (frame_override >= 0) ctl->frame = frame_override;
    }
  }
}

// ---------------------------------------------------------------------------
// Fused iteration.
// ---------------------------------------------------------------------------

// Side bits of vertex (bx, by) against the K segments of this thread: bit
// K-1-s is the sign of orient(p_s, p_{s+1}, b) = dx*by - dy*bx + nc.
template <int K>
__device__ __forceinline__ uint32_t pack_seg_sides(float bx, float by, const float (&dx)[K],
                                                   const float (&ndy)[K], const float (&nc)[K]) {
  uint32_t w = 0;
#pragma unroll
  for (int s = 0; s < K; ++s) {
    const float o = fmaf(dx[s], by, fmaf(ndy[s], bx, nc[s]));
    w = __builtin_amdgcn_alignbit(w, __float_as_uint(o), 31);
  }
  return w;
}

// Auto Truncation (Sec. "Auto Truncation") on the Tbest history ring.
__device__ bool at_fires(const float* hist, int k, int mode, int window, float delta, int q) {
  if (mode == 0 || q != 0 || window < 1) return false;
  if (mode == 1) {
    if (k < window) return false;
    float mean = 0.f;
    for (int i = k - window; i < k; ++i) mean += hist[i % kHist];
    mean /= (float)window;
    float var = 0.f;
    for (int i = k - window; i < k; ++i) {
      const float dv = hist[i % kHist] - mean;
      var += dv * dv;
    }
    var /= (float)window;
    return sqrtf(var) < delta;
  }
  if (mode == 2) {
    if (k <= window) return false;
    const float now = hist[(k - 1) % kHist], then = hist[(k - 1 - window) % kHist];
    const float scale = fabsf(now) > 1.f ? fabsf(now) : 1.f;
    return (then - now) < delta * scale;
  }
  return false;
}

// One outer step of the online hierarchical self-evolution (Sec. "HSEF"):
// outer particle g is group g's (w_init, C1, C2); its fitness is group g's
// best fitness; it moves by the grouped PSO update with the outer swarm's
// own hyper-parameters, each outer particle being its own group.
__device__ void hsef_step(const Pools& pl, const InstDesc& d, InstCtl* ctl, const float* s_gf) {
  __shared__ int s_otb, s_e;
  const int t = threadIdx.x, G = d.G;
  float* hy = pl.hyper + d.go * 6;
  float* op = pl.op + d.go * 3;
  float* ov = pl.ov + d.go * 3;
  float* opf = pl.opf + d.go;
  const float* oh = pl.outer_hyper + d.go * 6;
  const int col[3] = {3, 0, 1};
  if (t < G) {
    float F = s_gf[t];
    if (!isfinite(F)) F = INFINITY;
    if (F < opf[t]) {
      opf[t] = F;
      for (int j = 0; j < 3; ++j) op[t * 3 + j] = hy[t * 6 + col[j]];
    }
  }
  __syncthreads();
  if (t == 0) {
    int tb = 0;
    for (int g = 1; g < G; ++g)
      if (opf[g] < opf[tb]) tb = g;
    ctl->otb = tb;
    ctl->epoch_in_frame += 1;
    s_otb = tb;
    s_e = ctl->epoch_in_frame < d.T_outer ? ctl->epoch_in_frame : d.T_outer;
  }
  __syncthreads();
  if (t < G) {
    const float* h = oh + t * 6;
    const float w = h[3] - (h[3] - h[4]) / (float)d.T_outer * (float)s_e;
    const U4 r = philox((uint32_t)t, ctl->epoch_ctr, d.instance, TAG_HSEF, d.seed_lo, d.seed_hi);
    const float r1 = u01(r.v[0]), r2 = u01(r.v[1]), r3 = u01(r.v[2]);
    for (int j = 0; j < 3; ++j) {
      const float lo = j == 0 ? hy[t * 6 + 4] : 0.f, hi = j == 0 ? 1.f : 3.f;
      const float vmax = h[5] * (hi - lo) * 0.5f;
      const float x = hy[t * 6 + col[j]];
      const float pb = op[t * 3 + j], tbv = op[s_otb * 3 + j];
      float v = w * ov[t * 3 + j] + h[0] * r1 * (pb - x) + h[1] * r2 * (pb - x) +
                h[2] * r3 * (tbv - x);
      v = clampf(v, -vmax, vmax);
      ov[t * 3 + j] = v;
      hy[t * 6 + col[j]] = clampf(x + v, lo, hi);
    }
  }
  __syncthreads();
  if (t == 0) ctl->epoch_ctr += 1;
}

// Work of the last block of an instance to finish a launch.
__device__ void finish_iteration(const Pools& pl, const InstDesc& d, InstCtl* ctl, int k,
                                 int pending, uint32_t ctr, int flags) {
  __shared__ float s_gf[kMaxG];
  __shared__ int s_gn[kMaxG];
  __shared__ int s_tg, s_stop, s_at, s_q;
  const int t = threadIdx.x, G = d.G, N = d.N, D = 2 * d.W;
  if (!(flags & STEP_FIT)) {  // update-only launch
    if (t == 0) {
      ctl->ctr = ctr + (pending ? 1u : 0u);
      ctl->pending = 0;
      ctl->arrive = 0;
    }
    return;
  }
  const TileBest* tb = pl.tiles + d.to;
  for (int g = t; g < G; g += blockDim.x) {
    TileBest b = tb[g * d.tpg];
    for (int j = 1; j < d.tpg; ++j) {
      const TileBest c = tb[g * d.tpg + j];
      if (better(c.f, c.n, b.f, b.n)) b = c;
    }
    if (b.n >= N) b.n = 0;
    pl.gbest_n[d.go + g] = b.n;
    pl.gbest_f[d.go + g] = b.f;
    s_gn[g] = b.n;
    s_gf[g] = b.f;
  }
  __syncthreads();
  if (t == 0) {
    int tg = 0;
    for (int g = 1; g < G; ++g)
      if (s_gf[g] < s_gf[tg]) tg = g;
    s_tg = tg;
  }
  __syncthreads();
  const int tg = s_tg, tn = s_gn[tg];
  const float tf = s_gf[tg];
  const float* P = pl.P + d.xo;
  for (int e = t; e < G * D; e += blockDim.x) {
    const int g = e / D, dd = e - g * D;
    pl.gbest_pos[d.gpo + e] = P[(int64_t)(g * N + s_gn[g]) * D + dd];
  }
  for (int e = t; e < D; e += blockDim.x) pl.tbest_pos[d.dpo + e] = P[(int64_t)(tg * N + tn) * D + e];
  const int k_new = k + 1;
  const uint32_t ctr_new = ctr + (pending ? 1u : 0u);
  bool stop = false, at = false;
  if (flags & STEP_FRAME) {
    if (t == 0) {
      ctl->hist[(k_new - 1) % kHist] = tf;
      const int q = pl.PQ[d.po + tg * N + tn];
      const bool a = at_fires(ctl->hist, k_new, d.at_mode, d.at_window, d.at_delta, q);
      s_at = a;
      s_stop = a || k_new >= d.T;
      s_q = q;
    }
    __syncthreads();
    stop = s_stop;
    at = s_at;
    if (!stop && d.hsef_every > 0 && k_new % d.hsef_every == 0) hsef_step(pl, d, ctl, s_gf);
  }
  if (stop)
    for (int e = t; e < D; e += blockDim.x)
      pl.prev_path[d.dpo + e] = P[(int64_t)(tg * N + tn) * D + e];
  if (t == 0) {
    ctl->k = k_new;
    ctl->tb_g = tg;
    ctl->tb_n = tn;
    ctl->tb_f = tf;
    if (stop) {
      ctl->done = 1;
      ctl->pending = 0;
      ctl->ctr = ctr_new + 1u;
      ctl->truncated = at;
      ctl->res_cost = tf;
      ctl->res_len = pl.PL[d.po + tg * N + tn];
      ctl->res_q = s_q;
      ctl->res_iters = k_new;
      ctl->res_trunc = at;
      ctl->have_prev = 1;
      ctl->frame += 1;
    } else {
      ctl->pending = 1;
      ctl->ctr = ctr_new;
    }
    ctl->arrive = 0;
  }
}

// Thread layout: block = tile of `ppt` particles of one group, C threads per
// particle; thread chunk c handles path segments [cK, cK+K) between points
// cK .. cK+K (point 0 = start, W+1 = target, points past W+1 repeat the
// target so that their segments have zero length and cross nothing).
template <int K, bool FIT>
__device__ __forceinline__ void iteration(const Pools& pl, int flags) {
  __shared__ EdgeRec s_edge[kEdgeChunk];
  __shared__ int s_q[256];
  __shared__ float s_l[256];
  __shared__ float s_pf[256];
  __shared__ int s_imp[256];
  __shared__ int s_last;

  const int2 bt = pl.blk_tiles[blockIdx.x];
  const int inst = bt.x, tile = bt.y;
  const InstDesc& d = pl.desc[inst];
  InstCtl* ctl = pl.ctl + inst;
  if ((flags & STEP_FRAME) && ctl->done) return;
  const int k = ctl->k, pending = ctl->pending;
  const uint32_t ctr = ctl->ctr;
  const int N = d.N, W = d.W, D = 2 * W, C = d.C;
  const int g = tile / d.tpg;
  const int n0 = (tile - g * d.tpg) * d.ppt;
  const int t = threadIdx.x;
  const int slot = t / C, c = t - slot * C;
  const int n = n0 + slot;
  const bool active = slot < d.ppt && n < N;
  const int i = g * N + n;
  float* X = pl.X + d.xo + (int64_t)i * D;
  float* V = pl.V + d.xo + (int64_t)i * D;

  // ---- 1. path points of this chunk, with the pending update applied ------
  float px[K + 1], py[K + 1], vx[K + 1], vy[K + 1];
  if (active) {
    const float4 ends = pl.ends[inst];
    float w = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, vmx = 0.f, vmy = 0.f;
    const float* Pp = pl.P + d.xo + (int64_t)i * D;
    const float* Gb = pl.gbest_pos + d.gpo + g * D;
    const float* Tb = pl.tbest_pos + d.dpo;
    if (pending) {
      const float* h = pl.hyper + d.go * 6 + g * 6;
      const int kk = k < d.T ? k : d.T;
      w = h[3] - (h[3] - h[4]) / (float)d.T * (float)kk;
      const U4 r = philox((uint32_t)i, ctr, d.instance, TAG_UPDATE, d.seed_lo, d.seed_hi);
      a1 = h[0] * u01(r.v[0]);
      a2 = h[1] * u01(r.v[1]);
      a3 = h[2] * u01(r.v[2]);
      vmx = h[5] * d.width * 0.5f;
      vmy = h[5] * d.height * 0.5f;
    }
#pragma unroll
    for (int s = 0; s <= K; ++s) {
      int j = c * K + s;
      j = j > W + 1 ? W + 1 : j;
      float x, y, u = 0.f, v = 0.f;
      if (j == 0) {
        x = ends.x;
        y = ends.y;
      } else if (j == W + 1) {
        x = ends.z;
        y = ends.w;
      } else {
        const int q = j - 1;
        x = X[q];
        y = X[W + q];
        if (pending) {
          u = V[q];
          v = V[W + q];
          u = w * u + a1 * (Pp[q] - x) + a2 * (Gb[q] - x) + a3 * (Tb[q] - x);
          v = w * v + a1 * (Pp[W + q] - y) + a2 * (Gb[W + q] - y) + a3 * (Tb[W + q] - y);
          u = clampf(u, -vmx, vmx);
          v = clampf(v, -vmy, vmy);
          x = clampf(x + u, 0.f, d.width);
          y = clampf(y + v, 0.f, d.height);
        }
      }
      px[s] = x;
      py[s] = y;
      vx[s] = u;
      vy[s] = v;
    }
  }
  __syncthreads();  // every thread has read the old positions of its points
  if (active && pending) {
#pragma unroll
    for (int s = 1; s <= K; ++s) {
      const int j = c * K + s;
      if (j <= W) {
        X[j - 1] = px[s];
        X[W + j - 1] = py[s];
        V[j - 1] = vx[s];
        V[W + j - 1] = vy[s];
      }
    }
  }
  if (!FIT) {
    __threadfence();
    __syncthreads();
    if (t == 0) s_last = atomicAdd(&ctl->arrive, 1) == d.n_tiles - 1;
    __syncthreads();
    if (s_last) finish_iteration(pl, d, ctl, k, pending, ctr, flags & ~STEP_FIT);
    return;
  }

  // ---- 2. segment lines and lengths ----------------------------------------
  float dx[K], ndy[K], nc[K];
  float len = 0.f;
#pragma unroll
  for (int s = 0; s < K; ++s) {
    const float ddx = px[s + 1] - px[s], ddy = py[s + 1] - py[s];
    dx[s] = ddx;
    ndy[s] = -ddy;
    nc[s] = fmaf(ddy, px[s], -(ddx * py[s]));
    if (c * K + s <= W) len += sqrtf(ddx * ddx + ddy * ddy);
  }

  // ---- 3. crossings: segments x obstacle edges (edges staged in LDS) --------
  int cnt = 0;
  uint32_t w0 = 0, wp = 0;
  const EdgeRec* er = pl.edges + d.eo;
  for (int e0 = 0; e0 < d.n_edges; e0 += kEdgeChunk) {
    const int ne = d.n_edges - e0 < kEdgeChunk ? d.n_edges - e0 : kEdgeChunk;
    __syncthreads();
    {
      const float4* src = reinterpret_cast<const float4*>(er + e0);
      float4* dst = reinterpret_cast<float4*>(s_edge);
      for (int q = t; q < ne * 2; q += blockDim.x) dst[q] = src[q];
    }
    __syncthreads();
    if (active) {
      EdgeRec nx = s_edge[0];
      for (int e = 0; e < ne; ++e) {
        const EdgeRec r = nx;
        if (e + 1 < ne) nx = s_edge[e + 1];  // next record in flight while this one is used
        const int fl = __builtin_amdgcn_readfirstlane(r.flags);
        if (fl & EDGE_FIRST) {
          w0 = pack_seg_sides<K>(r.ax, r.ay, dx, ndy, nc);
          wp = w0;
        }
        uint32_t wn;
        if (fl & EDGE_LAST)
          wn = w0;
        else
          wn = pack_seg_sides<K>(r.bx, r.by, dx, ndy, nc);
        // side bits of the K+1 points against the edge's line: bit K-s
        uint32_t ew = 0;
#pragma unroll
        for (int s = 0; s <= K; ++s) {
          const float ev = fmaf(r.ex, py[s], fmaf(r.ney, px[s], r.nce));
          ew = __builtin_amdgcn_alignbit(ew, __float_as_uint(ev), 31);
        }
        // segment s straddles the edge's line iff points s and s+1 differ;
        // the edge straddles segment s's line iff its two vertices differ.
        cnt += __popc((wp ^ wn) & (ew ^ (ew >> 1)));
        wp = wn;
      }
    }
  }

  // ---- 4. per-particle fitness and Pbest ------------------------------------
  s_q[t] = cnt;
  s_l[t] = len;
  __syncthreads();
  if (active && c == 0) {
    int q = 0;
    float L = 0.f;
    for (int cc = 0; cc < C; ++cc) {
      q += s_q[t + cc];
      L += s_l[t + cc];
    }
    const float qf = (float)q;
    float pw = 1.f;
    for (int b = 0; b < d.beta; ++b) pw *= qf;
    const float fv = L + d.alpha * pw;
    const int64_t po = d.po + i;
    pl.f[po] = fv;
    pl.L[po] = L;
    pl.Q[po] = q;
    float pf = pl.Pf[po];
    const float fc = isfinite(fv) ? fv : INFINITY;
    const int imp = fc < pf;
    if (imp) {
      pl.Pf[po] = fc;
      pl.PL[po] = L;
      pl.PQ[po] = q;
      pf = fc;
    }
    s_imp[slot] = imp;
    s_pf[slot] = pf;
  }
  __syncthreads();
  if (active && s_imp[slot]) {
    float* Pw = pl.P + d.xo + (int64_t)i * D;
#pragma unroll
    for (int s = 1; s <= K; ++s) {
      const int j = c * K + s;
      if (j <= W) {
        Pw[j - 1] = px[s];
        Pw[W + j - 1] = py[s];
      }
    }
  }

  // ---- 5. tile argmin (lowest index on ties) --------------------------------
  if (t < 64) {
    float bf = INFINITY;
    int bn = 0x7fffffff;
    for (int sl = t; sl < d.ppt; sl += 64) {
      if (n0 + sl < N && better(s_pf[sl], n0 + sl, bf, bn)) {
        bf = s_pf[sl];
        bn = n0 + sl;
      }
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
      const float of = __shfl_xor(bf, m);
      const int on = __shfl_xor(bn, m);
      if (better(of, on, bf, bn)) {
        bf = of;
        bn = on;
      }
    }
    if (t == 0) pl.tiles[d.to + tile] = TileBest{bf, bn};
  }

  // ---- 6. the last block of this instance reduces the bests -----------------
  __threadfence();
  __syncthreads();
  if (t == 0) s_last = atomicAdd(&ctl->arrive, 1) == d.n_tiles - 1;
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  finish_iteration(pl, d, ctl, k, pending, ctr, flags);
}

// ---------------------------------------------------------------------------
void launch_geom(const Pools& pl, int n_inst, int move, hipStream_t s) {
  hipLaunchKernelGGL(geom_kernel, dim3(n_inst), dim3(256), 0, s, pl, move);
}

void launch_init(const Pools& pl, int n_blocks, int frame_override, int use_prev, hipStream_t s) {
  hipLaunchKernelGGL(init_kernel, dim3(n_blocks), dim3(256), 0, s, pl, frame_override, use_prev);
}

bool step_supported(int K) { return K == 4 || K == 8 || K == 12 || K == 16 || K == 24; }

// One fused iteration (fitness path) and the update-only flush, as separate
// kernels so that profiles separate them.
template <int K>
__global__ __launch_bounds__(256) void iter_kernel(Pools pl, int flags) {
  iteration<K, true>(pl, flags);
}
template <int K>
__global__ __launch_bounds__(256) void update_kernel(Pools pl, int flags) {
  iteration<K, false>(pl, flags);
}

template <int K>
static void launch_k(const Pools& pl, int n_blocks, int threads, int flags, hipStream_t s) {
  if (flags & STEP_FIT)
    hipLaunchKernelGGL(iter_kernel<K>, dim3(n_blocks), dim3(threads), 0, s, pl, flags);
  else
    hipLaunchKernelGGL(update_kernel<K>, dim3(n_blocks), dim3(threads), 0, s, pl, flags);
}

void launch_step(const Pools& pl, int K, int n_blocks, int threads, int flags, hipStream_t s) {
  switch (K) {
    case 4: launch_k<4>(pl, n_blocks, threads, flags, s); break;
    case 8: launch_k<8>(pl, n_blocks, threads, flags, s); break;
    case 12: launch_k<12>(pl, n_blocks, threads, flags, s); break;
    case 16: launch_k<16>(pl, n_blocks, threads, flags, s); break;
    case 24: launch_k<24>(pl, n_blocks, threads, flags, s); break;
    default: break;
  }
}

}  // namespace sepso
