// libsepso device code for path planning (gfx950, FP32 VALU).
//
// Kernels:
//   geom_kernel   -- obstacle/endpoint motion for one frame and the derived
//                    rectangle boxes / per-edge records the fitness reads;
//   init_kernel   -- uniform swarm and Priori Initialization;
//   iter_kernel   -- one fused DTPSO iteration per launch: the previous
//                    iteration's velocity/position update (Eq.(6)-(8)), the
//                    path fitness (Eq.(11)-(13)) and the Pbest update;
//   update_kernel -- the pending update alone (end of a stepping call);
//   reduce_kernel -- per instance: group and total bests, Auto Truncation,
//                    the online self-evolution step, control advance;
//   evolve_*      -- the evolution phase's higher level (H-SEPSO).
#include "common.h"
#include "kernels.h"
#include "rng.h"

namespace sepso {

__device__ __forceinline__ bool better(float fa, int na, float fb, int nb) {
  return fa < fb || (fa == fb && na < nb);
}

// Integer key of a float that orders as the values do (-0 just below +0).
__device__ __forceinline__ int float_key(float x) {
  const int b = __float_as_int(x);
  return b ^ ((b >> 31) & 0x7fffffff);
}

// The float of a key (the map is its own inverse).
__device__ __forceinline__ float key_float(int k) { return __int_as_float(k ^ ((k >> 31) & 0x7fffffff)); }

// Minimum (maximum) of v over the wave's 64 lanes, every lane taking part:
// pairs and quads (quad permutations), eights and sixteens (half-row and row
// mirrors) fold into the min/max instructions as DPP operands, so that every
// lane of a row of 16 holds the row's value; the four rows meet on the
// scalar unit.
__device__ __forceinline__ int wave_min_key(int v) {
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true));   // quad_perm 1,0,3,2
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true));   // quad_perm 2,3,0,1
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true));  // row_half_mirror
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, true));  // row_mirror
  return min(min(__builtin_amdgcn_readlane(v, 15), __builtin_amdgcn_readlane(v, 31)),
             min(__builtin_amdgcn_readlane(v, 47), __builtin_amdgcn_readlane(v, 63)));
}
__device__ __forceinline__ int wave_max_key(int v) {
  v = max(v, __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true));
  v = max(v, __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true));
  v = max(v, __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true));
  v = max(v, __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, true));
  return max(max(__builtin_amdgcn_readlane(v, 15), __builtin_amdgcn_readlane(v, 31)),
             max(__builtin_amdgcn_readlane(v, 47), __builtin_amdgcn_readlane(v, 63)));
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
  const InstDesc d = pl.desc[inst];  // by value: stores cannot make it reload
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
  const int2* kind = pl.pkind + d.pvo;
  for (int q = t; q < d.n_polys; q += blockDim.x) {
    const int v0 = pp[q], m = pp[q + 1] - v0;
    const int2 ks = kind[q];
    if (ks.x == 1) {  // axis-aligned rectangle: its bounding box
      float x0 = verts[v0].x, y0 = verts[v0].y, x1 = x0, y1 = y0;
      for (int j = 1; j < m; ++j) {
        x0 = fminf(x0, verts[v0 + j].x);
        x1 = fmaxf(x1, verts[v0 + j].x);
        y0 = fminf(y0, verts[v0 + j].y);
        y1 = fmaxf(y1, verts[v0 + j].y);
      }
      // + 0 turns a -0 corner into +0: every stored coordinate then has its
      // sign bit clear, and its bits order as its value does
      pl.rects[d.ro + ks.y] = make_float4(x0 + 0.f, y0 + 0.f, x1 + 0.f, y1 + 0.f);
      // centre and half sides (exact: the corners lie on a 1/256 grid)
      pl.rect_c[d.ro + ks.y] = make_float4((x0 + x1) * 0.5f, (y0 + y1) * 0.5f, (x1 - x0) * 0.5f,
                                           (y1 - y0) * 0.5f);
      continue;
    }
    if (ks.x >= 2) {  // convex: box keys, lines with the interior on their positive side, vertices
      CPoly& c = pl.cpolys[d.cpo + ks.y];
      const float sg = ks.x == 2 ? 1.f : -1.f;
      float x0 = verts[v0].x, y0 = verts[v0].y, x1 = x0, y1 = y0;
      for (int j = 0; j < m; ++j) {
        const float2 a = verts[v0 + j], b = verts[v0 + (j + 1 == m ? 0 : j + 1)];
        const float ex = b.x - a.x, ey = b.y - a.y;
        c.ex[j] = sg * ex;
        c.ney[j] = sg * -ey;
        c.nce[j] = sg * -fmaf(ex, a.y, -(ey * a.x));
        c.vx[j] = a.x;
        c.vy[j] = a.y;
        x0 = fminf(x0, a.x);
        x1 = fmaxf(x1, a.x);
        y0 = fminf(y0, a.y);
        y1 = fmaxf(y1, a.y);
      }
      c.kx0 = float_key(x0);
      c.ky0 = float_key(y0);
      c.kx1 = float_key(x1);
      c.ky1 = float_key(y1);
      c.n = m;
      continue;
    }
    EdgeRec* er = pl.edges + d.geo + ks.y;
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
      er[j] = r;
    }
  }
}

// ---------------------------------------------------------------------------
// Init: X ~ U(box), V ~ U(+-vmax); with a previous plan, the first n_pi
// particles of every group are drawn within +-radius of it (Priori
// Initialization).  Counter (particle*ceil(D/4) + d/4, frame, instance, tag),
// output d mod 4: one thread per quad of coordinates d = 4q..4q+3 of a
// particle makes each of its Philox calls once for all four.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void init_kernel(Pools pl, int frame_override, int use_prev) {
  const int2 bi = pl.blk_init[blockIdx.x];
  const int inst = bi.x;
  const InstDesc d = pl.desc[inst];  // by value: stores cannot make it reload
  InstCtl* ctl = pl.ctl + inst;
  const int W = d.W, D = 2 * W, DQ = (D + 3) / 4;
  const int nq = d.G * d.N * DQ;
  const int q = bi.y + (int)threadIdx.x;
  const int frame = frame_override >= 0 ? frame_override : ctl->frame;
  const bool learned = use_prev && ctl->use_learned;
  const bool pi = !learned && use_prev && d.use_pi && ctl->have_prev;
  if (q < nq) {
    const int i = q / DQ, d0 = 4 * (q - i * DQ);
    const int g = i / d.N, n = i - g * d.N;
    const float vl = pl.hyper[d.go * 6 + g * 6 + 5];
    const uint32_t c0 = (uint32_t)q;  // = i * ceil(D/4) + d0/4
    const U4 rx = philox(c0, (uint32_t)frame, d.instance, TAG_INIT_X, d.seed_lo, d.seed_hi);
    const U4 rv = philox(c0, (uint32_t)frame, d.instance, TAG_INIT_V, d.seed_lo, d.seed_hi);
    const bool near = (pi || learned) && n < d.n_pi;
    U4 rp{};
    if (near) rp = philox(c0, (uint32_t)frame, d.instance, TAG_PI, d.seed_lo, d.seed_hi);
    const int64_t o = d.xo + (int64_t)i * D + d0;
    float xq[4], vq[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int dd = min(d0 + u, D - 1);  // lanes past the particle's end compute, never store
      const float hi = dd < W ? d.width : d.height;
      const float vmax = vl * hi * 0.5f;
      float x = u01(rx.v[u]) * hi;
      if (near) {
        // Priori Initialization around the previous plan, or around this
        // group's learned proposal when the network supplied one
        const float r = d.pi_radius;
        const float c = learned ? pl.proposal[d.gpo + g * D + dd] : pl.prev_path[d.dpo + dd];
        x = clampf(c + (-r + u01(rp.v[u]) * (2.f * r)), 0.f, hi);
      }
      xq[u] = x;
      vq[u] = -vmax + u01(rv.v[u]) * (2.f * vmax);
    }
    if (d0 + 4 <= D && (o & 3) == 0) {  // a whole quad at a 16-byte boundary (pools are)
      const float4 x4 = make_float4(xq[0], xq[1], xq[2], xq[3]);
      st_stream(reinterpret_cast<float4*>(pl.X + o), x4);
      st_stream(reinterpret_cast<float4*>(pl.V + o), make_float4(vq[0], vq[1], vq[2], vq[3]));
      st_stream(reinterpret_cast<float4*>(pl.P + o), x4);
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (d0 + u < D) {
          pl.X[o + u] = xq[u];
          pl.V[o + u] = vq[u];
          pl.P[o + u] = xq[u];
        }
    }
    if (d0 == 0) {
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
  if (mode == 1 || mode == 3) {
    // mode 1: the full window must have elapsed; mode 3: the window is
    // whatever has elapsed (at least two values), capped at `window`
    int w = window;
    if (mode == 1 && k < window) return false;
    if (mode == 3) {
      if (k < 2) return false;
      w = k < window ? k : window;
    }
    float mean = 0.f;
    for (int i = k - w; i < k; ++i) mean += hist[i % kHist];
    mean /= (float)w;
    float var = 0.f;
    for (int i = k - w; i < k; ++i) {
      const float dv = hist[i % kHist] - mean;
      var += dv * dv;
    }
    var /= (float)w;
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


// Bests of one instance after an iteration (Algorithm 1, "update P, G, T"):
// Gbest_g = argmin of the Pbest fitness over group g (lowest index on ties),
// Tbest = argmin over groups; then Auto Truncation, the online outer step
// and the control-block advance.  One block per instance, after the tile
// kernels have finished (kernel boundary = visibility, no fences in tiles).
__global__ __launch_bounds__(512) void reduce_kernel(Pools pl, int flags) {
  __shared__ float s_gf[kMaxG];
  __shared__ int s_gn[kMaxG];
  __shared__ float s_hist[kHist];
  __shared__ int s_tg, s_stop, s_at, s_q;
  const int inst = blockIdx.x;
  const InstDesc d = pl.desc[inst];  // by value: stores cannot make it reload
  InstCtl* ctl = pl.ctl + inst;
  if ((flags & STEP_FRAME) && ctl->done) return;
  const int k = ctl->k, pending = ctl->pending;
  const uint32_t ctr = ctl->ctr;
  const int t = threadIdx.x, G = d.G, N = d.N, D = 2 * d.W;
  __syncthreads();  // every thread has read the control block before it advances
  if (!(flags & STEP_FIT)) {  // after an update-only launch
    if (t == 0) {
      ctl->ctr = ctr + (pending ? 1u : 0u);
      ctl->pending = 0;
    }
    return;
  }
  // the Auto-Truncation history ring, read while the Pbest scan runs (its
  // LDS copy is written after the scan, so that no wave waits for it first)
  const bool hist_lane = (flags & STEP_FRAME) && t < kHist;
  const float hv = hist_lane ? ctl->hist[t] : 0.f;
  // one wave per group (waves take groups in turn): lanes scan the group's
  // Pbest fitness, a shuffle argmin (lowest index on ties) picks Gbest
  const float* Pf = pl.Pf + d.po;
  const int lane = t & 63, wave = t >> 6, n_waves = blockDim.x >> 6;
  for (int g = wave; g < G; g += n_waves) {
    float bf = INFINITY;
    int bn = 0x7fffffff;
    for (int n0 = lane; n0 < N; n0 += 4 * 64) {  // four loads in flight per lane
      float f[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) f[u] = n0 + 64 * u < N ? Pf[g * N + n0 + 64 * u] : INFINITY;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (better(f[u], n0 + 64 * u, bf, bn)) {
          bf = f[u];
          bn = n0 + 64 * u;
        }
    }
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
      const float of = __shfl_xor(bf, m);
      const int on = __shfl_xor(bn, m);
      if (better(of, on, bf, bn)) {
        bf = of;
        bn = on;
      }
    }
    if (lane == 0) {
      const int n = bn < N ? bn : 0;
      s_gn[g] = n;
      s_gf[g] = bf;
      pl.gbest_n[d.go + g] = n;
      pl.gbest_f[d.go + g] = bf;
    }
  }
  if (hist_lane) s_hist[t] = hv;
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
  // Tbest's crossing count and length, read alongside the row copies
  int tq = 0;
  float tl = 0.f;
  if ((flags & STEP_FRAME) && t == 0) {
    tq = pl.PQ[d.po + tg * N + tn];
    tl = pl.PL[d.po + tg * N + tn];
  }
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
      s_hist[(k_new - 1) % kHist] = tf;
      const bool a = at_fires(s_hist, k_new, d.at_mode, d.at_window, d.at_delta, tq);
      s_at = a;
      s_stop = a || k_new >= d.T;
      s_q = tq;
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
      ctl->res_len = tl;
      ctl->res_q = s_q;
      ctl->res_iters = k_new;
      ctl->res_trunc = at;
      ctl->have_prev = 1;
      ctl->frame += 1;
    } else {
      ctl->pending = 1;
      ctl->ctr = ctr_new;
    }
  }
}


// Direct global -> LDS loads (no registers on the way): lane i of the wave
// writes its word at dst_wave + i, dst_wave the same for the whole wave.
__device__ __forceinline__ void lds_dma16(const void* src, void* dst_wave) {
  __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                   (__attribute__((address_space(3))) void*)dst_wave, 16, 0, 0);
}
__device__ __forceinline__ void lds_dma4(const void* src, void* dst_wave) {
  __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                   (__attribute__((address_space(3))) void*)dst_wave, 4, 0, 0);
}

// lds_dma16 with the non-temporal cache policy (aux bit 1): the swarm's
// positions stream like its other rows (ld_stream)
__device__ __forceinline__ void lds_dma16_stream(const void* src, void* dst_wave) {
  __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                   (__attribute__((address_space(3))) void*)dst_wave, 16, 0, 2);
}

// Edge records of the other polygons, from record first on, into the LDS
// staging area (float4 words, two loads in flight per thread).
__device__ __forceinline__ void stage_records(const Pools& pl, const InstDesc& d, float* s_stage,
                                              int first, int count) {
  const int t = threadIdx.x, B = blockDim.x;
  const float4* src = reinterpret_cast<const float4*>(pl.edges + d.geo + first);
  const int n4 = 2 * count;
  float4* dst = reinterpret_cast<float4*>(s_stage);
  for (int q = t; q < n4; q += 2 * B) {
    const float4 a = src[q];
    float4 b;
    if (q + B < n4) b = src[q + B];
    dst[q] = a;
    if (q + B < n4) dst[q + B] = b;
  }
}

// Phase C of the fused iteration: crossings of this thread's K segments with
// every obstacle edge of the instance.  Rectangles and convex polygons are
// read through the scalar cache; the other polygons' edge records are staged
// through LDS (s_stage: the first chunk was staged before the block's first
// barrier, later ones are staged here by all threads of the block between
// barriers).  Crossing
// words: bit K-1-s set when segment s properly crosses the edge (never for
// masked slots); ct counts them.
template <int K, int R>
__device__ __forceinline__ void crossings(const Pools& pl, const InstDesc& d, float* s_stage,
                                          bool active, int rg, const float (&px)[K + 1],
                                          const float (&py)[K + 1], const float (&dx)[K],
                                          const float (&ndy)[K], const float (&nc)[K], int& ct) {
  auto count = [&](uint32_t x) { ct += __popc(x); };
  // Bounding box of the wave's points (wave-uniform).  A segment lies in the
  // box of its end points, so a rectangle that is outside the box (touching
  // allowed) cannot be properly crossed by any of the wave's segments: its
  // sign tests could only mark points exactly on its lines, a degenerate
  // contact, and the whole rectangle is skipped.
  float bx0 = INFINITY, bx1 = -INFINITY, by0 = INFINITY, by1 = -INFINITY;
  if (active) {
#pragma unroll
    for (int s = 0; s <= K; ++s) {
      bx0 = fminf(bx0, px[s]);
      bx1 = fmaxf(bx1, px[s]);
      by0 = fminf(by0, py[s]);
      by1 = fmaxf(by1, py[s]);
    }
  }
  // Reduced over the wave as integer keys, then mapped back: the keys'
  // order is the floats' (-0 just below +0).
  const int kx0 = wave_min_key(float_key(bx0));
  const int kx1 = wave_max_key(float_key(bx1));
  const int ky0 = wave_min_key(float_key(by0));
  const int ky1 = wave_max_key(float_key(by1));
  bx0 = key_float(kx0);
  bx1 = key_float(kx1);
  by0 = key_float(ky0);
  by1 = key_float(ky1);
  // C.1 axis-aligned rectangles, read through the scalar cache: a record is
  // the same for every lane, so it stays in scalar registers and the culling
  // test runs on the scalar unit, on integer keys that order floats as their
  // values do (the key order puts -0 below +0, so it never culls more than
  // the float comparison would).
  //
  // A box is convex, so the proper crossings of a segment with its four
  // edges are (in general position) one when exactly one end point lies
  // strictly inside, none when both do, and two when both lie outside and
  // the segment meets the open box: its x and y ranges overlap the box's
  // and the box's corners are not all on one side of its line.  End-point
  // sides are exact sign tests of one coordinate difference; the corner
  // test is |o(centre)| < |dx| h/2 + |dy| w/2 (the corners' orientations
  // are o(centre) +- |dx| h/2 +- |dy| w/2), by two FMAs for o(centre) and
  // two for the difference, within the degenerate band of the exact value.
  // Where a test is degenerate the count may resolve it either way.
  constexpr uint32_t kOnes = (2u << K) - 1u;
  const uint32_t segmask = active ? (kOnes & ~1u) : 0u;
  {
    // lo < c < hi as one unsigned comparison of the coordinate's bits (the
    // box is not empty here; a coordinate of -0 lies on the map's border,
    // its bits test as outside).
    const uint32_t ny = (uint32_t)(ky1 - ky0 - 1), nx = (uint32_t)(kx1 - kx0 - 1);
    auto inside = [](float c, int lo, uint32_t n) { return (uint32_t)(__float_as_int(c) - lo - 1) < n; };
    // Words: bit K - s for point s; segment s (points s, s + 1) at bit K - s,
    // so its second point is the word shifted left by one.  Bits 1..K are the
    // segments (segmask); inactive lanes keep none.
    // sign bits of (c - p_s) (sub_c_p) or of (p_s - c)
    auto side_word = [&](const float (&p)[K + 1], float c, bool sub_c_p) {
      uint32_t w = 0;
#pragma unroll
      for (int s = 0; s <= K; ++s)
        w = __builtin_amdgcn_alignbit(w, __float_as_uint(sub_c_p ? c - p[s] : p[s] - c), 31);
      return w;
    };
    // Rectangles come in 64-byte quads (an instance's slice is padded to a
    // whole number of them), one scalar load per quad; wave group rg takes
    // quads rg, rg + R, ...  Padding rectangles are loaded, never tested.
    typedef float quad16 __attribute__((ext_vector_type(16)));
    const __attribute__((address_space(4))) quad16* rq =
        (const __attribute__((address_space(4))) quad16*)(pl.rects + d.ro);
    typedef float quad4 __attribute__((ext_vector_type(4)));
    const __attribute__((address_space(4))) quad4* cq =
        (const __attribute__((address_space(4))) quad4*)(pl.rect_c + d.ro);
    for (int c4 = rg; 4 * c4 < d.n_rects; c4 += R) {
      const quad16 blk = rq[c4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
      const float4 b = make_float4(blk[4 * q], blk[4 * q + 1], blk[4 * q + 2], blk[4 * q + 3]);  // x0, y0, x1, y1
      // stored coordinates have their sign bit clear: their bits are their keys
      if (4 * c4 + q >= d.n_rects || __float_as_int(b.z) <= kx0 || __float_as_int(b.x) >= kx1 ||
          __float_as_int(b.w) <= ky0 || __float_as_int(b.y) >= ky1)
        continue;
      // Point sides of the four lines (bit set: strictly on the box's side).
      // A line that does not pass strictly through the wave's box has every
      // point on the box's side of it or on it (the box is not culled); a
      // point on the line is then taken as on the box's side, as if moved
      // inward by an infinitesimal amount, which changes degenerate tests
      // only.
      const uint32_t lw = inside(b.x, kx0, nx) ? side_word(px, b.x, true) : kOnes;   // p.x > x0
      const uint32_t rw = inside(b.z, kx0, nx) ? side_word(px, b.z, false) : kOnes;  // p.x < x1
      const uint32_t bw = inside(b.y, ky0, ny) ? side_word(py, b.y, true) : kOnes;   // p.y > y0
      const uint32_t tw = inside(b.w, ky0, ny) ? side_word(py, b.w, false) : kOnes;  // p.y < y1
      const uint32_t in = lw & rw & bw & tw;
      count((in ^ (in << 1)) & segmask);  // one end strictly inside
      // both ends outside, ranges overlapping: candidates for two crossings
      const uint32_t ov = ((lw << 1) | lw) & ((rw << 1) | rw) & ((bw << 1) | bw) & ((tw << 1) | tw);
      const uint32_t cand = ov & ~((in << 1) | in) & segmask;
      if (__builtin_amdgcn_ballot_w64(cand != 0u) == 0ull) continue;
      const quad4 cr = cq[4 * c4 + q];  // centre and half sides, loaded only when needed
      const float xc = cr.x, yc = cr.y, hw = cr.z, hh = cr.w;
      uint32_t sw = 0;  // bit K - 1 - s: the line of segment s passes strictly through the box
#pragma unroll
      for (int s = 0; s < K; ++s) {
        const float oc = fmaf(dx[s], yc, fmaf(ndy[s], xc, nc[s]));
        const float dd = fmaf(-fabsf(ndy[s]), hw, fmaf(-fabsf(dx[s]), hh, fabsf(oc)));
        sw = __builtin_amdgcn_alignbit(sw, __float_as_uint(dd), 31);
      }
      const uint32_t thr = cand & (sw << 1);
      count(thr);
      count(thr);
      }
    }
  }
  // C.2 convex polygons other than rectangles, records read through the
  // scalar cache and dealt over the wave groups like the rectangles, culled
  // on their box keys.  The same in/out form: a segment crosses a convex
  // boundary once when exactly one end point is strictly inside (on the
  // positive side of every edge line), never when both are, and twice when
  // both are outside and no line separates it from the polygon -- neither
  // an edge line with both end points strictly outside (a whole polygon lies
  // on the inner side of each of its edge lines), nor the segment's own line
  // with every vertex on one side.  Point sides are the edge-line tests the
  // edge-by-edge path makes, vertex sides its segment-line tests (the
  // latter only for waves holding a candidate segment); where one is
  // degenerate the count may resolve it either way.
  {
    typedef __attribute__((address_space(4))) const CPoly ConstCPoly;
    typedef int ci8 __attribute__((ext_vector_type(8)));
    typedef float cf8 __attribute__((ext_vector_type(8)));
    typedef __attribute__((address_space(4))) const ci8 ConstCI8;
    typedef __attribute__((address_space(4))) const cf8 ConstCF8;
    ConstCPoly* cp = (ConstCPoly*)(pl.cpolys + d.cpo);
    for (int q = rg; q < d.n_cpolys; q += R) {
      ConstCPoly& c = cp[q];
      const ci8 h = *(ConstCI8*)&c.kx0;  // box keys and vertex count in one load
      if (h[2] <= kx0 || h[0] >= kx1 || h[3] <= ky0 || h[1] >= ky1) continue;
      const int n = h[4];
      // every slot is loaded (those past n hold no edge and are not used),
      // so that the loads go out together
      const cf8 cex = *(ConstCF8*)c.ex, cney = *(ConstCF8*)c.ney, cnce = *(ConstCF8*)c.nce;
      uint32_t outw = 0, sepe = 0;  // some edge line / the same edge line has the point outside
#pragma unroll
      for (int e = 0; e < kCPolyMax; ++e) {
        if (e >= n) break;
        const float ex = cex[e], ney = cney[e], nce = cnce[e];
        uint32_t ow = 0;
#pragma unroll
        for (int s = 0; s <= K; ++s) {
          const float ev = fmaf(ex, py[s], fmaf(ney, px[s], nce));
          ow = __builtin_amdgcn_alignbit(ow, __float_as_uint(ev), 31);
        }
        outw |= ow;
        sepe |= ow & (ow << 1);
      }
      const uint32_t in = ~outw & kOnes;
      count((in ^ (in << 1)) & segmask);  // one end strictly inside
      const uint32_t cand = ~(in | (in << 1)) & ~sepe & segmask;
      if (__builtin_amdgcn_ballot_w64(cand != 0u) == 0ull) continue;
      uint32_t allneg = ~0u, allpos = ~0u;  // bit K - 1 - s: every vertex on one side of segment s's line
      const cf8 cvx = *(ConstCF8*)c.vx, cvy = *(ConstCF8*)c.vy;
#pragma unroll
      for (int v = 0; v < kCPolyMax; ++v) {
        if (v >= n) break;
        const uint32_t vw = pack_seg_sides<K>(cvx[v], cvy[v], dx, ndy, nc);
        allneg &= vw;
        allpos &= ~vw;
      }
      const uint32_t thr = cand & ~((allneg | allpos) << 1);
      count(thr);
      count(thr);
    }
  }
  // C.3 other polygons, edge by edge, by wave group 0 (consecutive edges
  // share vertex words; the other groups still take part in the staging
  // barriers).  An edge outside the wave's box is skipped like a rectangle (a
  // proper crossing lies strictly inside both the segment and the edge); the
  // vertex words are then recomputed for the next edge instead of carried over.
  uint32_t w0 = 0, wp = 0;
  bool have_w0 = false, have_wp = false;
  const EdgeRec* s_edge = reinterpret_cast<const EdgeRec*>(s_stage);
  const int chunk = pl.stage_floats / 8;  // edge records per LDS pass
  for (int e0 = 0; e0 < d.n_gedges; e0 += chunk) {
    const int ne = d.n_gedges - e0 < chunk ? d.n_gedges - e0 : chunk;
    if (e0 > 0) {
      __syncthreads();
      stage_records(pl, d, s_stage, e0, ne);
      __syncthreads();
    }
    if (active && rg == 0) {
      for (int e = 0; e < ne; ++e) {
        const EdgeRec r = s_edge[e];
        const int fl = __builtin_amdgcn_readfirstlane(r.flags);
        if (fl & EDGE_FIRST) {
          have_w0 = false;
          have_wp = false;
        }
        if (fmaxf(r.ax, r.bx) <= bx0 || fminf(r.ax, r.bx) >= bx1 || fmaxf(r.ay, r.by) <= by0 ||
            fminf(r.ay, r.by) >= by1) {
          have_wp = false;
          continue;
        }
        if (!have_wp) {
          wp = pack_seg_sides<K>(r.ax, r.ay, dx, ndy, nc);
          if (fl & EDGE_FIRST) {
            w0 = wp;
            have_w0 = true;
          }
        }
        uint32_t wn;
        if ((fl & EDGE_LAST) && have_w0)
          wn = w0;  // the closing edge ends at the first vertex
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
        count((wp ^ wn) & (ew ^ (ew >> 1)));
        wp = wn;
        have_wp = true;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Fused iteration over one block = ppb consecutive particles of an instance
// (flat index g*N + n, possibly spanning groups; at most one particle per
// thread).
//
//  A. previous iteration's update, elementwise and coalesced over the
//     block's contiguous (particle, coordinate) range; new positions also
//     go to LDS, where they stay for the whole launch.  Every global read
//     the block needs -- its X, V, P range, the gbest rows of its groups and
//     Tbest, the hyper-parameters, its particles' old Pbest fitness and the
//     first chunk of obstacle records -- is issued before the first barrier,
//     so the block waits on memory about once;
//  B. a particle's W+1 segments are cut into C chunks of K; thread t takes
//     chunk t / ppb of particle t mod ppb (slots past the last segment are
//     masked out);
//  C. crossings of the K segments with every obstacle edge: rectangles and
//     convex polygons by their points' inside words (records through the
//     scalar cache), other polygons edge by edge (records staged in LDS):
//     one packed side word of the edge's end vertex against the K segment
//     lines and one of the K+1 points against the edge line, crossing bits
//     = both straddle;
//  D. per-particle Q and L summed in chunk order (deterministic), fitness
//     and Pbest; improved particles' positions go from LDS to P.
// ---------------------------------------------------------------------------
template <int K, int R, bool FIT>
__device__ __forceinline__ void iteration(const Pools& pl, int flags) {
  // dynamic LDS: positions | obstacle records | Tbest and the gbest rows of
  // the block's groups | an 8-word record per particle (Pbest flags in phase
  // D) | per group w, V_limit / 2, C1..C3 | per-thread crossings (the old
  // Pbest fitness of particle t until then) and lengths
  extern __shared__ __attribute__((aligned(16))) float s_dyn[];
  float* s_buf = s_dyn;
  float* s_stage = s_buf + pl.pos_floats;
  float* s_gb = s_stage + pl.stage_floats;
  float* s_c = s_gb + pl.gb_floats;
  float* s_wv = s_c + 8 * pl.ppb_max;
  int* s_q = reinterpret_cast<int*>(s_wv + 5 * pl.ngb_max);
  float* s_l = reinterpret_cast<float*>(s_q + blockDim.x);
  int* s_imp = reinterpret_cast<int*>(s_c);  // phase D: the records are dead by then

  const int2 bt = pl.blk_tiles[blockIdx.x];
  const int inst = bt.x, p0 = bt.y;
  const InstDesc d = pl.desc[inst];  // by value: stores cannot make it reload
  InstCtl* ctl = pl.ctl + inst;
  if ((flags & STEP_FRAME) && ctl->done) return;
  const int k = ctl->k, pending = ctl->pending;
  const uint32_t ctr = ctl->ctr;
  const int N = d.N, W = d.W, D = 2 * W, S = W + 2;
  const int np = min(d.ppb, d.G * N - p0);  // particles in this block
  const int t = threadIdx.x, B = blockDim.x;
  const float4 ends = pl.ends[inst];  // read before the block's first store

  // ---- A0. the block's global reads ------------------------------------------
  // The block's range starts 16-byte aligned (even particles per block) and
  // the pools are padded to whole float4 groups per instance, so the walk
  // goes by float4 groups of elements and reads and writes whole groups: an
  // instance's last group carries up to 3 padding floats, which are never
  // computed on and are written back as read.  Positions (group gi at LDS
  // word 4 gi), the first chunk of obstacle records, Tbest and the gbest
  // rows of the block's groups and the particles' old Pbest fitness go
  // straight to LDS; a thread's V and P groups and its particle's and group's
  // hyper-parameters to registers.  All of it is issued before the first
  // barrier, so that the block waits on memory once.
  const int lane = t & 63, w0 = t - lane;
  float4* X4 = reinterpret_cast<float4*>(pl.X + d.xo + (int64_t)p0 * D);
  float4* V4 = reinterpret_cast<float4*>(pl.V + d.xo + (int64_t)p0 * D);
  const float4* P4 = reinterpret_cast<const float4*>(pl.P + d.xo + (int64_t)p0 * D);
  const int nel = np * D, ng = (nel + 3) >> 2;
  float4* B4 = reinterpret_cast<float4*>(s_buf);
  constexpr int CH = 4;
  float4 va[CH], pa[CH];
  auto load = [&](int g0) {  // g0 = t + multiple of CH * B
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int gi = g0 + c * B;
      if (gi < ng) {
        lds_dma16_stream(X4 + gi, B4 + (gi - lane));
        if (pending) {
          va[c] = ld_stream(V4 + gi);
          pa[c] = ld_stream(P4 + gi);
        }
      }
    }
  };
  load(t);
  if (FIT) {
    // first chunk of the other polygons' edge records (float4 words)
    const int n4 = 2 * min(d.n_gedges, pl.stage_floats / 8);
    const float4* src = reinterpret_cast<const float4*>(pl.edges + d.geo);
    float4* dst = reinterpret_cast<float4*>(s_stage);
    for (int q = t; q < n4; q += B) lds_dma16(src + q, dst + (q - lane));
    // old Pbest fitness of particle t, parked in thread t's crossing slot
    if (t < np) lds_dma4(pl.Pf + d.po + p0 + t, s_q + w0);
  }
  const int g_lo = p0 / N, g_hi = (p0 + np - 1) / N, ngb = g_hi - g_lo + 1;
  const bool has_p = pending && t < np, has_g = pending && t < ngb;
  const int gp = (p0 + t) / N;  // the thread's particle's group
  float hpv[6], hgv[6];
  if (pending) {
    // Tbest row, then the gbest rows g_lo..g_hi (contiguous in the pool)
    const float* src_t = pl.tbest_pos + d.dpo;
    const float* src_g = pl.gbest_pos + d.gpo + g_lo * D;
    for (int q = t; q < D; q += B) lds_dma4(src_t + q, s_gb + (q - lane));
    for (int q = t; q < ngb * D; q += B) lds_dma4(src_g + q, s_gb + D + (q - lane));
    const float* hp = pl.hyper + (d.go + (has_p ? gp : 0)) * 6;
    const float* hg = pl.hyper + (d.go + g_lo + (has_g ? t : 0)) * 6;
#pragma unroll
    for (int i = 0; i < 6; ++i) hpv[i] = has_p ? hp[i] : 0.f;
#pragma unroll
    for (int i = 0; i < 6; ++i) hgv[i] = has_g ? hg[i] : 0.f;
  }

  // ---- A1. per-particle and per-group constants into LDS -------------------------
  // Per particle an 8-word record: one Philox call's r1..r3 scaled by the
  // group's C1..C3, the group's inertia of Eq.(6) and V_limit / 2, the LDS
  // offset of its gbest row and its group.  Per group the same inertia and
  // V_limit / 2 and C1..C3 (read by the per-coordinate variant).
  if (pending) {
    const int kk = k < d.T ? k : d.T;
    auto inertia = [&](const float* h) { return h[3] - (h[3] - h[4]) / (float)d.T * (float)kk; };
    auto put_group = [&](int gl, const float* h) {
      float* q = s_wv + 5 * gl;
      q[0] = inertia(h);
      q[1] = h[5] * 0.5f;
      q[2] = h[0];
      q[3] = h[1];
      q[4] = h[2];
    };
    if (has_p) {
      const U4 r = philox((uint32_t)(p0 + t), ctr, d.instance, TAG_UPDATE, d.seed_lo, d.seed_hi);
      const int gl = gp - g_lo;
      float4* rec = reinterpret_cast<float4*>(s_c + 8 * t);
      rec[0] = make_float4(hpv[0] * u01(r.v[0]), hpv[1] * u01(r.v[1]), hpv[2] * u01(r.v[2]),
                           inertia(hpv));
      rec[1] = make_float4(hpv[5] * 0.5f, __int_as_float((gl + 1) * D), __int_as_float(gl), 0.f);
    }
    if (has_g) put_group(t, hgv);
    for (int gl = t + B; gl < ngb; gl += B) put_group(gl, pl.hyper + (d.go + g_lo + gl) * 6);
  }
  __syncthreads();

  // ---- A2. update ---------------------------------------------------------------
  // The element loop walks (particle, coordinate) incrementally, without
  // divisions; groups past a thread's first CH are read chunk by chunk (the
  // thread's own lanes' words, so no barrier).  After the first barrier
  // nothing in the block waits on the vector-memory counter, which stores and
  // loads share: the stores drain while the block goes on.
  {
    const int qB = (4 * B) / D, rB = 4 * B - qB * D;
    int j = (4 * t) / D, dd = 4 * t - j * D;  // particle and coordinate of group's first element
    auto update = [&](int g0) {
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int gi = g0 + c * B, e = 4 * gi;
        if (gi < ng && pending) {
          float4 xv = B4[gi];
          float* xs = &xv.x;
          float* vs = &va[c].x;
          const float* ps = &pa[c].x;
          int jj = j, di = dd;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if (e + i < nel) {
              const float4 c0 = *reinterpret_cast<const float4*>(s_c + 8 * jj);
              const float4 c1 = *reinterpret_cast<const float4*>(s_c + 8 * jj + 4);
              const float w = c0.w, vlh = c1.x;
              float a1 = c0.x, a2 = c0.y, a3 = c0.z;
              if (d.rand_per_dim) {  // variant: factors per coordinate
                const float* q = s_wv + 5 * __float_as_int(c1.z);
                const U4 r = philox((uint32_t)((p0 + jj) * D + di), ctr, d.instance,
                                    TAG_UPDATE_DIM, d.seed_lo, d.seed_hi);
                a1 = q[2] * u01(r.v[0]);
                a2 = q[3] * u01(r.v[1]);
                a3 = q[4] * u01(r.v[2]);
              }
              const float hi = di < W ? d.width : d.height;
              const float vmax = vlh * hi;
              const float x = xs[i];
              const float gx = s_gb[__float_as_int(c1.y) + di], tx = s_gb[di];
              float v = w * vs[i] + a1 * (ps[i] - x) + a2 * (gx - x) + a3 * (tx - x);
              v = clampf(v, -vmax, vmax);
              vs[i] = v;
              xs[i] = clampf(x + v, 0.f, hi);
            }
            if (++di == D) {
              di = 0;
              ++jj;
            }
          }
          B4[gi] = xv;
          st_stream(X4 + gi, xv);
          st_stream(V4 + gi, va[c]);
        }
        dd += rB;
        j += qB;
        while (dd >= D) {
          dd -= D;
          ++j;
        }
      }
    };
    update(t);
    for (int g0 = t + CH * B; g0 < ng; g0 += CH * B) {
      load(g0);
      update(g0);
    }
  }
  if (!FIT) return;
  __syncthreads();

  // ---- B. this thread's K segments --------------------------------------------
  // A particle's W+1 segments are cut into C chunks of K.  The block's waves
  // form R groups of B/R threads (R = 1 unless the launch would leave most
  // CUs idle); in each group thread u takes chunk u / ppb of particle
  // u mod ppb, so the 64 lanes of a wave hold the same stretch of 64
  // neighbouring paths -- close together once the swarm converges, which is
  // what the culling in phase C feeds on -- and group r tests every R-th
  // rectangle from the r-th on.
  const int C = (W + K) / K;
  const int BR = R == 1 ? B : B / R;
  const int rg = R == 1 ? 0 : __builtin_amdgcn_readfirstlane(t / BR);  // whole waves: uniform
  const int u = t - rg * BR;
  const int c = u / d.ppb, jt = u - c * d.ppb;
  const bool active = c < C && jt < np;
  const int jc = active ? jt : 0;  // inactive lanes read a valid particle, count nothing
  const int i0 = c * K;           // first point index of the chunk
  // Point i0+s of the path (clamped to the target): start, waypoint, or
  // target.  Waypoints are read at a clamped index, without branches; only
  // point 0 of chunk 0 can be the start.
  float px[K + 1], py[K + 1];
  const float* sx = s_buf + jc * D;
#pragma unroll
  for (int s = 0; s <= K; ++s) {
    const int idx = min(i0 + s, S - 1);
    const int wi = min(max(idx - 1, 0), W - 1);
    const bool tgt = idx == S - 1;
    float x = sx[wi], y = sx[W + wi];
    x = tgt ? ends.z : x;
    y = tgt ? ends.w : y;
    if (s == 0) {
      x = idx == 0 ? ends.x : x;
      y = idx == 0 ? ends.y : y;
    }
    px[s] = x;
    py[s] = y;
  }
  float dx[K], ndy[K], nc[K];
  float len_sum = 0.f;
#pragma unroll
  for (int s = 0; s < K; ++s) {
    const float ddx = px[s + 1] - px[s], ddy = py[s + 1] - py[s];
    const bool seg = active && i0 + s < S - 1;  // segment i0+s of W+1
    // A slot that is no path segment gets the zero line: every vertex side
    // is +0 (coordinates are >= 0), so its side bits never differ and it
    // never counts as a crossing.
    dx[s] = seg ? ddx : 0.f;
    ndy[s] = seg ? -ddy : 0.f;
    nc[s] = seg ? fmaf(ddy, px[s], -(ddx * py[s])) : 0.f;
    if (seg) len_sum += __builtin_amdgcn_sqrtf(ddx * ddx + ddy * ddy);  // v_sqrt_f32, 1 ulp
  }
  if (rg != 0) len_sum = 0.f;  // each length is summed once, by group 0

  // ---- C. crossings ----------------------------------------------------------
  int ct = 0;
  crossings<K, R>(pl, d, s_stage, active, rg, px, py, dx, ndy, nc, ct);

  // ---- D. per-particle fitness and Pbest -------------------------------------
  const float pf_old = reinterpret_cast<const float*>(s_q)[t];  // before the slot is reused
  s_q[t] = ct;
  s_l[t] = len_sum;
  __syncthreads();
  if (t < np) {
    const int j = t;
    int q = 0;
    float L = 0.f;
    for (int cc = 0; cc < C; ++cc) {  // chunk order: deterministic
      for (int r = 0; r < R; ++r) q += s_q[r * BR + j + cc * d.ppb];
      L += s_l[j + cc * d.ppb];  // lengths from group 0 only
    }
    const float qf = (float)q;
    float pw = 1.f;
    for (int b = 0; b < d.beta; ++b) pw *= qf;
    const float fv = L + d.alpha * pw;
    const int64_t po = d.po + p0 + j;
    pl.f[po] = fv;
    pl.L[po] = L;
    pl.Q[po] = q;
    const float fc = isfinite(fv) ? fv : INFINITY;
    const int imp = fc < pf_old;
    if (imp) {
      pl.Pf[po] = fc;
      pl.PL[po] = L;
      pl.PQ[po] = q;
    }
    s_imp[j] = imp;
  }
  __syncthreads();
  // Improved particles' rows go to P from the LDS copy of the new positions,
  // by the same float4 walk as phase A.
  {
    float4* P4w = reinterpret_cast<float4*>(pl.P + d.xo + (int64_t)p0 * D);
    float* Ps = pl.P + d.xo + (int64_t)p0 * D;
    const int qB = (4 * B) / D, rB = 4 * B - qB * D;
    int j = (4 * t) / D, dd = 4 * t - j * D;
    for (int gi = t; gi < ng; gi += B) {
      const int e = 4 * gi;
      const int jl = j + (dd + 3 >= D ? 1 : 0);  // particle of the group's last element (dd + 3 < 2D)
      if (e + 4 <= nel && s_imp[j] && s_imp[jl]) {
        P4w[gi] = B4[gi];
      } else if (s_imp[j] || (jl < np && s_imp[jl])) {
        int jj = j, di = dd;
        for (int i = 0; i < 4; ++i) {
          if (e + i < nel && s_imp[jj]) Ps[e + i] = s_buf[e + i];
          if (++di == D) {
            di = 0;
            ++jj;
          }
        }
      }
      dd += rB;
      j += qB;
      while (dd >= D) {
        dd -= D;
        ++j;
      }
    }
  }
}

// One fused iteration (fitness path), the same with the rectangles dealt over
// R wave groups (launches with few blocks), and the update-only flush, as
// separate kernels so that profiles separate them.  Up to K = 8 the plain
// kernel is held to six waves per SIMD (80 VGPRs): its blocks spend most of
// their time waiting on the swarm's loads, and a sixth block per CU hides
// more of that than the four VGPRs it gives up cost.
template <int K>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(K <= 8 ? 6 : 1))) void
iter_kernel(Pools pl, int flags) {
  iteration<K, 1, true>(pl, flags);
}
template <int K, int R>
__global__ __launch_bounds__(256) void iter_kernel_split(Pools pl, int flags) {
  iteration<K, R, true>(pl, flags);
}
template <int K>
__global__ __launch_bounds__(256) void update_kernel(Pools pl, int flags) {
  iteration<K, 1, false>(pl, flags);
}

// ---------------------------------------------------------------------------
void launch_geom(const Pools& pl, int n_inst, int move, hipStream_t s) {
  hipLaunchKernelGGL(geom_kernel, dim3(n_inst), dim3(256), 0, s, pl, move);
}

void launch_init(const Pools& pl, int n_blocks, int frame_override, int use_prev, hipStream_t s) {
  hipLaunchKernelGGL(init_kernel, dim3(n_blocks), dim3(256), 0, s, pl, frame_override, use_prev);
}

size_t iter_lds_words(int pos_floats, int stage_floats, int gb_floats, int ngb_max, int ppb_max,
                      int threads) {
  return (size_t)pos_floats + stage_floats + gb_floats + 8 * (size_t)ppb_max + 5 * (size_t)ngb_max +
         2 * (size_t)threads;
}

size_t iter_lds_bytes(const Pools& pl, int threads) {
  return 4 * iter_lds_words(pl.pos_floats, pl.stage_floats, pl.gb_floats, pl.ngb_max, pl.ppb_max,
                            threads);
}

bool step_supported(int K) { return K == 4 || K == 8 || K == 12 || K == 16 || K == 24; }

template <int K>
static void launch_tiles_k(const Pools& pl, int n_blocks, int threads, int flags, hipStream_t s) {
  const size_t lds = iter_lds_bytes(pl, threads);
  if ((flags & STEP_FIT) && pl.rsplit == 4)
    hipLaunchKernelGGL((iter_kernel_split<K, 4>), dim3(n_blocks), dim3(threads), lds, s, pl, flags);
  else if ((flags & STEP_FIT) && pl.rsplit == 2)
    hipLaunchKernelGGL((iter_kernel_split<K, 2>), dim3(n_blocks), dim3(threads), lds, s, pl, flags);
  else if (flags & STEP_FIT)
    hipLaunchKernelGGL(iter_kernel<K>, dim3(n_blocks), dim3(threads), lds, s, pl, flags);
  else
    hipLaunchKernelGGL(update_kernel<K>, dim3(n_blocks), dim3(threads), lds, s, pl, flags);
}

bool launch_tiles(const Pools& pl, int K, int n_blocks, int threads, int flags, hipStream_t s) {
  if (n_blocks <= 0) return true;
  switch (K) {
    case 4: launch_tiles_k<4>(pl, n_blocks, threads, flags, s); return true;
    case 8: launch_tiles_k<8>(pl, n_blocks, threads, flags, s); return true;
    case 12: launch_tiles_k<12>(pl, n_blocks, threads, flags, s); return true;
    case 16: launch_tiles_k<16>(pl, n_blocks, threads, flags, s); return true;
    case 24: launch_tiles_k<24>(pl, n_blocks, threads, flags, s); return true;
    default: return false;
  }
}

void launch_reduce(const Pools& pl, int flags, hipStream_t s) {
  // few instances: eight waves per block, so that each of (typically) eight
  // groups gets a wave of its own and the launch's latency is one scan;
  // a full batch keeps four waves per block (more blocks resident)
  const int red_threads = pl.n_inst < 256 ? 512 : 256;
  hipLaunchKernelGGL(reduce_kernel, dim3(pl.n_inst), dim3(red_threads), 0, s, pl, flags);
}

// ---------------------------------------------------------------------------
// Evolution phase (Sec. "Hierarchical Self-evolving Framework", Eq.(9)): H
// particle i is lower-level instance i's whole (G_L, 6) hyper matrix; its
// fitness is that instance's frame result (the lowest fitness value of a full
// lower-level run).  Column c of a row is boxed to [lo[c], hi[c]].
// ---------------------------------------------------------------------------

// Where H particle i's position goes for the lower level: its own row of an
// external hyper array, or its batch instance's slice of the hyper pool.
__device__ __forceinline__ float* evolve_dst(const EvolveDev& ev, const Pools& pl, int i) {
  return ev.hyper_out ? ev.hyper_out + (int64_t)i * ev.Dh : pl.hyper + 6 * pl.desc[i].go;
}

// Uniform positions in the box, velocities in +-V_limit * half the column's
// extent; the lower level's hyper-parameters receive the positions.
__global__ __launch_bounds__(256) void evolve_init_kernel(EvolveDev ev, Pools pl) {
  const int n = ev.Gh * ev.Nh, Dh = ev.Dh, nb = (Dh + 3) / 4;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n * Dh) {
    const int i = e / Dh, d = e - i * Dh, c = d % 6, g = i / ev.Nh;
    const float lo = ev.lo[c], hi = ev.hi[c];
    const float vmax = ev.h_hyper[6 * g + 5] * (hi - lo) * 0.5f;
    const uint32_t c0 = (uint32_t)(i * nb + d / 4);
    const U4 rx = philox(c0, 0u, 0u, TAG_EVOLVE_X, ev.seed_lo, ev.seed_hi);
    const U4 rv = philox(c0, 0u, 0u, TAG_EVOLVE_V, ev.seed_lo, ev.seed_hi);
    const float x = lo + u01(rx.v[d & 3]) * (hi - lo);
    ev.X[e] = x;
    ev.P[e] = x;
    ev.V[e] = -vmax + u01(rv.v[d & 3]) * (2.f * vmax);
    evolve_dst(ev, pl, i)[d] = x;
  }
  if (e < n) {
    ev.Pf[e] = INFINITY;
    ev.lfv[e] = INFINITY;
  }
  if (e < ev.Gh) {
    ev.gbest_n[e] = 0;
    ev.gbest_f[e] = INFINITY;
  }
  if (e == 0) {
    ev.ctl->k = 0;
    ev.ctl->ctr = 0u;
    ev.ctl->tb_g = ev.ctl->tb_n = 0;
    ev.ctl->tb_f = INFINITY;
  }
}

// One evolution after the lower-level frame: H bests (Pbest = running
// minimum, Gbest = lowest Pbest of the group, lowest index on ties; Tbest =
// lowest Gbest), then the move of Eq.(6)-(8) with one (r1, r2, r3) per H
// particle; new positions go to the lower level's hyper-parameters.  One
// block.  Without injection the fitness is the batch instance's frame result.
__global__ __launch_bounds__(1024) void evolve_step_kernel(EvolveDev ev, Pools pl, int injected) {
  __shared__ float s_r[3 * kEvolveMaxH];
  __shared__ int s_imp[kEvolveMaxH];
  __shared__ float s_gf[kMaxG];
  __shared__ int s_gn[kMaxG];
  __shared__ int s_tg;
  const int t = threadIdx.x, nt = blockDim.x;
  const int Gh = ev.Gh, Nh = ev.Nh, n = Gh * Nh, Dh = ev.Dh;
  const int k = ev.ctl->k + 1;
  const uint32_t ctr = ev.ctl->ctr;
  for (int i = t; i < n; i += nt) {
    float f = injected ? ev.lfv_in[i] : pl.ctl[i].res_cost;
    if (!(fabsf(f) <= 3.402823466e38f)) f = INFINITY;  // NaN / inf -> +inf
    ev.lfv[i] = f;
    const bool imp = f < ev.Pf[i];
    if (imp) ev.Pf[i] = f;
    s_imp[i] = imp;
    const U4 r = philox((uint32_t)i, ctr, 0u, TAG_EVOLVE, ev.seed_lo, ev.seed_hi);
    s_r[3 * i + 0] = u01(r.v[0]);
    s_r[3 * i + 1] = u01(r.v[1]);
    s_r[3 * i + 2] = u01(r.v[2]);
  }
  __syncthreads();
  for (int e = t; e < n * Dh; e += nt)
    if (s_imp[e / Dh]) ev.P[e] = ev.X[e];
  if (t < Gh) {
    int b = 0;
    for (int m = 1; m < Nh; ++m)
      if (ev.Pf[t * Nh + m] < ev.Pf[t * Nh + b]) b = m;
    s_gn[t] = b;
    s_gf[t] = ev.Pf[t * Nh + b];
    ev.gbest_n[t] = b;
    ev.gbest_f[t] = s_gf[t];
  }
  __syncthreads();
  if (t == 0) {
    int tg = 0;
    for (int g = 1; g < Gh; ++g)
      if (s_gf[g] < s_gf[tg]) tg = g;
    s_tg = tg;
  }
  __syncthreads();
  const int tg = s_tg, tn = s_gn[tg];
  const int kk = k < ev.E ? k : ev.E;
  for (int e = t; e < n * Dh; e += nt) {
    const int i = e / Dh, d = e - i * Dh, c = d % 6, g = i / Nh;
    const float* hy = ev.h_hyper + 6 * g;
    const float w = hy[3] - (hy[3] - hy[4]) / (float)ev.E * (float)kk;
    const float lo = ev.lo[c], hi = ev.hi[c], vmax = hy[5] * (hi - lo) * 0.5f;
    const float x = ev.X[e], p = ev.P[e];
    const float gb = ev.P[(g * Nh + s_gn[g]) * Dh + d], tb = ev.P[(tg * Nh + tn) * Dh + d];
    float v = w * ev.V[e] + hy[0] * s_r[3 * i] * (p - x) + hy[1] * s_r[3 * i + 1] * (gb - x) +
              hy[2] * s_r[3 * i + 2] * (tb - x);
    v = clampf(v, -vmax, vmax);
    const float xn = clampf(x + v, lo, hi);
    ev.V[e] = v;
    ev.X[e] = xn;
    evolve_dst(ev, pl, i)[d] = xn;
  }
  if (t == 0) {
    ev.curve[(k - 1) % ev.E] = s_gf[tg];
    ev.ctl->k = k;
    ev.ctl->ctr = ctr + 1u;
    ev.ctl->tb_g = tg;
    ev.ctl->tb_n = tn;
    ev.ctl->tb_f = s_gf[tg];
  }
}

void launch_evolve_init(const EvolveDev& ev, const Pools& pl, hipStream_t s) {
  const int total = ev.Gh * ev.Nh * ev.Dh;
  hipLaunchKernelGGL(evolve_init_kernel, dim3((total + 255) / 256), dim3(256), 0, s, ev, pl);
}

void launch_evolve_step(const EvolveDev& ev, const Pools& pl, int injected, hipStream_t s) {
  hipLaunchKernelGGL(evolve_step_kernel, dim3(1), dim3(1024), 0, s, ev, pl, injected);
}

}  // namespace sepso
