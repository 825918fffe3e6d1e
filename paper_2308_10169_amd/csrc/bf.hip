// Benchmark-function workload (Table BFs; Sec. "Standard benchmark
// functions" and "Large-scale benchmark functions"): the same DTPSO step
// (Algorithm 1, Eq.(6)-(8)) minimising Sphere, Rosenbrock, Rastrigin or
// Griewank over [lo, hi]^D, for swarms up to HBM size (the paper's large
// case is 16K particles x 1K dimensions).
//
// The step is bound by HBM traffic: per element one read of X, V and P and
// one write of X and V (20 bytes); the group-best rows stay in L2.  One wave
// owns one particle row (rows padded to a multiple of 4 floats, float4
// accesses), so the fitness reduction is a wave reduction without LDS or
// barriers; four particles per 256-thread block.
//
//   bf_init_kernel   -- uniform swarm in the box;
//   bf_iter_kernel   -- pending move (with the previous iteration's bests),
//                       fitness of the new position, Pbest;
//   bf_reduce_kernel -- one block per group: Gbest (lowest Pbest, lowest
//                       index on ties) and its row; block 0 advances the
//                       control word.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/sepso.h"
#include "common.h"
#include "internal.h"
#include "kernels.h"
#include "rng.h"

namespace sepso {

enum : uint32_t { TAG_BF_UPDATE = 9, TAG_BF_INIT_X = 10, TAG_BF_INIT_V = 11 };
enum : int32_t { BF_SPHERE = 1, BF_ROSENBROCK = 2, BF_RASTRIGIN = 3, BF_GRIEWANK = 4 };

struct BFCtl {
  int32_t k;        // iterations evaluated
  uint32_t ctr;     // random stream position of the move
  int32_t pending;  // a move is owed before the next evaluation
  int32_t pad;
};

struct BFDev {
  int32_t func, G, N, D, Dp, T;  // G: groups of all swarms
  int32_t S, Gs;                 // independent swarms, groups per swarm (G = S * Gs)
  const int32_t* run;            // counter word 1 of the initial draws (NULL: 0)
  float lo, hi;
  uint32_t seed_lo, seed_hi;
  float *X, *V, *P;  // (G*N) x Dp
  float *f, *Pf;     // G*N
  int32_t* gbest_n;  // G
  float* gbest_f;    // G
  float* gbest_pos;  // G x Dp
  const float* hyper;  // G*6
  BFCtl* ctl;
};

__global__ __launch_bounds__(256) void bf_init_kernel(BFDev s) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)s.G * s.N * s.Dp;
  if (e >= total) return;
  const int i = (int)(e / s.Dp), d = (int)(e - (int64_t)i * s.Dp), g = i / s.N;
  float x = 0.f, v = 0.f;
  if (d < s.D) {
    // swarm sw's particle il: counter (il * Dp/4 + d/4, run, sw, tag)
    const int sw = g / s.Gs, il = i - sw * s.Gs * s.N;
    const uint32_t run = s.run ? (uint32_t)*s.run : 0u;
    const uint32_t c0 = (uint32_t)il * (uint32_t)(s.Dp / 4) + (uint32_t)(d / 4);
    const U4 rx = philox(c0, run, (uint32_t)sw, TAG_BF_INIT_X, s.seed_lo, s.seed_hi);
    const U4 rv = philox(c0, run, (uint32_t)sw, TAG_BF_INIT_V, s.seed_lo, s.seed_hi);
    const float vmax = s.hyper[6 * g + 5] * (s.hi - s.lo) * 0.5f;
    x = s.lo + u01(rx.v[d & 3]) * (s.hi - s.lo);
    v = -vmax + u01(rv.v[d & 3]) * (2.f * vmax);
  }
  s.X[e] = x;
  s.P[e] = x;
  s.V[e] = v;
  if (d == 0) {
    s.f[i] = INFINITY;
    s.Pf[i] = INFINITY;
  }
  if (e < s.G) {
    s.gbest_n[e] = 0;
    s.gbest_f[e] = INFINITY;
  }
  if (e == 0) *s.ctl = BFCtl{0, 0u, 0, 0};
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) x += __shfl_xor(x, m);
  return x;
}
__device__ __forceinline__ float wave_prod(float x) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) x *= __shfl_xor(x, m);
  return x;
}

// One coordinate's move (Eq.(7)-(8)) and one lane's four function terms:
// shared by the stepwise and the whole-run kernels, so that both compute the
// same FP32 operations in the same order.
__device__ __forceinline__ float bf_move(float x, float& v, float p, float gb, float tb, float w, float a1,
                                         float a2, float a3, float vmax, float lo, float hi) {
  float nv = w * v + a1 * (p - x) + a2 * (gb - x) + a3 * (tb - x);
  nv = clampf(nv, -vmax, vmax);
  v = nv;
  return clampf(x + nv, lo, hi);
}

// Terms of elements e .. e+3 (those below D) into acc (and prod for
// Griewank); prev = the element before e (Rosenbrock's pair).
template <int FUNC>
__device__ __forceinline__ void bf_terms(const float (&xv)[4], float prev, int e, int D, float& acc,
                                         float& prod) {
  if (FUNC == BF_ROSENBROCK) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int d = e + j;
      const float xm = j == 0 ? prev : xv[j - 1];
      if (d >= 1 && d < D) {
        const float a = xv[j] - xm * xm, b = 1.f - xm;
        acc += 100.f * a * a + b * b;
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int d = e + j;
      if (d < D) {
        const float x = xv[j];
        if (FUNC == BF_SPHERE) acc += x * x;
        if (FUNC == BF_RASTRIGIN) acc += x * x + 10.f * (1.f - cospif(2.f * x));
        if (FUNC == BF_GRIEWANK) {
          acc += x * x * (1.f / 4000.f);
          prod *= cosf(x / sqrtf((float)(d + 1)));
        }
      }
    }
  }
}

template <int FUNC, bool FIT>
__global__ __launch_bounds__(256) void bf_iter_kernel(BFDev s) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);  // particle of this wave
  if (i >= s.G * s.N) return;                          // whole wave leaves
  const BFCtl c = *s.ctl;
  const int g = i / s.N, D = s.D, Dp = s.Dp;
  const int sw = g / s.Gs, g0 = sw * s.Gs;  // this particle's swarm and its first group
  float4* X = reinterpret_cast<float4*>(s.X + (int64_t)i * Dp);
  float4* V = reinterpret_cast<float4*>(s.V + (int64_t)i * Dp);
  const float4* Pp = reinterpret_cast<const float4*>(s.P + (int64_t)i * Dp);

  // move coefficients (Eq.(6)-(7)) and the Tbest row = Gbest row of the
  // lowest group (lowest group index on ties)
  float w = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, vmax = 0.f;
  const float4 *Gb = nullptr, *Tb = nullptr;
  if (c.pending) {
    const float* h = s.hyper + 6 * g;
    const int kk = c.k < s.T ? c.k : s.T;
    w = h[3] - (h[3] - h[4]) / (float)s.T * (float)kk;
    vmax = h[5] * (s.hi - s.lo) * 0.5f;
    const U4 r = philox((uint32_t)(i - g0 * s.N), c.ctr, (uint32_t)sw, TAG_BF_UPDATE, s.seed_lo,
                        s.seed_hi);
    a1 = h[0] * u01(r.v[0]);
    a2 = h[1] * u01(r.v[1]);
    a3 = h[2] * u01(r.v[2]);
    // Tbest of this particle's own swarm
    float bf = lane < s.Gs ? s.gbest_f[g0 + lane] : INFINITY;
    int bn = lane < s.Gs ? lane : 0x7fffffff;
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
      const float of = __shfl_xor(bf, m);
      const int on = __shfl_xor(bn, m);
      if (of < bf || (of == bf && on < bn)) {
        bf = of;
        bn = on;
      }
    }
    const int tg = g0 + (bn < s.Gs ? bn : 0);
    Gb = reinterpret_cast<const float4*>(s.gbest_pos + (int64_t)g * Dp);
    Tb = reinterpret_cast<const float4*>(s.gbest_pos + (int64_t)tg * Dp);
  }

  float acc = 0.f, prod = 1.f, carry = 0.f;
  for (int e0 = 0; e0 < Dp; e0 += 256) {
    const int e = e0 + 4 * lane, q = e >> 2;
    float xv[4] = {0.f, 0.f, 0.f, 0.f};
    if (e < Dp) {
      float4 x4 = X[q];
      if (c.pending) {
        float4 v4 = V[q];
        const float4 p4 = Pp[q], g4 = Gb[q], t4 = Tb[q];
        float* xs = &x4.x;
        float* vs = &v4.x;
        const float* ps = &p4.x;
        const float* gs = &g4.x;
        const float* ts = &t4.x;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (e + j < D) xs[j] = bf_move(xs[j], vs[j], ps[j], gs[j], ts[j], w, a1, a2, a3, vmax, s.lo, s.hi);
        X[q] = x4;
        V[q] = v4;
      }
      xv[0] = x4.x;
      xv[1] = x4.y;
      xv[2] = x4.z;
      xv[3] = x4.w;
    }
    if (FIT) {
      // Rosenbrock pairs (x[j-1], x[j]): the element before this lane's
      // first comes from the previous lane, or for lane 0 from the previous
      // chunk
      float prev = 0.f;
      if (FUNC == BF_ROSENBROCK) {
        prev = __shfl_up(xv[3], 1);
        if (lane == 0) prev = carry;
        carry = __shfl(xv[3], 63);
      }
      bf_terms<FUNC>(xv, prev, e, D, acc, prod);
    }
  }
  if (!FIT) return;
  float fv = wave_sum(acc);
  if (FUNC == BF_GRIEWANK) fv = 1.f + fv - wave_prod(prod);
  if (!(fabsf(fv) <= 3.402823466e38f)) fv = INFINITY;
  const bool imp = fv < s.Pf[i];
  if (lane == 0) {
    s.f[i] = fv;
    if (imp) s.Pf[i] = fv;
  }
  if (imp) {  // wave-uniform; the row was just written, so it reads from L2
    float4* P = reinterpret_cast<float4*>(s.P + (int64_t)i * Dp);
    for (int q = lane; q < Dp / 4; q += 64) P[q] = X[q];
  }
}

__global__ __launch_bounds__(256) void bf_reduce_kernel(BFDev s, int fit) {
  __shared__ float s_f[256];
  __shared__ int s_n[256];
  const int g = blockIdx.x, t = threadIdx.x, N = s.N;
  if (fit) {
    float bf = INFINITY;
    int bn = 0x7fffffff;
    for (int n = t; n < N; n += blockDim.x) {
      const float f = s.Pf[g * N + n];
      if (f < bf || (f == bf && n < bn)) {
        bf = f;
        bn = n;
      }
    }
    s_f[t] = bf;
    s_n[t] = bn;
    __syncthreads();
    for (int m = blockDim.x / 2; m > 0; m >>= 1) {
      if (t < m) {
        const float of = s_f[t + m];
        const int on = s_n[t + m];
        if (of < s_f[t] || (of == s_f[t] && on < s_n[t])) {
          s_f[t] = of;
          s_n[t] = on;
        }
      }
      __syncthreads();
    }
    const int n = s_n[0] < N ? s_n[0] : 0;
    if (t == 0) {
      s.gbest_n[g] = n;
      s.gbest_f[g] = s_f[0];
    }
    const float4* src = reinterpret_cast<const float4*>(s.P + ((int64_t)g * N + n) * s.Dp);
    float4* dst = reinterpret_cast<float4*>(s.gbest_pos + (int64_t)g * s.Dp);
    for (int q = t; q < s.Dp / 4; q += blockDim.x) dst[q] = src[q];
  }
  if (g == 0 && t == 0) {  // the control word's only reader and writer in this launch
    const BFCtl c = *s.ctl;
    BFCtl n = c;
    n.ctr = c.ctr + (c.pending ? 1u : 0u);
    if (fit) {
      n.k = c.k + 1;
      n.pending = 1;
    } else {
      n.pending = 0;
    }
    *s.ctl = n;
  }
}

// Each swarm's total best fitness (the lowest of its groups' bests; non-finite
// as +inf), one thread per swarm.
__global__ __launch_bounds__(256) void bf_best_kernel(BFDev s, float* out) {
  const int sw = blockIdx.x * blockDim.x + threadIdx.x;
  if (sw >= s.S) return;
  float b = INFINITY;
  for (int g = sw * s.Gs; g < (sw + 1) * s.Gs; ++g) {
    const float f = s.gbest_f[g];
    if (f < b) b = f;
  }
  out[sw] = b;
}

// ---- whole run of a small swarm in one workgroup ----------------------------
// A swarm whose state fits in LDS (rows of at most 256 floats) runs all its
// iterations in one launch, one workgroup per swarm: the stepwise kernels'
// move, evaluation, Pbest and bests in the same order and arithmetic
// (bf_move, bf_terms, the same wave butterflies), with barriers instead of
// kernel boundaries, so the results are bit-identical.  The control word is
// read here and advanced by bf_ctl_kernel afterwards (every workgroup reads
// it unchanged).
constexpr int kBFRunThreads = 1024;

struct BFRunLds {
  int Q, L;      // float4 groups per row, lanes per particle (power of two >= Q)
  size_t bytes;  // dynamic LDS
};

inline BFRunLds bf_run_lds(int Gs, int N, int Dp) {
  BFRunLds r{};
  r.Q = Dp / 4;
  r.L = 1;
  while (r.L < r.Q) r.L *= 2;
  const size_t nS = (size_t)Gs * N;
  r.bytes = 16 * (3 * nS * r.Q + (size_t)Gs * r.Q) + 4 * (nS * 7 + 10 * (size_t)Gs);
  return r;
}

template <int FUNC>
__global__ __launch_bounds__(kBFRunThreads) void bf_run_kernel(BFDev s, int n_fit, int flush, int L) {
  extern __shared__ float4 s_dyn4[];
  __shared__ int s_tg;
  const int sw = blockIdx.x, t = threadIdx.x, B = blockDim.x;
  const int Gs = s.Gs, N = s.N, D = s.D, Q = s.Dp / 4, nS = Gs * N, g0 = sw * Gs;
  const int64_t r0 = (int64_t)g0 * N * Q;  // first float4 of the swarm's rows
  float4* sX = s_dyn4;
  float4* sV = sX + nS * Q;
  float4* sP = sV + nS * Q;
  float4* sG = sP + nS * Q;  // Gbest rows
  float* sPf = reinterpret_cast<float*>(sG + Gs * Q);
  float* sF = sPf + nS;
  float* sC = sF + nS;                            // per particle a1, a2, a3, (unused)
  int* sImp = reinterpret_cast<int*>(sC + 4 * nS);
  float* sGf = reinterpret_cast<float*>(sImp + nS);
  int* sGn = reinterpret_cast<int*>(sGf + Gs);
  float* sH = reinterpret_cast<float*>(sGn + Gs);  // per group C1, C2, C3, w_init, w_end, V_limit
  float* sW = sH + 6 * Gs;                         // per group inertia of the current move
  float* sVm = sW + Gs;                            // per group velocity bound

  const float4* X4 = reinterpret_cast<const float4*>(s.X) + r0;
  const float4* V4 = reinterpret_cast<const float4*>(s.V) + r0;
  const float4* P4 = reinterpret_cast<const float4*>(s.P) + r0;
  const float4* G4 = reinterpret_cast<const float4*>(s.gbest_pos) + (int64_t)g0 * Q;
  for (int q = t; q < nS * Q; q += B) {
    sX[q] = X4[q];
    sV[q] = V4[q];
    sP[q] = P4[q];
  }
  for (int q = t; q < Gs * Q; q += B) sG[q] = G4[q];
  for (int i = t; i < nS; i += B) {
    sPf[i] = s.Pf[(int64_t)g0 * N + i];
    sF[i] = s.f[(int64_t)g0 * N + i];
  }
  for (int g = t; g < Gs; g += B) {
    sGf[g] = s.gbest_f[g0 + g];
    sGn[g] = s.gbest_n[g0 + g];
    const float* h = s.hyper + 6 * (g0 + g);
    for (int j = 0; j < 6; ++j) sH[6 * g + j] = h[j];
    sVm[g] = h[5] * (s.hi - s.lo) * 0.5f;
  }
  const BFCtl c0 = *s.ctl;
  int k = c0.k, pending = c0.pending;
  uint32_t ctr = c0.ctr;
  __syncthreads();

  const int lane = t & 63, wave = t >> 6, n_waves = B >> 6;
  const int per_wave = 64 / L, seg = lane / L, ls = lane - seg * L;
  for (int step = 0; step < n_fit + flush; ++step) {
    const bool fit = step < n_fit;
    if (pending) {
      // Tbest of the swarm (lowest group best, lowest group on ties) and each
      // particle's r1, r2, r3 scaled by its group's C1, C2, C3
      if (t == 0) {
        int tg = 0;
        for (int g = 1; g < Gs; ++g)
          if (sGf[g] < sGf[tg]) tg = g;
        s_tg = tg;
      }
      const int kk = k < s.T ? k : s.T;
      for (int g = t; g < Gs; g += B) {
        const float* h = sH + 6 * g;
        sW[g] = h[3] - (h[3] - h[4]) / (float)s.T * (float)kk;
      }
      for (int i = t; i < nS; i += B) {
        const float* h = sH + 6 * (i / N);
        const U4 r = philox((uint32_t)i, ctr, (uint32_t)sw, TAG_BF_UPDATE, s.seed_lo, s.seed_hi);
        sC[4 * i + 0] = h[0] * u01(r.v[0]);
        sC[4 * i + 1] = h[1] * u01(r.v[1]);
        sC[4 * i + 2] = h[2] * u01(r.v[2]);
      }
      __syncthreads();
      const int tg = s_tg;
      for (int q = t; q < nS * Q; q += B) {
        const int i = q / Q, qq = q - i * Q, g = i / N, e = 4 * qq;
        const float w = sW[g], vmax = sVm[g];
        const float a1 = sC[4 * i], a2 = sC[4 * i + 1], a3 = sC[4 * i + 2];
        float4 x4 = sX[q], v4 = sV[q];
        const float4 p4 = sP[q], gb4 = sG[g * Q + qq], tb4 = sG[tg * Q + qq];
        float* xs = &x4.x;
        float* vs = &v4.x;
        const float* ps = &p4.x;
        const float* gs = &gb4.x;
        const float* ts = &tb4.x;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (e + j < D) xs[j] = bf_move(xs[j], vs[j], ps[j], gs[j], ts[j], w, a1, a2, a3, vmax, s.lo, s.hi);
        sX[q] = x4;
        sV[q] = v4;
      }
      __syncthreads();
    }
    if (fit) {
      // evaluation: L lanes per particle, lane ls holding elements 4 ls ..
      // 4 ls + 3 as the stepwise kernel's lane ls does; the butterfly's
      // steps below L add the exact zeros (ones) of the empty lanes there
      for (int base = wave * per_wave; base < nS; base += n_waves * per_wave) {
        const int i = base + seg;
        const bool ok = i < nS && ls < Q;
        float xv[4] = {0.f, 0.f, 0.f, 0.f};
        if (ok) {
          const float4 x4 = sX[i * Q + ls];
          xv[0] = x4.x;
          xv[1] = x4.y;
          xv[2] = x4.z;
          xv[3] = x4.w;
        }
        float prev = 0.f;
        if (FUNC == BF_ROSENBROCK) {
          prev = __shfl_up(xv[3], 1);
          if (ls == 0) prev = 0.f;
        }
        float acc = 0.f, prod = 1.f;
        bf_terms<FUNC>(xv, prev, ok ? 4 * ls : D, D, acc, prod);
        for (int m = L / 2; m > 0; m >>= 1) acc += __shfl_xor(acc, m);
        if (FUNC == BF_GRIEWANK) {
          for (int m = L / 2; m > 0; m >>= 1) prod *= __shfl_xor(prod, m);
        }
        float fv = acc;
        if (FUNC == BF_GRIEWANK) fv = 1.f + fv - prod;
        if (!(fabsf(fv) <= 3.402823466e38f)) fv = INFINITY;
        if (i < nS && ls == 0) {
          const int imp = fv < sPf[i];
          sF[i] = fv;
          if (imp) sPf[i] = fv;
          sImp[i] = imp;
        }
      }
      __syncthreads();
      for (int q = t; q < nS * Q; q += B)
        if (sImp[q / Q]) sP[q] = sX[q];
      // Gbest of every group: lowest Pbest, lowest index on ties
      for (int g = t; g < Gs; g += B) {
        float bf = INFINITY;
        int bn = 0;
        for (int n = 0; n < N; ++n) {
          const float f = sPf[g * N + n];
          if (f < bf) {
            bf = f;
            bn = n;
          }
        }
        sGf[g] = bf;
        sGn[g] = bn;
      }
      __syncthreads();
      for (int q = t; q < Gs * Q; q += B) {
        const int g = q / Q;
        sG[q] = sP[(g * N + sGn[g]) * Q + (q - g * Q)];
      }
      __syncthreads();
      k += 1;
    }
    ctr += pending ? 1u : 0u;
    pending = fit ? 1 : 0;
  }

  float4* Xo = reinterpret_cast<float4*>(s.X) + r0;
  float4* Vo = reinterpret_cast<float4*>(s.V) + r0;
  float4* Po = reinterpret_cast<float4*>(s.P) + r0;
  float4* Go = reinterpret_cast<float4*>(s.gbest_pos) + (int64_t)g0 * Q;
  for (int q = t; q < nS * Q; q += B) {
    Xo[q] = sX[q];
    Vo[q] = sV[q];
    Po[q] = sP[q];
  }
  for (int q = t; q < Gs * Q; q += B) Go[q] = sG[q];
  for (int i = t; i < nS; i += B) {
    s.Pf[(int64_t)g0 * N + i] = sPf[i];
    s.f[(int64_t)g0 * N + i] = sF[i];
  }
  for (int g = t; g < Gs; g += B) {
    s.gbest_f[g0 + g] = sGf[g];
    s.gbest_n[g0 + g] = sGn[g];
  }
}

// The control word after n_fit evaluated iterations and an optional flush
// (the stepwise reduce's bookkeeping, step by step).
__global__ void bf_ctl_kernel(BFDev s, int n_fit, int flush) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  BFCtl c = *s.ctl;
  // every step advances the counter by the move it owes: the first by the
  // pending flag it starts with, every later one by 1 (a fit step leaves a
  // move owed)
  const int steps = n_fit + flush;
  if (steps > 0) c.ctr += (c.pending ? 1u : 0u) + (uint32_t)(steps - 1);
  c.k += n_fit;
  if (steps > 0) c.pending = flush ? 0 : 1;
  *s.ctl = c;
}

bool bf_run_fits(const BFDev& s) {
  return s.Dp <= 256 && bf_run_lds(s.Gs, s.N, s.Dp).bytes <= 64 * 1024;
}

template <int FUNC>
void launch_bf_run_f(const BFDev& s, int n_fit, int flush, hipStream_t st) {
  const BFRunLds r = bf_run_lds(s.Gs, s.N, s.Dp);
  hipLaunchKernelGGL((bf_run_kernel<FUNC>), dim3(s.S), dim3(kBFRunThreads), r.bytes, st, s, n_fit, flush,
                     r.L);
}

// n_fit evaluated iterations (then a flush move when flush) of every swarm,
// in one launch plus the control-word update.
void launch_bf_run(const BFDev& s, int n_fit, int flush, hipStream_t st) {
  switch (s.func) {
    case BF_SPHERE: launch_bf_run_f<BF_SPHERE>(s, n_fit, flush, st); break;
    case BF_ROSENBROCK: launch_bf_run_f<BF_ROSENBROCK>(s, n_fit, flush, st); break;
    case BF_RASTRIGIN: launch_bf_run_f<BF_RASTRIGIN>(s, n_fit, flush, st); break;
    default: launch_bf_run_f<BF_GRIEWANK>(s, n_fit, flush, st); break;
  }
  hipLaunchKernelGGL(bf_ctl_kernel, dim3(1), dim3(64), 0, st, s, n_fit, flush);
}

void launch_bf_init(const BFDev& s, hipStream_t st) {
  const int64_t total = (int64_t)s.G * s.N * s.Dp;
  hipLaunchKernelGGL(bf_init_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, s);
}

template <int FUNC>
void launch_bf_iter(const BFDev& s, bool fit, hipStream_t st) {
  const int blocks = (s.G * s.N + 3) / 4;
  if (fit)
    hipLaunchKernelGGL((bf_iter_kernel<FUNC, true>), dim3(blocks), dim3(256), 0, st, s);
  else
    hipLaunchKernelGGL((bf_iter_kernel<FUNC, false>), dim3(blocks), dim3(256), 0, st, s);
}

void launch_bf_step(const BFDev& s, bool fit, hipStream_t st) {
  switch (s.func) {
    case BF_SPHERE: launch_bf_iter<BF_SPHERE>(s, fit, st); break;
    case BF_ROSENBROCK: launch_bf_iter<BF_ROSENBROCK>(s, fit, st); break;
    case BF_RASTRIGIN: launch_bf_iter<BF_RASTRIGIN>(s, fit, st); break;
    default: launch_bf_iter<BF_GRIEWANK>(s, fit, st); break;
  }
  hipLaunchKernelGGL(bf_reduce_kernel, dim3(s.G), dim3(256), 0, st, s, fit ? 1 : 0);
}

}  // namespace sepso

using namespace sepso;

struct sepso_bf {
  BFDev dev{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool broken = false;
  bool whole_run = false;  // small swarms: all iterations of a call in one launch
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

// Evolution phase over benchmark-function lower levels: swarm i of the
// lower-level handle is H particle i.
struct sepso_bf_evolve {
  sepso_bf* bf = nullptr;
  EvolveDev dev{};
  size_t bf_bytes = 0;
  float* lower_best = nullptr;     // n: each lower-level swarm's best after its run
  hipGraphExec_t graph = nullptr;  // one evolution: lower-level runs, their bests, the H step
};

namespace {

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

struct BFLayout {
  size_t ctl, xvp, fp, gb, gpos, hyper, total;
};

int bf_swarms(const sepso_bf_cfg* c) { return c->swarms < 1 ? 1 : c->swarms; }

// Shape checks; the hyper values are checked only when check_hyper is set
// (the evolution phase writes them itself).
sepso_status bf_check(const sepso_bf_cfg* c, bool check_hyper = true) {
  if (!c) return fail(SEPSO_E_ARG, "cfg is NULL");
  if (c->func < 1 || c->func > 4) return fail(SEPSO_E_ARG, "bf: func in 1..4");
  if (c->groups < 1 || c->groups > 64) return fail(SEPSO_E_ARG, "bf: groups in [1,64]");
  if (c->particles < 1 || c->dims < 1 || c->max_iters < 1)
    return fail(SEPSO_E_ARG, "bf: particles, dims, max_iters >= 1");
  if (c->path < 0 || c->path > 1) return fail(SEPSO_E_ARG, "bf: path in {0, 1}");
  const double S = bf_swarms(c);
  const double elems = S * c->groups * c->particles * ((c->dims + 3) / 4 * 4);
  if (elems > 4.0e9 || S * c->groups * c->particles > 2.0e9 || S * c->groups > 2.0e9 / 6)
    return fail(SEPSO_E_ARG, "bf: swarm too large");
  if ((double)c->groups * c->particles * ((c->dims + 3) / 4) > 4294967295.0)
    return fail(SEPSO_E_ARG, "bf: swarm too large for the 32-bit random counter");
  if (!(std::isfinite(c->lo) && std::isfinite(c->hi) && c->lo < c->hi))
    return fail(SEPSO_E_ARG, "bf: lo < hi finite");
  if (!check_hyper) return SEPSO_OK;
  if (!c->hyper) return fail(SEPSO_E_ARG, "bf: hyper is NULL");
  for (int64_t j = 0; j < 6 * (int64_t)S * c->groups; ++j)
    if (!std::isfinite(c->hyper[j]) || (j % 6 == 5 && c->hyper[j] < 0.f))
      return fail(SEPSO_E_ARG, "bf: hyper not finite or V_limit < 0");
  return SEPSO_OK;
}

BFLayout bf_layout(const sepso_bf_cfg* c) {
  const size_t G = (size_t)bf_swarms(c) * c->groups;
  const size_t n = G * c->particles, Dp = (size_t)(c->dims + 3) / 4 * 4;
  BFLayout L{};
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t at = o;
    o = a256(o + std::max<size_t>(b, 4));
    return at;
  };
  L.ctl = take(sizeof(BFCtl));
  L.xvp = take(4 * 3 * n * Dp);
  L.fp = take(4 * 2 * n);
  L.gb = take(8 * G);
  L.gpos = take(4 * G * Dp);
  L.hyper = take(4 * 6 * G);
  L.total = o;
  return L;
}

sepso_status bf_hip(sepso_bf* b, hipError_t e, const char* what) {
  b->broken = true;
  return fail(SEPSO_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define BFCHK(b, expr)                                  \
  do {                                                  \
    hipError_t _e = (expr);                             \
    if (_e != hipSuccess) return bf_hip(b, _e, #expr);  \
  } while (0)

sepso_status bf_usable(sepso_bf* b) {
  if (!b) return fail(SEPSO_E_ARG, "bf handle is NULL");
  if (b->broken) return fail(SEPSO_E_STATE, "handle is unusable after an earlier HIP error");
  return SEPSO_OK;
}

sepso_status bf_run(sepso_bf* b, int32_t n) {
  if (b->whole_run && n > 0) {
    launch_bf_run(b->dev, n, 1, b->stream);
  } else {
    for (int k = 0; k < n; ++k) launch_bf_step(b->dev, true, b->stream);
    if (n > 0) launch_bf_step(b->dev, false, b->stream);
  }
  BFCHK(b, hipGetLastError());
  return SEPSO_OK;
}

// Creates a handle on a checked cfg.  hyper_dev (device, S*G x 6) replaces
// the upload of cfg->hyper when given; run (device) is the counter word 1 of
// the initial draws (NULL: 0).  The swarm is initialised only when
// hyper_dev is NULL (otherwise its writer initialises it later).
sepso_status bf_create(const sepso_bf_cfg* cfg, void* d_ws, size_t ws_bytes, void* stream,
                       float** hyper_dev, const int32_t* run, sepso_bf** out) {
  const BFLayout L = bf_layout(cfg);
  if (!d_ws) return fail(SEPSO_E_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(d_ws) % 256) return fail(SEPSO_E_ARG, "workspace not 256-byte aligned");
  if (ws_bytes < L.total) return fail(SEPSO_E_NOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
  sepso_bf* b = new (std::nothrow) sepso_bf();
  if (!b) return fail(SEPSO_E_NOMEM, "host allocation failed");
  char* w = static_cast<char*>(d_ws);
  BFDev& d = b->dev;
  d.func = cfg->func;
  d.S = bf_swarms(cfg);
  d.Gs = cfg->groups;
  d.G = d.S * d.Gs;
  d.N = cfg->particles;
  d.D = cfg->dims;
  d.Dp = (cfg->dims + 3) / 4 * 4;
  d.T = cfg->max_iters;
  d.run = run;
  d.lo = cfg->lo;
  d.hi = cfg->hi;
  d.seed_lo = (uint32_t)(cfg->seed & 0xffffffffu);
  d.seed_hi = (uint32_t)(cfg->seed >> 32);
  const size_t n = (size_t)d.G * d.N;
  d.ctl = reinterpret_cast<BFCtl*>(w + L.ctl);
  d.X = reinterpret_cast<float*>(w + L.xvp);
  d.V = d.X + n * d.Dp;
  d.P = d.V + n * d.Dp;
  d.f = reinterpret_cast<float*>(w + L.fp);
  d.Pf = d.f + n;
  d.gbest_n = reinterpret_cast<int32_t*>(w + L.gb);
  d.gbest_f = reinterpret_cast<float*>(w + L.gb + 4 * (size_t)d.G);
  d.gbest_pos = reinterpret_cast<float*>(w + L.gpos);
  d.hyper = reinterpret_cast<const float*>(w + L.hyper);
  if (hyper_dev) *hyper_dev = reinterpret_cast<float*>(w + L.hyper);
  b->whole_run = cfg->path == 0 && bf_run_fits(d);
  if (stream) {
    b->stream = static_cast<hipStream_t>(stream);
  } else {
    hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete b;
      return fail(SEPSO_E_HIP, "hipStreamCreate: %s", hipGetErrorString(e));
    }
    b->own_stream = true;
  }
  hipError_t e = hipEventCreate(&b->ev0);
  if (e == hipSuccess) e = hipEventCreate(&b->ev1);
  if (e == hipSuccess && !hyper_dev) {
    e = hipMemcpyAsync(w + L.hyper, cfg->hyper, 24 * (size_t)d.G, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) {
      launch_bf_init(d, b->stream);
      e = hipGetLastError();
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) {
    sepso_status st = fail(SEPSO_E_HIP, "bf create: %s", hipGetErrorString(e));
    sepso_bf_destroy(b);
    return st;
  }
  *out = b;
  return SEPSO_OK;
}

}  // namespace

extern "C" {

sepso_status sepso_bf_workspace_bytes(const sepso_bf_cfg* cfg, size_t* bytes) {
  if (!bytes) return fail(SEPSO_E_ARG, "bytes is NULL");
  sepso_status st = bf_check(cfg);
  if (st != SEPSO_OK) return st;
  *bytes = bf_layout(cfg).total;
  return SEPSO_OK;
}

sepso_status sepso_bf_create(const sepso_bf_cfg* cfg, void* d_ws, size_t ws_bytes, void* stream,
                             sepso_bf** out) {
  if (!out) return fail(SEPSO_E_ARG, "out is NULL");
  *out = nullptr;
  sepso_status st = bf_check(cfg);
  if (st != SEPSO_OK) return st;
  return bf_create(cfg, d_ws, ws_bytes, stream, nullptr, nullptr, out);
}

sepso_status sepso_bf_destroy(sepso_bf* b) {
  if (!b) return fail(SEPSO_E_ARG, "bf handle is NULL");
  // teardown is best effort: a failure here leaves nothing to recover
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return SEPSO_OK;
}

sepso_status sepso_bf_step(sepso_bf* b, int32_t n) {
  sepso_status st = bf_usable(b);
  if (st != SEPSO_OK) return st;
  if (n < 0) return fail(SEPSO_E_ARG, "n must be >= 0");
  return bf_run(b, n);
}

sepso_status sepso_bf_profile(sepso_bf* b, int32_t n, float* ms_per_iter) {
  sepso_status st = bf_usable(b);
  if (st != SEPSO_OK) return st;
  if (n < 1 || !ms_per_iter) return fail(SEPSO_E_ARG, "n >= 1 and ms_per_iter required");
  BFCHK(b, hipEventRecord(b->ev0, b->stream));
  st = bf_run(b, n);
  if (st != SEPSO_OK) return st;
  BFCHK(b, hipEventRecord(b->ev1, b->stream));
  BFCHK(b, hipEventSynchronize(b->ev1));
  float ms = 0.f;
  BFCHK(b, hipEventElapsedTime(&ms, b->ev0, b->ev1));
  *ms_per_iter = ms / (float)n;
  return SEPSO_OK;
}

sepso_status sepso_bf_get_state(sepso_bf* b, sepso_bf_state* s) {
  sepso_status st = bf_usable(b);
  if (st != SEPSO_OK) return st;
  if (!s) return fail(SEPSO_E_ARG, "state is NULL");
  const BFDev& d = b->dev;
  const size_t n = (size_t)d.G * d.N;
  float* rows[3] = {s->X, s->V, s->P};
  const float* src[3] = {d.X, d.V, d.P};
  for (int a = 0; a < 3; ++a)
    if (rows[a])
      BFCHK(b, hipMemcpy2DAsync(rows[a], 4 * (size_t)d.D, src[a], 4 * (size_t)d.Dp, 4 * (size_t)d.D, n,
                                hipMemcpyDeviceToHost, b->stream));
  if (s->f) BFCHK(b, hipMemcpyAsync(s->f, d.f, 4 * n, hipMemcpyDeviceToHost, b->stream));
  if (s->Pf) BFCHK(b, hipMemcpyAsync(s->Pf, d.Pf, 4 * n, hipMemcpyDeviceToHost, b->stream));
  std::vector<int32_t> gn(d.G);
  std::vector<float> gf(d.G);
  BFCtl c{};
  BFCHK(b, hipMemcpyAsync(gn.data(), d.gbest_n, 4 * (size_t)d.G, hipMemcpyDeviceToHost, b->stream));
  BFCHK(b, hipMemcpyAsync(gf.data(), d.gbest_f, 4 * (size_t)d.G, hipMemcpyDeviceToHost, b->stream));
  BFCHK(b, hipMemcpyAsync(&c, d.ctl, sizeof(BFCtl), hipMemcpyDeviceToHost, b->stream));
  BFCHK(b, hipStreamSynchronize(b->stream));
  if (s->gbest_n) std::memcpy(s->gbest_n, gn.data(), 4 * (size_t)d.G);
  if (s->gbest_f) std::memcpy(s->gbest_f, gf.data(), 4 * (size_t)d.G);
  int tg = 0;
  for (int g = 1; g < d.G; ++g)
    if (gf[g] < gf[tg]) tg = g;
  s->tb_g = tg;
  s->tb_n = gn[tg];
  s->tb_f = gf[tg];
  s->k = c.k;
  s->ctr = c.ctr;
  s->pending = c.pending;
  return SEPSO_OK;
}

sepso_status sepso_bf_set_state(sepso_bf* b, const sepso_bf_state* s) {
  sepso_status st = bf_usable(b);
  if (st != SEPSO_OK) return st;
  if (!s) return fail(SEPSO_E_ARG, "state is NULL");
  const BFDev& d = b->dev;
  const size_t n = (size_t)d.G * d.N;
  if (s->gbest_n)
    for (int g = 0; g < d.G; ++g)
      if (s->gbest_n[g] < 0 || s->gbest_n[g] >= d.N) return fail(SEPSO_E_ARG, "gbest_n[%d] out of range", g);
  if (s->k < 0) return fail(SEPSO_E_ARG, "k must be >= 0");
  const float* rows[3] = {s->X, s->V, s->P};
  float* dst[3] = {d.X, d.V, d.P};
  for (int a = 0; a < 3; ++a)
    if (rows[a])
      BFCHK(b, hipMemcpy2DAsync(dst[a], 4 * (size_t)d.Dp, rows[a], 4 * (size_t)d.D, 4 * (size_t)d.D, n,
                                hipMemcpyHostToDevice, b->stream));
  if (s->f) BFCHK(b, hipMemcpyAsync(d.f, s->f, 4 * n, hipMemcpyHostToDevice, b->stream));
  if (s->Pf) BFCHK(b, hipMemcpyAsync(d.Pf, s->Pf, 4 * n, hipMemcpyHostToDevice, b->stream));
  if (s->gbest_n) BFCHK(b, hipMemcpyAsync(d.gbest_n, s->gbest_n, 4 * (size_t)d.G, hipMemcpyHostToDevice, b->stream));
  if (s->gbest_f) BFCHK(b, hipMemcpyAsync(d.gbest_f, s->gbest_f, 4 * (size_t)d.G, hipMemcpyHostToDevice, b->stream));
  // the Gbest rows follow from P and gbest_n
  if (s->P && s->gbest_n)
    for (int g = 0; g < d.G; ++g)
      BFCHK(b, hipMemcpyAsync(d.gbest_pos + (size_t)g * d.Dp, s->P + ((size_t)g * d.N + s->gbest_n[g]) * d.D,
                              4 * (size_t)d.D, hipMemcpyHostToDevice, b->stream));
  const BFCtl c{s->k, s->ctr, s->pending, 0};
  BFCHK(b, hipMemcpyAsync(d.ctl, &c, sizeof(BFCtl), hipMemcpyHostToDevice, b->stream));
  BFCHK(b, hipStreamSynchronize(b->stream));
  return SEPSO_OK;
}

// ---- evolution phase on the benchmark functions ---------------------------

static sepso_status bfe_sizes(const sepso_bf_cfg* lower, const sepso_evolve_cfg* cfg, sepso_bf_cfg* lc,
                              size_t* bf_bytes, size_t* h_bytes) {
  if (!lower || !cfg) return fail(SEPSO_E_ARG, "lower/cfg is NULL");
  sepso_status st = evolve_cfg_check(cfg);
  if (st != SEPSO_OK) return st;
  *lc = *lower;
  lc->swarms = cfg->h_groups * cfg->h_particles;
  lc->hyper = nullptr;
  st = bf_check(lc, false);
  if (st != SEPSO_OK) return st;
  *bf_bytes = a256(bf_layout(lc).total);
  *h_bytes = evolve_h_bytes(cfg, 6 * lower->groups) + a256(4 * (size_t)lc->swarms);
  return SEPSO_OK;
}

sepso_status sepso_bf_evolve_workspace_bytes(const sepso_bf_cfg* lower, const sepso_evolve_cfg* cfg,
                                             size_t* bytes) {
  if (!bytes) return fail(SEPSO_E_ARG, "bytes is NULL");
  sepso_bf_cfg lc;
  size_t a = 0, h = 0;
  sepso_status st = bfe_sizes(lower, cfg, &lc, &a, &h);
  if (st != SEPSO_OK) return st;
  *bytes = a + h;
  return SEPSO_OK;
}

sepso_status sepso_bf_evolve_create(const sepso_bf_cfg* lower, const sepso_evolve_cfg* cfg, void* d_ws,
                                    size_t ws_bytes, void* stream, sepso_bf_evolve** out) {
  if (!out) return fail(SEPSO_E_ARG, "out is NULL");
  *out = nullptr;
  sepso_bf_cfg lc;
  size_t a = 0, h = 0;
  sepso_status st = bfe_sizes(lower, cfg, &lc, &a, &h);
  if (st != SEPSO_OK) return st;
  if (!d_ws) return fail(SEPSO_E_ARG, "workspace is NULL");
  if (ws_bytes < a + h) return fail(SEPSO_E_NOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, a + h);
  sepso_bf_evolve* ev = new (std::nothrow) sepso_bf_evolve();
  if (!ev) return fail(SEPSO_E_NOMEM, "host allocation failed");
  EvolveDev& d = ev->dev;
  std::vector<float> hc;
  char* hbase = static_cast<char*>(d_ws) + a;
  evolve_h_carve(cfg, 6 * lower->groups, hbase, &d, &hc);
  ev->lower_best = reinterpret_cast<float*>(hbase + evolve_h_bytes(cfg, 6 * lower->groups));
  ev->bf_bytes = a;
  // the lower level's initial draws take the evolution counter (EvolveCtl's
  // first word) as word 1
  static_assert(offsetof(EvolveCtl, k) == 0, "EvolveCtl::k leads");
  st = bf_create(&lc, d_ws, a, stream, &d.hyper_out, reinterpret_cast<const int32_t*>(d.ctl), &ev->bf);
  if (st != SEPSO_OK) {
    delete ev;
    return st;
  }
  d.lfv_in = ev->lower_best;
  sepso_bf* b = ev->bf;
  hipError_t e = hipMemcpyAsync(const_cast<float*>(d.h_hyper), hc.data(), 4 * hc.size(),
                                hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) {
    launch_evolve_init(d, Pools{}, b->stream);
    launch_bf_init(b->dev, b->stream);  // the lower level's state is valid from here on
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) {
    st = fail(SEPSO_E_HIP, "bf evolve create: %s", hipGetErrorString(e));
    sepso_bf_destroy(b);
    delete ev;
    return st;
  }
  *out = ev;
  return SEPSO_OK;
}

sepso_status sepso_bf_evolve_destroy(sepso_bf_evolve* ev) {
  if (!ev) return fail(SEPSO_E_ARG, "evolve handle is NULL");
  if (ev->graph) (void)hipGraphExecDestroy(ev->graph);  // teardown: best effort
  sepso_bf_destroy(ev->bf);
  delete ev;
  return SEPSO_OK;
}

sepso_status sepso_bf_evolve_run(sepso_bf_evolve* ev, int32_t n, float* curve) {
  if (!ev) return fail(SEPSO_E_ARG, "evolve handle is NULL");
  sepso_bf* b = ev->bf;
  sepso_status st = bf_usable(b);
  if (st != SEPSO_OK) return st;
  if (n < 0) return fail(SEPSO_E_ARG, "n must be >= 0");
  if (curve && n > ev->dev.E) return fail(SEPSO_E_ARG, "curve holds at most `evolutions` values");
  const BFDev& d = b->dev;
  if (!ev->graph) {
    // fresh swarms (run = evolutions done), T evaluated iterations, every
    // swarm's best, the H step that writes the next hyper-parameters
    hipGraph_t g = nullptr;
    BFCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    launch_bf_init(d, b->stream);
    if (b->whole_run) {
      launch_bf_run(d, d.T, 0, b->stream);
    } else {
      for (int k = 0; k < d.T; ++k) launch_bf_step(d, true, b->stream);
    }
    hipLaunchKernelGGL(bf_best_kernel, dim3((d.S + 255) / 256), dim3(256), 0, b->stream, d, ev->lower_best);
    launch_evolve_step(ev->dev, Pools{}, 1, b->stream);
    hipError_t eq = hipGetLastError();
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (eq != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return bf_hip(b, eq, "bf evolution capture");
    }
    if (e != hipSuccess) return bf_hip(b, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&ev->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return bf_hip(b, e, "hipGraphInstantiate");
  }
  EvolveCtl c0{};
  if (curve) {
    BFCHK(b, hipMemcpyAsync(&c0, ev->dev.ctl, sizeof(EvolveCtl), hipMemcpyDeviceToHost, b->stream));
    BFCHK(b, hipStreamSynchronize(b->stream));
  }
  for (int k = 0; k < n; ++k) BFCHK(b, hipGraphLaunch(ev->graph, b->stream));
  if (curve && n > 0) BFCHK(b, evolve_h_curve(ev->dev, b->stream, c0.k, n, curve));
  BFCHK(b, hipStreamSynchronize(b->stream));
  return SEPSO_OK;
}

sepso_status sepso_bf_evolve_get_state(sepso_bf_evolve* ev, sepso_evolve_state* s) {
  if (!ev) return fail(SEPSO_E_ARG, "evolve handle is NULL");
  sepso_status st = bf_usable(ev->bf);
  if (st != SEPSO_OK) return st;
  if (!s) return fail(SEPSO_E_ARG, "state is NULL");
  BFCHK(ev->bf, evolve_h_state(ev->dev, ev->bf->stream, s));
  return SEPSO_OK;
}

sepso_status sepso_bf_evolve_best(sepso_bf_evolve* ev, float* hyper, float* lfv) {
  if (!ev) return fail(SEPSO_E_ARG, "evolve handle is NULL");
  sepso_status st = bf_usable(ev->bf);
  if (st != SEPSO_OK) return st;
  int k = 0;
  BFCHK(ev->bf, evolve_h_best(ev->dev, ev->bf->stream, hyper, lfv, &k));
  if (k == 0) return fail(SEPSO_E_STATE, "no evolution has run yet");
  return SEPSO_OK;
}

sepso_status sepso_bf_evolve_lower(sepso_bf_evolve* ev, sepso_bf** bf) {
  if (!ev || !bf) return fail(SEPSO_E_ARG, "evolve/out is NULL");
  *bf = ev->bf;
  return SEPSO_OK;
}

}  // extern "C"
