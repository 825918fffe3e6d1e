// Learned initializer (device code): occupancy raster of each instance's
// map, a BF16 MLP (FP32 accumulation on gfx950 MFMA) that proposes one
// initial path per group, its MSE backward pass and Adam with FP32 master
// weights.  GEMMs run on v_mfma_f32_16x16x32_bf16.
#include "common.h"
#include "mlp.h"

namespace sepso {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  const uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(r >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------------------------
// Input features of instance i (row i of X): 64 x 64 occupancy (cell centre
// inside any obstacle polygon, even-odd rule) followed by start and target
// normalised by the map size; zero padding up to kLinInPad.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void raster_kernel(Pools pl, uint16_t* X, int ldx,
                                                     int32_t* eligible) {
  const int inst = blockIdx.x;
  const InstDesc& d = pl.desc[inst];
  const float2* verts = pl.verts + d.eo;
  const int32_t* pp = pl.poly_ptr + d.plo;
  uint16_t* row = X + (int64_t)inst * ldx;
  for (int cell = threadIdx.x; cell < kRaster * kRaster; cell += blockDim.x) {
    const int r = cell / kRaster, c = cell - r * kRaster;
    const float px = (c + 0.5f) * d.width / kRaster, py = (r + 0.5f) * d.height / kRaster;
    int inside = 0;
    for (int q = 0; q < d.n_polys && !inside; ++q) {
      const int v0 = pp[q], m = pp[q + 1] - v0;
      int odd = 0;
      for (int j = 0; j < m; ++j) {
        const float2 a = verts[v0 + j], b = verts[v0 + (j + 1 == m ? 0 : j + 1)];
        if ((a.y > py) != (b.y > py)) {
          const float xc = a.x + (py - a.y) * (b.x - a.x) / (b.y - a.y);
          if (px < xc) odd ^= 1;
        }
      }
      inside = odd;
    }
    row[cell] = inside ? 0x3F80 : 0;  // 1.0 or 0.0
  }
  if (threadIdx.x < kLinInPad - kRaster * kRaster) {
    const int j = threadIdx.x;
    const float4 e = pl.ends[inst];
    float v = 0.f;
    if (j == 0) v = e.x / d.width;
    if (j == 1) v = e.y / d.height;
    if (j == 2) v = e.z / d.width;
    if (j == 3) v = e.w / d.height;
    row[kRaster * kRaster + j] = to_bf16(v);
  }
  if (threadIdx.x == 0) eligible[inst] = (d.G == kLinGroups && d.W == kLinW) ? 1 : 0;
}

// The GEMM epilogue applied to one FP32 result C(row, col) = v.
__device__ __forceinline__ void apply_epi(const Epi& ep, int row, int col, float v) {
  const int64_t o = (int64_t)row * ep.ldo + col;
  switch (ep.mode) {
    case EPI_BIAS_RELU_BF16:
      v += ep.bias[col];
      ep.out_bf16[o] = to_bf16(v > 0.f ? v : 0.f);
      break;
    case EPI_BIAS_F32:
      ep.out_f32[o] = v + ep.bias[col];
      break;
    case EPI_F32:
      ep.out_f32[o] = v;
      break;
    case EPI_MASK: {
      const float dz = from_bf16(ep.mask[o]) > 0.f ? v : 0.f;
      ep.out_f32[o] = dz;
      ep.out_bf16[o] = to_bf16(dz);
      break;
    }
  }
}

// ---------------------------------------------------------------------------
// C[M x N] = op(A)[M x K] * op(B)[K x N], BF16 in, FP32 accumulate.
//   A_KM = false: A(m, k) = A[m*lda + k]   A_KM = true: A(m, k) = A[k*lda + m]
//   B_KN = false: B(k, n) = B[n*ldb + k]   B_KN = true: B(k, n) = B[k*ldb + n]
// Block tile 64 x 64, four waves of 32 x 32 (2 x 2 MFMA 16x16x32 tiles).
// Requires K % 32 == 0; M % 8 == 0 when A_KM; N % 8 == 0 when B_KN.
// Split K: block z takes k-steps [z*kper, (z+1)*kper) of 32 and, when
// `part` is given, stores its raw sums as slice z of part (M x N each) for
// splitk_epi_kernel; otherwise it applies the epilogue itself.
// ---------------------------------------------------------------------------
template <bool A_KM, bool B_KN>
__global__ __launch_bounds__(256) void gemm_kernel(const uint16_t* __restrict__ A, int lda,
                                                   const uint16_t* __restrict__ B, int ldb, int M,
                                                   int N, int K, int kper, float* part, Epi ep) {
  constexpr int LDS = 40;  // padded row (k) length
  __shared__ __attribute__((aligned(16))) uint16_t As[64 * LDS];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[64 * LDS];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  f32x4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int kbeg = blockIdx.z * kper * 32, kend = min(K, kbeg + kper * 32);
  for (int k0 = kbeg; k0 < kend; k0 += 32) {
    if (!A_KM) {
      const int row = t >> 2, kc = (t & 3) * 8;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (m0 + row < M) v = *reinterpret_cast<const uint4*>(A + (int64_t)(m0 + row) * lda + k0 + kc);
      *reinterpret_cast<uint4*>(&As[row * LDS + kc]) = v;
    } else {
      const int kr = t >> 3, mc = (t & 7) * 8;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (m0 + mc < M) v = *reinterpret_cast<const uint4*>(A + (int64_t)(k0 + kr) * lda + m0 + mc);
      const uint16_t* h = reinterpret_cast<const uint16_t*>(&v);
      for (int i = 0; i < 8; ++i) As[(mc + i) * LDS + kr] = h[i];
    }
    if (!B_KN) {
      const int row = t >> 2, kc = (t & 3) * 8;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (n0 + row < N) v = *reinterpret_cast<const uint4*>(B + (int64_t)(n0 + row) * ldb + k0 + kc);
      *reinterpret_cast<uint4*>(&Bs[row * LDS + kc]) = v;
    } else {
      const int kr = t >> 3, nc = (t & 7) * 8;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (n0 + nc < N) v = *reinterpret_cast<const uint4*>(B + (int64_t)(k0 + kr) * ldb + n0 + nc);
      const uint16_t* h = reinterpret_cast<const uint16_t*>(&v);
      for (int i = 0; i < 8; ++i) Bs[(nc + i) * LDS + kr] = h[i];
    }
    __syncthreads();
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
    bf16x8 a[2], b[2];
    for (int i = 0; i < 2; ++i) {
      a[i] = *reinterpret_cast<const bf16x8*>(&As[(wm + i * 16 + r16) * LDS + kq]);
      b[i] = *reinterpret_cast<const bf16x8*>(&Bs[(wn + i * 16 + r16) * LDS + kq]);
    }
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  // D layout: lane holds column (lane % 16), rows 4*(lane/16) .. +3
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + i * 16 + (lane >> 4) * 4 + r;
        const int col = n0 + wn + j * 16 + (lane & 15);
        if (row >= M || col >= N) continue;
        if (part)
          part[((int64_t)blockIdx.z * M + row) * N + col] = acc[i][j][r];
        else
          apply_epi(ep, row, col, acc[i][j][r]);
      }
}

// One 32-wide k half-step of a 128-row operand tile (rows of the output
// dimension x 32 k) into two registers per thread.  K-contiguous source
// (KM = false): row t/2, k 16*(t&1) .. +15.  K-major source: k rows 2*(t/16)
// and +1 at columns 8*(t%16) .. +7.  Rows (columns) past R, and a half-step
// past the slice's end (valid = false), give zeros.
template <bool KM>
__device__ __forceinline__ void fetch128(const uint16_t* __restrict__ P, int ld, int r0, int R,
                                         int k0, int t, bool valid, uint4& r0v, uint4& r1v) {
  // an invalid row (column) or half-step reads the tile's first row at the
  // slice's first k, which exists, and is zeroed: every load is unconditional
  const uint4 zero = make_uint4(0, 0, 0, 0);
  if (!KM) {
    const int row = t >> 1, kc = (t & 1) * 16;
    const bool ok = valid && r0 + row < R;
    const uint16_t* src = P + (int64_t)(ok ? r0 + row : r0) * ld + (valid ? k0 : 0) + kc;
    r0v = *reinterpret_cast<const uint4*>(src);
    r1v = *reinterpret_cast<const uint4*>(src + 8);
    if (!ok) r0v = r1v = zero;
  } else {
    const int kr = 2 * (t >> 4), mc = (t & 15) * 8;
    const bool ok = valid && r0 + mc < R;
    const uint16_t* src = P + (int64_t)((valid ? k0 : 0) + kr) * ld + (ok ? r0 + mc : r0);
    r0v = *reinterpret_cast<const uint4*>(src);
    r1v = *reinterpret_cast<const uint4*>(src + ld);
    if (!ok) r0v = r1v = zero;
  }
}

// LDS position (in halves) of k offset k of tile row `row`: the row's eight
// 16-byte chunks of k are permuted by the row's bits 4..6, so that the
// transposing stores below (lanes 0..15 of a wave write rows 8 apart at one
// k) land in sixteen different banks, while the MFMA operand reads (sixteen
// consecutive rows from a multiple of 16, one chunk) keep one permutation
// per instruction and stay conflict-free on the padded rows.
template <int LDS>
__device__ __forceinline__ int swz128(int row, int k) {
  return row * LDS + ((((k >> 3) ^ (row >> 4)) & 7) << 3) + (k & 7);
}

// The registers of fetch128 into an LDS tile of rows of LDS halves (k
// contiguous, chunks permuted by swz128) at k offset kh; a K-major operand is
// transposed two k values at a time (one 32-bit store per row).
template <bool KM, int LDS>
__device__ __forceinline__ void stash128(uint16_t* S, int kh, int t, const uint4& r0v,
                                         const uint4& r1v) {
  if (!KM) {
    const int row = t >> 1, kc = kh + (t & 1) * 16;
    *reinterpret_cast<uint4*>(&S[swz128<LDS>(row, kc)]) = r0v;
    *reinterpret_cast<uint4*>(&S[swz128<LDS>(row, kc + 8)]) = r1v;
  } else {
    const int kr = kh + 2 * (t >> 4), mc = (t & 15) * 8;
    const uint32_t u0[4] = {r0v.x, r0v.y, r0v.z, r0v.w}, u1[4] = {r1v.x, r1v.y, r1v.z, r1v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {  // columns 2i, 2i+1: (k, k+1) as one 32-bit word each
      *reinterpret_cast<uint32_t*>(&S[swz128<LDS>(mc + 2 * i, kr)]) =
          __builtin_amdgcn_perm(u1[i], u0[i], 0x05040100u);
      *reinterpret_cast<uint32_t*>(&S[swz128<LDS>(mc + 2 * i + 1, kr)]) =
          __builtin_amdgcn_perm(u1[i], u0[i], 0x07060302u);
    }
  }
}

// The same product on a 128 x 128 block tile for large problems: four waves
// of 64 x 64 (4 x 4 MFMA 16x16x32 tiles, 64 accumulator registers) or eight
// of 64 x 32 (4 x 2 tiles; waves 0-3 load the A tile, waves 4-7 the B tile),
// k-steps of 64 (two MFMA k-steps; a slice's last may be 32 wide) through one
// LDS buffer -- the next step's global loads are in flight in registers while
// the current step's MFMAs run, two barriers per step.  One buffer (37 KB)
// lets four blocks share a CU where two buffers allowed two; the waves spend
// most of their time waiting, and the extra blocks hide more of it (layer-1
// weight gradient at 8192 rows: 102 -> 84 us).  Same contract as gemm_kernel.
template <bool A_KM, bool B_KN, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void gemm128_kernel(const uint16_t* __restrict__ A, int lda,
                                                             const uint16_t* __restrict__ B, int ldb,
                                                             int M, int N, int K, int kper, float* part,
                                                             Epi ep) {
  constexpr int T = 128, LDS = 72;  // padded row (k) length
  constexpr int NJ = WAVES == 8 ? 2 : 4;  // 16-column MFMA tiles per wave
  __shared__ __attribute__((aligned(16))) uint16_t As[T * LDS];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[T * LDS];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m0 = blockIdx.y * T, n0 = blockIdx.x * T;
  // four waves: 2 x 2 of 64 x 64; eight waves: 2 x 4 of 64 x 32
  const int wm = WAVES == 8 ? (w >> 2) * 64 : (w >> 1) * 64;
  const int wn = WAVES == 8 ? (w & 3) * 32 : (w & 1) * 64;
  f32x4 acc[4][NJ];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int kbeg = blockIdx.z * kper * 32, kend = min(K, kbeg + kper * 32);
  // with eight waves, waves 0-3 carry A and waves 4-7 carry B (in ra*)
  const int tt = t & 255;
  const bool carry_a = WAVES == 4 || t < 256;
  uint4 ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;
  auto fetch = [&](int k0) {
    const bool hi = k0 + 32 < kend;
    if (WAVES == 4) {
      fetch128<A_KM>(A, lda, m0, M, k0, t, true, ra0, ra1);
      fetch128<A_KM>(A, lda, m0, M, k0 + 32, t, hi, ra2, ra3);
      fetch128<B_KN>(B, ldb, n0, N, k0, t, true, rb0, rb1);
      fetch128<B_KN>(B, ldb, n0, N, k0 + 32, t, hi, rb2, rb3);
    } else if (carry_a) {
      fetch128<A_KM>(A, lda, m0, M, k0, tt, true, ra0, ra1);
      fetch128<A_KM>(A, lda, m0, M, k0 + 32, tt, hi, ra2, ra3);
    } else {
      fetch128<B_KN>(B, ldb, n0, N, k0, tt, true, ra0, ra1);
      fetch128<B_KN>(B, ldb, n0, N, k0 + 32, tt, hi, ra2, ra3);
    }
  };
  auto stash = [&]() {
    if (WAVES == 4) {
      stash128<A_KM, LDS>(As, 0, t, ra0, ra1);
      stash128<A_KM, LDS>(As, 32, t, ra2, ra3);
      stash128<B_KN, LDS>(Bs, 0, t, rb0, rb1);
      stash128<B_KN, LDS>(Bs, 32, t, rb2, rb3);
    } else if (carry_a) {
      stash128<A_KM, LDS>(As, 0, tt, ra0, ra1);
      stash128<A_KM, LDS>(As, 32, tt, ra2, ra3);
    } else {
      stash128<B_KN, LDS>(Bs, 0, tt, ra0, ra1);
      stash128<B_KN, LDS>(Bs, 32, tt, ra2, ra3);
    }
  };
  if (kbeg < kend) {
    fetch(kbeg);
    stash();
  }
  __syncthreads();
  const int r16 = lane & 15, kq = (lane >> 4) * 8;
  for (int k0 = kbeg; k0 < kend; k0 += 64) {
    const bool more = k0 + 64 < kend;
    if (more) fetch(k0 + 64);  // in flight during this step's MFMAs
#pragma unroll
    for (int kk = 0; kk < 64; kk += 32) {  // the upper half of a short last step is zeros
      bf16x8 a[4], b[NJ];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        a[i] = *reinterpret_cast<const bf16x8*>(&As[swz128<LDS>(wm + i * 16 + r16, kk + kq)]);
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        b[j] = *reinterpret_cast<const bf16x8*>(&Bs[swz128<LDS>(wn + j * 16 + r16, kk + kq)]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();  // every wave has read this step's tiles
    if (more) stash();
    __syncthreads();
  }
  // D layout: lane holds column (lane % 16), rows 4*(lane/16) .. +3
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + i * 16 + (lane >> 4) * 4 + r;
        const int col = n0 + wn + j * 16 + (lane & 15);
        if (row >= M || col >= N) continue;
        if (part)
          part[((int64_t)blockIdx.z * M + row) * N + col] = acc[i][j][r];
        else
          apply_epi(ep, row, col, acc[i][j][r]);
      }
}

// Sum of the S split-K slices of part in slice order, then the epilogue.
__global__ __launch_bounds__(256) void splitk_epi_kernel(const float* __restrict__ part, int S,
                                                         int M, int N, Epi ep) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, MN = (int64_t)M * N;
  if (i >= MN) return;
  float v = part[i];
  int z = 1;
  for (; z + 4 <= S; z += 4) {  // four loads in flight, the sum still in slice order
    const float a = part[z * MN + i], b = part[(z + 1) * MN + i];
    const float c = part[(z + 2) * MN + i], e = part[(z + 3) * MN + i];
    v += a;
    v += b;
    v += c;
    v += e;
  }
  for (; z < S; ++z) v += part[z * MN + i];
  const int ii = (int)i, row = ii / N;  // M N <= the split-K workspace, far below 2^31
  apply_epi(ep, row, ii - row * N, v);
}

// dy = 2 (y - target) / (B * n) (FP32 and BF16) and per-row squared-error
// sums: one wave per row (four rows per block), each lane summing columns
// lane, lane + 64, ... in order, then a butterfly over the wave.  A lane's
// loads (up to eight) are all issued before its first store.
__global__ __launch_bounds__(256) void loss_kernel(const float* y, const float* target, int B,
                                                   int n, float* dy, uint16_t* dy16,
                                                   float* row_sq) {
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= B) return;  // whole waves
  float acc = 0.f;
  const float scale = 2.f / ((float)B * (float)n);
  const float* yr = y + (int64_t)r * n;
  const float* tr = target + (int64_t)r * n;
  for (int j0 = lane; j0 < n; j0 += 8 * 64) {  // every load of the pass in flight at once
    float e[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = j0 + 64 * u;
      e[u] = j < n ? yr[j] - tr[j] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = j0 + 64 * u;
      if (j < n) {
        acc += e[u] * e[u];
        dy[(int64_t)r * n + j] = scale * e[u];
        dy16[(int64_t)r * n + j] = to_bf16(scale * e[u]);
      }
    }
  }
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) acc += __shfl_xor(acc, m);
  if (lane == 0) row_sq[r] = acc;
}

// Mean of the per-row squared errors (one block of 1024 threads, fixed order:
// thread t sums rows t, t + 1024, ... eight loads at a time, then a butterfly
// per wave and the sixteen wave sums in wave order).
__global__ __launch_bounds__(1024) void loss_sum_kernel(const float* row_sq, int B, float scale,
                                                        float* out) {
  __shared__ float s[16];
  const int t = threadIdx.x, lane = t & 63;
  float acc = 0.f;
  for (int r0 = t; r0 < B; r0 += 8 * 1024) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = r0 + u * 1024 < B ? row_sq[r0 + u * 1024] : 0.f;
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) acc += __shfl_xor(acc, m);
  if (lane == 0) s[t >> 6] = acc;
  __syncthreads();
  if (t == 0) {
    float tot = 0.f;
    for (int w = 0; w < 16; ++w) tot += s[w];
    out[0] = tot * scale;
  }
}

// Training targets of instance i: its final group bests, normalised by the
// map size (row i of T, Eq.(10) layout per group).
__global__ __launch_bounds__(256) void targets_kernel(Pools pl, float* T, int ldt) {
  const int inst = blockIdx.x;
  const InstDesc& d = pl.desc[inst];
  const int D = 2 * d.W;
  for (int j = threadIdx.x; j < d.G * D && j < ldt; j += blockDim.x) {
    const int dd = j % D;
    T[(int64_t)inst * ldt + j] = pl.gbest_pos[d.gpo + j] / (dd < d.W ? d.width : d.height);
  }
}

// Column sums of a B x n FP32 matrix (bias gradients), in a fixed order:
// block (x, y) takes 64 columns of the row chunk [cr y, cr y + cr), its
// wave w sums rows w, w+4, ... of the chunk (eight loads in flight per lane)
// and the four partial sums are added in wave order into part[y][col];
// colsum_fin_kernel then adds the chunks in a fixed order.  Chunks are 256
// rows when that still gives 128 blocks or more, else 32 (a small batch: more
// blocks, one round of loads per wave).
__global__ __launch_bounds__(256) void colsum_kernel(const float* dz, int B, int n, int cr,
                                                     float* part) {
  __shared__ float ps[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + lane;
  const int r0 = blockIdx.y * cr, r1 = min(B, r0 + cr);
  float s = 0.f;
  if (j < n) {
#pragma unroll 8
    for (int r = r0 + w; r < r1; r += 4) s += dz[(int64_t)r * n + j];
  }
  ps[w][lane] = s;
  __syncthreads();
  if (w == 0 && j < n) part[(int64_t)blockIdx.y * n + j] = ((ps[0][lane] + ps[1][lane]) + ps[2][lane]) + ps[3][lane];
}

// 32 columns per block, eight threads per column: thread `sub` adds chunks
// sub, sub + 8, ... in order, then the eight sums are added pairwise in a
// fixed tree (the same order on every call).
__global__ __launch_bounds__(256) void colsum_fin_kernel(const float* part, int R, int n, float* out) {
  __shared__ float ps[8][32];
  const int c = threadIdx.x & 31, sub = threadIdx.x >> 5;
  const int j = blockIdx.x * 32 + c;
  float s = 0.f;
  if (j < n) {
#pragma unroll 4
    for (int y = sub; y < R; y += 8) s += part[(int64_t)y * n + j];
  }
  ps[sub][c] = s;
  __syncthreads();
  if (sub == 0 && j < n)
    out[j] = ((ps[0][c] + ps[1][c]) + (ps[2][c] + ps[3][c])) + ((ps[4][c] + ps[5][c]) + (ps[6][c] + ps[7][c]));
}

// Adam on FP32 master weights, refreshing the BF16 copies used by the GEMMs,
// over up to kAdamMaxSets parameter tensors in one launch: block b belongs
// to the set whose block range holds it.
__global__ __launch_bounds__(256) void adam_sets_kernel(AdamSets a, float lr, float b1, float b2,
                                                        float eps, float c1, float c2) {
  int k = 0;
  while (k + 1 < a.n && (int64_t)blockIdx.x >= a.first_block[k + 1]) ++k;
  const int64_t i = ((int64_t)blockIdx.x - a.first_block[k]) * blockDim.x + threadIdx.x;
  if (i >= a.count[k]) return;
  const float gi = a.g[k][i];
  const float mi = b1 * a.m[k][i] + (1.f - b1) * gi;
  const float vi = b2 * a.v[k][i] + (1.f - b2) * gi * gi;
  a.m[k][i] = mi;
  a.v[k][i] = vi;
  const float pi = a.p[k][i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  a.p[k][i] = pi;
  if (a.p16[k]) a.p16[k][i] = to_bf16(pi);
}

__global__ __launch_bounds__(256) void cvt_bf16_kernel(const float* p, uint16_t* p16, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p16[i] = to_bf16(p[i]);
}

// Accept the network's proposals: eligible instances with a finite output
// get per-group initial paths (clamped to the map); others fall back.
__global__ __launch_bounds__(256) void proposal_kernel(Pools pl, const float* Y, int ldy,
                                                       const int32_t* eligible) {
  const int inst = blockIdx.x;
  const InstDesc& d = pl.desc[inst];
  __shared__ int s_ok;
  if (threadIdx.x == 0) s_ok = eligible[inst];
  __syncthreads();
  const int D = 2 * d.W;
  if (s_ok) {
    for (int j = threadIdx.x; j < kLinOut; j += blockDim.x)
      if (!isfinite(Y[(int64_t)inst * ldy + j])) atomicAnd(&s_ok, 0);
  }
  __syncthreads();
  if (s_ok) {
    for (int j = threadIdx.x; j < d.G * D; j += blockDim.x) {
      const int dd = j % D;
      const float hi = dd < d.W ? d.width : d.height;
      float u = Y[(int64_t)inst * ldy + j];
      u = u < 0.f ? 0.f : (u > 1.f ? 1.f : u);
      pl.proposal[d.gpo + j] = u * hi;
    }
  }
  if (threadIdx.x == 0) pl.ctl[inst].use_learned = s_ok;
}

// ---------------------------------------------------------------------------
void launch_raster(const Pools& pl, int n_inst, uint16_t* X, int ldx, int32_t* eligible,
                   hipStream_t s) {
  hipLaunchKernelGGL(raster_kernel, dim3(n_inst), dim3(256), 0, s, pl, X, ldx, eligible);
}

void launch_gemm(bool a_km, bool b_kn, const uint16_t* A, int lda, const uint16_t* B, int ldb,
                 int M, int N, int K, const Epi& ep, float* ws, int64_t ws_floats, hipStream_t s) {
  // 128 x 128 tiles once they alone give a quarter of the CUs a tile; then
  // split K until the grid has two blocks per CU, as far as the k-steps and
  // the workspace allow
  // (measured: even two-step slices pay for their slice sum at the training
  // shapes; 512 blocks against 256 took the batch-8192 step from 0.83 to
  // 0.73 ms).
  // A long reduction over a transposed operand (the weight gradients of the
  // 512-wide layers, K = the batch) also takes the 128 tiles, split up to 16
  // ways: their transposed stash is the conflict-free one.
  const int tiles128 = ((N + 127) / 128) * ((M + 127) / 128);
  const bool long_k = K >= 2048 && (a_km || b_kn);
  const int T = tiles128 >= 64 || long_k ? 128 : 64;
  const int smax = T == 128 && tiles128 < 64 ? 16 : 8;
  const int tiles = ((N + T - 1) / T) * ((M + T - 1) / T), steps = K / 32;
  int S = 1;
  // a short reduction on a grid that already gives every CU a block keeps
  // its epilogue in the product kernel (the slice sum would cost more)
  const bool whole = T == 128 && tiles >= 256 && K <= 1024;
  while (!whole && S < smax && tiles * S < 512 && S * 2 <= steps &&
         (int64_t)S * 2 * M * N <= ws_floats)
    S *= 2;
  const int kper = steps > 0 ? (steps + S - 1) / S : 1;
  S = steps > 0 ? (steps + kper - 1) / kper : 1;
  float* part = S > 1 ? ws : nullptr;
  const dim3 grid((N + T - 1) / T, (M + T - 1) / T, S);
  if (T == 128 && K >= 2048 && tiles128 >= 64) {
    // large products (the first layer's): four waves of 64 x 64 (fewer LDS
    // reads per MFMA; the grid alone fills the CUs)
    const dim3 blk(256);
    if (!a_km && !b_kn)
      hipLaunchKernelGGL((gemm128_kernel<false, false, 4>), grid, blk, 0, s, A, lda, B, ldb, M, N, K, kper, part, ep);
    else if (!a_km && b_kn)
      hipLaunchKernelGGL((gemm128_kernel<false, true, 4>), grid, blk, 0, s, A, lda, B, ldb, M, N, K, kper, part, ep);
    else if (a_km && b_kn)
      hipLaunchKernelGGL((gemm128_kernel<true, true, 4>), grid, blk, 0, s, A, lda, B, ldb, M, N, K, kper, part, ep);
    else
      hipLaunchKernelGGL((gemm128_kernel<true, false, 4>), grid, blk, 0, s, A, lda, B, ldb, M, N, K, kper, part, ep);
  } else if (T == 128) {
    // the rest: eight waves of 64 x 32 (more waves to cover the loads' latency)
    const dim3 blk(512);
    if (!a_km && !b_kn)
      hipLaunchKernelGGL((gemm128_kernel<false, false, 8>), grid, blk, 0, s, A, lda, B, ldb, M, N, K, kper, part, ep);
    else if (!a_km && b_kn)
      hipLaunchKernelGGL((gemm128_kernel<false, true, 8>), grid, blk, 0, s, A, lda, B, ldb, M, N, K, kper, part, ep);
    else if (a_km && b_kn)
      hipLaunchKernelGGL((gemm128_kernel<true, true, 8>), grid, blk, 0, s, A, lda, B, ldb, M, N, K, kper, part, ep);
    else
      hipLaunchKernelGGL((gemm128_kernel<true, false, 8>), grid, blk, 0, s, A, lda, B, ldb, M, N, K, kper, part, ep);
  } else if (!a_km && !b_kn)
    hipLaunchKernelGGL((gemm_kernel<false, false>), grid, dim3(256), 0, s, A, lda, B, ldb, M, N, K, kper, part, ep);
  else if (!a_km && b_kn)
    hipLaunchKernelGGL((gemm_kernel<false, true>), grid, dim3(256), 0, s, A, lda, B, ldb, M, N, K, kper, part, ep);
  else if (a_km && b_kn)
    hipLaunchKernelGGL((gemm_kernel<true, true>), grid, dim3(256), 0, s, A, lda, B, ldb, M, N, K, kper, part, ep);
  else
    hipLaunchKernelGGL((gemm_kernel<true, false>), grid, dim3(256), 0, s, A, lda, B, ldb, M, N, K, kper, part, ep);
  if (part) {
    const int64_t MN = (int64_t)M * N;
    hipLaunchKernelGGL(splitk_epi_kernel, dim3((unsigned)((MN + 255) / 256)), dim3(256), 0, s,
                       part, S, M, N, ep);
  }
}

void launch_loss(const float* y, const float* target, int B, int n, float* dy, uint16_t* dy16,
                 float* row_sq, hipStream_t s) {
  hipLaunchKernelGGL(loss_kernel, dim3((B + 3) / 4), dim3(256), 0, s, y, target, B, n, dy, dy16, row_sq);
}

void launch_loss_sum(const float* row_sq, int B, float scale, float* out, hipStream_t s) {
  hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(1024), 0, s, row_sq, B, scale, out);
}

void launch_targets(const Pools& pl, int n_inst, float* T, int ldt, hipStream_t s) {
  hipLaunchKernelGGL(targets_kernel, dim3(n_inst), dim3(256), 0, s, pl, T, ldt);
}

void launch_colsum(const float* dz, int B, int n, float* out, float* ws, hipStream_t s) {
  const int nb = (n + 63) / 64;
  const int cr = (int64_t)nb * ((B + 255) / 256) >= 128 ? 256 : 32;
  const int R = (B + cr - 1) / cr;
  hipLaunchKernelGGL(colsum_kernel, dim3(nb, R), dim3(256), 0, s, dz, B, n, cr, ws);
  hipLaunchKernelGGL(colsum_fin_kernel, dim3((n + 31) / 32), dim3(256), 0, s, ws, R, n, out);
}

void launch_adam_sets(AdamSets a, float lr, float b1, float b2, float eps, float c1, float c2,
                      hipStream_t s) {
  int64_t blocks = 0;
  for (int k = 0; k < a.n; ++k) {
    a.first_block[k] = blocks;
    blocks += (a.count[k] + 255) / 256;
  }
  if (blocks == 0) return;
  hipLaunchKernelGGL(adam_sets_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a, lr, b1, b2, eps,
                     c1, c2);
}

void launch_cvt_bf16(const float* p, uint16_t* p16, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(cvt_bf16_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, p16, count);
}

void launch_proposal(const Pools& pl, int n_inst, const float* Y, int ldy, const int32_t* eligible,
                     hipStream_t s) {
  hipLaunchKernelGGL(proposal_kernel, dim3(n_inst), dim3(256), 0, s, pl, Y, ldy, eligible);
}

}  // namespace sepso
