// Path fitness of given paths on a polygonal map (Eq.(11)-(13)): polyline
// length L over [start, waypoints, target], Q = proper crossings of the W+1
// segments with every polygon edge, F = L + alpha * Q^beta.  Stateless: the
// caller passes device inputs and outputs and a device workspace.
//
//   fit_edges_kernel -- one thread per vertex: the edge from it to the next
//                       vertex of its polygon (the last closes the polygon);
//   fit_seg_kernel   -- one thread per (path, segment): the segment's length
//                       and its proper crossings with every edge (records
//                       staged through LDS), as per-segment partial results;
//   fit_sum_kernel   -- one thread per path: L and Q summed in segment order
//                       (deterministic), F.
//
// Orientation arithmetic: a segment p -> q is kept as (dx, dy) and the line
// constant nc = dy*p.x - dx*p.y, so orient(p, q, v) = dx*v.y - dy*v.x + nc
// is two FMAs; an edge a -> b likewise as (ex, ey) and ce = ex*a.y - ey*a.x.
// A test counts when both pairs of orientations have strictly opposite
// signs; touching and collinear contacts never count.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "../../include/sepso.h"
#include "internal.h"

namespace sepso {
namespace {

constexpr int kFitThreads = 256;
constexpr int kFitStage = 512;  // edge records per LDS pass (16 KiB)

struct FitEdge {
  float ax, ay, bx, by;  // end points
  float ex, ey, ce, pad; // b - a and the line constant
};
static_assert(sizeof(FitEdge) == 32, "FitEdge is 32 bytes");

__global__ __launch_bounds__(kFitThreads) void fit_edges_kernel(int n_polys, const int32_t* pptr,
                                                                const float* verts, int n_vert,
                                                                FitEdge* out) {
  const int j = blockIdx.x * kFitThreads + threadIdx.x;
  if (j >= n_vert) return;
  // polygon q with pptr[q] <= j < pptr[q + 1] (binary search; q stays in
  // [0, n_polys) whatever the offsets hold)
  int lo = 0, hi = n_polys;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pptr[mid] <= j)
      lo = mid;
    else
      hi = mid;
  }
  int nx = j + 1 < pptr[lo + 1] ? j + 1 : pptr[lo];
  if (nx < 0 || nx >= n_vert) nx = j;  // malformed offsets: a zero-length edge, no access outside
  FitEdge r;
  r.ax = verts[2 * j];
  r.ay = verts[2 * j + 1];
  r.bx = verts[2 * nx];
  r.by = verts[2 * nx + 1];
  r.ex = r.bx - r.ax;
  r.ey = r.by - r.ay;
  r.ce = fmaf(r.ex, r.ay, -(r.ey * r.ax));
  r.pad = 0.f;
  out[j] = r;
}

__device__ __forceinline__ bool opposite(float a, float b) {
  return (a < 0.f && b > 0.f) || (a > 0.f && b < 0.f);
}

__global__ __launch_bounds__(kFitThreads) void fit_seg_kernel(const FitEdge* edges, int n_edges,
                                                              const float* ends, const float* paths,
                                                              int n_seg, int W, int32_t* seg_q,
                                                              float* seg_l) {
  __shared__ FitEdge s_e[kFitStage];
  const int t = threadIdx.x;
  const int i = blockIdx.x * kFitThreads + t;
  const bool active = i < n_seg;
  const int S = W + 1;  // segments per path
  const int path = active ? i / S : 0, s = active ? i - path * S : 0;
  const float* x = paths + (int64_t)path * 2 * W;
  // points s and s + 1 of [start, w_1..w_W, target]
  auto point = [&](int k, float& px, float& py) {
    if (k == 0) {
      px = ends[0];
      py = ends[1];
    } else if (k == W + 1) {
      px = ends[2];
      py = ends[3];
    } else {
      px = x[k - 1];
      py = x[W + k - 1];
    }
  };
  float px = 0.f, py = 0.f, qx = 0.f, qy = 0.f;
  if (active) {
    point(s, px, py);
    point(s + 1, qx, qy);
  }
  const float dx = qx - px, dy = qy - py;
  const float nc = fmaf(dy, px, -(dx * py));
  int count = 0;
  for (int e0 = 0; e0 < n_edges; e0 += kFitStage) {
    const int ne = n_edges - e0 < kFitStage ? n_edges - e0 : kFitStage;
    __syncthreads();
    {
      const float4* src = reinterpret_cast<const float4*>(edges + e0);
      float4* dst = reinterpret_cast<float4*>(s_e);
      for (int q = t; q < 2 * ne; q += kFitThreads) dst[q] = src[q];
    }
    __syncthreads();
    if (active) {
      for (int e = 0; e < ne; ++e) {
        const FitEdge r = s_e[e];
        const float o1 = fmaf(dx, r.ay, fmaf(-dy, r.ax, nc));
        const float o2 = fmaf(dx, r.by, fmaf(-dy, r.bx, nc));
        const float o3 = fmaf(r.ex, py, fmaf(-r.ey, px, -r.ce));
        const float o4 = fmaf(r.ex, qy, fmaf(-r.ey, qx, -r.ce));
        count += (opposite(o1, o2) && opposite(o3, o4)) ? 1 : 0;
      }
    }
  }
  if (active) {
    seg_q[i] = count;
    seg_l[i] = __builtin_amdgcn_sqrtf(dx * dx + dy * dy);  // v_sqrt_f32, within 1 ulp
  }
}

__global__ __launch_bounds__(kFitThreads) void fit_sum_kernel(const int32_t* seg_q,
                                                              const float* seg_l, int n_paths,
                                                              int W, float alpha, int beta,
                                                              float* f, float* L, int32_t* Q) {
  const int p = blockIdx.x * kFitThreads + threadIdx.x;
  if (p >= n_paths) return;
  const int S = W + 1;
  int q = 0;
  float l = 0.f;
  for (int s = 0; s < S; ++s) {  // segment order: deterministic
    q += seg_q[(int64_t)p * S + s];
    l += seg_l[(int64_t)p * S + s];
  }
  const float qf = (float)q;
  float pw = 1.f;
  for (int b = 0; b < beta; ++b) pw *= qf;
  f[p] = l + alpha * pw;
  L[p] = l;
  Q[p] = q;
}

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

struct FitLayout {
  size_t edges, seg_q, seg_l, total;
};

FitLayout fit_layout(int64_t n_vert, int64_t n_paths, int W) {
  FitLayout l;
  const int64_t n_seg = n_paths * (W + 1);
  l.edges = 0;
  l.seg_q = a256(sizeof(FitEdge) * (size_t)n_vert);
  l.seg_l = l.seg_q + a256(sizeof(int32_t) * (size_t)n_seg);
  l.total = l.seg_l + a256(sizeof(float) * (size_t)n_seg);
  return l;
}

sepso_status fit_check(int32_t n_polys, int32_t n_vert, int32_t n_paths, int32_t W, float alpha,
                       int32_t beta) {
  if (n_polys < 0 || n_vert < 0) return fail(SEPSO_E_ARG, "fitness: n_polys and n_vert must be >= 0");
  if (n_vert > 0 && n_polys < 1) return fail(SEPSO_E_ARG, "fitness: vertices without polygons");
  if (n_paths < 0) return fail(SEPSO_E_ARG, "fitness: n_paths must be >= 0");
  if (W < 1 || W > kMaxW) return fail(SEPSO_E_ARG, "fitness: waypoints must be in [1, %d]", kMaxW);
  if ((int64_t)n_paths * (W + 1) > 0x7fffffffLL)
    return fail(SEPSO_E_ARG, "fitness: n_paths * (waypoints + 1) exceeds 2^31 - 1");
  if (beta < 1) return fail(SEPSO_E_ARG, "fitness: beta must be >= 1");
  if (!std::isfinite(alpha)) return fail(SEPSO_E_ARG, "fitness: alpha must be finite");
  return SEPSO_OK;
}

sepso_status fit_run(int32_t n_polys, int32_t n_vert, const int32_t* d_pptr, const float* d_verts,
                     const float* d_ends, const float* d_paths, int32_t n_paths, int32_t W,
                     float alpha, int32_t beta, float* d_f, float* d_L, int32_t* d_Q, char* ws,
                     hipStream_t s) {
  const FitLayout l = fit_layout(n_vert, n_paths, W);
  FitEdge* edges = reinterpret_cast<FitEdge*>(ws + l.edges);
  int32_t* seg_q = reinterpret_cast<int32_t*>(ws + l.seg_q);
  float* seg_l = reinterpret_cast<float*>(ws + l.seg_l);
  const int n_seg = n_paths * (W + 1);
  if (n_vert > 0)
    hipLaunchKernelGGL(fit_edges_kernel, dim3((n_vert + kFitThreads - 1) / kFitThreads),
                       dim3(kFitThreads), 0, s, n_polys, d_pptr, d_verts, n_vert, edges);
  hipLaunchKernelGGL(fit_seg_kernel, dim3((n_seg + kFitThreads - 1) / kFitThreads), dim3(kFitThreads),
                     0, s, edges, n_vert, d_ends, d_paths, n_seg, W, seg_q, seg_l);
  hipLaunchKernelGGL(fit_sum_kernel, dim3((n_paths + kFitThreads - 1) / kFitThreads),
                     dim3(kFitThreads), 0, s, seg_q, seg_l, n_paths, W, alpha, beta, d_f, d_L, d_Q);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(SEPSO_E_HIP, "fitness launch: %s", hipGetErrorString(e));
  return SEPSO_OK;
}

sepso_status fit_pointers(int32_t n_vert, const int32_t* d_pptr, const float* d_verts,
                          const float* d_ends, const float* d_paths, int32_t n_paths, float* d_f,
                          float* d_L, int32_t* d_Q) {
  if (n_vert > 0 && (!d_pptr || !d_verts))
    return fail(SEPSO_E_ARG, "fitness: poly_ptr and verts must be device pointers");
  if (n_paths > 0 && (!d_ends || !d_paths || !d_f || !d_L || !d_Q))
    return fail(SEPSO_E_ARG, "fitness: ends, paths and the outputs must be device pointers");
  return SEPSO_OK;
}

}  // namespace
}  // namespace sepso

using namespace sepso;

extern "C" {

sepso_status sepso_fitness_workspace_bytes(int32_t n_vert, int32_t n_paths, int32_t waypoints,
                                           size_t* bytes) {
  if (!bytes) return fail(SEPSO_E_ARG, "fitness: bytes is NULL");
  if (n_vert < 0 || n_paths < 0) return fail(SEPSO_E_ARG, "fitness: sizes must be >= 0");
  if (waypoints < 1 || waypoints > kMaxW)
    return fail(SEPSO_E_ARG, "fitness: waypoints must be in [1, %d]", kMaxW);
  *bytes = fit_layout(n_vert, n_paths, waypoints).total;
  return SEPSO_OK;
}

sepso_status sepso_fitness(int32_t n_polys, int32_t n_vert, const int32_t* d_poly_ptr,
                           const float* d_verts, const float* d_ends, const float* d_paths,
                           int32_t n_paths, int32_t waypoints, float alpha, int32_t beta,
                           float* d_f, float* d_L, int32_t* d_Q, void* d_ws, size_t ws_bytes,
                           void* stream) {
  sepso_status st = fit_check(n_polys, n_vert, n_paths, waypoints, alpha, beta);
  if (st == SEPSO_OK)
    st = fit_pointers(n_vert, d_poly_ptr, d_verts, d_ends, d_paths, n_paths, d_f, d_L, d_Q);
  if (st != SEPSO_OK) return st;
  if (n_paths == 0) return SEPSO_OK;
  const size_t need = fit_layout(n_vert, n_paths, waypoints).total;
  if (!d_ws || (reinterpret_cast<uintptr_t>(d_ws) & 255))
    return fail(SEPSO_E_ARG, "fitness: workspace must be a 256-byte aligned device pointer");
  if (ws_bytes < need)
    return fail(SEPSO_E_NOMEM, "fitness: workspace of %zu bytes, %zu needed", ws_bytes, need);
  return fit_run(n_polys, n_vert, d_poly_ptr, d_verts, d_ends, d_paths, n_paths, waypoints, alpha,
                 beta, d_f, d_L, d_Q, static_cast<char*>(d_ws), static_cast<hipStream_t>(stream));
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free variant: the workspace is a file-scope device array of
// kFitScratchBytes, one per GPU, shared by every call on that GPU.  Host code
// never uses the array's name as an address: its device address is looked up
// once per device (hipGetSymbolAddress, with that device current) and kept.
// ---------------------------------------------------------------------------
namespace sepso {
namespace {

constexpr size_t kFitScratchBytes = size_t(8) << 20;  // 8 MiB per GPU
constexpr int kFitMaxDevices = 64;

__device__ __align__(256) char scratch[kFitScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kFitMaxDevices] = {};

sepso_status scratch_ptr(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(SEPSO_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kFitMaxDevices)
    return fail(SEPSO_E_UNSUPPORTED, "fitness: device %d beyond the %d supported", dev, kFitMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SEPSO_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SEPSO_OK;
}

}  // namespace
}  // namespace sepso

extern "C" {

sepso_status sepso_fitness_noalloc(int32_t n_polys, int32_t n_vert, const int32_t* d_poly_ptr,
                                   const float* d_verts, const float* d_ends, const float* d_paths,
                                   int32_t n_paths, int32_t waypoints, float alpha, int32_t beta,
                                   float* d_f, float* d_L, int32_t* d_Q, void* stream) {
  sepso_status st = fit_check(n_polys, n_vert, n_paths, waypoints, alpha, beta);
  if (st == SEPSO_OK)
    st = fit_pointers(n_vert, d_poly_ptr, d_verts, d_ends, d_paths, n_paths, d_f, d_L, d_Q);
  if (st != SEPSO_OK) return st;
  if (n_paths == 0) return SEPSO_OK;
  const size_t need = fit_layout(n_vert, n_paths, waypoints).total;
  if (need > kFitScratchBytes)
    return fail(SEPSO_E_ARG,
                "fitness_noalloc: %d paths of %d waypoints on %d vertices need %zu bytes of "
                "scratch; the allocation-free variant holds %zu (use sepso_fitness with a workspace)",
                n_paths, waypoints, n_vert, need, kFitScratchBytes);
  void* ws = nullptr;
  st = scratch_ptr(&ws);
  if (st != SEPSO_OK) return st;
  return fit_run(n_polys, n_vert, d_poly_ptr, d_verts, d_ends, d_paths, n_paths, waypoints, alpha,
                 beta, d_f, d_L, d_Q, static_cast<char*>(ws), static_cast<hipStream_t>(stream));
}

}  // extern "C"
