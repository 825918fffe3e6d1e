// Learned initializer, host side: workspace carve-up, weight handling,
// forward / backward / Adam sequencing, on-device training-set collection
// from planner results, and the hook that feeds proposals to a batch's
// frame graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"
#include "mlp.h"

using namespace sepso;

namespace {

const int kInPad[4] = {kLinInPad, kLinHidden, kLinHidden, kLinHidden};
const int kInReal[4] = {kLinIn, kLinHidden, kLinHidden, kLinHidden};
const int kOutN[4] = {kLinHidden, kLinHidden, kLinHidden, kLinOut};
constexpr int kLossHist = 1 << 16;
// split-K slices (FP32): up to four of the layer-1 weight gradient
constexpr int64_t kSplitWs = 4 * kLinHidden * kLinInPad;

int64_t n_params() {
  int64_t n = 0;
  for (int l = 0; l < 4; ++l) n += (int64_t)kOutN[l] * kInReal[l] + kOutN[l];
  return n;
}

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

// Byte layout of the learned-initializer workspace; assigns pointers when
// L is given.
size_t lin_layout(int max_rows, int64_t max_samples, sepso_lin* L, char* base) {
  size_t o = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + o : nullptr;
    o = a256(o + std::max<size_t>(bytes, 4));
    return p;
  };
  for (int l = 0; l < 4; ++l) {
    const size_t nw = (size_t)kOutN[l] * kInPad[l], nb = kOutN[l];
    char* p;
    p = take(4 * nw); if (L) L->W32[l] = (float*)p;
    p = take(4 * nb); if (L) L->b32[l] = (float*)p;
    p = take(2 * nw); if (L) L->W16[l] = (uint16_t*)p;
    p = take(4 * nw); if (L) L->mW[l] = (float*)p;
    p = take(4 * nw); if (L) L->vW[l] = (float*)p;
    p = take(4 * nb); if (L) L->mb[l] = (float*)p;
    p = take(4 * nb); if (L) L->vb[l] = (float*)p;
    p = take(4 * nw); if (L) L->gW[l] = (float*)p;
    p = take(4 * nb); if (L) L->gb[l] = (float*)p;
  }
  char* p;
  p = take(2 * (size_t)max_rows * kLinInPad); if (L) L->X16 = (uint16_t*)p;
  for (int l = 0; l < 3; ++l) {
    p = take(2 * (size_t)max_rows * kLinHidden); if (L) L->A16[l] = (uint16_t*)p;
    p = take(4 * (size_t)max_rows * kLinHidden); if (L) L->dZ[l] = (float*)p;
    p = take(2 * (size_t)max_rows * kLinHidden); if (L) L->dZ16[l] = (uint16_t*)p;
  }
  p = take(4 * (size_t)max_rows * kLinOut); if (L) L->Y = (float*)p;
  p = take(4 * (size_t)max_rows * kLinOut); if (L) L->T = (float*)p;
  p = take(4 * (size_t)max_rows * kLinOut); if (L) L->dY = (float*)p;
  p = take(2 * (size_t)max_rows * kLinOut); if (L) L->dY16 = (uint16_t*)p;
  p = take(4 * (size_t)max_rows); if (L) L->rowsq = (float*)p;
  p = take(4 * (size_t)max_rows); if (L) L->eligible = (int32_t*)p;
  p = take(4 * (size_t)kLossHist); if (L) L->dloss = (float*)p;
  p = take(4 * (size_t)kSplitWs); if (L) L->splitk = (float*)p;
  p = take(2 * (size_t)max_samples * kLinInPad); if (L) L->DX = (uint16_t*)p;
  p = take(4 * (size_t)max_samples * kLinOut); if (L) L->DT = (float*)p;
  return o;
}

uint16_t host_bf16(float f) {  // round to nearest even
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

sepso_status lin_hip(sepso_lin* L, hipError_t e, const char* what) {
  L->broken = true;
  return fail(SEPSO_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define LHIP(L, expr)                                    \
  do {                                                   \
    hipError_t _e = (expr);                              \
    if (_e != hipSuccess) return lin_hip(L, _e, #expr);  \
  } while (0)

sepso_status lin_usable(sepso_lin* L) {
  if (!L) return fail(SEPSO_E_ARG, "learned initializer handle is NULL");
  if (L->broken) return fail(SEPSO_E_STATE, "learned initializer unusable after a HIP error");
  return SEPSO_OK;
}

void forward(sepso_lin* L, const uint16_t* X, int M, hipStream_t s) {
  const uint16_t* in = X;
  int ldi = kLinInPad;
  for (int l = 0; l < 3; ++l) {
    const Epi ep{EPI_BIAS_RELU_BF16, L->b32[l], nullptr, L->A16[l], nullptr, kLinHidden};
    launch_gemm(false, false, in, ldi, L->W16[l], kInPad[l], M, kLinHidden, kInPad[l], ep, L->splitk, kSplitWs, s);
    in = L->A16[l];
    ldi = kLinHidden;
  }
  const Epi ep{EPI_BIAS_F32, L->b32[3], L->Y, nullptr, nullptr, kLinOut};
  launch_gemm(false, false, L->A16[2], kLinHidden, L->W16[3], kLinHidden, M, kLinOut, kLinHidden, ep, L->splitk, kSplitWs, s);
}

// Gradients of the mean squared error for rows X (B rows) against targets T.
void backward(sepso_lin* L, const uint16_t* X, const float* T, int B, float* loss_slot,
              hipStream_t s) {
  launch_loss(L->Y, T, B, kLinOut, L->dY, L->dY16, L->rowsq, s);
  launch_loss_sum(L->rowsq, B, 1.f / ((float)B * kLinOut), loss_slot, s);
  launch_colsum(L->dY, B, kLinOut, L->gb[3], L->splitk, s);
  launch_gemm(true, true, L->dY16, kLinOut, L->A16[2], kLinHidden, kLinOut, kLinHidden, B,
              Epi{EPI_F32, nullptr, L->gW[3], nullptr, nullptr, kLinHidden}, L->splitk, kSplitWs, s);
  launch_gemm(false, true, L->dY16, kLinOut, L->W16[3], kLinHidden, B, kLinHidden, kLinOut,
              Epi{EPI_MASK, nullptr, L->dZ[2], L->dZ16[2], L->A16[2], kLinHidden}, L->splitk, kSplitWs, s);
  for (int l = 2; l >= 1; --l) {
    launch_colsum(L->dZ[l], B, kLinHidden, L->gb[l], L->splitk, s);
    launch_gemm(true, true, L->dZ16[l], kLinHidden, L->A16[l - 1], kLinHidden, kLinHidden,
                kLinHidden, B, Epi{EPI_F32, nullptr, L->gW[l], nullptr, nullptr, kLinHidden}, L->splitk, kSplitWs, s);
    launch_gemm(false, true, L->dZ16[l], kLinHidden, L->W16[l], kLinHidden, B, kLinHidden,
                kLinHidden, Epi{EPI_MASK, nullptr, L->dZ[l - 1], L->dZ16[l - 1], L->A16[l - 1], kLinHidden}, L->splitk, kSplitWs, s);
  }
  launch_colsum(L->dZ[0], B, kLinHidden, L->gb[0], L->splitk, s);
  launch_gemm(true, true, L->dZ16[0], kLinHidden, X, kLinInPad, kLinHidden, kLinInPad, B,
              Epi{EPI_F32, nullptr, L->gW[0], nullptr, nullptr, kLinInPad}, L->splitk, kSplitWs, s);
}

void adam(sepso_lin* L, float lr, hipStream_t s) {
  L->adam_t += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  // bias corrections from the same (FP32) decay rates the moments use
  const float c1 = (float)(1.0 - std::pow((double)b1, L->adam_t));
  const float c2 = (float)(1.0 - std::pow((double)b2, L->adam_t));
  // all eight tensors (weights and biases of the four layers) in one launch
  AdamSets a{};
  for (int l = 0; l < 4; ++l) {
    const int w = 2 * l, b = 2 * l + 1;
    a.p[w] = L->W32[l]; a.g[w] = L->gW[l]; a.m[w] = L->mW[l]; a.v[w] = L->vW[l];
    a.p16[w] = L->W16[l]; a.count[w] = (int64_t)kOutN[l] * kInPad[l];
    a.p[b] = L->b32[l]; a.g[b] = L->gb[l]; a.m[b] = L->mb[l]; a.v[b] = L->vb[l];
    a.p16[b] = nullptr; a.count[b] = kOutN[l];
  }
  a.n = 8;
  launch_adam_sets(a, lr, b1, b2, eps, c1, c2, s);
}

// Upload host FP32 rows (n x kLinIn) as BF16 rows of stride kLinInPad.
sepso_status upload_inputs(sepso_lin* L, const float* x, int n) {
  std::vector<uint16_t> h((size_t)n * kLinInPad, 0);
  for (int r = 0; r < n; ++r)
    for (int j = 0; j < kLinIn; ++j) h[(size_t)r * kLinInPad + j] = host_bf16(x[(size_t)r * kLinIn + j]);
  LHIP(L, hipMemcpyAsync(L->X16, h.data(), 2 * h.size(), hipMemcpyHostToDevice, L->stream));
  LHIP(L, hipStreamSynchronize(L->stream));
  return SEPSO_OK;
}

}  // namespace

namespace sepso {
void lin_enqueue_proposals(sepso_lin* L, sepso_batch* b) {
  launch_raster(b->pl, b->n, L->X16, kLinInPad, L->eligible, b->stream);
  forward(L, L->X16, b->n, b->stream);
  launch_proposal(b->pl, b->n, L->Y, kLinOut, L->eligible, b->stream);
}
}  // namespace sepso

extern "C" {

sepso_status sepso_lin_workspace_bytes(int32_t max_rows, int64_t max_samples, size_t* bytes) {
  if (!bytes || max_rows < 32 || max_rows % 32 || max_samples < 0)
    return fail(SEPSO_E_ARG, "need bytes, max_rows >= 32 and a multiple of 32, max_samples >= 0");
  *bytes = lin_layout(max_rows, max_samples, nullptr, nullptr);
  return SEPSO_OK;
}

sepso_status sepso_lin_create(int32_t max_rows, int64_t max_samples, uint64_t seed, void* d_ws,
                              size_t ws_bytes, void* stream, sepso_lin** out) {
  if (!out) return fail(SEPSO_E_ARG, "out is NULL");
  *out = nullptr;
  size_t need = 0;
  sepso_status st = sepso_lin_workspace_bytes(max_rows, max_samples, &need);
  if (st != SEPSO_OK) return st;
  if (!d_ws || reinterpret_cast<uintptr_t>(d_ws) % 256)
    return fail(SEPSO_E_ARG, "workspace NULL or not 256-byte aligned");
  if (ws_bytes < need) return fail(SEPSO_E_NOMEM, "workspace too small: %zu < %zu", ws_bytes, need);
  sepso_lin* L = new (std::nothrow) sepso_lin();
  if (!L) return fail(SEPSO_E_NOMEM, "host allocation failed");
  L->max_rows = max_rows;
  L->max_samples = max_samples;
  L->ws = static_cast<char*>(d_ws);
  lin_layout(max_rows, max_samples, L, L->ws);
  hipError_t e = hipSuccess;
  if (stream) {
    L->stream = static_cast<hipStream_t>(stream);
  } else {
    e = hipStreamCreateWithFlags(&L->stream, hipStreamNonBlocking);
    L->own_stream = e == hipSuccess;
  }
  // zero everything (padding columns, Adam moments, activations)
  if (e == hipSuccess) e = hipMemsetAsync(L->ws, 0, need, L->stream);
  // seeded uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases
  uint64_t x = seed * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  auto next = [&]() {  // splitmix64
    x += 0x9E3779B97F4A7C15ull;
    uint64_t z = x;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  for (int l = 0; l < 4 && e == hipSuccess; ++l) {
    const double a = 1.0 / std::sqrt((double)kInReal[l]);
    std::vector<float> w((size_t)kOutN[l] * kInPad[l], 0.f);
    for (int o = 0; o < kOutN[l]; ++o)
      for (int i = 0; i < kInReal[l]; ++i)
        w[(size_t)o * kInPad[l] + i] = (float)(-a + 2.0 * a * ((next() >> 11) * (1.0 / 9007199254740992.0)));
    e = hipMemcpyAsync(L->W32[l], w.data(), 4 * w.size(), hipMemcpyHostToDevice, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (e == hipSuccess) launch_cvt_bf16(L->W32[l], L->W16[l], (int64_t)w.size(), L->stream);
  }
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess) e = hipHostMalloc((void**)&L->h_loss, 4 * kLossHist, hipHostMallocDefault);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (e != hipSuccess) {
    sepso_status s2 = fail(SEPSO_E_HIP, "lin create: %s", hipGetErrorString(e));
    if (L->own_stream) (void)hipStreamDestroy(L->stream);  // unwinding a failed create
    if (L->h_loss) (void)hipHostFree(L->h_loss);
    delete L;
    return s2;
  }
  *out = L;
  return SEPSO_OK;
}

sepso_status sepso_lin_destroy(sepso_lin* L) {
  if (!L) return fail(SEPSO_E_ARG, "handle is NULL");
  if (L->h_loss) (void)hipHostFree(L->h_loss);  // teardown: best effort
  if (L->own_stream) (void)hipStreamDestroy(L->stream);
  delete L;
  return SEPSO_OK;
}

int64_t sepso_lin_param_count(void) { return n_params(); }

sepso_status sepso_lin_set_weights(sepso_lin* L, const float* flat) {
  sepso_status st = lin_usable(L);
  if (st != SEPSO_OK) return st;
  if (!flat) return fail(SEPSO_E_ARG, "weights NULL");
  for (int64_t i = 0; i < n_params(); ++i)
    if (!std::isfinite(flat[i])) return fail(SEPSO_E_ARG, "weights must be finite");
  const float* p = flat;
  for (int l = 0; l < 4; ++l) {
    std::vector<float> w((size_t)kOutN[l] * kInPad[l], 0.f);
    for (int o = 0; o < kOutN[l]; ++o)
      for (int i = 0; i < kInReal[l]; ++i) w[(size_t)o * kInPad[l] + i] = *p++;
    LHIP(L, hipMemcpyAsync(L->W32[l], w.data(), 4 * w.size(), hipMemcpyHostToDevice, L->stream));
    LHIP(L, hipMemcpyAsync(L->b32[l], p, 4 * kOutN[l], hipMemcpyHostToDevice, L->stream));
    p += kOutN[l];
    LHIP(L, hipStreamSynchronize(L->stream));
    launch_cvt_bf16(L->W32[l], L->W16[l], (int64_t)w.size(), L->stream);
  }
  LHIP(L, hipGetLastError());
  LHIP(L, hipStreamSynchronize(L->stream));
  return SEPSO_OK;
}

sepso_status sepso_lin_get_weights(sepso_lin* L, float* flat) {
  sepso_status st = lin_usable(L);
  if (st != SEPSO_OK) return st;
  if (!flat) return fail(SEPSO_E_ARG, "weights NULL");
  float* p = flat;
  for (int l = 0; l < 4; ++l) {
    std::vector<float> w((size_t)kOutN[l] * kInPad[l]);
    LHIP(L, hipMemcpyAsync(w.data(), L->W32[l], 4 * w.size(), hipMemcpyDeviceToHost, L->stream));
    LHIP(L, hipMemcpyAsync(p + (size_t)kOutN[l] * kInReal[l], L->b32[l], 4 * kOutN[l],
                           hipMemcpyDeviceToHost, L->stream));
    LHIP(L, hipStreamSynchronize(L->stream));
    for (int o = 0; o < kOutN[l]; ++o)
      for (int i = 0; i < kInReal[l]; ++i) *p++ = w[(size_t)o * kInPad[l] + i];
    p += kOutN[l];
  }
  return SEPSO_OK;
}

sepso_status sepso_lin_forward(sepso_lin* L, const float* x, int32_t n, float* y) {
  sepso_status st = lin_usable(L);
  if (st != SEPSO_OK) return st;
  if (!x || !y || n < 1 || n > L->max_rows) return fail(SEPSO_E_ARG, "need x, y and 1 <= n <= max_rows");
  st = upload_inputs(L, x, n);
  if (st != SEPSO_OK) return st;
  forward(L, L->X16, n, L->stream);
  LHIP(L, hipGetLastError());
  LHIP(L, hipMemcpyAsync(y, L->Y, 4 * (size_t)n * kLinOut, hipMemcpyDeviceToHost, L->stream));
  LHIP(L, hipStreamSynchronize(L->stream));
  return SEPSO_OK;
}

sepso_status sepso_lin_grads(sepso_lin* L, const float* x, const float* t, int32_t n, float* loss,
                             float* grads) {
  sepso_status st = lin_usable(L);
  if (st != SEPSO_OK) return st;
  if (!x || !t || !grads || n < 32 || n % 32 || n > L->max_rows)
    return fail(SEPSO_E_ARG, "need x, t, grads and n a multiple of 32 within max_rows");
  st = upload_inputs(L, x, n);
  if (st != SEPSO_OK) return st;
  LHIP(L, hipMemcpyAsync(L->T, t, 4 * (size_t)n * kLinOut, hipMemcpyHostToDevice, L->stream));
  forward(L, L->X16, n, L->stream);
  backward(L, L->X16, L->T, n, L->dloss, L->stream);
  LHIP(L, hipGetLastError());
  LHIP(L, hipMemcpyAsync(L->h_loss, L->dloss, 4, hipMemcpyDeviceToHost, L->stream));
  float* p = grads;
  for (int l = 0; l < 4; ++l) {
    std::vector<float> g((size_t)kOutN[l] * kInPad[l]);
    LHIP(L, hipMemcpyAsync(g.data(), L->gW[l], 4 * g.size(), hipMemcpyDeviceToHost, L->stream));
    LHIP(L, hipMemcpyAsync(p + (size_t)kOutN[l] * kInReal[l], L->gb[l], 4 * kOutN[l],
                           hipMemcpyDeviceToHost, L->stream));
    LHIP(L, hipStreamSynchronize(L->stream));
    for (int o = 0; o < kOutN[l]; ++o)
      for (int i = 0; i < kInReal[l]; ++i) *p++ = g[(size_t)o * kInPad[l] + i];
    p += kOutN[l];
  }
  if (loss) *loss = L->h_loss[0];
  return SEPSO_OK;
}

sepso_status sepso_lin_collect(sepso_lin* L, sepso_batch* b) {
  sepso_status st = lin_usable(L);
  if (st != SEPSO_OK) return st;
  if (!b || b->broken) return fail(SEPSO_E_ARG, "batch NULL or unusable");
  if (b->frames_done < 1) return fail(SEPSO_E_STATE, "plan a frame before collecting its results");
  for (auto& d : b->desc)
    if (d.G != kLinGroups || d.W != kLinW)
      return fail(SEPSO_E_UNSUPPORTED, "collection needs %d groups of %d waypoints", kLinGroups, kLinW);
  if (L->n_samples + b->n > L->max_samples) return fail(SEPSO_E_NOMEM, "training set is full");
  uint16_t* X = L->DX + (size_t)L->n_samples * kLinInPad;
  float* T = L->DT + (size_t)L->n_samples * kLinOut;
  launch_raster(b->pl, b->n, X, kLinInPad, L->eligible, b->stream);
  launch_targets(b->pl, b->n, T, kLinOut, b->stream);
  LHIP(L, hipGetLastError());
  LHIP(L, hipStreamSynchronize(b->stream));
  L->n_samples += b->n;
  return SEPSO_OK;
}

sepso_status sepso_lin_samples(sepso_lin* L, int64_t* n) {
  if (!L || !n) return fail(SEPSO_E_ARG, "NULL argument");
  *n = L->n_samples;
  return SEPSO_OK;
}

sepso_status sepso_lin_train(sepso_lin* L, int32_t steps, int32_t batch, float lr, float* loss_out) {
  sepso_status st = lin_usable(L);
  if (st != SEPSO_OK) return st;
  if (steps < 1 || steps > kLossHist || batch < 32 || batch % 32 || batch > L->max_rows ||
      !(lr > 0.f) || L->n_samples < batch)
    return fail(SEPSO_E_ARG, "need 1 <= steps <= %d, batch a multiple of 32 <= max_rows and <= samples, lr > 0",
                kLossHist);
  const int64_t nb = L->n_samples / batch;
  for (int s = 0; s < steps; ++s) {
    const int64_t slot = s % nb;
    const uint16_t* X = L->DX + (size_t)slot * batch * kLinInPad;
    const float* T = L->DT + (size_t)slot * batch * kLinOut;
    forward(L, X, batch, L->stream);
    backward(L, X, T, batch, L->dloss + s, L->stream);
    adam(L, lr, L->stream);
  }
  LHIP(L, hipGetLastError());
  if (loss_out) {
    LHIP(L, hipMemcpyAsync(L->h_loss, L->dloss, 4 * (size_t)steps, hipMemcpyDeviceToHost, L->stream));
    LHIP(L, hipStreamSynchronize(L->stream));
    std::memcpy(loss_out, L->h_loss, 4 * (size_t)steps);
  }
  LHIP(L, hipStreamSynchronize(L->stream));
  return SEPSO_OK;
}

sepso_status sepso_lin_features(sepso_lin* L, sepso_batch* b, float* out) {
  sepso_status st = lin_usable(L);
  if (st != SEPSO_OK) return st;
  if (!b || !out || b->n > L->max_rows) return fail(SEPSO_E_ARG, "batch/out NULL or batch too large");
  launch_raster(b->pl, b->n, L->X16, kLinInPad, L->eligible, b->stream);
  LHIP(L, hipGetLastError());
  std::vector<uint16_t> h((size_t)b->n * kLinInPad);
  LHIP(L, hipMemcpyAsync(h.data(), L->X16, 2 * h.size(), hipMemcpyDeviceToHost, b->stream));
  LHIP(L, hipStreamSynchronize(b->stream));
  for (int r = 0; r < b->n; ++r)
    for (int j = 0; j < kLinIn; ++j) {
      const uint32_t u = (uint32_t)h[(size_t)r * kLinInPad + j] << 16;
      std::memcpy(&out[(size_t)r * kLinIn + j], &u, 4);
    }
  return SEPSO_OK;
}

sepso_status sepso_lin_attach(sepso_batch* b, sepso_lin* L) {
  if (!b) return fail(SEPSO_E_ARG, "batch is NULL");
  if (L && b->n > L->max_rows) return fail(SEPSO_E_ARG, "batch has more instances than max_rows");
  if (L && L->broken) return fail(SEPSO_E_STATE, "learned initializer unusable");
  b->lin = L;
  for (int m = 0; m < 2; ++m)
    if (b->graph[m]) {
      (void)hipGraphExecDestroy(b->graph[m]);  // retired; re-captured with the new initializer
      b->graph[m] = nullptr;
    }
  if (!L) {  // back to plain initialisation
    for (int i = 0; i < b->n; ++i) {
      InstCtl c;
      hipError_t e = hipMemcpy(&c, b->pl.ctl + i, sizeof(InstCtl), hipMemcpyDeviceToHost);
      if (e == hipSuccess) {
        c.use_learned = 0;
        e = hipMemcpy(b->pl.ctl + i, &c, sizeof(InstCtl), hipMemcpyHostToDevice);
      }
      if (e != hipSuccess) {
        b->broken = true;
        return fail(SEPSO_E_HIP, "detach: %s", hipGetErrorString(e));
      }
    }
  }
  return SEPSO_OK;
}

sepso_status sepso_lin_attach_ctx(sepso_ctx* ctx, sepso_lin* L) {
  if (!ctx) return fail(SEPSO_E_ARG, "ctx is NULL");
  return sepso_lin_attach(ctx->b, L);
}

}  // extern "C"
