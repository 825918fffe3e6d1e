// Learned initializer: launchers of the device kernels (mlp.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "common.h"

namespace sepso {

enum : int { EPI_BIAS_RELU_BF16 = 0, EPI_BIAS_F32 = 1, EPI_F32 = 2, EPI_MASK = 3 };

// GEMM epilogue: what happens to each FP32 accumulator C(row, col).
struct Epi {
  int mode;              // EPI_*
  const float* bias;     // per column (EPI_BIAS_*)
  float* out_f32;        // row stride ldo
  uint16_t* out_bf16;    // row stride ldo
  const uint16_t* mask;  // ReLU mask source (BF16 activations), row stride ldo
  int ldo;
};

void launch_raster(const Pools& pl, int n_inst, uint16_t* X, int ldx, int32_t* eligible,
                   hipStream_t s);
// ws: FP32 split-K workspace of ws_floats (S x M x N are used when K is split).
void launch_gemm(bool a_km, bool b_kn, const uint16_t* A, int lda, const uint16_t* B, int ldb,
                 int M, int N, int K, const Epi& ep, float* ws, int64_t ws_floats, hipStream_t s);
void launch_loss(const float* y, const float* target, int B, int n, float* dy, uint16_t* dy16,
                 float* row_sq, hipStream_t s);
// ws: FP32 scratch of ceil(B / 256) x n (row-chunk partial sums).
void launch_colsum(const float* dz, int B, int n, float* out, float* ws, hipStream_t s);
void launch_loss_sum(const float* row_sq, int B, float scale, float* out, hipStream_t s);
void launch_targets(const Pools& pl, int n_inst, float* T, int ldt, hipStream_t s);
// Parameter tensors updated by one Adam launch (p16 may be NULL per set).
constexpr int kAdamMaxSets = 8;
struct AdamSets {
  float* p[kAdamMaxSets];
  const float* g[kAdamMaxSets];
  float* m[kAdamMaxSets];
  float* v[kAdamMaxSets];
  uint16_t* p16[kAdamMaxSets];
  int64_t count[kAdamMaxSets];
  int64_t first_block[kAdamMaxSets];  // filled by launch_adam_sets
  int n;
};
void launch_adam_sets(AdamSets a, float lr, float b1, float b2, float eps, float c1, float c2,
                      hipStream_t s);
void launch_cvt_bf16(const float* p, uint16_t* p16, int64_t count, hipStream_t s);
void launch_proposal(const Pools& pl, int n_inst, const float* Y, int ldy, const int32_t* eligible,
                     hipStream_t s);

}  // namespace sepso
