// Device helpers shared by the HIP translation units: the Philox4x32-10
// counter-based generator, its 24-bit uniform, and a clamp.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

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

// x clamped to [lo, hi] for lo <= hi and x not NaN: the median of the three,
// one v_med3_f32 (the same value as comparing and selecting).
__device__ __forceinline__ float clampf(float x, float lo, float hi) {
  return __builtin_amdgcn_fmed3f(x, lo, hi);
}

}  // namespace sepso
