// Blocks of the planner's random streams, for inspection (sepso_philox).
#include "kernels.h"
#include "rng.h"

namespace sepso {

// Blocks of the random streams, for inspection: out[i] = Philox4x32-10 of the
// counter (first + i, c1, c2, c3) under key (k0, k1), the function every draw
// of the planner goes through.
__global__ __launch_bounds__(256) void philox_kernel(uint32_t first, uint32_t c1, uint32_t c2,
                                                     uint32_t c3, uint32_t k0, uint32_t k1,
                                                     int64_t n, uint4* out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const U4 r = philox(first + (uint32_t)i, c1, c2, c3, k0, k1);
    out[i] = make_uint4(r.v[0], r.v[1], r.v[2], r.v[3]);
  }
}

void launch_philox(uint32_t first, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t key, int64_t n,
                   uint32_t* out, hipStream_t s) {
  const int64_t want = (n + 255) / 256;
  const int blocks = (int)(want < 4096 ? want : 4096);
  hipLaunchKernelGGL(philox_kernel, dim3(blocks), dim3(256), 0, s, first, c1, c2, c3,
                     (uint32_t)key, (uint32_t)(key >> 32), n, reinterpret_cast<uint4*>(out));
}

}  // namespace sepso
