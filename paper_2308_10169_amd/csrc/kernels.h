// Host-side launchers of the device kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "common.h"

namespace sepso {

void launch_geom(const Pools& pl, int n_inst, int move, hipStream_t s);
void launch_philox(uint32_t first, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t key, int64_t n,
                   uint32_t* out, hipStream_t s);
void launch_init(const Pools& pl, int n_blocks, int frame_override, int use_prev, hipStream_t s);
bool step_supported(int K);
// 32-bit words of dynamic LDS the fused iteration takes per block.
size_t iter_lds_words(int pos_floats, int stage_floats, int gb_floats, int ngb_max, int ppb_max,
                      int threads);
// One iteration's tile kernel (fused, or the update alone without
// STEP_FIT) over n_blocks entries of pl.blk_tiles; false for an unsupported K.
bool launch_tiles(const Pools& pl, int K, int n_blocks, int threads, int flags, hipStream_t s);
// The per-instance reduce that follows the tile kernels of an iteration.
void launch_reduce(const Pools& pl, int flags, hipStream_t s);
void launch_evolve_init(const EvolveDev& ev, const Pools& pl, hipStream_t s);
void launch_evolve_step(const EvolveDev& ev, const Pools& pl, int injected, hipStream_t s);

}  // namespace sepso
