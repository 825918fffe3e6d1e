// Host-side internals shared by the C-ABI translation units: error state,
// workspace layout, and the batch / context / learned-initializer handles.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/sepso.h"
#include "common.h"

namespace sepso {

inline thread_local std::string g_err;

inline sepso_status fail(sepso_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

// Workspace carve-up of a batch (byte offsets of every pool).
struct Layout {
  size_t desc, ctl, X, V, P, f, L, Pf, PL, Q, PQ, edges, verts, pptr, pvel, ends, endv, gbn, gbf, hyper, ohyper, ov, op, opf, gpos, tpos, prev, prop, blkt, blki, total;
  int64_t sumPD = 0, sumP = 0, sumTilesMax = 0;
  int64_t sumE = 0, sumPP = 0, sumPoly = 0, sumG = 0, sumGD = 0, sumD = 0, initBlocks = 0;
  int64_t sumR = 0, sumGE = 0, sumCP = 0;  // rectangles, edges of other polygons, convex polygons
  size_t rects = 0, pkind = 0, cpolys = 0;
};

}  // namespace sepso

struct sepso_lin;

namespace sepso {
// Instances that share one tile shape of the fused iteration: one launch per
// bucket and iteration over its slice of the block table.
struct TileBucket {
  sepso_tune tune{16, 256};
  std::vector<int> inst;      // instance indices
  int first_block = 0, n_blocks = 0;
  Pools pl{};                 // the batch's pools with this bucket's block slice and LDS sizing
};
}  // namespace sepso

struct sepso_batch {
  int n = 0;
  std::vector<sepso::InstDesc> desc;
  std::vector<int> n_vert;
  std::vector<int32_t> h_pptr;  // polygon offsets of instance 0
  std::vector<float> h_hyper0;  // every instance's hyper-parameters as created
  std::vector<int2> h_kind;     // polygon kinds of instance 0
  std::vector<int64_t> path_off;
  sepso::Layout lay{};
  sepso::Pools pl{};
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool broken = false;
  sepso_tune tune{16, 256};    // the tile of every instance when there is one bucket
  std::vector<sepso::TileBucket> buckets;  // always >= 1 after creation
  std::vector<hipStream_t> bstreams;       // side streams for concurrent bucket launches
  std::vector<hipEvent_t> bevents;         // [0] fork, [1 + j] bucket j done
  int tile_blocks = 0;
  int frames_done = 0;
  int tune_gen = 0;  // bumped whenever the tile plan changes (captured graphs go stale)
  // pinned host mirrors
  sepso::InstCtl* h_ctl = nullptr;
  float* h_paths = nullptr;
  hipGraphExec_t graph[2] = {nullptr, nullptr};  // [0] no motion, [1] motion step first
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  sepso_lin* lin = nullptr;  // attached learned initializer (not owned)
};

struct sepso_ctx {
  sepso_batch* b;
};

// Learned initializer: BF16 MLP 4100 -> 512 -> 512 -> 512 -> 320 with FP32
// master weights and Adam state, activations for up to max_rows rows, and an
// on-device training set of up to max_samples (input, target) rows.
struct sepso_lin {
  int max_rows = 0;
  int64_t max_samples = 0, n_samples = 0;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool broken = false;
  int adam_t = 0;
  float* W32[4];
  float* b32[4];
  uint16_t* W16[4];
  float *mW[4], *vW[4], *mb[4], *vb[4];
  float* gW[4];
  float* gb[4];
  uint16_t* X16;     // max_rows x kLinInPad
  uint16_t* A16[3];  // max_rows x 512
  float* Y;          // max_rows x 320
  float* T;          // max_rows x 320
  float* dY;
  uint16_t* dY16;
  float* dZ[3];
  uint16_t* dZ16[3];
  float* rowsq;
  float* dloss;       // loss per training step
  float* splitk;      // split-K GEMM slices
  int32_t* eligible;  // max_rows
  uint16_t* DX;       // max_samples x kLinInPad
  float* DT;          // max_samples x 320
  float* h_loss = nullptr;  // pinned, max_rows
};

namespace sepso {
// Higher level of the evolution phase (H-SEPSO), shared by the path-planning
// and the benchmark-function lower levels (api.cpp).
sepso_status evolve_cfg_check(const sepso_evolve_cfg* cfg);
// Device bytes of the H state for H particles of Dh values each.
size_t evolve_h_bytes(const sepso_evolve_cfg* cfg, int Dh);
// Carves the H state out of base (evolve_h_bytes bytes) into d's pointers and
// sizes; consts receives the host image of d->h_hyper, lo and hi (6 Gh + 12
// floats, contiguous from d->h_hyper) for the caller to upload.
void evolve_h_carve(const sepso_evolve_cfg* cfg, int Dh, char* base, EvolveDev* d,
                    std::vector<float>* consts);
// Synchronous reads of the H state on stream st.
hipError_t evolve_h_state(const EvolveDev& d, hipStream_t st, sepso_evolve_state* s);
// Total-best row and LFV; *k = evolutions done (nothing else is read when 0).
hipError_t evolve_h_best(const EvolveDev& d, hipStream_t st, float* hyper, float* lfv, int* k);
// Enqueues the copy of the curve entries of evolutions k0 + 1 .. k0 + n.
hipError_t evolve_h_curve(const EvolveDev& d, hipStream_t st, int k0, int n, float* curve);

// Learned-initializer hooks used by the frame loop (lin.cpp).
void lin_enqueue_proposals(sepso_lin* lin, sepso_batch* b);
}  // namespace sepso
