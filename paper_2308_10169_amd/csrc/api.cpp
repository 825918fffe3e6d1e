// libsepso host side: argument validation, workspace carve-up, the C-ABI
// entry points, and graph capture of whole planning frames.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sepso.h"
#include "common.h"
#include "internal.h"
#include "kernels.h"

using namespace sepso;

namespace {

// Table hyper8 (DTPSO / H-SEPSO defaults): default outer-swarm hyper.
const float kHyper8[8][6] = {
    {2, 1, 1, 0.4f, 0.2f, 0.2f}, {1, 1, 2, 0.7f, 0.3f, 0.1f}, {2, 2, 1, 0.8f, 0.1f, 0.6f},
    {2, 2, 1, 0.8f, 0.6f, 0.4f}, {2, 1, 2, 0.2f, 0.1f, 0.3f}, {2, 1, 2, 0.9f, 0.5f, 0.5f},
    {1, 2, 2, 0.4f, 0.1f, 0.8f}, {1, 2, 2, 0.9f, 0.3f, 0.3f}};

bool finite(float x) { return std::isfinite(x); }

sepso_status check_map(const sepso_map* m, int idx) {
  if (!m) return fail(SEPSO_E_ARG, "map[%d] is NULL", idx);
  if (!(finite(m->width) && finite(m->height) && m->width > 0.f && m->height > 0.f))
    return fail(SEPSO_E_ARG, "map[%d]: width/height must be finite and > 0", idx);
  if (m->n_polys < 0 || m->n_polys > (1 << 20))
    return fail(SEPSO_E_ARG, "map[%d]: n_polys out of range", idx);
  for (int e = 0; e < 2; ++e) {
    const float* p = e ? m->target : m->start;
    if (!(finite(p[0]) && finite(p[1]) && p[0] >= 0.f && p[0] <= m->width && p[1] >= 0.f &&
          p[1] <= m->height))
      return fail(SEPSO_E_ARG, "map[%d]: %s outside the map", idx, e ? "target" : "start");
  }
  for (int j = 0; j < 4; ++j)
    if (!finite(m->endpoint_vel[j])) return fail(SEPSO_E_ARG, "map[%d]: endpoint_vel", idx);
  if (m->n_polys == 0) return SEPSO_OK;
  if (!m->poly_ptr || !m->verts) return fail(SEPSO_E_ARG, "map[%d]: poly_ptr/verts NULL", idx);
  if (m->poly_ptr[0] != 0) return fail(SEPSO_E_ARG, "map[%d]: poly_ptr[0] != 0", idx);
  for (int q = 0; q < m->n_polys; ++q)
    if (m->poly_ptr[q + 1] - m->poly_ptr[q] < 3)
      return fail(SEPSO_E_ARG, "map[%d]: polygon %d has < 3 vertices", idx, q);
  const int nv = m->poly_ptr[m->n_polys];
  if (nv > (1 << 22)) return fail(SEPSO_E_ARG, "map[%d]: too many vertices", idx);
  for (int j = 0; j < nv; ++j) {
    const float x = m->verts[2 * j], y = m->verts[2 * j + 1];
    if (!(finite(x) && finite(y) && x >= 0.f && x <= m->width && y >= 0.f && y <= m->height))
      return fail(SEPSO_E_ARG, "map[%d]: vertex %d outside the map", idx, j);
  }
  if (m->poly_vel)
    for (int q = 0; q < 2 * m->n_polys; ++q)
      if (!finite(m->poly_vel[q])) return fail(SEPSO_E_ARG, "map[%d]: poly_vel", idx);
  return SEPSO_OK;
}

sepso_status check_swarm(const sepso_swarm* s, int idx) {
  if (!s) return fail(SEPSO_E_ARG, "swarm[%d] is NULL", idx);
  if (s->groups < 1 || s->groups > kMaxG) return fail(SEPSO_E_ARG, "swarm[%d]: groups in [1,%d]", idx, kMaxG);
  if (s->particles < 1) return fail(SEPSO_E_ARG, "swarm[%d]: particles >= 1", idx);
  if (s->waypoints < 1 || s->waypoints > kMaxW)
    return fail(SEPSO_E_ARG, "swarm[%d]: waypoints in [1,%d]", idx, kMaxW);
  if (s->max_iters < 1) return fail(SEPSO_E_ARG, "swarm[%d]: max_iters >= 1", idx);
  const double elems = (double)s->groups * s->particles * 2.0 * s->waypoints;
  if (elems > 1.0e9) return fail(SEPSO_E_ARG, "swarm[%d]: swarm too large", idx);
  if (!s->hyper) return fail(SEPSO_E_ARG, "swarm[%d]: hyper is NULL", idx);
  for (int j = 0; j < 6 * s->groups; ++j)
    if (!finite(s->hyper[j])) return fail(SEPSO_E_ARG, "swarm[%d]: hyper not finite", idx);
  for (int g = 0; g < s->groups; ++g)
    if (s->hyper[6 * g + 5] < 0.f) return fail(SEPSO_E_ARG, "swarm[%d]: V_limit < 0", idx);
  if (s->hsef_hyper)
    for (int j = 0; j < 6 * s->groups; ++j)
      if (!finite(s->hsef_hyper[j]) || (j % 6 == 5 && s->hsef_hyper[j] < 0.f))
        return fail(SEPSO_E_ARG, "swarm[%d]: hsef_hyper not finite or V_limit < 0", idx);
  if (!(finite(s->alpha) && s->alpha >= 0.f)) return fail(SEPSO_E_ARG, "swarm[%d]: alpha", idx);
  if (s->beta < 1 || s->beta > 16) return fail(SEPSO_E_ARG, "swarm[%d]: beta in [1,16]", idx);
  if (!(finite(s->pi_gamma) && s->pi_gamma >= 0.f && s->pi_gamma <= 1.f))
    return fail(SEPSO_E_ARG, "swarm[%d]: pi_gamma in [0,1]", idx);
  if (!(finite(s->pi_radius) && s->pi_radius >= 0.f))
    return fail(SEPSO_E_ARG, "swarm[%d]: pi_radius >= 0", idx);
  if (s->at_mode < 0 || s->at_mode > 3) return fail(SEPSO_E_ARG, "swarm[%d]: at_mode", idx);
  if (s->at_window < 1 || s->at_window >= kHist)
    return fail(SEPSO_E_ARG, "swarm[%d]: at_window in [1,%d]", idx, kHist - 1);
  if (!finite(s->at_delta)) return fail(SEPSO_E_ARG, "swarm[%d]: at_delta", idx);
  if (s->hsef_every < 0) return fail(SEPSO_E_ARG, "swarm[%d]: hsef_every >= 0", idx);
  if (s->rand_per_dim != 0 && s->rand_per_dim != 1)
    return fail(SEPSO_E_ARG, "swarm[%d]: rand_per_dim is 0 or 1", idx);
  return SEPSO_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// An axis-aligned rectangle: four vertices whose consecutive edges are
// alternately horizontal and vertical (either orientation).
bool is_axis_rect(const float* v, int m) {
  if (m != 4) return false;
  bool prev_h = false;
  for (int j = 0; j < 4; ++j) {
    const float ax = v[2 * j], ay = v[2 * j + 1];
    const float bx = v[2 * ((j + 1) % 4)], by = v[2 * ((j + 1) % 4) + 1];
    const bool h = ay == by && ax != bx, vt = ax == bx && ay != by;
    if (!h && !vt) return false;
    if (j > 0 && h == prev_h) return false;
    prev_h = h;
  }
  return true;
}

// A simple convex polygon of at most kCPolyMax vertices: every turn
// strictly the same way (cross products of consecutive edges, exact in
// double for the coordinates a map holds) and one turn around in total (so
// that a pentagram, whose turns also agree, does not pass).  Returns +1
// (counter-clockwise), -1 (clockwise) or 0 (not such a polygon).
int convex_turn(const float* v, int m) {
  if (m < 3 || m > kCPolyMax) return 0;
  int sign = 0;
  double turn = 0.0;
  for (int j = 0; j < m; ++j) {
    const double ax = v[2 * j], ay = v[2 * j + 1];
    const double bx = v[2 * ((j + 1) % m)], by = v[2 * ((j + 1) % m) + 1];
    const double cx = v[2 * ((j + 2) % m)], cy = v[2 * ((j + 2) % m) + 1];
    const double cr = (bx - ax) * (cy - by) - (by - ay) * (cx - bx);
    const int sg = cr > 0.0 ? 1 : cr < 0.0 ? -1 : 0;
    if (sg == 0 || (sign != 0 && sg != sign)) return 0;
    sign = sg;
    double a = std::atan2(cy - by, cx - bx) - std::atan2(by - ay, bx - ax);
    while (a > M_PI) a -= 2.0 * M_PI;
    while (a < -M_PI) a += 2.0 * M_PI;
    turn += a;
  }
  return std::fabs(std::fabs(turn) - 2.0 * M_PI) < 1.0 ? sign : 0;
}

// Per polygon of a map: (1, slot among rectangles), (2 counter-clockwise or
// 3 clockwise, slot among convex polygons) or (0, first slot among the
// other polygons' edges).
void classify_polys(const sepso_map& m, std::vector<int2>* kind, int* n_rects, int* n_gedges,
                    int* n_cpolys) {
  kind->assign(m.n_polys, make_int2(0, 0));
  int nr = 0, ne = 0, nc = 0;
  for (int q = 0; q < m.n_polys; ++q) {
    const int v0 = m.poly_ptr[q], cnt = m.poly_ptr[q + 1] - v0;
    if (is_axis_rect(m.verts + 2 * v0, cnt)) {
      (*kind)[q] = make_int2(1, nr++);
    } else if (const int turn = convex_turn(m.verts + 2 * v0, cnt)) {
      (*kind)[q] = make_int2(turn > 0 ? 2 : 3, nc++);
    } else {
      (*kind)[q] = make_int2(0, ne);
      ne += cnt;
    }
  }
  *n_rects = nr;
  *n_gedges = ne;
  if (n_cpolys) *n_cpolys = nc;
}

Layout plan_layout(const sepso_map* maps, const sepso_swarm* sw, int n, std::vector<InstDesc>* desc) {
  Layout L{};
  if (desc) desc->assign(n, InstDesc{});
  std::vector<int2> kind;
  for (int i = 0; i < n; ++i) {
    const int G = sw[i].groups, N = sw[i].particles, W = sw[i].waypoints, D = 2 * W;
    const int64_t P = (int64_t)G * N;
    int n_rects = 0, n_gedges = 0, n_cpolys = 0;
    classify_polys(maps[i], &kind, &n_rects, &n_gedges, &n_cpolys);
    if (desc) {
      InstDesc& d = (*desc)[i];
      d.n_rects = n_rects;
      d.n_gedges = n_gedges;
      d.n_cpolys = n_cpolys;
      d.ro = (int32_t)L.sumR;
      d.geo = (int32_t)L.sumGE;
      d.cpo = (int32_t)L.sumCP;
    }
    L.sumR += (n_rects + 3) & ~3;  // whole 64-byte quads per instance
    L.sumGE += n_gedges;
    L.sumCP += n_cpolys;
    if (desc) {
      InstDesc& d = (*desc)[i];
      d.G = G;
      d.N = N;
      d.W = W;
      d.T = sw[i].max_iters;
      d.n_polys = maps[i].n_polys;
      d.n_edges = maps[i].n_polys ? maps[i].poly_ptr[maps[i].n_polys] : 0;
      d.width = maps[i].width;
      d.height = maps[i].height;
      d.alpha = sw[i].alpha;
      d.beta = sw[i].beta;
      d.use_pi = sw[i].use_pi ? 1 : 0;
      d.n_pi = (int)std::ceil((double)sw[i].pi_gamma * (double)N);
      d.pi_radius = sw[i].pi_radius;
      d.at_mode = sw[i].at_mode;
      d.at_window = sw[i].at_window;
      d.at_delta = sw[i].at_delta;
      d.hsef_every = sw[i].hsef_every;
      d.T_outer = sw[i].hsef_every > 0 ? (sw[i].max_iters + sw[i].hsef_every - 1) / sw[i].hsef_every : 1;
      d.seed_lo = (uint32_t)(sw[i].seed & 0xffffffffu);
      d.seed_hi = (uint32_t)(sw[i].seed >> 32);
      d.instance = sw[i].instance;
      d.rand_per_dim = sw[i].rand_per_dim;
      d.xo = L.sumPD;
      d.po = L.sumP;
      d.eo = (int32_t)L.sumE;
      d.plo = (int32_t)L.sumPP;
      d.pvo = (int32_t)L.sumPoly;
      d.go = (int32_t)L.sumG;
      d.gpo = (int32_t)L.sumGD;
      d.dpo = (int32_t)L.sumD;
    }
    L.sumPD += (P * D + 3) & ~int64_t(3);  // 16-byte aligned per instance (float4 walks)
    L.sumP += P;
    L.sumTilesMax += P;  // at most one tile per particle
    L.sumE += maps[i].n_polys ? maps[i].poly_ptr[maps[i].n_polys] : 0;
    L.sumPP += maps[i].n_polys + 1;
    L.sumPoly += maps[i].n_polys;
    L.sumG += G;
    L.sumGD += (int64_t)G * D;
    L.sumD += D;
    L.initBlocks += (P * ((D + 3) / 4) + 255) / 256;  // one init thread per 4 coordinates
  }
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align256(o + std::max<size_t>(bytes, 4));
    return at;
  };
  L.desc = take(sizeof(InstDesc) * n);
  L.ctl = take(sizeof(InstCtl) * n);
  L.X = take(4 * L.sumPD);
  L.V = take(4 * L.sumPD);
  L.P = take(4 * L.sumPD);
  L.f = take(4 * L.sumP);
  L.L = take(4 * L.sumP);
  L.Pf = take(4 * L.sumP);
  L.PL = take(4 * L.sumP);
  L.Q = take(4 * L.sumP);
  L.PQ = take(4 * L.sumP);
  L.edges = take(sizeof(EdgeRec) * L.sumGE);
  L.cpolys = take(sizeof(CPoly) * L.sumCP);
  L.rects = take(32 * L.sumR);  // boxes, then centres and half sides
  L.pkind = take(8 * L.sumPoly);
  L.verts = take(8 * L.sumE);
  L.pptr = take(4 * L.sumPP);
  L.pvel = take(8 * L.sumPoly);
  L.ends = take(16 * n);
  L.endv = take(16 * n);
  L.gbn = take(4 * L.sumG);
  L.gbf = take(4 * L.sumG);
  L.hyper = take(24 * L.sumG);
  L.ohyper = take(24 * L.sumG);
  L.ov = take(12 * L.sumG);
  L.op = take(12 * L.sumG);
  L.opf = take(4 * L.sumG);
  L.gpos = take(4 * L.sumGD);
  L.tpos = take(4 * L.sumD);
  L.prev = take(4 * L.sumD);
  L.prop = take(4 * L.sumGD);
  L.blkt = take(8 * L.sumTilesMax);
  L.blki = take(8 * L.initBlocks);
  L.total = o;
  return L;
}

// Particles per block of the fused iteration: C = ceil((W+1)/K) chunks of K
// segments per particle, one thread per chunk; even, so that every block
// starts 16-byte aligned.
int tile_ppb(int W, int K, int B, int R) { return std::max(2, ((B / R) / ((W + K) / K)) & ~1); }

// Wave groups a block's rectangles are dealt over: 1 for a launch with
// enough blocks, else doubled (while whole waves remain: B/R >= 64) as long
// as the launch stays within two blocks per CU of the 256 -- small instances
// then run their crossing tests on up to four times as many waves.
constexpr int kCUs = 256;

int tile_rsplit(const std::vector<InstDesc>& desc, int K, int B) {
  auto blocks = [&](int R) {
    int64_t n = 0;
    for (const InstDesc& d : desc) {
      const int ppb = tile_ppb(d.W, K, B, R);
      n += ((int64_t)d.G * d.N + ppb - 1) / ppb;
    }
    return n;
  };
  int R = 1;
  while (2 * R <= B / 64 && blocks(2 * R) <= 2 * kCUs) R *= 2;
  return R;
}

// Dynamic LDS areas of the fused iteration for a tile shape: maxima over the
// instances (floats; counts of groups and particles per block).
struct TileLds {
  int pos, stage, gb, ngb, ppb;
};

TileLds tile_lds(const std::vector<InstDesc>& desc, int K, int B) {
  TileLds L{8, 8, 4, 1, 2};
  const int R = tile_rsplit(desc, K, B);
  for (const InstDesc& d : desc) {
    const int ppb = tile_ppb(d.W, K, B, R), D = 2 * d.W;
    const int ngb = std::min(d.G, (ppb - 1) / d.N + 2);  // groups ppb consecutive particles span
    L.pos = std::max(L.pos, ppb * D);
    L.stage = std::max(L.stage, std::min(kStageFloats, 8 * d.n_gedges));
    L.gb = std::max(L.gb, (ngb + 1) * D);
    L.ngb = std::max(L.ngb, ngb);
    L.ppb = std::max(L.ppb, ppb);
  }
  L.pos = (L.pos + 7) & ~7;      // records after it 32-byte aligned
  L.stage = (L.stage + 7) & ~7;
  L.gb = (L.gb + 3) & ~3;        // per-particle float4 words after it
  return L;
}

// A tile shape suits a batch when a thread's K segments are not mostly empty
// for the shortest path (K <= 2(W+2)), B*K <= 4096, and the fused
// iteration's LDS for this batch stays within 64 KiB.
bool tune_ok(int K, int B, const std::vector<InstDesc>& desc) {
  int w_min = kMaxW;
  for (const InstDesc& d : desc) w_min = std::min(w_min, d.W);
  if (!(step_supported(K) && (B == 64 || B == 128 || B == 256) && K <= 2 * (w_min + 2) &&
        B * K <= 4096))
    return false;
  const TileLds L = tile_lds(desc, K, B);
  return 4 * iter_lds_words(L.pos, L.stage, L.gb, L.ngb, L.ppb, B) <= 65536;
}

// (4, 64) suits every batch: its LDS need stays far below 64 KiB.
sepso_tune default_tune(const std::vector<InstDesc>& desc) {
  for (int K : {8, 4})
    if (tune_ok(K, 128, desc)) return sepso_tune{K, 128};
  return sepso_tune{4, 64};
}

constexpr const char* kTuneRule =
    "tune: seg_per_thread in {4,8,12,16,24} and <= 2*(waypoints+2), block_threads in {64,128,256}, "
    "product <= 4096, fused-iteration LDS <= 64 KiB";

}  // namespace

namespace {

sepso_status hip_fail(sepso_batch* b, hipError_t e, const char* what) {
  if (b) b->broken = true;
  return fail(SEPSO_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(b, expr)                                  \
  do {                                                   \
    hipError_t _e = (expr);                              \
    if (_e != hipSuccess) return hip_fail(b, _e, #expr); \
  } while (0)

#define LAUNCHCHK(b, what)                             \
  do {                                                 \
    hipError_t _e = hipGetLastError();                 \
    if (_e != hipSuccess) return hip_fail(b, _e, what); \
  } while (0)

// One bucket holding every instance, with one tile shape.
void set_single(sepso_batch* b, const sepso_tune& t) {
  b->tune = t;
  b->buckets.assign(1, TileBucket{});
  b->buckets[0].tune = t;
  for (int i = 0; i < b->n; ++i) b->buckets[0].inst.push_back(i);
}

// Block geometry for the buckets' tiles: each block of the fused iteration
// takes ppb consecutive particles (tile_ppb) of one instance; fills the desc
// fields and, per bucket, its LDS sizing, wave groups and slice of the block
// -> (instance, first particle) table, heaviest blocks first (the dispatcher
// hands blocks out in order).
void plan_tiles(sepso_batch* b, std::vector<int2>* blk) {
  if (b->buckets.empty()) set_single(b, b->tune);
  blk->clear();
  for (TileBucket& bk : b->buckets) {
    const int K = bk.tune.seg_per_thread, B = bk.tune.block_threads;
    std::vector<InstDesc> sub;
    for (int i : bk.inst) sub.push_back(b->desc[i]);
    const int R = tile_rsplit(sub, K, B);
    std::vector<std::pair<double, int>> order;
    for (int i : bk.inst) {
      InstDesc& d = b->desc[i];
      d.ppb = tile_ppb(d.W, K, B, R);
      d.n_blocks = (d.G * d.N + d.ppb - 1) / d.ppb;
      order.push_back({(double)d.n_edges * d.ppb * (d.W + 2), i});
    }
    const TileLds L = tile_lds(sub, K, B);
    bk.pl = b->pl;
    bk.pl.rsplit = R;
    bk.pl.pos_floats = L.pos;
    bk.pl.stage_floats = L.stage;
    bk.pl.gb_floats = L.gb;
    bk.pl.ngb_max = L.ngb;
    bk.pl.ppb_max = L.ppb;
    std::stable_sort(order.begin(), order.end(), [](const std::pair<double, int>& a,
                                                    const std::pair<double, int>& c) {
      return a.first > c.first;
    });
    bk.first_block = (int)blk->size();
    for (auto& o : order) {
      const InstDesc& d = b->desc[o.second];
      for (int t = 0; t < d.n_blocks; ++t) blk->push_back(make_int2(o.second, t * d.ppb));
    }
    bk.n_blocks = (int)blk->size() - bk.first_block;
    bk.pl.blk_tiles = b->pl.blk_tiles + bk.first_block;
  }
  b->tile_blocks = (int)blk->size();
}

sepso_status upload_tiles(sepso_batch* b) {
  std::vector<int2> blk;
  plan_tiles(b, &blk);
  HIPCHK(b, hipMemcpyAsync(b->ws + b->lay.desc, b->desc.data(), sizeof(InstDesc) * b->n,
                           hipMemcpyHostToDevice, b->stream));
  HIPCHK(b, hipMemcpyAsync(b->ws + b->lay.blkt, blk.data(), sizeof(int2) * blk.size(),
                           hipMemcpyHostToDevice, b->stream));
  HIPCHK(b, hipStreamSynchronize(b->stream));
  b->tune_gen += 1;
  for (int m = 0; m < 2; ++m)
    if (b->graph[m]) {
      (void)hipGraphExecDestroy(b->graph[m]);  // retired; re-captured on next use
      b->graph[m] = nullptr;
    }
  return SEPSO_OK;
}

void destroy_batch(sepso_batch* b) {
  if (!b) return;
  for (int m = 0; m < 2; ++m)
    if (b->graph[m]) (void)hipGraphExecDestroy(b->graph[m]);
  // teardown is best effort: a failure here leaves nothing to recover
  for (hipStream_t x : b->bstreams) (void)hipStreamDestroy(x);
  for (hipEvent_t x : b->bevents) (void)hipEventDestroy(x);
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
  if (b->h_ctl) (void)hipHostFree(b->h_ctl);
  if (b->h_paths) (void)hipHostFree(b->h_paths);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

template <class T>
T* at(sepso_batch* b, size_t off) {
  return reinterpret_cast<T*>(b->ws + off);
}

sepso_status create_batch(const sepso_map* maps, const sepso_swarm* sw, int n, void* d_ws,
                          size_t ws_bytes, void* stream, const sepso_tune* tune, sepso_batch** out) {
  if (!out) return fail(SEPSO_E_ARG, "out is NULL");
  *out = nullptr;
  if (n < 1) return fail(SEPSO_E_ARG, "n_inst must be >= 1");
  if (!maps || !sw) return fail(SEPSO_E_ARG, "maps/swarms NULL");
  for (int i = 0; i < n; ++i) {
    sepso_status st = check_map(&maps[i], i);
    if (st != SEPSO_OK) return st;
    st = check_swarm(&sw[i], i);
    if (st != SEPSO_OK) return st;
  }
  if (!d_ws) return fail(SEPSO_E_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(d_ws) % 256) return fail(SEPSO_E_ARG, "workspace not 256-byte aligned");
  sepso_batch* b = new (std::nothrow) sepso_batch();
  if (!b) return fail(SEPSO_E_NOMEM, "host allocation failed");
  b->n = n;
  b->lay = plan_layout(maps, sw, n, &b->desc);
  b->tune = default_tune(b->desc);
  if (tune) {
    if (!tune_ok(tune->seg_per_thread, tune->block_threads, b->desc)) {
      delete b;
      return fail(SEPSO_E_ARG, "%s", kTuneRule);
    }
    b->tune = *tune;
  }
  set_single(b, b->tune);
  if (ws_bytes < b->lay.total) {
    const size_t need = b->lay.total;
    delete b;
    return fail(SEPSO_E_NOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  }
  b->ws = static_cast<char*>(d_ws);
  if (stream) {
    b->stream = static_cast<hipStream_t>(stream);
  } else {
    // graph capture needs a non-legacy stream; default priority
    hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete b;
      return fail(SEPSO_E_HIP, "hipStreamCreate: %s", hipGetErrorString(e));
    }
    b->own_stream = true;
  }
  const Layout& L = b->lay;
  Pools& pl = b->pl;
  pl.n_inst = n;
  pl.desc = at<InstDesc>(b, L.desc);
  pl.ctl = at<InstCtl>(b, L.ctl);
  pl.X = at<float>(b, L.X);
  pl.V = at<float>(b, L.V);
  pl.P = at<float>(b, L.P);
  pl.f = at<float>(b, L.f);
  pl.L = at<float>(b, L.L);
  pl.Pf = at<float>(b, L.Pf);
  pl.PL = at<float>(b, L.PL);
  pl.Q = at<int32_t>(b, L.Q);
  pl.PQ = at<int32_t>(b, L.PQ);
  pl.edges = at<EdgeRec>(b, L.edges);
  pl.cpolys = at<CPoly>(b, L.cpolys);
  pl.rects = at<float4>(b, L.rects);
  pl.rect_c = pl.rects + L.sumR;
  pl.pkind = at<int2>(b, L.pkind);
  pl.verts = at<float2>(b, L.verts);
  pl.poly_ptr = at<int32_t>(b, L.pptr);
  pl.poly_vel = at<float2>(b, L.pvel);
  pl.ends = at<float4>(b, L.ends);
  pl.end_vel = at<float4>(b, L.endv);
  pl.gbest_n = at<int32_t>(b, L.gbn);
  pl.gbest_f = at<float>(b, L.gbf);
  pl.hyper = at<float>(b, L.hyper);
  pl.outer_hyper = at<float>(b, L.ohyper);
  pl.ov = at<float>(b, L.ov);
  pl.op = at<float>(b, L.op);
  pl.opf = at<float>(b, L.opf);
  pl.gbest_pos = at<float>(b, L.gpos);
  pl.tbest_pos = at<float>(b, L.tpos);
  pl.prev_path = at<float>(b, L.prev);
  pl.proposal = at<float>(b, L.prop);
  pl.blk_tiles = at<int2>(b, L.blkt);
  pl.blk_init = at<int2>(b, L.blki);

  // host-side images of the static pools
  std::vector<float> verts(2 * L.sumE), pvel(2 * L.sumPoly, 0.f), ends(4 * n), endv(4 * n);
  std::vector<float> hyper(6 * L.sumG), ohyper(6 * L.sumG);
  std::vector<int32_t> pptr(L.sumPP);
  std::vector<int2> blki, pkind(std::max<int64_t>(1, L.sumPoly));
  b->n_vert.resize(n);
  b->path_off.resize(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    const InstDesc& d = b->desc[i];
    {
      std::vector<int2> kind;
      int nr = 0, ne = 0;
      classify_polys(maps[i], &kind, &nr, &ne, nullptr);
      for (int q = 0; q < d.n_polys; ++q) pkind[d.pvo + q] = kind[q];
      if (i == 0) b->h_kind = kind;
    }
    const sepso_map& m = maps[i];
    b->n_vert[i] = d.n_edges;
    for (int j = 0; j < 2 * d.n_edges; ++j) verts[2 * d.eo + j] = m.verts[j];
    for (int q = 0; q <= d.n_polys; ++q) pptr[d.plo + q] = d.n_polys ? m.poly_ptr[q] : 0;
    if (m.poly_vel)
      for (int q = 0; q < 2 * d.n_polys; ++q) pvel[2 * d.pvo + q] = m.poly_vel[q];
    ends[4 * i + 0] = m.start[0];
    ends[4 * i + 1] = m.start[1];
    ends[4 * i + 2] = m.target[0];
    ends[4 * i + 3] = m.target[1];
    for (int j = 0; j < 4; ++j) endv[4 * i + j] = m.endpoint_vel[j];
    for (int j = 0; j < 6 * d.G; ++j) {
      hyper[6 * d.go + j] = sw[i].hyper[j];
      ohyper[6 * d.go + j] = sw[i].hsef_hyper ? sw[i].hsef_hyper[j] : kHyper8[(j / 6) % 8][j % 6];
    }
    const int64_t PQ4 = (int64_t)d.G * d.N * ((2 * d.W + 3) / 4);  // coordinate quads
    for (int64_t q = 0; q < PQ4; q += 256) blki.push_back(make_int2(i, (int)q));
    b->path_off[i + 1] = b->path_off[i] + 2 * d.W;
  }
  b->h_pptr.assign(pptr.begin(), pptr.begin() + b->desc[0].n_polys + 1);
  b->h_hyper0 = hyper;
  std::vector<InstCtl> ctl(n);
  std::memset(ctl.data(), 0, sizeof(InstCtl) * n);
  for (int i = 0; i < n; ++i) ctl[i].tb_f = INFINITY;

  auto h2d = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
    if (!bytes) return hipSuccess;
    return hipMemcpyAsync(b->ws + off, src, bytes, hipMemcpyHostToDevice, b->stream);
  };
  hipError_t e = hipSuccess;
  const hipError_t errs[] = {
      h2d(L.ctl, ctl.data(), sizeof(InstCtl) * n),
      h2d(L.verts, verts.data(), 4 * verts.size()),
      h2d(L.pptr, pptr.data(), 4 * pptr.size()),
      h2d(L.pkind, pkind.data(), 8 * L.sumPoly),
      h2d(L.pvel, pvel.data(), 4 * pvel.size()),
      h2d(L.ends, ends.data(), 4 * ends.size()),
      h2d(L.endv, endv.data(), 4 * endv.size()),
      h2d(L.hyper, hyper.data(), 4 * hyper.size()),  // kept in b->h_hyper0 below
      h2d(L.ohyper, ohyper.data(), 4 * ohyper.size()),
      h2d(L.blki, blki.data(), sizeof(int2) * blki.size())};
  for (hipError_t x : errs)
    if (x != hipSuccess) e = x;
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_ctl, sizeof(InstCtl) * n, hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&b->h_paths, sizeof(float) * std::max<int64_t>(1, b->path_off[n]), hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreate(&b->ev0);
  if (e == hipSuccess) e = hipEventCreate(&b->ev1);
  if (e != hipSuccess) {
    sepso_status st = fail(SEPSO_E_HIP, "create: %s", hipGetErrorString(e));
    destroy_batch(b);
    return st;
  }
  sepso_status st = upload_tiles(b);
  if (st != SEPSO_OK) {
    destroy_batch(b);
    return st;
  }
  launch_geom(pl, n, 0, b->stream);
  launch_init(pl, (int)blki.size(), 0, 0, b->stream);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) {
    st = fail(SEPSO_E_HIP, "create launch: %s", hipGetErrorString(e));
    destroy_batch(b);
    return st;
  }
  *out = b;
  return SEPSO_OK;
}

sepso_status usable(sepso_batch* b) {
  if (!b) return fail(SEPSO_E_ARG, "handle is NULL");
  if (b->broken) return fail(SEPSO_E_STATE, "handle is unusable after an earlier HIP error");
  return SEPSO_OK;
}

int init_blocks(sepso_batch* b) { return (int)b->lay.initBlocks; }

// One iteration of every instance: each bucket's tile kernel, then the
// per-instance reduce.  With fork (graph capture) the buckets after the
// first go out on side streams that branch off before them and join before
// the reduce, so that their launches can run side by side; otherwise they
// follow one another on s.  Events, when given, bracket the tile kernels.
hipError_t enqueue_iteration(sepso_batch* b, int flags, bool fork, hipEvent_t before = nullptr,
                             hipEvent_t after = nullptr) {
  hipStream_t s = b->stream;
  hipError_t e = hipSuccess;
  if (before) e = hipEventRecord(before, s);
  const int nb = (int)b->buckets.size();
  const bool par = fork && nb > 1 && (int)b->bstreams.size() >= nb - 1 && (int)b->bevents.size() >= nb;
  if (par && e == hipSuccess) e = hipEventRecord(b->bevents[0], s);
  for (int j = 0; j < nb && e == hipSuccess; ++j) {
    const TileBucket& bk = b->buckets[j];
    hipStream_t sj = par && j > 0 ? b->bstreams[j - 1] : s;
    if (sj != s) e = hipStreamWaitEvent(sj, b->bevents[0], 0);
    if (e == hipSuccess &&
        !launch_tiles(bk.pl, bk.tune.seg_per_thread, bk.n_blocks, bk.tune.block_threads, flags, sj))
      e = hipErrorInvalidValue;
    if (e == hipSuccess && sj != s) e = hipEventRecord(b->bevents[j], sj);
    if (e == hipSuccess && sj != s) e = hipStreamWaitEvent(s, b->bevents[j], 0);
  }
  if (after && e == hipSuccess) e = hipEventRecord(after, s);
  if (e == hipSuccess) launch_reduce(b->pl, flags, s);
  return e;
}

// Enqueue one whole frame of every instance; the first error of the
// enqueued work (launch errors included).
hipError_t enqueue_frame(sepso_batch* b, bool move) {
  if (move) launch_geom(b->pl, b->n, 1, b->stream);
  if (b->lin) lin_enqueue_proposals(b->lin, b);
  launch_init(b->pl, init_blocks(b), -1, 1, b->stream);
  int tmax = 0;
  for (auto& d : b->desc) tmax = std::max(tmax, d.T);
  hipError_t e = hipSuccess;
  for (int k = 0; k < tmax && e == hipSuccess; ++k)
    e = enqueue_iteration(b, STEP_FIT | STEP_FRAME, true);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->h_ctl, b->pl.ctl, sizeof(InstCtl) * b->n, hipMemcpyDeviceToHost,
                       b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->h_paths, b->pl.prev_path, sizeof(float) * b->path_off[b->n],
                       hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipGetLastError();
  return e;
}

sepso_status run_frame(sepso_batch* b, bool move, float* ms) {
  const int m = move ? 1 : 0;
  if (!b->graph[m]) {
    hipGraph_t g = nullptr;
    HIPCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    const hipError_t eq = enqueue_frame(b, move);
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (eq != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return hip_fail(b, eq, "frame capture");
    }
    if (e != hipSuccess) return hip_fail(b, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b->graph[m], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);  // the instantiated graph keeps what it needs
    if (e != hipSuccess) return hip_fail(b, e, "hipGraphInstantiate");
  }
  HIPCHK(b, hipEventRecord(b->ev0, b->stream));
  HIPCHK(b, hipGraphLaunch(b->graph[m], b->stream));
  HIPCHK(b, hipEventRecord(b->ev1, b->stream));
  HIPCHK(b, hipEventSynchronize(b->ev1));
  if (ms) HIPCHK(b, hipEventElapsedTime(ms, b->ev0, b->ev1));
  b->frames_done += 1;
  return SEPSO_OK;
}

void fill_result(const InstCtl& c, float ms, sepso_frame_result* r) {
  r->cost = c.res_cost;
  r->length = c.res_len;
  r->crossings = c.res_q;
  r->iters = c.res_iters;
  r->truncated = c.res_trunc;
  r->used_learned = c.use_learned;
  r->device_ms = ms;
}

sepso_status get_state_inst(sepso_batch* b, int i, sepso_state* st) {
  const InstDesc& d = b->desc[i];
  const size_t PD = (size_t)d.G * d.N * 2 * d.W, P = (size_t)d.G * d.N;
  auto d2h = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    if (!dst || !bytes) return hipSuccess;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, b->stream);
  };
  HIPCHK(b, d2h(st->X, b->pl.X + d.xo, 4 * PD));
  HIPCHK(b, d2h(st->V, b->pl.V + d.xo, 4 * PD));
  HIPCHK(b, d2h(st->P, b->pl.P + d.xo, 4 * PD));
  HIPCHK(b, d2h(st->f, b->pl.f + d.po, 4 * P));
  HIPCHK(b, d2h(st->L, b->pl.L + d.po, 4 * P));
  HIPCHK(b, d2h(st->Pf, b->pl.Pf + d.po, 4 * P));
  HIPCHK(b, d2h(st->PL, b->pl.PL + d.po, 4 * P));
  HIPCHK(b, d2h(st->Q, b->pl.Q + d.po, 4 * P));
  HIPCHK(b, d2h(st->PQ, b->pl.PQ + d.po, 4 * P));
  HIPCHK(b, d2h(st->gbest_n, b->pl.gbest_n + d.go, 4 * d.G));
  HIPCHK(b, d2h(st->gbest_f, b->pl.gbest_f + d.go, 4 * d.G));
  HIPCHK(b, d2h(st->hyper, b->pl.hyper + 6 * d.go, 24 * d.G));
  HIPCHK(b, d2h(b->h_ctl + i, b->pl.ctl + i, sizeof(InstCtl)));
  HIPCHK(b, hipStreamSynchronize(b->stream));
  const InstCtl& c = b->h_ctl[i];
  st->tbest_g = c.tb_g;
  st->tbest_n = c.tb_n;
  st->tbest_f = c.tb_f;
  st->k = c.k;
  st->ctr = c.ctr;
  st->frame = c.frame;
  return SEPSO_OK;
}

}  // namespace

// ============================== C ABI =======================================
extern "C" {

const char* sepso_last_error(void) { return g_err.c_str(); }
const char* sepso_version(void) { return "libsepso 0.1 (gfx950)"; }

sepso_status sepso_philox(uint32_t first, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t key,
                          int64_t n, uint32_t* d_out, void* stream) {
  if (n < 0) return fail(SEPSO_E_ARG, "n must be >= 0");
  if (n > ((int64_t)1 << 32)) return fail(SEPSO_E_ARG, "n exceeds the 32-bit counter word");
  if (n > 0 && !d_out) return fail(SEPSO_E_ARG, "out is NULL");
  if (reinterpret_cast<uintptr_t>(d_out) % 16) return fail(SEPSO_E_ARG, "out not 16-byte aligned");
  if (n == 0) return SEPSO_OK;
  launch_philox(first, c1, c2, c3, key, n, d_out, static_cast<hipStream_t>(stream));
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(SEPSO_E_HIP, "philox launch: %s", hipGetErrorString(e));
  return SEPSO_OK;
}

sepso_status sepso_batch_workspace_bytes(const sepso_map* maps, const sepso_swarm* swarms,
                                         int32_t n_inst, size_t* bytes) {
  if (!bytes) return fail(SEPSO_E_ARG, "bytes is NULL");
  if (n_inst < 1 || !maps || !swarms) return fail(SEPSO_E_ARG, "need n_inst >= 1 maps and swarms");
  for (int i = 0; i < n_inst; ++i) {
    sepso_status st = check_map(&maps[i], i);
    if (st != SEPSO_OK) return st;
    st = check_swarm(&swarms[i], i);
    if (st != SEPSO_OK) return st;
  }
  *bytes = plan_layout(maps, swarms, n_inst, nullptr).total;
  return SEPSO_OK;
}

sepso_status sepso_workspace_bytes(const sepso_map* map, const sepso_swarm* swarm, size_t* bytes) {
  return sepso_batch_workspace_bytes(map, swarm, 1, bytes);
}

sepso_status sepso_batch_create(const sepso_map* maps, const sepso_swarm* swarms, int32_t n_inst,
                                void* d_ws, size_t ws_bytes, void* stream, const sepso_tune* tune,
                                sepso_batch** out) {
  return create_batch(maps, swarms, n_inst, d_ws, ws_bytes, stream, tune, out);
}

sepso_status sepso_create(const sepso_map* map, const sepso_swarm* swarm, void* d_ws,
                          size_t ws_bytes, void* stream, sepso_ctx** out) {
  if (!out) return fail(SEPSO_E_ARG, "out is NULL");
  *out = nullptr;
  sepso_batch* b = nullptr;
  sepso_status st = create_batch(map, swarm, 1, d_ws, ws_bytes, stream, nullptr, &b);
  if (st != SEPSO_OK) return st;
  sepso_ctx* c = new (std::nothrow) sepso_ctx{b};
  if (!c) {
    destroy_batch(b);
    return fail(SEPSO_E_NOMEM, "host allocation failed");
  }
  *out = c;
  return SEPSO_OK;
}

sepso_status sepso_destroy(sepso_ctx* ctx) {
  if (!ctx) return fail(SEPSO_E_ARG, "ctx is NULL");
  destroy_batch(ctx->b);
  delete ctx;
  return SEPSO_OK;
}

sepso_status sepso_batch_destroy(sepso_batch* b) {
  if (!b) return fail(SEPSO_E_ARG, "batch is NULL");
  destroy_batch(b);
  return SEPSO_OK;
}

static sepso_status step_batch(sepso_batch* b, int32_t n) {
  sepso_status st = usable(b);
  if (st != SEPSO_OK) return st;
  if (n < 0) return fail(SEPSO_E_ARG, "n must be >= 0");
  hipError_t e = hipSuccess;
  for (int k = 0; k < n && e == hipSuccess; ++k) e = enqueue_iteration(b, STEP_FIT, false);
  if (n > 0 && e == hipSuccess) e = enqueue_iteration(b, 0, false);
  if (e != hipSuccess) return hip_fail(b, e, "step launch");
  LAUNCHCHK(b, "step launch");
  return SEPSO_OK;
}

sepso_status sepso_step(sepso_ctx* ctx, int32_t n) {
  if (!ctx) return fail(SEPSO_E_ARG, "ctx is NULL");
  return step_batch(ctx->b, n);
}

sepso_status sepso_step_frame(sepso_ctx* ctx, int32_t n) {
  if (!ctx) return fail(SEPSO_E_ARG, "ctx is NULL");
  sepso_batch* b = ctx->b;
  sepso_status st = usable(b);
  if (st != SEPSO_OK) return st;
  if (n < 0) return fail(SEPSO_E_ARG, "n must be >= 0");
  hipError_t e = hipSuccess;
  for (int k = 0; k < n && e == hipSuccess; ++k) e = enqueue_iteration(b, STEP_FIT | STEP_FRAME, false);
  if (n > 0 && e == hipSuccess)  // the pending update (nothing once the frame has ended)
    e = enqueue_iteration(b, STEP_FRAME, false);
  if (e != hipSuccess) return hip_fail(b, e, "step launch");
  LAUNCHCHK(b, "step launch");
  return SEPSO_OK;
}

sepso_status sepso_get_outer(sepso_ctx* ctx, sepso_outer* o) {
  if (!ctx || !o) return fail(SEPSO_E_ARG, "ctx/outer is NULL");
  sepso_batch* b = ctx->b;
  sepso_status s = usable(b);
  if (s != SEPSO_OK) return s;
  const InstDesc& d = b->desc[0];
  auto d2h = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    if (!dst) return hipSuccess;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, b->stream);
  };
  HIPCHK(b, d2h(o->ov, b->pl.ov + 3 * d.go, 12 * (size_t)d.G));
  HIPCHK(b, d2h(o->op, b->pl.op + 3 * d.go, 12 * (size_t)d.G));
  HIPCHK(b, d2h(o->opf, b->pl.opf + d.go, 4 * (size_t)d.G));
  HIPCHK(b, hipMemcpyAsync(b->h_ctl, b->pl.ctl, sizeof(InstCtl), hipMemcpyDeviceToHost, b->stream));
  HIPCHK(b, hipStreamSynchronize(b->stream));
  o->otb = b->h_ctl[0].otb;
  o->epoch_in_frame = b->h_ctl[0].epoch_in_frame;
  o->epoch_ctr = b->h_ctl[0].epoch_ctr;
  return SEPSO_OK;
}

sepso_status sepso_set_outer(sepso_ctx* ctx, const sepso_outer* o) {
  if (!ctx || !o) return fail(SEPSO_E_ARG, "ctx/outer is NULL");
  sepso_batch* b = ctx->b;
  sepso_status s = usable(b);
  if (s != SEPSO_OK) return s;
  const InstDesc& d = b->desc[0];
  if (o->otb < 0 || o->otb >= d.G || o->epoch_in_frame < 0)
    return fail(SEPSO_E_ARG, "set_outer: otb or epoch_in_frame out of range");
  auto h2d = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    if (!src) return hipSuccess;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, b->stream);
  };
  HIPCHK(b, h2d(b->pl.ov + 3 * d.go, o->ov, 12 * (size_t)d.G));
  HIPCHK(b, h2d(b->pl.op + 3 * d.go, o->op, 12 * (size_t)d.G));
  HIPCHK(b, h2d(b->pl.opf + d.go, o->opf, 4 * (size_t)d.G));
  HIPCHK(b, hipMemcpyAsync(b->h_ctl, b->pl.ctl, sizeof(InstCtl), hipMemcpyDeviceToHost, b->stream));
  HIPCHK(b, hipStreamSynchronize(b->stream));
  b->h_ctl[0].otb = o->otb;
  b->h_ctl[0].epoch_in_frame = o->epoch_in_frame;
  b->h_ctl[0].epoch_ctr = o->epoch_ctr;
  HIPCHK(b, hipMemcpyAsync(b->pl.ctl, b->h_ctl, sizeof(InstCtl), hipMemcpyHostToDevice, b->stream));
  HIPCHK(b, hipStreamSynchronize(b->stream));
  return SEPSO_OK;
}

sepso_status sepso_reinit(sepso_ctx* ctx, int32_t frame, int32_t use_prev) {
  if (!ctx) return fail(SEPSO_E_ARG, "ctx is NULL");
  sepso_batch* b = ctx->b;
  sepso_status st = usable(b);
  if (st != SEPSO_OK) return st;
  if (frame < 0) return fail(SEPSO_E_ARG, "frame must be >= 0");
  launch_init(b->pl, init_blocks(b), frame, use_prev ? 1 : 0, b->stream);
  LAUNCHCHK(b, "init launch");
  return SEPSO_OK;
}

sepso_status sepso_plan_frame(sepso_ctx* ctx, const sepso_map* next, sepso_frame_result* out,
                              float* out_path) {
  if (!ctx) return fail(SEPSO_E_ARG, "ctx is NULL");
  sepso_batch* b = ctx->b;
  sepso_status st = usable(b);
  if (st != SEPSO_OK) return st;
  if (!out) return fail(SEPSO_E_ARG, "out is NULL");
  const InstDesc& d = b->desc[0];
  bool move = b->frames_done > 0;
  if (next) {
    st = check_map(next, 0);
    if (st != SEPSO_OK) return st;
    if (next->n_polys != d.n_polys)
      return fail(SEPSO_E_ARG, "next map must keep the polygon structure (n_polys)");
    for (int q = 0; q <= d.n_polys && d.n_polys; ++q)
      if (next->poly_ptr[q] != b->h_pptr[q]) return fail(SEPSO_E_ARG, "next map: poly_ptr differs");
    {
      std::vector<int2> kind;
      int nr = 0, ne = 0;
      classify_polys(*next, &kind, &nr, &ne, nullptr);
      for (int q = 0; q < d.n_polys; ++q)
        if (kind[q].x != b->h_kind[q].x)
          return fail(SEPSO_E_ARG, "next map: polygon %d changed kind (rectangle, convex, general)", q);
    }
    std::vector<float> e4 = {next->start[0], next->start[1], next->target[0], next->target[1]};
    HIPCHK(b, hipMemcpyAsync(b->pl.verts + d.eo, next->verts, 8 * (size_t)d.n_edges,
                             hipMemcpyHostToDevice, b->stream));
    HIPCHK(b, hipMemcpyAsync(b->pl.ends, e4.data(), 16, hipMemcpyHostToDevice, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    launch_geom(b->pl, 1, 0, b->stream);
    LAUNCHCHK(b, "geometry launch");
    move = false;
  }
  float ms = 0.f;
  st = run_frame(b, move, &ms);
  if (st != SEPSO_OK) return st;
  fill_result(b->h_ctl[0], ms, out);
  if (out_path) std::memcpy(out_path, b->h_paths, sizeof(float) * 2 * d.W);
  return SEPSO_OK;
}

sepso_status sepso_get_state(sepso_ctx* ctx, sepso_state* st) {
  if (!ctx || !st) return fail(SEPSO_E_ARG, "ctx/state is NULL");
  sepso_status s = usable(ctx->b);
  if (s != SEPSO_OK) return s;
  return get_state_inst(ctx->b, 0, st);
}

sepso_status sepso_batch_get_state(sepso_batch* b, int32_t i, sepso_state* st) {
  sepso_status s = usable(b);
  if (s != SEPSO_OK) return s;
  if (!st || i < 0 || i >= b->n) return fail(SEPSO_E_ARG, "bad instance index or state");
  return get_state_inst(b, i, st);
}

sepso_status sepso_set_state(sepso_ctx* ctx, const sepso_state* st) {
  if (!ctx || !st) return fail(SEPSO_E_ARG, "ctx/state is NULL");
  sepso_batch* b = ctx->b;
  sepso_status s = usable(b);
  if (s != SEPSO_OK) return s;
  const InstDesc& d = b->desc[0];
  const size_t PD = (size_t)d.G * d.N * 2 * d.W, P = (size_t)d.G * d.N;
  if (st->tbest_g < 0 || st->tbest_g >= d.G || st->tbest_n < 0 || st->tbest_n >= d.N || st->k < 0)
    return fail(SEPSO_E_ARG, "set_state: scalar fields out of range");
  if (st->X)
    for (size_t j = 0; j < PD; ++j) {
      const float lim = (j % (2 * d.W)) < (size_t)d.W ? d.width : d.height;
      if (!(st->X[j] >= 0.f && st->X[j] <= lim))
        return fail(SEPSO_E_ARG, "set_state: X[%zu] outside the map", j);
    }
  if (st->hyper)
    for (int j = 0; j < 6 * d.G; ++j)
      if (!finite(st->hyper[j]) || (j % 6 == 5 && st->hyper[j] < 0.f))
        return fail(SEPSO_E_ARG, "set_state: hyper not finite or V_limit < 0");
  auto h2d = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    if (!src || !bytes) return hipSuccess;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, b->stream);
  };
  HIPCHK(b, h2d(b->pl.X + d.xo, st->X, 4 * PD));
  HIPCHK(b, h2d(b->pl.V + d.xo, st->V, 4 * PD));
  HIPCHK(b, h2d(b->pl.P + d.xo, st->P, 4 * PD));
  HIPCHK(b, h2d(b->pl.f + d.po, st->f, 4 * P));
  HIPCHK(b, h2d(b->pl.L + d.po, st->L, 4 * P));
  HIPCHK(b, h2d(b->pl.Pf + d.po, st->Pf, 4 * P));
  HIPCHK(b, h2d(b->pl.PL + d.po, st->PL, 4 * P));
  HIPCHK(b, h2d(b->pl.Q + d.po, st->Q, 4 * P));
  HIPCHK(b, h2d(b->pl.PQ + d.po, st->PQ, 4 * P));
  HIPCHK(b, h2d(b->pl.gbest_n + d.go, st->gbest_n, 4 * d.G));
  HIPCHK(b, h2d(b->pl.gbest_f + d.go, st->gbest_f, 4 * d.G));
  HIPCHK(b, h2d(b->pl.hyper + 6 * d.go, st->hyper, 24 * d.G));
  HIPCHK(b, hipMemcpyAsync(b->h_ctl, b->pl.ctl, sizeof(InstCtl), hipMemcpyDeviceToHost, b->stream));
  HIPCHK(b, hipStreamSynchronize(b->stream));
  InstCtl c = b->h_ctl[0];
  c.k = st->k;
  c.ctr = st->ctr;
  c.frame = st->frame;
  c.tb_g = st->tbest_g;
  c.tb_n = st->tbest_n;
  c.tb_f = st->tbest_f;
  c.pending = 0;
  c.done = 0;
  c.arrive = 0;
  b->h_ctl[0] = c;
  HIPCHK(b, hipMemcpyAsync(b->pl.ctl, b->h_ctl, sizeof(InstCtl), hipMemcpyHostToDevice, b->stream));
  HIPCHK(b, hipStreamSynchronize(b->stream));
  return SEPSO_OK;
}

sepso_status sepso_get_geometry(sepso_ctx* ctx, float* verts, float* endpoints) {
  if (!ctx) return fail(SEPSO_E_ARG, "ctx is NULL");
  sepso_batch* b = ctx->b;
  sepso_status s = usable(b);
  if (s != SEPSO_OK) return s;
  const InstDesc& d = b->desc[0];
  if (verts && d.n_edges)
    HIPCHK(b, hipMemcpyAsync(verts, b->pl.verts + d.eo, 8 * (size_t)d.n_edges, hipMemcpyDeviceToHost, b->stream));
  if (endpoints)
    HIPCHK(b, hipMemcpyAsync(endpoints, b->pl.ends, 16, hipMemcpyDeviceToHost, b->stream));
  HIPCHK(b, hipStreamSynchronize(b->stream));
  return SEPSO_OK;
}

static sepso_status profile_batch(sepso_batch* b, int32_t n, float* avg_ms) {
  sepso_status s = usable(b);
  if (s != SEPSO_OK) return s;
  if (n < 1 || !avg_ms) return fail(SEPSO_E_ARG, "n >= 1 and avg_ms required");
  // events bracket each fused-iteration launch alone (not the reduce after it)
  std::vector<hipEvent_t> ev(2 * (size_t)n, nullptr);
  hipError_t e = hipSuccess;
  for (size_t q = 0; q < ev.size() && e == hipSuccess; ++q) e = hipEventCreate(&ev[q]);
  float total = 0.f;
  if (e == hipSuccess) {
    for (int k = 0; k < n && e == hipSuccess; ++k)
      e = enqueue_iteration(b, STEP_FIT, false, ev[2 * k], ev[2 * k + 1]);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = enqueue_iteration(b, 0, false);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    for (int k = 0; k < n && e == hipSuccess; ++k) {
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]);
      total += ms;
    }
  }
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  if (e != hipSuccess) return hip_fail(b, e, "profile");
  *avg_ms = total / (float)n;
  return SEPSO_OK;
}

sepso_status sepso_profile_step(sepso_ctx* ctx, int32_t n, float* avg_ms) {
  if (!ctx) return fail(SEPSO_E_ARG, "ctx is NULL");
  return profile_batch(ctx->b, n, avg_ms);
}

sepso_status sepso_batch_profile_step(sepso_batch* b, int32_t n, float* avg_ms) {
  return profile_batch(b, n, avg_ms);
}

sepso_status sepso_batch_path_offsets(sepso_batch* b, int64_t* offsets) {
  if (!b || !offsets) return fail(SEPSO_E_ARG, "batch/offsets NULL");
  std::memcpy(offsets, b->path_off.data(), sizeof(int64_t) * (b->n + 1));
  return SEPSO_OK;
}

sepso_status sepso_batch_plan(sepso_batch* b, int32_t n_frames, sepso_frame_result* out,
                              float* out_paths) {
  sepso_status st = usable(b);
  if (st != SEPSO_OK) return st;
  if (n_frames < 1 || !out) return fail(SEPSO_E_ARG, "n_frames >= 1 and out required");
  for (int f = 0; f < n_frames; ++f) {
    float ms = 0.f;
    st = run_frame(b, b->frames_done > 0, &ms);
    if (st != SEPSO_OK) return st;
    for (int i = 0; i < b->n; ++i) fill_result(b->h_ctl[i], 0.f, &out[(size_t)f * b->n + i]);
  }
  if (out_paths) std::memcpy(out_paths, b->h_paths, sizeof(float) * b->path_off[b->n]);
  return SEPSO_OK;
}

sepso_status sepso_batch_history(sepso_batch* b, float* out) {
  if (!b || !out) return fail(SEPSO_E_ARG, "batch/out NULL");
  for (int i = 0; i < b->n; ++i) std::memcpy(out + (size_t)i * kHist, b->h_ctl[i].hist, 4 * kHist);
  return SEPSO_OK;
}

sepso_status sepso_batch_work(sepso_batch* b, double* tests, double* elems) {
  if (!b) return fail(SEPSO_E_ARG, "batch is NULL");
  double t = 0, e = 0;
  for (auto& d : b->desc) {
    t += (double)d.G * d.N * (d.W + 1) * d.n_edges;
    e += (double)d.G * d.N * 2 * d.W;
  }
  if (tests) *tests = t;
  if (elems) *elems = e;
  return SEPSO_OK;
}

namespace {

// Back to the state of a new batch: control blocks as created (random-stream
// counters, frame index, previous plan and learned-start flags zero), the
// hyper-parameters as created (the online outer step moves them during a
// frame), then the frame-0 initial swarm.  Synchronous.
sepso_status restart(sepso_batch* b) {
  std::vector<InstCtl> ctl(b->n);
  std::memset(ctl.data(), 0, sizeof(InstCtl) * b->n);
  for (InstCtl& c : ctl) c.tb_f = INFINITY;
  HIPCHK(b, hipMemcpyAsync(b->pl.ctl, ctl.data(), sizeof(InstCtl) * b->n, hipMemcpyHostToDevice,
                           b->stream));
  HIPCHK(b, hipMemcpyAsync(b->pl.hyper, b->h_hyper0.data(), sizeof(float) * b->h_hyper0.size(),
                           hipMemcpyHostToDevice, b->stream));
  launch_init(b->pl, init_blocks(b), 0, 0, b->stream);
  LAUNCHCHK(b, "init launch");
  HIPCHK(b, hipStreamSynchronize(b->stream));
  b->frames_done = 0;
  return SEPSO_OK;
}

}  // namespace

sepso_status sepso_autotune(sepso_batch* b, sepso_tune* best) {
  sepso_status st = usable(b);
  if (st != SEPSO_OK) return st;
  const int Ks[] = {4, 8, 12, 16, 24};
  const int Bs[] = {64, 128, 256};
  sepso_tune win = b->tune;
  float win_ms = INFINITY;
  for (int K : Ks)
    for (int B : Bs) {
      if (!tune_ok(K, B, b->desc)) continue;
      set_single(b, sepso_tune{K, B});
      st = upload_tiles(b);
      if (st != SEPSO_OK) return st;
      float ms = 0.f;
      st = profile_batch(b, 1, &ms);  // warm-up
      if (st != SEPSO_OK) return st;
      st = profile_batch(b, 3, &ms);
      if (st != SEPSO_OK) return st;
      if (ms < win_ms) {
        win_ms = ms;
        win = b->tune;
      }
    }
  set_single(b, win);
  st = upload_tiles(b);
  if (st == SEPSO_OK) st = restart(b);
  if (st != SEPSO_OK) return st;
  if (best) *best = win;
  return SEPSO_OK;
}

namespace {

// Key of a batch for the tune cache: FNV-1a over the device architecture name
// and the shape fields of every instance that decide the tile's cost.
// Fingerprint of the device-code sources this library was built from
// (passed in by the build; 0 for a build that does not pass it).
#ifndef SEPSO_KERNELS_ID
#define SEPSO_KERNELS_ID 0ull
#endif

uint64_t tune_key(const sepso_batch* b) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void* p, size_t n) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
      h ^= c[i];
      h *= 1099511628211ull;
    }
  };
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    mix(prop.gcnArchName, strnlen(prop.gcnArchName, sizeof(prop.gcnArchName)));
  // a build of other kernel sources may rank the tiles differently
  const uint64_t src = SEPSO_KERNELS_ID;
  mix(&src, sizeof(src));
  mix(&b->n, sizeof(b->n));
  for (const InstDesc& d : b->desc) {
    const int32_t f[6] = {d.G, d.N, d.W, d.n_rects, d.n_cpolys, d.n_gedges};
    mix(f, sizeof(f));
  }
  return h;
}

}  // namespace

sepso_status sepso_autotune_cached(sepso_batch* b, const char* cache_path, sepso_tune* best) {
  sepso_status st = usable(b);
  if (st != SEPSO_OK) return st;
  if (!cache_path) return fail(SEPSO_E_ARG, "cache_path is NULL");
  const uint64_t key = tune_key(b);
  if (FILE* f = fopen(cache_path, "r")) {
    char line[256];
    bool hit = false;
    sepso_tune t{};
    while (!hit && fgets(line, sizeof line, f)) {
      unsigned long long k = 0;
      int K = 0, B = 0;
      if (sscanf(line, "%llx %d %d", &k, &K, &B) == 3 && k == key && tune_ok(K, B, b->desc)) {
        t = sepso_tune{K, B};
        hit = true;
      }
    }
    const bool bad = ferror(f) != 0;
    fclose(f);
    if (bad) return fail(SEPSO_E_ARG, "tune cache %s: read error", cache_path);
    if (hit) {
      set_single(b, t);
      st = upload_tiles(b);
      if (st == SEPSO_OK) st = restart(b);
      if (st != SEPSO_OK) return st;
      if (best) *best = t;
      return SEPSO_OK;
    }
  }
  sepso_tune win{};
  st = sepso_autotune(b, &win);
  if (st != SEPSO_OK) return st;
  FILE* f = fopen(cache_path, "a");
  if (!f) return fail(SEPSO_E_ARG, "tune cache %s: cannot open for writing", cache_path);
  const bool ok = fprintf(f, "%016llx %d %d\n", (unsigned long long)key, win.seg_per_thread,
                          win.block_threads) > 0;
  if (fclose(f) != 0 || !ok) return fail(SEPSO_E_ARG, "tune cache %s: write failed", cache_path);
  if (best) *best = win;
  return SEPSO_OK;
}

sepso_status sepso_batch_set_tune(sepso_batch* b, const sepso_tune* tune) {
  if (!b || !tune) return fail(SEPSO_E_ARG, "batch/tune NULL");
  sepso_status st = usable(b);
  if (st != SEPSO_OK) return st;
  if (!tune_ok(tune->seg_per_thread, tune->block_threads, b->desc))
    return fail(SEPSO_E_ARG, "%s", kTuneRule);
  set_single(b, *tune);
  return upload_tiles(b);
}

}  // extern "C"

namespace {

constexpr int kMaxBuckets = 8;

// Side streams (default priority) and fork / join events for the buckets.
sepso_status ensure_bucket_streams(sepso_batch* b) {
  const int nb = (int)b->buckets.size();
  while ((int)b->bstreams.size() < nb - 1) {
    hipStream_t x = nullptr;
    HIPCHK(b, hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
    b->bstreams.push_back(x);
  }
  while ((int)b->bevents.size() < nb) {
    hipEvent_t x = nullptr;
    HIPCHK(b, hipEventCreateWithFlags(&x, hipEventDisableTiming));
    b->bevents.push_back(x);
  }
  return SEPSO_OK;
}

// Mean device time of bucket j's tile kernel alone over n launches (events
// around it; each launch is followed by the reduce of every instance).
sepso_status profile_bucket(sepso_batch* b, int j, int n, float* avg_ms) {
  const TileBucket& bk = b->buckets[j];
  std::vector<hipEvent_t> ev(2 * (size_t)n, nullptr);
  hipError_t e = hipSuccess;
  for (size_t q = 0; q < ev.size() && e == hipSuccess; ++q) e = hipEventCreate(&ev[q]);
  float total = 0.f;
  for (int k = 0; k < n && e == hipSuccess; ++k) {
    e = hipEventRecord(ev[2 * k], b->stream);
    if (e == hipSuccess && !launch_tiles(bk.pl, bk.tune.seg_per_thread, bk.n_blocks,
                                         bk.tune.block_threads, STEP_FIT, b->stream))
      e = hipErrorInvalidValue;
    if (e == hipSuccess) e = hipEventRecord(ev[2 * k + 1], b->stream);
    if (e == hipSuccess) launch_reduce(b->pl, STEP_FIT, b->stream);
  }
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  for (int k = 0; k < n && e == hipSuccess; ++k) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]);
    total += ms;
  }
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  if (e != hipSuccess) return hip_fail(b, e, "profile bucket");
  *avg_ms = total / (float)n;
  return SEPSO_OK;
}

// Tune-cache key of one bucket: as the batch key, over the bucket's instances.
uint64_t bucket_key(const sepso_batch* b, const TileBucket& bk) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void* p, size_t n) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
      h ^= c[i];
      h *= 1099511628211ull;
    }
  };
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    mix(prop.gcnArchName, strnlen(prop.gcnArchName, sizeof(prop.gcnArchName)));
  const uint64_t src = SEPSO_KERNELS_ID;
  mix(&src, sizeof(src));
  const char tag[] = "bucket";
  mix(tag, sizeof(tag));
  const int32_t n = (int32_t)bk.inst.size();
  mix(&n, sizeof(n));
  for (int i : bk.inst) {
    const InstDesc& d = b->desc[i];
    const int32_t f[6] = {d.G, d.N, d.W, d.n_rects, d.n_cpolys, d.n_gedges};
    mix(f, sizeof(f));
  }
  return h;
}

std::vector<InstDesc> bucket_desc(const sepso_batch* b, const std::vector<int>& inst) {
  std::vector<InstDesc> sub;
  for (int i : inst) sub.push_back(b->desc[i]);
  return sub;
}

// Instances split by waypoint count (the tile's chunk fit) into at most
// max_b buckets of about equal size, equal counts kept together.
std::vector<std::vector<int>> split_by_waypoints(const sepso_batch* b, int max_b) {
  std::vector<int> idx(b->n);
  for (int i = 0; i < b->n; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return b->desc[x].W < b->desc[y].W; });
  std::vector<std::vector<int>> out(1);
  const int target = (b->n + max_b - 1) / max_b;
  for (size_t k = 0; k < idx.size(); ++k) {
    if (!out.back().empty() && (int)out.back().size() >= target && (int)out.size() < max_b &&
        b->desc[idx[k]].W != b->desc[idx[k - 1]].W)
      out.emplace_back();
    out.back().push_back(idx[k]);
  }
  for (auto& v : out) std::sort(v.begin(), v.end());
  return out;
}

void report_tiles(const sepso_batch* b, sepso_tune* tiles, int32_t* bucket_of, int32_t* n_buckets) {
  for (size_t j = 0; j < b->buckets.size(); ++j) {
    if (tiles) tiles[j] = b->buckets[j].tune;
    if (bucket_of)
      for (int i : b->buckets[j].inst) bucket_of[i] = (int32_t)j;
  }
  if (n_buckets) *n_buckets = (int32_t)b->buckets.size();
}

}  // namespace

extern "C" {

sepso_status sepso_batch_set_tiles(sepso_batch* b, int32_t n_buckets, const int32_t* bucket_of,
                                   const sepso_tune* tiles) {
  sepso_status st = usable(b);
  if (st != SEPSO_OK) return st;
  if (n_buckets < 1 || n_buckets > kMaxBuckets || !bucket_of || !tiles)
    return fail(SEPSO_E_ARG, "set_tiles: 1 <= n_buckets <= %d, bucket_of and tiles required", kMaxBuckets);
  std::vector<TileBucket> bks(n_buckets);
  for (int i = 0; i < b->n; ++i) {
    if (bucket_of[i] < 0 || bucket_of[i] >= n_buckets)
      return fail(SEPSO_E_ARG, "set_tiles: bucket_of[%d] = %d out of range", i, bucket_of[i]);
    bks[bucket_of[i]].inst.push_back(i);
  }
  for (int j = 0; j < n_buckets; ++j) {
    if (bks[j].inst.empty()) return fail(SEPSO_E_ARG, "set_tiles: bucket %d is empty", j);
    if (!tune_ok(tiles[j].seg_per_thread, tiles[j].block_threads, bucket_desc(b, bks[j].inst)))
      return fail(SEPSO_E_ARG, "set_tiles: bucket %d: %s", j, kTuneRule);
    bks[j].tune = tiles[j];
  }
  b->buckets = std::move(bks);
  b->tune = tiles[0];
  st = ensure_bucket_streams(b);
  if (st != SEPSO_OK) return st;
  return upload_tiles(b);
}

sepso_status sepso_autotune_buckets(sepso_batch* b, int32_t max_buckets, const char* cache_path,
                                    sepso_tune* tiles, int32_t* bucket_of, int32_t* n_buckets,
                                    float* frame_ms) {
  sepso_status st = usable(b);
  if (st != SEPSO_OK) return st;
  if (max_buckets < 1 || max_buckets > kMaxBuckets || !tiles)
    return fail(SEPSO_E_ARG, "autotune_buckets: 1 <= max_buckets <= %d and tiles required", kMaxBuckets);
  // the one-tile baseline
  sepso_tune global{};
  st = sepso_autotune(b, &global);
  if (st != SEPSO_OK) return st;
  const std::vector<std::vector<int>> parts = split_by_waypoints(b, max_buckets);
  if (parts.size() < 2) {
    if (frame_ms) frame_ms[0] = frame_ms[1] = NAN;
    report_tiles(b, tiles, bucket_of, n_buckets);
    return SEPSO_OK;
  }
  // cached tiles of these buckets
  std::vector<std::pair<unsigned long long, sepso_tune>> cache;
  if (cache_path)
    if (FILE* f = fopen(cache_path, "r")) {
      char line[256];
      while (fgets(line, sizeof line, f)) {
        unsigned long long k = 0;
        int K = 0, B = 0;
        if (sscanf(line, "%llx %d %d", &k, &K, &B) == 3) cache.push_back({k, sepso_tune{K, B}});
      }
      const bool bad = ferror(f) != 0;
      fclose(f);
      if (bad) return fail(SEPSO_E_ARG, "tune cache %s: read error", cache_path);
    }
  std::vector<TileBucket> bks(parts.size());
  for (size_t j = 0; j < parts.size(); ++j) {
    bks[j].inst = parts[j];
    bks[j].tune = default_tune(bucket_desc(b, parts[j]));
  }
  b->buckets = bks;
  st = ensure_bucket_streams(b);
  if (st != SEPSO_OK) return st;
  std::vector<std::pair<unsigned long long, sepso_tune>> fresh;
  const int Ks[] = {4, 8, 12, 16, 24};
  const int Bs[] = {64, 128, 256};
  for (size_t j = 0; j < b->buckets.size(); ++j) {
    const std::vector<InstDesc> sub = bucket_desc(b, b->buckets[j].inst);
    const unsigned long long key = bucket_key(b, b->buckets[j]);
    bool hit = false;
    for (auto& c : cache)
      if (c.first == key && tune_ok(c.second.seg_per_thread, c.second.block_threads, sub)) {
        b->buckets[j].tune = c.second;
        hit = true;
      }
    if (hit) continue;
    sepso_tune win = b->buckets[j].tune;
    float win_ms = INFINITY;
    for (int K : Ks)
      for (int B : Bs) {
        if (!tune_ok(K, B, sub)) continue;
        b->buckets[j].tune = sepso_tune{K, B};
        st = upload_tiles(b);
        float ms = 0.f;
        if (st == SEPSO_OK) st = profile_bucket(b, (int)j, 1, &ms);  // warm-up
        if (st == SEPSO_OK) st = profile_bucket(b, (int)j, 3, &ms);
        if (st != SEPSO_OK) return st;
        if (ms < win_ms) {
          win_ms = ms;
          win = b->buckets[j].tune;
        }
      }
    b->buckets[j].tune = win;
    fresh.push_back({key, win});
  }
  // one frame from the frame-0 swarm each way; the faster plan stays
  std::vector<TileBucket> chosen = b->buckets;
  float ms_buckets = 0.f, ms_global = 0.f;
  st = upload_tiles(b);
  if (st == SEPSO_OK) st = restart(b);
  if (st == SEPSO_OK) st = run_frame(b, false, &ms_buckets);
  if (st != SEPSO_OK) return st;
  set_single(b, global);
  st = upload_tiles(b);
  if (st == SEPSO_OK) st = restart(b);
  if (st == SEPSO_OK) st = run_frame(b, false, &ms_global);
  if (st != SEPSO_OK) return st;
  if (frame_ms) {
    frame_ms[0] = ms_buckets;
    frame_ms[1] = ms_global;
  }
  if (ms_buckets < ms_global) {
    b->buckets = chosen;
    b->tune = chosen[0].tune;
    st = upload_tiles(b);
    if (st != SEPSO_OK) return st;
  }
  st = restart(b);
  if (st != SEPSO_OK) return st;
  if (cache_path && !fresh.empty()) {
    FILE* f = fopen(cache_path, "a");
    if (!f) return fail(SEPSO_E_ARG, "tune cache %s: cannot open for writing", cache_path);
    bool ok = true;
    for (auto& c : fresh)
      ok = ok && fprintf(f, "%016llx %d %d\n", c.first, c.second.seg_per_thread,
                         c.second.block_threads) > 0;
    if (fclose(f) != 0 || !ok) return fail(SEPSO_E_ARG, "tune cache %s: write failed", cache_path);
  }
  report_tiles(b, tiles, bucket_of, n_buckets);
  return SEPSO_OK;
}

sepso_status sepso_set_tune(sepso_ctx* ctx, const sepso_tune* tune) {
  if (!ctx) return fail(SEPSO_E_ARG, "ctx is NULL");
  return sepso_batch_set_tune(ctx->b, tune);
}

sepso_status sepso_autotune_ctx(sepso_ctx* ctx, sepso_tune* best) {
  if (!ctx) return fail(SEPSO_E_ARG, "ctx is NULL");
  return sepso_autotune(ctx->b, best);
}

}  // extern "C"

// ============================ evolution phase ===============================

struct sepso_evolve {
  sepso_batch* b = nullptr;   // lower level: instance i = H particle i
  sepso::EvolveDev dev{};
  size_t batch_bytes = 0;
  hipGraphExec_t graph = nullptr;  // one lower-level frame + the H step
  int graph_gen = -1;              // tile plan the graph was captured with
};

namespace sepso {

namespace {
const float kEvolveLo[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
const float kEvolveHi[6] = {3.f, 3.f, 3.f, 1.f, 1.f, 1.f};
}  // namespace

sepso_status evolve_cfg_check(const sepso_evolve_cfg* cfg) {
  if (!cfg) return fail(SEPSO_E_ARG, "evolve cfg is NULL");
  if (cfg->h_groups < 1 || cfg->h_groups > kMaxG)
    return fail(SEPSO_E_ARG, "evolve: h_groups in [1,%d]", kMaxG);
  if (cfg->h_particles < 1 || (int64_t)cfg->h_groups * cfg->h_particles > kEvolveMaxH)
    return fail(SEPSO_E_ARG, "evolve: h_particles >= 1 and h_groups*h_particles <= %d", kEvolveMaxH);
  if (cfg->evolutions < 1) return fail(SEPSO_E_ARG, "evolve: evolutions >= 1");
  const float* lo = cfg->lo ? cfg->lo : kEvolveLo;
  const float* hi = cfg->hi ? cfg->hi : kEvolveHi;
  for (int c = 0; c < 6; ++c)
    if (!(finite(lo[c]) && finite(hi[c]) && lo[c] < hi[c]))
      return fail(SEPSO_E_ARG, "evolve: lo[%d] < hi[%d] finite", c, c);
  if (lo[5] < 0.f) return fail(SEPSO_E_ARG, "evolve: V_limit lower bound < 0");
  if (cfg->h_hyper)
    for (int j = 0; j < 6 * cfg->h_groups; ++j)
      if (!finite(cfg->h_hyper[j]) || (j % 6 == 5 && cfg->h_hyper[j] < 0.f))
        return fail(SEPSO_E_ARG, "evolve: h_hyper");
  return SEPSO_OK;
}

size_t evolve_h_bytes(const sepso_evolve_cfg* cfg, int Dh) {
  const size_t n = (size_t)cfg->h_groups * cfg->h_particles;
  return align256(sizeof(EvolveCtl)) + align256(4 * 3 * n * Dh) + align256(4 * 2 * n) +
         align256(8 * (size_t)cfg->h_groups) + align256(4 * (6 * (size_t)cfg->h_groups + 12)) +
         align256(4 * n) + align256(4 * (size_t)cfg->evolutions);
}

void evolve_h_carve(const sepso_evolve_cfg* cfg, int Dh, char* base, EvolveDev* d,
                    std::vector<float>* consts) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base + off;
    off += align256(bytes);
    return p;
  };
  const int n = cfg->h_groups * cfg->h_particles;
  d->Gh = cfg->h_groups;
  d->Nh = cfg->h_particles;
  d->Dh = Dh;
  d->E = cfg->evolutions;
  d->seed_lo = (uint32_t)(cfg->seed & 0xffffffffu);
  d->seed_hi = (uint32_t)(cfg->seed >> 32);
  const size_t nD = (size_t)n * Dh;
  d->ctl = reinterpret_cast<EvolveCtl*>(take(sizeof(EvolveCtl)));
  float* xvp = reinterpret_cast<float*>(take(4 * 3 * nD));
  d->X = xvp;
  d->V = xvp + nD;
  d->P = xvp + 2 * nD;
  float* pl2 = reinterpret_cast<float*>(take(4 * 2 * (size_t)n));
  d->Pf = pl2;
  d->lfv = pl2 + n;
  char* gb = take(8 * (size_t)d->Gh);
  d->gbest_n = reinterpret_cast<int32_t*>(gb);
  d->gbest_f = reinterpret_cast<float*>(gb + 4 * d->Gh);
  float* cst = reinterpret_cast<float*>(take(4 * (6 * (size_t)d->Gh + 12)));
  d->h_hyper = cst;
  d->lo = cst + 6 * d->Gh;
  d->hi = cst + 6 * d->Gh + 6;
  d->lfv_in = reinterpret_cast<float*>(take(4 * (size_t)n));
  d->curve = reinterpret_cast<float*>(take(4 * (size_t)d->E));
  consts->assign(6 * d->Gh + 12, 0.f);
  for (int j = 0; j < 6 * d->Gh; ++j)
    (*consts)[j] = cfg->h_hyper ? cfg->h_hyper[j] : kHyper8[(j / 6) % 8][j % 6];
  for (int c = 0; c < 6; ++c) {
    (*consts)[6 * d->Gh + c] = cfg->lo ? cfg->lo[c] : kEvolveLo[c];
    (*consts)[6 * d->Gh + 6 + c] = cfg->hi ? cfg->hi[c] : kEvolveHi[c];
  }
}

hipError_t evolve_h_state(const EvolveDev& d, hipStream_t st, sepso_evolve_state* s) {
  const size_t n = (size_t)d.Gh * d.Nh, nD = n * d.Dh;
  hipError_t e = hipSuccess;
  auto d2h = [&](void* dst, const void* src, size_t bytes) {
    if (dst && e == hipSuccess) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st);
  };
  EvolveCtl c{};
  d2h(s->X, d.X, 4 * nD);
  d2h(s->V, d.V, 4 * nD);
  d2h(s->P, d.P, 4 * nD);
  d2h(s->Pf, d.Pf, 4 * n);
  d2h(s->lfv, d.lfv, 4 * n);
  d2h(s->gbest_n, d.gbest_n, 4 * (size_t)d.Gh);
  d2h(s->gbest_f, d.gbest_f, 4 * (size_t)d.Gh);
  d2h(&c, d.ctl, sizeof(EvolveCtl));
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  s->tb_g = c.tb_g;
  s->tb_n = c.tb_n;
  s->tb_f = c.tb_f;
  s->k = c.k;
  s->ctr = c.ctr;
  return hipSuccess;
}

hipError_t evolve_h_best(const EvolveDev& d, hipStream_t st, float* hyper, float* lfv, int* k) {
  EvolveCtl c{};
  hipError_t e = hipMemcpyAsync(&c, d.ctl, sizeof(EvolveCtl), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  *k = c.k;
  if (c.k == 0) return hipSuccess;
  if (hyper) {
    const size_t row = (size_t)(c.tb_g * d.Nh + c.tb_n) * d.Dh;
    e = hipMemcpyAsync(hyper, d.P + row, 4 * (size_t)d.Dh, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  if (lfv) *lfv = c.tb_f;
  return e;
}

hipError_t evolve_h_curve(const EvolveDev& d, hipStream_t st, int k0, int n, float* curve) {
  const int E = d.E, first = k0 % E;
  const int n1 = std::min(n, E - first);
  hipError_t e = hipMemcpyAsync(curve, d.curve + first, 4 * (size_t)n1, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && n > n1)
    e = hipMemcpyAsync(curve + n1, d.curve, 4 * (size_t)(n - n1), hipMemcpyDeviceToHost, st);
  return e;
}

}  // namespace sepso

namespace {

struct EvolveInputs {
  std::vector<sepso_map> maps;
  std::vector<sepso_swarm> swarms;
  std::vector<float> placeholder;  // lower-level hyper until the H init writes it
  size_t batch_bytes = 0, h_bytes = 0;
};

sepso_status evolve_inputs(const sepso_map* map, const sepso_swarm* lower,
                           const sepso_evolve_cfg* cfg, EvolveInputs* in) {
  if (!map || !lower || !cfg) return fail(SEPSO_E_ARG, "map/lower/cfg is NULL");
  sepso_status st = evolve_cfg_check(cfg);
  if (st != SEPSO_OK) return st;
  const int n = cfg->h_groups * cfg->h_particles;
  sepso_swarm t = *lower;
  if (t.groups < 1 || t.groups > kMaxG) return fail(SEPSO_E_ARG, "lower: groups in [1,%d]", kMaxG);
  in->placeholder.resize(6 * t.groups);
  for (int j = 0; j < 6 * t.groups; ++j) in->placeholder[j] = kHyper8[(j / 6) % 8][j % 6];
  if (!t.hyper) t.hyper = in->placeholder.data();
  t.use_pi = 0;
  t.at_mode = 0;
  t.hsef_every = 0;
  in->maps.assign(n, *map);
  in->swarms.assign(n, t);
  for (int i = 0; i < n; ++i) in->swarms[i].instance = (uint32_t)i;
  st = sepso_batch_workspace_bytes(in->maps.data(), in->swarms.data(), n, &in->batch_bytes);
  if (st != SEPSO_OK) return st;
  in->batch_bytes = align256(in->batch_bytes);
  in->h_bytes = evolve_h_bytes(cfg, 6 * t.groups);
  return SEPSO_OK;
}

sepso_status evolve_usable(sepso_evolve* ev) {
  if (!ev) return fail(SEPSO_E_ARG, "evolve handle is NULL");
  return usable(ev->b);
}

}  // namespace

extern "C" {

sepso_status sepso_evolve_workspace_bytes(const sepso_map* map, const sepso_swarm* lower,
                                          const sepso_evolve_cfg* cfg, size_t* bytes) {
  if (!bytes) return fail(SEPSO_E_ARG, "bytes is NULL");
  EvolveInputs in;
  sepso_status st = evolve_inputs(map, lower, cfg, &in);
  if (st != SEPSO_OK) return st;
  *bytes = in.batch_bytes + in.h_bytes;
  return SEPSO_OK;
}

sepso_status sepso_evolve_create(const sepso_map* map, const sepso_swarm* lower,
                                 const sepso_evolve_cfg* cfg, void* d_ws, size_t ws_bytes,
                                 void* stream, sepso_evolve** out) {
  if (!out) return fail(SEPSO_E_ARG, "out is NULL");
  *out = nullptr;
  EvolveInputs in;
  sepso_status st = evolve_inputs(map, lower, cfg, &in);
  if (st != SEPSO_OK) return st;
  if (!d_ws) return fail(SEPSO_E_ARG, "workspace is NULL");
  if (ws_bytes < in.batch_bytes + in.h_bytes)
    return fail(SEPSO_E_NOMEM, "workspace too small: %zu < %zu bytes", ws_bytes,
                in.batch_bytes + in.h_bytes);
  const int n = cfg->h_groups * cfg->h_particles;
  sepso_evolve* ev = new (std::nothrow) sepso_evolve();
  if (!ev) return fail(SEPSO_E_NOMEM, "host allocation failed");
  st = create_batch(in.maps.data(), in.swarms.data(), n, d_ws, in.batch_bytes, stream, nullptr, &ev->b);
  if (st != SEPSO_OK) {
    delete ev;
    return st;
  }
  ev->batch_bytes = in.batch_bytes;
  EvolveDev& d = ev->dev;
  std::vector<float> hc;
  evolve_h_carve(cfg, 6 * lower->groups, static_cast<char*>(d_ws) + in.batch_bytes, &d, &hc);
  sepso_batch* b = ev->b;
  hipError_t e = hipMemcpyAsync(const_cast<float*>(d.h_hyper), hc.data(), 4 * hc.size(),
                                hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) {
    launch_evolve_init(d, b->pl, b->stream);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) {
    st = fail(SEPSO_E_HIP, "evolve create: %s", hipGetErrorString(e));
    destroy_batch(b);
    delete ev;
    return st;
  }
  *out = ev;
  return SEPSO_OK;
}

sepso_status sepso_evolve_destroy(sepso_evolve* ev) {
  if (!ev) return fail(SEPSO_E_ARG, "evolve handle is NULL");
  if (ev->graph) (void)hipGraphExecDestroy(ev->graph);  // teardown: best effort
  destroy_batch(ev->b);
  delete ev;
  return SEPSO_OK;
}

sepso_status sepso_evolve_run(sepso_evolve* ev, int32_t n, float* curve) {
  sepso_status st = evolve_usable(ev);
  if (st != SEPSO_OK) return st;
  if (n < 0) return fail(SEPSO_E_ARG, "n must be >= 0");
  if (curve && n > ev->dev.E) return fail(SEPSO_E_ARG, "curve holds at most `evolutions` values");
  sepso_batch* b = ev->b;
  if (ev->graph && ev->graph_gen != b->tune_gen) {
    (void)hipGraphExecDestroy(ev->graph);  // retired: the tile plan changed
    ev->graph = nullptr;
  }
  if (!ev->graph) {
    ev->graph_gen = b->tune_gen;
    hipGraph_t g = nullptr;
    HIPCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    hipError_t eq = enqueue_frame(b, false);
    launch_evolve_step(ev->dev, b->pl, 0, b->stream);
    if (eq == hipSuccess) eq = hipGetLastError();
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (eq != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return hip_fail(b, eq, "evolution capture");
    }
    if (e != hipSuccess) return hip_fail(b, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&ev->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);  // the instantiated graph keeps what it needs
    if (e != hipSuccess) return hip_fail(b, e, "hipGraphInstantiate");
  }
  EvolveCtl c0{};
  if (curve) {
    HIPCHK(b, hipMemcpyAsync(&c0, ev->dev.ctl, sizeof(EvolveCtl), hipMemcpyDeviceToHost, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
  }
  for (int k = 0; k < n; ++k) HIPCHK(b, hipGraphLaunch(ev->graph, b->stream));
  b->frames_done += n;
  if (curve && n > 0) HIPCHK(b, evolve_h_curve(ev->dev, b->stream, c0.k, n, curve));
  HIPCHK(b, hipStreamSynchronize(b->stream));
  return SEPSO_OK;
}

sepso_status sepso_evolve_inject(sepso_evolve* ev, const float* lfv) {
  sepso_status st = evolve_usable(ev);
  if (st != SEPSO_OK) return st;
  if (!lfv) return fail(SEPSO_E_ARG, "lfv is NULL");
  sepso_batch* b = ev->b;
  const int n = ev->dev.Gh * ev->dev.Nh;
  HIPCHK(b, hipMemcpyAsync(const_cast<float*>(ev->dev.lfv_in), lfv, 4 * (size_t)n,
                           hipMemcpyHostToDevice, b->stream));
  launch_evolve_step(ev->dev, b->pl, 1, b->stream);
  LAUNCHCHK(b, "evolve step launch");
  HIPCHK(b, hipStreamSynchronize(b->stream));
  return SEPSO_OK;
}

sepso_status sepso_evolve_get_state(sepso_evolve* ev, sepso_evolve_state* s) {
  sepso_status st = evolve_usable(ev);
  if (st != SEPSO_OK) return st;
  if (!s) return fail(SEPSO_E_ARG, "state is NULL");
  HIPCHK(ev->b, evolve_h_state(ev->dev, ev->b->stream, s));
  return SEPSO_OK;
}

sepso_status sepso_evolve_best(sepso_evolve* ev, float* hyper, float* lfv) {
  sepso_status st = evolve_usable(ev);
  if (st != SEPSO_OK) return st;
  int k = 0;
  HIPCHK(ev->b, evolve_h_best(ev->dev, ev->b->stream, hyper, lfv, &k));
  if (k == 0) return fail(SEPSO_E_STATE, "no evolution has run yet");
  return SEPSO_OK;
}

sepso_status sepso_evolve_lower(sepso_evolve* ev, sepso_batch** b) {
  if (!ev || !b) return fail(SEPSO_E_ARG, "evolve/out is NULL");
  *b = ev->b;
  return SEPSO_OK;
}

}  // extern "C"
