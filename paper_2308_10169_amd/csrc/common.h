// Shared host/device definitions of libsepso: per-instance descriptors,
// mutable control blocks and the obstacle-edge record.  Everything lives in
// the caller's workspace; see layout.cpp for the carve-up.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sepso {

constexpr int kMaxW = 64;        // interior waypoints per path
constexpr int kMaxG = 64;        // groups per instance
constexpr int kHist = 64;        // Auto-Truncation history ring
constexpr int kStageFloats = 2048;  // general-polygon edge records staged in LDS per pass (256)

// Learned initializer: 64 x 64 occupancy raster + start/target (4 values)
// -> 3 x 512 hidden -> 8 groups x 20 waypoints x 2 coordinates.
constexpr int kRaster = 64;
constexpr int kLinIn = kRaster * kRaster + 4;   // 4100
constexpr int kLinInPad = 4128;                 // multiple of 32
constexpr int kLinHidden = 512;
constexpr int kLinGroups = 8, kLinW = 20;
constexpr int kLinOut = kLinGroups * 2 * kLinW; // 320

// Philox counter tags: which random stream a draw belongs to.
enum Tag : uint32_t { TAG_UPDATE = 0, TAG_INIT_X = 1, TAG_INIT_V = 2, TAG_PI = 3, TAG_HSEF = 4,
                      TAG_EVOLVE = 6, TAG_EVOLVE_X = 7, TAG_EVOLVE_V = 8, TAG_UPDATE_DIM = 12 };

// Edge flags.
enum : int32_t { EDGE_FIRST = 1, EDGE_LAST = 2 };

// One polygon edge a -> b, stored so that the fitness kernel can (i) test
// which side of every path segment the end vertex b lies on and (ii) test
// which side of the edge's line every path point lies on:
//   side(p) = sign(ex * p.y - ey * p.x - (ex * a.y - ey * a.x)).
// The first edge of a polygon also carries its start vertex a (= v0), whose
// side is reused by the polygon's closing edge.
struct EdgeRec {
  float bx, by;     // end vertex
  float ex, ney;    // b - a  (ney = -(b.y - a.y))
  float nce;        // -(ex * a.y - ey * a.x)
  float ax, ay;     // start vertex (meaningful on the first edge of a polygon)
  int32_t flags;    // EDGE_FIRST / EDGE_LAST
};
static_assert(sizeof(EdgeRec) == 32, "EdgeRec is 32 bytes");

// One convex polygon of at most kCPolyMax vertices (every turn strictly the
// same way), 192 bytes read through the scalar cache: integer keys of its
// bounding box (ordering as the floats do), its vertex count, then per edge
// the line coefficients oriented so that the interior is on the positive
// side -- ev(p) = ex * p.y + ney * p.x + nce -- and per vertex its
// coordinates.
constexpr int kCPolyMax = 8;
struct CPoly {
  int32_t kx0, ky0, kx1, ky1;
  int32_t n;
  int32_t pad[3];
  float ex[kCPolyMax], ney[kCPolyMax], nce[kCPolyMax];
  float vx[kCPolyMax], vy[kCPolyMax];
};
static_assert(sizeof(CPoly) == 192, "CPoly is 192 bytes");

// Read-only description of one instance (sizes, constants, pool offsets).
struct InstDesc {
  int32_t G, N, W, T;
  int32_t n_edges, n_polys;
  int32_t ppb;           // particles per block of the fused iteration
  int32_t n_blocks;      // ceil(G*N / ppb)
  float width, height;
  float alpha; int32_t beta;
  int32_t use_pi, n_pi;  // PI on, particles per group that get it
  float pi_radius;
  int32_t at_mode, at_window; float at_delta;
  int32_t hsef_every, T_outer;
  uint32_t seed_lo, seed_hi, instance;
  int32_t rand_per_dim;  // one (r1, r2, r3) per coordinate instead of per particle
  int64_t xo;            // X, V, P pools: G*N*2W floats
  int64_t po;            // per-particle pools: G*N
  int32_t eo;            // vertices (n_edges float2)
  int32_t n_rects;       // polygons that are axis-aligned rectangles
  int32_t n_gedges;      // edges of the other non-convex polygons
  int32_t n_cpolys;      // convex polygons (other than rectangles)
  int32_t cpo;           // their records (n_cpolys CPoly)
  int32_t ro;            // rectangle records (n_rects float4: x0, y0, x1, y1)
  int32_t geo;           // general edge records (n_gedges)
  int32_t plo;           // poly_ptr pool (n_polys+1)
  int32_t pvo;           // poly_vel pool (n_polys float2)
  int32_t go;            // group pools: G (gbest_n/f, outer Pbest fitness), G*6 hyper, G*3 outer
  int32_t gpo;           // gbest positions: G*2W
  int32_t dpo;           // per-instance path pools (Tbest, previous plan): 2W
};

// Mutable per-instance control block (device resident).
struct InstCtl {
  int32_t k;             // iterations with bests done in the current plan
  int32_t pending;       // iteration k's velocity/position update not applied yet
  int32_t done;          // the current frame has ended
  int32_t frame;         // frames planned so far (random stream position for inits)
  uint32_t ctr;          // counter of iteration k's update draws
  uint32_t epoch_ctr;    // outer-swarm steps taken (random stream position)
  int32_t tb_g, tb_n;    // total best
  float tb_f;
  int32_t arrive;        // blocks finished in the current launch
  int32_t epoch_in_frame, otb;
  int32_t truncated;
  int32_t have_prev;     // a previous plan exists (PI allowed)
  float res_cost, res_len;
  int32_t res_q, res_iters, res_trunc, use_learned;
  float hist[kHist];     // Tbest fitness after iterations 1..k (ring)
};


}  // namespace sepso

namespace sepso {

// Device pointers of every pool in the workspace (passed by value).
struct Pools {
  int32_t n_inst;
  // fused-iteration LDS areas (floats), maxima over the instances
  int32_t pos_floats;    // a block's new positions (ppb * 2W)
  int32_t stage_floats;  // one chunk of general-polygon edge records
  int32_t gb_floats;     // Tbest and the gbest rows of a block's groups
  int32_t ngb_max;       // groups a block spans
  int32_t ppb_max;       // particles per block
  int32_t rsplit;        // wave groups the rectangles are dealt over (1, 2 or 4)
  const InstDesc* desc;
  InstCtl* ctl;
  float *X, *V, *P;
  float *f, *L, *Pf, *PL;
  int32_t *Q, *PQ;
  EdgeRec* edges;    // general polygons' edges
  CPoly* cpolys;     // convex polygons
  float4* rects;     // axis-aligned rectangles (x0, y0, x1, y1), x0 < x1, y0 < y1
  float4* rect_c;    // their centres and half sides (xc, yc, w/2, h/2)
  int2* pkind;       // per polygon: (1 = rectangle / 2, 3 = convex, counter-clockwise or not / 0 = general, slot in its pool)
  float2* verts;
  int32_t* poly_ptr;
  float2* poly_vel;
  float4* ends;      // start.xy, target.xy per instance
  float4* end_vel;   // per instance
  int32_t* gbest_n;
  float* gbest_f;
  float* hyper;      // G*6 per instance
  const float* outer_hyper;
  float* ov;         // G*3
  float* op;         // G*3
  float* opf;        // G
  float* gbest_pos;  // G*2W
  float* tbest_pos;  // 2W
  float* prev_path;  // 2W
  float* proposal;   // G*2W learned initial path per group (layout of gbest_pos)
  const int2* blk_tiles;  // fused-iteration block -> (instance, first particle)
  const int2* blk_init;   // init block -> (instance, first element)
};

// Evolution phase: the higher-level swarm (H-SEPSO) over whole lower-level
// hyper matrices.  H particle i drives lower-level instance i.
constexpr int kEvolveMaxH = 1024;  // H particles (one block moves them all)

struct EvolveCtl {
  int32_t k;      // evolutions done
  uint32_t ctr;   // random stream position of the move
  int32_t tb_g, tb_n;
  float tb_f;
  int32_t pad[3];
};

struct EvolveDev {
  int32_t Gh, Nh, Dh, E;       // H groups, particles per group, dims (6 G_L), schedule length
  uint32_t seed_lo, seed_hi;
  float *X, *V, *P;            // Gh*Nh*Dh
  float* Pf;                   // Gh*Nh
  float* lfv;                  // fitness of the last evolution
  int32_t* gbest_n;            // Gh
  float* gbest_f;              // Gh
  const float* h_hyper;        // Gh*6
  const float* lo;             // 6 per-column bounds
  const float* hi;             // 6
  const float* lfv_in;         // injected fitness (n) or null: lower level's frame result
  float* curve;                // total best after evolution k, at (k-1) mod E
  EvolveCtl* ctl;
  float* hyper_out;            // lower-level hyper rows (n x Dh), or null: the batch's hyper pool
};

// Kernel flags of the fused iteration.
enum : int32_t { STEP_FIT = 1, STEP_FRAME = 2 };

}  // namespace sepso
