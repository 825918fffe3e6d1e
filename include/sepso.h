/*
 * libsepso -- MI355X (gfx950) planner hot path of SEPSO: grouped particle
 * swarm optimisation in tensor form with a path fitness of polyline length
 * plus a crossing penalty, its application-phase frame loop, and batched
 * planning of many independent instances.
 *
 * Paper: Xin, Li, Zhang, Li, "Efficient Real-time Path Planning with
 * Self-evolving Particle Swarm Optimization in Dynamic Scenarios".
 *
 * Conventions (all entry points):
 *  - Every function returns sepso_status; SEPSO_OK is 0.  sepso_last_error()
 *    returns a thread-local message for the last failure.  No C++ exception
 *    crosses this boundary.
 *  - Arguments are validated before any device work: on SEPSO_E_ARG nothing
 *    has been launched and nothing has changed.
 *  - A HIP failure (SEPSO_E_HIP) is sticky: the handle refuses further work
 *    (SEPSO_E_STATE) until it is destroyed.
 *  - Host input structs and arrays are copied during the call; the caller
 *    keeps ownership.  Host outputs go to caller-allocated buffers.
 *  - Device memory is a caller-provided workspace (size from the matching
 *    *_workspace_bytes call, 256-byte aligned base), which must stay valid
 *    and untouched until the handle is destroyed.  The library allocates no
 *    device memory of its own; it allocates a small pinned host buffer per
 *    handle for results.
 *  - Work is enqueued on the caller's HIP stream (hipStream_t passed as
 *    void*; NULL = the default stream).  Functions documented as
 *    "asynchronous" return before the device work completes.
 *  - A handle is single-threaded; distinct handles are independent.
 *
 * Particle layout (Eq.(10)): a path of W interior waypoints is the vector
 * [x_1..x_W, y_1..y_W]; swarm arrays are (G, N, 2W) row-major FP32.
 */
#ifndef SEPSO_H
#define SEPSO_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sepso_status {
  SEPSO_OK = 0,
  SEPSO_E_ARG = 1,         /* invalid argument; nothing launched */
  SEPSO_E_NOMEM = 2,       /* workspace too small or host allocation failed */
  SEPSO_E_HIP = 3,         /* HIP runtime error (sticky) */
  SEPSO_E_STATE = 4,       /* handle unusable (earlier HIP error) or wrong call order */
  SEPSO_E_UNSUPPORTED = 5  /* valid request the library does not support */
} sepso_status;

const char* sepso_last_error(void);
const char* sepso_version(void);

/* The planner's random numbers are Philox4x32-10 blocks (Salmon et al.,
 * SC'11; the random factors of Eq.(4) and the initial, PI and evolution
 * draws).  For checking the streams: d_out (device, 16-byte aligned, 4*n
 * words) receives, for i < n, the block of counter (first + i mod 2^32, c1,
 * c2, c3) under the 64-bit key (low word first).  The planner's draws use
 * counter (index, step, instance, stream tag) and key = the swarm's seed.
 * Asynchronous on stream (NULL = the default stream); n <= 2^32. */
sepso_status sepso_philox(uint32_t first, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t key,
                          int64_t n, uint32_t* d_out, void* stream);

/* Polygonal map (Sec. "Map representation"): obstacles are closed polygons
 * given by their vertices; a path collides where one of its segments
 * properly crosses a polygon edge.  Map = [0,width] x [0,height]. */
typedef struct sepso_map {
  float width, height;
  int32_t n_polys;           /* >= 0 */
  const int32_t* poly_ptr;   /* n_polys+1 vertex offsets, poly_ptr[0] = 0, >= 3 vertices each */
  const float* verts;        /* poly_ptr[n_polys] vertices, (x, y) pairs */
  float start[2], target[2]; /* path end points, inside the map */
  const float* poly_vel;     /* n_polys (vx, vy) per frame for the device motion model, or NULL = static */
  float endpoint_vel[4];     /* start (vx, vy), target (vx, vy) per frame */
} sepso_map;

/* One planner instance: DTPSO (Algorithm 1) over G groups of N particles
 * with W waypoints, the fitness of Eq.(11)-(13), and the application-phase
 * mechanisms (Priori Initialization, Auto Truncation, online HSEF). */
typedef struct sepso_swarm {
  int32_t groups, particles, waypoints; /* G >= 1, N >= 1, 1 <= W <= 64 */
  int32_t max_iters;                    /* T >= 1: inertia schedule length and per-frame cap */
  const float* hyper;                   /* G x 6: C1, C2, C3, w_init, w_end, V_limit (Table hyper8 layout) */
  float alpha; int32_t beta;            /* penalty alpha * Q^beta, beta >= 1 (Eq.13) */
  int32_t use_pi; float pi_gamma, pi_radius; /* Priori Initialization: fraction and half-width */
  int32_t at_mode, at_window; float at_delta; /* Auto Truncation (needs a collision-free best):
                                                 0 off; 1 population std of the last `window`
                                                 Tbest values < delta (full window); 2 relative
                                                 gain over `window` iterations < delta; 3 as 1
                                                 over the last min(k, window) values, k >= 2 */
  int32_t hsef_every;                   /* online self-evolution period in iterations (0 = off) */
  const float* hsef_hyper;              /* G x 6 hyper of the outer swarm (NULL = Table hyper8 rows) */
  uint64_t seed;                        /* Philox4x32-10 key */
  uint32_t instance;                    /* Philox counter word 2 */
  int32_t rand_per_dim;                 /* 0: one (r1, r2, r3) per particle and iteration (the
                                           paper's R of shape (4, G, N)); 1: variant with one
                                           per coordinate, counter (particle*2W + coordinate,
                                           iteration, instance, 12) */
} sepso_swarm;

typedef struct sepso_frame_result {
  float cost;          /* Tbest fitness F = L + alpha Q^beta */
  float length;        /* L of the returned path */
  int32_t crossings;   /* Q of the returned path */
  int32_t iters;       /* iterations run in this frame */
  int32_t truncated;   /* Auto Truncation fired */
  int32_t used_learned;/* 1: the attached learned initializer's proposal seeded this
                          frame's Priori Initialization; 0: plain PI or uniform */
  float device_ms;     /* device time of the frame (0 when batched) */
} sepso_frame_result;

/* Host views for state inspection / injection (any pointer may be NULL to
 * skip that array).  Sizes: X, V, P: G*N*2W; f, L, Pf, PL: G*N floats;
 * Q, PQ: G*N int32; gbest_n: G int32; gbest_f: G floats; hyper: G*6. */
typedef struct sepso_state {
  float *X, *V, *P;
  float *f, *L, *Pf, *PL;
  int32_t *Q, *PQ;
  int32_t* gbest_n; float* gbest_f;
  float* hyper;
  int32_t tbest_g, tbest_n; float tbest_f;
  int32_t k;           /* iterations done in the current plan */
  uint32_t ctr;        /* global iteration counter (random-stream position) */
  int32_t frame;       /* frames planned so far */
} sepso_state;

/* Tile configuration of the fused iteration kernel.  Valid for a batch when
 * K <= 2*(smallest waypoint count + 2), K * block_threads <= 4096 and the
 * kernel's LDS for the batch's shapes stays within 64 KiB (otherwise
 * SEPSO_E_ARG). */
typedef struct sepso_tune {
  int32_t seg_per_thread; /* K: path segments per thread, one of 4, 8, 12, 16, 24 */
  int32_t block_threads;  /* 64, 128, 256 */
} sepso_tune;

typedef struct sepso_ctx sepso_ctx;
typedef struct sepso_batch sepso_batch;

/* ---- path fitness --------------------------------------------------------
 * Fitness of given paths on a polygonal map (Eq.(11)-(13), Sec. "Map
 * representation"): path r is [start, w_1..w_W, target] with the waypoints
 * in the Eq.(10) layout, paths[r*2W + i] = x_{i+1}, paths[r*2W + W + i] =
 * y_{i+1}; L = sum of the W+1 segment lengths; Q = number of proper
 * crossings (both pairs of orientations strictly of opposite sign; touching
 * and collinear contacts do not count) of the segments with every polygon
 * edge (v_j, v_{j+1}), the last vertex joined to the first; F = L +
 * alpha * Q^beta.  FP32 throughout.
 * Device inputs: poly_ptr (n_polys+1 int32 vertex offsets, non-decreasing,
 * poly_ptr[0] = 0, poly_ptr[n_polys] = n_vert), verts (n_vert (x, y)
 * pairs), ends (4 floats: start x, y, target x, y), paths (n_paths x 2W).
 * Device outputs: f, L (n_paths floats), Q (n_paths int32).  The workspace
 * (size from sepso_fitness_workspace_bytes, 256-byte aligned) holds the
 * edge records and per-segment partial results; it is free again when the
 * work has completed.  Asynchronous on stream (NULL = the default stream);
 * n_paths = 0 launches nothing.  1 <= waypoints <= 64, beta >= 1, alpha
 * finite, n_paths * (W + 1) < 2^31, else SEPSO_E_ARG; a workspace that is
 * too small gives SEPSO_E_NOMEM; a launch failure gives SEPSO_E_HIP. */
sepso_status sepso_fitness_workspace_bytes(int32_t n_vert, int32_t n_paths, int32_t waypoints,
                                           size_t* bytes);
sepso_status sepso_fitness(int32_t n_polys, int32_t n_vert, const int32_t* d_poly_ptr,
                           const float* d_verts, const float* d_ends, const float* d_paths,
                           int32_t n_paths, int32_t waypoints, float alpha, int32_t beta,
                           float* d_f, float* d_L, int32_t* d_Q, void* d_workspace,
                           size_t workspace_bytes, void* stream);

/* sepso_fitness without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the edge records and per-segment partial results live
 * in a fixed 8 MiB device array that the library holds on each GPU it runs
 * on until the process ends.  The call allocates nothing (no hipMalloc,
 * hipFree or allocating library routine).  Requests whose workspace
 * (sepso_fitness_workspace_bytes) would exceed 8 MiB give SEPSO_E_ARG.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (different streams or threads, work still in flight) race; calls
 * ordered on one stream do not.  Same arguments, results and errors as
 * sepso_fitness otherwise. */
sepso_status sepso_fitness_noalloc(int32_t n_polys, int32_t n_vert, const int32_t* d_poly_ptr,
                                   const float* d_verts, const float* d_ends, const float* d_paths,
                                   int32_t n_paths, int32_t waypoints, float alpha, int32_t beta,
                                   float* d_f, float* d_L, int32_t* d_Q, void* stream);

/* ---- single instance ---------------------------------------------------- */
sepso_status sepso_workspace_bytes(const sepso_map* map, const sepso_swarm* swarm, size_t* bytes);

/* Validates and copies the map and swarm, carves the workspace, uploads the
 * geometry and initialises the swarm uniformly (frame 0).  Asynchronous. */
sepso_status sepso_create(const sepso_map* map, const sepso_swarm* swarm, void* d_workspace,
                          size_t workspace_bytes, void* stream, sepso_ctx** out);
sepso_status sepso_destroy(sepso_ctx* ctx);

/* n iterations of Algorithm 1 (fitness -> Pbest/Gbest/Tbest -> inertia ->
 * velocity clip -> position clip), no host synchronisation.  Asynchronous. */
sepso_status sepso_step(sepso_ctx* ctx, int32_t n);

/* One application-phase frame: next map (host copy) or, with next == NULL,
 * one step of the device motion model for frames after the first; swarm
 * init with Priori Initialization from the last frame's plan; iterations
 * with online HSEF until Auto Truncation or max_iters.  Synchronises once;
 * writes *out and the plan's 2W path values to out_path (may be NULL).
 * A next map keeps the polygon structure: the same poly_ptr, and every
 * polygon of the same kind as in the first map (axis-aligned rectangle;
 * convex polygon of at most 8 vertices turning the same way; any other),
 * else SEPSO_E_ARG and nothing runs. */
sepso_status sepso_plan_frame(sepso_ctx* ctx, const sepso_map* next, sepso_frame_result* out,
                              float* out_path);

/* n iterations of the current frame as sepso_plan_frame runs them: bests
 * with Auto Truncation and, every hsef_every iterations, the online outer
 * step (Sec. "HSEF"), up to max_iters; once the frame has ended (truncated
 * or at max_iters) further calls do nothing until sepso_reinit or
 * sepso_set_state.  The last iteration's update is applied before the call
 * returns, as in sepso_step.  Asynchronous. */
sepso_status sepso_step_frame(sepso_ctx* ctx, int32_t n);

/* Online self-evolution state (Sec. "HSEF"): outer particle g is group g's
 * (w_init, C1, C2); ov, op (G x 3 in that order) are its velocity and best
 * position, opf (G) its best fitness; otb the outer total best, epoch_in_frame
 * the outer steps of this frame (inertia schedule position), epoch_ctr the
 * outer random-stream position.  Any array may be NULL.  Synchronous. */
typedef struct sepso_outer {
  float *ov, *op, *opf;
  int32_t otb, epoch_in_frame;
  uint32_t epoch_ctr;
} sepso_outer;
sepso_status sepso_get_outer(sepso_ctx* ctx, sepso_outer* o);
sepso_status sepso_set_outer(sepso_ctx* ctx, const sepso_outer* o);

/* Re-initialise the swarm for frame index `frame` (uniform; with
 * use_prev != 0 and PI enabled, Priori Initialization from the last plan).
 * Asynchronous. */
sepso_status sepso_reinit(sepso_ctx* ctx, int32_t frame, int32_t use_prev);

/* Copy the device state out / in.  Synchronous. */
sepso_status sepso_get_state(sepso_ctx* ctx, sepso_state* st);
sepso_status sepso_set_state(sepso_ctx* ctx, const sepso_state* st);

/* Current obstacle vertices and endpoints (after device motion): verts gets
 * 2*n_vert floats, endpoints 4 floats (start, target).  Synchronous. */
sepso_status sepso_get_geometry(sepso_ctx* ctx, float* verts, float* endpoints);

/* Mean device time of one fused iteration kernel over n back-to-back
 * launches (HIP events on the handle's stream).  Advances the swarm. */
sepso_status sepso_profile_step(sepso_ctx* ctx, int32_t n, float* avg_ms);

/* Tile shape of the fused iteration: set explicitly, or chosen by timing
 * candidates (the swarm is re-initialised for frame 0 afterwards). */
sepso_status sepso_set_tune(sepso_ctx* ctx, const sepso_tune* tune);
sepso_status sepso_autotune_ctx(sepso_ctx* ctx, sepso_tune* best);

/* ---- batch of independent instances ------------------------------------ */
sepso_status sepso_batch_workspace_bytes(const sepso_map* maps, const sepso_swarm* swarms,
                                         int32_t n_inst, size_t* bytes);
/* tune may be NULL (defaults).  Asynchronous (geometry upload + init). */
sepso_status sepso_batch_create(const sepso_map* maps, const sepso_swarm* swarms, int32_t n_inst,
                                void* d_workspace, size_t workspace_bytes, void* stream,
                                const sepso_tune* tune, sepso_batch** out);
sepso_status sepso_batch_destroy(sepso_batch* b);
/* Offsets of each instance's path in the flat out_paths array (n_inst+1). */
sepso_status sepso_batch_path_offsets(sepso_batch* b, int64_t* offsets);
/* n_frames frames of every instance (device motion model between frames),
 * one captured graph per frame, one synchronisation per frame.  out holds
 * n_inst * n_frames results (frame-major); out_paths (may be NULL) gets the
 * last frame's paths. */
sepso_status sepso_batch_plan(sepso_batch* b, int32_t n_frames, sepso_frame_result* out,
                              float* out_paths);
/* State of instance i of a batch (same views as sepso_get_state). */
sepso_status sepso_batch_get_state(sepso_batch* b, int32_t i, sepso_state* st);
sepso_status sepso_batch_profile_step(sepso_batch* b, int32_t n, float* avg_ms);
/* Choose seg_per_thread / block_threads by timing candidates on this batch;
 * the winner is applied to the batch and written to *best (may be NULL).
 * Afterwards the batch is as new: control blocks (random-stream positions,
 * frame index, previous plans) and hyper-parameters reset and the frame-0
 * swarm initialised.
 * Synchronous. */
sepso_status sepso_autotune(sepso_batch* b, sepso_tune* best);
/* sepso_autotune with a persistent cache: cache_path is a text file of lines
 * "<key> <K> <block_threads>", the key a 64-bit hash (16 hex digits) of the
 * device architecture name, a fingerprint of the library's device-code
 * sources (a rebuilt library does not reuse another build's tiles) and every
 * instance's groups, particles, waypoints, rectangles, convex polygons and
 * other-polygon edges.  When the file holds this
 * batch's key with a valid tile, that tile is applied without timing
 * (and the batch is reset as after sepso_autotune);
 * otherwise the batch is autotuned and a line is appended.  A missing file is
 * created; a file that cannot be read or written gives SEPSO_E_ARG, and an
 * unreadable line is skipped.  Synchronous.  best may be NULL. */
sepso_status sepso_autotune_cached(sepso_batch* b, const char* cache_path, sepso_tune* best);
/* Apply a tile configuration to every instance (same bounds as sepso_set_tune,
 * with the smallest waypoint count of the batch). */
sepso_status sepso_batch_set_tune(sepso_batch* b, const sepso_tune* tune);
/* Tiles per bucket of instances: bucket_of[i] in [0, n_buckets) names
 * instance i's bucket (every bucket non-empty, n_buckets <= 8) and tiles[j]
 * bucket j's tile (the sepso_batch_set_tune bounds over its instances).  Each
 * iteration then launches one fused-iteration kernel per bucket (side by side
 * in the frame's captured graph), then the per-instance reduce.  Results do
 * not depend on the bucketing beyond a tile's own summation order of the
 * path length.  Synchronous. */
sepso_status sepso_batch_set_tiles(sepso_batch* b, int32_t n_buckets, const int32_t* bucket_of,
                                   const sepso_tune* tiles);
/* Per-bucket autotuning: the batch's instances are split by waypoint count
 * into at most max_buckets (<= 8) buckets of about equal size; each bucket's
 * tile is the fastest candidate of its own fused-iteration launch (or, with
 * cache_path, a line of the cache file under the bucket's key: the batch key
 * of sepso_autotune_cached taken over the bucket's instances; timed buckets
 * are appended).  One frame from the frame-0 swarm is then planned with the
 * buckets and one with sepso_autotune's single tile; the faster stays.
 * tiles (max_buckets entries) receives the tile of each bucket used,
 * bucket_of (n_inst, may be NULL) each instance's bucket, *n_buckets (may be
 * NULL) the number of buckets (1: one tile for all), frame_ms (2 floats, may
 * be NULL) the device time of the compared frames (buckets, one tile; NaN
 * when the batch has a single waypoint count).  Afterwards the batch is as
 * new, as after sepso_autotune (hyper-parameters as created).  Synchronous. */
sepso_status sepso_autotune_buckets(sepso_batch* b, int32_t max_buckets, const char* cache_path,
                                    sepso_tune* tiles, int32_t* bucket_of, int32_t* n_buckets,
                                    float* frame_ms);
/* Work counters of one full iteration of every instance: segment x edge
 * tests and swarm elements (for throughput reporting). */
sepso_status sepso_batch_work(sepso_batch* b, double* tests_per_iter, double* elems_per_iter);
/* Tbest fitness after each iteration of the last planned frame, per
 * instance: out gets n_inst x 64 floats (entries past the frame's iteration
 * count are stale). */
sepso_status sepso_batch_history(sepso_batch* b, float* out);

/* ---- learned initializer ------------------------------------------------
 * An MLP (BF16 weights and activations, FP32 accumulation on MFMA) maps a
 * 64 x 64 occupancy raster of the map (cell centre inside an obstacle) plus
 * start and target (normalised by the map size) -- 4100 inputs -- through
 * three ReLU layers of 512 to 320 outputs: one initial 20-waypoint path per
 * group for 8 groups, normalised to [0,1].  When attached to a batch it runs
 * at every frame start and takes the place of the previous plan in Priori
 * Initialization (group g's first ceil(gamma*N) particles are drawn within
 * +-pi_radius of proposal g); instances that are not 8 x (N, 20) or whose
 * proposal is not finite fall back to plain Priori Initialization.
 * Parameters (flat FP32): W1 (512 x 4100), b1, W2 (512 x 512), b2, W3, b3,
 * W4 (320 x 512), b4 -- weights row-major (out, in).  Training: MSE against
 * targets, Adam (0.9, 0.999, 1e-8) on FP32 master weights. */
typedef struct sepso_lin sepso_lin;
int64_t sepso_lin_param_count(void);
/* max_rows (multiple of 32): rows of one forward/backward pass (batch
 * instances or minibatch); max_samples: on-device training-set capacity. */
sepso_status sepso_lin_workspace_bytes(int32_t max_rows, int64_t max_samples, size_t* bytes);
/* Weights seeded uniformly in +-1/sqrt(fan_in), biases zero.  Synchronous. */
sepso_status sepso_lin_create(int32_t max_rows, int64_t max_samples, uint64_t seed,
                              void* d_workspace, size_t workspace_bytes, void* stream,
                              sepso_lin** out);
sepso_status sepso_lin_destroy(sepso_lin* lin);
sepso_status sepso_lin_set_weights(sepso_lin* lin, const float* flat);
sepso_status sepso_lin_get_weights(sepso_lin* lin, float* flat);
/* Host rows x (n x 4100, rounded to BF16) -> outputs y (n x 320). */
sepso_status sepso_lin_forward(sepso_lin* lin, const float* x, int32_t n, float* y);
/* Loss and flat parameter gradients for n rows (n a multiple of 32). */
sepso_status sepso_lin_grads(sepso_lin* lin, const float* x, const float* targets, int32_t n,
                             float* loss, float* grads);
/* Append every instance of a planned batch (8 groups x 20 waypoints each)
 * to the training set: its features and its final group bests. */
sepso_status sepso_lin_collect(sepso_lin* lin, sepso_batch* b);
sepso_status sepso_lin_samples(sepso_lin* lin, int64_t* n);
/* steps Adam steps over consecutive minibatches of the training set;
 * loss_out (may be NULL) gets the loss of each step. */
sepso_status sepso_lin_train(sepso_lin* lin, int32_t steps, int32_t batch, float lr,
                             float* loss_out);
/* Network input features of the batch's current maps (n_inst x 4100). */
sepso_status sepso_lin_features(sepso_lin* lin, sepso_batch* b, float* out);
/* Use lin's proposals at every frame start of b (NULL detaches). */
sepso_status sepso_lin_attach(sepso_batch* b, sepso_lin* lin);
sepso_status sepso_lin_attach_ctx(sepso_ctx* ctx, sepso_lin* lin);

/* ---- benchmark-function workload ----------------------------------------
 * Table BFs with the Sec. "Standard / Large-scale benchmark functions" setup:
 * DTPSO (Algorithm 1, Eq.(6)-(8)) minimising func = 1 Sphere, 2 Rosenbrock,
 * 3 Rastrigin, 4 Griewank (textbook definitions, minimum 0) over [lo, hi]^D
 * with G groups of N particles and per-group hyper-parameters (Table hyper8
 * layout).  FP32 state; particle rows padded to a multiple of 4 floats in
 * the workspace.  Random streams: Philox4x32-10, key = seed, counter (c0, c1,
 * s, tag): tags 10 / 11 draw the initial positions / velocities (c0 = 4-value
 * block of the swarm-local flat (particle, dim) index, c1 = 0), tag 9 the move
 * (c0 = swarm-local particle, c1 = ctr, words 0..2 = r1, r2, r3); s is the
 * swarm.  With swarms = S > 1 the handle holds S independent swarms of G
 * groups side by side (group rows s*G .. s*G + G - 1), each with its own
 * Tbest, stepped together: the batched lower levels of the evolution phase
 * and the independent trials of the application phase. */
typedef struct sepso_bf_cfg {
  int32_t func;                  /* 1..4 */
  int32_t groups, particles, dims; /* G in [1, 64] per swarm, N >= 1, D >= 1 */
  int32_t max_iters;             /* T >= 1: inertia schedule length (Eq.6) */
  const float* hyper;            /* S*G x 6 (C1, C2, C3, w_init, w_end, V_limit >= 0) */
  float lo, hi;                  /* search box, lo < hi; V clipped to V_limit (hi - lo) / 2 */
  uint64_t seed;
  int32_t swarms;                /* S independent swarms; 0 or 1 = one */
  int32_t path;                  /* 0: a swarm whose rows (D <= 256) and state fit in 64 KiB of
                                    LDS runs each call's iterations in one launch, one
                                    workgroup per swarm; 1: always two launches per
                                    iteration.  Both give bit-identical results. */
} sepso_bf_cfg;

/* Host views (any pointer may be NULL), with G_all = S*G groups: X, V, P:
 * G_all*N*D row-major; f, Pf: G_all*N; gbest_n, gbest_f: G_all.  tb_* is
 * derived from gbest_f over all groups (lowest group, lowest index on ties).
 * pending = a move is owed before the next evaluation (0 after every
 * sepso_bf_step call). */
typedef struct sepso_bf_state {
  float *X, *V, *P;
  float *f, *Pf;
  int32_t* gbest_n; float* gbest_f;
  int32_t tb_g, tb_n; float tb_f;
  int32_t k;           /* iterations evaluated */
  uint32_t ctr;        /* random-stream position of the move */
  int32_t pending;
} sepso_bf_state;

typedef struct sepso_bf sepso_bf;
sepso_status sepso_bf_workspace_bytes(const sepso_bf_cfg* cfg, size_t* bytes);
/* Validates, initialises the swarm (synchronous); workspace caller-owned,
 * 256-byte aligned; stream NULL = an internal non-blocking stream. */
sepso_status sepso_bf_create(const sepso_bf_cfg* cfg, void* d_workspace, size_t workspace_bytes,
                             void* stream, sepso_bf** out);
sepso_status sepso_bf_destroy(sepso_bf* bf);
/* n iterations of Algorithm 1 (evaluate, bests, move), asynchronous. */
sepso_status sepso_bf_step(sepso_bf* bf, int32_t n);
/* As sepso_bf_step, timed with events on the handle's stream: device
 * milliseconds per iteration (synchronous). */
sepso_status sepso_bf_profile(sepso_bf* bf, int32_t n, float* ms_per_iter);
sepso_status sepso_bf_get_state(sepso_bf* bf, sepso_bf_state* st);
/* Injects state (NULL arrays are left as they are); the Gbest rows are
 * rebuilt from P and gbest_n when both are given.  Synchronous. */
sepso_status sepso_bf_set_state(sepso_bf* bf, const sepso_bf_state* st);

/* ---- evolution phase ------------------------------------------------------
 * Sec. "Hierarchical Self-evolving Framework", Eq.(9), and the path-planning
 * evolution that produced Table hyper8path.  The higher-level swarm H-SEPSO
 * (h_groups x h_particles particles, hyper-parameters h_hyper, Table hyper8 by
 * default) moves, with the DTPSO update of Eq.(6)-(8), over whole lower-level
 * hyper matrices: particle i holds G_L rows of (C1, C2, C3, w_init, w_end,
 * V_limit), row-major, column c boxed to [lo[c], hi[c]].  Its fitness is the
 * lowest fitness value (Tbest fitness after max_iters iterations) of a full
 * lower-level run on `map` with those values: instance i of an internal batch
 * runs one frame per evolution from a fresh random swarm (Philox frame
 * counter = evolution index), with no obstacle motion, Priori Initialization,
 * Auto Truncation or online self-evolution (the template's use_pi, at_mode,
 * hsef_every and instance are overridden; its hyper may be NULL).
 * Random streams of the higher level: Philox4x32-10 with key cfg->seed and
 * counter (c0, c1, 0, tag): tag 7 / 8 draw the initial positions / velocities
 * (c0 = 4-value block of the flat (particle, dim) index, c1 = 0), tag 6 the
 * move (c0 = particle, c1 = evolution counter, words 0..2 = r1, r2, r3). */
typedef struct sepso_evolve_cfg {
  int32_t h_groups;      /* 1..64 */
  int32_t h_particles;   /* per group; h_groups * h_particles <= 1024 */
  int32_t evolutions;    /* E >= 1: inertia schedule length (Eq.6) and curve capacity */
  const float* h_hyper;  /* h_groups x 6, V_limit >= 0; NULL = Table hyper8 rows */
  const float* lo;       /* 6 per-column lower bounds; NULL = 0 for every column */
  const float* hi;       /* 6 per-column upper bounds (> lo); NULL = (3, 3, 3, 1, 1, 1) */
  uint64_t seed;
} sepso_evolve_cfg;

/* Host views of the higher level (any pointer may be NULL).  n = h_groups *
 * h_particles, Dh = 6 * G_L: X, V, P: n x Dh; Pf, lfv: n (lfv = fitness of
 * the last evolution); gbest_n / gbest_f: h_groups. */
typedef struct sepso_evolve_state {
  float *X, *V, *P;
  float *Pf, *lfv;
  int32_t* gbest_n; float* gbest_f;
  int32_t tb_g, tb_n; float tb_f;
  int32_t k;             /* evolutions done */
  uint32_t ctr;          /* random-stream position of the move */
} sepso_evolve_state;

typedef struct sepso_evolve sepso_evolve;
/* Device workspace (caller-owned, 256-byte aligned) for the lower-level batch
 * of n instances plus the higher level's state. */
sepso_status sepso_evolve_workspace_bytes(const sepso_map* map, const sepso_swarm* lower,
                                          const sepso_evolve_cfg* cfg, size_t* bytes);
/* Validates, uploads, and initialises the higher level (synchronous). */
sepso_status sepso_evolve_create(const sepso_map* map, const sepso_swarm* lower,
                                 const sepso_evolve_cfg* cfg, void* d_workspace,
                                 size_t workspace_bytes, void* stream, sepso_evolve** out);
sepso_status sepso_evolve_destroy(sepso_evolve* ev);
/* n evolutions (one captured graph each: lower-level frame of every H
 * particle, then the H bests and move), one synchronisation at the end.
 * curve (n floats, n <= evolutions; may be NULL) receives the total-best LFV
 * after each. */
sepso_status sepso_evolve_run(sepso_evolve* ev, int32_t n, float* curve);
/* One higher-level step with the given fitness values (n floats; non-finite
 * counts as +inf) in place of lower-level runs: a seam for checking the
 * higher level on its own.  Synchronous. */
sepso_status sepso_evolve_inject(sepso_evolve* ev, const float* lfv);
sepso_status sepso_evolve_get_state(sepso_evolve* ev, sepso_evolve_state* st);
/* Best hyper matrix found so far (Dh floats, the total-best H Pbest) and its
 * LFV; SEPSO_E_STATE before the first evolution. */
sepso_status sepso_evolve_best(sepso_evolve* ev, float* hyper, float* lfv);
/* The lower-level batch (owned by ev): for sepso_batch_get_state and tuning. */
sepso_status sepso_evolve_lower(sepso_evolve* ev, sepso_batch** b);

/* ---- evolution phase on the benchmark functions ---------------------------
 * Sec. "Evolution Phase on Benchmark Functions": the same higher level
 * (sepso_evolve_cfg, H state and random streams as above, Dh = 6 G) over
 * benchmark-function lower levels.  H particle i's lower level is swarm i of
 * one sepso_bf handle with S = h_groups * h_particles swarms (lower->swarms
 * and lower->hyper are ignored); every evolution starts each swarm afresh
 * (initial draws with c1 = evolutions done), runs lower->max_iters evaluated
 * iterations with the H particle's values as its (G, 6) hyper matrix, and
 * takes the swarm's lowest fitness value as the particle's fitness (Eq.(9)). */
typedef struct sepso_bf_evolve sepso_bf_evolve;
sepso_status sepso_bf_evolve_workspace_bytes(const sepso_bf_cfg* lower, const sepso_evolve_cfg* cfg,
                                             size_t* bytes);
/* Validates, initialises both levels (synchronous); workspace caller-owned,
 * 256-byte aligned; stream NULL = an internal non-blocking stream. */
sepso_status sepso_bf_evolve_create(const sepso_bf_cfg* lower, const sepso_evolve_cfg* cfg,
                                    void* d_workspace, size_t workspace_bytes, void* stream,
                                    sepso_bf_evolve** out);
sepso_status sepso_bf_evolve_destroy(sepso_bf_evolve* ev);
/* n evolutions (one captured graph each: every swarm's run, their bests, the
 * H step), one synchronisation at the end; curve (n <= evolutions floats, may
 * be NULL) receives the total-best LFV after each. */
sepso_status sepso_bf_evolve_run(sepso_bf_evolve* ev, int32_t n, float* curve);
sepso_status sepso_bf_evolve_get_state(sepso_bf_evolve* ev, sepso_evolve_state* st);
/* Best hyper matrix (Dh floats) and its LFV; SEPSO_E_STATE before the first
 * evolution. */
sepso_status sepso_bf_evolve_best(sepso_bf_evolve* ev, float* hyper, float* lfv);
/* The lower-level handle (owned by ev): for sepso_bf_get_state. */
sepso_status sepso_bf_evolve_lower(sepso_bf_evolve* ev, sepso_bf** bf);

#ifdef __cplusplus
}
#endif
#endif
