/*
 * SEPSO oracle: plain, slow, single-threaded FP64 reference of the planner's
 * hot path.  TEST INFRASTRUCTURE ONLY: nothing in the product library may
 * include, link or call this code; only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark do.  It shares no code with the HIP path.
 *
 * Paper: "Efficient Real-time Path Planning with Self-evolving Particle Swarm
 * Optimization in Dynamic Scenarios" (Xin, Li, Zhang, Li).  Citations below
 * name the paper's section, equation, algorithm or table.
 *
 * Conventions shared with the GPU path by *specification* (not by code):
 *   - particle layout, Eq.(10): X[g][n][0..W-1] = x_1..x_W, X[g][n][W..2W-1] = y_1..y_W
 *   - random numbers: Philox4x32-10 (Salmon et al., SC'11), key = seed,
 *     counter = (c0, c1, c2 = instance, c3 = tag), u = (word >> 8) * 2^-24.
 */
#ifndef SEPSO_ORACLE_H
#define SEPSO_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox counter tags (which stream a draw belongs to). */
enum { ORC_TAG_UPDATE = 0, ORC_TAG_INIT_X = 1, ORC_TAG_INIT_V = 2, ORC_TAG_PI = 3,
       ORC_TAG_HSEF = 4, ORC_TAG_LEARNED = 5, ORC_TAG_EVOLVE = 6, ORC_TAG_EVOLVE_X = 7,
       ORC_TAG_EVOLVE_V = 8, ORC_TAG_BF_UPDATE = 9, ORC_TAG_BF_INIT_X = 10,
       ORC_TAG_BF_INIT_V = 11, ORC_TAG_UPDATE_DIM = 12 };

/* Philox4x32 with 10 rounds, written from Salmon et al. (SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* 24-bit uniform in [0,1): exact in FP32 and FP64. */
double orc_u01(uint32_t word);

/* Polygonal map, Sec. "Map representation": obstacles are closed polygons
 * (CSR over vertices), path runs from start to target. */
typedef struct orc_map {
  double width, height;
  int32_t n_polys;
  const int32_t* poly_ptr; /* n_polys + 1 */
  const double* verts;     /* n_vert * 2, (x, y) */
  double start[2], target[2];
} orc_map;

/* Exact-orientation classification of one segment x edge test:
 * 1 = robust crossing, 0 = robust non-crossing, -1 = degenerate (|orient| < tau). */
int32_t orc_classify(const double p[2], const double q[2], const double a[2],
                     const double b[2], double tau);
/* Strict proper-crossing predicate in FP64 (o1*o2 < 0 and o3*o4 < 0). */
int32_t orc_crosses(const double p[2], const double q[2], const double a[2], const double b[2]);

/* Fitness, Eq.(11)-(13), of n_paths paths of W interior waypoints each.
 * Outputs (any may be NULL): f = L + alpha*Q^beta with Q the FP64 strict
 * count, L (Eq.12), Q (strict FP64 count), q_yes (robust crossings) and
 * n_deg (degenerate tests) under threshold tau. */
void orc_fitness(const orc_map* m, int32_t n_paths, int32_t W, const double* X,
                 double alpha, int32_t beta, double tau, double* f, double* L,
                 int32_t* Q, int32_t* q_yes, int32_t* n_deg);

/* Swarm state of one planning instance (DTPSO, Algorithm 1). All arrays are
 * owned by the caller. */
typedef struct orc_swarm {
  int32_t G, N, W, T;      /* groups, particles per group, waypoints, iterations */
  double width, height;    /* search box [0,width] x [0,height] */
  double* hyper;           /* G*6: C1, C2, C3, w_init, w_end, V_limit */
  double alpha; int32_t beta;
  uint64_t seed; uint32_t instance;
  double *X, *V, *P;       /* G*N*D */
  double *f, *L;           /* G*N: last evaluated fitness and length */
  int32_t* Q;              /* G*N: last evaluated crossing count */
  double *Pf, *PL;         /* G*N: fitness and length at Pbest */
  int32_t* PQ;             /* G*N: crossing count at Pbest */
  int32_t* gbest_n;        /* G */
  double* gbest_f;         /* G */
  int32_t tbest_g, tbest_n;
  double tbest_f;
  int32_t k;               /* iteration index within the current plan */
  uint32_t ctr;            /* global iteration counter (random stream position) */
  int32_t rand_per_dim;    /* 0: one (r1, r2, r3) per particle; 1: one per coordinate,
                              counter (particle*2W + coordinate, ctr, instance, UPDATE_DIM) */
} orc_swarm;

void orc_eval(orc_swarm* s, const orc_map* m);        /* f, L, Q of X */
void orc_bests(orc_swarm* s);                          /* Pbest, Gbest, Tbest from f */
void orc_update(orc_swarm* s);                         /* omega, V, X update */
void orc_step(orc_swarm* s, const orc_map* m);         /* one Algorithm-1 iteration */
/* Initialise X, V (frame index `frame`); prev_path != NULL enables Priori
 * Initialisation of the first ceil(gamma*N) particles of each group. */
void orc_init(orc_swarm* s, int32_t frame, const double* prev_path, double pi_gamma,
              double pi_radius);

/* Online hierarchical self-evolution state (outer swarm over each group's
 * (w_init, C1, C2)). */
typedef struct orc_hsef {
  const double* outer_hyper; /* G*6 hyper of the outer swarm (Table hyper8 rows) */
  double* ov;                /* G*3 outer velocities */
  double* op;                /* G*3 outer Pbest positions */
  double* opf;               /* G outer Pbest fitness */
  int32_t otb;               /* outer total-best index */
  int32_t epoch_in_frame, T_outer;
  uint32_t epoch_ctr;        /* global outer-step counter (random stream position) */
} orc_hsef;
void orc_hsef_reset_frame(const orc_swarm* s, orc_hsef* h);
void orc_hsef_step(orc_swarm* s, orc_hsef* h);

/* Auto Truncation decision after iteration k (1-based); hist[i] = Tbest
 * fitness after iteration i+1. mode 1: population std over the last `window`
 * values < delta; mode 2: hist[k-window] - hist[k] < delta*max(1,|hist[k]|);
 * mode 3: as mode 1 over the last min(k, window) values once k >= 2.
 * All require the current best path to be collision-free. */
int32_t orc_at_check(const double* hist, int32_t k, int32_t mode, int32_t window,
                     double delta, int32_t q_tbest);

/* Obstacle / endpoint motion for one frame (reflecting walls). Mutates the
 * vertices, velocities and endpoints in place. */
void orc_sim_step(double width, double height, int32_t n_polys, const int32_t* poly_ptr,
                  double* verts, double* poly_vel, double* start, double* target,
                  double* endpoint_vel);

typedef struct orc_frame_cfg {
  int32_t use_pi; double pi_gamma, pi_radius;
  int32_t at_mode, at_window; double at_delta;
  int32_t hsef_every;
} orc_frame_cfg;

typedef struct orc_frame_result {
  double cost, length;
  int32_t crossings, iters, truncated;
} orc_frame_result;

/* One application-phase frame: init (PI when frame > 0 and enabled), then
 * iterations with AT and online HSEF until truncation or T. prev_path is the
 * previous frame's best path (D values) or NULL; out_path receives this
 * frame's best path; hist is scratch of T doubles. */
void orc_plan_frame(orc_swarm* s, orc_hsef* h, const orc_map* m, const orc_frame_cfg* c,
                    int32_t frame, const double* prev_path, double* out_path, double* hist,
                    orc_frame_result* res);

/* Evolution phase, Sec. "Hierarchical Self-evolving Framework" / Eq.(9):
 * the higher-level swarm H-SEPSO (Gh groups of Nh particles, hyper-parameters
 * h_hyper, Table hyper8) moves over whole lower-level hyper matrices (Dh =
 * 6*G_L values, row-major (G_L, 6)); column c of a row is boxed to
 * [lo[c], hi[c]].  Its fitness is the lower level's lowest fitness value
 * after a full run, supplied by the caller.  Random streams: counter
 * (c0, c1, 0, tag) with tags EVOLVE_X / EVOLVE_V (init, c1 = 0) and EVOLVE
 * (move, c0 = H particle, c1 = ctr).  All arrays owned by the caller. */
typedef struct orc_evolve {
  int32_t Gh, Nh, Dh, E;     /* E: evolutions of the inertia schedule, Eq.(6) */
  const double* h_hyper;     /* Gh*6 */
  const double* lo;          /* 6: per-column lower bound */
  const double* hi;          /* 6: per-column upper bound */
  uint64_t seed;
  double *X, *V, *P;         /* Gh*Nh*Dh */
  double* Pf;                /* Gh*Nh */
  int32_t* gbest_n;          /* Gh */
  double* gbest_f;           /* Gh */
  int32_t tb_g, tb_n;
  double tb_f;
  int32_t k;                 /* evolutions done */
  uint32_t ctr;              /* random stream position of the move */
} orc_evolve;
void orc_evolve_init(orc_evolve* h);
/* bests from lfv (Gh*Nh values) then the move of Eq.(6)-(8) */
void orc_evolve_step(orc_evolve* h, const double* lfv);

/* Benchmark-function workload (Table BFs): DTPSO over [lo, hi]^D on one of
 * the four functions.  Random streams: counter (c0, c1, instance, tag), tags
 * BF_INIT_X / BF_INIT_V (c0 = 4-value block of the flat index, c1 = run) and
 * BF_UPDATE (c0 = particle, c1 = ctr). */
enum { ORC_BF_SPHERE = 1, ORC_BF_ROSENBROCK = 2, ORC_BF_RASTRIGIN = 3, ORC_BF_GRIEWANK = 4 };
double orc_bf_value(int32_t func, int32_t D, const double* x);
typedef struct orc_bf {
  int32_t func, G, N, D, T;
  double lo, hi;
  const double* hyper;       /* G*6 (Table hyper8 rows) */
  uint64_t seed;
  double *X, *V, *P;         /* G*N*D */
  double *f, *Pf;            /* G*N */
  int32_t* gbest_n;          /* G */
  double* gbest_f;           /* G */
  int32_t tb_g, tb_n;
  double tb_f;
  int32_t k;
  uint32_t ctr;
  uint32_t instance;         /* counter word 2 of every draw: independent swarms */
  uint32_t run;              /* counter word 1 of the initial draws: independent runs */
} orc_bf;
void orc_bf_init(orc_bf* s);
void orc_bf_eval(orc_bf* s);     /* f = function value of X */
void orc_bf_advance(orc_bf* s);  /* bests from f, then the move with index k; ctr += 1 */
void orc_bf_step(orc_bf* s);     /* k += 1, eval, advance (Algorithm 1) */

#ifdef __cplusplus
}
#endif
#endif
