// SEPSO oracle, core: random numbers, geometry/fitness and one DTPSO
// iteration.  TEST INFRASTRUCTURE ONLY (see orc.h).  Plain FP64, one thread,
// no blocking or reordering beyond what the paper's definitions state.
#include "orc.h"

#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

static const double kInf = std::numeric_limits<double>::infinity();

// ---------------------------------------------------------------------------
// Philox4x32-10, from the description in Salmon, Moraes, Dror, Shaw,
// "Parallel Random Numbers: As Easy as 1, 2, 3" (SC'11): each round multiplies
// words 0 and 2 by two fixed odd constants, keeps the low halves as the new
// words 1 and 3, and mixes the high halves with the other two words and the
// round key; the 2-word key is bumped by two Weyl constants between rounds.
// ---------------------------------------------------------------------------
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint64_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t p0 = M0 * (uint64_t)c0;
    const uint64_t p1 = M1 * (uint64_t)c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

double orc_u01(uint32_t word) { return (double)(word >> 8) * (1.0 / 16777216.0); }

static void draw4(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t inst, uint32_t tag,
                  double u[4]) {
  const uint32_t ctr[4] = {c0, c1, inst, tag};
  const uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  for (int i = 0; i < 4; ++i) u[i] = orc_u01(w[i]);
}

// ---------------------------------------------------------------------------
// Geometry, Sec. "Map representation" and Eq.(11)-(13): a path collides with
// an obstacle where one of its segments properly crosses one of the polygon's
// edges; Q counts every such (segment, edge) pair.
// ---------------------------------------------------------------------------

// Signed doubled area of triangle (a, b, c): > 0 when c is left of a->b.
static double orient(const double a[2], const double b[2], const double c[2]) {
  return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]);
}

static bool opposite(double s, double t) { return (s < 0.0 && t > 0.0) || (s > 0.0 && t < 0.0); }
static bool same_side(double s, double t) { return (s < 0.0 && t < 0.0) || (s > 0.0 && t > 0.0); }

int32_t orc_crosses(const double p[2], const double q[2], const double a[2], const double b[2]) {
  const double o1 = orient(p, q, a), o2 = orient(p, q, b);
  const double o3 = orient(a, b, p), o4 = orient(a, b, q);
  return opposite(o1, o2) && opposite(o3, o4) ? 1 : 0;
}

int32_t orc_classify(const double p[2], const double q[2], const double a[2], const double b[2],
                     double tau) {
  if (p[0] == q[0] && p[1] == q[1]) return 0;  // a point crosses nothing
  const double o1 = orient(p, q, a), o2 = orient(p, q, b);
  const double o3 = orient(a, b, p), o4 = orient(a, b, q);
  const bool big12 = std::fabs(o1) >= tau && std::fabs(o2) >= tau;
  const bool big34 = std::fabs(o3) >= tau && std::fabs(o4) >= tau;
  if ((big12 && same_side(o1, o2)) || (big34 && same_side(o3, o4))) return 0;
  if (big12 && big34 && opposite(o1, o2) && opposite(o3, o4)) return 1;
  return -1;
}

static double int_pow(int32_t q, int32_t beta) {
  double r = 1.0;
  for (int32_t i = 0; i < beta; ++i) r *= (double)q;
  return r;
}

void orc_fitness(const orc_map* m, int32_t n_paths, int32_t W, const double* X, double alpha,
                 int32_t beta, double tau, double* f, double* L, int32_t* Q, int32_t* q_yes,
                 int32_t* n_deg) {
  const int32_t D = 2 * W;
  std::vector<double> pts(2 * (W + 2));
  for (int32_t pi = 0; pi < n_paths; ++pi) {
    const double* x = X + (size_t)pi * D;
    // Path points: start, the W interior waypoints of Eq.(10), target.
    pts[0] = m->start[0];
    pts[1] = m->start[1];
    for (int32_t i = 0; i < W; ++i) {
      pts[2 * (i + 1)] = x[i];
      pts[2 * (i + 1) + 1] = x[W + i];
    }
    pts[2 * (W + 1)] = m->target[0];
    pts[2 * (W + 1) + 1] = m->target[1];

    // Eq.(12): sum of the W+1 leg lengths.
    double len = 0.0;
    for (int32_t i = 0; i <= W; ++i) {
      const double dx = pts[2 * (i + 1)] - pts[2 * i];
      const double dy = pts[2 * (i + 1) + 1] - pts[2 * i + 1];
      len += std::sqrt(dx * dx + dy * dy);
    }

    // Eq.(13): Q = number of (path segment, obstacle edge) crossings.
    int32_t q = 0, yes = 0, deg = 0;
    for (int32_t i = 0; i <= W; ++i) {
      const double* p = &pts[2 * i];
      const double* r = &pts[2 * (i + 1)];
      for (int32_t poly = 0; poly < m->n_polys; ++poly) {
        const int32_t v0 = m->poly_ptr[poly], v1 = m->poly_ptr[poly + 1];
        const int32_t nv = v1 - v0;
        for (int32_t j = 0; j < nv; ++j) {
          const double* a = m->verts + 2 * (v0 + j);
          const double* b = m->verts + 2 * (v0 + (j + 1) % nv);
          q += orc_crosses(p, r, a, b);
          const int32_t c = orc_classify(p, r, a, b, tau);
          if (c == 1) ++yes;
          if (c < 0) ++deg;
        }
      }
    }
    if (f) f[pi] = len + alpha * int_pow(q, beta);
    if (L) L[pi] = len;
    if (Q) Q[pi] = q;
    if (q_yes) q_yes[pi] = yes;
    if (n_deg) n_deg[pi] = deg;
  }
}

// ---------------------------------------------------------------------------
// DTPSO iteration, Algorithm 1 with the grouped update of Eq.(4)-(5) in its
// tensor form Eq.(6)-(8).
// ---------------------------------------------------------------------------

static double map_hi(const orc_swarm* s, int32_t d) { return d < s->W ? s->width : s->height; }

void orc_eval(orc_swarm* s, const orc_map* m) {
  const int32_t P = s->G * s->N;
  const double S = m->width > m->height ? m->width : m->height;
  orc_fitness(m, P, s->W, s->X, s->alpha, s->beta, 1e-6 * S * S, s->f, s->L, s->Q, nullptr,
              nullptr);
}

// Algorithm 1, "update P, G, T when better fitness is identified": Pbest is
// the historical best of each particle (strictly better replaces it), Gbest
// the best Pbest of each group, Tbest the best over all groups; ties keep the
// lowest index.
void orc_bests(orc_swarm* s) {
  const int32_t G = s->G, N = s->N, D = 2 * s->W;
  for (int32_t i = 0; i < G * N; ++i) {
    double fi = s->f[i];
    if (!std::isfinite(fi)) fi = kInf;
    if (fi < s->Pf[i]) {
      std::memcpy(s->P + (size_t)i * D, s->X + (size_t)i * D, sizeof(double) * D);
      s->Pf[i] = fi;
      s->PL[i] = s->L[i];
      s->PQ[i] = s->Q[i];
    }
  }
  for (int32_t g = 0; g < G; ++g) {
    int32_t best = 0;
    for (int32_t n = 1; n < N; ++n)
      if (s->Pf[g * N + n] < s->Pf[g * N + best]) best = n;
    s->gbest_n[g] = best;
    s->gbest_f[g] = s->Pf[g * N + best];
  }
  int32_t tg = 0;
  for (int32_t g = 1; g < G; ++g)
    if (s->gbest_f[g] < s->gbest_f[tg]) tg = g;
  s->tbest_g = tg;
  s->tbest_n = s->gbest_n[tg];
  s->tbest_f = s->gbest_f[tg];
}

// Eq.(6): per-group linearly decreasing inertia; Eq.(4)/(7): velocity from
// inertia plus the Pbest, Gbest and Tbest attractors, one random factor per
// particle and attractor (R is (4,G,N) in Table EXP_TOF); velocity clipped to
// +-V_limit * half the box extent; Eq.(5)/(8): position step, clipped to the box.
void orc_update(orc_swarm* s) {
  const int32_t G = s->G, N = s->N, W = s->W, D = 2 * W;
  const int32_t k = s->k < s->T ? s->k : s->T;
  const double* Tb = s->P + (size_t)(s->tbest_g * N + s->tbest_n) * D;
  for (int32_t g = 0; g < G; ++g) {
    const double* h = s->hyper + 6 * g;
    const double C1 = h[0], C2 = h[1], C3 = h[2], wi = h[3], we = h[4], vl = h[5];
    const double w = wi - (wi - we) / (double)s->T * (double)k;
    const double* Gb = s->P + (size_t)(g * N + s->gbest_n[g]) * D;
    for (int32_t n = 0; n < N; ++n) {
      const int32_t i = g * N + n;
      double r[4];
      draw4(s->seed, (uint32_t)i, s->ctr, s->instance, ORC_TAG_UPDATE, r);
      double* x = s->X + (size_t)i * D;
      double* v = s->V + (size_t)i * D;
      const double* p = s->P + (size_t)i * D;
      for (int32_t d = 0; d < D; ++d) {
        if (s->rand_per_dim)  // variant: independent factors per coordinate
          draw4(s->seed, (uint32_t)(i * D + d), s->ctr, s->instance, ORC_TAG_UPDATE_DIM, r);
        const double hi = map_hi(s, d);
        const double vmax = vl * hi / 2.0;
        double vn = w * v[d] + C1 * r[0] * (p[d] - x[d]) + C2 * r[1] * (Gb[d] - x[d]) +
                    C3 * r[2] * (Tb[d] - x[d]);
        vn = vn < -vmax ? -vmax : (vn > vmax ? vmax : vn);
        double xn = x[d] + vn;
        xn = xn < 0.0 ? 0.0 : (xn > hi ? hi : xn);
        v[d] = vn;
        x[d] = xn;
      }
    }
  }
}

void orc_step(orc_swarm* s, const orc_map* m) {
  s->k += 1;
  orc_eval(s, m);
  orc_bests(s);
  orc_update(s);
  s->ctr += 1;
}

// Initial swarm: uniform positions in the box and uniform velocities in
// +-vmax.  With a previous plan, Priori Initialisation (Sec. "Priori
// Initialization") places the first ceil(gamma*N) particles of every group
// uniformly within +-radius of that plan instead.
void orc_init(orc_swarm* s, int32_t frame, const double* prev_path, double pi_gamma,
              double pi_radius) {
  const int32_t G = s->G, N = s->N, W = s->W, D = 2 * W;
  const int32_t nb = (D + 3) / 4;
  const int32_t n_pi = prev_path ? (int32_t)std::ceil(pi_gamma * (double)N) : 0;
  for (int32_t g = 0; g < G; ++g) {
    const double vl = s->hyper[6 * g + 5];
    for (int32_t n = 0; n < N; ++n) {
      const int32_t i = g * N + n;
      for (int32_t d = 0; d < D; ++d) {
        const uint32_t c0 = (uint32_t)(i * nb + d / 4);
        const double hi = map_hi(s, d), vmax = vl * hi / 2.0;
        double ux[4], uv[4];
        draw4(s->seed, c0, (uint32_t)frame, s->instance, ORC_TAG_INIT_X, ux);
        draw4(s->seed, c0, (uint32_t)frame, s->instance, ORC_TAG_INIT_V, uv);
        double x = 0.0 + ux[d % 4] * (hi - 0.0);
        if (n < n_pi) {
          double up[4];
          draw4(s->seed, c0, (uint32_t)frame, s->instance, ORC_TAG_PI, up);
          x = prev_path[d] + (-pi_radius + up[d % 4] * (2.0 * pi_radius));
          x = x < 0.0 ? 0.0 : (x > hi ? hi : x);
        }
        s->X[(size_t)i * D + d] = x;
        s->V[(size_t)i * D + d] = -vmax + uv[d % 4] * (2.0 * vmax);
        s->P[(size_t)i * D + d] = x;
      }
      s->Pf[i] = kInf;
      s->PL[i] = kInf;
      s->PQ[i] = 0;
      s->f[i] = kInf;
      s->L[i] = kInf;
      s->Q[i] = 0;
    }
    s->gbest_n[g] = 0;
    s->gbest_f[g] = kInf;
  }
  s->tbest_g = 0;
  s->tbest_n = 0;
  s->tbest_f = kInf;
  s->k = 0;
}

// Many Philox calls at once (statistics and cross-implementation tests).
extern "C" void orc_philox_many(int64_t n, const uint32_t* ctrs, const uint32_t key[2],
                                uint32_t* out) {
  for (int64_t i = 0; i < n; ++i) orc_philox4x32_10(ctrs + 4 * i, key, out + 4 * i);
}
