// SEPSO oracle, evolution phase (Sec. "Hierarchical Self-evolving Framework",
// Eq.(9)): the higher-level swarm H-SEPSO is a DTPSO whose particles are whole
// hyper-parameter matrices of the lower-level swarm (G_L rows of C1, C2, C3,
// w_init, w_end, V_limit, flattened row by row) and whose fitness is the
// lowest fitness value the lower-level swarm reaches with them.  The lower
// level runs are the caller's (one orc_plan_frame per H particle); this file
// holds the higher level: initialisation, bests and the move.
//
// TEST INFRASTRUCTURE ONLY (see orc.h).
#include <cmath>
#include <cstring>
#include <limits>

#include "orc.h"

static const double kInf = std::numeric_limits<double>::infinity();

static void draw4(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t tag, double u[4]) {
  const uint32_t ctr[4] = {c0, c1, 0u, tag};
  const uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  for (int i = 0; i < 4; ++i) u[i] = orc_u01(w[i]);
}

// Uniform positions in the per-column box [lo, hi] and velocities in
// +-V_limit * half the column's extent (V_limit of the particle's H group).
void orc_evolve_init(orc_evolve* h) {
  const int32_t Dh = h->Dh, nb = (Dh + 3) / 4;
  for (int32_t g = 0; g < h->Gh; ++g) {
    const double vl = h->h_hyper[6 * g + 5];
    for (int32_t n = 0; n < h->Nh; ++n) {
      const int32_t i = g * h->Nh + n;
      for (int32_t d = 0; d < Dh; ++d) {
        const double lo = h->lo[d % 6], hi = h->hi[d % 6], vmax = vl * (hi - lo) / 2.0;
        double ux[4], uv[4];
        const uint32_t c0 = (uint32_t)(i * nb + d / 4);
        draw4(h->seed, c0, 0u, ORC_TAG_EVOLVE_X, ux);
        draw4(h->seed, c0, 0u, ORC_TAG_EVOLVE_V, uv);
        const double x = lo + ux[d % 4] * (hi - lo);
        h->X[(size_t)i * Dh + d] = x;
        h->P[(size_t)i * Dh + d] = x;
        h->V[(size_t)i * Dh + d] = -vmax + uv[d % 4] * (2.0 * vmax);
      }
      h->Pf[i] = kInf;
    }
    h->gbest_n[g] = 0;
    h->gbest_f[g] = kInf;
  }
  h->tb_g = h->tb_n = 0;
  h->tb_f = kInf;
  h->k = 0;
  h->ctr = 0;
}

// One evolution after the lower-level runs: Algorithm 1's bests and move with
// the H particles, fitness lfv[i] of particle i (non-finite counts as +inf).
void orc_evolve_step(orc_evolve* h, const double* lfv) {
  const int32_t Gh = h->Gh, Nh = h->Nh, Dh = h->Dh;
  h->k += 1;
  for (int32_t i = 0; i < Gh * Nh; ++i) {
    const double fi = std::isfinite(lfv[i]) ? lfv[i] : kInf;
    if (fi < h->Pf[i]) {
      h->Pf[i] = fi;
      std::memcpy(h->P + (size_t)i * Dh, h->X + (size_t)i * Dh, sizeof(double) * Dh);
    }
  }
  for (int32_t g = 0; g < Gh; ++g) {
    int32_t b = 0;
    for (int32_t n = 1; n < Nh; ++n)
      if (h->Pf[g * Nh + n] < h->Pf[g * Nh + b]) b = n;
    h->gbest_n[g] = b;
    h->gbest_f[g] = h->Pf[g * Nh + b];
  }
  int32_t tg = 0;
  for (int32_t g = 1; g < Gh; ++g)
    if (h->gbest_f[g] < h->gbest_f[tg]) tg = g;
  h->tb_g = tg;
  h->tb_n = h->gbest_n[tg];
  h->tb_f = h->gbest_f[tg];

  const int32_t k = h->k < h->E ? h->k : h->E;
  const double* Tb = h->P + (size_t)(tg * Nh + h->tb_n) * Dh;
  for (int32_t g = 0; g < Gh; ++g) {
    const double* hy = h->h_hyper + 6 * g;
    const double C1 = hy[0], C2 = hy[1], C3 = hy[2], wi = hy[3], we = hy[4], vl = hy[5];
    const double w = wi - (wi - we) / (double)h->E * (double)k;  // Eq.(6)
    const double* Gb = h->P + (size_t)(g * Nh + h->gbest_n[g]) * Dh;
    for (int32_t n = 0; n < Nh; ++n) {
      const int32_t i = g * Nh + n;
      double r[4];
      draw4(h->seed, (uint32_t)i, h->ctr, ORC_TAG_EVOLVE, r);
      double* x = h->X + (size_t)i * Dh;
      double* v = h->V + (size_t)i * Dh;
      const double* p = h->P + (size_t)i * Dh;
      for (int32_t d = 0; d < Dh; ++d) {
        const double lo = h->lo[d % 6], hi = h->hi[d % 6], vmax = vl * (hi - lo) / 2.0;
        double vn = w * v[d] + C1 * r[0] * (p[d] - x[d]) + C2 * r[1] * (Gb[d] - x[d]) +
                    C3 * r[2] * (Tb[d] - x[d]);  // Eq.(7)
        vn = vn < -vmax ? -vmax : (vn > vmax ? vmax : vn);
        double xn = x[d] + vn;  // Eq.(8)
        xn = xn < lo ? lo : (xn > hi ? hi : xn);
        v[d] = vn;
        x[d] = xn;
      }
    }
  }
  h->ctr += 1;
}
