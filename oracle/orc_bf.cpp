// SEPSO oracle, benchmark-function workload (Table BFs; Sec. "Standard
// benchmark functions" and "Large-scale benchmark functions"): DTPSO
// (Algorithm 1, Eq.(6)-(8)) minimising Sphere, Rosenbrock, Rastrigin or
// Griewank over the box [lo, hi]^D.  Plain FP64 loops.
//
// TEST INFRASTRUCTURE ONLY (see orc.h).
#include <cmath>
#include <cstring>
#include <limits>

#include "orc.h"

static const double kInf = std::numeric_limits<double>::infinity();
static const double kPi = 3.14159265358979323846;

static void draw4(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t tag, double u[4]) {
  const uint32_t ctr[4] = {c0, c1, c2, tag};
  const uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  for (int i = 0; i < 4; ++i) u[i] = orc_u01(w[i]);
}

// The four functions of Table BFs, textbook definitions (minimum 0 at the
// origin, Rosenbrock at (1, ..., 1)).
double orc_bf_value(int32_t func, int32_t D, const double* x) {
  double s = 0.0;
  switch (func) {
    case ORC_BF_SPHERE:
      for (int32_t i = 0; i < D; ++i) s += x[i] * x[i];
      return s;
    case ORC_BF_ROSENBROCK:
      for (int32_t i = 0; i + 1 < D; ++i) {
        const double a = x[i + 1] - x[i] * x[i], b = 1.0 - x[i];
        s += 100.0 * a * a + b * b;
      }
      return s;
    case ORC_BF_RASTRIGIN:
      for (int32_t i = 0; i < D; ++i) s += x[i] * x[i] - 10.0 * std::cos(2.0 * kPi * x[i]);
      return 10.0 * D + s;
    case ORC_BF_GRIEWANK: {
      double p = 1.0;
      for (int32_t i = 0; i < D; ++i) {
        s += x[i] * x[i] / 4000.0;
        p *= std::cos(x[i] / std::sqrt((double)(i + 1)));
      }
      return 1.0 + s - p;
    }
    default:
      return std::numeric_limits<double>::quiet_NaN();
  }
}

void orc_bf_init(orc_bf* s) {
  const int32_t G = s->G, N = s->N, D = s->D, nb = (D + 3) / 4;
  const double lo = s->lo, hi = s->hi;
  for (int32_t g = 0; g < G; ++g) {
    const double vmax = s->hyper[6 * g + 5] * (hi - lo) / 2.0;
    for (int32_t n = 0; n < N; ++n) {
      const int32_t i = g * N + n;
      for (int32_t d = 0; d < D; ++d) {
        double ux[4], uv[4];
        const uint32_t c0 = (uint32_t)(i * nb + d / 4);
        draw4(s->seed, c0, s->run, s->instance, ORC_TAG_BF_INIT_X, ux);
        draw4(s->seed, c0, s->run, s->instance, ORC_TAG_BF_INIT_V, uv);
        const double x = lo + ux[d % 4] * (hi - lo);
        s->X[(size_t)i * D + d] = x;
        s->P[(size_t)i * D + d] = x;
        s->V[(size_t)i * D + d] = -vmax + uv[d % 4] * (2.0 * vmax);
      }
      s->f[i] = kInf;
      s->Pf[i] = kInf;
    }
    s->gbest_n[g] = 0;
    s->gbest_f[g] = kInf;
  }
  s->tb_g = s->tb_n = 0;
  s->tb_f = kInf;
  s->k = 0;
  s->ctr = 0;
}

// Fitness of every particle's current position.
void orc_bf_eval(orc_bf* s) {
  for (int32_t i = 0; i < s->G * s->N; ++i) {
    const double fi = orc_bf_value(s->func, s->D, s->X + (size_t)i * s->D);
    s->f[i] = std::isfinite(fi) ? fi : kInf;
  }
}

// Bests from the fitness in f (Pbest on strict improvement, Gbest the
// group's lowest Pbest, lowest index on ties, Tbest the lowest Gbest), then
// the move of Eq.(6)-(8) with iteration index k.
void orc_bf_advance(orc_bf* s) {
  const int32_t G = s->G, N = s->N, D = s->D;
  for (int32_t i = 0; i < G * N; ++i) {
    const double fi = std::isfinite(s->f[i]) ? s->f[i] : kInf;
    if (fi < s->Pf[i]) {
      s->Pf[i] = fi;
      std::memcpy(s->P + (size_t)i * D, s->X + (size_t)i * D, sizeof(double) * D);
    }
  }
  for (int32_t g = 0; g < G; ++g) {
    int32_t b = 0;
    for (int32_t n = 1; n < N; ++n)
      if (s->Pf[g * N + n] < s->Pf[g * N + b]) b = n;
    s->gbest_n[g] = b;
    s->gbest_f[g] = s->Pf[g * N + b];
  }
  int32_t tg = 0;
  for (int32_t g = 1; g < G; ++g)
    if (s->gbest_f[g] < s->gbest_f[tg]) tg = g;
  s->tb_g = tg;
  s->tb_n = s->gbest_n[tg];
  s->tb_f = s->gbest_f[tg];

  const int32_t k = s->k < s->T ? s->k : s->T;
  const double lo = s->lo, hi = s->hi;
  const double* Tb = s->P + (size_t)(tg * N + s->tb_n) * D;
  for (int32_t g = 0; g < G; ++g) {
    const double* h = s->hyper + 6 * g;
    const double C1 = h[0], C2 = h[1], C3 = h[2], wi = h[3], we = h[4];
    const double vmax = h[5] * (hi - lo) / 2.0;
    const double w = wi - (wi - we) / (double)s->T * (double)k;  // Eq.(6)
    const double* Gb = s->P + (size_t)(g * N + s->gbest_n[g]) * D;
    for (int32_t n = 0; n < N; ++n) {
      const int32_t i = g * N + n;
      double r[4];
      draw4(s->seed, (uint32_t)i, s->ctr, s->instance, ORC_TAG_BF_UPDATE, r);
      double* x = s->X + (size_t)i * D;
      double* v = s->V + (size_t)i * D;
      const double* p = s->P + (size_t)i * D;
      for (int32_t d = 0; d < D; ++d) {
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
  s->ctr += 1;
}

// One Algorithm-1 iteration: evaluate, bests, then the move.
void orc_bf_step(orc_bf* s) {
  s->k += 1;
  orc_bf_eval(s);
  orc_bf_advance(s);
}
