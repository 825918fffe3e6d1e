// SEPSO oracle, application-phase frame loop: online hierarchical
// self-evolution, Auto Truncation, obstacle motion and one planning frame.
// TEST INFRASTRUCTURE ONLY (see orc.h).  Plain FP64, one thread.
#include <cmath>
#include <limits>

#include "orc.h"

static const double kInf = std::numeric_limits<double>::infinity();

static void draw4(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t inst, uint32_t tag,
                  double u[4]) {
  const uint32_t ctr[4] = {c0, c1, inst, tag};
  const uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  for (int i = 0; i < 4; ++i) u[i] = orc_u01(w[i]);
}

static double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

// Outer particle g carries group g's (w_init, C1, C2); the three columns of
// the (G,6) hyper-matrix that the outer swarm moves.
static const int kOuterCol[3] = {3, 0, 1};

static void outer_bounds(const orc_swarm* s, int32_t g, int j, double* lo, double* hi) {
  if (j == 0) {  // w_init stays within [w_end, 1]
    *lo = s->hyper[6 * g + 4];
    *hi = 1.0;
  } else {  // acceleration constants within [0, 3]
    *lo = 0.0;
    *hi = 3.0;
  }
}

// Each frame restarts the outer swarm's memory: the map changed, so old
// Lowest-Fitness-Values (Eq.9) no longer compare with new ones.
void orc_hsef_reset_frame(const orc_swarm* s, orc_hsef* h) {
  for (int32_t g = 0; g < s->G; ++g) {
    for (int j = 0; j < 3; ++j) {
      h->op[3 * g + j] = s->hyper[6 * g + kOuterCol[j]];
      h->ov[3 * g + j] = 0.0;
    }
    h->opf[g] = kInf;
  }
  h->otb = 0;
  h->epoch_in_frame = 0;
}

// One outer (H-SEPSO) step, Sec. "Hierarchical Self-evolving Framework": the
// outer particles are hyper-parameter sets, their fitness is the lowest
// fitness value the inner swarm reached with them (Eq.9; here each group's
// current best), and they move by the same grouped update, Eq.(4)-(6), with
// each outer particle forming its own group and the outer swarm using the
// fixed DTPSO defaults (Table hyper8).
void orc_hsef_step(orc_swarm* s, orc_hsef* h) {
  const int32_t G = s->G;
  for (int32_t g = 0; g < G; ++g) {
    double F = s->gbest_f[g];
    if (!std::isfinite(F)) F = kInf;
    if (F < h->opf[g]) {
      h->opf[g] = F;
      for (int j = 0; j < 3; ++j) h->op[3 * g + j] = s->hyper[6 * g + kOuterCol[j]];
    }
  }
  int32_t tb = 0;
  for (int32_t g = 1; g < G; ++g)
    if (h->opf[g] < h->opf[tb]) tb = g;
  h->otb = tb;
  h->epoch_in_frame += 1;
  const int32_t e = h->epoch_in_frame < h->T_outer ? h->epoch_in_frame : h->T_outer;
  for (int32_t g = 0; g < G; ++g) {
    const double* oh = h->outer_hyper + 6 * g;
    const double C1 = oh[0], C2 = oh[1], C3 = oh[2], wi = oh[3], we = oh[4], vl = oh[5];
    const double w = wi - (wi - we) / (double)h->T_outer * (double)e;
    double r[4];
    draw4(s->seed, (uint32_t)g, h->epoch_ctr, s->instance, ORC_TAG_HSEF, r);
    for (int j = 0; j < 3; ++j) {
      double lo, hi;
      outer_bounds(s, g, j, &lo, &hi);
      const double vmax = vl * (hi - lo) / 2.0;
      const double x = s->hyper[6 * g + kOuterCol[j]];
      const double pb = h->op[3 * g + j];  // own Pbest, also its group's best
      const double tbv = h->op[3 * tb + j];
      double v = w * h->ov[3 * g + j] + C1 * r[0] * (pb - x) + C2 * r[1] * (pb - x) +
                 C3 * r[2] * (tbv - x);
      v = clampd(v, -vmax, vmax);
      h->ov[3 * g + j] = v;
      s->hyper[6 * g + kOuterCol[j]] = clampd(x + v, lo, hi);
    }
  }
  h->epoch_ctr += 1;
}

// Sec. "Auto Truncation": stop once the lowest fitness value has settled
// over the truncation window and the current best path is collision-free.
int32_t orc_at_check(const double* hist, int32_t k, int32_t mode, int32_t window, double delta,
                     int32_t q_tbest) {
  if (mode == 0 || q_tbest != 0 || window < 1) return 0;
  if (mode == 1 || mode == 3) {
    // mode 1: the full window must have elapsed; mode 3: the window is
    // whatever has elapsed (at least two values), capped at `window`
    int32_t w = window;
    if (mode == 1 && k < window) return 0;
    if (mode == 3) {
      if (k < 2) return 0;
      w = k < window ? k : window;
    }
    double mean = 0.0;
    for (int32_t i = k - w; i < k; ++i) mean += hist[i];
    mean /= (double)w;
    double var = 0.0;
    for (int32_t i = k - w; i < k; ++i) var += (hist[i] - mean) * (hist[i] - mean);
    var /= (double)w;
    return std::sqrt(var) < delta ? 1 : 0;
  }
  if (mode == 2) {
    if (k <= window) return 0;
    const double now = hist[k - 1], then = hist[k - 1 - window];
    const double scale = std::fabs(now) > 1.0 ? std::fabs(now) : 1.0;
    return (then - now) < delta * scale ? 1 : 0;
  }
  return 0;
}

// Moving obstacles translate by their velocity each frame and bounce off the
// map border (velocity component reversed, overshoot mirrored back); the
// start and target points move the same way.
static void bounce_axis(double* coords, int32_t n, int32_t stride, double* vel, double hi) {
  double mn = coords[0], mx = coords[0];
  for (int32_t i = 1; i < n; ++i) {
    mn = coords[i * stride] < mn ? coords[i * stride] : mn;
    mx = coords[i * stride] > mx ? coords[i * stride] : mx;
  }
  double shift = 0.0;
  if (mn < 0.0)
    shift = -2.0 * mn;
  else if (mx > hi)
    shift = -2.0 * (mx - hi);
  if (shift != 0.0) {
    for (int32_t i = 0; i < n; ++i) coords[i * stride] += shift;
    *vel = -*vel;
  }
}

void orc_sim_step(double width, double height, int32_t n_polys, const int32_t* poly_ptr,
                  double* verts, double* poly_vel, double* start, double* target,
                  double* endpoint_vel) {
  for (int32_t p = 0; p < n_polys; ++p) {
    const int32_t v0 = poly_ptr[p], nv = poly_ptr[p + 1] - v0;
    double* vx = verts + 2 * v0;
    if (poly_vel[2 * p] == 0.0 && poly_vel[2 * p + 1] == 0.0) continue;
    for (int32_t i = 0; i < nv; ++i) {
      vx[2 * i] += poly_vel[2 * p];
      vx[2 * i + 1] += poly_vel[2 * p + 1];
    }
    bounce_axis(vx, nv, 2, &poly_vel[2 * p], width);
    bounce_axis(vx + 1, nv, 2, &poly_vel[2 * p + 1], height);
  }
  double* pts[2] = {start, target};
  for (int e = 0; e < 2; ++e) {
    double* pt = pts[e];
    double* ve = endpoint_vel + 2 * e;
    pt[0] += ve[0];
    pt[1] += ve[1];
    bounce_axis(pt, 1, 1, &ve[0], width);
    bounce_axis(pt + 1, 1, 1, &ve[1], height);
  }
}

void orc_plan_frame(orc_swarm* s, orc_hsef* h, const orc_map* m, const orc_frame_cfg* c,
                    int32_t frame, const double* prev_path, double* out_path, double* hist,
                    orc_frame_result* res) {
  const bool pi = c->use_pi && frame > 0 && prev_path != nullptr;
  orc_init(s, frame, pi ? prev_path : nullptr, c->pi_gamma, c->pi_radius);
  if (c->hsef_every > 0) orc_hsef_reset_frame(s, h);
  int32_t truncated = 0;
  for (;;) {
    s->k += 1;
    orc_eval(s, m);
    orc_bests(s);
    hist[s->k - 1] = s->tbest_f;
    const int32_t tq = s->PQ[s->tbest_g * s->N + s->tbest_n];
    bool stop = false;
    if (orc_at_check(hist, s->k, c->at_mode, c->at_window, c->at_delta, tq)) {
      truncated = 1;
      stop = true;
    }
    if (s->k >= s->T) stop = true;
    if (stop) {
      s->ctr += 1;
      break;
    }
    if (c->hsef_every > 0 && s->k % c->hsef_every == 0) orc_hsef_step(s, h);
    orc_update(s);
    s->ctr += 1;
  }
  const int32_t D = 2 * s->W;
  const int32_t ti = s->tbest_g * s->N + s->tbest_n;
  for (int32_t d = 0; d < D; ++d) out_path[d] = s->P[(size_t)ti * D + d];
  res->cost = s->tbest_f;
  res->length = s->PL[ti];
  res->crossings = s->PQ[ti];
  res->iters = s->k;
  res->truncated = truncated;
}
