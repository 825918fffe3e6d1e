// SEPSO oracle, learned initializer: FP64 forward and backward of the
// path-proposal MLP (Linear-ReLU stack, linear output, mean squared error),
// with optional rounding to BF16 at the points where the device stores
// BF16 values, and the Adam step that trains it.  TEST INFRASTRUCTURE ONLY
// (see orc.h).  Plain loops.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

extern "C" {

// Round to the nearest BF16 value (8 significant bits, ties to even),
// written from the definition: scale the significand to an integer range and
// round half to even.
double orc_bf16(double x) {
  if (x == 0.0 || !std::isfinite(x)) return x;
  int e;
  const double m = std::frexp(x, &e);    // x = m * 2^e, 0.5 <= |m| < 1
  const double s = std::ldexp(m, 8);      // 8 significant bits -> |s| in [128, 256)
  double r = std::floor(s);
  const double frac = s - r;
  if (frac > 0.5 || (frac == 0.5 && std::fmod(r, 2.0) != 0.0)) r += 1.0;
  return std::ldexp(r, e - 8);
}

// Network: sizes[0] inputs -> sizes[1..L-1] ReLU hidden -> sizes[L] linear.
// W[l] is sizes[l+1] x sizes[l] row-major, b[l] has sizes[l+1] entries.
// With `round` != 0, inputs, weights and the hidden activations fed to the
// next layer are rounded to BF16, as are the output-gradient and the hidden
// pre-activation gradients fed to the weight-gradient products; all sums
// are exact-order FP64.
//   y     : B x sizes[L] outputs
//   loss  : mean over B * sizes[L] of (y - target)^2
//   gW,gb : gradients of loss (may be NULL to skip the backward pass)
//   gWmag : (may be NULL) per weight-gradient element a magnitude that bounds
//           how far BF16 storage of intermediate values can move it: the same
//           chain of products run on absolute values, |x| forward through
//           |W| and |b| (Mag(a)), 2 (Mag(y) + |t|) / (B n) backward through
//           |W| with every unit kept (Mag(dz), so ReLU decisions that flip
//           are covered), and gWmag[l] = sum over the batch of
//           Mag(dz) Mag(a).  Each rounding moves a value by at most 2^-8 of
//           its Mag, and the roundings add up along the chain.
void orc_mlp(int32_t L, const int32_t* sizes, const double* const* W, const double* const* b,
             int32_t B, const double* x, const double* target, int32_t round, double* y,
             double* loss, double* const* gW, double* const* gb, double* const* gWmag) {
  auto R = [&](double v) { return round ? orc_bf16(v) : v; };
  std::vector<std::vector<double>> a(L + 1), z(L + 1);
  a[0].resize((size_t)B * sizes[0]);
  for (size_t i = 0; i < a[0].size(); ++i) a[0][i] = R(x[i]);
  std::vector<std::vector<double>> Wr(L);
  for (int l = 0; l < L; ++l) {
    Wr[l].resize((size_t)sizes[l + 1] * sizes[l]);
    for (size_t i = 0; i < Wr[l].size(); ++i) Wr[l][i] = R(W[l][i]);
  }
  for (int l = 0; l < L; ++l) {
    const int ni = sizes[l], no = sizes[l + 1];
    z[l + 1].assign((size_t)B * no, 0.0);
    a[l + 1].assign((size_t)B * no, 0.0);
    for (int r = 0; r < B; ++r)
      for (int o = 0; o < no; ++o) {
        double s = 0.0;
        for (int i = 0; i < ni; ++i) s += Wr[l][(size_t)o * ni + i] * a[l][(size_t)r * ni + i];
        s += b[l][o];
        z[l + 1][(size_t)r * no + o] = s;
        if (l + 1 < L)
          a[l + 1][(size_t)r * no + o] = R(s > 0.0 ? s : 0.0);
        else
          a[l + 1][(size_t)r * no + o] = s;
      }
  }
  // magnitude forward pass (only for gWmag)
  std::vector<std::vector<double>> m(gWmag ? L + 1 : 0);
  if (gWmag) {
    m[0].resize(a[0].size());
    for (size_t i = 0; i < a[0].size(); ++i) m[0][i] = std::fabs(a[0][i]);
    for (int l = 0; l < L; ++l) {
      const int ni = sizes[l], no = sizes[l + 1];
      m[l + 1].assign((size_t)B * no, 0.0);
      for (int r = 0; r < B; ++r)
        for (int o = 0; o < no; ++o) {
          double s = std::fabs(b[l][o]);
          for (int i = 0; i < ni; ++i) s += std::fabs(Wr[l][(size_t)o * ni + i]) * m[l][(size_t)r * ni + i];
          m[l + 1][(size_t)r * no + o] = s;
        }
    }
  }
  const int no = sizes[L];
  double acc = 0.0;
  for (size_t i = 0; i < (size_t)B * no; ++i) {
    if (y) y[i] = a[L][i];
    if (target) acc += (a[L][i] - target[i]) * (a[L][i] - target[i]);
  }
  if (loss) *loss = acc / ((double)B * no);
  if (!gW || !target) return;
  // d loss / d z_L
  std::vector<double> dz((size_t)B * no), mdz;
  for (size_t i = 0; i < dz.size(); ++i) dz[i] = 2.0 * (a[L][i] - target[i]) / ((double)B * no);
  if (gWmag) {
    mdz.resize(dz.size());
    for (size_t i = 0; i < dz.size(); ++i) mdz[i] = 2.0 * (m[L][i] + std::fabs(target[i])) / ((double)B * no);
  }
  for (int l = L - 1; l >= 0; --l) {
    const int ni = sizes[l], nO = sizes[l + 1];
    std::vector<double> dzr(dz.size());
    for (size_t i = 0; i < dz.size(); ++i) dzr[i] = R(dz[i]);
    for (int o = 0; o < nO; ++o) {
      double sb = 0.0;
      for (int r = 0; r < B; ++r) sb += dz[(size_t)r * nO + o];
      gb[l][o] = sb;
      for (int i = 0; i < ni; ++i) {
        double s = 0.0;
        for (int r = 0; r < B; ++r) s += dzr[(size_t)r * nO + o] * a[l][(size_t)r * ni + i];
        gW[l][(size_t)o * ni + i] = s;
        if (gWmag) {
          double sm = 0.0;
          for (int r = 0; r < B; ++r) sm += mdz[(size_t)r * nO + o] * m[l][(size_t)r * ni + i];
          gWmag[l][(size_t)o * ni + i] = sm;
        }
      }
    }
    if (l == 0) break;
    if (gWmag) {
      std::vector<double> mprev((size_t)B * ni, 0.0);
      for (int r = 0; r < B; ++r)
        for (int i = 0; i < ni; ++i) {
          double s = 0.0;
          for (int o = 0; o < nO; ++o) s += mdz[(size_t)r * nO + o] * std::fabs(Wr[l][(size_t)o * ni + i]);
          mprev[(size_t)r * ni + i] = s;
        }
      mdz.swap(mprev);
    }
    std::vector<double> dprev((size_t)B * ni, 0.0);
    for (int r = 0; r < B; ++r)
      for (int i = 0; i < ni; ++i) {
        double s = 0.0;
        for (int o = 0; o < nO; ++o) s += dzr[(size_t)r * nO + o] * Wr[l][(size_t)o * ni + i];
        dprev[(size_t)r * ni + i] = z[l][(size_t)r * ni + i] > 0.0 ? s : 0.0;  // ReLU'
      }
    dz.swap(dprev);
  }
}

// Occupancy raster: cell (r, c) of an n x n grid over [0,width] x [0,height]
// is 1 when its centre lies inside any polygon (even-odd crossing rule).
void orc_raster(double width, double height, int32_t n_polys, const int32_t* poly_ptr,
                const double* verts, int32_t n, double* out) {
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) {
      const double px = (c + 0.5) * width / n, py = (r + 0.5) * height / n;
      int inside = 0;
      for (int q = 0; q < n_polys && !inside; ++q) {
        const int v0 = poly_ptr[q], m = poly_ptr[q + 1] - v0;
        int odd = 0;
        for (int j = 0; j < m; ++j) {
          const double* a = verts + 2 * (v0 + j);
          const double* bb = verts + 2 * (v0 + (j + 1) % m);
          if ((a[1] > py) != (bb[1] > py)) {
            const double xc = a[0] + (py - a[1]) * (bb[0] - a[0]) / (bb[1] - a[1]);
            if (px < xc) odd ^= 1;
          }
        }
        inside = odd;
      }
      out[r * n + c] = inside;
    }
}

}  // extern "C"

extern "C" {

// One step of Adam (Kingma and Ba, "Adam: A Method for Stochastic
// Optimization", ICLR 2015, Algorithm 1) over n parameters, in FP64: the
// moment estimates m, v are updated in place, t is the 1-based step index
// used by the bias corrections, and each parameter moves by
//   -lr * m_hat / (sqrt(v_hat) + eps),  m_hat = m / (1 - b1^t),  v_hat = v / (1 - b2^t).
void orc_adam_step(int64_t n, double* p, const double* g, double* m, double* v, int32_t t,
                   double lr, double b1, double b2, double eps) {
  const double c1 = 1.0 - std::pow(b1, (double)t), c2 = 1.0 - std::pow(b2, (double)t);
  for (int64_t i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    const double mh = m[i] / c1, vh = v[i] / c2;
    p[i] -= lr * mh / (std::sqrt(vh) + eps);
  }
}

}  // extern "C"
