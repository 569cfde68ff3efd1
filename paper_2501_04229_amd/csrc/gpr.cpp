// Gaussian-process regression of the splitting parameter on the problem size
// (Section 3.3): the paper maps the grid size n of small systems of one
// structure to their best alpha and predicts alpha for large n.
//
// Model, with x = the size feature and y = the target (the callers use
// x = log2 n, y = log10 alpha):
//   y(x) = b0 + b1 x + f(x) + e,  f ~ GP(0, sf2 exp(-(x - x')^2 / (2 l^2))),
//   e ~ N(0, sn2),
// the linear mean by ordinary least squares (b1 = 0 when the x are all equal),
// the GP on its residuals (none when every residual is at most
// 1e-12 max(1, max |y|): the data are a line up to rounding).  Hyperparameters maximise the log marginal
// likelihood of the residuals: l over 25 log-spaced values in
// [0.1 s, 10 s] (s = spread of x, 1 if zero), eta = sn2 / sf2 over 13
// log-spaced values in [1e-6, 1], and sf2 profiled out (its maximiser is
// e^T Kt^-1 e / m for Kt = K / sf2).  Ties keep the first grid point in
// (l, eta) order.  Predictions are the latent posterior mean and standard
// deviation (noise excluded; the uncertainty of the linear mean is not added).
//
// Host code: plain double arithmetic, no device work.
#include <cmath>
#include <new>
#include <vector>

#include "gadi.h"

struct gadi_gpr {
  int m = 0;
  std::vector<double> x;      // training inputs
  std::vector<double> alpha;  // Kt^-1 e
  std::vector<double> L;      // Cholesky factor of Kt (row-major, lower)
  double b0 = 0.0, b1 = 0.0;
  double ell = 1.0, sf2 = 0.0, eta = 0.0, lml = 0.0;
};

namespace {

constexpr int kEllGrid = 25;
constexpr int kEtaGrid = 13;

// Cholesky of the m x m symmetric positive definite a (row-major) into l;
// false if a pivot is not positive.
bool cholesky(const std::vector<double>& a, int m, std::vector<double>& l) {
  l.assign((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = a[(size_t)i * m + j];
      for (int k = 0; k < j; ++k) s -= l[(size_t)i * m + k] * l[(size_t)j * m + k];
      if (i == j) {
        if (!(s > 0.0)) return false;
        l[(size_t)i * m + i] = std::sqrt(s);
      } else {
        l[(size_t)i * m + j] = s / l[(size_t)j * m + j];
      }
    }
  return true;
}

// Solves L L^T v = r in place.
void chol_solve(const std::vector<double>& l, int m, std::vector<double>& v) {
  for (int i = 0; i < m; ++i) {
    double s = v[i];
    for (int k = 0; k < i; ++k) s -= l[(size_t)i * m + k] * v[k];
    v[i] = s / l[(size_t)i * m + i];
  }
  for (int i = m - 1; i >= 0; --i) {
    double s = v[i];
    for (int k = i + 1; k < m; ++k) s -= l[(size_t)k * m + i] * v[k];
    v[i] = s / l[(size_t)i * m + i];
  }
}

double kern(double a, double b, double ell) {
  const double d = (a - b) / ell;
  return std::exp(-0.5 * d * d);
}

}  // namespace

extern "C" gadi_status gadi_gpr_fit(const double* x, const double* y, int32_t m, gadi_gpr** out) {
  if (!out) return GADI_EINVAL;
  *out = nullptr;
  // the grid search factors 325 m x m matrices: O(100 m^3) flops, about a second at the limit
  if (!x || !y || m < 1 || m > 256) return GADI_EINVAL;
  for (int i = 0; i < m; ++i)
    if (!std::isfinite(x[i]) || !std::isfinite(y[i])) return GADI_EINVAL;
  gadi_gpr* g = new (std::nothrow) gadi_gpr();
  if (!g) return GADI_ENOMEM;
  g->m = m;
  g->x.assign(x, x + m);
  // linear mean by least squares
  double mx = 0.0, my = 0.0;
  for (int i = 0; i < m; ++i) {
    mx += x[i];
    my += y[i];
  }
  mx /= m;
  my /= m;
  double sxx = 0.0, sxy = 0.0, lo = x[0], hi = x[0];
  for (int i = 0; i < m; ++i) {
    sxx += (x[i] - mx) * (x[i] - mx);
    sxy += (x[i] - mx) * (y[i] - my);
    lo = std::fmin(lo, x[i]);
    hi = std::fmax(hi, x[i]);
  }
  g->b1 = sxx > 0.0 ? sxy / sxx : 0.0;
  g->b0 = my - g->b1 * mx;
  std::vector<double> e(m);
  double emax = 0.0, ymax = 1.0;
  for (int i = 0; i < m; ++i) {
    e[i] = y[i] - g->b0 - g->b1 * x[i];
    emax = std::fmax(emax, std::fabs(e[i]));
    ymax = std::fmax(ymax, std::fabs(y[i]));
  }
  const double spread = hi > lo ? hi - lo : 1.0;
  g->alpha.assign(m, 0.0);
  g->L.assign((size_t)m * m, 0.0);
  if (!(emax > 1e-12 * ymax)) {
    // linear data up to rounding: the GP part is zero
    g->ell = spread;
    g->sf2 = 0.0;
    g->eta = 1.0;
    g->lml = INFINITY;
    *out = g;
    return GADI_OK;
  }
  const double kLog2Pi = std::log(2.0 * M_PI);
  bool found = false;
  std::vector<double> K((size_t)m * m), l, v;
  for (int a = 0; a < kEllGrid; ++a) {
    const double ell = spread * std::pow(10.0, -1.0 + 2.0 * a / (kEllGrid - 1));
    for (int b = 0; b < kEtaGrid; ++b) {
      const double eta = std::pow(10.0, -6.0 + 6.0 * b / (kEtaGrid - 1));
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) K[(size_t)i * m + j] = kern(x[i], x[j], ell) + (i == j ? eta : 0.0);
      if (!cholesky(K, m, l)) continue;
      v = e;
      chol_solve(l, m, v);
      double q = 0.0, logdet = 0.0;
      for (int i = 0; i < m; ++i) {
        q += e[i] * v[i];
        logdet += std::log(l[(size_t)i * m + i]);
      }
      if (!(q > 0.0)) continue;
      const double sf2 = q / m;
      // log N(e; 0, sf2 Kt) at the profiled sf2
      const double lml = -0.5 * m * std::log(sf2) - logdet - 0.5 * m - 0.5 * m * kLog2Pi;
      if (!found || lml > g->lml) {
        found = true;
        g->lml = lml;
        g->ell = ell;
        g->eta = eta;
        g->sf2 = sf2;
        g->alpha = v;
        g->L = l;
      }
    }
  }
  if (!found) {
    delete g;
    return GADI_EINVAL;
  }
  *out = g;
  return GADI_OK;
}

extern "C" gadi_status gadi_gpr_predict(const gadi_gpr* g, const double* xq, int32_t q, double* mean, double* sd) {
  if (!g || !xq || q < 0 || (q > 0 && !mean)) return GADI_EINVAL;
  const int m = g->m;
  std::vector<double> k(m);
  for (int t = 0; t < q; ++t) {
    if (!std::isfinite(xq[t])) return GADI_EINVAL;
    double mu = g->b0 + g->b1 * xq[t];
    double var = 0.0;
    if (g->sf2 > 0.0) {
      for (int i = 0; i < m; ++i) {
        k[i] = kern(xq[t], g->x[i], g->ell);
        mu += k[i] * g->alpha[i];
      }
      // latent variance sf2 (1 - k^T Kt^-1 k) through the forward solve L w = k
      for (int i = 0; i < m; ++i) {
        double s = k[i];
        for (int j = 0; j < i; ++j) s -= g->L[(size_t)i * m + j] * k[j];
        k[i] = s / g->L[(size_t)i * m + i];
      }
      double kk = 0.0;
      for (int i = 0; i < m; ++i) kk += k[i] * k[i];
      var = g->sf2 * (1.0 - kk);
    }
    mean[t] = mu;
    if (sd) sd[t] = std::sqrt(var > 0.0 ? var : 0.0);
  }
  return GADI_OK;
}

extern "C" gadi_status gadi_gpr_params(const gadi_gpr* g, double* out) {
  if (!g || !out) return GADI_EINVAL;
  out[0] = g->b0;
  out[1] = g->b1;
  out[2] = g->ell;
  out[3] = g->sf2;
  out[4] = g->eta * g->sf2;
  out[5] = g->lml;
  return GADI_OK;
}

extern "C" gadi_status gadi_gpr_destroy(gadi_gpr* g) {
  if (!g) return GADI_EINVAL;
  delete g;
  return GADI_OK;
}
