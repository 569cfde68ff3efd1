// Host-side code under AddressSanitizer and UndefinedBehaviorSanitizer: the
// C oracle (split, products, GADI, Gershgorin bounds) on a small 2-D
// convection-diffusion system and the size-based GPR of libgadi's host code.
// Built and run by tests/test_cpu_sanitize.py; exits non-zero on a wrong
// result, and the sanitizers abort on any memory or undefined-behaviour error.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "gadi.h"

extern "C" {
struct oracle_sys;
oracle_sys* oracle_setup(int n, const int* rp, const int* col, const double* val);
void oracle_free(oracle_sys* s);
int oracle_split_ok(const oracle_sys* s);
int oracle_spmv(const oracle_sys* s, int which, const double* x, double* y);
int oracle_gadi(const oracle_sys* s, const double* b, double* x, double alpha, double omega, double tol, double eps_h,
                double eps_s, int maxit_out, int maxit_in, int* sweeps, int64_t* inner_h, int64_t* inner_s,
                double* relres, double* hist, int hist_len);
int oracle_gershgorin(const oracle_sys* s, double* out);
}

// 5-point stencil of the h^2-scaled 2-D convection-diffusion operator, n x n
// interior grid, beta on both axes (sub -1 - r, super -1 + r, r = beta h / 2).
static void convdiff2d(int n, double beta, std::vector<int>& rp, std::vector<int>& col, std::vector<double>& val) {
  const double r = beta / (2.0 * (n + 1));
  const int N = n * n;
  rp.assign(1, 0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const int row = i * n + j;
      auto add = [&](int c, double v) {
        col.push_back(c);
        val.push_back(v);
      };
      if (i > 0) add(row - n, -1.0 - r);
      if (j > 0) add(row - 1, -1.0 - r);
      add(row, 4.0);
      if (j + 1 < n) add(row + 1, -1.0 + r);
      if (i + 1 < n) add(row + n, -1.0 + r);
      rp.push_back((int)col.size());
    }
  (void)N;
}

int main() {
  const int n = 12, N = n * n;
  std::vector<int> rp, col;
  std::vector<double> val;
  convdiff2d(n, 10.0, rp, col, val);
  oracle_sys* s = oracle_setup(N, rp.data(), col.data(), val.data());
  if (!s || !oracle_split_ok(s)) return 2;
  std::vector<double> ones(N, 1.0), b(N), y(N), x(N, 0.0), hist(64);
  if (oracle_spmv(s, 0, ones.data(), b.data()) != 0) return 3;
  for (int which = 1; which <= 2; ++which)
    if (oracle_spmv(s, which, ones.data(), y.data()) != 0) return 4;
  int sweeps = 0;
  int64_t ih = 0, is = 0;
  double rel = 0.0;
  const int st = oracle_gadi(s, b.data(), x.data(), 0.5, 0.5, 1e-10, 1e-6, 1e-6, 2000, 500, &sweeps, &ih, &is, &rel,
                             hist.data(), (int)hist.size());
  if (st != 0 || !(rel <= 1e-10)) return 5;
  double err = 0.0;
  for (int i = 0; i < N; ++i) err = std::fmax(err, std::fabs(x[i] - 1.0));
  if (!(err < 1e-7)) return 6;
  double g[4];
  if (oracle_gershgorin(s, g) != 0 || !(g[0] >= 0.0) || !(g[1] > g[0])) return 7;
  oracle_free(s);

  // GPR: log10 alpha on log2 n, a line plus a bump; predictions between the points
  const double xs[5] = {3.0, 3.58, 4.0, 4.58, 5.0};
  double ys[5];
  for (int i = 0; i < 5; ++i) ys[i] = -0.3 * xs[i] + 0.05 * std::sin(3.0 * xs[i]);
  gadi_gpr* gp = nullptr;
  if (gadi_gpr_fit(xs, ys, 5, &gp) != GADI_OK || !gp) return 8;
  const double xq[3] = {3.3, 5.5, 7.0};
  double mean[3], sd[3], params[8];
  if (gadi_gpr_predict(gp, xq, 3, mean, sd) != GADI_OK) return 9;
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(mean[i]) || !(sd[i] >= 0.0)) return 10;
  if (gadi_gpr_params(gp, params) != GADI_OK) return 11;
  gadi_gpr_destroy(gp);
  std::printf("host driver ok: %d sweeps, error %.3g, gpr mean %.4f %.4f %.4f\n", sweeps, err, mean[0], mean[1],
              mean[2]);
  return 0;
}
