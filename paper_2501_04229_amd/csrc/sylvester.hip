// GADI-AB for the continuous Sylvester equation A X + X B = C (Section 4.3).
//
// L(X) = A X + X B is split into M(X) = A X and N(X) = X B, so the two inner
// solves of Algorithm 1 become many independent tridiagonal solves: step 2
// solves (alpha I + A) z = r for every column of R, step 3 solves
// (alpha I + B)^T y = g for every row of G = (2 - omega) alpha Z.  All columns
// (rows) share one LU factorisation, computed on the host per alpha.  A
// column's recurrences are split into chunks of kChunk rows:
//
//   forward   y_i = v_i - l_i y_{i-1}             (l_i = sub_{i-1} / p_{i-1})
//   backward  z_i = (y_i - sup_i z_{i+1}) / p_i
//
// Run inside a chunk [s, e) with y_{s-1} = 0 and z_e = 0 they give y^, z^;
// the true values are y_i = y^_i + f_i y_{s-1} and
// z_i = z^_i + y_{s-1} q_i + z_e h_i, where f, q, h depend on the matrix only
// (precomputed).  A short chain per column then fixes the chunk boundary
// values y_{s-1} (forward) and z_e (backward).  Kernels per sweep:
//   residual (double) -> partial sums -> column chunks -> column chains ->
//   column correction (writes G, tracks max |G|) -> row chunks (LDS tiles)
//   -> row chains -> row correction fused with the update of X (double).
// X, C and the work arrays are m x n row-major.
#include <cmath>
#include <cstdio>
#include <vector>

#include "device_common.h"

namespace gadi {

constexpr int kChunk = 64;         // rows of a chunk of the recurrences
constexpr int kSylBlock = 256;     // threads of the elementwise kernels
constexpr int kSylMax = 1 << 15;   // largest m or n

// Coefficients of one direction's solves (device, inner type IT): per row i
// of the (alpha I + T) system: l_i, 1/p_i, sup_i, f_i, q_i, h_i.
template <class IT>
struct Factors {
  const IT* l;
  const IT* ip;
  const IT* sup;
  const IT* f;
  const IT* q;
  const IT* h;
  int len;  // system size (m for columns, n for rows)
};

// Half-precision storage of an inner right-hand side or solution: round to
// binary16 and back (MODE 1), else unchanged.
template <int MODE, class IT>
__device__ __forceinline__ IT stor(IT v) {
  if constexpr (MODE == 1) return (IT)__half2float(__float2half_rn((float)v));
  else return v;
}

// Device-side loop control of one solve: the host enqueues sweeps in batches
// and reads this record between batches; every kernel of a sweep returns at
// once when `done` is set.
struct SylCtl {
  double rho0;    // ||R_0||_F
  double res;     // last ||R_k||_F / ||R_0||_F
  double scale1;  // power of two that brings max |R_k| into [1/2, 1)
  double tol;
  int sweeps;     // corrections issued
  int maxit;
  int done;
  int status;
};

// ---------------------------------------------------------------------- residual
// R = C - A X - X B in double; per-block sum of squares and max |r| into part.
template <class IT>
__global__ void __launch_bounds__(kSylBlock) syl_residual_kernel(
    const double* __restrict__ X, const double* __restrict__ C, const double* __restrict__ a_sub,
    const double* __restrict__ a_diag, const double* __restrict__ a_sup, const double* __restrict__ b_sub,
    const double* __restrict__ b_diag, const double* __restrict__ b_sup, IT* __restrict__ R, int m, int n,
    double* __restrict__ part, const SylCtl* __restrict__ ctl) {
  __shared__ double sh[kSylBlock / 64][2];
  if (ctl->done) return;
  const size_t total = (size_t)m * n;
  double s2 = 0.0, mx = 0.0;
  for (size_t k = (size_t)blockIdx.x * kSylBlock + threadIdx.x; k < total; k += (size_t)gridDim.x * kSylBlock) {
    const int i = (int)(k / n), j = (int)(k % n);
    const double x = X[k];
    double ax = a_diag[i] * x;
    if (i > 0) ax += a_sub[i - 1] * X[k - n];
    if (i < m - 1) ax += a_sup[i] * X[k + n];
    double xb = x * b_diag[j];
    if (j > 0) xb += X[k - 1] * b_sup[j - 1];
    if (j < n - 1) xb += X[k + 1] * b_sub[j];
    const double r = C[k] - ax - xb;
    R[k] = (IT)r;
    s2 += r * r;
    mx = fmax(mx, fabs(r));
  }
  s2 = wave_sum(s2);
  mx = wave_max(mx);
  if ((threadIdx.x & 63) == 0) {
    sh[threadIdx.x >> 6][0] = s2;
    sh[threadIdx.x >> 6][1] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < kSylBlock / 64; ++w) {
      a += sh[w][0];
      b = fmax(b, sh[w][1]);
    }
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = b;
  }
}

// Fixed-order combination of the residual partials and the stopping test of
// Algorithm 1; clears the max |G| word for the sweep that follows.
__global__ void syl_reduce_kernel(const double* __restrict__ part, int nparts, SylCtl* __restrict__ ctl,
                                  double* __restrict__ hist, int hist_cap, int scale_rhs, unsigned* __restrict__ gmax) {
  if (threadIdx.x != 0 || ctl->done) return;
  double a = 0.0, b = 0.0;
  for (int k = 0; k < nparts; ++k) {
    a += part[2 * k];
    b = fmax(b, part[2 * k + 1]);
  }
  const double rho = sqrt(a);
  const int k = ctl->sweeps;
  if (k == 0) ctl->rho0 = rho;
  const double rho0 = ctl->rho0;
  const double res = rho0 > 0.0 ? rho / rho0 : 0.0;
  ctl->res = res;
  if (hist && k < hist_cap) hist[k] = res;
  if (rho <= ctl->tol * rho0) {
    ctl->status = GADI_OK;
    ctl->done = 1;
  } else if (!isfinite(rho) || rho > 1e6 * rho0) {
    ctl->status = GADI_EDIVERGED;
    ctl->done = 1;
  } else if (k >= ctl->maxit) {
    ctl->status = GADI_EMAXIT;
    ctl->done = 1;
  } else {
    int e1;
    (void)frexp(b, &e1);
    e1 = e1 < -120 ? -120 : (e1 > 120 ? 120 : e1);
    ctl->scale1 = scale_rhs ? ldexp(1.0, -e1) : 1.0;
    ctl->sweeps = k + 1;  // the kernels that follow apply this correction
  }
  *gmax = 0u;
}

// ---------------------------------------------------------------------- column solves
// One thread per (column j, chunk c): local recurrences over the chunk's rows.
// v_i = stor(R_ij * scale) (MODE 1: half storage of the right-hand side).
template <class IT, int MODE>
__global__ void __launch_bounds__(kSylBlock) syl_col_local_kernel(const IT* __restrict__ R, Factors<IT> F,
                                                                  const SylCtl* __restrict__ ctl, int n,
                                                                  IT* __restrict__ Zh, IT* __restrict__ yend,
                                                                  IT* __restrict__ zbeg) {
  if (ctl->done) return;
  const IT scale = (IT)ctl->scale1;
  const int j = blockIdx.x * kSylBlock + threadIdx.x;
  const int c = blockIdx.y;
  const int s = c * kChunk, e = (s + kChunk < F.len) ? s + kChunk : F.len;
  if (j >= n) return;
  IT y[kChunk];
  IT prev = 0;
#pragma unroll
  for (int k = 0; k < kChunk; ++k) {
    const int i = s + k;
    if (i < e) {
      const IT v = stor<MODE>(R[(size_t)i * n + j] * scale);
      prev = v - (k == 0 ? IT(0) : F.l[i] * prev);
      y[k] = prev;
    }
  }
  IT z = 0;
#pragma unroll
  for (int k = kChunk - 1; k >= 0; --k) {
    const int i = s + k;
    if (i < e) {
      z = (y[k] - F.sup[i] * z) * F.ip[i];
      Zh[(size_t)i * n + j] = z;
    }
  }
  yend[(size_t)c * n + j] = prev;  // y^ of the chunk's last row
  zbeg[(size_t)c * n + j] = z;
}

// One thread per column: the chunk-boundary chains.  B_c = y_{s_c - 1}
// (B_0 = 0), E_c = z_{e_c} (E_last = 0).  The chain inputs are loaded kBatch
// chunks at a time, so the loads of a batch are in flight together.
constexpr int kBatch = 16;

template <class IT>
__global__ void __launch_bounds__(kSylBlock) syl_chain_kernel(const IT* __restrict__ yend, const IT* __restrict__ zbeg,
                                                              Factors<IT> F, int nchunks, int width,
                                                              IT* __restrict__ Bc, IT* __restrict__ Ec,
                                                              const SylCtl* __restrict__ ctl) {
  if (ctl->done) return;
  const int j = blockIdx.x * kSylBlock + threadIdx.x;
  if (j >= width) return;
  IT b = 0;
  for (int c0 = 0; c0 < nchunks; c0 += kBatch) {
    IT ye[kBatch], ff[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int c = c0 + u;
      if (c < nchunks) {
        const int e = (c + 1) * kChunk < F.len ? (c + 1) * kChunk : F.len;
        ye[u] = yend[(size_t)c * width + j];
        ff[u] = F.f[e - 1];
      }
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int c = c0 + u;
      if (c < nchunks) {
        Bc[(size_t)c * width + j] = b;
        b = ye[u] + ff[u] * b;
      }
    }
  }
  IT ez = 0;
  for (int c1 = nchunks - 1; c1 >= 0; c1 -= kBatch) {
    IT zb[kBatch], bb[kBatch], qq[kBatch], hh[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int c = c1 - u;
      if (c >= 0) {
        const int s = c * kChunk;
        zb[u] = zbeg[(size_t)c * width + j];
        bb[u] = Bc[(size_t)c * width + j];
        qq[u] = F.q[s];
        hh[u] = F.h[s];
      }
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int c = c1 - u;
      if (c >= 0) {
        Ec[(size_t)c * width + j] = ez;
        ez = zb[u] + bb[u] * qq[u] + ez * hh[u];
      }
    }
  }
}

// z = z^ + B q + E h per element; G = (2 - omega) alpha z (in place of Zh),
// block max of |G| into gmax (bits of a non-negative float: monotone).
template <class IT>
__global__ void __launch_bounds__(kSylBlock) syl_col_fix_kernel(IT* __restrict__ Zh, const IT* __restrict__ Bc,
                                                                const IT* __restrict__ Ec, Factors<IT> F, IT gscale,
                                                                int m, int n, unsigned* __restrict__ gmax,
                                                                const SylCtl* __restrict__ ctl) {
  __shared__ float sh[kSylBlock / 64];
  if (ctl->done) return;
  const size_t total = (size_t)m * n;
  float mx = 0.f;
  for (size_t k = (size_t)blockIdx.x * kSylBlock + threadIdx.x; k < total; k += (size_t)gridDim.x * kSylBlock) {
    const int i = (int)(k / n), j = (int)(k % n);
    const int c = i / kChunk;
    const IT z = Zh[k] + Bc[(size_t)c * n + j] * F.q[i] + Ec[(size_t)c * n + j] * F.h[i];
    const IT g = gscale * z;
    Zh[k] = g;
    mx = fmaxf(mx, fabsf((float)g));
  }
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    float b = 0.f;
    for (int w = 0; w < kSylBlock / 64; ++w) b = fmaxf(b, sh[w]);
    atomicMax(gmax, __float_as_uint(b));
  }
}

// Power-of-two scale that brings max |g| into [1/2, 1) (1 if g is zero).
__device__ __forceinline__ float g_scale(const unsigned* gmax) {
  const float mx = __uint_as_float(*gmax);
  if (!(mx > 0.f) || !isfinite(mx)) return 1.f;
  int e;
  (void)frexpf(mx, &e);
  e = e < -120 ? -120 : (e > 120 ? 120 : e);
  return ldexpf(1.f, -e);
}

// ---------------------------------------------------------------------- row solves
// One wavefront per tile of 64 rows x kChunk columns: the tile passes through
// LDS so that global loads and stores run along the rows; lane t then runs the
// chunk-local recurrences of row r0 + t.  v_ij = stor(G_ij * 2^-e2).
template <class IT, int MODE>
__global__ void __launch_bounds__(64) syl_row_local_kernel(const IT* __restrict__ G, Factors<IT> F,
                                                           const unsigned* __restrict__ gmax, int m, int n,
                                                           IT* __restrict__ Zh, IT* __restrict__ yend,
                                                           IT* __restrict__ zbeg, const SylCtl* __restrict__ ctl) {
  __shared__ IT tile[64][kChunk + 1];
  if (ctl->done) return;
  const int t = threadIdx.x;
  const int c = blockIdx.x;
  const int r0 = blockIdx.y * 64;
  const int s = c * kChunk, e = (s + kChunk < n) ? s + kChunk : n;
  const IT sc = (IT)g_scale(gmax);
  for (int k = 0; k < 64; ++k) {
    const int i = r0 + k, j = s + t;
    tile[k][t] = (i < m && j < e) ? stor<MODE>(G[(size_t)i * n + j] * sc) : IT(0);
  }
  __syncthreads();
  const int row = r0 + t;
  IT y[kChunk];
  IT prev = 0;
#pragma unroll
  for (int k = 0; k < kChunk; ++k) {
    const int j = s + k;
    if (j < e) {
      const IT v = tile[t][k];
      prev = v - (k == 0 ? IT(0) : F.l[j] * prev);
      y[k] = prev;
    }
  }
  IT z = 0;
#pragma unroll
  for (int k = kChunk - 1; k >= 0; --k) {
    const int j = s + k;
    if (j < e) {
      z = (y[k] - F.sup[j] * z) * F.ip[j];
      tile[t][k] = z;
    }
  }
  if (row < m) {
    yend[(size_t)c * m + row] = prev;
    zbeg[(size_t)c * m + row] = z;
  }
  __syncthreads();
  for (int k = 0; k < 64; ++k) {
    const int i = r0 + k, j = s + t;
    if (i < m && j < e) Zh[(size_t)i * n + j] = tile[k][t];
  }
}

// y = z^ + B q + E h along the rows, stored in the inner precision, then
// X += y 2^(e1 + e2) in double.
template <class IT, int MODE>
__global__ void __launch_bounds__(kSylBlock) syl_row_fix_update_kernel(const IT* __restrict__ Zh,
                                                                       const IT* __restrict__ Bc,
                                                                       const IT* __restrict__ Ec, Factors<IT> F,
                                                                       const unsigned* __restrict__ gmax,
                                                                       const SylCtl* __restrict__ ctl, int m, int n,
                                                                       double* __restrict__ X) {
  if (ctl->done) return;
  const size_t total = (size_t)m * n;
  const double unscale = 1.0 / (ctl->scale1 * (double)g_scale(gmax));
  for (size_t k = (size_t)blockIdx.x * kSylBlock + threadIdx.x; k < total; k += (size_t)gridDim.x * kSylBlock) {
    const int i = (int)(k / n), j = (int)(k % n);
    const int c = j / kChunk;
    const IT y = stor<MODE>(Zh[k] + Bc[(size_t)c * m + i] * F.q[j] + Ec[(size_t)c * m + i] * F.h[j]);
    X[k] += (double)y * unscale;
  }
}

// ---------------------------------------------------------------------- host side

struct SylSystem {
  int m = 0, n = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  std::vector<double> a_sub, a_diag, a_sup, b_sub, b_diag, b_sup;  // host copies (length m or n, padded)
  double* dA = nullptr;  // [3][m]: sub, diag, sup of A (sub[i] at i, last entries 0)
  double* dB = nullptr;  // [3][n]
  double* dX = nullptr;
  double* dC = nullptr;
  void* R = nullptr;     // m*n inner type
  void* Zh = nullptr;    // m*n inner type
  void* chain = nullptr; // yend, zbeg, B, E: 4 * chunks * max(m, n)
  void* coef = nullptr;  // 6 * (m + n) inner type
  double* part = nullptr;
  SylCtl* ctl = nullptr;       // device
  SylCtl* ctl_host = nullptr;  // pinned host copy
  double* dhist = nullptr;
  int hist_cap = 0;
  unsigned* gmax = nullptr;
  int nparts = 0;
  std::vector<double> hist;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

}  // namespace gadi

struct gadi_sylv {
  gadi::SylSystem s;
};

namespace gadi {

static int chunks_of(int len) { return (len + kChunk - 1) / kChunk; }

// LU factors of (alpha I + T) (T given by sub/diag/sup, optionally rounded to
// half first) and the chunk coefficients f, q, h, in double.
static void factor(const std::vector<double>& sub0, const std::vector<double>& diag0, const std::vector<double>& sup0,
                   int len, double alpha, bool half, std::vector<double>& out) {
  auto rd = [&](double v) { return half ? (double)__half2float(__float2half_rn((float)v)) : v; };
  std::vector<double> sub(len, 0.0), d(len), sup(len, 0.0);
  for (int i = 0; i < len; ++i) {
    d[i] = rd(diag0[i]) + alpha;
    if (i + 1 < len) {
      sub[i] = rd(sub0[i]);
      sup[i] = rd(sup0[i]);
    }
  }
  out.assign(6 * (size_t)len, 0.0);
  double* l = out.data();
  double* ip = l + len;
  double* su = ip + len;
  double* f = su + len;
  double* q = f + len;
  double* h = q + len;
  double p = d[0];
  l[0] = 0.0;
  ip[0] = 1.0 / p;
  for (int i = 1; i < len; ++i) {
    l[i] = sub[i - 1] / p;
    p = d[i] - l[i] * sup[i - 1];
    ip[i] = 1.0 / p;
  }
  for (int i = 0; i < len; ++i) su[i] = (i + 1 < len) ? sup[i] : 0.0;
  for (int s = 0; s < len; s += kChunk) {
    const int e = s + kChunk < len ? s + kChunk : len;
    // f: y_i's dependence on y_{s-1}; q: the backward solve of f; h: z_i's on z_e
    for (int i = s; i < e; ++i) f[i] = (i == s ? -l[i] : -l[i] * f[i - 1]);
    for (int i = e - 1; i >= s; --i) {
      q[i] = (f[i] - (i + 1 < e ? su[i] * q[i + 1] : 0.0)) * ip[i];
      h[i] = -su[i] * ip[i] * (i + 1 < e ? h[i + 1] : 1.0);
    }
  }
}

template <class IT>
static gadi_status upload_coef(SylSystem& S, const std::vector<double>& col, const std::vector<double>& row) {
  std::vector<IT> buf(6 * (size_t)(S.m + S.n));
  for (size_t k = 0; k < col.size(); ++k) buf[k] = (IT)col[k];
  for (size_t k = 0; k < row.size(); ++k) buf[col.size() + k] = (IT)row[k];
  GADI_HIP_CHECK(hipMemcpyAsync(S.coef, buf.data(), buf.size() * sizeof(IT), hipMemcpyHostToDevice, S.stream));
  GADI_HIP_CHECK(hipStreamSynchronize(S.stream));
  return GADI_OK;
}

template <class IT>
static Factors<IT> factors_at(const SylSystem& S, int which) {
  const IT* base = (const IT*)S.coef + (which == 0 ? 0 : 6 * (size_t)S.m);
  const int len = which == 0 ? S.m : S.n;
  return Factors<IT>{base, base + len, base + 2 * len, base + 3 * len, base + 4 * len, base + 5 * len, len};
}

static int grid_of(size_t total) {
  size_t g = (total + kSylBlock - 1) / kSylBlock;
  return (int)(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

// One sweep: residual and stopping test, then steps 2-4; every kernel is a
// no-op once the device-side control has stopped the solve.
template <class IT, int MODE>
static void enqueue_sweep(SylSystem& S, double alpha, double omega) {
  const int m = S.m, n = S.n;
  const int pc = chunks_of(m), pr = chunks_of(n);
  const size_t w = (size_t)(m > n ? m : n);
  const size_t pw = (size_t)(pc > pr ? pc : pr) * w;
  IT* yend = (IT*)S.chain;
  IT* zbeg = yend + pw;
  IT* Bc = zbeg + pw;
  IT* Ec = Bc + pw;
  const Factors<IT> Fc = factors_at<IT>(S, 0), Fr = factors_at<IT>(S, 1);
  IT* R = (IT*)S.R;
  IT* Zh = (IT*)S.Zh;
  hipLaunchKernelGGL((syl_residual_kernel<IT>), dim3(S.nparts), dim3(kSylBlock), 0, S.stream, S.dX, S.dC, S.dA,
                     S.dA + m, S.dA + 2 * m, S.dB, S.dB + n, S.dB + 2 * n, R, m, n, S.part, S.ctl);
  hipLaunchKernelGGL(syl_reduce_kernel, dim3(1), dim3(64), 0, S.stream, S.part, S.nparts, S.ctl, S.dhist, S.hist_cap,
                     MODE == 2 ? 0 : 1, S.gmax);
  hipLaunchKernelGGL((syl_col_local_kernel<IT, MODE>), dim3((n + kSylBlock - 1) / kSylBlock, pc), dim3(kSylBlock), 0,
                     S.stream, R, Fc, S.ctl, n, Zh, yend, zbeg);
  hipLaunchKernelGGL((syl_chain_kernel<IT>), dim3((n + kSylBlock - 1) / kSylBlock), dim3(kSylBlock), 0, S.stream,
                     yend, zbeg, Fc, pc, n, Bc, Ec, S.ctl);
  hipLaunchKernelGGL((syl_col_fix_kernel<IT>), dim3(grid_of((size_t)m * n)), dim3(kSylBlock), 0, S.stream, Zh, Bc, Ec,
                     Fc, (IT)((2.0 - omega) * alpha), m, n, S.gmax, S.ctl);
  // G is in Zh; the row solves write their chunk-local solutions to R
  hipLaunchKernelGGL((syl_row_local_kernel<IT, MODE>), dim3(pr, (m + 63) / 64), dim3(64), 0, S.stream, Zh, Fr, S.gmax,
                     m, n, R, yend, zbeg, S.ctl);
  hipLaunchKernelGGL((syl_chain_kernel<IT>), dim3((m + kSylBlock - 1) / kSylBlock), dim3(kSylBlock), 0, S.stream,
                     yend, zbeg, Fr, pr, m, Bc, Ec, S.ctl);
  hipLaunchKernelGGL((syl_row_fix_update_kernel<IT, MODE>), dim3(grid_of((size_t)m * n)), dim3(kSylBlock), 0,
                     S.stream, R, Bc, Ec, Fr, S.gmax, S.ctl, m, n, S.dX);
}

template <class IT, int MODE>
static gadi_status run(SylSystem& S, double alpha, double omega, double tol, int maxit, bool record,
                       gadi_solve_info* info) {
  std::vector<double> fc, fr;
  factor(S.a_sub, S.a_diag, S.a_sup, S.m, alpha, MODE == 1, fc);
  // the row solves use (alpha I + B)^T: sub and sup exchanged
  factor(S.b_sup, S.b_diag, S.b_sub, S.n, alpha, MODE == 1, fr);
  gadi_status st = upload_coef<IT>(S, fc, fr);
  if (st != GADI_OK) return st;
  if (record && maxit + 1 > S.hist_cap) {
    if (S.dhist) (void)hipFree(S.dhist);
    S.dhist = nullptr;
    S.hist_cap = 0;
    GADI_HIP_CHECK(hipMalloc((void**)&S.dhist, sizeof(double) * (maxit + 1)));
    S.hist_cap = maxit + 1;
  }
  SylCtl c0{};
  c0.tol = tol;
  c0.maxit = maxit;
  c0.status = GADI_EMAXIT;
  *S.ctl_host = c0;
  GADI_HIP_CHECK(hipMemcpyAsync(S.ctl, S.ctl_host, sizeof(SylCtl), hipMemcpyHostToDevice, S.stream));
  const double* hist = record ? S.dhist : nullptr;
  GADI_HIP_CHECK(hipEventRecord(S.ev0, S.stream));
  // batches of sweeps between reads of the control record, growing with the sweep count
  int issued = 0;
  for (;;) {
    const int batch = issued < 8 ? 4 : (issued < 256 ? 16 : 64);
    for (int b = 0; b < batch; ++b) enqueue_sweep<IT, MODE>(S, alpha, omega);
    issued += batch;
    GADI_HIP_CHECK(hipGetLastError());
    GADI_HIP_CHECK(hipMemcpyAsync(S.ctl_host, S.ctl, sizeof(SylCtl), hipMemcpyDeviceToHost, S.stream));
    GADI_HIP_CHECK(hipStreamSynchronize(S.stream));
    if (S.ctl_host->done) break;
  }
  GADI_HIP_CHECK(hipEventRecord(S.ev1, S.stream));
  GADI_HIP_CHECK(hipEventSynchronize(S.ev1));
  float ms = 0.f;
  GADI_HIP_CHECK(hipEventElapsedTime(&ms, S.ev0, S.ev1));
  const SylCtl c = *S.ctl_host;
  S.hist.clear();
  if (record) {
    const int k = c.sweeps + 1 < S.hist_cap ? c.sweeps + 1 : S.hist_cap;
    S.hist.resize(k);
    GADI_HIP_CHECK(hipMemcpy(S.hist.data(), hist, sizeof(double) * k, hipMemcpyDeviceToHost));
  }
  if (info) {
    info->status = c.status;
    info->outer_sweeps = c.sweeps;
    info->inner_H = c.sweeps;
    info->inner_S = c.sweeps;
    info->relres = c.res;
    info->seconds = ms * 1e-3;
  }
  return (gadi_status)c.status;
}

}  // namespace gadi

using namespace gadi;

extern "C" gadi_status gadi_sylv_setup(int32_t m, int32_t n, const double* a_sub, const double* a_diag,
                                       const double* a_sup, const double* b_sub, const double* b_diag,
                                       const double* b_sup, gadi_sylv** out) {
  if (!out) return GADI_EINVAL;
  *out = nullptr;
  if (m < 1 || n < 1 || m > kSylMax || n > kSylMax || !a_diag || !b_diag) return GADI_EINVAL;
  if ((m > 1 && (!a_sub || !a_sup)) || (n > 1 && (!b_sub || !b_sup))) return GADI_EINVAL;
  gadi_sylv* h = new (std::nothrow) gadi_sylv();
  if (!h) return GADI_ENOMEM;
  SylSystem& S = h->s;
  S.m = m;
  S.n = n;
  S.a_diag.assign(a_diag, a_diag + m);
  S.b_diag.assign(b_diag, b_diag + n);
  S.a_sub.assign(m, 0.0);
  S.a_sup.assign(m, 0.0);
  S.b_sub.assign(n, 0.0);
  S.b_sup.assign(n, 0.0);
  for (int i = 0; i + 1 < m; ++i) {
    S.a_sub[i] = a_sub[i];
    S.a_sup[i] = a_sup[i];
  }
  for (int i = 0; i + 1 < n; ++i) {
    S.b_sub[i] = b_sub[i];
    S.b_sup[i] = b_sup[i];
  }
  auto fail = [&](gadi_status st) {
    gadi_sylv_destroy(h);
    return st;
  };
  if (hipGetDevice(&S.device) != hipSuccess) return fail(GADI_EHIP);
  const size_t mn = (size_t)m * n;
  const size_t w = (size_t)(m > n ? m : n);
  const size_t pmax = (size_t)(chunks_of(m) > chunks_of(n) ? chunks_of(m) : chunks_of(n));
  S.nparts = grid_of(mn);
  std::vector<double> a3(3 * (size_t)m), b3(3 * (size_t)n);
  for (int i = 0; i < m; ++i) {
    a3[i] = S.a_sub[i];
    a3[m + i] = S.a_diag[i];
    a3[2 * (size_t)m + i] = S.a_sup[i];
  }
  for (int i = 0; i < n; ++i) {
    b3[i] = S.b_sub[i];
    b3[n + i] = S.b_diag[i];
    b3[2 * (size_t)n + i] = S.b_sup[i];
  }
  if (hipMalloc((void**)&S.dA, a3.size() * 8) != hipSuccess || hipMalloc((void**)&S.dB, b3.size() * 8) != hipSuccess ||
      hipMalloc((void**)&S.dX, mn * 8) != hipSuccess || hipMalloc((void**)&S.dC, mn * 8) != hipSuccess ||
      hipMalloc(&S.R, mn * 8) != hipSuccess || hipMalloc(&S.Zh, mn * 8) != hipSuccess ||
      hipMalloc(&S.chain, 4 * pmax * w * 8) != hipSuccess || hipMalloc(&S.coef, 6 * (size_t)(m + n) * 8) != hipSuccess ||
      hipMalloc((void**)&S.part, 2 * (size_t)S.nparts * 8) != hipSuccess ||
      hipMalloc((void**)&S.ctl, sizeof(SylCtl)) != hipSuccess ||
      hipHostMalloc((void**)&S.ctl_host, sizeof(SylCtl)) != hipSuccess ||
      hipMalloc((void**)&S.gmax, 4) != hipSuccess ||
      hipEventCreate(&S.ev0) != hipSuccess || hipEventCreate(&S.ev1) != hipSuccess)
    return fail(GADI_ENOMEM);
  if (hipMemcpy(S.dA, a3.data(), a3.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(S.dB, b3.data(), b3.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
    return fail(GADI_EHIP);
  *out = h;
  return GADI_OK;
}

extern "C" gadi_status gadi_sylv_solve(gadi_sylv* h, const double* C, double* X, double alpha, double omega,
                                       double tol, const gadi_options* opts, gadi_solve_info* info) {
  if (info) {
    info->status = GADI_EINVAL;
    info->outer_sweeps = 0;
    info->inner_H = info->inner_S = 0;
    info->relres = 0.0;
    info->seconds = 0.0;
    info->alpha = alpha;
    info->omega = omega;
    info->fell_back = 0;
    info->barriers = 0;
    info->barrier_seconds = 0.0;
  }
  if (!h || !C || !X) return GADI_EINVAL;
  if (!(alpha > 0.0) || !std::isfinite(alpha) || !(omega >= 0.0 && omega < 2.0) || !(tol >= 0.0) ||
      !std::isfinite(tol))
    return GADI_EINVAL;
  gadi_options o;
  if (opts) o = *opts;
  else gadi_default_options(&o, GADI_PREC_FP16_IR);
  if (o.prec < GADI_PREC_FP64 || o.prec > GADI_PREC_FP32_IR || o.maxit_outer < 0) return GADI_EINVAL;
  SylSystem& S = h->s;
  GADI_HIP_CHECK(hipSetDevice(S.device));
  const size_t bytes = (size_t)S.m * S.n * sizeof(double);
  const hipMemcpyKind kin = o.on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  const hipMemcpyKind kout = o.on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  GADI_HIP_CHECK(hipMemcpyAsync(S.dC, C, bytes, kin, S.stream));
  GADI_HIP_CHECK(hipMemcpyAsync(S.dX, X, bytes, kin, S.stream));
  gadi_status st;
  const bool rec = o.record_history != 0;
  if (o.prec == GADI_PREC_FP64) st = run<double, 2>(S, alpha, omega, tol, o.maxit_outer, rec, info);
  else if (o.prec == GADI_PREC_FP32_IR) st = run<float, 0>(S, alpha, omega, tol, o.maxit_outer, rec, info);
  else st = run<float, 1>(S, alpha, omega, tol, o.maxit_outer, rec, info);
  if (st == GADI_EHIP || st == GADI_EINVAL || st == GADI_ENOMEM) return st;
  GADI_HIP_CHECK(hipMemcpyAsync(X, S.dX, bytes, kout, S.stream));
  GADI_HIP_CHECK(hipStreamSynchronize(S.stream));
  return st;
}

extern "C" int32_t gadi_sylv_get_history(gadi_sylv* h, double* out, int32_t cap) {
  if (!h || !out || cap <= 0) return 0;
  const int k = (int)h->s.hist.size() < cap ? (int)h->s.hist.size() : cap;
  for (int i = 0; i < k; ++i) out[i] = h->s.hist[i];
  return k;
}

extern "C" gadi_status gadi_sylv_set_stream(gadi_sylv* h, void* hip_stream) {
  if (!h) return GADI_EINVAL;
  h->s.stream = (hipStream_t)hip_stream;
  return GADI_OK;
}

extern "C" gadi_status gadi_sylv_destroy(gadi_sylv* h) {
  if (!h) return GADI_EINVAL;
  SylSystem& S = h->s;
  void* ptrs[] = {S.dA, S.dB, S.dX, S.dC, S.R, S.Zh, S.chain, S.coef, S.part, S.ctl, S.dhist, S.gmax};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (S.ctl_host) (void)hipHostFree(S.ctl_host);
  if (S.ev0) (void)hipEventDestroy(S.ev0);
  if (S.ev1) (void)hipEventDestroy(S.ev1);
  delete h;
  return GADI_OK;
}
