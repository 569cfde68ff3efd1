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
//   residual (double) -> partial sums and stopping test -> column chunks ->
//   column chains (also bound max |G|) -> row chunks, which apply the column
//   correction and form G while staging LDS tiles -> row chains -> row
//   correction fused with the update of X (double).
// X, C and the work arrays are m x n row-major.
#include <cmath>
#include <cstdio>
#include <vector>

#include "device_common.h"

namespace gadi {

constexpr int kChunk = 64;         // rows of a chunk of the recurrences
constexpr int kSylBlock = 256;     // threads of the elementwise kernels
constexpr int kSylMax = 1 << 15;   // largest m or n
constexpr int kRowsPer = 16;       // rows per block of the residual and update kernels
static_assert(kChunk == 64, "the row tiles of the row solves are one column chunk high");

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
  const IT* qm;  // per chunk: max |q_i|, max |h_i| over the chunk's rows
  const IT* hm;
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
// R = C - A X - X B in double.  Block (bx, by): columns bx*256 + t, rows
// [by*kRowsPer, ...); X rows roll through registers, the column neighbours come
// from the lanes' shared cache lines.  Per-block sum of squares and max |r|
// into part.
template <class IT>
__global__ void __launch_bounds__(kSylBlock) syl_residual_kernel(
    const double* __restrict__ X, const double* __restrict__ C, const double* __restrict__ a_sub,
    const double* __restrict__ a_diag, const double* __restrict__ a_sup, const double* __restrict__ b_sub,
    const double* __restrict__ b_diag, const double* __restrict__ b_sup, IT* __restrict__ R, int m, int n,
    double* __restrict__ part, const SylCtl* __restrict__ ctl) {
  __shared__ double sh[kSylBlock / 64][2];
  if (ctl->done) return;
  const int j = blockIdx.x * kSylBlock + threadIdx.x;
  const int i0 = blockIdx.y * kRowsPer;
  const int i1 = i0 + kRowsPer < m ? i0 + kRowsPer : m;
  double s2 = 0.0, mx = 0.0;
  if (j < n) {
    // Every load of the block's rows is issued before the arithmetic.
    // Out-of-range neighbours are read at a clamped in-range index and meet a
    // zero coefficient: sub/sup of A and B end with a zero entry.
    const double bd = b_diag[j];
    const double bl = j > 0 ? b_sup[j > 0 ? j - 1 : 0] : 0.0;  // B[j-1][j]
    const double br = b_sub[j];                                // B[j+1][j] (0 in the last column)
    const int dl = j > 0 ? 1 : 0, dr = j + 1 < n ? 1 : 0;
    double xv[kRowsPer + 2], cv[kRowsPer], xl[kRowsPer], xr[kRowsPer];
#pragma unroll
    for (int r = 0; r < kRowsPer + 2; ++r) {
      int i = i0 - 1 + r;
      i = i < 0 ? 0 : (i < m ? i : m - 1);
      xv[r] = X[(size_t)i * n + j];
    }
#pragma unroll
    for (int r = 0; r < kRowsPer; ++r) {
      const size_t k = (size_t)(i0 + r < m ? i0 + r : m - 1) * n + j;
      cv[r] = C[k];
      xl[r] = X[k - dl];
      xr[r] = X[k + dr];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 0; r < kRowsPer; ++r) {
      const int i = i0 + r;
      if (i < i1) {
        const double al = i > 0 ? a_sub[i > 0 ? i - 1 : 0] : 0.0;
        const double ax = a_diag[i] * xv[r + 1] + al * xv[r] + a_sup[i] * xv[r + 2];
        const double xb = xv[r + 1] * bd + xl[r] * bl + xr[r] * br;
        const double res = cv[r] - ax - xb;
        R[(size_t)i * n + j] = (IT)res;
        s2 += res * res;
        mx = fmax(mx, fabs(res));
      }
    }
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
    const int blk = blockIdx.y * gridDim.x + blockIdx.x;
    part[2 * blk] = a;
    part[2 * blk + 1] = b;
  }
}

// Fixed-order combination of the residual partials and the stopping test of
// Algorithm 1; clears the max |G| word for the sweep that follows.
__global__ void __launch_bounds__(kSylBlock) syl_reduce_kernel(const double* __restrict__ part, int nparts,
                                                               SylCtl* __restrict__ ctl, double* __restrict__ hist,
                                                               int hist_cap, int scale_rhs,
                                                               unsigned* __restrict__ gmax) {
  __shared__ double sh[kSylBlock / 64][2];
  if (ctl->done) return;
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < nparts; k += kSylBlock) {
    a += part[2 * k];
    b = fmax(b, part[2 * k + 1]);
  }
  a = wave_sum(a);
  b = wave_max(b);
  if ((threadIdx.x & 63) == 0) {
    sh[threadIdx.x >> 6][0] = a;
    sh[threadIdx.x >> 6][1] = b;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  a = 0.0;
  b = 0.0;
  for (int w = 0; w < kSylBlock / 64; ++w) {
    a += sh[w][0];
    b = fmax(b, sh[w][1]);
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

// Lane k's value of v for the whole wavefront (k wave-uniform).
template <class T>
__device__ __forceinline__ T lane_value(T v, int k) {
  if constexpr (sizeof(T) == 8) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, k);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), k);
    return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), k));
  }
}

// ---------------------------------------------------------------------- column solves
// One thread per (column j, chunk c): local recurrences over the chunk's rows.
// v_i = stor(R_ij * scale) (MODE 1: half storage of the right-hand side).  The
// chunk's rows are loaded at once (clamped indexes, no branches between the
// loads); lane k of each wavefront holds the coefficients of row s + k, which
// the recurrences read with lane broadcasts.  All lanes stay active until the
// broadcasts are done.
template <class IT, int MODE>
__global__ void __launch_bounds__(kSylBlock) syl_col_local_kernel(const IT* __restrict__ R, Factors<IT> F,
                                                                  const SylCtl* __restrict__ ctl, int n,
                                                                  IT* __restrict__ Zh, IT* __restrict__ yend,
                                                                  IT* __restrict__ zbeg, IT* __restrict__ zmx) {
  if (ctl->done) return;
  const IT scale = (IT)ctl->scale1;
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  const int s = c * kChunk;
  const int len = F.len - s < kChunk ? F.len - s : kChunk;
  const int ic = s + (lane < len ? lane : len - 1);
  const IT lk = F.l[ic], sk = F.sup[ic], pk = F.ip[ic];
  const int jc = j < n ? j : n - 1;
  IT y[kChunk];
#pragma unroll
  for (int k = 0; k < kChunk; ++k) y[k] = R[(size_t)(s + (k < len ? k : len - 1)) * n + jc];
  __builtin_amdgcn_sched_barrier(0);  // every load of the chunk in flight before the recurrences
  IT prev = 0;
#pragma unroll
  for (int k = 0; k < kChunk; ++k) {
    const IT v = stor<MODE>(y[k] * scale);
    const IT np = k == 0 ? v : v - lane_value(lk, k) * prev;
    prev = k < len ? np : prev;
    y[k] = prev;
  }
  IT z = 0, zm = 0;
#pragma unroll
  for (int k = kChunk - 1; k >= 0; --k) {
    const IT nz = (y[k] - lane_value(sk, k) * z) * lane_value(pk, k);
    z = k < len ? nz : z;
    if (k < len && j < n) Zh[(size_t)(s + k) * n + j] = z;
    zm = fmax(zm, fabs(z));
  }
  if (j < n) {
    yend[(size_t)c * n + j] = prev;  // y^ of the chunk's last row
    zbeg[(size_t)c * n + j] = z;
    zmx[(size_t)c * n + j] = zm;
  }
}

// The chunk-boundary chains: B_c = y_{s_c - 1} (B_0 = 0), E_c = z_{e_c}
// (E_last = 0).  Across chunks each chain is an affine recurrence,
//   B_{c+1} = yend_c + f_{e_c - 1} B_c,
//   E_{c-1} = zbeg_c + B_c q_{s_c} + h_{s_c} E_c,
// so it runs as a two-level scan: a block holds kChainCols columns and splits
// each column's chunks into kChainParts consecutive ranges, one per thread.
// A thread composes the affine maps of its range, one thread per column chains
// the composed maps through LDS, and every thread then reruns its range from
// its true entry value, writing the boundary values.  A range of at most
// kChainBatch chunks keeps its inputs in registers through both chains (one
// round of loads); a longer one reloads them per pass, and its backward chain
// reads back the B_c its own thread wrote.  With zmx given (column direction), the kernel
// also bounds max |G| = |gscale| max |z| by max over chunks of
// max|z^| + |B_c| max|q| + |E_c| max|h| into gmax.
constexpr int kChainCols = 16;
constexpr int kChainParts = 16;
constexpr int kChainBlock = kChainCols * kChainParts;
constexpr int kChainBatch = 4;  // chunks whose loads are issued together

template <class IT>
__global__ void __launch_bounds__(kChainBlock) syl_chain_kernel(const IT* __restrict__ yend, const IT* __restrict__ zbeg,
                                                              Factors<IT> F, int nchunks, int width,
                                                              IT* __restrict__ Bc, IT* __restrict__ Ec,
                                                              const IT* __restrict__ zmx, IT gscale,
                                                              unsigned* __restrict__ gmax,
                                                              const SylCtl* __restrict__ ctl) {
  if (ctl->done) return;
  __shared__ IT s_c[kChainParts][kChainCols], s_m[kChainParts][kChainCols];
  __shared__ float s_bound[kChainBlock / 64];
  const int col = threadIdx.x % kChainCols, part = threadIdx.x / kChainCols;
  const int j = blockIdx.x * kChainCols + col;
  const bool live = j < width;
  const int jc = live ? j : width - 1;
  const int per = (nchunks + kChainParts - 1) / kChainParts;
  const int lo = part * per < nchunks ? part * per : nchunks;
  const int hi = lo + per < nchunks ? lo + per : nchunks;
  // entry values of the parts, from the composed maps (cst, mul) of every part:
  // forward = true chains part 0 upward, else part kChainParts - 1 downward
  auto chain_parts = [&](IT cst, IT mul, bool forward) -> IT {
    s_c[part][col] = cst;
    s_m[part][col] = mul;
    __syncthreads();
    if (part == 0) {
      IT v = 0;
      for (int k = 0; k < kChainParts; ++k) {
        const int p = forward ? k : kChainParts - 1 - k;
        const IT c = s_c[p][col], m = s_m[p][col];
        s_c[p][col] = v;
        v = c + m * v;
      }
    }
    __syncthreads();
    const IT entry = s_c[part][col];
    __syncthreads();  // the arrays are reused by the next chain
    return entry;
  };
  // block maximum of the column bound into gmax
  auto chain_bound = [&](IT bound) {
    if (!zmx) return;
    float v = live ? (float)(fabs(gscale) * bound) : 0.f;
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) s_bound[threadIdx.x / 64] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      float mx = s_bound[0];
      for (int w = 1; w < kChainBlock / 64; ++w) mx = fmaxf(mx, s_bound[w]);
      atomicMax(gmax, __float_as_uint(mx));
    }
  };
  if (per <= kChainBatch) {
    // a range of at most kChainBatch chunks: every input of the range is
    // loaded at once and kept in registers through both chains
    IT ye[kChainBatch], ff[kChainBatch], zb[kChainBatch], qq[kChainBatch], hh[kChainBatch], zm[kChainBatch],
        bb[kChainBatch];
#pragma unroll
    for (int u = 0; u < kChainBatch; ++u) {
      // an empty range has lo = hi = nchunks: its clamped loads stay in bounds
      const int c = lo + u < hi ? lo + u : hi - 1;
      const int s = c * kChunk;
      const int e = (c + 1) * kChunk < F.len ? (c + 1) * kChunk : F.len;
      ye[u] = yend[(size_t)c * width + jc];
      ff[u] = F.f[e - 1];
      zb[u] = zbeg[(size_t)c * width + jc];
      qq[u] = F.q[s];
      hh[u] = F.h[s];
      zm[u] = zmx ? zmx[(size_t)c * width + jc] : IT(0);
    }
    IT cst = 0, mul = 1;
#pragma unroll
    for (int u = 0; u < kChainBatch; ++u)
      if (lo + u < hi) {
        cst = ye[u] + ff[u] * cst;
        mul = ff[u] * mul;
      }
    IT b = chain_parts(cst, mul, true);
#pragma unroll
    for (int u = 0; u < kChainBatch; ++u) {
      bb[u] = b;
      if (lo + u < hi) {
        if (live) Bc[(size_t)(lo + u) * width + j] = b;
        b = ye[u] + ff[u] * b;
      }
    }
    cst = 0;
    mul = 1;
#pragma unroll
    for (int u = kChainBatch - 1; u >= 0; --u)
      if (lo + u < hi) {
        cst = zb[u] + bb[u] * qq[u] + hh[u] * cst;
        mul = hh[u] * mul;
      }
    IT ez = chain_parts(cst, mul, false);
    IT bound = 0;
#pragma unroll
    for (int u = kChainBatch - 1; u >= 0; --u) {
      const int c = lo + u;
      if (c < hi) {
        if (live) Ec[(size_t)c * width + j] = ez;
        if (zmx) bound = fmax(bound, zm[u] + fabs(bb[u]) * F.qm[c] + fabs(ez) * F.hm[c]);
        ez = zb[u] + bb[u] * qq[u] + ez * hh[u];
      }
    }
    chain_bound(bound);
    return;
  }
  // forward chain: compose, chain the parts, rerun writing B_c
  IT cst = 0, mul = 1;
  for (int c0 = lo; c0 < hi; c0 += kChainBatch) {
    IT ye[kChainBatch], ff[kChainBatch];
#pragma unroll
    for (int u = 0; u < kChainBatch; ++u) {
      const int c = c0 + u < hi ? c0 + u : hi - 1;
      const int e = (c + 1) * kChunk < F.len ? (c + 1) * kChunk : F.len;
      ye[u] = yend[(size_t)c * width + jc];
      ff[u] = F.f[e - 1];
    }
#pragma unroll
    for (int u = 0; u < kChainBatch; ++u)
      if (c0 + u < hi) {
        cst = ye[u] + ff[u] * cst;
        mul = ff[u] * mul;
      }
  }
  IT b = chain_parts(cst, mul, true);
  for (int c0 = lo; c0 < hi; c0 += kChainBatch) {
    IT ye[kChainBatch], ff[kChainBatch];
#pragma unroll
    for (int u = 0; u < kChainBatch; ++u) {
      const int c = c0 + u < hi ? c0 + u : hi - 1;
      const int e = (c + 1) * kChunk < F.len ? (c + 1) * kChunk : F.len;
      ye[u] = yend[(size_t)c * width + jc];
      ff[u] = F.f[e - 1];
    }
#pragma unroll
    for (int u = 0; u < kChainBatch; ++u) {
      const int c = c0 + u;
      if (c < hi) {
        if (live) Bc[(size_t)c * width + j] = b;
        b = ye[u] + ff[u] * b;
      }
    }
  }
  // backward chain over the same ranges, chunks in descending order; a live
  // thread reads back the B_c it wrote above
  cst = 0;
  mul = 1;
  for (int c1 = hi - 1; c1 >= lo; c1 -= kChainBatch) {
    IT kk[kChainBatch], hh[kChainBatch];
#pragma unroll
    for (int u = 0; u < kChainBatch; ++u) {
      const int c = c1 - u >= lo ? c1 - u : lo;
      const int s = c * kChunk;
      const IT bb = live ? Bc[(size_t)c * width + j] : IT(0);
      kk[u] = zbeg[(size_t)c * width + jc] + bb * F.q[s];
      hh[u] = F.h[s];
    }
#pragma unroll
    for (int u = 0; u < kChainBatch; ++u)
      if (c1 - u >= lo) {
        cst = kk[u] + hh[u] * cst;
        mul = hh[u] * mul;
      }
  }
  IT ez = chain_parts(cst, mul, false);
  IT bound = 0;
  for (int c1 = hi - 1; c1 >= lo; c1 -= kChainBatch) {
    IT zb[kChainBatch], bb[kChainBatch], qq[kChainBatch], hh[kChainBatch], zm[kChainBatch];
#pragma unroll
    for (int u = 0; u < kChainBatch; ++u) {
      const int c = c1 - u >= lo ? c1 - u : lo;
      const int s = c * kChunk;
      zb[u] = zbeg[(size_t)c * width + jc];
      bb[u] = live ? Bc[(size_t)c * width + j] : IT(0);
      qq[u] = F.q[s];
      hh[u] = F.h[s];
      zm[u] = zmx ? zmx[(size_t)c * width + jc] : IT(0);
    }
#pragma unroll
    for (int u = 0; u < kChainBatch; ++u) {
      const int c = c1 - u;
      if (c >= lo) {
        if (live) Ec[(size_t)c * width + j] = ez;
        if (zmx) bound = fmax(bound, zm[u] + fabs(bb[u]) * F.qm[c] + fabs(ez) * F.hm[c]);
        ez = zb[u] + bb[u] * qq[u] + ez * hh[u];
      }
    }
  }
  chain_bound(bound);
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
// One wavefront per tile of 64 rows (one column chunk) x kChunk columns; lane t
// runs the chunk-local recurrences of row r0 + t.  The tile passes through LDS
// in slabs of kSlab columns so that global loads and stores run along the
// rows.  Reading a slab finishes the column solves, z = z^ + B q + E h, and
// forms v_ij = stor(G_ij 2^-e2) with G = (2 - omega) alpha z.  Lane t holds
// the row solve's coefficients and the column chains of column s + t, and the
// column coefficients q, h of row r0 + t.
constexpr int kSlab = 16;

template <class IT, int MODE>
__global__ void __launch_bounds__(64) syl_row_local_kernel(const IT* __restrict__ Zc, const IT* __restrict__ Bcol,
                                                           const IT* __restrict__ Ecol, Factors<IT> Fc, IT gscale,
                                                           Factors<IT> F, const unsigned* __restrict__ gmax, int m,
                                                           int n, IT* __restrict__ Zh, IT* __restrict__ yend,
                                                           IT* __restrict__ zbeg, const SylCtl* __restrict__ ctl) {
  __shared__ IT tile[64][kSlab + 1];
  if (ctl->done) return;
  const int t = threadIdx.x;
  const int c = blockIdx.x;
  const int r0 = blockIdx.y * 64;
  const int s = c * kChunk;
  const int len = n - s < kChunk ? n - s : kChunk;
  const IT sc = (IT)g_scale(gmax) * gscale;
  const int jt = s + (t < len ? t : len - 1);
  const IT lk = F.l[jt], sk = F.sup[jt], pk = F.ip[jt];
  const IT bq = Bcol[(size_t)blockIdx.y * n + jt], eh = Ecol[(size_t)blockIdx.y * n + jt];
  const int row = r0 + t;
  const int rc = row < m ? row : m - 1;
  const IT qr = Fc.q[rc], hr = Fc.h[rc];
  const int sl = t % kSlab, sr = t / kSlab;  // slab column and first row of this lane's slab loads
  constexpr int kPer = 64 * kSlab / 64;      // slab elements per lane
  IT y[kChunk];
  IT prev = 0;
#pragma unroll
  for (int q = 0; q < kChunk / kSlab; ++q) {
    const int col = q * kSlab + sl;
    const int jj = s + (col < len ? col : len - 1);
    IT v[kPer];
#pragma unroll
    for (int kk = 0; kk < kPer; ++kk) {
      const int i = r0 + sr + (64 / kSlab) * kk;
      v[kk] = Zc[(size_t)(i < m ? i : m - 1) * n + jj];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int kk = 0; kk < kPer; ++kk) tile[sr + (64 / kSlab) * kk][sl] = v[kk];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSlab; ++k) {
      const int kc = q * kSlab + k;
      const IT zc = tile[t][k] + lane_value(bq, kc) * qr + lane_value(eh, kc) * hr;
      const IT vv = stor<MODE>(zc * sc);
      const IT np = kc == 0 ? vv : vv - lane_value(lk, kc) * prev;
      prev = kc < len ? np : prev;
      y[kc] = prev;
    }
    __syncthreads();
  }
  IT z = 0;
#pragma unroll
  for (int q = kChunk / kSlab - 1; q >= 0; --q) {
#pragma unroll
    for (int k = kSlab - 1; k >= 0; --k) {
      const int kc = q * kSlab + k;
      const IT nz = (y[kc] - lane_value(sk, kc) * z) * lane_value(pk, kc);
      z = kc < len ? nz : z;
      tile[t][k] = z;
    }
    __syncthreads();
    const int col = q * kSlab + sl;
#pragma unroll
    for (int kk = 0; kk < kPer; ++kk) {
      const int i = r0 + sr + (64 / kSlab) * kk;
      if (i < m && col < len) Zh[(size_t)i * n + s + col] = tile[sr + (64 / kSlab) * kk][sl];
    }
    __syncthreads();
  }
  if (row < m) {
    yend[(size_t)c * m + row] = prev;
    zbeg[(size_t)c * m + row] = z;
  }
}

// y = z^ + B q + E h along the rows, stored in the inner precision, then
// X += y 2^(e1 + e2) in double.  Block (bx, by): columns bx*256 + t, rows
// [by*kRowsPer, ...); a wavefront's 64 columns lie in one chunk, so B and E
// are wave-uniform loads.
template <class IT, int MODE>
__global__ void __launch_bounds__(kSylBlock) syl_row_fix_update_kernel(const IT* __restrict__ Zh,
                                                                       const IT* __restrict__ Bc,
                                                                       const IT* __restrict__ Ec, Factors<IT> F,
                                                                       const unsigned* __restrict__ gmax,
                                                                       const SylCtl* __restrict__ ctl, int m, int n,
                                                                       double* __restrict__ X) {
  if (ctl->done) return;
  const int j = blockIdx.x * kSylBlock + threadIdx.x;
  if (j >= n) return;
  const double unscale = 1.0 / (ctl->scale1 * (double)g_scale(gmax));
  const int c = j / kChunk;
  const IT q = F.q[j], h = F.h[j];
  const int i0 = blockIdx.y * kRowsPer;
  IT zv[kRowsPer], bv[kRowsPer], ev[kRowsPer];
  double xo[kRowsPer];
#pragma unroll
  for (int r = 0; r < kRowsPer; ++r) {
    const int i = i0 + r < m ? i0 + r : m - 1;
    const size_t k = (size_t)i * n + j;
    zv[r] = Zh[k];
    bv[r] = Bc[(size_t)c * m + i];
    ev[r] = Ec[(size_t)c * m + i];
    xo[r] = X[k];
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int r = 0; r < kRowsPer; ++r) {
    const int i = i0 + r;
    if (i < m) {
      const IT y = stor<MODE>(zv[r] + bv[r] * q + ev[r] * h);
      X[(size_t)i * n + j] = xo[r] + (double)y * unscale;
    }
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
  void* chain = nullptr; // yend, zbeg, B, E, max|z^|: 5 * chunks * max(m, n)
  void* coef = nullptr;  // per direction l, 1/p, sup, f, q, h and per-chunk max|q|, max|h|
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
  const int nch = (len + kChunk - 1) / kChunk;
  out.assign(6 * (size_t)len + 2 * (size_t)nch, 0.0);
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
    double qm = 0.0, hm = 0.0;
    for (int i = s; i < e; ++i) {
      qm = std::fmax(qm, std::fabs(q[i]));
      hm = std::fmax(hm, std::fabs(h[i]));
    }
    // rounded up by a few ulps so that the bound survives the conversion to the inner type
    out[6 * (size_t)len + s / kChunk] = qm * (1.0 + 1e-6);
    out[6 * (size_t)len + nch + s / kChunk] = hm * (1.0 + 1e-6);
  }
}

template <class IT>
static gadi_status upload_coef(SylSystem& S, const std::vector<double>& col, const std::vector<double>& row) {
  std::vector<IT> buf(col.size() + row.size());
  for (size_t k = 0; k < col.size(); ++k) buf[k] = (IT)col[k];
  for (size_t k = 0; k < row.size(); ++k) buf[col.size() + k] = (IT)row[k];
  GADI_HIP_CHECK(hipMemcpyAsync(S.coef, buf.data(), buf.size() * sizeof(IT), hipMemcpyHostToDevice, S.stream));
  GADI_HIP_CHECK(hipStreamSynchronize(S.stream));
  return GADI_OK;
}

static size_t coef_len(int len) { return 6 * (size_t)len + 2 * (size_t)((len + kChunk - 1) / kChunk); }

template <class IT>
static Factors<IT> factors_at(const SylSystem& S, int which) {
  const IT* base = (const IT*)S.coef + (which == 0 ? 0 : coef_len(S.m));
  const int len = which == 0 ? S.m : S.n;
  const int nch = (len + kChunk - 1) / kChunk;
  const IT* qm = base + 6 * (size_t)len;
  return Factors<IT>{base,           base + len,     base + 2 * len, base + 3 * len, base + 4 * len,
                     base + 5 * len, qm,             qm + nch,       len};
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
  IT* zmx = Ec + pw;
  const Factors<IT> Fc = factors_at<IT>(S, 0), Fr = factors_at<IT>(S, 1);
  const IT gs = (IT)((2.0 - omega) * alpha);
  IT* R = (IT*)S.R;
  IT* Zh = (IT*)S.Zh;
  const dim3 g2((n + kSylBlock - 1) / kSylBlock, (m + kRowsPer - 1) / kRowsPer);
  hipLaunchKernelGGL((syl_residual_kernel<IT>), g2, dim3(kSylBlock), 0, S.stream, S.dX, S.dC, S.dA, S.dA + m,
                     S.dA + 2 * m, S.dB, S.dB + n, S.dB + 2 * n, R, m, n, S.part, S.ctl);
  hipLaunchKernelGGL(syl_reduce_kernel, dim3(1), dim3(kSylBlock), 0, S.stream, S.part, S.nparts, S.ctl, S.dhist,
                     S.hist_cap, MODE == 2 ? 0 : 1, S.gmax);
  // column chunks: one wavefront per block unless 256-thread blocks already
  // give a few blocks per compute unit
  const int cb = (size_t)((n + kSylBlock - 1) / kSylBlock) * pc >= 1024 ? kSylBlock : 64;
  hipLaunchKernelGGL((syl_col_local_kernel<IT, MODE>), dim3((n + cb - 1) / cb, pc), dim3(cb), 0, S.stream, R, Fc,
                     S.ctl, n, Zh, yend, zbeg, zmx);
  hipLaunchKernelGGL((syl_chain_kernel<IT>), dim3((n + kChainCols - 1) / kChainCols), dim3(kChainBlock), 0, S.stream,
                     yend, zbeg, Fc, pc, n, Bc, Ec, zmx, gs, S.gmax, S.ctl);
  // the row solves read z^ (Zh) and the column chains (Bc, Ec), and write their
  // chunk-local solutions to R and their chain inputs to yend, zbeg
  hipLaunchKernelGGL((syl_row_local_kernel<IT, MODE>), dim3(pr, (m + 63) / 64), dim3(64), 0, S.stream, Zh, Bc, Ec, Fc,
                     gs, Fr, S.gmax, m, n, R, yend, zbeg, S.ctl);
  hipLaunchKernelGGL((syl_chain_kernel<IT>), dim3((m + kChainCols - 1) / kChainCols), dim3(kChainBlock), 0, S.stream,
                     yend, zbeg, Fr, pr, m, Bc, Ec, (const IT*)nullptr, IT(0), S.gmax, S.ctl);
  hipLaunchKernelGGL((syl_row_fix_update_kernel<IT, MODE>), g2, dim3(kSylBlock), 0, S.stream, R, Bc, Ec, Fr, S.gmax,
                     S.ctl, m, n, S.dX);
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
  {
    const hipError_t e = hipGetDevice(&S.device);
    if (e != hipSuccess) return fail(fail_hip(e, "hipGetDevice", __FILE__, __LINE__));
  }
  const size_t mn = (size_t)m * n;
  const size_t w = (size_t)(m > n ? m : n);
  static_assert(((kSylMax + kSylBlock - 1) / kSylBlock) * ((kSylMax + kRowsPer - 1) / kRowsPer) < (1 << 30),
                "partials fit int");
  const size_t pmax = (size_t)(chunks_of(m) > chunks_of(n) ? chunks_of(m) : chunks_of(n));
  S.nparts = ((n + kSylBlock - 1) / kSylBlock) * ((m + kRowsPer - 1) / kRowsPer);
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
      hipMalloc(&S.chain, 5 * pmax * w * 8) != hipSuccess || hipMalloc(&S.coef, (coef_len(m) + coef_len(n)) * 8) != hipSuccess ||
      hipMalloc((void**)&S.part, 2 * (size_t)S.nparts * 8) != hipSuccess ||
      hipMalloc((void**)&S.ctl, sizeof(SylCtl)) != hipSuccess ||
      hipHostMalloc((void**)&S.ctl_host, sizeof(SylCtl)) != hipSuccess ||
      hipMalloc((void**)&S.gmax, 4) != hipSuccess ||
      hipEventCreate(&S.ev0) != hipSuccess || hipEventCreate(&S.ev1) != hipSuccess)
    return fail(GADI_ENOMEM);
  for (int k = 0; k < 2; ++k) {
    const hipError_t e = k == 0 ? hipMemcpy(S.dA, a3.data(), a3.size() * 8, hipMemcpyHostToDevice)
                                : hipMemcpy(S.dB, b3.data(), b3.size() * 8, hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(fail_hip(e, "hipMemcpy of the coefficients", __FILE__, __LINE__));
  }
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
