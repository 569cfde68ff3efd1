// The refinement loop of Algorithm 1 (Section 2.1), written once and run under
// two synchronisation policies: device-wide (one large system per cooperative
// launch, solve.hip) and block-local (one system per block, batched.hip).
//
// One outer sweep:
//   a1  r = b - A x in double, ||r||_2^2 and ||r||_inf                 (step 1)
//   a2  stop if ||r|| <= tol ||r_0||, diverged, or sweep limit        (while test)
//   a3  CG on (alpha I + H) z = r * 2^-e1 with e1 from ||r||_inf      (step 2)
//   a4  g = (2 - omega) z * 2^-e2 with e2 from ||z||_inf               (step 3 rhs)
//   a5  CGNE on (I + S/alpha) u = g:
//         CG on (I - S^2/alpha^2) w = g, u = (I - S/alpha) w          (step 3)
//   a6  x += u * 2^(e1 + e2) in double                                (step 4)
// Dividing the S-step by alpha turns (alpha I + S) y = (2 - omega) alpha z into
// (I + S/alpha) y = (2 - omega) z, so alpha never enters a stored half value;
// the exact power-of-two scalings keep every half-precision right-hand side
// in [1/2, 1) in max norm.
//
// The CG recurrences fold the direction update into the product phase:
// q_{k+1} = K p_{k+1} = K r_{k+1} + beta q_k, so each CG step needs two
// reductions and one operator product.
#pragma once

#include <cmath>

#include "device_common.h"

namespace gadi {

struct SolveArgs {
  int n, npad, ntiles, maxit_out, maxit_in, hist_cap;
  const int32_t* slice_ptr;
  const int32_t* col;
  const int32_t* slice_dia;
  const int32_t* dia_off;
  const double* a_off;
  const double* a_diag;
  const void* h_off;
  const void* s_off;
  const void* h_diag;
  const double* b;
  double* x;
  void* r;
  void* z;
  void* w;
  void* v[8];  // storage-precision vectors: r (2), w (2), s (2), p, t
  double alpha, omega, tol, eps_h, eps_s;
  SyncState* sync;
  unsigned long long* flags;
  double* part;
  double* result;
  DevInfo* info;
  double* hist;
  long long timeout;
  // Batched sweeps only: best work (operator products) of a converged trial
  // of this system so far; a trial stops (EMAXIT) once its own work exceeds it.
  unsigned long long* prune;
  // optional per-phase profile of block 0: wall-clock ticks [10], phase counts [10]
  long long* prof;
};

// Reduction into out[4] under the caller's synchronisation policy; leaves the
// solve if a device-wide barrier timed out.
#define ALLREDUCE(a0, a1, a2, a3)                                  \
  do {                                                             \
    bool ok_;                                                      \
    const Red4 r_ = red.reduce((a0), (a1), (a2), (a3), ok_);       \
    if (!ok_) return false;                                        \
    out[0] = r_.v[0];                                              \
    out[1] = r_.v[1];                                              \
    out[2] = r_.v[2];                                              \
    out[3] = r_.v[3];                                              \
  } while (0)

// Synchronisation policy of one large system: every block of a cooperative
// launch owns a band of rows; phases are separated by device-wide barriers.
template <int BLOCK>
struct GridRed {
  Grid g;
  __device__ __forceinline__ Red4 reduce(double s0, double s1, double s2, double m3, bool& ok) {
    return grid_allreduce<BLOCK>(g, s0, s1, s2, m3, ok);
  }
  // pruning needs one value seen identically by every block; not offered here
  __device__ __forceinline__ unsigned long long broadcast_load(const unsigned long long*) { return ~0ull; }
  __device__ __forceinline__ void publish_min(unsigned long long*, unsigned long long) {}
};

// Synchronisation policy of the batched sweep: one block owns a whole system,
// so a phase ends at a block barrier and reductions stay in LDS (combined in
// wavefront order, a fixed order).
template <int BLOCK>
struct BlockRed {
  long long barriers = 0;
  __device__ __forceinline__ Red4 reduce(double s0, double s1, double s2, double m3, bool& ok) {
    constexpr int NW = BLOCK / 64;
    __shared__ double sh[NW][4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const double a0 = wave_sum(s0), a1 = wave_sum(s1), a2 = wave_sum(s2), a3 = wave_max(m3);
    if (lane == 0) {
      sh[wid][0] = a0;
      sh[wid][1] = a1;
      sh[wid][2] = a2;
      sh[wid][3] = a3;
    }
    __syncthreads();
    Red4 r;
    r.v[0] = r.v[1] = r.v[2] = r.v[3] = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      r.v[0] += sh[w][0];
      r.v[1] += sh[w][1];
      r.v[2] += sh[w][2];
      r.v[3] = fmax(r.v[3], sh[w][3]);
    }
    __syncthreads();  // sh is rewritten by the next call
    ++barriers;
    ok = true;
    return r;
  }
  // thread 0 reads, the block agrees on the value
  __device__ __forceinline__ unsigned long long broadcast_load(const unsigned long long* p) {
    __shared__ unsigned long long v;
    if (threadIdx.x == 0) v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const unsigned long long r = v;
    __syncthreads();
    return r;
  }
  __device__ __forceinline__ void publish_min(unsigned long long* p, unsigned long long v) {
    if (threadIdx.x == 0) atomicMin(p, v);
  }
};

// The same, charging the block-0 time since the previous reduction to phase
// `id` of the optional per-phase profile (a.prof: ticks[10], counts[10]).
#define ALLREDUCE_P(id, a0, a1, a2, a3)                                    \
  do {                                                                     \
    if (a.prof && blockIdx.x == 0 && threadIdx.x == 0) {                   \
      const long long now_ = wall_clock64();                               \
      a.prof[(id)] += now_ - t_mark;                                       \
      a.prof[10 + (id)] += 1;                                              \
    }                                                                      \
    ALLREDUCE(a0, a1, a2, a3);                                             \
    if (a.prof && blockIdx.x == 0 && threadIdx.x == 0) t_mark = wall_clock64(); \
  } while (0)

static __device__ __forceinline__ int clamp_exp(int e) { return e < -120 ? -120 : (e > 120 ? 120 : e); }

// The refinement loop of Algorithm 1 for rows [t0 * BLOCK, t1 * BLOCK) of one
// system.  Returns false if a barrier timed out; otherwise fills `res`.
//
// Both inner solves use the Chronopoulos-Gear form of CG: with w = K r and
// s = K p carried by recurrence, the two inner products of a step,
// gamma = r.r and delta = r.K r, come from one reduction.  Step k updates
//   s_k = w_k + beta_k s_{k-1},  p_k = r_k + beta_k p_{k-1},
//   z += a_k p_k,  r_{k+1} = r_k - a_k s_k,  w_{k+1} = K r_{k+1},
// with beta_k = gamma_k / gamma_{k-1} and a_k = gamma_k / (delta_k - beta_k gamma_k / a_{k-1}).
// (FUSED = true.)  The other variant (FUSED = false) is Hestenes-Stiefel CG
// with q_{k+1} = K p_{k+1} = K r_{k+1} + beta q_k folded into the product
// phase: two phases per CG step, three per CGNE step, but no recomputation.
// The product K r_{k+1} needs r_{k+1} at neighbouring rows, which other
// blocks are writing in the same phase; each block recomputes those values
// from r_k, w_k, s_{k-1} (read from the previous phase's buffers, hence
// ping-pong buffers for r, w, s) with the same fused operations and the same
// roundings as their owner, so every copy is bit-identical.  A CG step on
// alpha I + H is one phase; a CGNE step on I - (S/alpha)^2 is two (the
// second product needs the first one's result at neighbouring rows).
template <class AT>
__device__ __forceinline__ AT fma_at(AT a, AT b, AT c);
template <>
__device__ __forceinline__ float fma_at<float>(float a, float b, float c) {
  return fmaf(a, b, c);
}
template <>
__device__ __forceinline__ double fma_at<double>(double a, double b, double c) {
  return fma(a, b, c);
}

template <class Mode, int BLOCK, bool FUSED, class Red>
__device__ __forceinline__ bool solve_body(const SolveArgs& a, Red& red, int t0, int t1, DevInfo& res_out) {
  using MT = typename Mode::MT;
  using VT = typename Mode::VT;
  using ST = typename Mode::ST;
  using RT = typename Mode::RT;
  using AT = typename Mode::AT;

  const int tid = threadIdx.x;

  const Pattern pat{a.slice_ptr, a.col, a.slice_dia, a.dia_off, a.n - 1};
  const MT* __restrict__ hoff = (const MT*)a.h_off;
  const MT* __restrict__ soff = (const MT*)a.s_off;
  const MT* __restrict__ hdiag = (const MT*)a.h_diag;
  RT* __restrict__ r = (RT*)a.r;
  ST* __restrict__ z = (ST*)a.z;
  ST* __restrict__ wsol = (ST*)a.w;
  VT* const R[2] = {(VT*)a.v[0], (VT*)a.v[1]};
  VT* const W[2] = {(VT*)a.v[2], (VT*)a.v[3]};
  VT* const Sv[2] = {(VT*)a.v[4], (VT*)a.v[5]};
  VT* __restrict__ P = (VT*)a.v[6];
  VT* __restrict__ T = (VT*)a.v[7];
  double* __restrict__ x = a.x;
  const double* __restrict__ b = a.b;

  const AT alpha = (AT)a.alpha;
  const AT inv_alpha = (AT)(1.0 / a.alpha);
  const AT two_m_omega = (AT)(2.0 - a.omega);
  const double eps_h2 = a.eps_h * a.eps_h;
  const double eps_s2 = a.eps_s * a.eps_s;
  const int overflow_status = Mode::id == GADI_PREC_FP16_IR ? GADI_EOVERFLOW16 : GADI_EDIVERGED;

  // value rounded to the storage type and read back
  auto rnd = [](AT v) { return ld<AT>(st<VT>(v)); };

  double out[4];
  long long t_mark = (a.prof && blockIdx.x == 0 && threadIdx.x == 0) ? wall_clock64() : 0;
  double rho0 = 0.0, res = 0.0;
  int status = GADI_EMAXIT;
  int sweep = 0;
  long long ih = 0, is = 0;

  for (;;) {
    // ---------------------------------------------------------- a1: residual
    {
      double s0 = 0.0, m3 = 0.0;
      for (int t = t0; t < t1; ++t) {
        const int row = t * BLOCK + tid;
        const double ax = a.a_diag[row] * x[row] +
                          row_sum<double>(row, pat, a.a_off, [&](int c) { return x[c]; });
        const double ri = b[row] - ax;
        r[row] = (RT)ri;
        s0 += ri * ri;
        m3 = fmax(m3, fabs(ri));
      }
      ALLREDUCE_P(0, s0, 0.0, 0.0, m3);
    }
    const double rho = sqrt(out[0]);
    const double rmax = out[3];
    if (sweep == 0) rho0 = rho;
    res = rho0 > 0.0 ? rho / rho0 : 0.0;
    if (a.hist && sweep < a.hist_cap && blockIdx.x == 0 && tid == 0) a.hist[sweep] = res;
    if (rho <= a.tol * rho0) {
      status = GADI_OK;
      break;
    }
    if (!isfinite(rho) || rho > 1e6 * rho0) {
      status = GADI_EDIVERGED;
      break;
    }
    if (sweep >= a.maxit_out) {
      status = GADI_EMAXIT;
      break;
    }
    if (a.prune) {
      const unsigned long long wk = (unsigned long long)(ih + 2 * is + 3 * (long long)sweep);
      if (wk > red.broadcast_load(a.prune)) {
        status = GADI_EMAXIT;
        break;
      }
    }

    // ---------------------------------------------------------- a3: CG on alpha I + H
    int e1;
    (void)frexp(rmax, &e1);
    e1 = clamp_exp(e1);
    const AT sc1 = (AT)ldexp(1.0, -e1);
    double zmax = 0.0;
    int it = 0;
    if constexpr (FUSED) {
      {
        // r_0 = r * 2^-e1 in storage precision, w_0 = K r_0
        double g0 = 0.0, d0 = 0.0;
        for (int t = t0; t < t1; ++t) {
          const int row = t * BLOCK + tid;
          const AT ri = rnd((AT)r[row] * sc1);
          const AT kr = (alpha + ld<AT>(hdiag[row])) * ri +
                        row_sum<AT>(row, pat, hoff, [&](int c) { return rnd((AT)r[c] * sc1); });
          const AT wi = rnd(kr);
          R[0][row] = st<VT>(ri);
          W[0][row] = st<VT>(wi);
          g0 += (double)ri * (double)ri;
          d0 += (double)wi * (double)ri;
        }
        ALLREDUCE_P(1, g0, d0, 0.0, 0.0);
      }
      double gam = out[0], del = out[1];
      const double gam0 = gam;
      if (gam0 > 0.0) {
        double gam_prev = 1.0, a_prev = 1.0;
        for (int k = 0;; ++k) {
          const double beta = k == 0 ? 0.0 : gam / gam_prev;
          const double den = k == 0 ? del : del - beta * gam / a_prev;
          if (!(den > 0.0) || !isfinite(den)) {
            if (k == 0) status = isfinite(den) ? GADI_ENOTSPD : overflow_status;
            break;
          }
          const double ak = gam / den;
          const AT akt = (AT)ak, bkt = (AT)beta;
          const VT* __restrict__ rk = R[k & 1];
          const VT* __restrict__ wk = W[k & 1];
          const VT* __restrict__ sprev = Sv[(k + 1) & 1];
          VT* __restrict__ snew = Sv[k & 1];
          VT* __restrict__ rnew = R[(k + 1) & 1];
          VT* __restrict__ wnew = W[(k + 1) & 1];
          // r_{k+1} at row c, computed exactly as its owner computes it
          auto r_next = [&](int c) {
            const AT sc = k == 0 ? ld<AT>(wk[c]) : rnd(fma_at<AT>(bkt, ld<AT>(sprev[c]), ld<AT>(wk[c])));
            return rnd(fma_at<AT>(-akt, sc, ld<AT>(rk[c])));
          };
          double g1 = 0.0, d1 = 0.0, m3 = 0.0;
          for (int t = t0; t < t1; ++t) {
            const int row = t * BLOCK + tid;
            const AT ri = ld<AT>(rk[row]);
            const AT si = k == 0 ? ld<AT>(wk[row]) : rnd(fma_at<AT>(bkt, ld<AT>(sprev[row]), ld<AT>(wk[row])));
            const AT pi = k == 0 ? ri : rnd(fma_at<AT>(bkt, ld<AT>(P[row]), ri));
            const ST zi = (k == 0 ? ST(0) : z[row]) + (ST)(akt * pi);
            const AT rn = rnd(fma_at<AT>(-akt, si, ri));
            const AT kr = (alpha + ld<AT>(hdiag[row])) * rn + row_sum<AT>(row, pat, hoff, r_next);
            const AT wn = rnd(kr);
            snew[row] = st<VT>(si);
            P[row] = st<VT>(pi);
            z[row] = zi;
            rnew[row] = st<VT>(rn);
            wnew[row] = st<VT>(wn);
            g1 += (double)rn * (double)rn;
            d1 += (double)wn * (double)rn;
            m3 = fmax(m3, fabs((double)zi));
          }
          ALLREDUCE_P(2, g1, d1, 0.0, m3);
          gam_prev = gam;
          a_prev = ak;
          gam = out[0];
          del = out[1];
          zmax = out[3];
          it = k + 1;
          if (gam <= eps_h2 * gam0 || it >= a.maxit_in || !isfinite(gam)) break;
        }
      }
    } else {
      VT* __restrict__ vr = R[0];
      VT* __restrict__ vp = P;
      VT* __restrict__ vq = W[0];
      double pq, rr, rr0;
      {
        double s0 = 0.0, s1 = 0.0;
        for (int t = t0; t < t1; ++t) {
          const int row = t * BLOCK + tid;
          const VT pi = st<VT>((AT)r[row] * sc1);
          const AT api = ld<AT>(pi);
          const AT kp = (alpha + ld<AT>(hdiag[row])) * api +
                        row_sum<AT>(row, pat, hoff, [&](int c) { return ld<AT>(st<VT>((AT)r[c] * sc1)); });
          const VT qi = st<VT>(kp);
          vr[row] = pi;
          vp[row] = pi;
          vq[row] = qi;
          s0 += (double)api * (double)ld<AT>(qi);
          s1 += (double)api * (double)api;
        }
        ALLREDUCE_P(1, s0, s1, 0.0, 0.0);
        pq = out[0];
        rr0 = out[1];
        rr = rr0;
      }
      if (rr0 > 0.0) {
        for (;;) {
          if (!(pq > 0.0) || !isfinite(pq)) {
            if (it == 0) status = isfinite(pq) ? GADI_ENOTSPD : (Mode::id == GADI_PREC_FP16_IR ? GADI_EOVERFLOW16 : GADI_EDIVERGED);
            break;
          }
          const AT ak = (AT)(rr / pq);
          double s0 = 0.0, m3 = 0.0;
          for (int t = t0; t < t1; ++t) {
            const int row = t * BLOCK + tid;
            const AT pi = ld<AT>(vp[row]);
            const ST zi = (it == 0 ? ST(0) : z[row]) + (ST)(ak * pi);
            z[row] = zi;
            const VT ri = st<VT>(ld<AT>(vr[row]) - ak * ld<AT>(vq[row]));
            vr[row] = ri;
            const double dr = (double)ld<AT>(ri);
            s0 += dr * dr;
            m3 = fmax(m3, fabs((double)zi));
          }
          ALLREDUCE_P(3, s0, 0.0, 0.0, m3);
          const double rr_new = out[0];
          zmax = out[3];
          ++it;
          if (rr_new <= eps_h2 * rr0 || it >= a.maxit_in || !isfinite(rr_new)) break;
          const AT beta = (AT)(rr_new / rr);
          rr = rr_new;
          s0 = 0.0;
          for (int t = t0; t < t1; ++t) {
            const int row = t * BLOCK + tid;
            const AT ri = ld<AT>(vr[row]);
            const AT kr = (alpha + ld<AT>(hdiag[row])) * ri +
                          row_sum<AT>(row, pat, hoff, [&](int c) { return ld<AT>(vr[c]); });
            const VT pn = st<VT>(ri + beta * ld<AT>(vp[row]));
            const VT qn = st<VT>(kr + beta * ld<AT>(vq[row]));
            vp[row] = pn;
            vq[row] = qn;
            s0 += (double)ld<AT>(pn) * (double)ld<AT>(qn);
          }
          ALLREDUCE_P(2, s0, 0.0, 0.0, 0.0);
          pq = out[0];
        }
      }
    }
    ih += it;
    if (status != GADI_EMAXIT) break;  // inner breakdown on the first step
    if (!isfinite(zmax)) {
      status = overflow_status;
      break;
    }

    // ---------------------------------------------------------- a4/a5: CGNE on I + S/alpha
    int its = 0;
    if (it > 0 && zmax > 0.0) {
      int e2;
      (void)frexp((double)two_m_omega * zmax, &e2);
      e2 = clamp_exp(e2);
      const AT sc2 = (AT)ldexp(1.0, -e2);
      auto g_at = [&](int c) { return rnd(two_m_omega * (AT)z[c] * sc2); };
      if constexpr (FUSED) {
        // r_0 = g, t = (S/alpha) g
        {
          double g0 = 0.0;
          for (int t = t0; t < t1; ++t) {
            const int row = t * BLOCK + tid;
            const AT gi = g_at(row);
            const AT tv = inv_alpha * row_sum<AT>(row, pat, soff, g_at);
            R[0][row] = st<VT>(gi);
            T[row] = st<VT>(tv);
            g0 += (double)gi * (double)gi;
          }
          ALLREDUCE_P(4, g0, 0.0, 0.0, 0.0);
        }
        const double gs0 = out[0];
        // w_0 = r_0 - (S/alpha) t
        {
          double d0 = 0.0;
          for (int t = t0; t < t1; ++t) {
            const int row = t * BLOCK + tid;
            const AT ri = ld<AT>(R[0][row]);
            const AT wi = rnd(ri - inv_alpha * row_sum<AT>(row, pat, soff, [&](int c) { return ld<AT>(T[c]); }));
            W[0][row] = st<VT>(wi);
            d0 += (double)wi * (double)ri;
          }
          ALLREDUCE_P(4, 0.0, d0, 0.0, 0.0);
        }
        double gam = gs0, del = out[1];
        if (gs0 > 0.0) {
          double gam_prev = 1.0, a_prev = 1.0;
          for (int k = 0;; ++k) {
            const double beta = k == 0 ? 0.0 : gam / gam_prev;
            const double den = k == 0 ? del : del - beta * gam / a_prev;
            if (!(den > 0.0) || !isfinite(den)) {
              if (k == 0) status = isfinite(den) ? GADI_ENOTSPD : overflow_status;
              break;
            }
            const double ak = gam / den;
            const AT akt = (AT)ak, bkt = (AT)beta;
            const VT* __restrict__ rk = R[k & 1];
            const VT* __restrict__ wk = W[k & 1];
            const VT* __restrict__ sprev = Sv[(k + 1) & 1];
            VT* __restrict__ snew = Sv[k & 1];
            VT* __restrict__ rnew = R[(k + 1) & 1];
            VT* __restrict__ wnew = W[(k + 1) & 1];
            auto r_next = [&](int c) {
              const AT sc = k == 0 ? ld<AT>(wk[c]) : rnd(fma_at<AT>(bkt, ld<AT>(sprev[c]), ld<AT>(wk[c])));
              return rnd(fma_at<AT>(-akt, sc, ld<AT>(rk[c])));
            };
            // step + t = (S/alpha) r_{k+1}
            double g1 = 0.0;
            for (int t = t0; t < t1; ++t) {
              const int row = t * BLOCK + tid;
              const AT ri = ld<AT>(rk[row]);
              const AT si = k == 0 ? ld<AT>(wk[row]) : rnd(fma_at<AT>(bkt, ld<AT>(sprev[row]), ld<AT>(wk[row])));
              const AT pi = k == 0 ? ri : rnd(fma_at<AT>(bkt, ld<AT>(P[row]), ri));
              wsol[row] = (k == 0 ? ST(0) : wsol[row]) + (ST)(akt * pi);
              const AT rn = rnd(fma_at<AT>(-akt, si, ri));
              const AT tv = inv_alpha * row_sum<AT>(row, pat, soff, r_next);
              snew[row] = st<VT>(si);
              P[row] = st<VT>(pi);
              rnew[row] = st<VT>(rn);
              T[row] = st<VT>(tv);
              g1 += (double)rn * (double)rn;
            }
            ALLREDUCE_P(5, g1, 0.0, 0.0, 0.0);
            gam_prev = gam;
            a_prev = ak;
            gam = out[0];
            its = k + 1;
            if (gam <= eps_s2 * gs0 || its >= a.maxit_in || !isfinite(gam)) break;
            // w_{k+1} = r_{k+1} - (S/alpha) t
            double d1 = 0.0;
            for (int t = t0; t < t1; ++t) {
              const int row = t * BLOCK + tid;
              const AT rn = ld<AT>(rnew[row]);
              const AT wn = rnd(rn - inv_alpha * row_sum<AT>(row, pat, soff, [&](int c) { return ld<AT>(T[c]); }));
              wnew[row] = st<VT>(wn);
              d1 += (double)wn * (double)rn;
            }
            ALLREDUCE_P(6, 0.0, d1, 0.0, 0.0);
            del = out[1];
          }
        }
      } else {
        VT* __restrict__ vr = R[0];
        VT* __restrict__ vp = P;
        VT* __restrict__ vq = W[0];
        VT* __restrict__ vt = T;
        ST* __restrict__ w = wsol;
        double rrs0;
        {
          double s1 = 0.0;
          for (int t = t0; t < t1; ++t) {
            const int row = t * BLOCK + tid;
            const VT gi = st<VT>(two_m_omega * (AT)z[row] * sc2);
            const AT tv = inv_alpha * row_sum<AT>(row, pat, soff, [&](int c) {
                            return ld<AT>(st<VT>(two_m_omega * (AT)z[c] * sc2));
                          });
            vr[row] = gi;
            vp[row] = gi;
            vt[row] = st<VT>(tv);
            const double dg = (double)ld<AT>(gi);
            s1 += dg * dg;
          }
          ALLREDUCE_P(4, 0.0, s1, 0.0, 0.0);
          rrs0 = out[1];
        }
        double rrs = rrs0;
        if (rrs0 > 0.0) {
          for (;;) {
            // q = p - (S/alpha) t, with t = (S/alpha) p
            double s0 = 0.0;
            for (int t = t0; t < t1; ++t) {
              const int row = t * BLOCK + tid;
              const AT pi = ld<AT>(vp[row]);
              const AT qv = pi - inv_alpha * row_sum<AT>(row, pat, soff, [&](int c) { return ld<AT>(vt[c]); });
              const VT qi = st<VT>(qv);
              vq[row] = qi;
              s0 += (double)pi * (double)ld<AT>(qi);
            }
            ALLREDUCE_P(6, s0, 0.0, 0.0, 0.0);
            const double pqs = out[0];
            if (!(pqs > 0.0) || !isfinite(pqs)) {
              if (its == 0) status = isfinite(pqs) ? GADI_ENOTSPD : (Mode::id == GADI_PREC_FP16_IR ? GADI_EOVERFLOW16 : GADI_EDIVERGED);
              break;
            }
            const AT ak = (AT)(rrs / pqs);
            s0 = 0.0;
            for (int t = t0; t < t1; ++t) {
              const int row = t * BLOCK + tid;
              const AT pi = ld<AT>(vp[row]);
              w[row] = (its == 0 ? ST(0) : w[row]) + (ST)(ak * pi);
              const VT ri = st<VT>(ld<AT>(vr[row]) - ak * ld<AT>(vq[row]));
              vr[row] = ri;
              const double dr = (double)ld<AT>(ri);
              s0 += dr * dr;
            }
            ALLREDUCE_P(7, s0, 0.0, 0.0, 0.0);
            const double rr_new = out[0];
            ++its;
            if (rr_new <= eps_s2 * rrs0 || its >= a.maxit_in || !isfinite(rr_new)) break;
            const AT beta = (AT)(rr_new / rrs);
            rrs = rr_new;
            for (int t = t0; t < t1; ++t) {
              const int row = t * BLOCK + tid;
              const AT ri = ld<AT>(vr[row]);
              const AT sr = inv_alpha * row_sum<AT>(row, pat, soff, [&](int c) { return ld<AT>(vr[c]); });
              vt[row] = st<VT>(sr + beta * ld<AT>(vt[row]));
              vp[row] = st<VT>(ri + beta * ld<AT>(vp[row]));
            }
            ALLREDUCE_P(5, 0.0, 0.0, 0.0, 0.0);
          }
        }
      }
      is += its;
      if (status != GADI_EMAXIT) break;

      // ---------------------------------------------------------- a6: x += (I - S/alpha) w * 2^(e1+e2)
      if (its > 0) {
        const double unscale = ldexp(1.0, e1 + e2);
        for (int t = t0; t < t1; ++t) {
          const int row = t * BLOCK + tid;
          const AT ui = (AT)wsol[row] - inv_alpha * row_sum<AT>(row, pat, soff, [&](int c) { return (AT)wsol[c]; });
          x[row] += (double)ui * unscale;
        }
        ALLREDUCE_P(8, 0.0, 0.0, 0.0, 0.0);
      }
    }
    ++sweep;
  }

  if (a.prune && status == GADI_OK)
    red.publish_min(a.prune, (unsigned long long)(ih + 2 * is + 3 * (long long)sweep));
  res_out.status = status;
  res_out.sweeps = sweep;
  res_out.inner_h = ih;
  res_out.inner_s = is;
  res_out.relres = res;
  res_out.rho0 = rho0;
  return true;
}

}  // namespace gadi
