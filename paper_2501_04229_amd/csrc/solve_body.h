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
// Each phase runs over the rows a block owns and ends in one reduction (a
// device-wide barrier under the cooperative launch, a block barrier in the
// batched launch).
#pragma once

#include <cmath>
#include <type_traits>

#include "device_common.h"

namespace gadi {

struct SolveArgs {
  int n, npad, ntiles, maxit_out, maxit_in, hist_cap;
  const int32_t* slice_ptr;
  const int32_t* col;
  const int32_t* slice_dia;
  const int32_t* dia_off;
  // column offsets shared by every slice when the layout is uniformly
  // diagonal-style (System::dia_uniform slots per slice), else unused
  int32_t dia_u[kDiaMax];
  const void* a_off;   // Mode::AV values of A on the pattern
  const void* a_diag;  // Mode::AV diagonal of A
  const void* h_off;
  const void* s_off;
  const void* h_diag;
  // H and S in the half layout of the uniform pattern (the positive offsets
  // only, half_pad zero rows in front; System::h_half), or null
  const void* h_half;
  const void* s_half;
  int half_pad;
  const double* b;
  void* x;  // Mode::XT solution
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
  // Batched sweeps only: least work of a converged trial of this system so
  // far, in phases of the fused inner solvers (a CG step 1, a CGNE step 2,
  // the rest of a sweep 5); a trial stops (EMAXIT) once its own work exceeds it.
  unsigned long long* prune;
  // optional per-phase profile of block 0: wall-clock ticks [10], phase counts [10]
  long long* prof;
  int barrier;  // device-wide barrier: 0 relay, 1 XCC-hierarchical, 2 XCC-hierarchical without a master
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
// Every block also records its time of each of the first kPhaseRec phases
// (load-balance diagnostics), and block 0 the phase ids.
#define ALLREDUCE_P(id, a0, a1, a2, a3)                                        \
  do {                                                                         \
    if (a.prof && threadIdx.x == 0) {                                          \
      const long long now_ = wall_clock64();                                   \
      if (blockIdx.x == 0) {                                                   \
        a.prof[(id)] += now_ - t_mark;                                         \
        a.prof[10 + (id)] += 1;                                                \
      }                                                                        \
      if (nphase < kPhaseRec) {                                                \
        a.prof[kProfPhase + (size_t)nphase * kMaxBlocks + blockIdx.x] = now_ - t_mark; \
        if (blockIdx.x == 0) a.prof[kProfPhaseId + nphase] = (id);             \
      }                                                                        \
      ++nphase;                                                                \
    }                                                                          \
    ALLREDUCE(a0, a1, a2, a3);                                                 \
    if (a.prof && threadIdx.x == 0) t_mark = wall_clock64();                   \
  } while (0)

static __device__ __forceinline__ int clamp_exp(int e) { return e < -120 ? -120 : (e > 120 ? 120 : e); }

// fused multiply-add in the arithmetic type (fixes the rounding of the
// recomputed r_{k+1})
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

// Sparsity-pattern policies of the row products, in two steps so that a
// phase can issue every load of a row before any arithmetic: gather(row, val,
// load) returns the row's stored values and load(c) for each of its columns;
// dot<AT>(g, eval) returns sum_j val_j * eval(load(c_j)) in slot order.
// PatDia<W> serves a uniformly diagonal-style layout: W slots per slice with
// the same column offsets in every slice, held in scalar registers, so no
// address depends on loaded metadata.  PatGeneric reads the per-slice layout
// metadata (explicit or diagonal-style slices); its gather only records the
// row and the loads happen inside dot.
// Element i of p addressed as p plus a 32-bit byte offset, so that a load or
// store takes a scalar base and one 32-bit offset register (every array the
// solver indexes this way is below 4 GiB).
template <class T>
__device__ __forceinline__ const T& at(const T* p, unsigned i) {
  return *(const T*)((const char*)p + i * (unsigned)sizeof(T));
}
template <class T>
__device__ __forceinline__ T& at(T* p, unsigned i) {
  return *(T*)((char*)p + i * (unsigned)sizeof(T));
}

template <int W>
struct PatDia {
  int off[W];
  int nmax;
  template <bool SKEW, class MT>
  __host__ __device__ __forceinline__ const MT* mirror(const MT* p, const MT*) const {
    return p;
  }
  template <class MT, class R>
  struct G {
    MT v[W];
    R x[W];
  };
  // Indices are unsigned 32-bit so that loads address from a scalar base
  // plus a 32-bit offset (every array here is below 4 GiB).
  template <class MT, class LD>
  __device__ __forceinline__ auto gather(unsigned row, const MT* __restrict__ val, LD&& load) const {
    G<MT, decltype(load(0u))> g;
    // slice s starts at s * W * kSlice; slot j of lane l at + j * kSlice + l
    const unsigned k0 = (row & ~(unsigned)(kSlice - 1)) * W + (row & (kSlice - 1));
#pragma unroll
    for (int j = 0; j < W; ++j) {
      g.v[j] = at(val, k0 + j * kSlice);
      const int cc = (int)row + off[j];
      g.x[j] = load((unsigned)(cc < 0 ? 0 : (cc > nmax ? nmax : cc)));
    }
    return g;
  }
  template <class AT, class Gt, class EV>
  __device__ __forceinline__ AT dot(const Gt& g, EV&& eval) const {
    AT acc = 0;
#pragma unroll
    for (int j = 0; j < W; ++j) acc += ld<AT>(g.v[j]) * eval(g.x[j]);
    return acc;
  }
};

// Values of a matrix that is symmetric (SKEW = false: H) or skew-symmetric
// (SKEW = true: S) in value, as PatDiaSym reads them.
template <class MT, bool SKEW>
struct MirrorVals {
  const MT* p;
};

template <class MT>
__device__ __forceinline__ MT neg_of(MT v) {
  return -v;
}
template <>
__device__ __forceinline__ __half neg_of(__half v) {
  return __hneg(v);
}
template <>
__device__ __forceinline__ e4m3 neg_of(e4m3 v) {
  return e4m3{(uint8_t)(v.bits ^ 0x80u)};
}

// PatDia<W> for the symmetric offset sets of H and S (off[j] = -off[W-1-j],
// ascending: the pattern is that of A + A^T).  H_ij = H_ji and S_ij = -S_ji
// hold exactly for the stored values (both entries are computed from the same
// A_ij, A_ji and rounded to nearest, which commutes with negation), so H and S
// are read from a half layout that keeps the W/2 positive offsets of each row
// (W/2 slots per slice, `pad` zero rows in front): the entry at offset -d of
// row i is the entry at +d of row i - d (negated for S).  Both reads are
// contiguous streams; the value bytes of the H and S products halve, and every
// value is the one the full layout stores (a zero may change sign), so the
// products are those of PatDia.  Plain pointers (A) take the full layout.
template <int W>
struct PatDiaSym : PatDia<W> {
  int pad;  // zero rows in front of row 0 of the half layout (a multiple of kSlice, >= off[W-1])
  using PatDia<W>::gather;
  template <bool SKEW, class MT>
  __host__ __device__ __forceinline__ MirrorVals<MT, SKEW> mirror(const MT*, const MT* half) const {
    return {half};
  }
  template <class MT, bool SKEW, class LD>
  __device__ __forceinline__ auto gather(unsigned row, MirrorVals<MT, SKEW> mv, LD&& load) const {
    constexpr int H = W / 2;
    typename PatDia<W>::template G<MT, decltype(load(0u))> g;
#pragma unroll
    for (int j = 0; j < W; ++j) {
      const int cc = (int)row + this->off[j];
      g.x[j] = load((unsigned)(cc < 0 ? 0 : (cc > this->nmax ? this->nmax : cc)));
      // row rr of the half layout holds the entries at +d; a negative offset
      // reads the mirrored slot of row cc
      const unsigned rr = (unsigned)((j >= H ? (int)row : cc) + pad);
      const int slot = j >= H ? j - H : W - 1 - j - H;
      MT v = at(mv.p, (rr & ~(unsigned)(kSlice - 1)) * H + (unsigned)(slot * kSlice) + (rr & (kSlice - 1)));
      if constexpr (SKEW) {
        if (j < H) v = neg_of(v);
      }
      g.v[j] = v;
    }
    return g;
  }
};

struct PatGeneric {
  Pattern p;
  template <bool SKEW, class MT>
  __host__ __device__ __forceinline__ const MT* mirror(const MT* p, const MT*) const {
    return p;
  }
  template <class MT, class LD>
  struct G {
    int row;
    const MT* val;
    LD load;
  };
  template <class MT, class LD>
  __device__ __forceinline__ G<MT, std::decay_t<LD>> gather(unsigned row, const MT* __restrict__ val, LD&& load) const {
    return {(int)row, val, load};
  }
  template <class AT, class Gt, class EV>
  __device__ __forceinline__ AT dot(const Gt& g, EV&& eval) const {
    return row_sum<AT>(g.row, p, g.val, [&](unsigned c) { return eval(g.load(c)); });
  }
};

// Runs one phase over this thread's rows in three steps per row: load(row)
// performs every load of the row, math(l) the arithmetic, store(row, out)
// the writes and the row's terms of the thread's partial sums.  The loads of
// U tiles are issued before any of their arithmetic (a scheduling barrier
// keeps the compiler from interleaving them), so a wavefront has all of them
// in flight at once; partial sums still run over the rows in ascending order.
template <int BLOCK, int U, class L, class M, class S>
__device__ __forceinline__ void for_rows(int t0, int t1, L&& load, M&& math, S&& store) {
  const unsigned tid = threadIdx.x;
  int t = t0;
  if constexpr (U > 1) {
    using LT = decltype(load(0u));
    for (; t + U <= t1; t += U) {
      LT l[U];
#pragma unroll
      for (int u = 0; u < U; ++u) l[u] = load((unsigned)(t + u) * BLOCK + tid);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < U; ++u) store((unsigned)(t + u) * BLOCK + tid, math(l[u]));
    }
  }
  for (; t < t1; ++t) {
    const unsigned row = (unsigned)t * BLOCK + tid;
    const auto l = load(row);
    __builtin_amdgcn_sched_barrier(0);
    store(row, math(l));
  }
}

template <bool B>
using bool_c = std::integral_constant<bool, B>;

// Calls f(bool_c<true>) when first, else f(bool_c<false>): the first step of
// a recurrence becomes its own straight-line code instead of a branch per load.
template <class F>
__device__ __forceinline__ void first_or_rest(bool first, F&& f) {
  if (first) f(bool_c<true>{});
  else f(bool_c<false>{});
}

template <class T>
__device__ __forceinline__ T* pick(int k, T* p0, T* p1) {
  return (k & 1) ? p1 : p0;
}

// The refinement loop of Algorithm 1 for rows [t0 * BLOCK, t1 * BLOCK) of one
// system.  Returns false if a barrier timed out; otherwise fills `res`.
//
// The inner solves exist in three forms (FORM).
// FORM 1: the Chronopoulos-Gear form of CG: with w = K r and s = K p carried
// by recurrence, the two inner products of a step, gamma = r.r and delta =
// r.K r, come from one reduction.  Step k updates
//   s_k = w_k + beta_k s_{k-1},  p_k = r_k + beta_k p_{k-1},
//   z += a_k p_k,  r_{k+1} = r_k - a_k s_k,  w_{k+1} = K r_{k+1},
// with beta_k = gamma_k / gamma_{k-1} and a_k = gamma_k / (delta_k - beta_k gamma_k / a_{k-1}).
// The product K r_{k+1} needs r_{k+1} at neighbouring rows, which other
// blocks are writing in the same phase; each block recomputes those values
// from r_k, w_k, s_{k-1} (read from the previous phase's buffers, hence
// ping-pong buffers for r, w, s) with the same fused operations and the same
// roundings as their owner, so every copy is bit-identical.  A CG step on
// alpha I + H is one phase; a CGNE step on I - (S/alpha)^2 is two (the
// second product needs the first one's result at neighbouring rows).
// FORM 0: Hestenes-Stiefel CG with q_{k+1} = K p_{k+1} = K r_{k+1} +
// beta q_k folded into the product phase: two phases per CG step, three per
// CGNE step, and no recomputation.
// FORM 2: the same Chronopoulos-Gear scalars with one more recurrence,
// u_k = K s_k = K w_k + beta_k u_{k-1}, so that the step's product is K w_k
// on a vector the previous phase completed (the pipelined arrangement of
// Ghysels and Vanroose): one phase per CG step and no recomputation, w in
// ping-pong buffers.  Its CGNE is Craig's method on (I + S/alpha) y = g:
//   v = (I + S/alpha) p_k,  y += a_k p_k,  r_{k+1} = r_k - a_k v,
//   p_{k+1} = (I - S/alpha) r_{k+1} + beta_k p_k,
// a_k = |r_k|^2 / |p_k|^2, beta_k = |r_{k+1}|^2 / |r_k|^2: two phases per
// step, one product each, and y = (I - S/alpha) w comes out directly, so the
// update a6 needs no product.  In exact arithmetic its iterates are those of
// CG on (I - (S/alpha)^2) w = g mapped by I - S/alpha, with the same residuals.
// FORM 3: the Hestenes-Stiefel CG of form 0 with Craig's CGNE of form 2.
template <class Mode, int BLOCK, int FORM, int U, class Red, class Pat>
__device__ __forceinline__ bool solve_body(const SolveArgs& a, Red& red, const Pat& pat, int t0, int t1,
                                           DevInfo& res_out) {
  using MT = typename Mode::MT;
  using VT = typename Mode::VT;
  using ST = typename Mode::ST;
  using RT = typename Mode::RT;
  using AT = typename Mode::AT;

  const MT* __restrict__ hoff = (const MT*)a.h_off;
  const MT* __restrict__ soff = (const MT*)a.s_off;
  // H and S as the pattern reads them (the symmetric pattern reads half of each)
  const auto hv = pat.template mirror<false>(hoff, (const MT*)a.h_half);
  const auto sv = pat.template mirror<true>(soff, (const MT*)a.s_half);
  using DT = typename Mode::DT;
  const DT* __restrict__ hdiag = (const DT*)a.h_diag;
  RT* __restrict__ r = (RT*)a.r;
  ST* __restrict__ z = (ST*)a.z;
  ST* __restrict__ wsol = (ST*)a.w;
  VT* const R0 = (VT*)a.v[0];
  VT* const R1 = (VT*)a.v[1];
  VT* const W0 = (VT*)a.v[2];
  VT* const W1 = (VT*)a.v[3];
  VT* const S0 = (VT*)a.v[4];
  VT* const S1 = (VT*)a.v[5];
  VT* __restrict__ P = (VT*)a.v[6];
  VT* __restrict__ T = (VT*)a.v[7];
  using XT = typename Mode::XT;
  using FT = typename Mode::FT;
  using AV = typename Mode::AV;
  XT* __restrict__ x = (XT*)a.x;
  const AV* __restrict__ aoff = (const AV*)a.a_off;
  const AV* __restrict__ adiag = (const AV*)a.a_diag;
  const double* __restrict__ b = a.b;

  // the lean loops of the Hestenes-Stiefel CG and of Craig's CGNE (and their
  // start phases) hold few loads per row: 512-thread blocks keep twice the
  // tiles in flight there
  constexpr int UL = (BLOCK == 512 && U > 1) ? 2 * U : U;
  const AT alpha = (AT)a.alpha;
  const AT inv_alpha = (AT)(1.0 / a.alpha);
  const AT two_m_omega = (AT)(2.0 - a.omega);
  const double eps_h2 = a.eps_h * a.eps_h;
  const double eps_s2 = a.eps_s * a.eps_s;
  // a non-finite inner quantity is a half-precision overflow in every mode that
  // stores its Krylov vectors in half (fp16, h-d-s, h-s-s, fp8)
  const int overflow_status = std::is_same<VT, __half>::value ? GADI_EOVERFLOW16 : GADI_EDIVERGED;

  // value rounded to the storage type and read back
  auto rnd = [](AT v) { return ld<AT>(st<VT>(v)); };
  auto ldv = [](VT v) { return ld<AT>(v); };

  double out[4];
  long long t_mark = (a.prof && threadIdx.x == 0) ? wall_clock64() : 0;
  int nphase = 0;
  double rho0 = 0.0, res = 0.0;
  int status = GADI_EMAXIT;
  int sweep = 0;
  long long ih = 0, is = 0;

  // Operands of the recomputed r_{k+1} at a neighbouring row (form 1).
  struct Rk3 {
    VT sp, w, r;
  };
  struct Rk2 {
    VT w, r;
  };

  // forms 2, 3: x alternates between a.x and R1; a pending correction a6
  [[maybe_unused]] XT* xcur = x;
  [[maybe_unused]] XT* const xalt = (XT*)a.v[1];
  [[maybe_unused]] bool pend = false;
  [[maybe_unused]] double unscale_p = 0.0;
  for (;;) {
    // ---------------------------------------------------------- a1: residual
    // Forms 2 and 3 apply the previous sweep's correction a6 here: each row's
    // corrected x, and its neighbours' (recomputed with the same operations, so
    // every copy is bit-identical), enter the residual, and the corrected x is
    // written to the other x buffer (R1 of the Krylov vectors, unused by these
    // forms): one phase fewer per sweep.
    {
      // the residual's double-precision rows hold the most loads: at most two tiles in flight
      constexpr int UR = U > 2 ? 2 : U;
      double s0 = 0.0, m3 = 0.0;
      bool applied = false;
      if constexpr (FORM >= 2) {
        if (pend) {
          struct XY {
            XT x;
            ST y;
          };
          struct RX {
            double r;
            XT x;
          };
          XT* __restrict__ xo = xcur;
          XT* __restrict__ xn = xcur == x ? xalt : x;
          const double us = unscale_p;
          auto corr = [us](XT xv, ST yv) { return (XT)(xv + (XT)((double)ld<AT>(yv) * us)); };
          auto gxy = [&](unsigned c) { return XY{at(xo, c), at(wsol, c)}; };
          for_rows<BLOCK, UR>(
              t0, t1,
              [&](unsigned row) {
                struct {
                  AV d;
                  XY xy;
                  double br;
                  decltype(pat.gather(0u, aoff, gxy)) g;
                } l{at(adiag, row), XY{at(xo, row), at(wsol, row)}, at(b, row), pat.gather(row, aoff, gxy)};
                return l;
              },
              [&](const auto& l) {
                const XT xr = corr(l.xy.x, l.xy.y);
                const FT ax = (FT)l.d * (FT)xr +
                              pat.template dot<FT>(l.g, [&](const XY& v) { return (FT)corr(v.x, v.y); });
                return RX{(double)((FT)l.br - ax), xr};
              },
              [&](unsigned row, const RX& o) {
                at(r, row) = (RT)o.r;
                at(xn, row) = o.x;
                s0 += o.r * o.r;
                m3 = fmax(m3, fabs(o.r));
              });
          xcur = xn;
          pend = false;
          applied = true;
        }
      }
      if (!applied) {
        XT* __restrict__ xr_ = xcur;
        auto gx = [&](unsigned c) { return at(xr_, c); };
        for_rows<BLOCK, UR>(
            t0, t1,
            [&](unsigned row) {
              struct {
                AV d;
                XT xr;
                double br;
                decltype(pat.gather(0u, aoff, gx)) g;
              } l{at(adiag, row), at(xr_, row), at(b, row), pat.gather(row, aoff, gx)};
              return l;
            },
            [&](const auto& l) {
              // in the residual precision u_f (double unless a single-precision mode)
              const FT ax = (FT)l.d * (FT)l.xr + pat.template dot<FT>(l.g, [](XT v) { return (FT)v; });
              return (double)((FT)l.br - ax);
            },
            [&](unsigned row, double ri) {
              at(r, row) = (RT)ri;
              s0 += ri * ri;
              m3 = fmax(m3, fabs(ri));
            });
      }
      ALLREDUCE_P(0, s0, 0.0, 0.0, m3);
    }
    const double rho = sqrt(out[0]);
    const double rmax = out[3];
    if (sweep == 0) rho0 = rho;
    res = rho0 > 0.0 ? rho / rho0 : 0.0;
    if (a.hist && sweep < a.hist_cap && blockIdx.x == 0 && threadIdx.x == 0) a.hist[sweep] = res;
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
      const unsigned long long wk = (unsigned long long)(ih + 2 * is + 5 * (long long)sweep);
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
    auto gr = [&](unsigned c) { return at(r, c); };
    if constexpr (FORM == 1 || FORM == 2) {
      struct RW {
        AT r, w;
      };
      {
        // r_0 = r * 2^-e1 in storage precision, w_0 = K r_0
        double g0 = 0.0, d0 = 0.0;
        for_rows<BLOCK, U>(
            t0, t1,
            [&](unsigned row) {
              struct {
                RT rr;
                DT hd;
                decltype(pat.gather(0u, hv, gr)) g;
              } l{at(r, row), at(hdiag, row), pat.gather(row, hv, gr)};
              return l;
            },
            [&](const auto& l) {
              const AT ri = rnd((AT)l.rr * sc1);
              const AT kr = (alpha + ld<AT>(l.hd)) * ri + pat.template dot<AT>(l.g, [&](RT v) { return rnd((AT)v * sc1); });
              return RW{ri, rnd(kr)};
            },
            [&](unsigned row, const RW& o) {
              at(R0, row) = st<VT>(o.r);
              at(W0, row) = st<VT>(o.w);
              g0 += (double)o.r * (double)o.r;
              d0 += (double)o.w * (double)o.r;
            });
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
          double g1 = 0.0, d1 = 0.0, m3 = 0.0;
          if constexpr (FORM == 1) {
            const VT* __restrict__ rk = pick(k, R0, R1);
            const VT* __restrict__ wk = pick(k, W0, W1);
            const VT* __restrict__ sprev = pick(k + 1, S0, S1);
            VT* __restrict__ snew = pick(k, S0, S1);
            VT* __restrict__ rnew = pick(k + 1, R0, R1);
            VT* __restrict__ wnew = pick(k + 1, W0, W1);
            struct O {
              AT s, p, rn, wn;
              ST z;
            };
            auto store = [&](unsigned row, const O& o) {
              at(snew, row) = st<VT>(o.s);
              at(P, row) = st<VT>(o.p);
              at(z, row) = o.z;
              at(rnew, row) = st<VT>(o.rn);
              at(wnew, row) = st<VT>(o.wn);
              g1 += (double)o.rn * (double)o.rn;
              d1 += (double)o.wn * (double)o.rn;
              m3 = fmax(m3, fabs((double)ld<AT>(o.z)));
            };
            if (k == 0) {
              // s_0 = w_0, p_0 = r_0; r_1 at row c = r_0 - a_0 w_0
              auto gl = [&](unsigned c) { return Rk2{at(wk, c), at(rk, c)}; };
              auto r_next = [&](const Rk2& v) { return rnd(fma_at<AT>(-akt, ldv(v.w), ldv(v.r))); };
              for_rows<BLOCK, U>(
                  t0, t1,
                  [&](unsigned row) {
                    struct {
                      VT r, w;
                      DT hd;
                      decltype(pat.gather(0u, hv, gl)) g;
                    } l{at(rk, row), at(wk, row), at(hdiag, row), pat.gather(row, hv, gl)};
                    return l;
                  },
                  [&](const auto& l) {
                    O o;
                    const AT ri = ldv(l.r);
                    o.s = ldv(l.w);
                    o.p = ri;
                    o.z = st<ST>(akt * ri);
                    o.rn = rnd(fma_at<AT>(-akt, o.s, ri));
                    o.wn = rnd((alpha + ld<AT>(l.hd)) * o.rn + pat.template dot<AT>(l.g, r_next));
                    return o;
                  },
                  store);
            } else {
              // s_k = w_k + b_k s_{k-1} and r_{k+1} = r_k - a_k s_k at row c,
              // computed exactly as the row's owner computes them
              auto gl = [&](unsigned c) { return Rk3{at(sprev, c), at(wk, c), at(rk, c)}; };
              auto r_next = [&](const Rk3& v) {
                return rnd(fma_at<AT>(-akt, rnd(fma_at<AT>(bkt, ldv(v.sp), ldv(v.w))), ldv(v.r)));
              };
              for_rows<BLOCK, U>(
                  t0, t1,
                  [&](unsigned row) {
                    struct {
                      VT r, w, sp, p;
                      ST z;
                      DT hd;
                      decltype(pat.gather(0u, hv, gl)) g;
                    } l{at(rk, row), at(wk, row), at(sprev, row), at(P, row), at(z, row), at(hdiag, row), pat.gather(row, hv, gl)};
                    return l;
                  },
                  [&](const auto& l) {
                    O o;
                    const AT ri = ldv(l.r);
                    o.s = rnd(fma_at<AT>(bkt, ldv(l.sp), ldv(l.w)));
                    o.p = rnd(fma_at<AT>(bkt, ldv(l.p), ri));
                    o.z = st<ST>(ld<AT>(l.z) + akt * o.p);
                    o.rn = rnd(fma_at<AT>(-akt, o.s, ri));
                    o.wn = rnd((alpha + ld<AT>(l.hd)) * o.rn + pat.template dot<AT>(l.g, r_next));
                    return o;
                  },
                  store);
            }
          } else {
            // pipelined: the product is K w_k; r stays in R0, s in S0, u in S1
            const VT* __restrict__ wk = pick(k, W0, W1);
            VT* __restrict__ wnew = pick(k + 1, W0, W1);
            auto gw = [&](unsigned c) { return at(wk, c); };
            struct O {
              AT s, u, p, rn, wn;
              ST z;
            };
            auto store = [&](unsigned row, const O& o) {
              at(S0, row) = st<VT>(o.s);
              at(S1, row) = st<VT>(o.u);
              at(P, row) = st<VT>(o.p);
              at(z, row) = o.z;
              at(R0, row) = st<VT>(o.rn);
              at(wnew, row) = st<VT>(o.wn);
              g1 += (double)o.rn * (double)o.rn;
              d1 += (double)o.wn * (double)o.rn;
              m3 = fmax(m3, fabs((double)ld<AT>(o.z)));
            };
            if (k == 0) {
              // u_0 = K w_0, s_0 = w_0, p_0 = r_0
              for_rows<BLOCK, U>(
                  t0, t1,
                  [&](unsigned row) {
                    struct {
                      VT r, w;
                      DT hd;
                      decltype(pat.gather(0u, hv, gw)) g;
                    } l{at(R0, row), at(wk, row), at(hdiag, row), pat.gather(row, hv, gw)};
                    return l;
                  },
                  [&](const auto& l) {
                    O o;
                    const AT ri = ldv(l.r), wi = ldv(l.w);
                    o.u = rnd((alpha + ld<AT>(l.hd)) * wi + pat.template dot<AT>(l.g, ldv));
                    o.s = wi;
                    o.p = ri;
                    o.z = st<ST>(akt * ri);
                    o.rn = rnd(fma_at<AT>(-akt, o.s, ri));
                    o.wn = rnd(fma_at<AT>(-akt, o.u, wi));
                    return o;
                  },
                  store);
            } else {
              for_rows<BLOCK, U>(
                  t0, t1,
                  [&](unsigned row) {
                    struct {
                      VT r, w, s, u, p;
                      ST z;
                      DT hd;
                      decltype(pat.gather(0u, hv, gw)) g;
                    } l{at(R0, row), at(wk, row), at(S0, row), at(S1, row), at(P, row), at(z, row), at(hdiag, row),
                        pat.gather(row, hv, gw)};
                    return l;
                  },
                  [&](const auto& l) {
                    O o;
                    const AT ri = ldv(l.r), wi = ldv(l.w);
                    const AT kw = (alpha + ld<AT>(l.hd)) * wi + pat.template dot<AT>(l.g, ldv);
                    o.u = rnd(fma_at<AT>(bkt, ldv(l.u), kw));
                    o.s = rnd(fma_at<AT>(bkt, ldv(l.s), wi));
                    o.p = rnd(fma_at<AT>(bkt, ldv(l.p), ri));
                    o.z = st<ST>(ld<AT>(l.z) + akt * o.p);
                    o.rn = rnd(fma_at<AT>(-akt, o.s, ri));
                    o.wn = rnd(fma_at<AT>(-akt, o.u, wi));
                    return o;
                  },
                  store);
            }
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
      VT* __restrict__ vr = R0;
      VT* __restrict__ vp = P;
      VT* __restrict__ vq = W0;
      double pq, rr, rr0;
      {
        struct O {
          VT p, q;
        };
        double s0 = 0.0, s1 = 0.0;
        for_rows<BLOCK, UL>(
            t0, t1,
            [&](unsigned row) {
              struct {
                RT rr;
                DT hd;
                decltype(pat.gather(0u, hv, gr)) g;
              } l{at(r, row), at(hdiag, row), pat.gather(row, hv, gr)};
              return l;
            },
            [&](const auto& l) {
              const VT pi = st<VT>((AT)l.rr * sc1);
              const AT kp = (alpha + ld<AT>(l.hd)) * ld<AT>(pi) +
                            pat.template dot<AT>(l.g, [&](RT v) { return ld<AT>(st<VT>((AT)v * sc1)); });
              return O{pi, st<VT>(kp)};
            },
            [&](unsigned row, const O& o) {
              at(vr, row) = o.p;
              at(vp, row) = o.p;
              at(vq, row) = o.q;
              const double api = (double)ld<AT>(o.p);
              s0 += api * (double)ld<AT>(o.q);
              s1 += api * api;
            });
        ALLREDUCE_P(1, s0, s1, 0.0, 0.0);
        pq = out[0];
        rr0 = out[1];
        rr = rr0;
      }
      if (rr0 > 0.0) {
        for (;;) {
          if (!(pq > 0.0) || !isfinite(pq)) {
            if (it == 0) status = isfinite(pq) ? GADI_ENOTSPD : overflow_status;
            break;
          }
          const AT ak = (AT)(rr / pq);
          double s0 = 0.0, m3 = 0.0;
          first_or_rest(it == 0, [&](auto first_c) {
            constexpr bool FIRST = decltype(first_c)::value;
            struct O {
              ST z;
              VT r;
            };
            for_rows<BLOCK, UL>(
                t0, t1,
                [&](unsigned row) {
                  struct {
                    VT p, r, q;
                    ST z;
                  } l{at(vp, row), at(vr, row), at(vq, row), FIRST ? st<ST>(AT(0)) : at(z, row)};
                  return l;
                },
                [&](const auto& l) {
                  const AT pi = ldv(l.p);
                  O o;
                  if constexpr (FIRST) o.z = st<ST>(ak * pi);
                  else o.z = st<ST>(ld<AT>(l.z) + ak * pi);
                  o.r = st<VT>(ldv(l.r) - ak * ldv(l.q));
                  return o;
                },
                [&](unsigned row, const O& o) {
                  at(z, row) = o.z;
                  at(vr, row) = o.r;
                  const double dr = (double)ld<AT>(o.r);
                  s0 += dr * dr;
                  m3 = fmax(m3, fabs((double)ld<AT>(o.z)));
                });
          });
          ALLREDUCE_P(3, s0, 0.0, 0.0, m3);
          const double rr_new = out[0];
          zmax = out[3];
          ++it;
          if (rr_new <= eps_h2 * rr0 || it >= a.maxit_in || !isfinite(rr_new)) break;
          const AT beta = (AT)(rr_new / rr);
          rr = rr_new;
          s0 = 0.0;
          {
            struct O {
              VT p, q;
            };
            auto gv = [&](unsigned c) { return at(vr, c); };
            for_rows<BLOCK, UL>(
                t0, t1,
                [&](unsigned row) {
                  struct {
                    VT r, p, q;
                    DT hd;
                    decltype(pat.gather(0u, hv, gv)) g;
                  } l{at(vr, row), at(vp, row), at(vq, row), at(hdiag, row), pat.gather(row, hv, gv)};
                  return l;
                },
                [&](const auto& l) {
                  const AT ri = ldv(l.r);
                  const AT kr = (alpha + ld<AT>(l.hd)) * ri + pat.template dot<AT>(l.g, ldv);
                  return O{st<VT>(ri + beta * ldv(l.p)), st<VT>(kr + beta * ldv(l.q))};
                },
                [&](unsigned row, const O& o) {
                  at(vp, row) = o.p;
                  at(vq, row) = o.q;
                  s0 += (double)ld<AT>(o.p) * (double)ld<AT>(o.q);
                });
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
      // g = (2 - omega) z 2^-e2 rounded to the storage type, from a loaded z
      auto g_of = [&](ST zc) { return rnd(two_m_omega * ld<AT>(zc) * sc2); };
      auto gz = [&](unsigned c) { return at(z, c); };
      auto gT = [&](unsigned c) { return at(T, c); };
      if constexpr (FORM >= 2) {
        // Craig's method: r in R0, p in P, y in wsol
        double gs0, pp;
        {
          // r_0 = g, p_0 = (I - S/alpha) g
          struct O {
            AT g, p;
          };
          double s0 = 0.0, s1 = 0.0;
          for_rows<BLOCK, UL>(
              t0, t1,
              [&](unsigned row) {
                struct {
                  ST z;
                  decltype(pat.gather(0u, sv, gz)) g;
                } l{at(z, row), pat.gather(row, sv, gz)};
                return l;
              },
              [&](const auto& l) {
                const AT gi = g_of(l.z);
                return O{gi, rnd(gi - inv_alpha * pat.template dot<AT>(l.g, g_of))};
              },
              [&](unsigned row, const O& o) {
                at(R0, row) = st<VT>(o.g);
                at(P, row) = st<VT>(o.p);
                s0 += (double)o.g * (double)o.g;
                s1 += (double)o.p * (double)o.p;
              });
          ALLREDUCE_P(4, s0, s1, 0.0, 0.0);
          gs0 = out[0];
          pp = out[1];
        }
        double gam = gs0;
        if (gs0 > 0.0) {
          auto gp = [&](unsigned c) { return at(P, c); };
          auto gr0 = [&](unsigned c) { return at(R0, c); };
          for (;;) {
            if (!(pp > 0.0) || !isfinite(pp)) {
              if (its == 0) status = isfinite(pp) ? GADI_ENOTSPD : overflow_status;
              break;
            }
            const AT ak = (AT)(gam / pp);
            // y += a_k p_k, r_{k+1} = r_k - a_k (I + S/alpha) p_k
            double s0 = 0.0;
            struct O {
              ST y;
              VT r;
            };
            auto store = [&](unsigned row, const O& o) {
              at(wsol, row) = o.y;
              at(R0, row) = o.r;
              const double dr = (double)ld<AT>(o.r);
              s0 += dr * dr;
            };
            if (its == 0) {
              for_rows<BLOCK, UL>(
                  t0, t1,
                  [&](unsigned row) {
                    struct {
                      VT p, r;
                      decltype(pat.gather(0u, sv, gp)) g;
                    } l{at(P, row), at(R0, row), pat.gather(row, sv, gp)};
                    return l;
                  },
                  [&](const auto& l) {
                    const AT pi = ldv(l.p);
                    const AT v = pi + inv_alpha * pat.template dot<AT>(l.g, ldv);
                    return O{st<ST>(ak * pi), st<VT>(ldv(l.r) - ak * v)};
                  },
                  store);
            } else {
              for_rows<BLOCK, UL>(
                  t0, t1,
                  [&](unsigned row) {
                    struct {
                      VT p, r;
                      ST y;
                      decltype(pat.gather(0u, sv, gp)) g;
                    } l{at(P, row), at(R0, row), at(wsol, row), pat.gather(row, sv, gp)};
                    return l;
                  },
                  [&](const auto& l) {
                    const AT pi = ldv(l.p);
                    const AT v = pi + inv_alpha * pat.template dot<AT>(l.g, ldv);
                    return O{st<ST>(ld<AT>(l.y) + ak * pi), st<VT>(ldv(l.r) - ak * v)};
                  },
                  store);
            }
            ALLREDUCE_P(7, s0, 0.0, 0.0, 0.0);
            const double gnew = out[0];
            ++its;
            if (gnew <= eps_s2 * gs0 || its >= a.maxit_in || !isfinite(gnew)) break;
            const AT beta = (AT)(gnew / gam);
            gam = gnew;
            // p_{k+1} = (I - S/alpha) r_{k+1} + beta_k p_k
            double s1 = 0.0;
            for_rows<BLOCK, UL>(
                t0, t1,
                [&](unsigned row) {
                  struct {
                    VT r, p;
                    decltype(pat.gather(0u, sv, gr0)) g;
                  } l{at(R0, row), at(P, row), pat.gather(row, sv, gr0)};
                  return l;
                },
                [&](const auto& l) {
                  const AT ri = ldv(l.r);
                  return st<VT>(ri - inv_alpha * pat.template dot<AT>(l.g, ldv) + beta * ldv(l.p));
                },
                [&](unsigned row, VT pn) {
                  at(P, row) = pn;
                  const double dp = (double)ld<AT>(pn);
                  s1 += dp * dp;
                });
            ALLREDUCE_P(5, s1, 0.0, 0.0, 0.0);
            pp = out[0];
          }
        }
      } else if constexpr (FORM == 1) {
        // r_0 = g, t = (S/alpha) g
        {
          struct O {
            AT g, t;
          };
          double g0 = 0.0;
          for_rows<BLOCK, U>(
              t0, t1,
              [&](unsigned row) {
                struct {
                  ST z;
                  decltype(pat.gather(0u, sv, gz)) g;
                } l{at(z, row), pat.gather(row, sv, gz)};
                return l;
              },
              [&](const auto& l) { return O{g_of(l.z), inv_alpha * pat.template dot<AT>(l.g, g_of)}; },
              [&](unsigned row, const O& o) {
                at(R0, row) = st<VT>(o.g);
                at(T, row) = st<VT>(o.t);
                g0 += (double)o.g * (double)o.g;
              });
          ALLREDUCE_P(4, g0, 0.0, 0.0, 0.0);
        }
        const double gs0 = out[0];
        // w_0 = r_0 - (S/alpha) t
        {
          struct O {
            AT r, w;
          };
          double d0 = 0.0;
          for_rows<BLOCK, U>(
              t0, t1,
              [&](unsigned row) {
                struct {
                  VT r;
                  decltype(pat.gather(0u, sv, gT)) g;
                } l{at(R0, row), pat.gather(row, sv, gT)};
                return l;
              },
              [&](const auto& l) {
                const AT ri = ldv(l.r);
                return O{ri, rnd(ri - inv_alpha * pat.template dot<AT>(l.g, ldv))};
              },
              [&](unsigned row, const O& o) {
                at(W0, row) = st<VT>(o.w);
                d0 += (double)o.w * (double)o.r;
              });
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
            const VT* __restrict__ rk = pick(k, R0, R1);
            const VT* __restrict__ wk = pick(k, W0, W1);
            const VT* __restrict__ sprev = pick(k + 1, S0, S1);
            VT* __restrict__ snew = pick(k, S0, S1);
            VT* __restrict__ rnew = pick(k + 1, R0, R1);
            VT* __restrict__ wnew = pick(k + 1, W0, W1);
            // step + t = (S/alpha) r_{k+1}
            double g1 = 0.0;
            struct O {
              AT s, p, rn, t;
              ST w;
            };
            auto store = [&](unsigned row, const O& o) {
              at(snew, row) = st<VT>(o.s);
              at(P, row) = st<VT>(o.p);
              at(wsol, row) = o.w;
              at(rnew, row) = st<VT>(o.rn);
              at(T, row) = st<VT>(o.t);
              g1 += (double)o.rn * (double)o.rn;
            };
            if (k == 0) {
              auto gl = [&](unsigned c) { return Rk2{at(wk, c), at(rk, c)}; };
              auto r_next = [&](const Rk2& v) { return rnd(fma_at<AT>(-akt, ldv(v.w), ldv(v.r))); };
              for_rows<BLOCK, U>(
                  t0, t1,
                  [&](unsigned row) {
                    struct {
                      VT r, w;
                      decltype(pat.gather(0u, sv, gl)) g;
                    } l{at(rk, row), at(wk, row), pat.gather(row, sv, gl)};
                    return l;
                  },
                  [&](const auto& l) {
                    O o;
                    const AT ri = ldv(l.r);
                    o.s = ldv(l.w);
                    o.p = ri;
                    o.w = st<ST>(akt * ri);
                    o.rn = rnd(fma_at<AT>(-akt, o.s, ri));
                    o.t = inv_alpha * pat.template dot<AT>(l.g, r_next);
                    return o;
                  },
                  store);
            } else {
              auto gl = [&](unsigned c) { return Rk3{at(sprev, c), at(wk, c), at(rk, c)}; };
              auto r_next = [&](const Rk3& v) {
                return rnd(fma_at<AT>(-akt, rnd(fma_at<AT>(bkt, ldv(v.sp), ldv(v.w))), ldv(v.r)));
              };
              for_rows<BLOCK, U>(
                  t0, t1,
                  [&](unsigned row) {
                    struct {
                      VT r, w, sp, p;
                      ST ws;
                      decltype(pat.gather(0u, sv, gl)) g;
                    } l{at(rk, row), at(wk, row), at(sprev, row), at(P, row), at(wsol, row), pat.gather(row, sv, gl)};
                    return l;
                  },
                  [&](const auto& l) {
                    O o;
                    const AT ri = ldv(l.r);
                    o.s = rnd(fma_at<AT>(bkt, ldv(l.sp), ldv(l.w)));
                    o.p = rnd(fma_at<AT>(bkt, ldv(l.p), ri));
                    o.w = st<ST>(ld<AT>(l.ws) + akt * o.p);
                    o.rn = rnd(fma_at<AT>(-akt, o.s, ri));
                    o.t = inv_alpha * pat.template dot<AT>(l.g, r_next);
                    return o;
                  },
                  store);
            }
            ALLREDUCE_P(5, g1, 0.0, 0.0, 0.0);
            gam_prev = gam;
            a_prev = ak;
            gam = out[0];
            its = k + 1;
            if (gam <= eps_s2 * gs0 || its >= a.maxit_in || !isfinite(gam)) break;
            // w_{k+1} = r_{k+1} - (S/alpha) t
            double d1 = 0.0;
            {
              struct O2 {
                AT r, w;
              };
              for_rows<BLOCK, U>(
                  t0, t1,
                  [&](unsigned row) {
                    struct {
                      VT r;
                      decltype(pat.gather(0u, sv, gT)) g;
                    } l{at(rnew, row), pat.gather(row, sv, gT)};
                    return l;
                  },
                  [&](const auto& l) {
                    const AT rn = ldv(l.r);
                    return O2{rn, rnd(rn - inv_alpha * pat.template dot<AT>(l.g, ldv))};
                  },
                  [&](unsigned row, const O2& o) {
                    at(wnew, row) = st<VT>(o.w);
                    d1 += (double)o.w * (double)o.r;
                  });
            }
            ALLREDUCE_P(6, 0.0, d1, 0.0, 0.0);
            del = out[1];
          }
        }
      } else {
        VT* __restrict__ vr = R0;
        VT* __restrict__ vp = P;
        VT* __restrict__ vq = W0;
        VT* __restrict__ vt = T;
        ST* __restrict__ w = wsol;
        double rrs0;
        {
          struct O {
            VT g, t;
          };
          double s1 = 0.0;
          for_rows<BLOCK, U>(
              t0, t1,
              [&](unsigned row) {
                struct {
                  ST z;
                  decltype(pat.gather(0u, sv, gz)) g;
                } l{at(z, row), pat.gather(row, sv, gz)};
                return l;
              },
              [&](const auto& l) {
                const VT gi = st<VT>(two_m_omega * ld<AT>(l.z) * sc2);
                const AT tv = inv_alpha * pat.template dot<AT>(l.g, [&](ST zc) {
                                return ld<AT>(st<VT>(two_m_omega * ld<AT>(zc) * sc2));
                              });
                return O{gi, st<VT>(tv)};
              },
              [&](unsigned row, const O& o) {
                at(vr, row) = o.g;
                at(vp, row) = o.g;
                at(vt, row) = o.t;
                const double dg = (double)ld<AT>(o.g);
                s1 += dg * dg;
              });
          ALLREDUCE_P(4, 0.0, s1, 0.0, 0.0);
          rrs0 = out[1];
        }
        double rrs = rrs0;
        if (rrs0 > 0.0) {
          auto gvt = [&](unsigned c) { return at(vt, c); };
          auto gvr = [&](unsigned c) { return at(vr, c); };
          for (;;) {
            // q = p - (S/alpha) t, with t = (S/alpha) p
            double s0 = 0.0;
            {
              struct O {
                AT p;
                VT q;
              };
              for_rows<BLOCK, U>(
                  t0, t1,
                  [&](unsigned row) {
                    struct {
                      VT p;
                      decltype(pat.gather(0u, sv, gvt)) g;
                    } l{at(vp, row), pat.gather(row, sv, gvt)};
                    return l;
                  },
                  [&](const auto& l) {
                    const AT pi = ldv(l.p);
                    return O{pi, st<VT>(pi - inv_alpha * pat.template dot<AT>(l.g, ldv))};
                  },
                  [&](unsigned row, const O& o) {
                    at(vq, row) = o.q;
                    s0 += (double)o.p * (double)ld<AT>(o.q);
                  });
            }
            ALLREDUCE_P(6, s0, 0.0, 0.0, 0.0);
            const double pqs = out[0];
            if (!(pqs > 0.0) || !isfinite(pqs)) {
              if (its == 0) status = isfinite(pqs) ? GADI_ENOTSPD : overflow_status;
              break;
            }
            const AT ak = (AT)(rrs / pqs);
            s0 = 0.0;
            first_or_rest(its == 0, [&](auto first_c) {
              constexpr bool FIRST = decltype(first_c)::value;
              struct O {
                ST w;
                VT r;
              };
              for_rows<BLOCK, U>(
                  t0, t1,
                  [&](unsigned row) {
                    struct {
                      VT p, r, q;
                      ST w;
                    } l{at(vp, row), at(vr, row), at(vq, row), FIRST ? st<ST>(AT(0)) : at(w, row)};
                    return l;
                  },
                  [&](const auto& l) {
                    const AT pi = ldv(l.p);
                    O o;
                    if constexpr (FIRST) o.w = st<ST>(ak * pi);
                    else o.w = st<ST>(ld<AT>(l.w) + ak * pi);
                    o.r = st<VT>(ldv(l.r) - ak * ldv(l.q));
                    return o;
                  },
                  [&](unsigned row, const O& o) {
                    at(w, row) = o.w;
                    at(vr, row) = o.r;
                    const double dr = (double)ld<AT>(o.r);
                    s0 += dr * dr;
                  });
            });
            ALLREDUCE_P(7, s0, 0.0, 0.0, 0.0);
            const double rr_new = out[0];
            ++its;
            if (rr_new <= eps_s2 * rrs0 || its >= a.maxit_in || !isfinite(rr_new)) break;
            const AT beta = (AT)(rr_new / rrs);
            rrs = rr_new;
            {
              struct O {
                VT t, p;
              };
              for_rows<BLOCK, U>(
                  t0, t1,
                  [&](unsigned row) {
                    struct {
                      VT r, t, p;
                      decltype(pat.gather(0u, sv, gvr)) g;
                    } l{at(vr, row), at(vt, row), at(vp, row), pat.gather(row, sv, gvr)};
                    return l;
                  },
                  [&](const auto& l) {
                    const AT sr = inv_alpha * pat.template dot<AT>(l.g, ldv);
                    return O{st<VT>(sr + beta * ldv(l.t)), st<VT>(ldv(l.r) + beta * ldv(l.p))};
                  },
                  [&](unsigned row, const O& o) {
                    at(vt, row) = o.t;
                    at(vp, row) = o.p;
                  });
            }
            ALLREDUCE_P(5, 0.0, 0.0, 0.0, 0.0);
          }
        }
      }
      is += its;
      if (status != GADI_EMAXIT) break;

      // ---------------------------------------------------------- a6: x += (I - S/alpha) w * 2^(e1+e2)
      if constexpr (FORM >= 2) {
        // Craig's iterate is already (I - S/alpha) w: x += y 2^(e1+e2) is
        // applied by the next residual phase
        if (its > 0) {
          pend = true;
          unscale_p = ldexp(1.0, e1 + e2);
        }
      } else if (its > 0) {
        const double unscale = ldexp(1.0, e1 + e2);
        auto gw = [&](unsigned c) { return at(wsol, c); };
        for_rows<BLOCK, U>(
            t0, t1,
            [&](unsigned row) {
              struct {
                ST w;
                XT x;
                decltype(pat.gather(0u, sv, gw)) g;
              } l{at(wsol, row), at(x, row), pat.gather(row, sv, gw)};
              return l;
            },
            [&](const auto& l) {
              const AT ui = ld<AT>(l.w) - inv_alpha * pat.template dot<AT>(l.g, [](ST v) { return ld<AT>(v); });
              // the update in the solution precision u
              return (XT)(l.x + (XT)((double)ui * unscale));
            },
            [&](unsigned row, XT xn) { at(x, row) = xn; });
        ALLREDUCE_P(8, 0.0, 0.0, 0.0, 0.0);
      }
    }
    ++sweep;
  }

  if constexpr (FORM >= 2) {
    // the solution is wherever the last residual phase left it
    if (xcur != x)
      for_rows<BLOCK, U>(
          t0, t1, [&](unsigned row) { return at(xalt, row); }, [](XT v) { return v; },
          [&](unsigned row, XT v) { at(x, row) = v; });
  }
  if (a.prune && status == GADI_OK)
    red.publish_min(a.prune, (unsigned long long)(ih + 2 * is + 5 * (long long)sweep));
  res_out.status = status;
  res_out.sweeps = sweep;
  res_out.inner_h = ih;
  res_out.inner_s = is;
  res_out.relres = res;
  res_out.rho0 = rho0;
  return true;
}

}  // namespace gadi
