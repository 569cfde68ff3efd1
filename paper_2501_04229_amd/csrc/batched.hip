// Batched (alpha, omega) sweep: many systems of uneven size, up to 16
// parameter trials each, solved in one persistent launch captured in a HIP
// graph.  This is the parameter sweep behind the predictor's training set
// (Section 3.3 builds its training set from near-optimal parameters of small
// systems of the same structure).
//
// Work unit: one system and a pack of up to kPack of its trials, run in
// lockstep as a multi-right-hand-side solve: every phase of Algorithm 1 loads
// the system's matrix row once and applies it to each active trial of the
// pack; a trial that has finished its inner solve (or its whole solve) is
// masked out of the phase.  The phases and their arithmetic are those of the
// single-system solver with the one-reduction (Chronopoulos-Gear) inner
// solves, so a trial's iterates match a single solve's up to the order of its
// sums.
//
// A unit is processed by a group of `gsize` blocks on one XCD, each block
// owning a contiguous band of row tiles; the blocks of a group meet at a group
// barrier (a relay through the group's first block, as the device-wide
// barrier of the single-system solver) after every phase, and a one-block
// group synchronises in LDS only.  Groups pull units from a device queue,
// largest systems first.  The launch shape -- threads per block and blocks
// per group, i.e. the rows a block owns -- is chosen per batch shape by a
// timed one-sweep trial of every candidate, weighted by the load imbalance
// the largest unit causes.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <numeric>
#include <vector>

#include <unistd.h>

#include "solve_body.h"

namespace gadi {

gadi_status ensure_fp32_public(System& s);

constexpr int kPack = 4;                 // trials per unit
constexpr int kRed = 4 * kPack + 2;      // reduction payload (see GroupSync)
constexpr int kGenW = 16;                // widest row of a per-slice-metadata layout
constexpr int kVecs = 12;                // vectors per trial in the workspace

// One system of the batch, device view.
struct BSys {
  int n, npad, uni;  // uni: offsets per slice of a uniform diagonal layout, 0 = per-slice metadata
  int32_t dia_u[kDiaMax];
  const int32_t* slice_ptr;
  const int32_t* col;
  const int32_t* slice_dia;
  const int32_t* dia_off;
  const double* a_off;
  const double* a_diag;
  const void* h_off;
  const void* s_off;
  const void* h_diag;
  const double* b;  // [npad], zero padded
  long long xoff;   // offset of trial 0's solution in the output buffer, -1 if not wanted
};

struct BArgs {
  const BSys* sys;
  const int* order;  // unit ids (system * npacks + pack), largest systems first
  int nunits, nsys, ntrial, npacks, grid_per_system;
  const double* alpha;
  const double* omega;
  double tol, eps;
  int maxit_out, maxit_in;
  int gsize;        // blocks per group
  char* ws;         // per-group workspace: kVecs * kPack vector slots
  size_t slot;      // bytes per vector slot
  size_t ws_stride; // bytes per group
  int* queue;
  DevInfo* info;    // [nsys * ntrial]
  double* xout;
  unsigned long long* best_work;  // [nsys] or null: prune dominated trials
  unsigned long long* flags;      // [G * kFlagStride] arrival epochs
  double* part;                   // [G][2][kRed] partial results
  double* result;                 // [ngroups][2][kRed]
  unsigned long long* release;    // [ngroups * kFlagStride]
  int* abort;
  long long timeout;
  unsigned* done;  // optional: units finished per group, in mapped host memory (progress reports)
};

// Reduction payload: slots [3t, 3t+3) sums of trial t, [3P + t] a maximum of
// trial t, slot 4P a sum (broadcast of the unit index), slot 4P + 1 a maximum
// (the pruning bound, negated).
__device__ __forceinline__ bool red_is_max(int i) { return (i >= 3 * kPack && i < 4 * kPack) || i == 4 * kPack + 1; }

// Synchronisation of one group: LDS only for a one-block group; otherwise
// every block publishes its block partials and an arrival epoch, the group's
// first block combines the partials in rank order (a fixed order) and releases
// the group through one word; agent-scope release / acquire fences order the
// phase data.  A wait beyond `timeout` ticks sets the abort flag, and every
// block then leaves.
template <int BLOCK>
struct GroupSync {
  unsigned long long* flags;
  double* part;
  double* result;
  unsigned long long* release;
  int* abort;
  long long timeout;
  int gsize;
  unsigned group, rank, lb;
  unsigned long long epoch;
  long long phases;

  __device__ __forceinline__ bool reduce(double (&v)[kRed]) {
    constexpr int NW = BLOCK / 64;
    __shared__ double sh[NW][kRed];
    __shared__ double out[kRed];
    __shared__ int sh_abort;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
#pragma unroll
    for (int i = 0; i < kRed; ++i) {
      const double w = red_is_max(i) ? wave_max(v[i]) : wave_sum(v[i]);
      if (lane == 0) sh[wid][i] = w;
    }
    if (tid == 0) sh_abort = 0;
    __syncthreads();
    ++phases;
    if (tid < kRed) {
      double acc = red_is_max(tid) ? -INFINITY : 0.0;
      for (int w = 0; w < NW; ++w) acc = red_is_max(tid) ? fmax(acc, sh[w][tid]) : acc + sh[w][tid];
      out[tid] = acc;
    }
    const int gs = gsize;
    if (gs > 1) {
      epoch += 1;
      const unsigned par = (unsigned)(epoch & 1ull);
      __syncthreads();
      if (tid < kRed) part[((size_t)lb * 2 + par) * kRed + tid] = out[tid];
      __syncthreads();
      if (tid == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(flags + (size_t)lb * kFlagStride, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      const unsigned first = group * (unsigned)gs;
      double* res = result + ((size_t)group * 2 + par) * kRed;
      if (rank == 0) {
        const long long t_start = wall_clock64();
        for (;;) {
          int mine = 1;
          for (int k = tid; k < gs; k += BLOCK)
            if (__hip_atomic_load(flags + (size_t)(first + k) * kFlagStride, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT) < epoch)
              mine = 0;
          if (__syncthreads_and(mine)) break;
          const int expired = (tid == 0) && (wall_clock64() - t_start > timeout ||
                                             __hip_atomic_load(abort, __ATOMIC_RELAXED,
                                                               __HIP_MEMORY_SCOPE_AGENT) != 0);
          if (__syncthreads_or(expired)) {
            if (tid == 0) {
              __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              sh_abort = 1;
            }
            break;
          }
        }
        if (tid == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __syncthreads();
        if (tid < kRed) {
          double acc = red_is_max(tid) ? -INFINITY : 0.0;
          for (int k = 0; k < gs; ++k) {
            const double pv = part[((size_t)(first + k) * 2 + par) * kRed + tid];
            acc = red_is_max(tid) ? fmax(acc, pv) : acc + pv;
          }
          res[tid] = acc;
        }
        __syncthreads();
        if (tid == 0) {
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          __hip_atomic_store(release + (size_t)group * kFlagStride, epoch, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
        }
      } else if (tid == 0) {
        const long long t_start = wall_clock64();
        unsigned spins = 0;
        while (__hip_atomic_load(release + (size_t)group * kFlagStride, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT) < epoch) {
          __builtin_amdgcn_s_sleep(1);
          if ((++spins & 255u) == 0u) {
            if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                wall_clock64() - t_start > timeout) {
              __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              sh_abort = 1;
              break;
            }
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      __syncthreads();
      if (tid < kRed) out[tid] = res[tid];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kRed; ++i) v[i] = out[i];
    const bool ok = sh_abort == 0;
    __syncthreads();  // sh and out are rewritten by the next call
    return ok;
  }
};

// A row of the shared sparsity pattern: its stored values and (clamped)
// columns, loaded once per phase and applied to every active trial.
template <class MT, int W>
struct RowView {
  MT v[W];
  unsigned c[W];
};

template <int W>
struct PatU {  // uniform diagonal layout: W offsets in scalar registers
  int off[W];
  int nmax;
  template <class MT>
  __device__ __forceinline__ RowView<MT, W> row(unsigned row, const MT* __restrict__ val) const {
    RowView<MT, W> r;
    const unsigned k0 = (row & ~(unsigned)(kSlice - 1)) * W + (row & (kSlice - 1));
#pragma unroll
    for (int j = 0; j < W; ++j) {
      r.v[j] = at(val, k0 + j * kSlice);
      const int cc = (int)row + off[j];
      r.c[j] = (unsigned)(cc < 0 ? 0 : (cc > nmax ? nmax : cc));
    }
    return r;
  }
};

struct PatM {  // per-slice metadata (explicit or diagonal-style slices), at most kGenW slots
  Pattern p;
  template <class MT>
  __device__ __forceinline__ RowView<MT, kGenW> row(unsigned row, const MT* __restrict__ val) const {
    RowView<MT, kGenW> r;
    const int s = __builtin_amdgcn_readfirstlane((int)(row >> 6));
    const int beg = p.sp[s];
    const int w = (p.sp[s + 1] - beg) >> 6;
    const int k0 = beg + (int)(row & (kSlice - 1));
    const int dia = p.dia[s];
#pragma unroll
    for (int j = 0; j < kGenW; ++j) {
      if (j < w) {
        r.v[j] = val[k0 + j * kSlice];
        if (dia) {
          const int cc = (int)row + p.doff[(size_t)s * kDiaMax + j];
          r.c[j] = (unsigned)(cc < 0 ? 0 : (cc > p.nmax ? p.nmax : cc));
        } else {
          r.c[j] = (unsigned)p.col[k0 + j * kSlice];
        }
      } else {
        r.v[j] = MT{};
        r.c[j] = row;
      }
    }
    return r;
  }
};

template <class AT, class MT, int W, class F>
__device__ __forceinline__ AT rdot(const RowView<MT, W>& r, F&& f) {
  AT acc = 0;
#pragma unroll
  for (int j = 0; j < W; ++j) acc += ld<AT>(r.v[j]) * f(j, r.c[j]);
  return acc;
}

__device__ __forceinline__ bool has(unsigned m, int t) { return (m >> t) & 1u; }

// f(integral_constant<int, t>) for each trial t in mask m, t a compile-time
// constant so that the per-trial partial sums stay in registers
template <int T = 0, class F>
__device__ __forceinline__ void each_trial(unsigned m, F&& f) {
  if constexpr (T < kPack) {
    if (has(m, T)) f(std::integral_constant<int, T>{});
    each_trial<T + 1>(m, f);
  }
}

// Per-trial scalars of the unit a block is running, in LDS: updated by thread
// 0 after each reduction (a block barrier follows), read by every thread.
template <class AT>
struct UnitState {
  AT alpha[kPack], inv_alpha[kPack], tmo[kPack], sc[kPack], akt[kPack], bkt[kPack];
  double rho0[kPack], res[kPack], rmax[kPack], gam[kPack], del[kPack], gam0[kPack], gprev[kPack], aprev[kPack];
  double zmax[kPack], akd[kPack], unscale[kPack];
  int status[kPack], sweep[kPack], it[kPack], its[kPack], e1[kPack], e2[kPack];
  long long ih[kPack], is[kPack];
  unsigned live;  // trials still iterating
  unsigned mask;  // trials of the current phase
  unsigned next;  // trials of the following phase
};

// Algorithm 1 for the trials of one unit, rows [t0 * BLOCK, t1 * BLOCK) of
// system S, in lockstep.  Within a phase each row's matrix values and columns
// are loaded once; the active trials then follow one another, each issuing all
// of its loads before its arithmetic.  Fills the per-trial records; returns
// false if a group barrier timed out.
template <class Mode, int BLOCK, int W, class Pat>
__device__ __forceinline__ bool unit_body(const BArgs& ba, GroupSync<BLOCK>& gs, const Pat& pat, const BSys& S, int si,
                          int pack, int ntr, char* ws, int t0, int t1) {
  using MT = typename Mode::MT;
  using VT = typename Mode::VT;
  using ST = typename Mode::ST;
  using RT = typename Mode::RT;
  using AT = typename Mode::AT;
  using DT = typename Mode::DT;
  using XT = typename Mode::XT;
  using FT = typename Mode::FT;
  using AV = typename Mode::AV;
  __shared__ UnitState<AT> U;
  const unsigned tid = threadIdx.x;
  const bool lead = tid == 0;
  const size_t slot = ba.slot;
  // vector v of trial t
  auto vec = [&](int v, int t) { return ws + ((size_t)v * kPack + t) * slot; };
  enum { X = 0, R = 1, Z = 2, WS = 3, R0 = 4, R1 = 5, W0 = 6, W1 = 7, S0 = 8, S1 = 9, PV = 10, TV = 11 };

  const MT* __restrict__ hoff = (const MT*)S.h_off;
  const MT* __restrict__ soff = (const MT*)S.s_off;
  const DT* __restrict__ hdiag = (const DT*)S.h_diag;
  const AV* __restrict__ aoff = (const AV*)S.a_off;
  const AV* __restrict__ adiag = (const AV*)S.a_diag;
  const double* __restrict__ b = S.b;
  const double eps2 = ba.eps * ba.eps;
  const int overflow_status = std::is_same<VT, __half>::value ? GADI_EOVERFLOW16 : GADI_EDIVERGED;

  if (lead) {
    U.live = 0;
#pragma unroll
    for (int t = 0; t < kPack; ++t) {
      const int gi = ba.grid_per_system ? si * ba.ntrial + pack * kPack + t : pack * kPack + t;
      const bool on = t < ntr;
      const double al = on ? ba.alpha[gi] : 1.0;
      U.alpha[t] = (AT)al;
      U.inv_alpha[t] = (AT)(1.0 / al);
      U.tmo[t] = (AT)(2.0 - (on ? ba.omega[gi] : 0.0));
      U.rho0[t] = U.res[t] = 0.0;
      U.status[t] = GADI_EMAXIT;
      U.sweep[t] = 0;
      U.ih[t] = U.is[t] = 0;
      if (on) U.live |= 1u << t;
    }
  }
  __syncthreads();
  auto rnd = [](AT v) { return ld<AT>(st<VT>(v)); };
  auto ldv = [](VT v) { return ld<AT>(v); };
  double red[kRed];
  auto clear = [&]() {
#pragma unroll
    for (int i = 0; i < kRed; ++i) red[i] = red_is_max(i) ? -INFINITY : 0.0;
  };
  auto rows = [&](auto&& f) {
    for (int tile = t0; tile < t1; ++tile) f((unsigned)tile * BLOCK + tid);
  };
  // thread 0 updates the unit state from the reduction; the block then sees it
  auto update = [&](auto&& f) {
    if (lead) f();
    __syncthreads();
  };
  // operand loads of one trial issued together, then its arithmetic
  auto fence = []() { __builtin_amdgcn_sched_barrier(0); };

  {
    // x_0 = 0 for every trial (other blocks read it at neighbouring rows: a barrier follows)
    const unsigned m = U.live;
    rows([&](unsigned row) {
#pragma unroll
      for (int t = 0; t < kPack; ++t)
        if (has(m, t)) at((XT*)vec(X, t), row) = XT(0);
    });
  }
  clear();
  if (!gs.reduce(red)) return false;

  for (;;) {
    // ------------------------------------------------ a1: r = b - A x, ||r||^2, ||r||_inf
    {
      const unsigned m = U.live;
      clear();
      rows([&](unsigned row) {
        const auto rv = pat.row(row, aoff);
        const AV d = at(adiag, row);
        const double br = at(b, row);
        each_trial(m, [&](auto tc) {
          constexpr int t = decltype(tc)::value;
            const XT* xt = (const XT*)vec(X, t);
            const XT xo = at(xt, row);
            XT xn[W];
#pragma unroll
            for (int j = 0; j < W; ++j) xn[j] = at(xt, rv.c[j]);
            fence();
            const FT ax = (FT)d * (FT)xo + rdot<FT>(rv, [&](int j, unsigned) { return (FT)xn[j]; });
            const double ri = (double)((FT)br - ax);
            at((RT*)vec(R, t), row) = (RT)ri;
            red[3 * t] += ri * ri;
            red[3 * kPack + t] = fmax(red[3 * kPack + t], fabs(ri));
          });
      });
      if (ba.best_work && lead)
        red[4 * kPack + 1] = -(double)__hip_atomic_load(ba.best_work + si, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (!gs.reduce(red)) return false;
    }
    update([&]() {
      const double best = -red[4 * kPack + 1];
      U.mask = 0;
#pragma unroll
      for (int t = 0; t < kPack; ++t) {
        if (!has(U.live, t)) continue;
        const double rho = sqrt(red[3 * t]);
        if (U.sweep[t] == 0) U.rho0[t] = rho;
        U.res[t] = U.rho0[t] > 0.0 ? rho / U.rho0[t] : 0.0;
        const long long wk = U.ih[t] + 2 * U.is[t] + 5ll * U.sweep[t];
        int stop = -1;
        if (rho <= ba.tol * U.rho0[t]) stop = GADI_OK;
        else if (!isfinite(rho) || rho > 1e6 * U.rho0[t]) stop = GADI_EDIVERGED;
        else if (U.sweep[t] >= ba.maxit_out) stop = GADI_EMAXIT;
        else if (ba.best_work && (double)wk > best) stop = GADI_EPRUNED;
        if (stop >= 0) {
          U.status[t] = stop;
          U.live &= ~(1u << t);
          if (stop == GADI_OK && ba.best_work && gs.rank == 0) atomicMin(ba.best_work + si, (unsigned long long)wk);
          continue;
        }
        U.rmax[t] = red[3 * kPack + t];
        int e1 = 0;
        (void)frexp(U.rmax[t], &e1);
        U.e1[t] = clamp_exp(e1);
        U.sc[t] = (AT)ldexp(1.0, -U.e1[t]);
      }
    });
    if (!U.live) break;

    // ------------------------------------------------ a3: CG on (alpha I + H) z = r 2^-e1
    {
      const unsigned m = U.live;
      clear();
      rows([&](unsigned row) {
        const auto rv = pat.row(row, hoff);
        const AT hd = ld<AT>(at(hdiag, row));
        each_trial(m, [&](auto tc) {
          constexpr int t = decltype(tc)::value;
            const AT sc1 = U.sc[t];
            const RT* rt = (const RT*)vec(R, t);
            const RT ro = at(rt, row);
            RT rn[W];
#pragma unroll
            for (int j = 0; j < W; ++j) rn[j] = at(rt, rv.c[j]);
            fence();
            const AT ri = rnd((AT)ro * sc1);
            const AT kr = (U.alpha[t] + hd) * ri + rdot<AT>(rv, [&](int j, unsigned) { return rnd((AT)rn[j] * sc1); });
            const AT wi = rnd(kr);
            at((VT*)vec(R0, t), row) = st<VT>(ri);
            at((VT*)vec(W0, t), row) = st<VT>(wi);
            red[3 * t] += (double)ri * (double)ri;
            red[3 * t + 1] += (double)wi * (double)ri;
          });
      });
      if (!gs.reduce(red)) return false;
    }
    update([&]() {
      U.mask = 0;
#pragma unroll
      for (int t = 0; t < kPack; ++t) {
        U.gam[t] = U.gam0[t] = red[3 * t];
        U.del[t] = red[3 * t + 1];
        U.gprev[t] = U.aprev[t] = 1.0;
        U.zmax[t] = 0.0;
        U.it[t] = 0;
        if (has(U.live, t) && U.gam0[t] > 0.0) U.mask |= 1u << t;
      }
    });
    for (int k = 0; U.mask; ++k) {
      // step coefficients; a breakdown ends that trial's inner solve
      update([&]() {
#pragma unroll
        for (int t = 0; t < kPack; ++t) {
          if (!has(U.mask, t)) continue;
          const double beta = k == 0 ? 0.0 : U.gam[t] / U.gprev[t];
          const double den = k == 0 ? U.del[t] : U.del[t] - beta * U.gam[t] / U.aprev[t];
          if (!(den > 0.0) || !isfinite(den)) {
            if (k == 0) U.status[t] = isfinite(den) ? GADI_ENOTSPD : overflow_status;
            U.mask &= ~(1u << t);
            continue;
          }
          U.akd[t] = U.gam[t] / den;
          U.akt[t] = (AT)U.akd[t];
          U.bkt[t] = (AT)beta;
        }
      });
      const unsigned m = U.mask;
      if (!m) break;
      const int rk = k & 1;  // ping-pong: r_k, w_k in slot rk; s_{k-1} in 1 - rk
      const bool first = k == 0;
      clear();
      rows([&](unsigned row) {
        const auto rv = pat.row(row, hoff);
        const AT hd = ld<AT>(at(hdiag, row));
        each_trial(m, [&](auto tc) {
          constexpr int t = decltype(tc)::value;
            const AT akt = U.akt[t], bkt = U.bkt[t];
            const VT* rkp = (const VT*)vec(R0 + rk, t);
            const VT* wkp = (const VT*)vec(W0 + rk, t);
            const VT* spp = (const VT*)vec(S0 + 1 - rk, t);
            const VT r_ = at(rkp, row), w_ = at(wkp, row);
            VT sp_{}, p_{};
            ST z_ = st<ST>(AT(0));
            VT nr[W], nw[W], ns[W];
#pragma unroll
            for (int j = 0; j < W; ++j) {
              nr[j] = at(rkp, rv.c[j]);
              nw[j] = at(wkp, rv.c[j]);
            }
            if (!first) {
              sp_ = at(spp, row);
              p_ = at((const VT*)vec(PV, t), row);
              z_ = at((const ST*)vec(Z, t), row);
#pragma unroll
              for (int j = 0; j < W; ++j) ns[j] = at(spp, rv.c[j]);
            }
            fence();
            const AT ri = ldv(r_);
            AT s, p;
            ST z;
            if (first) {
              s = ldv(w_);
              p = ri;
              z = st<ST>(akt * ri);
            } else {
              s = rnd(fma_at<AT>(bkt, ldv(sp_), ldv(w_)));
              p = rnd(fma_at<AT>(bkt, ldv(p_), ri));
              z = st<ST>(ld<AT>(z_) + akt * p);
            }
            const AT rn = rnd(fma_at<AT>(-akt, s, ri));
            // r_{k+1} at the neighbouring rows, computed as their owners compute it
            const AT kr = (U.alpha[t] + hd) * rn + rdot<AT>(rv, [&](int j, unsigned) {
                            const AT sj = first ? ldv(nw[j]) : rnd(fma_at<AT>(bkt, ldv(ns[j]), ldv(nw[j])));
                            return rnd(fma_at<AT>(-akt, sj, ldv(nr[j])));
                          });
            const AT wn = rnd(kr);
            at((VT*)vec(S0 + rk, t), row) = st<VT>(s);
            at((VT*)vec(PV, t), row) = st<VT>(p);
            at((ST*)vec(Z, t), row) = z;
            at((VT*)vec(R0 + 1 - rk, t), row) = st<VT>(rn);
            at((VT*)vec(W0 + 1 - rk, t), row) = st<VT>(wn);
            red[3 * t] += (double)rn * (double)rn;
            red[3 * t + 1] += (double)wn * (double)rn;
            red[3 * kPack + t] = fmax(red[3 * kPack + t], fabs((double)ld<AT>(z)));
          });
      });
      if (!gs.reduce(red)) return false;
      update([&]() {
#pragma unroll
        for (int t = 0; t < kPack; ++t) {
          if (!has(U.mask, t)) continue;
          U.gprev[t] = U.gam[t];
          U.aprev[t] = U.akd[t];
          U.gam[t] = red[3 * t];
          U.del[t] = red[3 * t + 1];
          U.zmax[t] = red[3 * kPack + t];
          U.it[t] = k + 1;
          if (U.gam[t] <= eps2 * U.gam0[t] || U.it[t] >= ba.maxit_in || !isfinite(U.gam[t]))
            U.mask &= ~(1u << t);
        }
      });
    }
    // end of the CG solves; trials with a usable z go on to the S-step
    update([&]() {
      U.mask = 0;
#pragma unroll
      for (int t = 0; t < kPack; ++t) {
        U.its[t] = 0;
        if (!has(U.live, t)) continue;
        U.ih[t] += U.it[t];
        if (U.status[t] != GADI_EMAXIT) {  // inner breakdown on the first step
          U.live &= ~(1u << t);
          continue;
        }
        if (!isfinite(U.zmax[t])) {
          U.status[t] = overflow_status;
          U.live &= ~(1u << t);
          continue;
        }
        int e2 = 0;
        (void)frexp((double)U.tmo[t] * U.zmax[t], &e2);
        U.e2[t] = clamp_exp(e2);
        U.sc[t] = (AT)ldexp(1.0, -U.e2[t]);
        if (U.it[t] > 0 && U.zmax[t] > 0.0) U.mask |= 1u << t;
      }
    });

    // ------------------------------------------------ a4/a5: CGNE on (I + S/alpha) u = (2 - omega) z 2^-e2
    if (U.mask) {
      // r_0 = g, t = (S/alpha) g
      {
        const unsigned m = U.mask;
        clear();
        rows([&](unsigned row) {
          const auto rv = pat.row(row, soff);
          each_trial(m, [&](auto tc) {
            constexpr int t = decltype(tc)::value;
              const ST* zt = (const ST*)vec(Z, t);
              const ST zo = at(zt, row);
              ST zn[W];
#pragma unroll
              for (int j = 0; j < W; ++j) zn[j] = at(zt, rv.c[j]);
              fence();
              const AT g = rnd(U.tmo[t] * ld<AT>(zo) * U.sc[t]);
              const AT tv = U.inv_alpha[t] * rdot<AT>(rv, [&](int j, unsigned) {
                              return rnd(U.tmo[t] * ld<AT>(zn[j]) * U.sc[t]);
                            });
              at((VT*)vec(R0, t), row) = st<VT>(g);
              at((VT*)vec(TV, t), row) = st<VT>(tv);
              red[3 * t] += (double)g * (double)g;
            });
        });
        if (!gs.reduce(red)) return false;
      }
      update([&]() {
#pragma unroll
        for (int t = 0; t < kPack; ++t) U.gam0[t] = red[3 * t];
      });
      // w_0 = r_0 - (S/alpha) t
      {
        const unsigned m = U.mask;
        clear();
        rows([&](unsigned row) {
          const auto rv = pat.row(row, soff);
          each_trial(m, [&](auto tc) {
            constexpr int t = decltype(tc)::value;
              const VT ro = at((const VT*)vec(R0, t), row);
              const VT* tt = (const VT*)vec(TV, t);
              VT tn[W];
#pragma unroll
              for (int j = 0; j < W; ++j) tn[j] = at(tt, rv.c[j]);
              fence();
              const AT ri = ldv(ro);
              const AT wi = rnd(ri - U.inv_alpha[t] * rdot<AT>(rv, [&](int j, unsigned) { return ldv(tn[j]); }));
              at((VT*)vec(W0, t), row) = st<VT>(wi);
              red[3 * t + 1] += (double)wi * (double)ri;
            });
        });
        if (!gs.reduce(red)) return false;
      }
      update([&]() {
        const unsigned m = U.mask;
        U.mask = 0;
#pragma unroll
        for (int t = 0; t < kPack; ++t) {
          U.gam[t] = U.gam0[t];
          U.del[t] = red[3 * t + 1];
          U.gprev[t] = U.aprev[t] = 1.0;
          if (has(m, t) && U.gam0[t] > 0.0) U.mask |= 1u << t;
        }
      });
      for (int k = 0; U.mask; ++k) {
        update([&]() {
#pragma unroll
          for (int t = 0; t < kPack; ++t) {
            if (!has(U.mask, t)) continue;
            const double beta = k == 0 ? 0.0 : U.gam[t] / U.gprev[t];
            const double den = k == 0 ? U.del[t] : U.del[t] - beta * U.gam[t] / U.aprev[t];
            if (!(den > 0.0) || !isfinite(den)) {
              if (k == 0) U.status[t] = isfinite(den) ? GADI_ENOTSPD : overflow_status;
              U.mask &= ~(1u << t);
              continue;
            }
            U.akd[t] = U.gam[t] / den;
            U.akt[t] = (AT)U.akd[t];
            U.bkt[t] = (AT)beta;
          }
        });
        unsigned m = U.mask;
        if (!m) break;
        const int rk = k & 1;
        const bool first = k == 0;
        // s, p, w += a p, r_{k+1}, t = (S/alpha) r_{k+1}
        clear();
        rows([&](unsigned row) {
          const auto rv = pat.row(row, soff);
          each_trial(m, [&](auto tc) {
            constexpr int t = decltype(tc)::value;
              const AT akt = U.akt[t], bkt = U.bkt[t];
              const VT* rkp = (const VT*)vec(R0 + rk, t);
              const VT* wkp = (const VT*)vec(W0 + rk, t);
              const VT* spp = (const VT*)vec(S0 + 1 - rk, t);
              const VT r_ = at(rkp, row), w_ = at(wkp, row);
              VT sp_{}, p_{};
              ST ws_ = st<ST>(AT(0));
              VT nr[W], nw[W], ns[W];
#pragma unroll
              for (int j = 0; j < W; ++j) {
                nr[j] = at(rkp, rv.c[j]);
                nw[j] = at(wkp, rv.c[j]);
              }
              if (!first) {
                sp_ = at(spp, row);
                p_ = at((const VT*)vec(PV, t), row);
                ws_ = at((const ST*)vec(WS, t), row);
#pragma unroll
                for (int j = 0; j < W; ++j) ns[j] = at(spp, rv.c[j]);
              }
              fence();
              const AT ri = ldv(r_);
              AT s, p;
              ST wv;
              if (first) {
                s = ldv(w_);
                p = ri;
                wv = st<ST>(akt * ri);
              } else {
                s = rnd(fma_at<AT>(bkt, ldv(sp_), ldv(w_)));
                p = rnd(fma_at<AT>(bkt, ldv(p_), ri));
                wv = st<ST>(ld<AT>(ws_) + akt * p);
              }
              const AT rn = rnd(fma_at<AT>(-akt, s, ri));
              const AT tv = U.inv_alpha[t] * rdot<AT>(rv, [&](int j, unsigned) {
                              const AT sj = first ? ldv(nw[j]) : rnd(fma_at<AT>(bkt, ldv(ns[j]), ldv(nw[j])));
                              return rnd(fma_at<AT>(-akt, sj, ldv(nr[j])));
                            });
              at((VT*)vec(S0 + rk, t), row) = st<VT>(s);
              at((VT*)vec(PV, t), row) = st<VT>(p);
              at((ST*)vec(WS, t), row) = wv;
              at((VT*)vec(R0 + 1 - rk, t), row) = st<VT>(rn);
              at((VT*)vec(TV, t), row) = st<VT>(tv);
              red[3 * t] += (double)rn * (double)rn;
            });
        });
        if (!gs.reduce(red)) return false;
        update([&]() {
#pragma unroll
          for (int t = 0; t < kPack; ++t) {
            if (!has(U.mask, t)) continue;
            U.gprev[t] = U.gam[t];
            U.aprev[t] = U.akd[t];
            U.gam[t] = red[3 * t];
            U.its[t] = k + 1;
            if (U.gam[t] <= eps2 * U.gam0[t] || U.its[t] >= ba.maxit_in || !isfinite(U.gam[t]))
              U.mask &= ~(1u << t);
          }
        });
        m = U.mask;
        if (!m) break;
        // w_{k+1} = r_{k+1} - (S/alpha) t
        clear();
        rows([&](unsigned row) {
          const auto rv = pat.row(row, soff);
          each_trial(m, [&](auto tc) {
            constexpr int t = decltype(tc)::value;
              const VT ro = at((const VT*)vec(R0 + 1 - rk, t), row);
              const VT* tt = (const VT*)vec(TV, t);
              VT tn[W];
#pragma unroll
              for (int j = 0; j < W; ++j) tn[j] = at(tt, rv.c[j]);
              fence();
              const AT rn = ldv(ro);
              const AT wn = rnd(rn - U.inv_alpha[t] * rdot<AT>(rv, [&](int j, unsigned) { return ldv(tn[j]); }));
              at((VT*)vec(W0 + 1 - rk, t), row) = st<VT>(wn);
              red[3 * t + 1] += (double)wn * (double)rn;
            });
        });
        if (!gs.reduce(red)) return false;
        update([&]() {
#pragma unroll
          for (int t = 0; t < kPack; ++t)
            if (has(U.mask, t)) U.del[t] = red[3 * t + 1];
        });
      }
    }
    update([&]() {
      U.mask = 0;
#pragma unroll
      for (int t = 0; t < kPack; ++t) {
        if (!has(U.live, t)) continue;
        U.is[t] += U.its[t];
        if (U.status[t] != GADI_EMAXIT) {
          U.live &= ~(1u << t);
          continue;
        }
        if (U.its[t] > 0) {
          U.mask |= 1u << t;
          U.unscale[t] = ldexp(1.0, U.e1[t] + U.e2[t]);
        }
      }
    });

    // ------------------------------------------------ a6: x += (I - S/alpha) w 2^(e1 + e2)
    if (U.mask) {
      const unsigned m = U.mask;
      rows([&](unsigned row) {
        const auto rv = pat.row(row, soff);
        each_trial(m, [&](auto tc) {
          constexpr int t = decltype(tc)::value;
            const ST* wt = (const ST*)vec(WS, t);
            const ST wo = at(wt, row);
            const XT xo = at((const XT*)vec(X, t), row);
            ST wn[W];
#pragma unroll
            for (int j = 0; j < W; ++j) wn[j] = at(wt, rv.c[j]);
            fence();
            const AT ui = ld<AT>(wo) - U.inv_alpha[t] * rdot<AT>(rv, [&](int j, unsigned) { return ld<AT>(wn[j]); });
            at((XT*)vec(X, t), row) = (XT)(xo + (XT)((double)ui * U.unscale[t]));
          });
      });
      clear();
      if (!gs.reduce(red)) return false;
    }
    update([&]() {
#pragma unroll
      for (int t = 0; t < kPack; ++t)
        if (has(U.live, t)) ++U.sweep[t];
    });
  }

  if (gs.rank == 0 && lead) {
    for (int t = 0; t < ntr; ++t) {
      DevInfo r{};
      r.status = U.status[t];
      r.sweeps = U.sweep[t];
      r.inner_h = U.ih[t];
      r.inner_s = U.is[t];
      r.relres = U.res[t];
      r.rho0 = U.rho0[t];
      ba.info[(size_t)si * ba.ntrial + pack * kPack + t] = r;
    }
  }
  // trial 0's solution
  if (pack == 0 && S.xoff >= 0)
    rows([&](unsigned row) {
      if ((int)row < S.n) ba.xout[S.xoff + row] = (double)at((const XT*)vec(X, 0), row);
    });
  __syncthreads();  // U is reset by the next unit
  return true;
}

template <class Mode, int BLOCK>
__global__ void __launch_bounds__(BLOCK) batched_kernel(BArgs ba) {
  __shared__ int sh_unit;
  // blocks of one XCD form the groups: logical index lb, group lb / gsize
  const unsigned lb = logical_block(blockIdx.x, gridDim.x);
  GroupSync<BLOCK> gs{ba.flags, ba.part, ba.result, ba.release, ba.abort, ba.timeout, ba.gsize,
                      lb / (unsigned)ba.gsize, lb % (unsigned)ba.gsize, lb, 0ull, 0ll};
  char* ws = ba.ws + ba.ws_stride * gs.group;
  double red[kRed];
  unsigned units_done = 0;
  for (;;) {
    // the group's first block takes the next unit and the group barrier broadcasts it
#pragma unroll
    for (int i = 0; i < kRed; ++i) red[i] = red_is_max(i) ? -INFINITY : 0.0;
    if (threadIdx.x == 0) {
      sh_unit = gs.rank == 0 ? atomicAdd(ba.queue, 1) : 0;
      red[4 * kPack] = (double)sh_unit;
    }
    if (!gs.reduce(red)) return;
    const int k = (int)red[4 * kPack];
    if (k >= ba.nunits) break;
    const int u = ba.order[k];
    const int si = u / ba.npacks, pack = u % ba.npacks;
    const int ntr = min(kPack, ba.ntrial - pack * kPack);
    const BSys S = ba.sys[si];
    const int ntiles = S.npad / BLOCK;
    const int t0 = (int)((long long)ntiles * gs.rank / ba.gsize);
    const int t1 = (int)((long long)ntiles * (gs.rank + 1) / ba.gsize);
    const long long t_start = wall_clock64();
    const long long ph0 = gs.phases;
    bool ok;
    if (S.uni == 4) {
      PatU<4> pat;
#pragma unroll
      for (int j = 0; j < 4; ++j) pat.off[j] = S.dia_u[j];
      pat.nmax = S.n - 1;
      ok = unit_body<Mode, BLOCK, 4>(ba, gs, pat, S, si, pack, ntr, ws, t0, t1);
    } else if (S.uni == 6) {
      PatU<6> pat;
#pragma unroll
      for (int j = 0; j < 6; ++j) pat.off[j] = S.dia_u[j];
      pat.nmax = S.n - 1;
      ok = unit_body<Mode, BLOCK, 6>(ba, gs, pat, S, si, pack, ntr, ws, t0, t1);
    } else {
      const PatM pat{Pattern{S.slice_ptr, S.col, S.slice_dia, S.dia_off, S.n - 1}};
      ok = unit_body<Mode, BLOCK, kGenW>(ba, gs, pat, S, si, pack, ntr, ws, t0, t1);
    }
    if (!ok) return;
    if (gs.rank == 0 && threadIdx.x == 0) {
      for (int t = 0; t < ntr; ++t) {
        DevInfo& r = ba.info[(size_t)si * ba.ntrial + pack * kPack + t];
        r.barriers = gs.phases - ph0;
        r.barrier_ticks = wall_clock64() - t_start;  // the unit's wall-clock ticks
      }
      if (ba.done) __hip_atomic_store(ba.done + gs.group, ++units_done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

// Queue, barrier state and pruning bounds start fresh in every launch (a
// kernel, not a memset, so the launch can be captured in a graph).
__global__ void reset_batch_kernel(BArgs ba, int nblocks, int ngroups) {
  const int i0 = blockIdx.x * blockDim.x + threadIdx.x, step = gridDim.x * blockDim.x;
  if (i0 == 0) {
    *ba.queue = 0;
    *ba.abort = 0;
  }
  for (int i = i0; i < nblocks * kFlagStride; i += step) ba.flags[i] = 0ull;
  for (int i = i0; i < ngroups * kFlagStride; i += step) ba.release[i] = 0ull;
  if (ba.best_work)
    for (int i = i0; i < ba.nsys; i += step) ba.best_work[i] = ~0ull;
}

template <class Mode, int BLOCK>
static gadi_status occupancy_t(int* nb) {
  GADI_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, batched_kernel<Mode, BLOCK>, BLOCK, 0));
  if (*nb < 1) *nb = 0;
  return GADI_OK;
}

// Resident blocks per compute unit of the batched kernel.
static gadi_status batched_occupancy(int prec, int block, int* nb) {
  *nb = 0;
#define OCC(M)                                       \
  switch (block) {                                   \
    case 512: return occupancy_t<M, 512>(nb);        \
    case 1024: return occupancy_t<M, 1024>(nb);      \
  }
  if (prec == GADI_PREC_FP16_IR) {
    OCC(ModeF16)
  } else if (prec == GADI_PREC_FP32_IR) {
    OCC(ModeF32)
  } else {
    OCC(ModeF64)
  }
#undef OCC
  return GADI_EINVAL;
}

// G never exceeds the blocks that fit on the device at once (occupancy times
// compute units), so every block of a group is resident while the launch runs
// alone; the group barrier's time limit ends the launch otherwise.  A plain
// launch, so that it can be captured in a graph.
template <class Mode, int BLOCK>
static gadi_status launch_batched_t(const BArgs& ba, int G, hipStream_t stream) {
  if (ba.gsize < 1 || G < ba.gsize || G % ba.gsize) return GADI_EINVAL;
  hipLaunchKernelGGL(reset_batch_kernel, dim3(64), dim3(256), 0, stream, ba, G, G / ba.gsize);
  hipLaunchKernelGGL((batched_kernel<Mode, BLOCK>), dim3((unsigned)G), dim3(BLOCK), 0, stream, ba);
  GADI_HIP_CHECK(hipGetLastError());
  return GADI_OK;
}

template <class Mode>
static gadi_status launch_batched_mode(const BArgs& ba, int block, int G, hipStream_t st) {
  switch (block) {
    case 512: return launch_batched_t<Mode, 512>(ba, G, st);
    case 1024: return launch_batched_t<Mode, 1024>(ba, G, st);
  }
  return GADI_EINVAL;
}

static gadi_status launch_batched(int prec, const BArgs& ba, int block, int G, hipStream_t st) {
  if (prec == GADI_PREC_FP16_IR) return launch_batched_mode<ModeF16>(ba, block, G, st);
  if (prec == GADI_PREC_FP32_IR) return launch_batched_mode<ModeF32>(ba, block, G, st);
  return launch_batched_mode<ModeF64>(ba, block, G, st);
}

// Record + launch through a HIP graph (captured once per call).  With
// `progress` (host view of ba.done), the wait reports each change of the
// finished-unit count on stderr.
static gadi_status run_graph(int prec, const BArgs& ba, int block, int G, hipStream_t stream,
                             volatile unsigned* progress, int ngroups) {
  hipStream_t cs = stream;
  bool own = false;
  if (!cs) {
    GADI_HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    own = true;
  }
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  gadi_status st = GADI_OK;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    st = launch_batched(prec, ba, block, G, cs);
    hipError_t e2 = hipStreamEndCapture(cs, &graph);
    if (st == GADI_OK && e2 != hipSuccess) st = fail_hip(e2, "hipStreamEndCapture", __FILE__, __LINE__);
  } else {
    st = fail_hip(e, "hipStreamBeginCapture", __FILE__, __LINE__);
  }
  if (st == GADI_OK) {
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipGraphLaunch(exec, cs);
    if (e == hipSuccess && progress) {
      unsigned seen = 0;
      for (;;) {
        e = hipStreamQuery(cs);
        if (e != hipErrorNotReady) break;
        unsigned d = 0;
        for (int q = 0; q < ngroups; ++q) d += progress[q];
        if (d != seen) {
          seen = d;
          std::fprintf(stderr, "gadi: batched units finished %u of %d\n", d, ba.nunits);
        }
        usleep(100000);
      }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(cs);
    if (e != hipSuccess) st = fail_hip(e, "graph launch", __FILE__, __LINE__);
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (own) (void)hipStreamDestroy(cs);
  return st;
}

// launch shape per batch shape: (prec, log2 max npad, log2 total rows, units bucket) -> (block, gsize)
static std::map<std::tuple<int, int, int, int>, std::pair<int, int>> g_batched_shape;

}  // namespace gadi

using namespace gadi;

extern "C" gadi_status gadi_ir_solve_batched(gadi_handle* const* hs, int32_t nsys, const double* const* b,
                                             double* const* x, const double* alpha, const double* omega,
                                             int32_t ntrial, double tol, const gadi_options* opts,
                                             gadi_solve_info* info) {
  if (!hs || !b || !alpha || !omega || !info || nsys < 1 || ntrial < 1 || ntrial > 16 || !(tol >= 0.0))
    return GADI_EINVAL;
  gadi_options o;
  if (opts) o = *opts;
  else gadi_default_options(&o, GADI_PREC_FP16_IR);
  const int ngrid = o.grid_per_system ? nsys * ntrial : ntrial;
  for (int t = 0; t < ngrid; ++t)
    if (!(alpha[t] > 0.0) || !std::isfinite(alpha[t]) || !(omega[t] >= 0.0 && omega[t] < 2.0)) return GADI_EINVAL;
  if (o.prec < GADI_PREC_FP64 || o.prec > GADI_PREC_FP32_IR || !(o.eps_inner > 0.0) || o.eps_inner >= 1.0 ||
      o.maxit_outer < 0 || o.maxit_inner < 1 || o.on_device)
    return GADI_EINVAL;
  for (int s = 0; s < nsys; ++s) {
    if (!hs[s] || !b[s]) return GADI_EINVAL;
    if (!hs[s]->sys.dia_uniform && hs[s]->sys.max_width > kGenW) return GADI_EINVAL;
  }
  hipStream_t stream = hs[0]->sys.stream;
  const int npacks = (ntrial + kPack - 1) / kPack;
  const int nunits = nsys * npacks;
  std::vector<BSys> hsys(nsys);
  int max_npad = 0;
  long long xtotal = 0, rows_total = 0;
  std::vector<long long> work(nsys);
  for (int s = 0; s < nsys; ++s) {
    System& S = hs[s]->sys;
    if (o.prec == GADI_PREC_FP32_IR) {
      gadi_status st = ensure_fp32_public(S);
      if (st != GADI_OK) return st;
    }
    BSys& d = hsys[s];
    d.n = S.n;
    d.npad = S.npad;
    d.uni = S.dia_uniform;
    for (int j = 0; j < kDiaMax; ++j) d.dia_u[j] = S.dia_u[j];
    d.slice_ptr = S.slice_ptr;
    d.col = S.col;
    d.slice_dia = S.slice_dia;
    d.dia_off = S.dia_off;
    d.a_off = S.a_off;
    d.a_diag = S.a_diag;
    if (o.prec == GADI_PREC_FP16_IR) {
      d.h_off = S.h_off16;
      d.s_off = S.s_off16;
      d.h_diag = S.h_diag16;
    } else if (o.prec == GADI_PREC_FP32_IR) {
      d.h_off = S.h_off32;
      d.s_off = S.s_off32;
      d.h_diag = S.h_diag32;
    } else {
      d.h_off = S.h_off64;
      d.s_off = S.s_off64;
      d.h_diag = S.h_diag64;
    }
    d.xoff = (x && x[s]) ? xtotal : -1;
    if (x && x[s]) xtotal += S.n;
    max_npad = std::max(max_npad, S.npad);
    work[s] = S.nslots + S.npad;
    rows_total += S.npad;
  }
  std::vector<size_t> boff(nsys);
  size_t btotal = 0;
  for (int s = 0; s < nsys; ++s) {
    boff[s] = btotal;
    btotal += (size_t)hsys[s].npad;
  }
  // units largest system first; the packs of a system stay together
  std::vector<int> sys_order(nsys);
  std::iota(sys_order.begin(), sys_order.end(), 0);
  std::stable_sort(sys_order.begin(), sys_order.end(), [&](int p, int q) { return work[p] > work[q]; });
  std::vector<int> order;
  order.reserve(nunits);
  for (int s : sys_order)
    for (int p = 0; p < npacks; ++p) order.push_back(s * npacks + p);

  int cus = 0, dev = 0, rate = 0;
  GADI_HIP_CHECK(hipGetDevice(&dev));
  GADI_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  GADI_HIP_CHECK(hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, dev));
  const double tick_hz = (rate > 0 ? rate : 100000) * 1000.0;
  const size_t slot = (((size_t)max_npad * sizeof(double)) + 255) & ~(size_t)255;
  const size_t ws_stride = slot * kVecs * kPack;

  // candidate launch shapes {threads per block, blocks per group}; each group
  // needs its workspace, within a 32 GiB budget
  const long long budget = 32ll << 30;
  struct Shape {
    int block, gsize, G;
  };
  std::vector<Shape> shapes;
  for (int block : {1024, 512}) {
    int occ = 0;
    gadi_status st = batched_occupancy(o.prec, block, &occ);
    if (st != GADI_OK) return st;
    if (occ < 1) continue;
    for (int g : {1, 2, 4, 8, 16}) {
      long long G = (long long)std::min(occ, 2) * cus;
      G = G / (8 * g) * (8 * g);  // whole groups on each XCD
      while (G > 0 && (G / g) * (long long)ws_stride > budget) G -= 8 * g;
      // no more groups than units
      while (G > 8 * g && G / g > nunits + 8) G -= 8 * g;
      if (G >= g && G <= kMaxBlocks) shapes.push_back({block, g, (int)G});
    }
  }
  if (shapes.empty()) return GADI_ENOMEM;
  int max_G = 0, max_groups = 0;
  for (const Shape& sh : shapes) {
    max_G = std::max(max_G, sh.G);
    max_groups = std::max(max_groups, sh.G / sh.gsize);
  }

  double *db = nullptr, *dal = nullptr, *dom = nullptr, *dx = nullptr, *dpart = nullptr, *dres = nullptr;
  BSys* dsys = nullptr;
  int *dorder = nullptr, *dq = nullptr, *dabort = nullptr;
  unsigned long long *dbest = nullptr, *dflags = nullptr, *drel = nullptr;
  DevInfo* dinfo = nullptr;
  char* dws = nullptr;
  gadi_status st = GADI_OK;
  auto cleanup = [&]() {
    void* ps[] = {db, dal, dom, dx, dsys, dorder, dq, dinfo, dws, dbest, dflags, drel, dpart, dres, dabort};
    for (void* p : ps)
      if (p) (void)hipFree(p);
  };
#define BCHECK(expr)                                                \
  do {                                                              \
    hipError_t e_ = (expr);                                         \
    if (e_ != hipSuccess) {                                         \
      st = fail_hip(e_, #expr, __FILE__, __LINE__);                 \
      cleanup();                                                    \
      return st;                                                    \
    }                                                               \
  } while (0)
  BCHECK(hipMalloc((void**)&db, sizeof(double) * btotal));
  BCHECK(hipMemset(db, 0, sizeof(double) * btotal));
  for (int s = 0; s < nsys; ++s) {
    BCHECK(hipMemcpy(db + boff[s], b[s], sizeof(double) * hsys[s].n, hipMemcpyHostToDevice));
    hsys[s].b = db + boff[s];
  }
  BCHECK(hipMalloc((void**)&dsys, sizeof(BSys) * nsys));
  BCHECK(hipMemcpy(dsys, hsys.data(), sizeof(BSys) * nsys, hipMemcpyHostToDevice));
  BCHECK(hipMalloc((void**)&dorder, sizeof(int) * nunits));
  BCHECK(hipMemcpy(dorder, order.data(), sizeof(int) * nunits, hipMemcpyHostToDevice));
  BCHECK(hipMalloc((void**)&dal, sizeof(double) * ngrid));
  BCHECK(hipMalloc((void**)&dom, sizeof(double) * ngrid));
  BCHECK(hipMemcpy(dal, alpha, sizeof(double) * ngrid, hipMemcpyHostToDevice));
  BCHECK(hipMemcpy(dom, omega, sizeof(double) * ngrid, hipMemcpyHostToDevice));
  BCHECK(hipMalloc((void**)&dq, sizeof(int)));
  BCHECK(hipMalloc((void**)&dabort, sizeof(int)));
  if (o.prune_dominated) BCHECK(hipMalloc((void**)&dbest, sizeof(unsigned long long) * nsys));
  BCHECK(hipMalloc((void**)&dinfo, sizeof(DevInfo) * nsys * ntrial));
  BCHECK(hipMemset(dinfo, 0, sizeof(DevInfo) * nsys * ntrial));
  BCHECK(hipMalloc((void**)&dx, sizeof(double) * (xtotal ? xtotal : 1)));
  BCHECK(hipMalloc((void**)&dws, ws_stride * (size_t)max_groups));
  BCHECK(hipMalloc((void**)&dflags, sizeof(unsigned long long) * kFlagStride * max_G));
  BCHECK(hipMalloc((void**)&drel, sizeof(unsigned long long) * kFlagStride * max_groups));
  BCHECK(hipMalloc((void**)&dpart, sizeof(double) * 2 * kRed * max_G));
  BCHECK(hipMalloc((void**)&dres, sizeof(double) * 2 * kRed * max_groups));

  BArgs ba{};
  ba.sys = dsys;
  ba.order = dorder;
  ba.nunits = nunits;
  ba.nsys = nsys;
  ba.ntrial = ntrial;
  ba.npacks = npacks;
  ba.grid_per_system = o.grid_per_system ? 1 : 0;
  ba.alpha = dal;
  ba.omega = dom;
  ba.tol = tol;
  ba.eps = o.eps_inner;
  ba.maxit_out = o.maxit_outer;
  ba.maxit_in = o.maxit_inner;
  ba.ws = dws;
  ba.slot = slot;
  ba.ws_stride = ws_stride;
  ba.queue = dq;
  ba.info = dinfo;
  ba.xout = dx;
  ba.best_work = dbest;
  ba.flags = dflags;
  ba.part = dpart;
  ba.result = dres;
  ba.release = drel;
  ba.abort = dabort;
  ba.timeout = (long long)(tick_hz * 20.0);

  // launch shape: env override, cached choice, or a timed one-sweep trial of
  // every candidate; the estimate scales the trial's time by the load the
  // largest unit puts on one block relative to the average block's
  int lg = 0, lr = 0;
  while ((1 << lg) < max_npad) ++lg;
  while ((1ll << lr) < rows_total) ++lr;
  const auto key = std::make_tuple((int)o.prec, lg, lr, nunits >= 256 ? 2 : (nunits >= 32 ? 1 : 0));
  Shape pick{0, 0, 0};
  const char* eb = std::getenv("GADI_BATCH_BLOCK");
  const char* eg = std::getenv("GADI_BATCH_GROUP");
  if (eb || eg) {
    const int want_b = eb ? std::atoi(eb) : 1024, want_g = eg ? std::atoi(eg) : 1;
    for (const Shape& sh : shapes)
      if (sh.block == want_b && sh.gsize == want_g) pick = sh;
    if (!pick.block) {
      cleanup();
      return GADI_EINVAL;
    }
  } else {
    auto it = g_batched_shape.find(key);
    if (it != g_batched_shape.end())
      for (const Shape& sh : shapes)
        if (sh.block == it->second.first && sh.gsize == it->second.second) pick = sh;
  }
  if (!pick.block) {
    hipEvent_t e0, e1;
    BCHECK(hipEventCreate(&e0));
    BCHECK(hipEventCreate(&e1));
    BArgs probe = ba;
    probe.maxit_out = ba.maxit_out < 1 ? ba.maxit_out : 1;
    double best = 1e300;
    const double biggest = (double)*std::max_element(work.begin(), work.end()) * npacks;
    double total = 0.0;
    for (long long w : work) total += (double)w * npacks;
    for (const Shape& sh : shapes) {
      probe.gsize = sh.gsize;
      BCHECK(hipEventRecord(e0, stream));
      st = launch_batched(o.prec, probe, sh.block, sh.G, stream);
      if (st != GADI_OK) break;
      BCHECK(hipEventRecord(e1, stream));
      BCHECK(hipEventSynchronize(e1));
      float ms = 0.f;
      BCHECK(hipEventElapsedTime(&ms, e0, e1));
      const double imbalance = std::max(1.0, (biggest / sh.gsize) / (total / sh.G));
      const double est = ms * imbalance;
      if (std::getenv("GADI_DEBUG"))
        std::fprintf(stderr, "gadi: batched tune block %d x group %d (%d blocks): %.3f ms, imbalance %.2f\n",
                     sh.block, sh.gsize, sh.G, ms, imbalance);
      if (est < best) {
        best = est;
        pick = sh;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != GADI_OK) {
      cleanup();
      return st;
    }
    g_batched_shape[key] = {pick.block, pick.gsize};
  }
  ba.gsize = pick.gsize;

  hipEvent_t t0, t1;
  BCHECK(hipEventCreate(&t0));
  BCHECK(hipEventCreate(&t1));
  // progress reports (GADI_PROGRESS=1): finished-unit counts per group in mapped host memory
  unsigned* hdone = nullptr;
  if (const char* ep = std::getenv("GADI_PROGRESS"))
    if (std::atoi(ep) > 0 &&
        hipHostMalloc((void**)&hdone, sizeof(unsigned) * (pick.G / pick.gsize), hipHostMallocMapped) == hipSuccess) {
      for (int q = 0; q < pick.G / pick.gsize; ++q) hdone[q] = 0;
      if (hipHostGetDevicePointer((void**)&ba.done, hdone, 0) != hipSuccess) {
        (void)hipHostFree(hdone);
        hdone = nullptr;
        ba.done = nullptr;
      }
    }
  BCHECK(hipEventRecord(t0, stream));
  st = run_graph(o.prec, ba, pick.block, pick.G, stream, hdone, pick.G / pick.gsize);
  if (hdone) (void)hipHostFree(hdone);
  BCHECK(hipEventRecord(t1, stream));
  BCHECK(hipEventSynchronize(t1));
  float total_ms = 0.f;
  BCHECK(hipEventElapsedTime(&total_ms, t0, t1));
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (st != GADI_OK) {
    cleanup();
    return st;
  }
  int abort_flag = 0;
  BCHECK(hipMemcpy(&abort_flag, dabort, sizeof(int), hipMemcpyDeviceToHost));
  std::vector<DevInfo> hinfo((size_t)nsys * ntrial);
  BCHECK(hipMemcpy(hinfo.data(), dinfo, sizeof(DevInfo) * nsys * ntrial, hipMemcpyDeviceToHost));
  for (int s = 0; s < nsys; ++s)
    if (hsys[s].xoff >= 0)
      BCHECK(hipMemcpy(x[s], dx + hsys[s].xoff, sizeof(double) * hsys[s].n, hipMemcpyDeviceToHost));
  gadi_status worst = abort_flag ? GADI_EBARRIER : GADI_OK;
  for (int u = 0; u < nsys * ntrial; ++u) {
    const DevInfo& r = hinfo[u];
    gadi_solve_info& out = info[u];
    out.status = abort_flag ? GADI_EBARRIER : r.status;
    out.outer_sweeps = r.sweeps;
    out.inner_H = r.inner_h;
    out.inner_S = r.inner_s;
    out.relres = r.relres;
    out.seconds = (double)r.barrier_ticks / tick_hz;  // the unit's (pack's) wall-clock time
    out.alpha = alpha[o.grid_per_system ? u : u % ntrial];
    out.omega = omega[o.grid_per_system ? u : u % ntrial];
    out.fell_back = 0;
    out.barriers = r.barriers;
    out.barrier_seconds = total_ms * 1e-3;  // whole batch: device time of the graph launch
    if (r.status == GADI_EMAXIT && worst == GADI_OK) worst = GADI_EMAXIT;
  }
  cleanup();
#undef BCHECK
  return worst;
}
