// Device helpers shared by the solver kernels: precision modes, conversions,
// the SELL-64 row product, and the device-wide barrier / all-reduce used by
// the persistent launches.
#pragma once

#include "internal.h"

namespace gadi {

// OCP FP8 E4M3 storage: sign, 4 exponent bits (bias 7), 3 mantissa bits; no
// infinities, largest finite 448.
struct e4m3 {
  uint8_t bits;
};

// Precision modes (u_r, u, u_f) of Algorithm 1.  Inner solves (u_r): MT the
// stored value type of H and S, DT that of the diagonal of H, VT the stored
// Krylov vectors, ST the inner
// solution accumulators, RT the stored outer residual, AT the arithmetic.
// Outer loop: XT the stored solution x and its update (u), FT the arithmetic
// of the residual r = b - A x (u_f) and AV the stored values of A it uses.
struct ModeF16 {  // (half, double, double)
  using MT = __half;
  using DT = __half;
  using VT = __half;
  using ST = __half;
  using RT = float;
  using AT = float;
  using XT = double;
  using FT = double;
  using AV = double;
  static constexpr int id = GADI_PREC_FP16_IR;
  static constexpr int tiles = 2;  // tiles per thread with loads in flight together
};
struct ModeF32 {  // (single, double, double)
  using MT = float;
  using DT = float;
  using VT = float;
  using ST = float;
  using RT = float;
  using AT = float;
  using XT = double;
  using FT = double;
  using AV = double;
  static constexpr int id = GADI_PREC_FP32_IR;
  static constexpr int tiles = 2;
};
struct ModeF64 {  // (double, double, double): plain GADI
  using MT = double;
  using DT = double;
  using VT = double;
  using ST = double;
  using RT = double;
  using AT = double;
  using XT = double;
  using FT = double;
  using AV = double;
  static constexpr int id = GADI_PREC_FP64;
  static constexpr int tiles = 1;
};
struct ModeHDS : ModeF16 {  // (half, double, single)
  using FT = float;
  using AV = float;
  static constexpr int id = GADI_PREC_H_D_S;
};
struct ModeHSS : ModeF16 {  // (half, single, single)
  using XT = float;
  using FT = float;
  using AV = float;
  static constexpr int id = GADI_PREC_H_S_S;
};
struct ModeSSS : ModeF32 {  // (single, single, single)
  using XT = float;
  using FT = float;
  using AV = float;
  static constexpr int id = GADI_PREC_S_S_S;
};
struct ModeF8 : ModeF16 {  // FP8 values of H and S, half diagonal and vectors; (double, double) outside
  using MT = e4m3;
  static constexpr int id = GADI_PREC_FP8_IR;
};

template <class AT>
__device__ __forceinline__ AT ld(__half v) {
  return (AT)__half2float(v);
}
template <class AT>
__device__ __forceinline__ AT ld(float v) {
  return (AT)v;
}
template <class AT>
__device__ __forceinline__ AT ld(double v) {
  return (AT)v;
}
// E4M3 -> AT, exact: the exponent and mantissa fields moved into the binary16
// fields (exponent field e -> e, mantissa m -> m << 7) give a binary16 value
// 2^-8 times the E4M3 value, for normal and subnormal codes alike.
template <class AT>
__device__ __forceinline__ AT ld(e4m3 v) {
  const unsigned b = v.bits;
  const unsigned short h = (unsigned short)(((b & 0x80u) << 8) | ((b & 0x7Fu) << 7));
  return (AT)(__half2float(__ushort_as_half(h)) * 256.0f);
}

template <class VT>
struct Cvt;
template <>
struct Cvt<__half> {
  template <class AT>
  static __device__ __forceinline__ __half to(AT v) {
    return __float2half_rn((float)v);
  }
};
template <>
struct Cvt<float> {
  template <class AT>
  static __device__ __forceinline__ float to(AT v) {
    return (float)v;
  }
};
template <>
struct Cvt<double> {
  template <class AT>
  static __device__ __forceinline__ double to(AT v) {
    return (double)v;
  }
};
template <class VT, class AT>
__device__ __forceinline__ VT st(AT v) {
  return Cvt<VT>::template to<AT>(v);
}

// Sparsity pattern shared by A, H and S in the packed layout (internal.h).
struct Pattern {
  const int32_t* sp;    // slice_ptr
  const int32_t* col;   // explicit slices only
  const int32_t* dia;   // offsets per diagonal-style slice, 0 = explicit
  const int32_t* doff;  // [nslices * kDiaMax] column offsets
  int nmax;             // last valid column (n - 1)
};

// Off-diagonal part of one row of an explicit SELL-64 slice:
// sum_j val_ij * fetch(col_ij) over the row's slots in ascending column
// order.  W slots, unrolled so that every index and value load is issued
// before the first gather.
template <int W, class AT, class MT, class F>
__device__ __forceinline__ AT row_sum_w(int k0, const int32_t* __restrict__ col, const MT* __restrict__ val,
                                        F&& fetch) {
  int c[W];
  MT v[W];
#pragma unroll
  for (int j = 0; j < W; ++j) {
    c[j] = col[k0 + j * kSlice];
    v[j] = val[k0 + j * kSlice];
  }
  AT acc = 0;
#pragma unroll
  for (int j = 0; j < W; ++j) acc += ld<AT>(v[j]) * fetch(c[j]);
  return acc;
}

// The same for a diagonal-style slice: the column of slot j is row + offs[j]
// (offs wave-uniform), clamped into [0, nmax] so that phantom entries (value
// 0) never address outside the vector.
template <int W, class AT, class MT, class F>
__device__ __forceinline__ AT row_sum_dia_w(int row, int k0, const int32_t* __restrict__ offs, int nmax,
                                            const MT* __restrict__ val, F&& fetch) {
  int c[W];
  MT v[W];
#pragma unroll
  for (int j = 0; j < W; ++j) {
    v[j] = val[k0 + j * kSlice];
    const int cc = row + offs[j];
    c[j] = cc < 0 ? 0 : (cc > nmax ? nmax : cc);
  }
  AT acc = 0;
#pragma unroll
  for (int j = 0; j < W; ++j) acc += ld<AT>(v[j]) * fetch(c[j]);
  return acc;
}

template <class AT, class MT, class F>
__device__ __forceinline__ AT row_sum(int row, const Pattern& P, const MT* __restrict__ val, F&& fetch) {
  // a wavefront covers exactly one slice, so the slice data are wave-uniform
  const int s = __builtin_amdgcn_readfirstlane(row >> 6);
  const int beg = P.sp[s];
  const int w = (P.sp[s + 1] - beg) >> 6;
  const int k0 = beg + (row & (kSlice - 1));
  if (P.dia[s]) {
    const int32_t* offs = P.doff + (size_t)s * kDiaMax;
    switch (w) {
      case 1: return row_sum_dia_w<1, AT>(row, k0, offs, P.nmax, val, fetch);
      case 2: return row_sum_dia_w<2, AT>(row, k0, offs, P.nmax, val, fetch);
      case 3: return row_sum_dia_w<3, AT>(row, k0, offs, P.nmax, val, fetch);
      case 4: return row_sum_dia_w<4, AT>(row, k0, offs, P.nmax, val, fetch);
      case 5: return row_sum_dia_w<5, AT>(row, k0, offs, P.nmax, val, fetch);
      case 6: return row_sum_dia_w<6, AT>(row, k0, offs, P.nmax, val, fetch);
      default: {
        AT acc = 0;
        for (int j = 0; j < w; ++j) {
          const int cc = row + offs[j];
          acc += ld<AT>(val[k0 + j * kSlice]) * fetch(cc < 0 ? 0 : (cc > P.nmax ? P.nmax : cc));
        }
        return acc;
      }
    }
  }
  const int32_t* __restrict__ col = P.col;
  switch (w) {
    case 0: return AT(0);
    case 1: return row_sum_w<1, AT>(k0, col, val, fetch);
    case 2: return row_sum_w<2, AT>(k0, col, val, fetch);
    case 3: return row_sum_w<3, AT>(k0, col, val, fetch);
    case 4: return row_sum_w<4, AT>(k0, col, val, fetch);
    case 5: return row_sum_w<5, AT>(k0, col, val, fetch);
    case 6: return row_sum_w<6, AT>(k0, col, val, fetch);
    default: {
      AT acc = 0;
      for (int j = 0; j < w; ++j) {
        const int k = k0 + j * kSlice;
        acc += ld<AT>(val[k]) * fetch(col[k]);
      }
      return acc;
    }
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Device-wide all-reduce + barrier for a persistent launch whose blocks are
// all resident (cooperative launch).  Each block contributes three sums and
// one maximum; every block receives the same four results.
//
// Arrival is contention free: a block publishes its partials, then its own
// flag word (one 64-byte line per block).  Block 0 polls all flags with all
// of its threads, combines the partials in block order (a fixed order, so the
// result never depends on arrival order), publishes the result and releases
// the grid through one word.  The agent-scope release before each flag store
// and the acquire after each observed flag make the data written before the
// barrier visible to every block after it.  A wait that exceeds `timeout`
// wall-clock ticks sets the abort flag; the function then returns false in
// every block and the caller must exit.
struct Grid {
  SyncState* sync;
  unsigned long long* flags;
  double* part;
  double* result;
  unsigned nblocks;
  unsigned long long epoch;
  long long timeout;
  long long wait_ticks;  // thread 0: wall-clock ticks this block spent inside barriers
  // XCC-hierarchical variants (kind 1, 2): this block's XCC, the XCC's block
  // count and the XCCs in use
  int kind = 0;
  unsigned xcc = 0, xcc_n = 0, xcc_mask = 0;
  unsigned long long h0 = 0;  // epoch at which the hierarchical barrier took over
};

// Per-XCC line k (0 block count, 1 arrivals, 2 arrival epoch) of XCC x.
__device__ __forceinline__ unsigned long long* xcc_line(unsigned long long* flags, int k, unsigned x) {
  return flags + (size_t)(kMaxBlocks + k * kMaxXcc + (int)x) * kFlagStride;
}

// Word x of the packed arrival epochs (direct variant): one word per XCC in
// consecutive words, so that one wavefront load reads every XCC's epoch.
__device__ __forceinline__ unsigned long long* xcc_epoch_word(unsigned long long* flags, unsigned x) {
  return flags + (size_t)(kMaxBlocks + 3 * kMaxXcc) * kFlagStride + x;
}

// The XCC (L2 domain) that runs the calling wave.
__device__ __forceinline__ unsigned current_xcc() {
  return (unsigned)__builtin_amdgcn_s_getreg((3 << 11) | 20) & 0xFu;  // HW_REG_XCC_ID, bits [3:0]
}

// Waits until this wave's outstanding vector memory operations, stores
// included, have completed (s_waitcnt vmcnt(0)).
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

struct Red4 {
  double v[4];
};

// XCC-hierarchical all-reduce.  A block that arrives has its phase stores in
// its XCC's L2 (every wave waited for them); it publishes its partials and
// counts itself in its XCC's arrival counter.  The XCC's last arriver writes
// the L2 back once for all of the XCC's blocks (one agent-scope release per
// XCC instead of one per block) and publishes the XCC's epoch.  Block 0 waits
// for every XCC in use, combines the partials in block order and releases the
// grid through one word; every block takes its own agent-scope acquire after
// it sees that word.  Timeouts set the abort flag as in the relay barrier.
template <int BLOCK>
static __device__ __forceinline__ Red4 xcc_allreduce(Grid& g, double (*sh)[4], int& sh_abort, long long t_enter,
                                                  bool& ok) {
  constexpr int NW = BLOCK / 64;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  g.epoch += 1;
  const unsigned parity = (unsigned)(g.epoch & 1ull);
  if (tid == 0) {
    double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
    for (int w = 0; w < NW; ++w) {
      t0 += sh[w][0];
      t1 += sh[w][1];
      t2 += sh[w][2];
      t3 = fmax(t3, sh[w][3]);
    }
    double* p = g.part + ((size_t)parity * kMaxBlocks + blockIdx.x) * 4;
    p[0] = t0;
    p[1] = t1;
    p[2] = t2;
    p[3] = t3;
    sh_abort = 0;
    wait_vmem();  // the partials are in the L2
    const unsigned long long target = (g.epoch - g.h0) * (unsigned long long)g.xcc_n;
    const unsigned long long before =
        __hip_atomic_fetch_add(xcc_line(g.flags, 1, g.xcc), 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (before + 1 == target) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(xcc_line(g.flags, 2, g.xcc), g.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (blockIdx.x == 0) {
    const long long t_start = wall_clock64();
    for (;;) {
      int mine = 1;
      if (tid < kMaxXcc && ((g.xcc_mask >> tid) & 1u))
        mine = __hip_atomic_load(xcc_line(g.flags, 2, (unsigned)tid), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >=
               g.epoch;
      if (__syncthreads_and(mine)) break;
      const int expired = (tid == 0) && (wall_clock64() - t_start > g.timeout ||
                                         __hip_atomic_load(&g.sync->abort, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT) != 0);
      if (__syncthreads_or(expired)) {
        if (tid == 0) {
          __hip_atomic_store(&g.sync->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          sh_abort = 1;
        }
        break;
      }
    }
    if (tid == 0) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      wait_vmem();
    }
    __syncthreads();
    double b0 = 0.0, b1 = 0.0, b2 = 0.0, b3 = 0.0;
    for (unsigned k = tid; k < g.nblocks; k += BLOCK) {
      const double* p = g.part + ((size_t)parity * kMaxBlocks + k) * 4;
      b0 += p[0];
      b1 += p[1];
      b2 += p[2];
      b3 = fmax(b3, p[3]);
    }
    b0 = wave_sum(b0);
    b1 = wave_sum(b1);
    b2 = wave_sum(b2);
    b3 = wave_max(b3);
    __syncthreads();
    if (lane == 0) {
      sh[wid][0] = b0;
      sh[wid][1] = b1;
      sh[wid][2] = b2;
      sh[wid][3] = b3;
    }
    __syncthreads();
    if (tid == 0) {
      double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0;
      for (int w = 0; w < NW; ++w) {
        r0 += sh[w][0];
        r1 += sh[w][1];
        r2 += sh[w][2];
        r3 = fmax(r3, sh[w][3]);
      }
      double* r = g.result + parity * 4;
      r[0] = r0;
      r[1] = r1;
      r[2] = r2;
      r[3] = r3;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(&g.sync->release, g.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  } else if (tid == 0) {
    const long long t_start = wall_clock64();
    unsigned spins = 0;
    while (__hip_atomic_load(&g.sync->release, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < g.epoch) {
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 255u) == 0u) {
        if (__hip_atomic_load(&g.sync->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
            wall_clock64() - t_start > g.timeout) {
          __hip_atomic_store(&g.sync->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          sh_abort = 1;
          break;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  Red4 out;
  const double* r = g.result + parity * 4;
  out.v[0] = r[0];
  out.v[1] = r[1];
  out.v[2] = r[2];
  out.v[3] = r[3];
  ok = sh_abort == 0;
  if (tid == 0) g.wait_ticks += wall_clock64() - t_enter;
  __syncthreads();  // shared state is rewritten by the next call
  return out;
}

// XCC-hierarchical all-reduce without a master (kind 2).  Arrival as in
// xcc_allreduce, except that an XCC's last arriver publishes the XCC's epoch
// in the packed word array.  Every block then waits for all XCCs in use with
// one wavefront (a lane per XCC, one load of the packed words per poll), takes
// its agent-scope acquire and combines the partials itself, in block order
// with the same code in every block, so every block computes the same bits.
// This saves the master's relay: its wait, its release of the result and the
// other blocks' wait for that release.  The partials are double-buffered by
// epoch parity: a block writes the buffer of epoch e + 2 only after every
// block has arrived at e + 1, hence finished reading the partials of e.
template <int BLOCK>
static __device__ __forceinline__ Red4 xcc_direct_allreduce(Grid& g, double (*sh)[4], int& sh_abort,
                                                         long long t_enter, bool& ok) {
  constexpr int NW = BLOCK / 64;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  g.epoch += 1;
  const unsigned parity = (unsigned)(g.epoch & 1ull);
  if (tid == 0) {
    double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
    for (int w = 0; w < NW; ++w) {
      t0 += sh[w][0];
      t1 += sh[w][1];
      t2 += sh[w][2];
      t3 = fmax(t3, sh[w][3]);
    }
    double* p = g.part + ((size_t)parity * kMaxBlocks + blockIdx.x) * 4;
    p[0] = t0;
    p[1] = t1;
    p[2] = t2;
    p[3] = t3;
    sh_abort = 0;
    wait_vmem();  // the partials are in the L2
    const unsigned long long target = (g.epoch - g.h0) * (unsigned long long)g.xcc_n;
    const unsigned long long before =
        __hip_atomic_fetch_add(xcc_line(g.flags, 1, g.xcc), 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (before + 1 == target) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(xcc_epoch_word(g.flags, g.xcc), g.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (wid == 0) {
    const long long t_start = wall_clock64();
    const bool watch = lane < kMaxXcc && ((g.xcc_mask >> lane) & 1u);
    unsigned spins = 0;
    for (;;) {
      int mine = 1;
      if (watch)
        mine = __hip_atomic_load(xcc_epoch_word(g.flags, (unsigned)lane), __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT) >= g.epoch;
      if (__all(mine)) break;
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 255u) == 0u) {
        const int expired = wall_clock64() - t_start > g.timeout ||
                            __hip_atomic_load(&g.sync->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        if (__any(expired)) {
          if (lane == 0) {
            __hip_atomic_store(&g.sync->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            sh_abort = 1;
          }
          break;
        }
      }
    }
    if (lane == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  double b0 = 0.0, b1 = 0.0, b2 = 0.0, b3 = 0.0;
  for (unsigned k = tid; k < g.nblocks; k += BLOCK) {
    const double* p = g.part + ((size_t)parity * kMaxBlocks + k) * 4;
    b0 += p[0];
    b1 += p[1];
    b2 += p[2];
    b3 = fmax(b3, p[3]);
  }
  b0 = wave_sum(b0);
  b1 = wave_sum(b1);
  b2 = wave_sum(b2);
  b3 = wave_max(b3);
  // sh (this block's arrival sums) was last read by thread 0 before the barrier above
  if (lane == 0) {
    sh[wid][0] = b0;
    sh[wid][1] = b1;
    sh[wid][2] = b2;
    sh[wid][3] = b3;
  }
  __syncthreads();
  Red4 out;
  out.v[0] = out.v[1] = out.v[2] = out.v[3] = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    out.v[0] += sh[w][0];
    out.v[1] += sh[w][1];
    out.v[2] += sh[w][2];
    out.v[3] = fmax(out.v[3], sh[w][3]);
  }
  ok = sh_abort == 0;
  if (tid == 0) g.wait_ticks += wall_clock64() - t_enter;
  __syncthreads();  // shared state is rewritten by the next call
  return out;
}

template <int BLOCK>
static __device__ __forceinline__ Red4 grid_allreduce_all(Grid& g, double s0, double s1, double s2, double m3,
                                                          bool& ok) {
  constexpr int NW = BLOCK / 64;
  __shared__ double sh[NW][4];
  __shared__ int sh_abort;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const long long t_enter = tid == 0 ? wall_clock64() : 0;
  {
    const double a0 = wave_sum(s0), a1 = wave_sum(s1), a2 = wave_sum(s2), a3 = wave_max(m3);
    if (lane == 0) {
      sh[wid][0] = a0;
      sh[wid][1] = a1;
      sh[wid][2] = a2;
      sh[wid][3] = a3;
    }
  }
  if (g.kind != 0) {
    wait_vmem();  // this wave's phase stores are in the L2 before the block arrives
    __syncthreads();
    return g.kind == 2 ? xcc_direct_allreduce<BLOCK>(g, sh, sh_abort, t_enter, ok)
                       : xcc_allreduce<BLOCK>(g, sh, sh_abort, t_enter, ok);
  }
  __syncthreads();
  g.epoch += 1;
  const unsigned parity = (unsigned)(g.epoch & 1ull);
  if (tid == 0) {
    double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      t0 += sh[w][0];
      t1 += sh[w][1];
      t2 += sh[w][2];
      t3 = fmax(t3, sh[w][3]);
    }
    double* p = g.part + ((size_t)parity * kMaxBlocks + blockIdx.x) * 4;
    p[0] = t0;
    p[1] = t1;
    p[2] = t2;
    p[3] = t3;
    sh_abort = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(g.flags + (size_t)blockIdx.x * kFlagStride, g.epoch, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
  if (blockIdx.x == 0) {
    // master: wait until every block has published this epoch
    const long long t_start = wall_clock64();
    for (;;) {
      int mine = 1;
      for (unsigned k = tid; k < g.nblocks; k += BLOCK)
        if (__hip_atomic_load(g.flags + (size_t)k * kFlagStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
            g.epoch)
          mine = 0;
      if (__syncthreads_and(mine)) break;
      const int expired = (tid == 0) && (wall_clock64() - t_start > g.timeout ||
                                         __hip_atomic_load(&g.sync->abort, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT) != 0);
      if (__syncthreads_or(expired)) {
        if (tid == 0) {
          __hip_atomic_store(&g.sync->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          sh_abort = 1;
        }
        break;
      }
    }
    if (tid == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __syncthreads();
    double b0 = 0.0, b1 = 0.0, b2 = 0.0, b3 = 0.0;
    for (unsigned k = tid; k < g.nblocks; k += BLOCK) {
      const double* p = g.part + ((size_t)parity * kMaxBlocks + k) * 4;
      b0 += p[0];
      b1 += p[1];
      b2 += p[2];
      b3 = fmax(b3, p[3]);
    }
    b0 = wave_sum(b0);
    b1 = wave_sum(b1);
    b2 = wave_sum(b2);
    b3 = wave_max(b3);
    __syncthreads();  // every wave has read sh[] above; reuse it
    if (lane == 0) {
      sh[wid][0] = b0;
      sh[wid][1] = b1;
      sh[wid][2] = b2;
      sh[wid][3] = b3;
    }
    __syncthreads();
    if (tid == 0) {
      double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        r0 += sh[w][0];
        r1 += sh[w][1];
        r2 += sh[w][2];
        r3 = fmax(r3, sh[w][3]);
      }
      double* r = g.result + parity * 4;
      r[0] = r0;
      r[1] = r1;
      r[2] = r2;
      r[3] = r3;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(&g.sync->release, g.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  } else if (tid == 0) {
    const long long t_start = wall_clock64();
    unsigned spins = 0;
    while (__hip_atomic_load(&g.sync->release, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < g.epoch) {
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 255u) == 0u) {
        if (__hip_atomic_load(&g.sync->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
            wall_clock64() - t_start > g.timeout) {
          __hip_atomic_store(&g.sync->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          sh_abort = 1;
          break;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  Red4 out;
  const double* r = g.result + parity * 4;
  out.v[0] = r[0];
  out.v[1] = r[1];
  out.v[2] = r[2];
  out.v[3] = r[3];
  ok = sh_abort == 0;
  if (tid == 0) g.wait_ticks += wall_clock64() - t_enter;
  __syncthreads();  // shared state is rewritten by the next call
  return out;
}

// The relay and the master XCC protocols out of line: the launch-start relay
// barrier and the non-default GADI_BARRIER choices call one copy, so that only
// the default protocol's code sits at every phase end (a kernel inlining all
// three at its ~40 call sites is about 3 times larger than the instruction
// cache).  The grid state goes by value and comes back with the result, so it
// stays in registers.
struct GridRet {
  Red4 out;
  unsigned long long epoch;
  long long wait_ticks;
  bool ok;
};
template <int BLOCK>
static __device__ __noinline__ GridRet grid_allreduce_ool(Grid g, double s0, double s1, double s2, double m3) {
  GridRet r;
  r.out = grid_allreduce_all<BLOCK>(g, s0, s1, s2, m3, r.ok);
  r.epoch = g.epoch;
  r.wait_ticks = g.wait_ticks;
  return r;
}

// Device-wide all-reduce of the solve kernel: the master-free XCC protocol
// inline, the others through grid_allreduce_ool.
template <int BLOCK>
static __device__ __forceinline__ Red4 grid_allreduce(Grid& g, double s0, double s1, double s2, double m3,
                                                      bool& ok) {
  if (g.kind == 2) {
    constexpr int NW = BLOCK / 64;
    __shared__ double sh[NW][4];
    __shared__ int sh_abort;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const long long t_enter = tid == 0 ? wall_clock64() : 0;
    const double a0 = wave_sum(s0), a1 = wave_sum(s1), a2 = wave_sum(s2), a3 = wave_max(m3);
    if (lane == 0) {
      sh[wid][0] = a0;
      sh[wid][1] = a1;
      sh[wid][2] = a2;
      sh[wid][3] = a3;
    }
    wait_vmem();  // this wave's phase stores are in the L2 before the block arrives
    __syncthreads();
    return xcc_direct_allreduce<BLOCK>(g, sh, sh_abort, t_enter, ok);
  }
  const GridRet r = grid_allreduce_ool<BLOCK>(g, s0, s1, s2, m3);
  g.epoch = r.epoch;
  g.wait_ticks = r.wait_ticks;
  ok = r.ok;
  return r.out;
}

// Logical block index: blocks are dealt to the 8 XCDs round-robin, so blocks
// b, b+8, ... share an XCD and its L2.  The remap gives each XCD a contiguous
// run of logical indices, hence a contiguous band of rows.
__device__ __forceinline__ unsigned logical_block(unsigned b, unsigned G) {
  return (G % 8u == 0u) ? (b % 8u) * (G / 8u) + b / 8u : b;
}

}  // namespace gadi
