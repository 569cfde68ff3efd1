// The persistent solve kernel and its launch, instantiated per precision mode
// in its own translation unit (solve_inst_*.hip) so that the modes compile in
// parallel; solve.hip holds the host side of gadi_ir_solve.
#pragma once

#include "solve_body.h"

namespace gadi {

int num_cus();
// GADI_SOLVE_PATTERN=generic: read the per-slice layout metadata even where
// the uniform offsets allow the mirrored diagonal pattern
bool generic_pattern_forced();

// One large system: persistent cooperative launch, one band of rows per block.
// PW = 0: per-slice layout metadata; PW = 4 or 6: uniformly diagonal-style
// layout with PW offsets per slice (SolveArgs::dia_u), a set symmetric about
// zero; H and S are read from their half layout (SolveArgs::h_half).
template <class Mode, int BLOCK, int FORM, int PW>
__global__ void __launch_bounds__(BLOCK) solve_kernel(SolveArgs a) {
  const long long t_begin = wall_clock64();
  GridRed<BLOCK> red{Grid{a.sync, a.flags, a.part, a.result, gridDim.x, 0ull, a.timeout, 0ll}};
  if (a.barrier != 0) {
    // XCC-hierarchical barrier: every block counts itself in the XCC that runs
    // it; after one relay barrier every block knows its XCC's block count and
    // the XCCs in use
    __shared__ unsigned sh_x[3];
    if (threadIdx.x == 0) {
      const unsigned x = current_xcc();
      __hip_atomic_fetch_add(xcc_line(a.flags, 0, x), 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      sh_x[0] = x;
    }
    bool ok0;
    (void)red.reduce(0.0, 0.0, 0.0, 0.0, ok0);
    if (!ok0) return;
    if (threadIdx.x == 0) {
      unsigned mask = 0;
      for (unsigned i = 0; i < (unsigned)kMaxXcc; ++i)
        if (__hip_atomic_load(xcc_line(a.flags, 0, i), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > 0) mask |= 1u << i;
      sh_x[1] = (unsigned)__hip_atomic_load(xcc_line(a.flags, 0, sh_x[0]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      sh_x[2] = mask;
    }
    __syncthreads();
    red.g.kind = a.barrier;
    red.g.xcc = sh_x[0];
    red.g.xcc_n = sh_x[1];
    red.g.xcc_mask = sh_x[2];
    red.g.h0 = red.g.epoch;  // arrivals are counted from here
    __syncthreads();
  }
  const unsigned lb = logical_block(blockIdx.x, gridDim.x);
  const int t0 = (int)((long long)a.ntiles * lb / gridDim.x);
  const int t1 = (int)((long long)a.ntiles * (lb + 1) / gridDim.x);
  DevInfo r{};
  bool ok;
  if constexpr (PW == 0) {
    // per-slice metadata: a row's loads depend on loaded metadata, one tile at a time
    const PatGeneric pat{Pattern{a.slice_ptr, a.col, a.slice_dia, a.dia_off, a.n - 1}};
    ok = solve_body<Mode, BLOCK, FORM, 1>(a, red, pat, t0, t1, r);
  } else {
    PatDiaSym<PW> pat;
#pragma unroll
    for (int j = 0; j < PW; ++j) pat.off[j] = a.dia_u[j];
    pat.nmax = a.n - 1;
    pat.pad = a.half_pad;
    // 512-thread blocks run 8 waves per compute unit with up to 256 registers
    // each: twice the row tiles in flight per thread of the 1024-thread blocks
    ok = solve_body<Mode, BLOCK, FORM, (BLOCK == 512 ? 2 * Mode::tiles : Mode::tiles)>(a, red, pat, t0, t1, r);
  }
  if (!ok) return;
  // per-block profile: ticks inside barriers and in the whole launch
  if (a.prof && threadIdx.x == 0) {
    a.prof[kProfHead + blockIdx.x] = red.g.wait_ticks;
    a.prof[kProfHead + kMaxBlocks + blockIdx.x] = wall_clock64() - t_begin;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    r.barriers = (long long)red.g.epoch;
    r.barrier_ticks = red.g.wait_ticks;
    *a.info = r;
  }
}

static __global__ void reset_sync_kernel(SyncState* s, unsigned long long* flags, DevInfo* info, long long* prof) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kFlagWords; i += gridDim.x * blockDim.x)
    flags[i] = 0ull;
  if (prof && blockIdx.x == 0 && threadIdx.x < 20) prof[threadIdx.x] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    s->arrive = 0ull;
    s->release = 0ull;
    s->abort = 0;
    info->status = GADI_EBARRIER;
    info->sweeps = 0;
    info->inner_h = 0;
    info->inner_s = 0;
    info->relres = 0.0;
    info->rho0 = 0.0;
    info->barriers = 0;
    info->barrier_ticks = 0;
  }
}

template <class Mode, int BLOCK, int FORM, int PW>
static gadi_status launch_t(System& s, SolveArgs a, int per_cu) {
  int nb = 0;
  GADI_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, solve_kernel<Mode, BLOCK, FORM, PW>, BLOCK, 0));
  if (nb < 1 || per_cu > nb) return GADI_EINVAL;  // not co-resident: not a valid shape
  const int ntiles = s.npad / BLOCK;
  long long G = (long long)per_cu * num_cus();
  if (G > ntiles) G = ntiles;
  if (G > kMaxBlocks) G = kMaxBlocks;
  if (G < 1) G = 1;
  a.ntiles = ntiles;
  hipLaunchKernelGGL(reset_sync_kernel, dim3(32), dim3(1024), 0, s.stream, a.sync, a.flags, a.info, a.prof);
  GADI_HIP_CHECK(hipGetLastError());
  void* kargs[] = {(void*)&a};
  GADI_HIP_CHECK(hipLaunchCooperativeKernel((const void*)solve_kernel<Mode, BLOCK, FORM, PW>, dim3((unsigned)G), dim3(BLOCK),
                                            kargs, 0, s.stream));
  s.last_blocks = (int)G;
  s.last_block_threads = BLOCK;
  return GADI_OK;
}

template <class Mode, int FORM, int PW>
static gadi_status launch_block(System& s, const SolveArgs& a, int block, int per_cu) {
  switch (block) {
    case 512:
      // the precision-study modes are built in one block size only
      if constexpr (Mode::id <= GADI_PREC_FP32_IR || Mode::id == GADI_PREC_FP8_IR)
        return launch_t<Mode, 512, FORM, PW>(s, a, per_cu);
      return GADI_EINVAL;
    case 1024: return launch_t<Mode, 1024, FORM, PW>(s, a, per_cu);
  }
  return GADI_EINVAL;
}

template <class Mode, int FORM>
gadi_status launch_mode(System& s, const SolveArgs& a, int block, int per_cu) {
  const bool half = s.dia_sym && a.h_half && a.s_half && !generic_pattern_forced();
  switch (half ? s.dia_uniform : 0) {
    case 4: return launch_block<Mode, FORM, 4>(s, a, block, per_cu);
    case 6: return launch_block<Mode, FORM, 6>(s, a, block, per_cu);
  }
  return launch_block<Mode, FORM, 0>(s, a, block, per_cu);
}

// one explicit instantiation per mode and inner-solver form (0 Hestenes-Stiefel,
// 1 Chronopoulos-Gear, 2 pipelined CG with Craig's CGNE, 3 Hestenes-Stiefel CG
// with Craig's CGNE), each mode in its own translation unit
#define GADI_DECLARE_MODE(M)                                                          \
  extern template gadi_status launch_mode<M, 0>(System&, const SolveArgs&, int, int); \
  extern template gadi_status launch_mode<M, 1>(System&, const SolveArgs&, int, int); \
  extern template gadi_status launch_mode<M, 2>(System&, const SolveArgs&, int, int); \
  extern template gadi_status launch_mode<M, 3>(System&, const SolveArgs&, int, int);
#define GADI_INSTANTIATE_MODE(M)                                               \
  template gadi_status launch_mode<M, 0>(System&, const SolveArgs&, int, int); \
  template gadi_status launch_mode<M, 1>(System&, const SolveArgs&, int, int); \
  template gadi_status launch_mode<M, 2>(System&, const SolveArgs&, int, int); \
  template gadi_status launch_mode<M, 3>(System&, const SolveArgs&, int, int);

}  // namespace gadi
