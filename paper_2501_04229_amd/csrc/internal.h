// Internal types of libgadi: the device layout of one system and the solver
// workspace.  Not part of the public ABI (include/gadi.h).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "gadi.h"

namespace gadi {

// Rows per SELL slice: one row per lane of a 64-wide wavefront.
constexpr int kSlice = 64;
// Threads (= rows) per block of the one-shot product kernels.
constexpr int kRowBlock = 256;
// Threads per block of the persistent solve kernels: 16 wavefronts, one block
// per compute unit; a block step covers kTile = kSolveBlock rows (16 slices).
constexpr int kSolveBlock = 1024;
constexpr int kTile = kSolveBlock;
// Row counts are padded to a whole number of solve tiles.
constexpr int kPadRows = kTile;
// Upper bound on blocks of any persistent launch (sizes the barrier buffers).
constexpr int kMaxBlocks = 4096;
// Stride between per-block arrival flags (one 64-byte line each).
constexpr int kFlagStride = 8;
// The XCC-hierarchical barrier keeps per-XCC lines after the per-block flags:
// line kMaxBlocks + k * kMaxXcc + x holds, for XCC x, k = 0 its block count,
// 1 its arrival count, 2 its arrival epoch; the direct variant packs the
// arrival epochs of all XCCs into the two lines after those (one word each).
constexpr int kMaxXcc = 16;
constexpr int kFlagWords = (kMaxBlocks + 3 * kMaxXcc) * kFlagStride + kMaxXcc;
// barrier of the solve kernel unless GADI_BARRIER says otherwise (0 relay, 1
// XCC-hierarchical with a master, 2 XCC-hierarchical without one)
constexpr int kDefaultBarrier = 2;
// Per-phase profile of block 0 (ticks [10], counts [10]), then per block the
// ticks inside barriers [kMaxBlocks] and in the whole launch [kMaxBlocks].
constexpr int kProfHead = 20;
// ... then each block's ticks of each of the first kPhaseRec phases
// [kPhaseRec][kMaxBlocks] and the phases' ids [kPhaseRec].
constexpr int kPhaseRec = 96;
constexpr int kProfPhase = kProfHead + 2 * 4096;
constexpr int kProfPhaseId = kProfPhase + kPhaseRec * 4096;
constexpr int kProfLen = kProfPhaseId + kPhaseRec;
// Largest number of distinct column offsets of a diagonal-style slice.
constexpr int kDiaMax = 8;
// largest system: its padded double vectors stay below 4 GiB
constexpr int kMaxRows = (1 << 29) - kPadRows;

#define GADI_HIP_CHECK(expr)                                \
  do {                                                      \
    hipError_t e_ = (expr);                                 \
    if (e_ != hipSuccess) return fail_hip(e_, #expr, __FILE__, __LINE__); \
  } while (0)

gadi_status fail_hip(hipError_t e, const char* what, const char* file, int line);

// Barrier / reduction state of a persistent launch (device memory).
struct SyncState {
  unsigned long long arrive;   // monotone arrival count
  unsigned long long release;  // epoch released by the last arriving block
  int abort;                   // set when a barrier wait timed out
  int pad[5];
};

// Result record written by the solve kernel.
struct DevInfo {
  int status;
  int sweeps;
  long long inner_h;
  long long inner_s;
  double relres;
  double rho0;
  long long barriers;
  long long barrier_ticks;
};

// One system in device layout.
//   Off-diagonal entries of the union pattern of A and A^T are packed as
//   SELL-64: slice s covers rows [64 s, 64 s + 64); its entries start at
//   slice_ptr[s]; slot j of row (64 s + l) is element slice_ptr[s] + 64 j + l.
//   The slice width is (slice_ptr[s+1] - slice_ptr[s]) / 64.  In an explicit
//   slice, padding slots hold col = row and value 0.  A diagonal-style slice
//   (slice_dia[s] > 0) has one slot per column offset dia_off[s][j]: slot j of
//   row i is the entry (i, i + dia_off[s][j]), value 0 where the row has no
//   such entry; its column indices are implied and never read.  Diagonals are
//   stored densely.
struct System {
  int n = 0;       // rows
  int npad = 0;    // rows rounded up to a tile
  int nslices = 0;
  int64_t nnz_a = 0;      // stored entries of A
  int64_t nnz_off = 0;    // off-diagonal entries of the union pattern
  int64_t nslots = 0;     // SELL slots including padding
  int max_width = 0;
  int device = 0;
  hipStream_t stream = nullptr;

  int64_t dia_slices = 0;
  int64_t dia_slots = 0;         // slots of diagonal-style slices
  int64_t explicit_entries = 0;  // structural entries in explicit slices
  int32_t* slice_dia = nullptr;  // [nslices]: number of offsets of a diagonal-style slice, 0 = explicit
  int32_t* dia_off = nullptr;    // [nslices * kDiaMax]: ascending column offsets col - row
  // > 0: every slice is diagonal-style with these same dia_uniform offsets
  int dia_uniform = 0;
  int32_t dia_u[kDiaMax] = {0, 0, 0, 0, 0, 0, 0, 0};
  // the uniform offsets are symmetric about zero (dia_u[k] = -dia_u[W-1-k])
  bool dia_sym = false;
  // H and S in the half layout of a symmetric uniform pattern, per value type
  // (0 fp16, 1 fp32, 2 fp64, 3 E4M3): per slice only the slots of the positive
  // offsets, with half_pad zero rows in front of row 0; built on first use
  void* h_half[4] = {nullptr, nullptr, nullptr, nullptr};
  void* s_half[4] = {nullptr, nullptr, nullptr, nullptr};
  int half_pad = 0;
  int32_t* slice_ptr = nullptr;  // [nslices + 1]
  int32_t* col = nullptr;        // [nslots]
  double* a_off = nullptr;       // [nslots] A values on the union pattern
  double* a_diag = nullptr;      // [npad]
  double* h_off64 = nullptr;     // [nslots] H = (A + A^T)/2
  double* s_off64 = nullptr;     // [nslots] S = (A - A^T)/2
  double* h_diag64 = nullptr;    // [npad]
  __half* h_off16 = nullptr;
  __half* s_off16 = nullptr;
  __half* h_diag16 = nullptr;
  uint8_t* h_off8 = nullptr;     // [nslots] E4M3 codes of H and S (FP8 mode), encoded on first use
  uint8_t* s_off8 = nullptr;
  int fp8_overflow = 0;          // an entry of H or S is beyond the E4M3 range
  float* h_off32 = nullptr;
  float* s_off32 = nullptr;
  float* h_diag32 = nullptr;
  float* a_off32 = nullptr;   // fp32 copy of A for single-precision residuals
  float* a_diag32 = nullptr;

  // solver workspace (lazily sized for the widest precision)
  void* ws = nullptr;
  size_t ws_bytes = 0;
  double* hist = nullptr;
  int hist_cap = 0;
  int hist_len = 0;
  SyncState* sync = nullptr;
  unsigned long long* flags = nullptr;  // [kMaxBlocks * kFlagStride]
  double* part = nullptr;    // [2][kMaxBlocks][4]
  double* result = nullptr;  // [2][4]
  DevInfo* info = nullptr;
  long long* prof = nullptr;  // [kProfLen] per-phase and per-block profile of the last solve
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // launch shape of the solve kernel per precision mode, chosen by the autotuner
  int tuned_block[7] = {0, 0, 0, 0, 0, 0, 0};
  int tuned_per_cu[7] = {0, 0, 0, 0, 0, 0, 0};
  int tuned_form[7] = {0, 0, 0, 0, 0, 0, 0};  // inner-solver form (solve_body.h)
  int last_blocks = 0;
  int last_form = -1;
  int last_block_threads = 0;
};

}  // namespace gadi

struct gadi_handle {
  gadi::System sys;
};

namespace gadi {
gadi_status ensure_workspace(System& s);
void free_system(System& s);
}  // namespace gadi
