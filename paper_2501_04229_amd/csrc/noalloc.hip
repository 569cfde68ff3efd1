// Allocation-free GADI-IR solve, for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc).  The solver's workspace -- padded copies of b and x, the
// Krylov vectors and the barrier / reduction state of the persistent launch --
// lives in one file-scope device array, `scratch`, instead of the handle's
// lazily allocated workspace.  Every call on a device shares that device's
// array: calls that overlap on one device race, and each call clears what must
// start at zero.
#include <mutex>

#include "solve_body.h"

namespace gadi {

gadi_status launch_solve_shape(System& s, int prec, SolveArgs a, int block, int per_cu, int form);
int barrier_kind();
double wall_clock_hz();

// 1 MiB of barrier / reduction state (about 0.53 MiB used), then 13 double-sized vectors of the
// padded length: the largest padded system is (256 MiB - 1 MiB) / 104 bytes
// per row = 2,573,753 rows (a 128^3 grid is 2,097,152).
constexpr size_t kScratchBytes = size_t(256) << 20;
constexpr size_t kCtrlBytes = size_t(1) << 20;
constexpr size_t kVecsPerRow = 13;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch[kMaxDevices];

// The device address of `scratch` on device `dev` (current): each device holds
// its own copy of the array, looked up once per device and kept.
static gadi_status scratch_base(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return GADI_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    GADI_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch[dev] = p;
  }
  *out = (unsigned char*)g_scratch[dev];
  return GADI_OK;
}

__global__ void noalloc_clear_kernel(double* __restrict__ p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

}  // namespace gadi

using namespace gadi;

extern "C" gadi_status gadi_ir_solve_noalloc(gadi_handle* h, const double* b, double* x, double alpha,
                                             double omega, double tol, const gadi_options* opts,
                                             gadi_solve_info* info) {
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
  if (!h || !b || !x) return GADI_EINVAL;
  if (!(alpha > 0.0) || !std::isfinite(alpha) || !(omega >= 0.0 && omega < 2.0) || !(tol >= 0.0) ||
      !std::isfinite(tol))
    return GADI_EINVAL;
  gadi_options o;
  if (opts) {
    o = *opts;
  } else {
    gadi_default_options(&o, GADI_PREC_FP16_IR);
    o.on_device = 1;
  }
  // device vectors only, no history, and the modes whose operators gadi_setup stores
  if (!o.on_device || o.record_history || (o.prec != GADI_PREC_FP16_IR && o.prec != GADI_PREC_FP64) ||
      !(o.eps_inner > 0.0) || o.eps_inner >= 1.0 || o.maxit_outer < 0 || o.maxit_inner < 1)
    return GADI_EINVAL;
  System& s = h->sys;
  const size_t np = (size_t)s.npad;
  if (kCtrlBytes + kVecsPerRow * np * sizeof(double) > kScratchBytes) {
    if (info) info->status = GADI_ENOMEM;
    return GADI_ENOMEM;
  }
  GADI_HIP_CHECK(hipSetDevice(s.device));
  unsigned char* base = nullptr;
  gadi_status st = scratch_base(s.device, &base);
  if (st != GADI_OK) return st;

  SyncState* sync = (SyncState*)base;
  unsigned long long* flags = (unsigned long long*)(base + 256);
  double* part = (double*)(flags + (size_t)kFlagWords);
  double* result = part + 2 * kMaxBlocks * 4;
  DevInfo* dinfo = (DevInfo*)(result + 8);
  double* db = (double*)(base + kCtrlBytes);
  double* dx = db + np;
  char* vbase = (char*)(dx + np);
  const size_t vbytes = np * sizeof(double);

  // every vector (b and x with their zero padding, the Krylov workspace) starts at zero
  hipLaunchKernelGGL(noalloc_clear_kernel, dim3(1024), dim3(256), 0, s.stream, db, (long long)(kVecsPerRow * np));
  GADI_HIP_CHECK(hipGetLastError());
  GADI_HIP_CHECK(hipMemcpyAsync(db, b, sizeof(double) * s.n, hipMemcpyDeviceToDevice, s.stream));
  GADI_HIP_CHECK(hipMemcpyAsync(dx, x, sizeof(double) * s.n, hipMemcpyDeviceToDevice, s.stream));

  SolveArgs a{};
  a.n = s.n;
  a.npad = s.npad;
  a.maxit_out = o.maxit_outer;
  a.maxit_in = o.maxit_inner;
  a.hist_cap = 0;
  a.slice_ptr = s.slice_ptr;
  a.col = s.col;
  a.slice_dia = s.slice_dia;
  a.dia_off = s.dia_off;
  for (int j = 0; j < kDiaMax; ++j) a.dia_u[j] = s.dia_u[j];
  a.a_off = s.a_off;
  a.a_diag = s.a_diag;
  a.b = db;
  a.x = dx;
  a.r = vbase;
  a.z = vbase + vbytes;
  a.w = vbase + 2 * vbytes;
  for (int v = 0; v < 8; ++v) a.v[v] = vbase + (3 + v) * vbytes;
  a.alpha = alpha;
  a.omega = omega;
  a.tol = tol;
  a.eps_h = o.eps_inner;
  a.eps_s = o.eps_inner;
  a.sync = sync;
  a.flags = flags;
  a.part = part;
  a.result = result;
  a.info = dinfo;
  a.hist = nullptr;
  a.prof = nullptr;
  a.barrier = barrier_kind();
  if (o.prec == GADI_PREC_FP16_IR) {
    a.h_off = s.h_off16;
    a.s_off = s.s_off16;
    a.h_diag = s.h_diag16;
  } else {
    a.h_off = s.h_off64;
    a.s_off = s.s_off64;
    a.h_diag = s.h_diag64;
  }
  // the half layout of H and S if a gadi_ir_solve has built it for this
  // precision, else the full layout through the generic pattern
  {
    const int kind = o.prec == GADI_PREC_FP16_IR ? 0 : 2;
    a.h_half = s.h_half[kind];
    a.s_half = s.s_half[kind];
    a.half_pad = s.half_pad;
  }
  // the launch shape the autotuner chose for this handle and precision (a
  // gadi_ir_solve call tunes it), else one 1024-thread block per compute unit
  // with the pipelined CG and Craig's CGNE
  const int p = o.prec;
  const int block = s.tuned_block[p] ? s.tuned_block[p] : 1024;
  const int per_cu = s.tuned_block[p] ? s.tuned_per_cu[p] : 1;
  const int form = s.tuned_block[p] ? s.tuned_form[p] : 2;
  if ((st = launch_solve_shape(s, p, a, block, per_cu, form)) != GADI_OK) return st;
  GADI_HIP_CHECK(hipMemcpyAsync(x, dx, sizeof(double) * s.n, hipMemcpyDeviceToDevice, s.stream));
  DevInfo di;
  int abort_flag = 0;
  GADI_HIP_CHECK(hipMemcpyAsync(&di, dinfo, sizeof(DevInfo), hipMemcpyDeviceToHost, s.stream));
  GADI_HIP_CHECK(hipMemcpyAsync(&abort_flag, &sync->abort, sizeof(int), hipMemcpyDeviceToHost, s.stream));
  GADI_HIP_CHECK(hipStreamSynchronize(s.stream));
  const gadi_status result_st = abort_flag ? GADI_EBARRIER : (gadi_status)di.status;
  if (info) {
    info->status = result_st;
    info->outer_sweeps = di.sweeps;
    info->inner_H = di.inner_h;
    info->inner_S = di.inner_s;
    info->relres = di.relres;
    info->barriers = di.barriers;
    info->barrier_seconds = (double)di.barrier_ticks / wall_clock_hz();
  }
  return result_st;
}
