// GADI-IR solve of one large system: one persistent, cooperatively launched
// kernel runs the whole refinement loop on the device, with device-wide
// all-reduces between phases (device_common.h); no host round trip happens
// inside a solve.  The block size and blocks per compute unit are chosen per
// system by a short timed trial of each candidate (autotune).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "solve_kernel.h"

namespace gadi {

template <class T>
__global__ void convert_kernel(const double* __restrict__ in, T* __restrict__ out, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = (T)in[i];
}

// ------------------------------------------------------------------ host side

static int g_num_cus = 0;
static long long g_wall_rate_khz = 0;

static gadi_status device_props() {
  if (g_num_cus) return GADI_OK;
  int dev = 0;
  GADI_HIP_CHECK(hipGetDevice(&dev));
  int cus = 0, rate = 0;
  GADI_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  GADI_HIP_CHECK(hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, dev));
  g_num_cus = cus > 0 ? cus : 1;
  g_wall_rate_khz = rate > 0 ? rate : 100000;
  return GADI_OK;
}

long long barrier_timeout_ticks() {
  // 20 s of wall clock: far above any legitimate phase, small enough to end a stuck launch
  return g_wall_rate_khz * 1000ll * 20ll;
}

int num_cus() { return g_num_cus; }

// Device-wide barrier of the solve kernel: 1 = XCC-hierarchical (one L2
// writeback per XCC and phase), 0 = relay through block 0 with every block's
// own release; GADI_BARRIER=relay|xcc overrides the default.
bool generic_pattern_forced() {
  const char* e = std::getenv("GADI_SOLVE_PATTERN");
  return e && std::string(e) == "generic";
}

int barrier_kind() {
  const char* e = std::getenv("GADI_BARRIER");
  if (e && std::string(e) == "relay") return 0;
  if (e && std::string(e) == "xcc") return 1;
  if (e && std::string(e) == "direct") return 2;
  return kDefaultBarrier;
}

gadi_status ensure_workspace(System& s) {
  GADI_HIP_CHECK(hipSetDevice(s.device));
  if (s.ws) return GADI_OK;
  // b, x (double) + r, z, w (double-sized) + 8 Krylov vectors (double-sized)
  // + one double staging vector for a single-precision solution
  s.ws_bytes = (size_t)s.npad * sizeof(double) * 14;
  GADI_HIP_CHECK(hipMalloc(&s.ws, s.ws_bytes));
  GADI_HIP_CHECK(hipMemset(s.ws, 0, s.ws_bytes));
  GADI_HIP_CHECK(hipMalloc((void**)&s.sync, sizeof(SyncState)));
  GADI_HIP_CHECK(hipMemset(s.sync, 0, sizeof(SyncState)));
  GADI_HIP_CHECK(hipMalloc((void**)&s.part, sizeof(double) * 2 * kMaxBlocks * 4));
  GADI_HIP_CHECK(hipMalloc((void**)&s.flags, sizeof(unsigned long long) * kFlagWords));
  GADI_HIP_CHECK(hipMalloc((void**)&s.result, sizeof(double) * 8));
  GADI_HIP_CHECK(hipMalloc((void**)&s.info, sizeof(DevInfo)));
  GADI_HIP_CHECK(hipMalloc((void**)&s.prof, sizeof(long long) * kProfLen));
  GADI_HIP_CHECK(hipMemset(s.prof, 0, sizeof(long long) * kProfLen));
  GADI_HIP_CHECK(hipEventCreate(&s.ev0));
  GADI_HIP_CHECK(hipEventCreate(&s.ev1));
  return GADI_OK;
}

static gadi_status ensure_fp32(System& s) {
  if (s.h_off32) return GADI_OK;
  GADI_HIP_CHECK(hipMalloc((void**)&s.h_off32, sizeof(float) * (s.nslots ? s.nslots : 1)));
  GADI_HIP_CHECK(hipMalloc((void**)&s.s_off32, sizeof(float) * (s.nslots ? s.nslots : 1)));
  GADI_HIP_CHECK(hipMalloc((void**)&s.h_diag32, sizeof(float) * s.npad));
  if (s.nslots) {
    hipLaunchKernelGGL(convert_kernel<float>, dim3(1024), dim3(256), 0, s.stream, s.h_off64, s.h_off32, (long long)s.nslots);
    hipLaunchKernelGGL(convert_kernel<float>, dim3(1024), dim3(256), 0, s.stream, s.s_off64, s.s_off32, (long long)s.nslots);
  }
  hipLaunchKernelGGL(convert_kernel<float>, dim3(1024), dim3(256), 0, s.stream, s.h_diag64, s.h_diag32, (long long)s.npad);
  GADI_HIP_CHECK(hipGetLastError());
  return GADI_OK;
}

// fp32 copy of A's values for residuals in single precision (u_f = single)
static gadi_status ensure_a32(System& s) {
  if (s.a_off32) return GADI_OK;
  GADI_HIP_CHECK(hipMalloc((void**)&s.a_off32, sizeof(float) * (s.nslots ? s.nslots : 1)));
  GADI_HIP_CHECK(hipMalloc((void**)&s.a_diag32, sizeof(float) * s.npad));
  if (s.nslots)
    hipLaunchKernelGGL(convert_kernel<float>, dim3(1024), dim3(256), 0, s.stream, s.a_off, s.a_off32, (long long)s.nslots);
  hipLaunchKernelGGL(convert_kernel<float>, dim3(1024), dim3(256), 0, s.stream, s.a_diag, s.a_diag32, (long long)s.npad);
  GADI_HIP_CHECK(hipGetLastError());
  return GADI_OK;
}

__global__ void widen_kernel(const float* __restrict__ in, double* __restrict__ out, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = (double)in[i];
}

__global__ void fill_zero_kernel(double* __restrict__ p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// Half layout of a symmetric uniform pattern (PatDiaSym): slice sl of the
// half array holds, for its 64 rows, the slots of the W/2 positive offsets of
// the full array's slice sl - P; the P leading slices are zero.
template <class T>
__global__ void halve_kernel(const T* __restrict__ full, T* __restrict__ half, long long nhalf, int W, long long P) {
  const int H = W / 2;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nhalf; i += (long long)gridDim.x * blockDim.x) {
    const long long sl = i / (H * kSlice);
    const long long rem = i - sl * H * kSlice;
    const long long q = rem / kSlice, l = rem - q * kSlice;
    half[i] = sl < P ? T(0) : full[(sl - P) * W * kSlice + (H + q) * kSlice + l];
  }
}

template <class T>
static gadi_status halve(System& s, const void* full, void** out, long long nhalf, long long P) {
  GADI_HIP_CHECK(hipMalloc(out, sizeof(T) * (size_t)nhalf));
  hipLaunchKernelGGL(halve_kernel<T>, dim3(1024), dim3(256), 0, s.stream, (const T*)full, (T*)*out, nhalf,
                     s.dia_uniform, P);
  GADI_HIP_CHECK(hipGetLastError());
  return GADI_OK;
}

// The half layout of H and S for value type `kind` (0 fp16, 1 fp32, 2 fp64,
// 3 E4M3) from their full arrays, once per handle and type.
gadi_status ensure_half(System& s, int kind, const void* hfull, const void* sfull) {
  if (!s.dia_sym || s.h_half[kind]) return GADI_OK;
  const long long P = (s.dia_u[s.dia_uniform - 1] + kSlice - 1) / kSlice;
  const long long nhalf = (P + s.nslices) * (long long)(s.dia_uniform / 2) * kSlice;
  s.half_pad = (int)(P * kSlice);
  gadi_status st = GADI_OK;
  void *h = nullptr, *sv = nullptr;
  switch (kind) {
    case 0:
      if ((st = halve<uint16_t>(s, hfull, &h, nhalf, P)) == GADI_OK) st = halve<uint16_t>(s, sfull, &sv, nhalf, P);
      break;
    case 1:
      if ((st = halve<uint32_t>(s, hfull, &h, nhalf, P)) == GADI_OK) st = halve<uint32_t>(s, sfull, &sv, nhalf, P);
      break;
    case 2:
      if ((st = halve<uint64_t>(s, hfull, &h, nhalf, P)) == GADI_OK) st = halve<uint64_t>(s, sfull, &sv, nhalf, P);
      break;
    default:
      if ((st = halve<uint8_t>(s, hfull, &h, nhalf, P)) == GADI_OK) st = halve<uint8_t>(s, sfull, &sv, nhalf, P);
  }
  if (st != GADI_OK) {
    if (h) (void)hipFree(h);
    if (sv) (void)hipFree(sv);
    return st;
  }
  s.h_half[kind] = h;
  s.s_half[kind] = sv;
  return GADI_OK;
}

gadi_status ensure_fp32_public(System& s) { return ensure_fp32(s); }

// E4M3 code of v, rounded to nearest-even in one step from double; `over` is
// set when |v| is beyond 464 (448 plus half its spacing) or not finite.  Within
// the binade [2^E, 2^(E+1)) the spacing is 2^(E-3); the subnormals share the
// spacing 2^-9 of the lowest binade E = -6.  With N = |v| / 2^(E-3) rounded
// (8..16, or 0..16 at E = -6) the code is 8 (E + 6) + N: N = 16 carries into
// the next binade's first code.
__device__ __forceinline__ uint8_t e4m3_rne(double v, bool& over) {
  const unsigned sign = signbit(v) ? 0x80u : 0u;
  const double a = fabs(v);
  if (!(a <= 464.0)) {
    over = true;
    return (uint8_t)(sign | 0x7Eu);
  }
  if (a == 0.0) return (uint8_t)sign;
  int k;
  (void)frexp(a, &k);  // a = f 2^k, f in [1/2, 1)
  int E = k - 1;
  if (E < -6) E = -6;
  const double N = rint(ldexp(a, 3 - E));
  const unsigned code = (unsigned)(8 * (E + 6)) + (unsigned)N;
  return (uint8_t)(sign | (code > 0x7Eu ? 0x7Eu : code));
}

__global__ void encode_e4m3_kernel(const double* __restrict__ in, uint8_t* __restrict__ out, long long n,
                                   unsigned* __restrict__ over) {
  bool o = false;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = e4m3_rne(in[i], o);
  if (o) atomicOr(over, 1u);
}

// E4M3 copies of the off-diagonal values of H and S for the FP8 mode, encoded
// once per handle from the double splitting (synchronises the stream).
static gadi_status ensure_fp8(System& s) {
  if (s.h_off8) return s.fp8_overflow ? GADI_EOVERFLOW16 : GADI_OK;
  const size_t n = s.nslots ? (size_t)s.nslots : 1;
  uint8_t *h8 = nullptr, *s8 = nullptr;
  unsigned* over = nullptr;
  unsigned flag = 0;
  // every exit below frees what this call allocated unless it is kept
  auto encode = [&]() -> gadi_status {
    GADI_HIP_CHECK(hipMalloc((void**)&h8, n));
    GADI_HIP_CHECK(hipMalloc((void**)&s8, n));
    GADI_HIP_CHECK(hipMalloc((void**)&over, sizeof(unsigned)));
    GADI_HIP_CHECK(hipMemsetAsync(over, 0, sizeof(unsigned), s.stream));
    if (s.nslots) {
      hipLaunchKernelGGL(encode_e4m3_kernel, dim3(1024), dim3(256), 0, s.stream, s.h_off64, h8, (long long)s.nslots,
                         over);
      hipLaunchKernelGGL(encode_e4m3_kernel, dim3(1024), dim3(256), 0, s.stream, s.s_off64, s8, (long long)s.nslots,
                         over);
    }
    GADI_HIP_CHECK(hipGetLastError());
    GADI_HIP_CHECK(hipMemcpyAsync(&flag, over, sizeof(unsigned), hipMemcpyDeviceToHost, s.stream));
    GADI_HIP_CHECK(hipStreamSynchronize(s.stream));
    return GADI_OK;
  };
  const gadi_status st = encode();
  if (over) (void)hipFree(over);
  if (st != GADI_OK) {
    if (h8) (void)hipFree(h8);
    if (s8) (void)hipFree(s8);
    return st;
  }
  s.h_off8 = h8;
  s.s_off8 = s8;
  s.fp8_overflow = flag != 0;
  return s.fp8_overflow ? GADI_EOVERFLOW16 : GADI_OK;
}

gadi_status ensure_fp8_public(System& s) { return ensure_fp8(s); }

#define GADI_MODES(X) X(ModeF16) X(ModeF32) X(ModeF64) X(ModeHDS) X(ModeHSS) X(ModeSSS) X(ModeF8)
GADI_MODES(GADI_DECLARE_MODE)

// form: the inner-solver form (0 Hestenes-Stiefel, 1 Chronopoulos-Gear, 2
// pipelined CG with Craig's CGNE, 3 Hestenes-Stiefel CG with Craig's CGNE)
template <int FORM>
static gadi_status launch_prec(System& s, int prec, const SolveArgs& a, int block, int per_cu) {
  switch (prec) {
    case GADI_PREC_FP16_IR: return launch_mode<ModeF16, FORM>(s, a, block, per_cu);
    case GADI_PREC_FP32_IR: return launch_mode<ModeF32, FORM>(s, a, block, per_cu);
    case GADI_PREC_H_D_S: return launch_mode<ModeHDS, FORM>(s, a, block, per_cu);
    case GADI_PREC_H_S_S: return launch_mode<ModeHSS, FORM>(s, a, block, per_cu);
    case GADI_PREC_S_S_S: return launch_mode<ModeSSS, FORM>(s, a, block, per_cu);
    case GADI_PREC_FP8_IR: return launch_mode<ModeF8, FORM>(s, a, block, per_cu);
  }
  return launch_mode<ModeF64, FORM>(s, a, block, per_cu);
}

static gadi_status launch_solve(System& s, int prec, const SolveArgs& a, int block, int per_cu, int form) {
  s.last_form = form;
  switch (form) {
    case 0: return launch_prec<0>(s, prec, a, block, per_cu);
    case 1: return launch_prec<1>(s, prec, a, block, per_cu);
    case 2: return launch_prec<2>(s, prec, a, block, per_cu);
    case 3: return launch_prec<3>(s, prec, a, block, per_cu);
  }
  return GADI_EINVAL;
}

// for the allocation-free entry point (noalloc.hip): the same launch with the
// synchronisation state and vectors the caller's SolveArgs name
gadi_status launch_solve_shape(System& s, int prec, SolveArgs a, int block, int per_cu, int form) {
  gadi_status st = device_props();
  if (st != GADI_OK) return st;
  a.timeout = barrier_timeout_ticks();
  return launch_solve(s, prec, a, block, per_cu, form);
}

double wall_clock_hz() { return (double)g_wall_rate_khz * 1000.0; }

// solution stored in single precision (u = single)
static bool single_solution(int prec) { return prec == GADI_PREC_H_S_S || prec == GADI_PREC_S_S_S; }
// residual in single precision (u_f = single)
static bool single_residual(int prec) {
  return prec == GADI_PREC_H_D_S || prec == GADI_PREC_H_S_S || prec == GADI_PREC_S_S_S;
}

// Autotuner: time three outer sweeps from x = 0 in every candidate (threads
// per block x blocks per compute unit x inner-solver form), after one
// untimed warm-up launch, best of two passes, and keep the lowest time per
// inner step.  Runs once per handle and precision; GADI_SOLVE_BLOCK,
// GADI_BLOCKS_PER_CU and GADI_SOLVE_FORM override it.
static gadi_status tune_solve(System& s, int prec, SolveArgs a, double* dx) {
  if (s.tuned_block[prec]) return GADI_OK;
  const char* eb = std::getenv("GADI_SOLVE_BLOCK");
  const char* ec = std::getenv("GADI_BLOCKS_PER_CU");
  const char* ef = std::getenv("GADI_SOLVE_FORM");
  if (eb || ec || ef) {
    s.tuned_block[prec] = eb ? std::atoi(eb) : 1024;
    s.tuned_per_cu[prec] = ec ? std::atoi(ec) : 1;
    s.tuned_form[prec] = ef ? std::atoi(ef) : 2;
    return GADI_OK;
  }
  // {threads per block, blocks per CU, inner-solver form}
  // (shapes that are not co-resident return EINVAL and are skipped)
  static const int cand[][3] = {{1024, 1, 0}, {1024, 2, 0}, {512, 4, 0}, {512, 2, 0}, {512, 1, 0},
                                {1024, 1, 1}, {1024, 2, 1}, {512, 4, 1}, {512, 2, 1}, {512, 1, 1},
                                {1024, 1, 2}, {1024, 2, 2}, {512, 4, 2}, {512, 2, 2}, {512, 1, 2},
                                {1024, 1, 3}, {1024, 2, 3}, {512, 4, 3}, {512, 2, 3}, {512, 1, 3}};
  a.maxit_out = a.maxit_out < 3 ? a.maxit_out : 3;
  a.hist = nullptr;
  a.hist_cap = 0;
  double best = 1e300;
  int bb = 1024, bc = 1, bf = 0;
  // the first launch also pays code loading and cold caches: run it untimed
  for (int pass = 0; pass < 3; ++pass) {
    for (const auto& c : cand) {
      hipLaunchKernelGGL(fill_zero_kernel, dim3(256), dim3(256), 0, s.stream, dx, (long long)s.npad);
      GADI_HIP_CHECK(hipEventRecord(s.ev0, s.stream));
      gadi_status st = launch_solve(s, prec, a, c[0], c[1], c[2]);
      if (st == GADI_EINVAL) continue;
      if (st != GADI_OK) return st;
      GADI_HIP_CHECK(hipEventRecord(s.ev1, s.stream));
      DevInfo di;
      GADI_HIP_CHECK(hipMemcpyAsync(&di, s.info, sizeof(DevInfo), hipMemcpyDeviceToHost, s.stream));
      GADI_HIP_CHECK(hipStreamSynchronize(s.stream));
      float ms = 0.f;
      GADI_HIP_CHECK(hipEventElapsedTime(&ms, s.ev0, s.ev1));
      // time per inner step (CG + CGNE steps + 4 per sweep) is comparable across variants
      const double steps = (double)(di.inner_h + di.inner_s + 4ll * di.sweeps);
      const double per = ms / (steps > 0 ? steps : 1.0);
      if (pass == 0) break;  // warm-up launch only
      if (std::getenv("GADI_DEBUG"))
        std::fprintf(stderr, "gadi: tune prec %d block %d x %d/CU form %d: %.2f us/step (%lld phases)\n", prec,
                     c[0], c[1], c[2], per * 1e3, (long long)di.barriers);
      if (per < best) {
        best = per;
        bb = c[0];
        bc = c[1];
        bf = c[2];
      }
    }
  }
  s.tuned_block[prec] = bb;
  s.tuned_per_cu[prec] = bc;
  s.tuned_form[prec] = bf;
  return GADI_OK;
}

}  // namespace gadi

using namespace gadi;

extern "C" gadi_status gadi_ir_solve(gadi_handle* h, const double* b, double* x, double alpha, double omega,
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
  if (!h || !b || !x) return GADI_EINVAL;
  if (!(alpha > 0.0) || !std::isfinite(alpha) || !(omega >= 0.0 && omega < 2.0) || !(tol >= 0.0) ||
      !std::isfinite(tol))
    return GADI_EINVAL;
  gadi_options o;
  if (opts) o = *opts;
  else gadi_default_options(&o, GADI_PREC_FP16_IR);
  if (o.prec < GADI_PREC_FP64 || o.prec > GADI_PREC_FP8_IR || !(o.eps_inner > 0.0) || o.eps_inner >= 1.0 ||
      o.maxit_outer < 0 || o.maxit_inner < 1)
    return GADI_EINVAL;
  System& s = h->sys;
  gadi_status st;
  if ((st = device_props()) != GADI_OK) return st;
  if ((st = ensure_workspace(s)) != GADI_OK) return st;
  const bool inner32 = o.prec == GADI_PREC_FP32_IR || o.prec == GADI_PREC_S_S_S;
  if (inner32 && (st = ensure_fp32(s)) != GADI_OK) return st;
  if (single_residual(o.prec) && (st = ensure_a32(s)) != GADI_OK) return st;
  if (o.prec == GADI_PREC_FP8_IR && (st = ensure_fp8(s)) != GADI_OK) {
    if (info) info->status = st;
    return st;
  }
  if (o.record_history) {
    int cap = o.maxit_outer + 1;
    if (cap > s.hist_cap) {
      if (s.hist) (void)hipFree(s.hist);
      s.hist = nullptr;
      s.hist_cap = 0;
      GADI_HIP_CHECK(hipMalloc((void**)&s.hist, sizeof(double) * cap));
      s.hist_cap = cap;
    }
  }
  const size_t np = (size_t)s.npad;
  double* db = (double*)s.ws;
  double* dx = db + np;
  char* vbase = (char*)(dx + np);
  const size_t vbytes = np * sizeof(double);
  const hipMemcpyKind kin = o.on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  const hipMemcpyKind kout = o.on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  GADI_HIP_CHECK(hipMemcpyAsync(db, b, sizeof(double) * s.n, kin, s.stream));

  SolveArgs a{};
  a.n = s.n;
  a.npad = s.npad;
  a.maxit_out = o.maxit_outer;
  a.maxit_in = o.maxit_inner;
  a.hist_cap = o.record_history ? s.hist_cap : 0;
  a.slice_ptr = s.slice_ptr;
  a.col = s.col;
  a.slice_dia = s.slice_dia;
  a.dia_off = s.dia_off;
  for (int j = 0; j < kDiaMax; ++j) a.dia_u[j] = s.dia_u[j];
  a.a_off = single_residual(o.prec) ? (const void*)s.a_off32 : (const void*)s.a_off;
  a.a_diag = single_residual(o.prec) ? (const void*)s.a_diag32 : (const void*)s.a_diag;
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
  a.sync = s.sync;
  a.flags = s.flags;
  a.part = s.part;
  a.result = s.result;
  a.info = s.info;
  a.hist = o.record_history ? s.hist : nullptr;
  a.timeout = barrier_timeout_ticks();
  a.prof = s.prof;
  a.barrier = barrier_kind();
  if (o.prec == GADI_PREC_FP16_IR || o.prec == GADI_PREC_H_D_S || o.prec == GADI_PREC_H_S_S) {
    a.h_off = s.h_off16;
    a.s_off = s.s_off16;
    a.h_diag = s.h_diag16;
  } else if (o.prec == GADI_PREC_FP8_IR) {
    a.h_off = s.h_off8;
    a.s_off = s.s_off8;
    a.h_diag = s.h_diag16;
  } else if (inner32) {
    a.h_off = s.h_off32;
    a.s_off = s.s_off32;
    a.h_diag = s.h_diag32;
  } else {
    a.h_off = s.h_off64;
    a.s_off = s.s_off64;
    a.h_diag = s.h_diag64;
  }
  {
    const int kind = (o.prec == GADI_PREC_FP16_IR || o.prec == GADI_PREC_H_D_S || o.prec == GADI_PREC_H_S_S) ? 0
                     : o.prec == GADI_PREC_FP8_IR                                                      ? 3
                     : inner32                                                                          ? 1
                                                                                                        : 2;
    if ((st = ensure_half(s, kind, a.h_off, a.s_off)) != GADI_OK) return st;
    a.h_half = s.h_half[kind];
    a.s_half = s.s_half[kind];
    a.half_pad = s.half_pad;
  }
  if ((st = tune_solve(s, o.prec, a, dx)) != GADI_OK) return st;
  // a single-precision solution lives in dx as floats; the caller's doubles
  // pass through the staging vector after the Krylov vectors
  double* stage = (double*)(vbase + 11 * vbytes);
  const bool xs = single_solution(o.prec);
  GADI_HIP_CHECK(hipMemcpyAsync(xs ? stage : dx, x, sizeof(double) * s.n, kin, s.stream));
  if (xs) {
    hipLaunchKernelGGL(fill_zero_kernel, dim3(256), dim3(256), 0, s.stream, dx, (long long)s.npad);
    hipLaunchKernelGGL(convert_kernel<float>, dim3(1024), dim3(256), 0, s.stream, stage, (float*)dx, (long long)s.n);
    GADI_HIP_CHECK(hipGetLastError());
  }
  GADI_HIP_CHECK(hipEventRecord(s.ev0, s.stream));
  st = launch_solve(s, o.prec, a, s.tuned_block[o.prec], s.tuned_per_cu[o.prec], s.tuned_form[o.prec]);
  if (st != GADI_OK) return st;
  GADI_HIP_CHECK(hipEventRecord(s.ev1, s.stream));
  if (xs) {
    hipLaunchKernelGGL(widen_kernel, dim3(1024), dim3(256), 0, s.stream, (const float*)dx, stage, (long long)s.n);
    GADI_HIP_CHECK(hipGetLastError());
  }
  GADI_HIP_CHECK(hipMemcpyAsync(x, xs ? stage : dx, sizeof(double) * s.n, kout, s.stream));
  DevInfo di;
  GADI_HIP_CHECK(hipMemcpyAsync(&di, s.info, sizeof(DevInfo), hipMemcpyDeviceToHost, s.stream));
  GADI_HIP_CHECK(hipStreamSynchronize(s.stream));
  float ms = 0.f;
  GADI_HIP_CHECK(hipEventElapsedTime(&ms, s.ev0, s.ev1));
  int abort_flag = 0;
  GADI_HIP_CHECK(hipMemcpy(&abort_flag, &s.sync->abort, sizeof(int), hipMemcpyDeviceToHost));
  gadi_status result = abort_flag ? GADI_EBARRIER : (gadi_status)di.status;
  s.hist_len = o.record_history ? (di.sweeps + 1 < s.hist_cap ? di.sweeps + 1 : s.hist_cap) : 0;
  if (info) {
    info->status = result;
    info->outer_sweeps = di.sweeps;
    info->inner_H = di.inner_h;
    info->inner_S = di.inner_s;
    info->relres = di.relres;
    info->seconds = ms * 1e-3;
    info->barriers = di.barriers;
    info->barrier_seconds = (double)di.barrier_ticks / ((double)g_wall_rate_khz * 1000.0);
  }
  return result;
}

extern "C" int32_t gadi_get_history(gadi_handle* h, double* out, int32_t cap) {
  if (!h || !out || cap <= 0 || !h->sys.hist) return 0;
  int n = h->sys.hist_len < cap ? h->sys.hist_len : cap;
  if (n <= 0) return 0;
  if (hipMemcpy(out, h->sys.hist, sizeof(double) * n, hipMemcpyDeviceToHost) != hipSuccess) return 0;
  return n;
}

extern "C" gadi_status gadi_get_phase_profile(gadi_handle* h, double* seconds, int64_t* counts) {
  if (!h || !seconds || !counts || !h->sys.prof) return GADI_EINVAL;
  long long buf[20];
  GADI_HIP_CHECK(hipMemcpy(buf, h->sys.prof, sizeof(buf), hipMemcpyDeviceToHost));
  for (int i = 0; i < 10; ++i) {
    seconds[i] = (double)buf[i] / ((double)g_wall_rate_khz * 1000.0);
    counts[i] = buf[10 + i];
  }
  return GADI_OK;
}

extern "C" int32_t gadi_solver_blocks(gadi_handle* h, int32_t* threads) {
  if (!h) return 0;
  if (threads) *threads = h->sys.last_block_threads;
  return h->sys.last_blocks;
}

extern "C" int32_t gadi_solver_form(gadi_handle* h) { return h ? h->sys.last_form : -1; }

extern "C" int32_t gadi_get_block_profile(gadi_handle* h, double* wait_seconds, double* total_seconds, int32_t cap) {
  if (!h || !h->sys.prof || h->sys.last_blocks <= 0) return 0;
  const int nb = h->sys.last_blocks < cap ? h->sys.last_blocks : cap;
  if (nb <= 0) return 0;
  std::vector<long long> buf(2 * kMaxBlocks);
  if (hipMemcpy(buf.data(), h->sys.prof + kProfHead, sizeof(long long) * 2 * kMaxBlocks, hipMemcpyDeviceToHost) !=
      hipSuccess)
    return 0;
  const double hz = (double)g_wall_rate_khz * 1000.0;
  for (int i = 0; i < nb; ++i) {
    if (wait_seconds) wait_seconds[i] = (double)buf[i] / hz;
    if (total_seconds) total_seconds[i] = (double)buf[kMaxBlocks + i] / hz;
  }
  return nb;
}

extern "C" int32_t gadi_get_phase_block_profile(gadi_handle* h, double* seconds, int32_t* ids, int32_t max_phases) {
  if (!h || !h->sys.prof || h->sys.last_blocks <= 0 || max_phases <= 0) return 0;
  const int nb = h->sys.last_blocks;
  const int np = max_phases < kPhaseRec ? max_phases : kPhaseRec;
  std::vector<long long> buf((size_t)kPhaseRec * kMaxBlocks + kPhaseRec);
  if (hipMemcpy(buf.data(), h->sys.prof + kProfPhase, sizeof(long long) * buf.size(), hipMemcpyDeviceToHost) !=
      hipSuccess)
    return 0;
  const double hz = (double)g_wall_rate_khz * 1000.0;
  for (int p = 0; p < np; ++p) {
    if (ids) ids[p] = (int32_t)buf[(size_t)kPhaseRec * kMaxBlocks + p];
    if (seconds)
      for (int b = 0; b < nb; ++b) seconds[(size_t)p * nb + b] = (double)buf[(size_t)p * kMaxBlocks + b] / hz;
  }
  return np;
}
