// GADI-IR solve: one persistent, cooperatively launched kernel runs the whole
// refinement loop of Algorithm 1 (Section 2.1) on the device.  Phases are
// separated by device-wide all-reduces (device_common.h); no host round trip
// happens inside a solve.
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
// device-wide reductions and one operator product.
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "device_common.h"

namespace gadi {

struct SolveArgs {
  int n, npad, ntiles, maxit_out, maxit_in, hist_cap;
  const int32_t* slice_ptr;
  const int32_t* col;
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
  void* vr;
  void* vp;
  void* vq;
  void* vt;
  double alpha, omega, tol, eps_h, eps_s;
  SyncState* sync;
  unsigned long long* flags;
  double* part;
  double* result;
  DevInfo* info;
  double* hist;
  long long timeout;
};

// Device-wide reduction into out[4]; leaves the kernel if a barrier timed out.
#define ALLREDUCE(a0, a1, a2, a3)                                              \
  do {                                                                         \
    bool ok_;                                                                  \
    const Red4 r_ = grid_allreduce<kSolveBlock>(g, (a0), (a1), (a2), (a3), ok_); \
    if (!ok_) return;                                                          \
    out[0] = r_.v[0];                                                          \
    out[1] = r_.v[1];                                                          \
    out[2] = r_.v[2];                                                          \
    out[3] = r_.v[3];                                                          \
  } while (0)

static __device__ __forceinline__ int clamp_exp(int e) { return e < -120 ? -120 : (e > 120 ? 120 : e); }

template <class Mode>
__global__ void __launch_bounds__(kSolveBlock) solve_kernel(SolveArgs a) {
  using MT = typename Mode::MT;
  using VT = typename Mode::VT;
  using ST = typename Mode::ST;
  using RT = typename Mode::RT;
  using AT = typename Mode::AT;

  Grid g{a.sync, a.flags, a.part, a.result, gridDim.x, 0ull, a.timeout, 0ll};
  const int tid = threadIdx.x;
  const unsigned lb = logical_block(blockIdx.x, gridDim.x);
  const int t0 = (int)((long long)a.ntiles * lb / gridDim.x);
  const int t1 = (int)((long long)a.ntiles * (lb + 1) / gridDim.x);

  const int32_t* __restrict__ sp = a.slice_ptr;
  const int32_t* __restrict__ col = a.col;
  const MT* __restrict__ hoff = (const MT*)a.h_off;
  const MT* __restrict__ soff = (const MT*)a.s_off;
  const MT* __restrict__ hdiag = (const MT*)a.h_diag;
  RT* __restrict__ r = (RT*)a.r;
  ST* __restrict__ z = (ST*)a.z;
  ST* __restrict__ w = (ST*)a.w;
  VT* __restrict__ vr = (VT*)a.vr;
  VT* __restrict__ vp = (VT*)a.vp;
  VT* __restrict__ vq = (VT*)a.vq;
  VT* __restrict__ vt = (VT*)a.vt;
  double* __restrict__ x = a.x;
  const double* __restrict__ b = a.b;

  const AT alpha = (AT)a.alpha;
  const AT inv_alpha = (AT)(1.0 / a.alpha);
  const AT two_m_omega = (AT)(2.0 - a.omega);
  const double eps_h2 = a.eps_h * a.eps_h;
  const double eps_s2 = a.eps_s * a.eps_s;

  double out[4];
  double rho0 = 0.0, res = 0.0;
  int status = GADI_EMAXIT;
  int sweep = 0;
  long long ih = 0, is = 0;

  for (;;) {
    // ---------------------------------------------------------- a1: residual
    {
      double s0 = 0.0, m3 = 0.0;
      for (int t = t0; t < t1; ++t) {
        const int row = t * kTile + tid;
        const double ax = a.a_diag[row] * x[row] +
                          row_sum<double>(row, sp, col, a.a_off, [&](int c) { return x[c]; });
        const double ri = b[row] - ax;
        r[row] = (RT)ri;
        s0 += ri * ri;
        m3 = fmax(m3, fabs(ri));
      }
      ALLREDUCE(s0, 0.0, 0.0, m3);
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

    // ---------------------------------------------------------- a3: CG on alpha I + H
    int e1;
    (void)frexp(rmax, &e1);
    e1 = clamp_exp(e1);
    const AT sc1 = (AT)ldexp(1.0, -e1);
    double pq, rr, rr0, zmax = 0.0;
    {
      double s0 = 0.0, s1 = 0.0;
      for (int t = t0; t < t1; ++t) {
        const int row = t * kTile + tid;
        const VT pi = st<VT>((AT)r[row] * sc1);
        const AT api = ld<AT>(pi);
        const AT kp = (alpha + ld<AT>(hdiag[row])) * api +
                      row_sum<AT>(row, sp, col, hoff, [&](int c) { return ld<AT>(st<VT>((AT)r[c] * sc1)); });
        const VT qi = st<VT>(kp);
        vr[row] = pi;
        vp[row] = pi;
        vq[row] = qi;
        s0 += (double)api * (double)ld<AT>(qi);
        s1 += (double)api * (double)api;
      }
      ALLREDUCE(s0, s1, 0.0, 0.0);
      pq = out[0];
      rr0 = out[1];
      rr = rr0;
    }
    int it = 0;
    if (rr0 > 0.0) {
      for (;;) {
        if (!(pq > 0.0) || !isfinite(pq)) {
          if (it == 0) status = isfinite(pq) ? GADI_ENOTSPD : (Mode::id == GADI_PREC_FP16_IR ? GADI_EOVERFLOW16 : GADI_EDIVERGED);
          break;
        }
        const AT ak = (AT)(rr / pq);
        double s0 = 0.0, m3 = 0.0;
        for (int t = t0; t < t1; ++t) {
          const int row = t * kTile + tid;
          const AT pi = ld<AT>(vp[row]);
          const ST zi = (it == 0 ? ST(0) : z[row]) + (ST)(ak * pi);
          z[row] = zi;
          const VT ri = st<VT>(ld<AT>(vr[row]) - ak * ld<AT>(vq[row]));
          vr[row] = ri;
          const double dr = (double)ld<AT>(ri);
          s0 += dr * dr;
          m3 = fmax(m3, fabs((double)zi));
        }
        ALLREDUCE(s0, 0.0, 0.0, m3);
        const double rr_new = out[0];
        zmax = out[3];
        ++it;
        if (rr_new <= eps_h2 * rr0 || it >= a.maxit_in || !isfinite(rr_new)) break;
        const AT beta = (AT)(rr_new / rr);
        rr = rr_new;
        s0 = 0.0;
        for (int t = t0; t < t1; ++t) {
          const int row = t * kTile + tid;
          const AT ri = ld<AT>(vr[row]);
          const AT kr = (alpha + ld<AT>(hdiag[row])) * ri +
                        row_sum<AT>(row, sp, col, hoff, [&](int c) { return ld<AT>(vr[c]); });
          const VT pn = st<VT>(ri + beta * ld<AT>(vp[row]));
          const VT qn = st<VT>(kr + beta * ld<AT>(vq[row]));
          vp[row] = pn;
          vq[row] = qn;
          s0 += (double)ld<AT>(pn) * (double)ld<AT>(qn);
        }
        ALLREDUCE(s0, 0.0, 0.0, 0.0);
        pq = out[0];
      }
    }
    ih += it;
    if (status != GADI_EMAXIT) break;  // inner breakdown on the first step
    if (!isfinite(zmax)) {
      status = Mode::id == GADI_PREC_FP16_IR ? GADI_EOVERFLOW16 : GADI_EDIVERGED;
      break;
    }

    // ---------------------------------------------------------- a4/a5: CGNE on I + S/alpha
    int its = 0;
    if (it > 0 && zmax > 0.0) {
      int e2;
      (void)frexp((double)two_m_omega * zmax, &e2);
      e2 = clamp_exp(e2);
      const AT sc2 = (AT)ldexp(1.0, -e2);
      double rrs0;
      {
        double s1 = 0.0;
        for (int t = t0; t < t1; ++t) {
          const int row = t * kTile + tid;
          const VT gi = st<VT>(two_m_omega * (AT)z[row] * sc2);
          const AT tv = inv_alpha * row_sum<AT>(row, sp, col, soff, [&](int c) {
                          return ld<AT>(st<VT>(two_m_omega * (AT)z[c] * sc2));
                        });
          vr[row] = gi;
          vp[row] = gi;
          vt[row] = st<VT>(tv);
          const double dg = (double)ld<AT>(gi);
          s1 += dg * dg;
        }
        ALLREDUCE(0.0, s1, 0.0, 0.0);
        rrs0 = out[1];
      }
      double rrs = rrs0;
      if (rrs0 > 0.0) {
        for (;;) {
          // q = p - (S/alpha) t, with t = (S/alpha) p
          double s0 = 0.0;
          for (int t = t0; t < t1; ++t) {
            const int row = t * kTile + tid;
            const AT pi = ld<AT>(vp[row]);
            const AT qv = pi - inv_alpha * row_sum<AT>(row, sp, col, soff, [&](int c) { return ld<AT>(vt[c]); });
            const VT qi = st<VT>(qv);
            vq[row] = qi;
            s0 += (double)pi * (double)ld<AT>(qi);
          }
          ALLREDUCE(s0, 0.0, 0.0, 0.0);
          const double pqs = out[0];
          if (!(pqs > 0.0) || !isfinite(pqs)) {
            if (its == 0) status = isfinite(pqs) ? GADI_ENOTSPD : (Mode::id == GADI_PREC_FP16_IR ? GADI_EOVERFLOW16 : GADI_EDIVERGED);
            break;
          }
          const AT ak = (AT)(rrs / pqs);
          s0 = 0.0;
          for (int t = t0; t < t1; ++t) {
            const int row = t * kTile + tid;
            const AT pi = ld<AT>(vp[row]);
            w[row] = (its == 0 ? ST(0) : w[row]) + (ST)(ak * pi);
            const VT ri = st<VT>(ld<AT>(vr[row]) - ak * ld<AT>(vq[row]));
            vr[row] = ri;
            const double dr = (double)ld<AT>(ri);
            s0 += dr * dr;
          }
          ALLREDUCE(s0, 0.0, 0.0, 0.0);
          const double rr_new = out[0];
          ++its;
          if (rr_new <= eps_s2 * rrs0 || its >= a.maxit_in || !isfinite(rr_new)) break;
          const AT beta = (AT)(rr_new / rrs);
          rrs = rr_new;
          for (int t = t0; t < t1; ++t) {
            const int row = t * kTile + tid;
            const AT ri = ld<AT>(vr[row]);
            const AT sr = inv_alpha * row_sum<AT>(row, sp, col, soff, [&](int c) { return ld<AT>(vr[c]); });
            vt[row] = st<VT>(sr + beta * ld<AT>(vt[row]));
            vp[row] = st<VT>(ri + beta * ld<AT>(vp[row]));
          }
          ALLREDUCE(0.0, 0.0, 0.0, 0.0);
        }
      }
      is += its;
      if (status != GADI_EMAXIT) break;

      // ---------------------------------------------------------- a6: x += (I - S/alpha) w * 2^(e1+e2)
      if (its > 0) {
        const double unscale = ldexp(1.0, e1 + e2);
        for (int t = t0; t < t1; ++t) {
          const int row = t * kTile + tid;
          const AT ui = (AT)w[row] - inv_alpha * row_sum<AT>(row, sp, col, soff, [&](int c) { return (AT)w[c]; });
          x[row] += (double)ui * unscale;
        }
        ALLREDUCE(0.0, 0.0, 0.0, 0.0);
      }
    }
    ++sweep;
  }

  if (blockIdx.x == 0 && tid == 0) {
    a.info->status = status;
    a.info->sweeps = sweep;
    a.info->inner_h = ih;
    a.info->inner_s = is;
    a.info->relres = res;
    a.info->rho0 = rho0;
    a.info->barriers = (long long)g.epoch;
    a.info->barrier_ticks = g.wait_ticks;
  }
}

__global__ void reset_sync_kernel(SyncState* s, unsigned long long* flags, DevInfo* info) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kMaxBlocks * kFlagStride; i += gridDim.x * blockDim.x)
    flags[i] = 0ull;
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

gadi_status ensure_workspace(System& s) {
  GADI_HIP_CHECK(hipSetDevice(s.device));
  if (s.ws) return GADI_OK;
  // b, x (double) + r, z, w (double-sized) + 4 Krylov vectors (double-sized)
  s.ws_bytes = (size_t)s.npad * sizeof(double) * 9;
  GADI_HIP_CHECK(hipMalloc(&s.ws, s.ws_bytes));
  GADI_HIP_CHECK(hipMemset(s.ws, 0, s.ws_bytes));
  GADI_HIP_CHECK(hipMalloc((void**)&s.sync, sizeof(SyncState)));
  GADI_HIP_CHECK(hipMemset(s.sync, 0, sizeof(SyncState)));
  GADI_HIP_CHECK(hipMalloc((void**)&s.part, sizeof(double) * 2 * kMaxBlocks * 4));
  GADI_HIP_CHECK(hipMalloc((void**)&s.flags, sizeof(unsigned long long) * kMaxBlocks * kFlagStride));
  GADI_HIP_CHECK(hipMalloc((void**)&s.result, sizeof(double) * 8));
  GADI_HIP_CHECK(hipMalloc((void**)&s.info, sizeof(DevInfo)));
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

template <class Mode>
static gadi_status launch_solve(System& s, const SolveArgs& args, int* blocks_out) {
  static int per_cu = 0;
  if (!per_cu) {
    int nb = 0;
    GADI_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, solve_kernel<Mode>, kSolveBlock, 0));
    per_cu = nb > 0 ? nb : 1;
    if (const char* env = std::getenv("GADI_BLOCKS_PER_CU")) {
      int v = std::atoi(env);
      if (v > 0 && v < per_cu) per_cu = v;
    }
  }
  long long G = (long long)per_cu * num_cus();
  if (G > s.npad / kTile) G = s.npad / kTile;
  if (G > kMaxBlocks) G = kMaxBlocks;
  if (G < 1) G = 1;
  *blocks_out = (int)G;
  SolveArgs a = args;
  void* kargs[] = {(void*)&a};
  GADI_HIP_CHECK(hipLaunchCooperativeKernel((const void*)solve_kernel<Mode>, dim3((unsigned)G), dim3(kSolveBlock), kargs, 0,
                                            s.stream));
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
  if (o.prec < GADI_PREC_FP64 || o.prec > GADI_PREC_FP32_IR || !(o.eps_inner > 0.0) || o.eps_inner >= 1.0 ||
      o.maxit_outer < 0 || o.maxit_inner < 1)
    return GADI_EINVAL;
  System& s = h->sys;
  gadi_status st;
  if ((st = device_props()) != GADI_OK) return st;
  if ((st = ensure_workspace(s)) != GADI_OK) return st;
  if (o.prec == GADI_PREC_FP32_IR && (st = ensure_fp32(s)) != GADI_OK) return st;
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
  GADI_HIP_CHECK(hipMemcpyAsync(dx, x, sizeof(double) * s.n, kin, s.stream));

  SolveArgs a{};
  a.n = s.n;
  a.npad = s.npad;
  a.ntiles = s.npad / kTile;
  a.maxit_out = o.maxit_outer;
  a.maxit_in = o.maxit_inner;
  a.hist_cap = o.record_history ? s.hist_cap : 0;
  a.slice_ptr = s.slice_ptr;
  a.col = s.col;
  a.a_off = s.a_off;
  a.a_diag = s.a_diag;
  a.b = db;
  a.x = dx;
  a.r = vbase;
  a.z = vbase + vbytes;
  a.w = vbase + 2 * vbytes;
  a.vr = vbase + 3 * vbytes;
  a.vp = vbase + 4 * vbytes;
  a.vq = vbase + 5 * vbytes;
  a.vt = vbase + 6 * vbytes;
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
  if (o.prec == GADI_PREC_FP16_IR) {
    a.h_off = s.h_off16;
    a.s_off = s.s_off16;
    a.h_diag = s.h_diag16;
  } else if (o.prec == GADI_PREC_FP32_IR) {
    a.h_off = s.h_off32;
    a.s_off = s.s_off32;
    a.h_diag = s.h_diag32;
  } else {
    a.h_off = s.h_off64;
    a.s_off = s.s_off64;
    a.h_diag = s.h_diag64;
  }
  hipLaunchKernelGGL(reset_sync_kernel, dim3(32), dim3(1024), 0, s.stream, s.sync, s.flags, s.info);
  GADI_HIP_CHECK(hipGetLastError());
  GADI_HIP_CHECK(hipEventRecord(s.ev0, s.stream));
  int blocks = 0;
  if (o.prec == GADI_PREC_FP16_IR) st = launch_solve<ModeF16>(s, a, &blocks);
  else if (o.prec == GADI_PREC_FP32_IR) st = launch_solve<ModeF32>(s, a, &blocks);
  else st = launch_solve<ModeF64>(s, a, &blocks);
  if (st != GADI_OK) return st;
  GADI_HIP_CHECK(hipEventRecord(s.ev1, s.stream));
  GADI_HIP_CHECK(hipMemcpyAsync(x, dx, sizeof(double) * s.n, kout, s.stream));
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

extern "C" int32_t gadi_solver_blocks(gadi_handle* h) {
  if (!h || device_props() != GADI_OK) return 0;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, solve_kernel<ModeF16>, kSolveBlock, 0) != hipSuccess) return 0;
  long long G = (long long)nb * num_cus();
  if (G > h->sys.npad / kTile) G = h->sys.npad / kTile;
  if (G > kMaxBlocks) G = kMaxBlocks;
  return (int32_t)(G < 1 ? 1 : G);
}
