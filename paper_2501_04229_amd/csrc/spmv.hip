// Stand-alone operator products on the packed SELL-64 layout (kernel-level
// parity checks and bandwidth measurement) and the Gershgorin feature pass.
#include <cmath>
#include <vector>

#include "solve_body.h"

namespace gadi {

gadi_status ensure_fp8_public(System& s);
gadi_status ensure_half(System& s, int kind, const void* hfull, const void* sfull);

// The products run the solver's row loop (solve_body.h): every load of U
// tiles of BLOCK rows is issued before their arithmetic, under the same
// pattern policies (uniform diagonal layout: offsets in scalar registers).
// A block owns U consecutive tiles (an XCD-contiguous remap of the blocks,
// as in the solver, measured slower here at 256^3).  x has the caller's
// length n: rows past n read x at row n - 1 (an unconditional load, so no
// branch drains the loads in flight) and write no y.
// threads per block: 512 for the half-precision products, 256 for the double
// product of A (each measured best at 256^3)
constexpr int kSpmvBlock16 = 512;
constexpr int kSpmvBlock64 = 256;

// y = A x in double (the residual's operator, step 1 of Algorithm 1)
template <int U, class Pat>
__global__ void __launch_bounds__(kSpmvBlock64) spmv_a64_kernel(Pat pat, const double* __restrict__ off,
                                                             const double* __restrict__ diag,
                                                             const double* __restrict__ x, double* __restrict__ y,
                                                             int n, int ntiles) {
  const int t0 = blockIdx.x * U, t1 = t0 + U < ntiles ? t0 + U : ntiles;
  auto gx = [&](unsigned c) { return at(x, c); };
  for_rows<kSpmvBlock64, U>(
      t0, t1,
      [&](unsigned row) {
        struct {
          double d, xr;
          decltype(pat.gather(0u, off, gx)) g;
        } l{at(diag, row), at(x, row < (unsigned)n ? row : (unsigned)n - 1u), pat.gather(row, off, gx)};
        return l;
      },
      [&](const auto& l) { return l.d * l.xr + pat.template dot<double>(l.g, [](double v) { return v; }); },
      [&](unsigned row, double v) {
        if (row < (unsigned)n) at(y, row) = v;
      });
}

// y = (alpha I + H) x: off-diagonal values (OV: a pointer to MT, or H's half
// layout under PatDiaSym), diagonal and vectors VT, arithmetic in AT
template <int U, class Pat, class OV, class VT, class AT>
__global__ void __launch_bounds__(kSpmvBlock16) spmv_h_kernel(Pat pat, OV off,
                                                           const VT* __restrict__ diag, const VT* __restrict__ x,
                                                           VT* __restrict__ y, AT alpha, int n, int ntiles) {
  const int t0 = blockIdx.x * U, t1 = t0 + U < ntiles ? t0 + U : ntiles;
  auto gx = [&](unsigned c) { return at(x, c); };
  for_rows<kSpmvBlock16, U>(
      t0, t1,
      [&](unsigned row) {
        struct {
          VT d, xr;
          decltype(pat.gather(0u, off, gx)) g;
        } l{at(diag, row), at(x, row < (unsigned)n ? row : (unsigned)n - 1u), pat.gather(row, off, gx)};
        return l;
      },
      [&](const auto& l) {
        return (alpha + ld<AT>(l.d)) * ld<AT>(l.xr) + pat.template dot<AT>(l.g, [](VT v) { return ld<AT>(v); });
      },
      [&](unsigned row, AT v) {
        if (row < (unsigned)n) at(y, row) = st<VT>(v);
      });
}

// y = (I + S / alpha) x, half in/out, float arithmetic (OV as above)
template <int U, class Pat, class OV>
__global__ void __launch_bounds__(kSpmvBlock16) spmv_s16_kernel(Pat pat, OV off,
                                                             const __half* __restrict__ x, __half* __restrict__ y,
                                                             float inv_alpha, int n, int ntiles) {
  const int t0 = blockIdx.x * U, t1 = t0 + U < ntiles ? t0 + U : ntiles;
  auto gx = [&](unsigned c) { return at(x, c); };
  for_rows<kSpmvBlock16, U>(
      t0, t1,
      [&](unsigned row) {
        struct {
          __half xr;
          decltype(pat.gather(0u, off, gx)) g;
        } l{at(x, row < (unsigned)n ? row : (unsigned)n - 1u), pat.gather(row, off, gx)};
        return l;
      },
      [&](const auto& l) {
        return __half2float(l.xr) + inv_alpha * pat.template dot<float>(l.g, [](__half v) { return __half2float(v); });
      },
      [&](unsigned row, float v) {
        if (row < (unsigned)n) at(y, row) = __float2half_rn(v);
      });
}

// Per-block Gershgorin extrema: [min(H_ii - R^H_i), max(H_ii + R^H_i), max R^S_i, min R^S_i]
__global__ void __launch_bounds__(kRowBlock) gershgorin_kernel(const int32_t* __restrict__ sp, const int32_t* __restrict__ col,
    const int32_t* __restrict__ dia, const int32_t* __restrict__ doff,
                                                             const double* __restrict__ hoff, const double* __restrict__ soff,
                                                             const double* __restrict__ hdiag, int n, double* __restrict__ out) {
  __shared__ double sh[4][4];
  const int row = blockIdx.x * kRowBlock + threadIdx.x;
  const int s = __builtin_amdgcn_readfirstlane(row >> 6);
  const int beg = sp[s];
  const int w = (sp[s + 1] - beg) >> 6;
  double rh = 0.0, rs = 0.0;
  for (int j = 0; j < w; ++j) {
    const int k = beg + j * kSlice + (row & (kSlice - 1));
    rh += fabs(hoff[k]);
    rs += fabs(soff[k]);
  }
  const bool valid = row < n;
  const double d = hdiag[row];
  double v0 = valid ? d - rh : INFINITY, v1 = valid ? d + rh : -INFINITY;
  double v2 = valid ? rs : -INFINITY, v3 = valid ? rs : INFINITY;
  for (int o = 32; o > 0; o >>= 1) {
    v0 = fmin(v0, __shfl_xor(v0, o, 64));
    v1 = fmax(v1, __shfl_xor(v1, o, 64));
    v2 = fmax(v2, __shfl_xor(v2, o, 64));
    v3 = fmin(v3, __shfl_xor(v3, o, 64));
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    sh[wid][0] = v0;
    sh[wid][1] = v1;
    sh[wid][2] = v2;
    sh[wid][3] = v3;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double* o = out + (size_t)blockIdx.x * 4;
    o[0] = fmin(fmin(sh[0][0], sh[1][0]), fmin(sh[2][0], sh[3][0]));
    o[1] = fmax(fmax(sh[0][1], sh[1][1]), fmax(sh[2][1], sh[3][1]));
    o[2] = fmax(fmax(sh[0][2], sh[1][2]), fmax(sh[2][2], sh[3][2]));
    o[3] = fmin(fmin(sh[0][3], sh[1][3]), fmin(sh[2][3], sh[3][3]));
  }
}

}  // namespace gadi

using namespace gadi;

// U16 / U64: tiles per block of the half and double products (4 and 2 on the
// uniform layout: measured best at 256^3).  H and S go
// through pat.mirror: their half layout under PatDiaSym, the full one otherwise.
template <int U16, int U64, class Pat>
static void launch_products(System& s, const Pat& pat, int which, double alpha, const void* x, void* y) {
  const int nt16 = s.npad / kSpmvBlock16, nt64 = s.npad / kSpmvBlock64;
  const dim3 g16((nt16 + U16 - 1) / U16), g64((nt64 + U64 - 1) / U64), b16(kSpmvBlock16), b64(kSpmvBlock64);
  switch (which) {
    case 0:
      hipLaunchKernelGGL((spmv_a64_kernel<U64, Pat>), g64, b64, 0, s.stream, pat, s.a_off, s.a_diag,
                         (const double*)x, (double*)y, s.n, nt64);
      break;
    case 1: {
      const auto hv = pat.template mirror<false>((const __half*)s.h_off16, (const __half*)s.h_half[0]);
      hipLaunchKernelGGL((spmv_h_kernel<U16, Pat, decltype(hv), __half, float>), g16, b16, 0, s.stream, pat, hv,
                         s.h_diag16, (const __half*)x, (__half*)y, (float)alpha, s.n, nt16);
      break;
    }
    case 2: {
      const auto sv = pat.template mirror<true>((const __half*)s.s_off16, (const __half*)s.s_half[0]);
      hipLaunchKernelGGL((spmv_s16_kernel<U16, Pat, decltype(sv)>), g16, b16, 0, s.stream, pat, sv,
                         (const __half*)x, (__half*)y, (float)(1.0 / alpha), s.n, nt16);
      break;
    }
    case 3: {
      const auto hv = pat.template mirror<false>((const double*)s.h_off64, (const double*)s.h_half[2]);
      // the double H product runs the 512-thread kernel with the double tiling
      hipLaunchKernelGGL((spmv_h_kernel<U64, Pat, decltype(hv), double, double>), dim3((nt16 + U64 - 1) / U64), b16, 0,
                         s.stream, pat, hv, s.h_diag64, (const double*)x, (double*)y, alpha, s.n, nt16);
      break;
    }
    case 4: {
      const auto hv = pat.template mirror<false>((const e4m3*)s.h_off8, (const e4m3*)s.h_half[3]);
      hipLaunchKernelGGL((spmv_h_kernel<U16, Pat, decltype(hv), __half, float>), g16, b16, 0, s.stream, pat, hv,
                         s.h_diag16, (const __half*)x, (__half*)y, (float)alpha, s.n, nt16);
      break;
    }
  }
}

// Symmetric uniform offsets: H and S from their half layout (PatDiaSym), A
// from the full one.
template <int W>
static PatDiaSym<W> uniform_pattern(const System& s) {
  PatDiaSym<W> p;
  for (int j = 0; j < W; ++j) p.off[j] = s.dia_u[j];
  p.nmax = s.n - 1;
  p.pad = s.half_pad;
  return p;
}

extern "C" gadi_status gadi_spmv(gadi_handle* h, int32_t which, double alpha, const void* x, void* y) {
  if (!h || !x || !y || which < 0 || which > 4) return GADI_EINVAL;
  if (which != 0 && !(alpha > 0.0)) return GADI_EINVAL;
  System& s = h->sys;
  GADI_HIP_CHECK(hipSetDevice(s.device));
  if (which == 4) {
    const gadi_status st = ensure_fp8_public(s);
    if (st != GADI_OK) return st;
  }
  // the half layout of H and S for this product's value type (built on first use)
  if (which != 0 && s.dia_sym) {
    const int kind = which == 3 ? 2 : (which == 4 ? 3 : 0);
    const void* hf = which == 3 ? (const void*)s.h_off64 : (which == 4 ? (const void*)s.h_off8 : (const void*)s.h_off16);
    const void* sf = which == 3 ? (const void*)s.s_off64 : (which == 4 ? (const void*)s.s_off8 : (const void*)s.s_off16);
    const gadi_status st = ensure_half(s, kind, hf, sf);
    if (st != GADI_OK) return st;
  }
  const bool half = s.dia_sym && (which == 0 || s.h_half[which == 3 ? 2 : (which == 4 ? 3 : 0)]);
  switch (half ? s.dia_uniform : 0) {
    case 4: launch_products<4, 2>(s, uniform_pattern<4>(s), which, alpha, x, y); break;
    case 6: launch_products<4, 2>(s, uniform_pattern<6>(s), which, alpha, x, y); break;
    default:
      launch_products<1, 1>(s, PatGeneric{Pattern{s.slice_ptr, s.col, s.slice_dia, s.dia_off, s.n - 1}}, which, alpha,
                         x, y);
  }
  GADI_HIP_CHECK(hipGetLastError());
  return GADI_OK;
}

extern "C" gadi_status gadi_features(gadi_handle* h, int32_t dim, int32_t grid, const double* beta, float* out) {
  if (!h || !out || dim < 1 || grid < 1 || !beta) return GADI_EINVAL;
  System& s = h->sys;
  GADI_HIP_CHECK(hipSetDevice(s.device));
  const int nb = s.npad / kRowBlock;
  double* dpart = nullptr;
  GADI_HIP_CHECK(hipMalloc((void**)&dpart, sizeof(double) * 4 * nb));
  hipLaunchKernelGGL(gershgorin_kernel, dim3(nb), dim3(kRowBlock), 0, s.stream, s.slice_ptr, s.col, s.slice_dia, s.dia_off, s.h_off64, s.s_off64,
                     s.h_diag64, s.n, dpart);
  hipError_t e = hipGetLastError();
  std::vector<double> part((size_t)4 * nb);
  if (e == hipSuccess) e = hipMemcpyAsync(part.data(), dpart, sizeof(double) * 4 * nb, hipMemcpyDeviceToHost, s.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s.stream);
  (void)hipFree(dpart);
  if (e != hipSuccess) return fail_hip(e, "gershgorin", __FILE__, __LINE__);
  double g0 = INFINITY, g1 = -INFINITY, g2 = -INFINITY, g3 = INFINITY;
  for (int i = 0; i < nb; ++i) {
    g0 = std::fmin(g0, part[4 * i + 0]);
    g1 = std::fmax(g1, part[4 * i + 1]);
    g2 = std::fmax(g2, part[4 * i + 2]);
    g3 = std::fmin(g3, part[4 * i + 3]);
  }
  double bsum = 0.0, bmax = -INFINITY;
  for (int a = 0; a < dim; ++a) {
    bsum += beta[a];
    bmax = std::fmax(bmax, beta[a]);
  }
  const double bmean = bsum / dim;
  if (!(bmean > 0.0)) return GADI_EINVAL;
  const double hgrid = 1.0 / (grid + 1.0);
  out[0] = (float)std::log((double)s.n);
  out[1] = (float)dim;
  out[2] = (float)std::log10(bmean);
  // scale-free quantities enter in log10 (floored at 1e-12 so beta = 0 stays finite)
  auto lg = [](double v) { return std::log10(v > 1e-12 ? v : 1e-12); };
  out[3] = (float)lg(bmax * hgrid / 2.0);
  // spectral scale of H: its smallest eigenvalue in closed form (a sum of
  // 1-D h^2-scaled Laplacians: dim (2 - 2 cos(pi h))) and the Gershgorin
  // bound of its largest
  (void)g0;
  out[4] = (float)lg(dim * (2.0 - 2.0 * std::cos(M_PI * hgrid)));
  out[5] = (float)lg(g1);
  out[6] = (float)lg(g2);
  out[7] = (float)lg(g3);
  return GADI_OK;
}
