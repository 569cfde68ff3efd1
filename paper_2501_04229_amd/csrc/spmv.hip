// Stand-alone operator products on the packed SELL-64 layout (kernel-level
// parity checks and bandwidth measurement) and the Gershgorin feature pass.
#include <cmath>
#include <vector>

#include "device_common.h"

namespace gadi {

// y = A x in double (the residual's operator, step 1 of Algorithm 1)
__global__ void __launch_bounds__(kRowBlock) spmv_a64_kernel(const int32_t* __restrict__ sp, const int32_t* __restrict__ col,
    const int32_t* __restrict__ dia, const int32_t* __restrict__ doff,
                                                           const double* __restrict__ off, const double* __restrict__ diag,
                                                           const double* __restrict__ x, double* __restrict__ y, int n) {
  const int row = blockIdx.x * kRowBlock + threadIdx.x;
  const double xi = row < n ? x[row] : 0.0;
  const double acc = diag[row] * xi + row_sum<double>(row, Pattern{sp, col, dia, doff, n - 1}, off, [&](int c) { return x[c]; });
  if (row < n) y[row] = acc;
}

// y = (alpha I + H) x with H, x, y in the value type MT, arithmetic in AT
template <class MT, class AT>
__global__ void __launch_bounds__(kRowBlock) spmv_h_kernel(const int32_t* __restrict__ sp, const int32_t* __restrict__ col,
    const int32_t* __restrict__ dia, const int32_t* __restrict__ doff,
                                                         const MT* __restrict__ off, const MT* __restrict__ diag,
                                                         const MT* __restrict__ x, MT* __restrict__ y, AT alpha, int n) {
  const int row = blockIdx.x * kRowBlock + threadIdx.x;
  const AT xi = row < n ? ld<AT>(x[row]) : AT(0);
  const AT acc = (alpha + ld<AT>(diag[row])) * xi + row_sum<AT>(row, Pattern{sp, col, dia, doff, n - 1}, off, [&](int c) { return ld<AT>(x[c]); });
  if (row < n) y[row] = st<MT>(acc);
}

// y = (I + S / alpha) x, half in/out, float arithmetic
__global__ void __launch_bounds__(kRowBlock) spmv_s16_kernel(const int32_t* __restrict__ sp, const int32_t* __restrict__ col,
    const int32_t* __restrict__ dia, const int32_t* __restrict__ doff,
                                                           const __half* __restrict__ off, const __half* __restrict__ x,
                                                           __half* __restrict__ y, float inv_alpha, int n) {
  const int row = blockIdx.x * kRowBlock + threadIdx.x;
  const float xi = row < n ? __half2float(x[row]) : 0.f;
  const float acc = xi + inv_alpha * row_sum<float>(row, Pattern{sp, col, dia, doff, n - 1}, off, [&](int c) { return __half2float(x[c]); });
  if (row < n) y[row] = __float2half_rn(acc);
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

extern "C" gadi_status gadi_spmv(gadi_handle* h, int32_t which, double alpha, const void* x, void* y) {
  if (!h || !x || !y || which < 0 || which > 3) return GADI_EINVAL;
  if ((which == 1 || which == 2 || which == 3) && !(alpha > 0.0)) return GADI_EINVAL;
  System& s = h->sys;
  GADI_HIP_CHECK(hipSetDevice(s.device));
  const dim3 grid(s.npad / kRowBlock), block(kRowBlock);
  switch (which) {
    case 0:
      hipLaunchKernelGGL(spmv_a64_kernel, grid, block, 0, s.stream, s.slice_ptr, s.col, s.slice_dia, s.dia_off, s.a_off, s.a_diag,
                         (const double*)x, (double*)y, s.n);
      break;
    case 1:
      hipLaunchKernelGGL((spmv_h_kernel<__half, float>), grid, block, 0, s.stream, s.slice_ptr, s.col, s.slice_dia, s.dia_off, s.h_off16,
                         s.h_diag16, (const __half*)x, (__half*)y, (float)alpha, s.n);
      break;
    case 2:
      hipLaunchKernelGGL(spmv_s16_kernel, grid, block, 0, s.stream, s.slice_ptr, s.col, s.slice_dia, s.dia_off, s.s_off16, (const __half*)x,
                         (__half*)y, (float)(1.0 / alpha), s.n);
      break;
    case 3:
      hipLaunchKernelGGL((spmv_h_kernel<double, double>), grid, block, 0, s.stream, s.slice_ptr, s.col, s.slice_dia, s.dia_off, s.h_off64,
                         s.h_diag64, (const double*)x, (double*)y, alpha, s.n);
      break;
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
