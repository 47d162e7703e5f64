// sft_series.hip -- time-domain companions of the SFT inner product, for studies of its
// accuracy (Sec. IV.A: r = 1 - sqrt(([d,h]) / <d,h>) against the direct integral):
//   series_kernel : the strain of one template at every sample time, with the waveform of the
//                   scans (FP64), h = A [F+ A+ cos(phi) + Fx Ax sin(phi)] (Sec. II.A projector);
//   tdp_kernel    : <x, y> = (2 / S) dt sum_j x_j y_j for a white one-sided PSD S (Eq. td_product
//                   of the whitened data of Eq. whitened_data), as FP64 partial sums per block
//                   combined in a fixed order (bitwise reproducible).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/sft.h"
#include "sft_device.h"

sft_status sft_set_error(sft_status st, const char* msg);

using namespace sftk;

namespace {

constexpr int kSeriesBlock = 256;

__global__ __launch_bounds__(kSeriesBlock) void series_kernel(int32_t wf, double mc, double q, double t_c, double phi_c,
                                                              double tsun, double t0, double dt, int64_t n,
                                                              const double* __restrict__ fplus,
                                                              const double* __restrict__ fcross, double a_plus,
                                                              double a_cross, double* __restrict__ h,
                                                              double* __restrict__ quant)
{
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double t = fma((double)j, dt, t0);
  const double tau = t_c - t;
  Chirp ch{};
  bool ok = tau > 0.0;
  if (ok) {
    if (wf == SFT_WF_PN35) {
      double qq = q;
      if (!(qq >= 1.0)) qq = 1.0 / qq;
      const double nu = qq / ((1.0 + qq) * (1.0 + qq));
      const double Mt = mc * pow(nu, -0.6) * tsun;
      ch = pn35_chirp(tau, nu, nu / (5.0 * Mt), Mt, pow(nu, 0.4), phi_c, 1.0, pn_coefficients(nu));
    } else {
      const double M = mc * tsun;
      ch = newton_chirp(tau, 1.0 / (5.0 * M), 1.0 / (8.0 * kPi * M), phi_c, 1.0);
    }
    ok = isfinite(ch.phase) && isfinite(ch.amp);
  }
  double v = 0.0;
  if (ok) {
    double s, c;
    sincos(reduce_2pi(ch.phase), &s, &c);
    const double fp = fplus ? fplus[j] : 1.0, fx = fcross ? fcross[j] : 0.0;
    v = ch.amp * (fp * a_plus * c + fx * a_cross * s);
  }
  h[j] = v;
  if (quant) {
    double* qo = quant + 5 * j;
    // with T = 1 the chirp's kappa, beta and dres are f, fdot and fddot / 8
    qo[0] = ok ? ch.amp : 0.0;
    qo[1] = ok ? ch.phase : 0.0;
    qo[2] = ok ? ch.kappa : 0.0;
    qo[3] = ok ? ch.beta : 0.0;
    qo[4] = ok ? 8.0 * ch.dres : 0.0;
  }
}

// block b sums x_j y_j over j in [b chunk, (b+1) chunk) with a Neumaier-compensated FP64 sum per
// thread (strided), then a fixed-order tree over the block's threads
__global__ __launch_bounds__(kSeriesBlock) void tdp_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                                           int64_t n, int64_t chunk, double* __restrict__ part)
{
  __shared__ double sh[kSeriesBlock];
  const int64_t j0 = (int64_t)blockIdx.x * chunk;
  const int64_t j1 = j0 + chunk < n ? j0 + chunk : n;
  double s = 0.0, c = 0.0;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
    const double v = x[j] * y[j];
    const double t = s + v;
    c += fabs(s) >= fabs(v) ? (s - t) + v : (v - t) + s;
    s = t;
  }
  sh[threadIdx.x] = s + c;
  __syncthreads();
  for (int w = kSeriesBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

}  // namespace

extern "C" sft_status sft_waveform_series(int32_t waveform, double mc, double q, double t_c, double phi_c, double tsun,
                                          double t0, double dt, int64_t n, const double* fplus, const double* fcross,
                                          double a_plus, double a_cross, double* h, double* quantities,
                                          void* hip_stream)
{
  if (!h) return sft_set_error(SFT_E_INVALID, "sft_waveform_series: null output");
  if (waveform != SFT_WF_NEWTON && waveform != SFT_WF_PN35)
    return sft_set_error(SFT_E_UNSUPPORTED, "sft_waveform_series: Newtonian or 3.5PN waveform only");
  if (n < 0 || !(dt > 0.0) || !(mc > 0.0) || !(tsun > 0.0))
    return sft_set_error(SFT_E_INVALID, "sft_waveform_series: bad argument");
  if (n == 0) return SFT_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t nb = (n + kSeriesBlock - 1) / kSeriesBlock;
  if (nb > INT32_MAX) return sft_set_error(SFT_E_RANGE, "sft_waveform_series: too many samples");
  hipLaunchKernelGGL(series_kernel, dim3((unsigned)nb), dim3(kSeriesBlock), 0, st, waveform, mc, q, t_c, phi_c, tsun,
                     t0, dt, n, fplus, fcross, a_plus, a_cross, h, quantities);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return sft_set_error(SFT_E_DEVICE, hipGetErrorString(e));
  return SFT_OK;
}

extern "C" sft_status sft_td_product(const double* x, const double* y, int64_t n, double dt, double psd,
                                     void* hip_stream, double* out)
{
  if (!x || !y || !out) return sft_set_error(SFT_E_INVALID, "sft_td_product: null argument");
  if (n < 1 || !(dt > 0.0) || !(psd > 0.0)) return sft_set_error(SFT_E_INVALID, "sft_td_product: bad argument");
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t chunk = 1 << 16;
  const int64_t nb = (n + chunk - 1) / chunk;
  double* part = nullptr;
  hipError_t e = hipMallocAsync((void**)&part, nb * sizeof(double), st);
  std::vector<double> hp(nb);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(tdp_kernel, dim3((unsigned)nb), dim3(kSeriesBlock), 0, st, x, y, n, chunk, part);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(hp.data(), part, nb * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (part) (void)hipFreeAsync(part, st);
  if (e != hipSuccess) return sft_set_error(SFT_E_DEVICE, hipGetErrorString(e));
  // the block partials in order, compensated
  double s = 0.0, c = 0.0;
  for (double v : hp) {
    const double t = s + v;
    c += std::fabs(s) >= std::fabs(v) ? (s - t) + v : (v - t) + s;
    s = t;
  }
  *out = (s + c) * dt * 2.0 / psd;
  return SFT_OK;
}
