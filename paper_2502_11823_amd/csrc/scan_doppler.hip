// scan_doppler.hip -- scan kernels of the Doppler form (one row per timestamp group, chirp at
// the emission time), plain and F-statistic: FP32 compensated sums on F32 storage and FP64
// sums on F64 storage (Dirichlet kernel), leading-order waveform.
#include "sft_scan.h"

using namespace sftk;

ScanFn scan_pick_doppler(int prec, int fs, int kern, int K)
{
  if (prec == SFT_PREC_FP64) {
    if (kern == KERN_DIRICHLET)
      return fs ? pick_doppler_k<double2, SFT_PREC_FP64, KERN_DIRICHLET, 1>(K)
                : pick_doppler_k<double2, SFT_PREC_FP64, KERN_DIRICHLET, 0>(K);
    return fs ? pick_doppler_k<double2, SFT_PREC_FP64, KERN_FRESNEL, 1>(K)
              : pick_doppler_k<double2, SFT_PREC_FP64, KERN_FRESNEL, 0>(K);
  }
  if (kern == KERN_DIRICHLET)
    return fs ? pick_doppler_k<float2, SFT_PREC_FP32_KAHAN, KERN_DIRICHLET, 1>(K)
              : pick_doppler_k<float2, SFT_PREC_FP32_KAHAN, KERN_DIRICHLET, 0>(K);
  return fs ? pick_doppler_k<float2, SFT_PREC_FP32_KAHAN, KERN_FRESNEL, 1>(K)
            : pick_doppler_k<float2, SFT_PREC_FP32_KAHAN, KERN_FRESNEL, 0>(K);
}
