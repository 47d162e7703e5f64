// scan_f32k_newton.hip -- scan kernels: FP32 compensated sums on F32 storage, leading-order waveform.
#include "sft_scan.h"

using namespace sftk;

ScanFn scan_pick_f32k_newton(int kern, int K, int nd)
{
  return pick_kern<float2, SFT_PREC_FP32_KAHAN, WF_NEWTON>(kern, K, nd);
}
