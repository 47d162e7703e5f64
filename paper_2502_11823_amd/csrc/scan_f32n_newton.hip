// scan_f32n_newton.hip -- scan kernels: FP32 plain sums on F32 storage, leading-order waveform.
#include "sft_scan.h"

using namespace sftk;

ScanFn scan_pick_f32n_newton(int kern, int K, int nd)
{
  return pick_kern<float2, SFT_PREC_FP32_NAIVE, WF_NEWTON>(kern, K, nd);
}
