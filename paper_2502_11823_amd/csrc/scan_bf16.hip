// scan_bf16.hip -- scan kernels: FP32 sums on BF16 storage, leading-order waveform.
#include "sft_scan.h"

using namespace sftk;

ScanFn scan_pick_bf16(int prec, int kern, int K, int nd)
{
  return prec == SFT_PREC_FP32_KAHAN ? pick_kern<bf16x2, SFT_PREC_FP32_KAHAN, WF_NEWTON>(kern, K, nd)
                                     : pick_kern<bf16x2, SFT_PREC_FP32_NAIVE, WF_NEWTON>(kern, K, nd);
}
