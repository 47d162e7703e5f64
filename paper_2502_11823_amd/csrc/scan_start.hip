// scan_start.hip -- scan kernels with the Taylor expansion at the SFT start (the paper's
// reference point; run-time window): every storage and precision, the closed-form waveforms,
// plain and F-statistic forms.
#include "sft_scan.h"

using namespace sftk;

ScanFn scan_pick_start(int storage, int prec, int wf, int kern, int nd, int fs)
{
  if (prec == SFT_PREC_FP64) {
    if (fs) return pick_start<double2, SFT_PREC_FP64, WF_NEWTON, 1>(kern, nd);
    return wf == WF_PN35 ? pick_start<double2, SFT_PREC_FP64, WF_PN35>(kern, nd)
                         : pick_start<double2, SFT_PREC_FP64, WF_NEWTON>(kern, nd);
  }
  if (storage == SFT_STORE_BF16)
    return prec == SFT_PREC_FP32_KAHAN ? pick_start<bf16x2, SFT_PREC_FP32_KAHAN, WF_NEWTON>(kern, nd)
                                       : pick_start<bf16x2, SFT_PREC_FP32_NAIVE, WF_NEWTON>(kern, nd);
  if (prec == SFT_PREC_FP32_KAHAN) {
    if (fs) return pick_start<float2, SFT_PREC_FP32_KAHAN, WF_NEWTON, 1>(kern, nd);
    return wf == WF_PN35 ? pick_start<float2, SFT_PREC_FP32_KAHAN, WF_PN35>(kern, nd)
                         : pick_start<float2, SFT_PREC_FP32_KAHAN, WF_NEWTON>(kern, nd);
  }
  return wf == WF_PN35 ? pick_start<float2, SFT_PREC_FP32_NAIVE, WF_PN35>(kern, nd)
                       : pick_start<float2, SFT_PREC_FP32_NAIVE, WF_NEWTON>(kern, nd);
}
