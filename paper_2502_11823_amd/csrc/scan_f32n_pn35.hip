// scan_f32n_pn35.hip -- scan kernels: FP32 plain sums on F32 storage, 3.5PN waveform.
#include "sft_scan.h"

using namespace sftk;

ScanFn scan_pick_f32n_pn35(int kern, int K, int nd)
{
  return pick_kern<float2, SFT_PREC_FP32_NAIVE, WF_PN35>(kern, K, nd);
}
