// scan_f32k_table.hip -- scan kernels: FP32 compensated sums on F32 storage, tabulated (surrogate) waveform.
#include "sft_scan.h"

using namespace sftk;

ScanFn scan_pick_f32k_table(int kern, int K, int nd)
{
  return pick_kern<float2, SFT_PREC_FP32_KAHAN, WF_TABLE>(kern, K, nd);
}
