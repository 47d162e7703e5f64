// scan_fstat.hip -- scan kernels of the F-statistic form (cross norm, FP64 norm sums):
// FP32 compensated sums on F32 storage and FP64 sums on F64 storage (Dirichlet kernel),
// leading-order waveform.
#include "sft_scan.h"

using namespace sftk;

ScanFn scan_pick_fstat(int prec, int kern, int K, int nd)
{
  if (prec == SFT_PREC_FP64) return pick_kern<double2, SFT_PREC_FP64, WF_NEWTON, 1>(kern, K, nd);
  return pick_kern<float2, SFT_PREC_FP32_KAHAN, WF_NEWTON, 1>(kern, K, nd);
}
