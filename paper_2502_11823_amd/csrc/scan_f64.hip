// scan_f64.hip -- scan kernels: FP64 sums on F64 storage (Dirichlet kernel): every waveform.
#include "sft_scan.h"

using namespace sftk;

ScanFn scan_pick_f64(int wf, int kern, int K, int nd)
{
  switch (wf) {
  case WF_PN35: return pick_kern<double2, SFT_PREC_FP64, WF_PN35>(kern, K, nd);
  case WF_TABLE: return pick_kern<double2, SFT_PREC_FP64, WF_TABLE>(kern, K, nd);
  default: return pick_kern<double2, SFT_PREC_FP64, WF_NEWTON>(kern, K, nd);
  }
}
