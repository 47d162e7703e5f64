// scan_f64.hip -- scan kernels: FP64 sums on F64 storage (Dirichlet kernel): every waveform.
#include "sft_scan.h"

using namespace sftk;

ScanFn scan_pick_f64(int wf, int K, int nd)
{
  switch (wf) {
  case WF_PN35: return pick_k<double2, SFT_PREC_FP64, KERN_DIRICHLET, WF_PN35>(K, nd);
  case WF_TABLE: return pick_k<double2, SFT_PREC_FP64, KERN_DIRICHLET, WF_TABLE>(K, nd);
  default: return pick_k<double2, SFT_PREC_FP64, KERN_DIRICHLET, WF_NEWTON>(K, nd);
  }
}
