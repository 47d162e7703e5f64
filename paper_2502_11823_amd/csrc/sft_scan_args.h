// sft_scan_args.h -- arguments of the bank-scan kernels, shared by the host code of
// libsft.so and the translation units that instantiate the scan kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sft.h"

// Rows that share a start time (detectors of one network) form a timestamp group;
// a group holds at most this many rows (more rows at one time start another group).
#define SFT_GROUP_MAX 4

struct ScanArgs {
  const void* bins;
  const void* psd;
  const double* g_tmid;    // [n_groups] midpoint time of each timestamp group
  const int32_t* g_rows;   // [n_groups][SFT_GROUP_MAX] SFT rows of the group, -1 = absent
  const double* fp;
  const double* fx;
  int32_t n_groups, n_ext, k_ext_lo, n_bins, k_lo, K;
  int32_t k_nyq;            // n / 2: window centres outside [0, k_nyq] have no data
  double T, beta_switch, tsun, delta_max;
  const double* mc;
  const double* q;
  const double* t_c;
  const double* phi_c;
  const int32_t* a_first;
  const int32_t* a_last;
  int64_t n_tmpl;
  int32_t chunk, n_chunks;  // groups per chunk, chunk count
  int32_t n_tiles;          // ceil(n_tmpl / blockDim.x)
  int32_t n_items;          // n_tiles * n_chunks work items, chunk-major
  int32_t persistent;       // 1: grid of resident blocks pulling items from *counter
  int32_t* counter;         // work-queue head (zeroed before the launch)
  double* part;      // [n_chunks][6 (+1 in the F-statistic form)][n_tmpl]
  uint32_t* pflags;  // [n_chunks][n_tmpl]
  const double* wtab;  // chirp table (WF_TABLE): 5 planes [n_groups][n_tmpl] kappa, phase, amp, beta, dres
  const double* sky;   // Doppler form: [n_tmpl][3] unit vectors toward the sources
  const double* g_eph; // Doppler form: [n_groups][9] detector r/c, v/c, a/c (one row per group)
};

enum { KERN_DIRICHLET = 0, KERN_FRESNEL = 1 };
// WF_TABLE: the chirp of every (template, group) comes precomputed from a table (the
// surrogate path fills it); an internal value, never accepted from the caller
enum { WF_NEWTON = SFT_WF_NEWTON, WF_PN35 = SFT_WF_PN35, WF_TABLE = 100 };

using ScanFn = void (*)(ScanArgs);

// Scan kernel for one arithmetic form, chosen by waveform (WF_*), kernel (KERN_*), window
// half-width K and the largest timestamp-group size nd.  Each is defined in its own
// translation unit (scan_*.hip), so that the kernel instantiations compile in parallel.
ScanFn scan_pick_f64(int wf, int kern, int K, int nd);
ScanFn scan_pick_f32k_newton(int kern, int K, int nd);
ScanFn scan_pick_f32k_pn35(int kern, int K, int nd);
ScanFn scan_pick_f32k_table(int kern, int K, int nd);
ScanFn scan_pick_f32n_newton(int kern, int K, int nd);
ScanFn scan_pick_f32n_pn35(int kern, int K, int nd);
ScanFn scan_pick_f32n_table(int kern, int K, int nd);
ScanFn scan_pick_bf16(int prec, int kern, int K, int nd);
// the F-statistic form (Newtonian waveform; prec SFT_PREC_FP32_KAHAN with F32 storage or
// SFT_PREC_FP64 with F64 storage and the Dirichlet kernel)
ScanFn scan_pick_fstat(int prec, int kern, int K, int nd);
// the Doppler form (one row per timestamp group; Newtonian waveform; fs selects the
// F-statistic form as well)
ScanFn scan_pick_doppler(int prec, int fs, int kern, int K);
// the Taylor expansion at the SFT start (run-time window)
ScanFn scan_pick_start(int storage, int prec, int wf, int kern, int nd, int fs);
