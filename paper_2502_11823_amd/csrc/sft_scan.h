// sft_scan.h -- the bank-scan kernel templates (device code).  Included only by the
// translation units scan_*.hip, each of which instantiates one arithmetic form.
//
// One lane per template, one work item per (template tile, chunk of timestamp groups).
// For every timestamp group of the chunk: FP64 chirp at the SFT midpoint, FP64 phase
// reduction, FP64 bin split, 2K+1 kernel weights and the bin contraction (Eq. with_f_1),
// the coherent accumulation of Eq. efficient and of the norm, in FP64 or FP32 (Kahan or
// plain).  Writes one partial per (template, chunk); the finalize kernel combines them.
// REF = 1: the Taylor expansion at the SFT start (the paper's form) instead of the midpoint.
// FS = 1 (the F-statistic form, Sec. II.B) also accumulates the cross norm
// sum F+ Fx A^2 T / S, and keeps the three norm sums in FP64.  DP = 1 (the Doppler form,
// Sec. III.B) evaluates the chirp at the emission time t + r.n/c of each SFT row's detector
// and carries the factor dt_s/dt into f and fdot (one row per timestamp group).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "sft_device.h"
#include "sft_scan_args.h"

namespace sftk {

// smallest window half-width for which the Fresnel loop splits the bins into series segments
#ifndef SFT_OUTER_MIN_K
#define SFT_OUTER_MIN_K 4
#endif

// unroll factor of the Dirichlet bin loop
#ifndef SFT_BIN_UNROLL
#define SFT_BIN_UNROLL 4
#endif

// accumulators
struct AccKahan {
  float s = 0.f, c = 0.f;
  __device__ inline void add(float x)
  {
    float y = x - c;
    float t = s + y;
    c = (t - s) - y;
    s = t;
  }
  __device__ inline double get() const { return (double)s - (double)c; }
};
struct AccNaive {
  float s = 0.f;
  __device__ inline void add(float x) { s += x; }
  __device__ inline double get() const { return (double)s; }
};
struct AccF64 {
  double s = 0.0;
  __device__ inline void add(double x) { s += x; }
  __device__ inline double get() const { return s; }
};

template <int PREC> struct PrecTraits;
template <> struct PrecTraits<SFT_PREC_FP64> { using R = double; using Acc = AccF64; };
template <> struct PrecTraits<SFT_PREC_FP32_KAHAN> { using R = float; using Acc = AccKahan; };
template <> struct PrecTraits<SFT_PREC_FP32_NAIVE> { using R = float; using Acc = AccNaive; };

__device__ inline float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Order of the window bins in the Dirichlet contraction.  Wide windows (K >= SFT_WIDE_K) go
// from the outside in (-K, K, -K+1, K-1, ..., 0), so that the running sum stays small until the
// dominant central bins arrive and the rounding of the many small far-bin terms is not taken
// against the full sum; narrow windows go left to right (same accuracy at that length, and
// faster: consecutive bins share the loads' address arithmetic).  The Fresnel loop orders its
// series segments from the edges inwards instead.
#ifndef SFT_WIDE_K
#define SFT_WIDE_K 16
#endif
__device__ inline int bin_order(int t, int K)
{
  return K >= SFT_WIDE_K ? ((t & 1) ? K - (t >> 1) : (t >> 1) - K) : t - K;
}

// Largest x over the active lanes of the wavefront, for x in [lo, hi] (wave-uniform bounds).
// The first active lane's value is the answer when no active lane exceeds it (the usual
// case: neighbouring templates share their windows); otherwise a binary search on lane
// votes above it (a compare's lane mask holds bits of active lanes only).
__device__ inline int wave_max_active(int x, int lo, int hi)
{
  const int c = __builtin_amdgcn_readfirstlane(x);
  if (!__ballot(x > c)) return c;
  lo = c + 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (__ballot(x >= mid)) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// [lo, hi] of x over the active lanes, when every active lane is within span of the first
// active lane's value; false otherwise.
__device__ inline bool wave_range(int x, int span, int& lo, int& hi)
{
  const int c = __builtin_amdgcn_readfirstlane(x);
  if (__ballot(x < c - span || x > c + span)) return false;
  hi = c + wave_max_active(x - c, 0, span);
  lo = c - wave_max_active(c - x, 0, span);
  return true;
}

// LDS stage of one timestamp group's bins for a wavefront: ND rows of stage_width bins from
// a wave-uniform start.  Compile-time windows (2K+1 bins) leave room for lanes whose windows
// start up to ~47 bins apart; the run-time K kernel holds K up to 64 with ~63 bins of spread.
// The 3.5PN kernels (two wavefronts per SIMD for their registers) gather instead: the stage's
// load -> LDS -> read chain per group costs them more latency than the gathers it replaces.
template <int KC, int WF>
__host__ __device__ constexpr int stage_width()
{
  return WF == WF_PN35 ? 0 : KC >= 0 ? (2 * KC + 1 + 47 + 63) / 64 * 64 : 192;
}

// The active lanes copy bins [sb, sb + wl) of each row into the wavefront's stage, bin p by
// the lane of rank p mod (active lanes) (coalesced; any exec mask).  The fences keep the
// previous group's LDS reads before these writes and the bin loops' reads after them (a
// wavefront's LDS instructions execute in order).
template <typename Bin, int ND, int WST>
__device__ inline void stage_window(Bin* sw, const Bin* const* rp, int sb, int wl)
{
  const uint64_t ex = __builtin_amdgcn_read_exec();
  const int nact = __builtin_popcountll(ex);
  const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(ex >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)ex, 0u));
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  for (int p = rank; p < wl; p += nact) {
    Bin v[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) v[d] = rp[d][sb + p];
#pragma unroll
    for (int d = 0; d < ND; ++d) sw[d * WST + p] = v[d];
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One lane per template, one grid row per chunk of timestamp groups.  The SFT rows of
// a group (one per detector) share the SFT midpoint, hence the chirp, the window and
// all 2K+1 kernel weights: those are evaluated once per group and contracted with the
// bins of each of the ND rows (the projector Lambda carries the detector dependence).
template <typename Bin, int PREC, int KERN, int KC, int ND, int WF, int FS, int DP, int REF>
__device__ __forceinline__ void scan_item(const ScanArgs& a, const int K, const int64_t m, const int c, const float2* tab,
                                          Bin* sw);

// Register budget: the FP32 Fresnel kernels with a compile-time window for groups of 2 or 3
// rows, and the one-row K = 32 kernel, with the Newtonian chirp fit 96 VGPRs without
// spilling, i.e. 5 wavefronts per SIMD instead of 4; the FP32 Dirichlet kernels with the
// 3.5PN chirp fit 168, i.e. 3 instead of 2.  The others are left to the compiler (1 = no
// constraint).
template <int PREC, int KERN, int KC, int ND, int WF>
constexpr int scan_min_waves()
{
  if (PREC != SFT_PREC_FP64 && KERN == KERN_FRESNEL && KC >= 0 && WF == WF_NEWTON &&
      (ND == 2 || ND == 3 || (ND == 1 && KC == 32)))
    return 5;
  if (PREC != SFT_PREC_FP64 && KERN == KERN_DIRICHLET && WF == WF_PN35) return 3;
  return 1;
}

template <typename Bin, int PREC, int KERN, int KC, int ND, int WF, int FS = 0, int DP = 0, int REF = 0>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(scan_min_waves<PREC, KERN, KC, ND, WF>())))
void scan_kernel(ScanArgs a)
{
  __shared__ float2 tab[SFT_G_NINT * (SFT_G_DEG + 1)];
  if (KERN == KERN_FRESNEL) {
    for (int i = threadIdx.x; i < SFT_G_NINT * (SFT_G_DEG + 1); i += blockDim.x)
      tab[i] = make_float2(sft_g_coef[i / (SFT_G_DEG + 1)][i % (SFT_G_DEG + 1)][0],
                           sft_g_coef[i / (SFT_G_DEG + 1)][i % (SFT_G_DEG + 1)][1]);
    __syncthreads();
  }

  __shared__ int s_item;
  // per wavefront (at most 4 per workgroup): the bins of the current timestamp group
  constexpr int WST = stage_width<KC, WF>();
  __shared__ Bin stage[4 * ND * (WST > 0 ? WST : 1)];
  const int K = KC >= 0 ? KC : a.K;
  // A work item is (template tile, chunk of timestamp groups), chunk-major so that
  // concurrently running blocks share the data rows of one chunk in L2.  A plain grid
  // runs one item per block; a persistent grid pulls items from a counter until the
  // queue is empty (every block reaches the exit test with the same item value).
  int item = (int)(blockIdx.y * gridDim.x + blockIdx.x);
  for (;;) {
    if (a.persistent) {
      __syncthreads();
      if (threadIdx.x == 0) s_item = atomicAdd(a.counter, 1);
      __syncthreads();
      item = s_item;
      if (item >= a.n_items) break;
    }
    const int tile = item % a.n_tiles;
    const int c = item / a.n_tiles;
    const int64_t m = (int64_t)tile * blockDim.x + threadIdx.x;
    if (m < a.n_tmpl)
      scan_item<Bin, PREC, KERN, KC, ND, WF, FS, DP, REF>(a, K, m, c, tab, stage + (threadIdx.x >> 6) * (ND * WST));
    if (!a.persistent) break;
  }
}

template <typename Bin, int PREC, int KERN, int KC, int ND, int WF, int FS, int DP, int REF>
__device__ __forceinline__ void scan_item(const ScanArgs& a, const int K, const int64_t m, const int c, const float2* tab,
                                          Bin* sw)
{
  constexpr int WST = stage_width<KC, WF>();
  using R = typename PrecTraits<PREC>::R;
  using Acc = typename PrecTraits<PREC>::Acc;
  using PS = typename std::conditional<PREC == SFT_PREC_FP64, double, float>::type;
  const int g0 = c * a.chunk;
  const int g1 = min(g0 + a.chunk, a.n_groups) - 1;
  const int lo = a.a_first ? (int)a.a_first[m] : 0;
  const int hi = a.a_last ? (int)a.a_last[m] : 0x7fffffff;

  const double T = a.T;
  double inv5M = 0.0, cf = 0.0;
  if constexpr (WF == WF_NEWTON) {
    const double M = a.mc[m] * a.tsun;
    inv5M = 1.0 / (5.0 * M);
    cf = T / (8.0 * kPi * M);
  }
  const double tc = a.t_c[m];
  const double phic = a.phi_c ? a.phi_c[m] : 0.0;
  // Doppler form: unit vector toward the source
  double nx = 0.0, ny = 0.0, nz = 0.0;
  if constexpr (DP != 0) {
    nx = a.sky[3 * m];
    ny = a.sky[3 * m + 1];
    nz = a.sky[3 * m + 2];
  }
  // 3.5PN: symmetric mass ratio, total mass, nu/(5M), nu^(2/5) and the series coefficients
  double nu = 0.25, Mt = 0.0, inv5Mnu = 0.0, nu25 = 0.0;
  PNCoef pcf{};
  if constexpr (WF == WF_PN35) {
    double qq = a.q ? a.q[m] : 1.0;
    if (!(qq >= 1.0)) qq = 1.0 / qq;
    nu = qq / ((1.0 + qq) * (1.0 + qq));
    Mt = a.mc[m] * pow(nu, -0.6) * a.tsun;
    inv5Mnu = nu / (5.0 * Mt);
    nu25 = pow(nu, 0.4);
    pcf = pn_coefficients(nu);
  }
  const Bin* __restrict__ bins = (const Bin*)a.bins;
  const PS* __restrict__ psd = (const PS*)a.psd;

  Acc zpr, zpi, zxr, zxi;
  // norm sums: FP64 in the F-statistic form, whose 2x2 norm matrix is inverted
  using NAcc = typename std::conditional<FS != 0, AccF64, Acc>::type;
  NAcc hp, hx, hpx;
  uint32_t fl = 0;

  // the group's rows and midpoint time are loaded one group ahead, so that their latency
  // overlaps the previous group's work
  int nrows[ND];
  double ntmid = 0.0;
  if (g0 <= g1) {
#pragma unroll
    for (int d = 0; d < ND; ++d) nrows[d] = a.g_rows[g0 * SFT_GROUP_MAX + d];
    ntmid = a.g_tmid[g0];
  }
  for (int g = g0; g <= g1; ++g) {
    int rows[ND];
    bool act[ND];
    bool any = false;
#pragma unroll
    for (int d = 0; d < ND; ++d) rows[d] = nrows[d];
    const double tmid = ntmid;
    if (g < g1) {
#pragma unroll
      for (int d = 0; d < ND; ++d) nrows[d] = a.g_rows[(g + 1) * SFT_GROUP_MAX + d];
      ntmid = a.g_tmid[g + 1];
    }
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      act[d] = rows[d] >= 0 && rows[d] >= lo && rows[d] <= hi;
      any = any || act[d];
    }
    if (!any) continue;
    // Doppler form: Roemer delay r.n/c and its rates v.n/c, a.n/c of the row's detector
    double dl = 0.0, dl1 = 0.0, dl2 = 0.0;
    if constexpr (DP != 0) {
      const double* e = a.g_eph + 9 * (int64_t)g;
      dl = fma(e[0], nx, fma(e[1], ny, e[2] * nz));
      dl1 = fma(e[3], nx, fma(e[4], ny, e[5] * nz));
      dl2 = fma(e[6], nx, fma(e[7], ny, e[8] * nz));
    }
    // the reference time of the Taylor expansion: the SFT midpoint, or its start
    const double tref = REF != 0 ? tmid - 0.5 * T : tmid;
    const double tau = DP != 0 ? tc - (tref + dl) : tc - tref;
    if (!(tau > 0.0)) {
      fl |= kFlagTau;
      continue;
    }
    {
      uint32_t nact = 0;
#pragma unroll
      for (int d = 0; d < ND; ++d) nact += act[d] ? 1u : 0u;
      fl += nact << kUsedShift;
    }
    Chirp ch;
    if constexpr (WF == WF_PN35) {
      ch = pn35_chirp(tau, nu, inv5Mnu, Mt, nu25, phic, T, pcf);
    } else if constexpr (WF == WF_TABLE) {
      const int64_t ps = (int64_t)a.n_groups * a.n_tmpl;
      const double* w = a.wtab + (int64_t)g * a.n_tmpl + m;
      ch.kappa = w[0];
      ch.phase = w[ps];
      ch.amp = w[2 * ps];
      ch.beta = w[3 * ps];
      ch.dres = w[4 * ps];
    } else {
      ch = newton_chirp(tau, inv5M, cf, phic, T);
    }
    if constexpr (DP != 0) {
      // f = f_s (1 + D'), fdot = fdot_s (1 + D')^2 + f_s D'' (in bins: times T and T^2),
      // fddot scaled by (1 + D')^3 for the validity flag
      const double g1 = 1.0 + dl1;
      const double ks = ch.kappa;
      ch.kappa = ks * g1;
      ch.beta = fma(ch.beta, g1 * g1, ks * dl2 * T);
      ch.dres *= g1 * g1 * g1;
    }
    // Start reference: the kernel over [0, 1] is the midpoint kernel at x + beta/2 times
    // exp(i (pi x + pi beta / 4)), with x = kappa - k; the (-1)^k of the midpoint form absorbs
    // exp(i pi (kappa - k)) up to exp(i pi kappa).  So the start form is the midpoint form with
    // the kernel argument kappa + beta/2 and the phase phi + pi kappa + pi beta / 4, the window
    // still centred on the start frequency; the validity lever is T instead of T / 2.
    // The drift in the shift is the kernel's: 0 where the Dirichlet limit is used.
    double kwin = ch.kappa;
    if constexpr (REF != 0) {
      const double bk = (KERN == KERN_FRESNEL && !(fabs(ch.beta) <= a.beta_switch)) ? ch.beta : 0.0;
      kwin = fma(0.5, bk, ch.kappa);
      ch.phase += kPi * fma(0.25, bk, ch.kappa);
      ch.dres *= 4.0;
    }
    if (a.delta_max > 0.0 && ch.dres > a.delta_max) fl |= kFlagTaylor;
    if (!(ch.kappa < 1.0e9)) {
      // frequency far above any stored band: no window bin and no norm bin exists
      fl |= kFlagOOB;
      continue;
    }
    const double kr = floor(ch.kappa + 0.5);
    const double delta = kwin - kr;
    const int k0 = (int)kr;
    if (k0 < 0 || k0 > a.k_nyq) {
      // frequency below DC or above Nyquist: no representation in the data (its norm bins
      // are outside the band too)
      fl |= kFlagOOB;
      continue;
    }
    const int i0 = k0 - K - a.k_ext_lo;
    const bool inband = (i0 >= 0) && (i0 + 2 * K < a.n_ext);
    const Bin* rp[ND];
#pragma unroll
    // an absent row of the group reads row 0 instead: its contraction is computed (keeping the
    // bin loop free of per-row branches, so the loads of all rows are issued together) and
    // never accumulated
    for (int d = 0; d < ND; ++d) rp[d] = bins + (int64_t)(rows[d] >= 0 ? rows[d] : 0) * a.n_ext;
    // Neighbouring templates share most of their windows: when every active lane of the
    // wavefront is in band and the union of the windows fits the stage, the lanes load the
    // union once, coalesced, into LDS and the bin loops read it there (stg); otherwise each
    // lane gathers its bins from global memory with range checks.
    bool stg = false;
    int sb = 0;
    if (WST > 0 && !__ballot(!inband)) {
      int wlo, whi;
      if (wave_range(i0, WST, wlo, whi) && whi - wlo + 2 * K + 1 <= WST) {
        stg = true;
        sb = wlo;
        stage_window<Bin, ND, WST>(sw, rp, sb, whi - wlo + 2 * K + 1);
      }
    }

    R cre[ND], cim[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) cre[d] = cim[d] = (R)0;
    bool dir = true;
    if constexpr (KERN == KERN_FRESNEL) dir = fabs(ch.beta) <= a.beta_switch;
    if (dir) {
      // H_j = sin(pi delta) / (pi (delta - j))
      const R dl = (R)delta;
      R sp;
      if constexpr (PREC == SFT_PREC_FP64) {
        sp = sin(kPi * delta) / kPi;
      } else {
        float s_, c_;
        phasor(kPi * delta, s_, c_);
        sp = s_ * kInvPiF;
      }
      auto drun = [&](auto stgc) {
        constexpr bool STG = decltype(stgc)::value;
#pragma unroll SFT_BIN_UNROLL
        for (int t = 0; t <= 2 * K; ++t) {
          const int j = bin_order(t, K);
          const int idx = i0 + j + K;
          if (!STG && !inband && (idx < 0 || idx >= a.n_ext)) {
            fl |= kFlagOOB;
            continue;
          }
          const R x = dl - (R)j;
          R h;
          if constexpr (PREC == SFT_PREC_FP64) h = (x == (R)0) ? (R)1 : sp / x;
          else h = (x == (R)0) ? (R)1 : (R)(sp * fast_rcp((float)x));
#pragma unroll
          for (int d = 0; d < ND; ++d) {
            R bre, bim;
            if constexpr (STG) BinIO<Bin>::load(sw + d * WST + (idx - sb), bre, bim);
            else BinIO<Bin>::load(rp[d] + idx, bre, bim);
            cre[d] = fma(bre, h, cre[d]);
            cim[d] = fma(bim, h, cim[d]);
          }
        }
      };
      if (stg) drun(std::true_type{});
      else drun(std::false_type{});
    } else if constexpr (KERN == KERN_FRESNEL && PREC == SFT_PREC_FP64) {
      // FP64 Fresnel weights, bin by bin.  With b = |beta|, the mirror x' = ds - jj (ds = +-delta,
      // jj = +-j, the lower signs for beta < 0, where F(x, beta) = conj F(-x, b)) and
      // p-+ = x' -+ b / 2:
      //   H_j = (-1)^j F(x, beta) = cj[ e(p-) E- - e(p+) E+
      //                                 + [p- < 0 <= p+] (-1)^jj (1+i) exp(-i pi x'^2 / b) / sqrt(2 b) ],
      // e(p) = sgn(p) G(sqrt(2 / b) |p|) / sqrt(2 b), E-+ = exp(i pi (-+ds + b / 4)), cj the
      // conjugate for beta < 0, G from fresnel_aux64.
      const bool neg = ch.beta < 0.0;
      const double b = fabs(ch.beta);
      const double ds = neg ? -delta : delta;
      const double isq2b = 1.0 / sqrt(2.0 * b), sq2ob = sqrt(2.0 / b);
      double emr, emi, epr, epi;
      sincos(kPi * (0.25 * b - ds), &emi, &emr);
      sincos(kPi * (0.25 * b + ds), &epi, &epr);
      auto frun = [&](auto stgc) {
        constexpr bool STG = decltype(stgc)::value;
        for (int t = 0; t <= 2 * K; ++t) {
          const int j = bin_order(t, K);
          const int idx = i0 + j + K;
          if (!STG && !inband && (idx < 0 || idx >= a.n_ext)) {
            fl |= kFlagOOB;
            continue;
          }
          const int jj = neg ? -j : j;
          const double xq = ds - (double)jj;
          const double pm = xq - 0.5 * b, pp = xq + 0.5 * b;
          const double2 gm = fresnel_aux64(fabs(pm) * sq2ob), gp = fresnel_aux64(fabs(pp) * sq2ob);
          const double sm = pm < 0.0 ? -isq2b : isq2b, sq = pp < 0.0 ? -isq2b : isq2b;
          double hr = sm * (gm.x * emr - gm.y * emi) - sq * (gp.x * epr - gp.y * epi);
          double hi = sm * (gm.x * emi + gm.y * emr) - sq * (gp.x * epi + gp.y * epr);
          if (pm < 0.0 && pp >= 0.0) {
            // |x'| <= b / 2 here, so x'^2 / b <= b / 4 needs no special reduction
            double st, ct;
            sincos(kPi * (xq * xq / b), &st, &ct);
            const double sg = (jj & 1) ? -isq2b : isq2b;
            hr = fma(sg, ct + st, hr);
            hi = fma(sg, ct - st, hi);
          }
          if (neg) hi = -hi;
#pragma unroll
          for (int d = 0; d < ND; ++d) {
            R bre, bim;
            if constexpr (STG) BinIO<Bin>::load(sw + d * WST + (idx - sb), bre, bim);
            else BinIO<Bin>::load(rp[d] + idx, bre, bim);
            cre[d] = fma(bre, hr, fma(-bim, hi, cre[d]));
            cim[d] = fma(bre, hi, fma(bim, hr, cim[d]));
          }
        }
      };
      if (stg) frun(std::true_type{});
      else frun(std::false_type{});
    } else if constexpr (KERN == KERN_FRESNEL) {
      // Fresnel weights; beta < 0 through F(x, beta) = conj F(-x, -beta).  The endpoint
      // phasors E-+ are common to all bins, so the bins accumulate b e(p-) and b e(p+)
      // and the phasors are applied once: C = E- S- - E+ S+ + S_stat.
      const bool neg = ch.beta < 0.0;
      const double bpos = fabs(ch.beta);
      const double ds64 = neg ? -delta : delta;
      const float bp = (float)bpos;
      const float ds = (float)ds64;
      const float rsb = rsqrtf(bp);
      const float sq2ob = 1.41421356237309505f * rsb;         // sqrt(2 / beta)
      const float isq2b = 0.70710678118654752f * rsb;         // 1 / sqrt(2 beta)
      const float tsc = 6.28318530717958648f * isq2b;         // 2 pi / sqrt(2 beta)
      const float bq = bp * kInvTwoPiF;                       // beta / (2 pi)
      const float dm = ds - 0.5f * bp, dp = ds + 0.5f * bp;   // p-+ of bin j are dm - j, dp - j
      // E- = exp(i(-pi delta + pi beta / 4)) from its own FP64-reduced phase (it scales every
      // term of the SFT, the stationary ones included), exp(i pi delta), rho = exp(2 pi i delta)
      // = E+ / E-, and E+ = E- rho
      float emi, emr, sd, cd;
      phasor(0.25 * kPi * bpos - kPi * ds64, emi, emr);
      phasor(kPi * ds64, sd, cd);
      const float rr = fmaf(cd, cd, -sd * sd), ri = 2.0f * cd * sd;
      const float epr = fmaf(emr, rr, -emi * ri), epi = fmaf(emr, ri, emi * rr);   // E+
      // 1 / beta and p- of bin 0 in FP64 for the stationary phase: FP32 estimate + two Newton steps
      double ib = (double)fast_rcp(bp);
      ib = ib * fma(-bpos, ib, 2.0);
      ib = ib * fma(-bpos, ib, 2.0);
      const double dm64 = ds64 - 0.5 * bpos;
      // Run-time K kernels (windows up to 129 bins, drifts beyond a hundred bins): p-+ of bin jj
      // as an exact integer plus an FP32 fraction split from the FP64 values, each rounded once
      // (to ulp(|p|) / 2); dm - jj in FP32 carries the rounding of beta / 2 (~ulp(beta)) into
      // every bin.  The compile-time windows (drift up to a few tens of bins) keep dm - jj: the
      // split costs them registers (a larger spill, ~5% of the ground scan).
      constexpr bool PSPLIT = KC < 0;
      const double dp64 = ds64 + 0.5 * bpos;
      const double nmr = PSPLIT ? rint(dm64) : 0.0, npr = PSPLIT ? rint(dp64) : 0.0;
      const int nmi = (int)nmr, npi = (int)npr;
      const float fm = (float)(dm64 - nmr), fpf = (float)(dp64 - npr);
      // central bin from its direct series (small drift and small delta)
      const bool cser = bp <= SFT_SERIES_BETA && fabsf(ds) <= SFT_SERIES_DELTA;
      // one row: sums of b e(p-) and b e(p+) (unused with several rows)
      // Bin sums: FP32 for the compile-time windows (17 or 65 bins); FP64 for the run-time K
      // kernels (windows up to 129 bins, where a plain FP32 running sum loses ~eps sqrt(N/2)
      // ~ 5e-7 of the SFT's term), with the products still formed in FP32.
      using BS = typename std::conditional<(KC < 0 && PREC != SFT_PREC_FP64), double, float>::type;
      BS smr = 0, smi = 0, spr = 0, spi = 0;
      BS wre[ND], wim[ND];
#pragma unroll
      for (int d = 0; d < ND; ++d) wre[d] = wim[d] = (BS)0;
      // Outer bins: jj >= jup or jj <= jdn puts both endpoints of a lane at or beyond the
      // asymptotic threshold |p| = SFT_G_VASYM sqrt(beta / 2), with no stationary point inside
      // the SFT (p- and p+ of one sign): jj >= dp + SFT_G_VASYM sqrt(beta / 2) gives
      // p+ = dp - jj <= -SFT_G_VASYM sqrt(beta / 2) (the rounding of the bound moves v by a
      // few ulp, where the dropped series terms stay below 1e-8 of the term).  With the bounds
      // taken over the active lanes of the wavefront, those bins take the asymptotic form
      // directly, without the per-lane range test.  Lane bounds are clamped to the window,
      // [-K-1, K+1], and keep the central bin jj = 0 out of the outer segments (it takes the
      // table path, or the direct series of a small-drift lane).
      // The same bounds for the larger thresholds at which the series may stop after one or
      // no power of W (ju1/jd1, ju0/jd0) nest outside jup/jdn:
      //   jd0 <= jd1 <= jdn < 0 < jup <= ju1 <= ju0.
      // Used for windows of SFT_OUTER_MIN_K bins or more a side (otherwise every bin takes
      // the table path).
      int jup = K + 1, jdn = -K - 1, ju1 = K + 1, jd1 = -K - 1, ju0 = K + 1, jd0 = -K - 1;
      if (K >= SFT_OUTER_MIN_K) {
        const float shb = bp * isq2b;   // sqrt(beta / 2) = beta / sqrt(2 beta)
        auto up = [&](float vt) {
          return (int)fminf(fmaxf(ceilf(fmaf(vt, shb, dp)), 1.0f), (float)(K + 1));
        };
        auto dn = [&](float vt) {
          return -(int)fmaxf(fminf(floorf(fmaf(-vt, shb, dm)), -1.0f), (float)(-K - 1));
        };
        jup = wave_max_active(up(SFT_G_VASYM), -K - 1, K + 1);
        jdn = -wave_max_active(dn(SFT_G_VASYM), -K - 1, K + 1);
        ju1 = wave_max_active(up(SFT_VASYM_W1), jup, K + 1);
        jd1 = -wave_max_active(dn(SFT_VASYM_W1), -jdn, K + 1);
        ju0 = wave_max_active(up(SFT_VASYM_W0), ju1, K + 1);
        jd0 = -wave_max_active(dn(SFT_VASYM_W0), -jd1, K + 1);
      }
      // E-+ / 2 pi with the imaginary parts of the beta < 0 mirror
      const float eqr = kInvTwoPiF * emr, eqy = kInvTwoPiF * (neg ? -emi : emi);
      const float fqr = kInvTwoPiF * epr, fqy = kInvTwoPiF * (neg ? -epi : epi);
      // rho (conjugated by the mirror): the bin weight is (E- / 2 pi) (e(p-) - rho e(p+))
      const float rhr = rr, rhi = neg ? -ri : ri;
      // One bin jj (jj = -j for beta < 0) of series tier TR: 0, 1 or 3 the asymptotic form cut
      // after TR powers of W, 4 the table with the stationary-point check (nothing for the
      // central bin of a small-drift lane, which is added after the loop).
      auto bin = [&](auto negc, auto checked, auto stgc, auto tierc, int jj) {
        constexpr bool NEG = decltype(negc)::value;
        constexpr bool CHK = decltype(checked)::value;
        constexpr bool STG = decltype(stgc)::value;
        constexpr int TR = decltype(tierc)::value;
        const int j = NEG ? -jj : jj;
        const int idx = i0 + j + K;
        if constexpr (CHK) {
          if (idx < 0 || idx >= a.n_ext) {
            fl |= kFlagOOB;
            return;
          }
        }
        // the bins first, so that their loads are in flight while the weights are formed
        float bre[ND], bim[ND];
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          if constexpr (STG) BinIO<Bin>::load(sw + d * WST + (idx - sb), bre[d], bim[d]);
          else BinIO<Bin>::load(rp[d] + idx, bre[d], bim[d]);
        }
        float pm, pp;
        if constexpr (PSPLIT) {
          pm = (float)(nmi - jj) + fm;
          pp = (float)(npi - jj) + fpf;
        } else {
          pm = dm - (float)jj;
          pp = dp - (float)jj;
        }
        float2 em, ep;
        if constexpr (TR < 4) {
          em = fres_endpoint_asym<TR>(pm, bq);
          ep = fres_endpoint_asym<TR>(pp, bq);
          if (NEG) {
            em.y = -em.y;
            ep.y = -ep.y;
          }
        } else {
          em = fres_endpoint2<ND == 1>(pm, bq, sq2ob, tsc, tab);
          ep = fres_endpoint2<ND == 1>(pp, bq, sq2ob, tsc, tab);
          if (NEG) {
            em.y = -em.y;
            ep.y = -ep.y;
          }
          if (pm < 0.0f && pp >= 0.0f) {
            // stationary point inside the SFT: h = (-1)^j (1+i) exp(-i pi x^2 / beta) / sqrt(2 beta),
            // x = delta - j, carried inside e(p-), which the sums multiply by E- / 2 pi.  As
            // x^2 - delta beta + beta^2 / 4 = (p-)^2 + j beta with j an integer,
            //   h / (E- / 2 pi) = 2 pi (1+i) exp(-i pi (p-)^2 / beta) / sqrt(2 beta),
            // with p- = delta - beta/2 - j and its phase reduced in FP64
            const double p64 = dm64 - (double)jj;
            const double hq = p64 * p64 * ib;
            float sr, cr;
            phasor(kPi * (hq - 2.0 * rint(0.5 * hq)), sr, cr);
            em.x += tsc * (cr + sr);
            em.y += NEG ? -tsc * (cr - sr) : tsc * (cr - sr);
          }
          if (jj == 0 && cser) {
            // central bin of a small-drift lane: added after the loop from its series
            em = make_float2(0.f, 0.f);
            ep = make_float2(0.f, 0.f);
          }
        }
        if constexpr (ND >= 2) {
          // several rows share the bin's weight H' = e(p-) - rho e(p+): one complex MAC per
          // row, E- / 2 pi applied once per row after the loop
          const float hr = fmaf(-rhr, ep.x, fmaf(rhi, ep.y, em.x));
          const float hi = fmaf(-rhr, ep.y, fmaf(-rhi, ep.x, em.y));
#pragma unroll
          for (int d = 0; d < ND; ++d) {
            if constexpr (std::is_same<BS, float>::value) {
              wre[d] = fmaf(bre[d], hr, fmaf(-bim[d], hi, wre[d]));
              wim[d] = fmaf(bre[d], hi, fmaf(bim[d], hr, wim[d]));
            } else {
              wre[d] += (BS)fmaf(bre[d], hr, -bim[d] * hi);
              wim[d] += (BS)fmaf(bre[d], hi, bim[d] * hr);
            }
          }
        } else {
          // one row: the bins accumulate b e(p-) and b e(p+)
          if constexpr (std::is_same<BS, float>::value) {
            smr = fmaf(bre[0], em.x, fmaf(-bim[0], em.y, smr));
            smi = fmaf(bre[0], em.y, fmaf(bim[0], em.x, smi));
            spr = fmaf(bre[0], ep.x, fmaf(-bim[0], ep.y, spr));
            spi = fmaf(bre[0], ep.y, fmaf(bim[0], ep.x, spi));
          } else {
            smr += (BS)fmaf(bre[0], em.x, -bim[0] * em.y);
            smi += (BS)fmaf(bre[0], em.y, bim[0] * em.x);
            spr += (BS)fmaf(bre[0], ep.x, -bim[0] * ep.y);
            spi += (BS)fmaf(bre[0], ep.y, bim[0] * ep.x);
          }
        }
      };
      // The bins as segments of one series tier each (bounds wave-uniform, so no per-bin
      // tier test), from the window's edges inwards: the smallest terms enter the FP32 sums
      // first and the central table bins last.
      auto run = [&](auto negc, auto checked, auto stgc) {
        using I0 = std::integral_constant<int, 0>;
        using I1 = std::integral_constant<int, 1>;
        using I3 = std::integral_constant<int, 3>;
        using I4 = std::integral_constant<int, 4>;
        for (int jj = -K; jj <= jd0; ++jj) bin(negc, checked, stgc, I0{}, jj);
        for (int jj = K; jj >= ju0; --jj) bin(negc, checked, stgc, I0{}, jj);
        for (int jj = jd0 + 1; jj <= jd1; ++jj) bin(negc, checked, stgc, I1{}, jj);
        for (int jj = ju0 - 1; jj >= ju1; --jj) bin(negc, checked, stgc, I1{}, jj);
        for (int jj = jd1 + 1; jj <= jdn; ++jj) bin(negc, checked, stgc, I3{}, jj);
        for (int jj = ju1 - 1; jj >= jup; --jj) bin(negc, checked, stgc, I3{}, jj);
        for (int jj = jdn + 1; jj < jup; ++jj) bin(negc, checked, stgc, I4{}, jj);
      };
      if (stg) {
        if (neg) run(std::true_type{}, std::false_type{}, std::true_type{});
        else run(std::false_type{}, std::false_type{}, std::true_type{});
      } else {
        if (neg) run(std::true_type{}, std::true_type{}, std::false_type{});
        else run(std::false_type{}, std::true_type{}, std::false_type{});
      }
      if constexpr (ND == 1) {
        // one row: the bins accumulated b e(p-) and b e(p+); apply the phasors once
        const float sr = (float)smr, si = (float)smi, qr = (float)spr, qi = (float)spi;
        cre[0] = (eqr * sr - eqy * si) - (fqr * qr - fqy * qi);
        cim[0] = (eqr * si + eqy * sr) - (fqr * qi + fqy * qr);
      } else {
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          const float cr = (float)wre[d], ci = (float)wim[d];
          cre[d] = eqr * cr - eqy * ci;
          cim[d] = eqr * ci + eqy * cr;
        }
      }
      // Central bin of a lane with small drift and small delta: its weight F(delta, beta) from
      // the direct series (the two endpoint terms are large there and cancel to a weight near
      // 1), evaluated here, outside the bin loops, and contracted with each row's bin k0.
      const int i_c = i0 + K;
      if (cser && (stg || (i_c >= 0 && i_c < a.n_ext))) {
        const float dl = (float)dm64 + 0.5f * bp;   // delta (mirrored for beta < 0)
        const float2 F = fres_central_series(neg ? -dl : dl, neg ? -bp : bp);
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          float bre, bim;
          if (stg) BinIO<Bin>::load(sw + d * WST + (i_c - sb), bre, bim);
          else BinIO<Bin>::load(rp[d] + i_c, bre, bim);
          cre[d] = fmaf(bre, F.x, fmaf(-bim, F.y, cre[d]));
          cim[d] = fmaf(bre, F.y, fmaf(bim, F.x, cim[d]));
        }
      }
    }
    // term_d = (-1)^{k0} A exp(i phi) C_d
    R pc, ps;
    if constexpr (PREC == SFT_PREC_FP64) {
      const double ph = reduce_2pi(ch.phase);
      double s_, c_;
      sincos(ph, &s_, &c_);
      ps = (R)s_;
      pc = (R)c_;
    } else {
      float s_, c_;
      phasor(ch.phase, s_, c_);
      ps = s_;
      pc = c_;
    }
    const R amp = (R)ch.amp;
    const R as = (k0 & 1) ? -amp : amp;
    const R apc = as * pc, aps = as * ps;
    // norm term A^2 T / S(f), S linear between bins floor(kappa) and floor(kappa) + 1
    const double kfl = floor(ch.kappa);
    const int ip = (int)kfl - a.k_lo;
    const bool psd_in = ip >= 0 && ip + 1 < a.n_bins;
    const R w = (R)(ch.kappa - kfl);
    const R a2t = amp * amp * (R)T;
    // the rows of the group are summed plainly, then the group enters the running
    // (compensated) sums once
    R gzpr = 0, gzpi = 0, gzxr = 0, gzxi = 0, ghp = 0, ghx = 0, ghpx = 0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      if (!act[d]) continue;
      const R tre = apc * cre[d] - aps * cim[d];
      const R tim = apc * cim[d] + aps * cre[d];
      const R fpa = (R)a.fp[rows[d]];
      const R fxa = (R)a.fx[rows[d]];
      gzpr = fma(fpa, tre, gzpr);
      gzpi = fma(fpa, tim, gzpi);
      gzxr = fma(fxa, tre, gzxr);
      gzxi = fma(fxa, tim, gzxi);
      if (!psd_in) {
        fl |= kFlagOOB;
        continue;
      }
      const R S0 = (R)psd[(int64_t)rows[d] * a.n_bins + ip];
      const R S1 = (R)psd[(int64_t)rows[d] * a.n_bins + ip + 1];
      if (!(S0 > (R)0) || !(S1 > (R)0)) {
        fl |= kFlagOOB;
        continue;
      }
      const R S = ((R)1 - w) * S0 + w * S1;
      R hterm;
      if constexpr (PREC == SFT_PREC_FP64) hterm = a2t / S;
      else hterm = a2t * (R)fast_rcp((float)S);
      ghp = fma(fpa * fpa, hterm, ghp);
      ghx = fma(fxa * fxa, hterm, ghx);
      if constexpr (FS != 0) ghpx = fma(fpa * fxa, hterm, ghpx);
    }
    zpr.add(gzpr);
    zpi.add(gzpi);
    zxr.add(gzxr);
    zxi.add(gzxi);
    hp.add(ghp);
    hx.add(ghx);
    if constexpr (FS != 0) hpx.add(ghpx);
  }

  const int64_t n = a.n_tmpl;
  double* p = a.part + (int64_t)c * (6 + FS) * n + m;
  p[0] = zpr.get();
  p[n] = zpi.get();
  p[2 * n] = zxr.get();
  p[3 * n] = zxi.get();
  p[4 * n] = hp.get();
  p[5 * n] = hx.get();
  if constexpr (FS != 0) p[6 * n] = hpx.get();
  a.pflags[(int64_t)c * n + m] = fl;
}

// ---------------------------------------------------------------------------- dispatch
// Newtonian: every detector-group width 1..4.  3.5PN: widths 1 and 4 (groups of 2 or 3
// rows run in the width-4 kernel, whose absent rows are skipped by a uniform test).
template <typename Bin, int PREC, int KERN, int KC, int WF, int FS, int REF = 0>
static ScanFn pick_nd(int nd)
{
  if constexpr (WF == WF_NEWTON) {
    switch (nd) {
    case 1: return scan_kernel<Bin, PREC, KERN, KC, 1, WF, FS, 0, REF>;
    case 2: return scan_kernel<Bin, PREC, KERN, KC, 2, WF, FS, 0, REF>;
    case 3: return scan_kernel<Bin, PREC, KERN, KC, 3, WF, FS, 0, REF>;
    default: return scan_kernel<Bin, PREC, KERN, KC, 4, WF, FS, 0, REF>;
    }
  } else {
    return nd == 1 ? scan_kernel<Bin, PREC, KERN, KC, 1, WF, FS, 0, REF> : scan_kernel<Bin, PREC, KERN, KC, 4, WF, FS, 0, REF>;
  }
}

// Start reference: the run-time-K kernels only (any K), so that the compile-time windows of the
// benchmark shapes carry no code for it.
template <typename Bin, int PREC, int WF, int FS = 0>
static ScanFn pick_start(int kern, int nd)
{
  return kern == KERN_DIRICHLET ? pick_nd<Bin, PREC, KERN_DIRICHLET, -1, WF, FS, 1>(nd)
                                : pick_nd<Bin, PREC, KERN_FRESNEL, -1, WF, FS, 1>(nd);
}

// FP64: the Dirichlet kernel with a compile-time window for K = 4 and a run-time one otherwise;
// the FP64 Fresnel weights (a reference mode, dominated by their special functions) with the
// run-time window only.
template <typename Bin, int PREC, int KERN, int WF, int FS = 0>
static ScanFn pick_k(int K, int nd)
{
  if constexpr (PREC == SFT_PREC_FP64) {
    if constexpr (KERN == KERN_FRESNEL) return pick_nd<Bin, PREC, KERN, -1, WF, FS>(nd);
    return K == 4 ? pick_nd<Bin, PREC, KERN, 4, WF, FS>(nd) : pick_nd<Bin, PREC, KERN, -1, WF, FS>(nd);
  } else {
    // one-row Fresnel scans with K = 32 (space-like banks) get a compile-time window too
    if constexpr (KERN == KERN_FRESNEL && WF == WF_NEWTON)
      if (K == 32 && nd == 1) return scan_kernel<Bin, PREC, KERN, 32, 1, WF, FS>;
    return K == 8 ? pick_nd<Bin, PREC, KERN, 8, WF, FS>(nd) : pick_nd<Bin, PREC, KERN, -1, WF, FS>(nd);
  }
}

template <typename Bin, int PREC, int WF, int FS = 0>
static ScanFn pick_kern(int kern, int K, int nd)
{
  return kern == KERN_DIRICHLET ? pick_k<Bin, PREC, KERN_DIRICHLET, WF, FS>(K, nd)
                                : pick_k<Bin, PREC, KERN_FRESNEL, WF, FS>(K, nd);
}

// Doppler form: one row per timestamp group
template <typename Bin, int PREC, int KERN, int FS>
static ScanFn pick_doppler_k(int K)
{
  if constexpr (PREC == SFT_PREC_FP64) {
    if constexpr (KERN == KERN_FRESNEL) return scan_kernel<Bin, PREC, KERN, -1, 1, WF_NEWTON, FS, 1>;
    return K == 4 ? scan_kernel<Bin, PREC, KERN, 4, 1, WF_NEWTON, FS, 1> : scan_kernel<Bin, PREC, KERN, -1, 1, WF_NEWTON, FS, 1>;
  } else {
    if constexpr (KERN == KERN_FRESNEL)
      if (K == 32) return scan_kernel<Bin, PREC, KERN, 32, 1, WF_NEWTON, FS, 1>;
    return K == 8 ? scan_kernel<Bin, PREC, KERN, 8, 1, WF_NEWTON, FS, 1> : scan_kernel<Bin, PREC, KERN, -1, 1, WF_NEWTON, FS, 1>;
  }
}

template <typename Bin, int PREC>
static ScanFn pick_wf(int wf, int kern, int K, int nd)
{
  switch (wf) {
  case WF_PN35: return pick_kern<Bin, PREC, WF_PN35>(kern, K, nd);
  case WF_TABLE: return pick_kern<Bin, PREC, WF_TABLE>(kern, K, nd);
  default: return pick_kern<Bin, PREC, WF_NEWTON>(kern, K, nd);
  }
}

}  // namespace sftk
