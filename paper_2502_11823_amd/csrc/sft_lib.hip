// sft_lib.hip -- libsft.so: C ABI (include/sft.h) and gfx950 kernels for the
// short-Fourier-transform inner product of Tenorio & Gerosa (arXiv:2502.11823).
//
// Kernels
//   load_kernel     : per-SFT whitening d~ = 2 x~ / S (Sec. III.B), conjugation,
//                     DC/Nyquist mirroring (footnote of Sec. III.C), conversion to the
//                     storage precision, PSD masking.  Once per dataset.
//   scan_kernel     : one template per lane, one SFT chunk per grid row.  For every
//                     SFT of the chunk: FP64 chirp at the SFT midpoint, FP64 phase
//                     reduction, FP64 bin split, 2K+1 kernel weights and the bin
//                     contraction (Eq. with_f_1), the coherent accumulation of
//                     Eq. efficient and of the norm, in FP64 or FP32 (Kahan or plain).
//                     Writes one partial per (template, chunk).
//   finalize_kernel : sums the partials of a template in chunk order (FP64), forms
//                     rho (Eq. det_short) and the flags.
// Reductions are in a fixed order, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <type_traits>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sft.h"
#include "sft_device.h"
#include "sft_mlp.h"

using namespace sftk;

// ============================================================================ errors
static thread_local std::string g_err;

static sft_status fail(sft_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static sft_status fail(sft_status st, const char* fmt, ...)
{
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_OR_FAIL(call)                                                                 \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(e_ == hipErrorOutOfMemory ? SFT_E_NOMEM : SFT_E_DEVICE, "%s: %s (%s:%d)", \
                  #call, hipGetErrorString(e_), __FILE__, __LINE__);                      \
  } while (0)

sft_status sft_set_error(sft_status st, const char* msg)
{
  g_err = msg;
  return st;
}

extern "C" const char* sft_last_error(void) { return g_err.c_str(); }
extern "C" const char* sft_version(void) { return "libsft 0.1.0 gfx950"; }

// ============================================================================ kernel timing
#include <mutex>
#include <vector>
static std::mutex g_tmu;
static std::vector<hipEvent_t> g_ev;   // pairs: [2i] before, [2i+1] after the scan kernel of record i
static int32_t g_tcap = 0, g_tused = 0;

static void timing_drop()
{
  for (hipEvent_t e : g_ev) (void)hipEventDestroy(e);
  g_ev.clear();
  g_tcap = g_tused = 0;
}

extern "C" sft_status sft_kernel_timing(int32_t n)
{
  std::lock_guard<std::mutex> lk(g_tmu);
  timing_drop();
  if (n <= 0) return SFT_OK;
  if (n > 4096) return fail(SFT_E_RANGE, "sft_kernel_timing: at most 4096 records");
  g_ev.resize(2 * (size_t)n, nullptr);
  for (auto& e : g_ev) {
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) {
      e = nullptr;
      timing_drop();
      return fail(SFT_E_DEVICE, "sft_kernel_timing: hipEventCreate: %s", hipGetErrorString(r));
    }
  }
  g_tcap = n;
  return SFT_OK;
}

extern "C" int32_t sft_kernel_times(float* ms, int32_t max)
{
  std::lock_guard<std::mutex> lk(g_tmu);
  for (int32_t i = 0; i < g_tused && i < max; ++i) {
    float t = -1.f;
    if (hipEventSynchronize(g_ev[2 * i + 1]) == hipSuccess &&
        hipEventElapsedTime(&t, g_ev[2 * i], g_ev[2 * i + 1]) != hipSuccess)
      t = -1.f;
    if (ms) ms[i] = t;
  }
  return g_tused;
}

// returns the event pair for this scan, or nulls when not recording
static void timing_slot(hipEvent_t* b, hipEvent_t* e)
{
  std::lock_guard<std::mutex> lk(g_tmu);
  *b = *e = nullptr;
  if (g_tused < g_tcap) {
    *b = g_ev[2 * g_tused];
    *e = g_ev[2 * g_tused + 1];
    ++g_tused;
  }
}

// ============================================================================ data handle
// Rows that share a start time (detectors of one network) form a timestamp group;
// a group holds at most this many rows (more rows at one time start another group).
#define SFT_GROUP_MAX 4
struct sft_data {
  int device;
  int32_t n_sft, n, k_lo, n_bins, storage;
  int32_t n_ext, k_ext_lo;  // stored rows cover bins k_ext_lo .. k_ext_lo + n_ext - 1 (mirrors included)
  double T;
  void* bins;     // [n_sft][n_ext] conj(2 x~ / S) in the storage type
  void* psd;      // [n_sft][n_bins] S (double for F64 storage, float otherwise); masked -> 0
  double* fp;     // [n_sft]
  double* fx;     // [n_sft]
  // timestamp groups: rows with equal start times (one per detector), in time order
  int32_t n_groups, nd;   // group count, largest group size (<= SFT_GROUP_MAX)
  double* g_tmid;         // [n_groups] SFT midpoint t_start + T/2
  int32_t* g_rows;        // [n_groups][SFT_GROUP_MAX] rows, -1 = absent
  int32_t cu_count;       // compute units of the device
  sft_tuning tune;        // launch shape of the scans on this handle (0 fields = automatic)
};

template <typename Bin> __device__ inline void store_bin(Bin* p, double re, double im);
template <> __device__ inline void store_bin<double2>(double2* p, double re, double im) { *p = make_double2(re, im); }
template <> __device__ inline void store_bin<float2>(float2* p, double re, double im) { *p = make_float2((float)re, (float)im); }
template <> __device__ inline void store_bin<bf16x2>(bf16x2* p, double re, double im)
{
  bf16x2 v;
  v.re = f32_to_bf16((float)re);
  v.im = f32_to_bf16((float)im);
  *p = v;
}

template <typename Bin, typename PS>
__global__ __launch_bounds__(256) void load_kernel(const double* __restrict__ xb, const double* __restrict__ psd,
                                                   int32_t n_sft, int32_t n, int32_t k_lo, int32_t n_bins,
                                                   int32_t n_ext, int32_t k_ext_lo,
                                                   Bin* __restrict__ bins, PS* __restrict__ psd_out)
{
  int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = (int64_t)n_sft * n_ext;
  if (gid >= total) return;
  int64_t a = gid / n_ext;
  int32_t e = (int32_t)(gid - a * n_ext);
  int32_t k = k_ext_lo + e;
  bool cj = false;
  int32_t km = k;
  if (km < 0) { km = -km; cj = true; }
  else if (km > n / 2) { km = n - km; cj = true; }
  int32_t i = km - k_lo;
  double re = 0.0, im = 0.0;
  if (i >= 0 && i < n_bins) {
    double S = psd[a * n_bins + i];
    if (S > 0.0 && S <= 1.79769313486231570e308) {
      re = 2.0 * xb[2 * (a * n_bins + i)] / S;
      im = 2.0 * xb[2 * (a * n_bins + i) + 1] / S;
      if (cj) im = -im;
      im = -im;  // stored operand is conj(d~)
    }
  }
  store_bin<Bin>(bins + gid, re, im);
  // the PSD rows (original band only)
  if (!cj && k >= k_lo && k < k_lo + n_bins) {
    double S = psd[a * n_bins + (k - k_lo)];
    psd_out[a * n_bins + (k - k_lo)] = (S > 0.0 && S <= 1.79769313486231570e308) ? (PS)S : (PS)0;
  }
}

// Group rows by start time: stable order by time, runs of equal t_start split into
// groups of at most SFT_GROUP_MAX rows.
static void build_groups(const double* t_start, int32_t n_sft, double T, std::vector<double>& tmid,
                         std::vector<int32_t>& rows, int32_t& nd)
{
  std::vector<int32_t> order(n_sft);
  for (int32_t i = 0; i < n_sft; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return t_start[x] < t_start[y]; });
  tmid.clear();
  rows.clear();
  nd = 1;
  int32_t i = 0;
  while (i < n_sft) {
    int32_t j = i;
    while (j < n_sft && j - i < SFT_GROUP_MAX && t_start[order[j]] == t_start[order[i]]) ++j;
    tmid.push_back(t_start[order[i]] + 0.5 * T);
    for (int32_t d = 0; d < SFT_GROUP_MAX; ++d) rows.push_back(i + d < j ? order[i + d] : -1);
    nd = std::max(nd, j - i);
    i = j;
  }
}

extern "C" sft_status sft_load_data(const sft_data_desc* d, const double* t_start, const double* x_bins,
                                    const double* psd, const double* fplus, const double* fcross,
                                    void* hip_stream, sft_data** out)
{
  if (!d || !t_start || !x_bins || !psd || !out) return fail(SFT_E_INVALID, "sft_load_data: null argument");
  *out = nullptr;
  if (d->n_sft < 1 || d->n_samples < 2 || (d->n_samples & 1) || !(d->t_sft > 0.0) || d->reserved != 0)
    return fail(SFT_E_INVALID, "sft_load_data: bad descriptor (n_sft=%d n=%d T=%g)", d->n_sft, d->n_samples, d->t_sft);
  if (d->k_lo < 0 || d->n_bins < 1 || d->k_lo + d->n_bins - 1 > d->n_samples / 2)
    return fail(SFT_E_INVALID, "sft_load_data: band [%d, %d) outside [0, n/2]", d->k_lo, d->k_lo + d->n_bins);
  if (d->storage != SFT_STORE_F64 && d->storage != SFT_STORE_F32 && d->storage != SFT_STORE_BF16)
    return fail(SFT_E_INVALID, "sft_load_data: unknown storage %d", d->storage);
  hipStream_t st = (hipStream_t)hip_stream;
  sft_data* h = new sft_data();
  std::memset(h, 0, sizeof(*h));
  HIP_OR_FAIL(hipGetDevice(&h->device));
  if (hipDeviceGetAttribute(&h->cu_count, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess ||
      h->cu_count < 1)
    h->cu_count = 256;
  h->n_sft = d->n_sft;
  h->n = d->n_samples;
  h->k_lo = d->k_lo;
  h->n_bins = d->n_bins;
  h->storage = d->storage;
  h->T = d->t_sft;
  int32_t g_lo = d->k_lo == 0 ? std::min(SFT_K_MAX, d->n_bins - 1) : 0;
  int32_t g_hi = (d->k_lo + d->n_bins - 1 == d->n_samples / 2) ? std::min(SFT_K_MAX, d->n_bins - 1) : 0;
  h->k_ext_lo = d->k_lo - g_lo;
  h->n_ext = d->n_bins + g_lo + g_hi;
  size_t nb = (size_t)d->n_sft * d->n_bins;
  size_t ne = (size_t)d->n_sft * h->n_ext;
  size_t bin_sz = d->storage == SFT_STORE_F64 ? sizeof(double2) : d->storage == SFT_STORE_F32 ? sizeof(float2) : sizeof(bf16x2);
  size_t ps_sz = d->storage == SFT_STORE_F64 ? sizeof(double) : sizeof(float);
  double *dx = nullptr, *dp = nullptr, *dts = nullptr;
  auto cleanup = [&]() {
    if (dx) (void)hipFree(dx);
    if (dp) (void)hipFree(dp);
    if (dts) (void)hipFree(dts);
  };
  hipError_t e = hipSuccess;
  if ((e = hipMalloc(&h->bins, ne * bin_sz)) != hipSuccess || (e = hipMalloc(&h->psd, nb * ps_sz)) != hipSuccess ||
      (e = hipMalloc(&h->fp, d->n_sft * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&h->fx, d->n_sft * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&dx, nb * 2 * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&dp, nb * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&dts, d->n_sft * sizeof(double))) != hipSuccess) {
    cleanup();
    sft_free_data(h);
    return fail(e == hipErrorOutOfMemory ? SFT_E_NOMEM : SFT_E_DEVICE, "sft_load_data: hipMalloc: %s", hipGetErrorString(e));
  }
  std::string err;
  do {
    if ((e = hipMemcpyAsync(dx, x_bins, nb * 2 * sizeof(double), hipMemcpyHostToDevice, st)) != hipSuccess) break;
    if ((e = hipMemcpyAsync(dp, psd, nb * sizeof(double), hipMemcpyHostToDevice, st)) != hipSuccess) break;
    if ((e = hipMemcpyAsync(dts, t_start, d->n_sft * sizeof(double), hipMemcpyHostToDevice, st)) != hipSuccess) break;
    if (fplus) e = hipMemcpyAsync(h->fp, fplus, d->n_sft * sizeof(double), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) break;
    if (fcross) e = hipMemcpyAsync(h->fx, fcross, d->n_sft * sizeof(double), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) break;
    if (!fplus || !fcross) {
      // defaults F+ = 1, Fx = 0 staged from the host
      double* tmp = new double[d->n_sft];
      if (!fplus) {
        for (int i = 0; i < d->n_sft; i++) tmp[i] = 1.0;
        e = hipMemcpy(h->fp, tmp, d->n_sft * sizeof(double), hipMemcpyHostToDevice);
      }
      if (e == hipSuccess && !fcross) {
        for (int i = 0; i < d->n_sft; i++) tmp[i] = 0.0;
        e = hipMemcpy(h->fx, tmp, d->n_sft * sizeof(double), hipMemcpyHostToDevice);
      }
      delete[] tmp;
      if (e != hipSuccess) break;
    }
    unsigned blocks = (unsigned)((ne + 255) / 256);
    switch (d->storage) {
    case SFT_STORE_F64:
      hipLaunchKernelGGL((load_kernel<double2, double>), dim3(blocks), dim3(256), 0, st, dx, dp, h->n_sft, h->n, h->k_lo,
                         h->n_bins, h->n_ext, h->k_ext_lo, (double2*)h->bins, (double*)h->psd);
      break;
    case SFT_STORE_F32:
      hipLaunchKernelGGL((load_kernel<float2, float>), dim3(blocks), dim3(256), 0, st, dx, dp, h->n_sft, h->n, h->k_lo,
                         h->n_bins, h->n_ext, h->k_ext_lo, (float2*)h->bins, (float*)h->psd);
      break;
    default:
      hipLaunchKernelGGL((load_kernel<bf16x2, float>), dim3(blocks), dim3(256), 0, st, dx, dp, h->n_sft, h->n, h->k_lo,
                         h->n_bins, h->n_ext, h->k_ext_lo, (bf16x2*)h->bins, (float*)h->psd);
      break;
    }
    if ((e = hipGetLastError()) != hipSuccess) break;
    {
      std::vector<double> tmid;
      std::vector<int32_t> grows;
      build_groups(t_start, d->n_sft, h->T, tmid, grows, h->nd);
      h->n_groups = (int32_t)tmid.size();
      if ((e = hipMalloc(&h->g_tmid, tmid.size() * sizeof(double))) != hipSuccess) break;
      if ((e = hipMalloc(&h->g_rows, grows.size() * sizeof(int32_t))) != hipSuccess) break;
      if ((e = hipMemcpyAsync(h->g_tmid, tmid.data(), tmid.size() * sizeof(double), hipMemcpyHostToDevice, st)) != hipSuccess) break;
      if ((e = hipMemcpyAsync(h->g_rows, grows.data(), grows.size() * sizeof(int32_t), hipMemcpyHostToDevice, st)) != hipSuccess) break;
      e = hipStreamSynchronize(st);   // the host vectors go out of scope here
    }
  } while (0);
  cleanup();
  if (e != hipSuccess) {
    sft_free_data(h);
    return fail(SFT_E_DEVICE, "sft_load_data: %s", hipGetErrorString(e));
  }
  *out = h;
  return SFT_OK;
}

extern "C" void sft_free_data(sft_data* h)
{
  if (!h) return;
  if (h->bins) (void)hipFree(h->bins);
  if (h->psd) (void)hipFree(h->psd);
  if (h->g_tmid) (void)hipFree(h->g_tmid);
  if (h->g_rows) (void)hipFree(h->g_rows);
  if (h->fp) (void)hipFree(h->fp);
  if (h->fx) (void)hipFree(h->fx);
  delete h;
}

extern "C" void sft_default_opts(sft_opts* o)
{
  if (!o) return;
  o->K = 8;
  o->kernel = SFT_KERNEL_AUTO;
  o->precision = SFT_PREC_FP32_KAHAN;
  o->waveform = SFT_WF_NEWTON;
  o->beta_switch = 1e-7;
  o->a_plus = 1.0;
  o->a_cross = 0.0;
  o->tsun = 4.925490947641267e-6;
  o->delta_max = 0.0;
  o->surrogate = nullptr;
}

// ============================================================================ scan
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
  double* part;      // [n_chunks][6][n_tmpl]
  uint32_t* pflags;  // [n_chunks][n_tmpl]
  const double* wtab;  // chirp table (WF_TABLE): 5 planes [n_groups][n_tmpl] kappa, phase, amp, beta, dres
};

enum { KERN_DIRICHLET = 0, KERN_FRESNEL = 1 };
// WF_TABLE: the chirp of every (template, group) comes precomputed from a table (the
// surrogate path fills it); an internal value, never accepted from the caller
enum { WF_NEWTON = SFT_WF_NEWTON, WF_PN35 = SFT_WF_PN35, WF_TABLE = 100 };

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
template <typename Bin, int PREC, int KERN, int KC, int ND, int WF>
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

template <typename Bin, int PREC, int KERN, int KC, int ND, int WF>
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
    if (m < a.n_tmpl) scan_item<Bin, PREC, KERN, KC, ND, WF>(a, K, m, c, tab, stage + (threadIdx.x >> 6) * (ND * WST));
    if (!a.persistent) break;
  }
}

template <typename Bin, int PREC, int KERN, int KC, int ND, int WF>
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

  Acc zpr, zpi, zxr, zxi, hp, hx;
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
    const double tau = tc - tmid;
    if (!(tau > 0.0)) {
      fl |= kFlagTau;
      continue;
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
    if (a.delta_max > 0.0 && ch.dres > a.delta_max) fl |= kFlagTaylor;
    if (!(ch.kappa < 1.0e9)) {
      // frequency far above any stored band: no window bin and no norm bin exists
      fl |= kFlagOOB;
      continue;
    }
    const double kr = floor(ch.kappa + 0.5);
    const double delta = ch.kappa - kr;
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
      // central bin from its direct series (small drift and small delta)
      const bool cser = bp <= SFT_SERIES_BETA && fabsf(ds) <= SFT_SERIES_DELTA;
      // one row: sums of b e(p-) and b e(p+) (unused with several rows)
      float smr = 0.f, smi = 0.f, spr = 0.f, spi = 0.f;
      // Outer bins: jj >= jup or jj <= jdn puts both endpoints of a lane at least one bin
      // beyond the asymptotic threshold |p| = SFT_G_VASYM sqrt(beta / 2), with no stationary
      // point inside the SFT (p- and p+ of one sign).  With the bounds taken over the active
      // lanes of the wavefront, those bins take the asymptotic form directly, without the
      // per-lane range test.  Lane bounds are clamped to the window, [-K-1, K+1].
      // The same bounds for the larger thresholds at which the series may stop after one or
      // no power of W (ju1/jd1, ju0/jd0) nest outside jup/jdn:
      //   jd0 <= jd1 <= jdn < 0 < jup <= ju1 <= ju0.
      // Used for windows of SFT_OUTER_MIN_K bins or more a side (otherwise every bin takes
      // the table path).
      int jup = K + 1, jdn = -K - 1, ju1 = K + 1, jd1 = -K - 1, ju0 = K + 1, jd0 = -K - 1;
      if (K >= SFT_OUTER_MIN_K) {
        const float shb = bp * isq2b;   // sqrt(beta / 2) = beta / sqrt(2 beta)
        auto up = [&](float vt) {
          return (int)fminf(fmaxf(ceilf(fmaf(vt, shb, dp)) + 1.0f, (float)(-K - 1)), (float)(K + 1));
        };
        auto dn = [&](float vt) {
          return -(int)fminf(fmaxf(floorf(fmaf(-vt, shb, dm)) - 1.0f, (float)(-K - 1)), (float)(K + 1));
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
        const float pm = dm - (float)jj, pp = dp - (float)jj;
        float2 em, ep;
        if constexpr (TR < 4) {
          em = fres_endpoint_asym<TR>(pm, bq);
          ep = fres_endpoint_asym<TR>(pp, bq);
          if (NEG) {
            em.y = -em.y;
            ep.y = -ep.y;
          }
        } else {
          em = fres_endpoint2(pm, bq, sq2ob, tsc, tab);
          ep = fres_endpoint2(pp, bq, sq2ob, tsc, tab);
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
            cre[d] = fmaf(bre[d], hr, fmaf(-bim[d], hi, cre[d]));
            cim[d] = fmaf(bre[d], hi, fmaf(bim[d], hr, cim[d]));
          }
        } else {
          // one row: the bins accumulate b e(p-) and b e(p+)
          smr = fmaf(bre[0], em.x, fmaf(-bim[0], em.y, smr));
          smi = fmaf(bre[0], em.y, fmaf(bim[0], em.x, smi));
          spr = fmaf(bre[0], ep.x, fmaf(-bim[0], ep.y, spr));
          spi = fmaf(bre[0], ep.y, fmaf(bim[0], ep.x, spi));
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
        cre[0] = (eqr * smr - eqy * smi) - (fqr * spr - fqy * spi);
        cim[0] = (eqr * smi + eqy * smr) - (fqr * spi + fqy * spr);
      } else {
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          const R cr = cre[d];
          cre[d] = eqr * cr - eqy * cim[d];
          cim[d] = eqr * cim[d] + eqy * cr;
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
    R gzpr = 0, gzpi = 0, gzxr = 0, gzxi = 0, ghp = 0, ghx = 0;
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
    }
    zpr.add(gzpr);
    zpi.add(gzpi);
    zxr.add(gzxr);
    zxi.add(gzxi);
    hp.add(ghp);
    hx.add(ghx);
  }

  const int64_t n = a.n_tmpl;
  double* p = a.part + (int64_t)c * 6 * n + m;
  p[0] = zpr.get();
  p[n] = zpi.get();
  p[2 * n] = zxr.get();
  p[3 * n] = zxi.get();
  p[4 * n] = hp.get();
  p[5 * n] = hx.get();
  a.pflags[(int64_t)c * n + m] = fl;
}

__global__ __launch_bounds__(256) void finalize_kernel(const double* __restrict__ part, const uint32_t* __restrict__ pflags,
                                                       int64_t n, int32_t n_chunks, double a_plus, double a_cross,
                                                       double* __restrict__ zp, double* __restrict__ zx,
                                                       double* __restrict__ hhp, double* __restrict__ hhx,
                                                       double* __restrict__ rho, uint32_t* __restrict__ flags,
                                                       const uint32_t* __restrict__ xflags)
{
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  double v[6] = {0, 0, 0, 0, 0, 0};
  uint32_t fl = 0;
  for (int c = 0; c < n_chunks; ++c) {
    const double* p = part + (int64_t)c * 6 * n + m;
#pragma unroll
    for (int q = 0; q < 6; ++q) v[q] += p[q * n];
    fl |= pflags[(int64_t)c * n + m];
  }
  const double re = a_plus * v[0] + a_cross * v[3];
  const double im = a_plus * v[1] - a_cross * v[2];
  const double hh = a_plus * a_plus * v[4] + a_cross * a_cross * v[5];
  double r;
  if (!(hh > 0.0)) {
    r = 0.0;
    fl |= kFlagEmpty;
  } else {
    r = sqrt(re * re + im * im) / sqrt(hh);
  }
  bool fin = isfinite(r);
  for (int q = 0; q < 6; ++q) fin = fin && isfinite(v[q]);
  if (!fin) fl |= kFlagNonfinite;
  if (xflags) fl |= xflags[m];
  zp[2 * m] = v[0];
  zp[2 * m + 1] = v[1];
  zx[2 * m] = v[2];
  zx[2 * m + 1] = v[3];
  hhp[m] = v[4];
  hhx[m] = v[5];
  rho[m] = r;
  flags[m] = fl;
}

// ---------------------------------------------------------------------------- dispatch
using ScanFn = void (*)(ScanArgs);

// Newtonian: every detector-group width 1..4.  3.5PN: widths 1 and 4 (groups of 2 or 3
// rows run in the width-4 kernel, whose absent rows are skipped by a uniform test).
template <typename Bin, int PREC, int KERN, int KC, int WF>
static ScanFn pick_nd(int nd)
{
  if constexpr (WF == WF_NEWTON) {
    switch (nd) {
    case 1: return scan_kernel<Bin, PREC, KERN, KC, 1, WF>;
    case 2: return scan_kernel<Bin, PREC, KERN, KC, 2, WF>;
    case 3: return scan_kernel<Bin, PREC, KERN, KC, 3, WF>;
    default: return scan_kernel<Bin, PREC, KERN, KC, 4, WF>;
    }
  } else {
    return nd == 1 ? scan_kernel<Bin, PREC, KERN, KC, 1, WF> : scan_kernel<Bin, PREC, KERN, KC, 4, WF>;
  }
}

template <typename Bin, int PREC, int KERN, int WF>
static ScanFn pick_k(int K, int nd)
{
  if (PREC == SFT_PREC_FP64) return K == 4 ? pick_nd<Bin, PREC, KERN, 4, WF>(nd) : pick_nd<Bin, PREC, KERN, -1, WF>(nd);
  // one-row Fresnel scans with K = 32 (space-like banks) get a compile-time window too
  if constexpr (KERN == KERN_FRESNEL && WF == WF_NEWTON)
    if (K == 32 && nd == 1) return scan_kernel<Bin, PREC, KERN, 32, 1, WF>;
  return K == 8 ? pick_nd<Bin, PREC, KERN, 8, WF>(nd) : pick_nd<Bin, PREC, KERN, -1, WF>(nd);
}

template <typename Bin, int PREC, int WF>
static ScanFn pick_kern(int kern, int K, int nd)
{
  return kern == KERN_DIRICHLET ? pick_k<Bin, PREC, KERN_DIRICHLET, WF>(K, nd) : pick_k<Bin, PREC, KERN_FRESNEL, WF>(K, nd);
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

// wf: WF_NEWTON, WF_PN35 or WF_TABLE (the surrogate path)
static ScanFn pick_kernel(const sft_data* d, const sft_opts* o, int wf)
{
  const int kern = o->kernel == SFT_KERNEL_DIRICHLET ? KERN_DIRICHLET : KERN_FRESNEL;
  if (o->precision == SFT_PREC_FP64) {
    switch (wf) {
    case WF_PN35: return pick_k<double2, SFT_PREC_FP64, KERN_DIRICHLET, WF_PN35>(o->K, d->nd);
    case WF_TABLE: return pick_k<double2, SFT_PREC_FP64, KERN_DIRICHLET, WF_TABLE>(o->K, d->nd);
    default: return pick_k<double2, SFT_PREC_FP64, KERN_DIRICHLET, WF_NEWTON>(o->K, d->nd);
    }
  }
  if (d->storage == SFT_STORE_F32)
    return o->precision == SFT_PREC_FP32_KAHAN ? pick_wf<float2, SFT_PREC_FP32_KAHAN>(wf, kern, o->K, d->nd)
                                               : pick_wf<float2, SFT_PREC_FP32_NAIVE>(wf, kern, o->K, d->nd);
  return o->precision == SFT_PREC_FP32_KAHAN ? pick_kern<bf16x2, SFT_PREC_FP32_KAHAN, WF_NEWTON>(kern, o->K, d->nd)
                                             : pick_kern<bf16x2, SFT_PREC_FP32_NAIVE, WF_NEWTON>(kern, o->K, d->nd);
}

__global__ void zero_counter_kernel(int32_t* c)
{
  if (threadIdx.x == 0) c[0] = 0;
}

static sft_status validate_scan(const sft_data* d, const sft_opts* o)
{
  if (!d || !o) return fail(SFT_E_INVALID, "scan: null data or options");
  if (o->K < 0 || o->K > SFT_K_MAX) return fail(SFT_E_RANGE, "scan: K=%d outside [0, %d]", o->K, SFT_K_MAX);
  if (o->kernel != SFT_KERNEL_DIRICHLET && o->kernel != SFT_KERNEL_FRESNEL && o->kernel != SFT_KERNEL_AUTO)
    return fail(SFT_E_INVALID, "scan: unknown kernel %d", o->kernel);
  if (o->waveform != SFT_WF_NEWTON && o->waveform != SFT_WF_PN35 && o->waveform != SFT_WF_SURROGATE)
    return fail(SFT_E_INVALID, "scan: unknown waveform %d", o->waveform);
  if (o->waveform == SFT_WF_SURROGATE && !o->surrogate)
    return fail(SFT_E_INVALID, "scan: the surrogate waveform needs opts.surrogate");
  if (o->waveform != SFT_WF_NEWTON && d->storage == SFT_STORE_BF16)
    return fail(SFT_E_UNSUPPORTED, "scan: the 3.5PN and surrogate waveforms need F32 or F64 storage");
  if (o->waveform == SFT_WF_SURROGATE) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != o->surrogate->device)
      return fail(SFT_E_INVALID, "scan: the surrogate lives on device %d, not on the current device", o->surrogate->device);
  }
  if (!(o->tsun > 0.0)) return fail(SFT_E_INVALID, "scan: tsun must be positive");
  if (o->precision == SFT_PREC_FP64) {
    if (d->storage != SFT_STORE_F64) return fail(SFT_E_UNSUPPORTED, "scan: FP64 precision needs F64 storage");
    if (o->kernel != SFT_KERNEL_DIRICHLET) return fail(SFT_E_UNSUPPORTED, "scan: FP64 precision supports the Dirichlet kernel only");
  } else if (o->precision == SFT_PREC_FP32_KAHAN || o->precision == SFT_PREC_FP32_NAIVE) {
    if (d->storage == SFT_STORE_F64) return fail(SFT_E_UNSUPPORTED, "scan: FP32 precision needs F32 or BF16 storage");
  } else {
    return fail(SFT_E_INVALID, "scan: unknown precision %d", o->precision);
  }
  return SFT_OK;
}

static sft_status validate_io(const sft_bank* bank, int64_t n, const sft_out* out)
{
  if (!bank || !out) return fail(SFT_E_INVALID, "scan: null bank or output");
  if (n < 0) return fail(SFT_E_INVALID, "scan: negative template count");
  if (n == 0) return SFT_OK;
  if (!bank->mc || !bank->t_c) return fail(SFT_E_INVALID, "scan: bank.mc and bank.t_c are required");
  if (!out->zp || !out->zx || !out->hhp || !out->hhx || !out->rho || !out->flags)
    return fail(SFT_E_INVALID, "scan: every output array is required");
  if (n > (int64_t)INT32_MAX) return fail(SFT_E_RANGE, "scan: too many templates");
  return SFT_OK;
}

static sft_status validate_tuning(const sft_tuning* t)
{
  if (!t) return fail(SFT_E_INVALID, "tuning: null");
  if (t->block != 0 && t->block != 64 && t->block != 128 && t->block != 256)
    return fail(SFT_E_RANGE, "tuning: block must be 0, 64, 128 or 256 (got %d)", t->block);
  if (t->chunk_groups < 0) return fail(SFT_E_RANGE, "tuning: chunk_groups must be >= 0");
  if (t->persistent != 0 && t->persistent != 1) return fail(SFT_E_RANGE, "tuning: persistent must be 0 or 1");
  return SFT_OK;
}

// A scan prepared for launch: arguments, launch shape and workspace layout.
struct Prepared {
  ScanArgs a;
  ScanFn fn;
  const uint32_t* xflags;  // extra per-template flags ORed in by the finalize kernel (or null)
  dim3 grid, block;
  size_t part_bytes, flag_bytes, counter_off, ws_bytes;
  int64_t n;
  double a_plus, a_cross;
};

static sft_status prepare_scan(const sft_data* d, const sft_bank* bank, int64_t n, const sft_opts* o,
                               const sft_tuning& t, Prepared& P, int wf = -1, const double* wtab = nullptr,
                               const uint32_t* xflags = nullptr)
{
  ScanArgs& a = P.a;
  std::memset(&a, 0, sizeof(a));
  a.bins = d->bins;
  a.psd = d->psd;
  a.g_tmid = d->g_tmid;
  a.g_rows = d->g_rows;
  a.fp = d->fp;
  a.fx = d->fx;
  a.n_groups = d->n_groups;
  a.n_ext = d->n_ext;
  a.k_ext_lo = d->k_ext_lo;
  a.n_bins = d->n_bins;
  a.k_lo = d->k_lo;
  a.K = o->K;
  a.k_nyq = d->n / 2;
  a.T = d->T;
  // the FRESNEL kernel uses the Dirichlet limit only at beta == 0
  a.beta_switch = o->kernel == SFT_KERNEL_AUTO ? o->beta_switch : 0.0;
  a.tsun = o->tsun;
  a.delta_max = o->delta_max;
  a.mc = bank->mc;
  a.q = bank->q;
  a.t_c = bank->t_c;
  a.phi_c = bank->phi_c;
  a.a_first = bank->a_first;
  a.a_last = bank->a_last;
  a.n_tmpl = n;
  a.wtab = wtab;
  P.xflags = xflags;
  P.fn = pick_kernel(d, o, wf >= 0 ? wf : o->waveform);
  const int B = t.block ? t.block : 256;
  a.n_tiles = (int32_t)((n + B - 1) / B);
  int nb_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb_cu, (const void*)P.fn, B, 0) != hipSuccess || nb_cu < 1)
    nb_cu = 1;
  const int64_t resident = (int64_t)nb_cu * d->cu_count;
  int64_t nc;
  if (t.chunk_groups > 0) {
    nc = (d->n_groups + t.chunk_groups - 1) / t.chunk_groups;
  } else {
    // automatic: chunks of about 1 MiB of bins (they stay in L2 while the tiles of the
    // chunk run) and at least ~4 work items per resident block (short last wave)
    const size_t bin_sz = d->storage == SFT_STORE_F64 ? 16 : d->storage == SFT_STORE_F32 ? 8 : 4;
    const size_t group_bytes = (size_t)d->nd * d->n_ext * bin_sz;
    const int64_t g_l2 = std::max<int64_t>(1, (int64_t)((1u << 20) / std::max<size_t>(group_bytes, 1)));
    nc = std::max<int64_t>((d->n_groups + g_l2 - 1) / g_l2, (4 * resident + a.n_tiles - 1) / a.n_tiles);
    nc = std::min<int64_t>(std::max<int64_t>(nc, 1), std::max(1, d->n_groups / 4));
  }
  nc = std::min<int64_t>(std::max<int64_t>(nc, 1), std::min<int64_t>(d->n_groups, 65535));
  a.chunk = (int32_t)((d->n_groups + nc - 1) / nc);
  a.n_chunks = (d->n_groups + a.chunk - 1) / a.chunk;
  if ((int64_t)a.n_tiles * a.n_chunks > INT32_MAX) return fail(SFT_E_RANGE, "scan: too many work items");
  a.n_items = a.n_tiles * a.n_chunks;
  a.persistent = t.block == 0 && t.chunk_groups == 0 && t.persistent == 0 ? 1 : t.persistent;
  P.block = dim3(B);
  if (a.persistent) P.grid = dim3((unsigned)std::min<int64_t>(a.n_items, resident));
  else P.grid = dim3((unsigned)a.n_tiles, (unsigned)a.n_chunks);
  P.part_bytes = (size_t)a.n_chunks * 6 * n * sizeof(double);
  P.flag_bytes = (size_t)a.n_chunks * n * sizeof(uint32_t);
  P.counter_off = (P.part_bytes + P.flag_bytes + 255) / 256 * 256;
  P.ws_bytes = P.counter_off + 256;
  P.n = n;
  P.a_plus = o->a_plus;
  P.a_cross = o->a_cross;
  return SFT_OK;
}

// Enqueue [zero counter,] scan, finalize on st.  ws holds P.ws_bytes bytes.
static hipError_t enqueue_scan(Prepared& P, void* ws, sft_out* out, hipStream_t st, bool timed)
{
  ScanArgs& a = P.a;
  a.part = (double*)ws;
  a.pflags = (uint32_t*)((char*)ws + P.part_bytes);
  a.counter = (int32_t*)((char*)ws + P.counter_off);
  if (a.persistent) {
    hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(64), 0, st, a.counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipEvent_t ev_b = nullptr, ev_e = nullptr;
  if (timed) timing_slot(&ev_b, &ev_e);
  if (ev_b) (void)hipEventRecord(ev_b, st);
  void* args[] = {&a};
  hipError_t e = hipLaunchKernel((const void*)P.fn, P.grid, P.block, args, 0, st);
  if (e == hipSuccess) e = hipGetLastError();
  if (ev_e) (void)hipEventRecord(ev_e, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)((P.n + 255) / 256)), dim3(256), 0, st, a.part, a.pflags, P.n,
                     a.n_chunks, P.a_plus, P.a_cross, out->zp, out->zx, out->hhp, out->hhx, out->rho, out->flags,
                     P.xflags);
  return hipGetLastError();
}

// ============================================================================ surrogate
// Parameters of the surrogate waveform shared by its kernels.
struct SurArgs {
  double mc_lo, mc_span, q_lo, q_span, lt_lo, lt_span;  // input normalisation
  double c_phi, c_amp, p, judge_tol, tsun;
  int32_t head;
};

static SurArgs sur_args(const sft_surrogate* s, double tsun)
{
  SurArgs a;
  a.mc_lo = s->d.mc_lo;
  a.mc_span = s->d.mc_hi - s->d.mc_lo;
  a.q_lo = s->d.q_lo;
  a.q_span = s->d.q_hi - s->d.q_lo;
  a.lt_lo = s->d.lt_lo;
  a.lt_span = s->d.lt_hi - s->d.lt_lo;
  a.c_phi = s->d.c_phi;
  a.c_amp = s->d.c_amp;
  a.p = s->d.head ? 0.125 : 0.375;
  a.judge_tol = s->d.judge_tol;
  a.tsun = tsun;
  a.head = s->d.head;
  return a;
}

// network inputs in [-1, 1]
__device__ inline void sur_inputs(const SurArgs& a, double mc, double q, double tau, double* u)
{
  u[0] = 2.0 * (mc - a.mc_lo) / a.mc_span - 1.0;
  u[1] = 2.0 * (q - a.q_lo) / a.q_span - 1.0;
  u[2] = 2.0 * (log(tau) - a.lt_lo) / a.lt_span - 1.0;
}

// mass parameters of the 3.5PN model: nu, total mass [s], nu / (5 M), nu^(2/5)
struct PNMass {
  double nu, Mt, inv5Mnu, nu25;
};
__device__ inline PNMass pn_mass(double mc, double q, double tsun)
{
  double qq = q;
  if (!(qq >= 1.0)) qq = 1.0 / qq;
  PNMass r;
  r.nu = qq / ((1.0 + qq) * (1.0 + qq));
  r.Mt = mc * pow(r.nu, -0.6) * tsun;
  r.inv5Mnu = r.nu / (5.0 * r.Mt);
  r.nu25 = pow(r.nu, 0.4);
  return r;
}

// 1PN + 1.5PN part of the 3.5PN phase, -(2/nu) Theta^(5/8) (p2 Theta^(-1/4) + p3 Theta^(-3/8)),
// and its tau-derivative
__device__ inline void pn_head(const PNMass& pm, const PNCoef& c, double tau, double& ph, double& dph)
{
  const double th = tau * pm.inv5Mnu;
  const double t38 = pow(th, 0.375), t14 = pow(th, 0.25);
  ph = -2.0 / pm.nu * (c.p2 * t38 + c.p3 * t14);
  dph = -2.0 / pm.nu * (0.375 * c.p2 * t38 + 0.25 * c.p3 * t14) / th * pm.inv5Mnu;
}

// training pairs: u [n][3], y [n][2] (FP32) from FP64 Newtonian and 3.5PN waveforms
__global__ __launch_bounds__(256) void sur_targets_kernel(SurArgs sa, const double* __restrict__ mc,
                                                          const double* __restrict__ q, const double* __restrict__ tau,
                                                          int64_t n, float* __restrict__ u, float* __restrict__ y)
{
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double m = mc[i], qq = q[i], t = tau[i];
  const double M = m * sa.tsun;
  const double inv5M = 1.0 / (5.0 * M);
  const Chirp cn = newton_chirp(t, inv5M, 1.0 / (8.0 * kPi * M), 0.0, 1.0);
  const PNMass pm = pn_mass(m, qq, sa.tsun);
  const PNCoef pc = pn_coefficients(pm.nu);
  const Chirp cp = pn35_chirp(t, pm.nu, pm.inv5Mnu, pm.Mt, pm.nu25, 0.0, 1.0, pc);
  double d = cp.phase - cn.phase;
  if (sa.head) {
    double hp, hd;
    pn_head(pm, pc, t, hp, hd);
    d -= hp;
  }
  const double Phi = pow(t * inv5M, sa.p);
  double uu[3];
  sur_inputs(sa, m, qq, t, uu);
  u[3 * i] = (float)uu[0];
  u[3 * i + 1] = (float)uu[1];
  u[3 * i + 2] = (float)uu[2];
  y[2 * i] = (float)(d / (sa.c_phi * Phi));
  y[2 * i + 1] = (float)(log(cp.amp / cn.amp) / sa.c_amp);
}

// network inputs of a template batch, row r = g * nb + m (group-major)
__global__ __launch_bounds__(256) void sur_inputs_kernel(SurArgs sa, const double* __restrict__ mc,
                                                         const double* __restrict__ q, const double* __restrict__ t_c,
                                                         const double* __restrict__ g_tmid, int64_t nb, int32_t n_groups,
                                                         double* __restrict__ U)
{
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nb * n_groups) return;
  const int64_t m = r % nb;
  const int g = (int)(r / nb);
  const double tau = t_c[m] - g_tmid[g];
  double u[3];
  sur_inputs(sa, mc[m], q ? q[m] : 1.0, tau > 0.0 ? tau : 1.0, u);
  U[3 * r] = u[0];
  U[3 * r + 1] = u[1];
  U[3 * r + 2] = u[2];
}

// One lane per template of the batch: the surrogate chirp of every group the template
// uses (Newtonian chirp plus the network's corrections), the judge against the 3.5PN
// chirp, and the chirp table the scan reads (the 3.5PN chirps for a rejected template).
__global__ __launch_bounds__(256) void sur_post_kernel(SurArgs sa, const double* __restrict__ mc,
                                                       const double* __restrict__ q, const double* __restrict__ t_c,
                                                       const double* __restrict__ phi_c, const int32_t* __restrict__ a_first,
                                                       const int32_t* __restrict__ a_last,
                                                       const double* __restrict__ g_tmid, const int32_t* __restrict__ g_rows,
                                                       int64_t nb, int32_t n_groups, double T,
                                                       const double* __restrict__ Y, const double* __restrict__ dY,
                                                       double* __restrict__ tab, uint32_t* __restrict__ xflags,
                                                       double* __restrict__ mismatch)
{
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nb) return;
  const int lo = a_first ? (int)a_first[m] : 0;
  const int hi = a_last ? (int)a_last[m] : 0x7fffffff;
  const double tc = t_c[m], phic = phi_c ? phi_c[m] : 0.0;
  const double M = mc[m] * sa.tsun;
  const double inv5M = 1.0 / (5.0 * M);
  const double cf = T / (8.0 * kPi * M);
  const PNMass pm = pn_mass(mc[m], q ? q[m] : 1.0, sa.tsun);
  const PNCoef pc = pn_coefficients(pm.nu);
  const double dlt = 2.0 / sa.lt_span;   // du_tau / d ln tau
  const int64_t ps = (int64_t)n_groups * nb;
  double sr = 0.0, si = 0.0, sw = 0.0;
  for (int g = 0; g < n_groups; ++g) {
    int n_act = 0;
    for (int d = 0; d < SFT_GROUP_MAX; ++d) {
      const int r = g_rows[g * SFT_GROUP_MAX + d];
      n_act += (r >= 0 && r >= lo && r <= hi) ? 1 : 0;
    }
    const double tau = tc - g_tmid[g];
    if (n_act == 0 || !(tau > 0.0)) continue;
    const int64_t r = (int64_t)g * nb + m;
    const double y1 = Y[2 * r], y2 = Y[2 * r + 1], dy1 = dY[2 * r];
    const Chirp cn = newton_chirp(tau, inv5M, cf, phic, T);
    const double Phi = pow(tau * inv5M, sa.p);
    double dphi = sa.c_phi * Phi * y1;
    double ddphi = sa.c_phi * Phi * (sa.p * y1 + dy1 * dlt) / tau;   // d(dphi)/dtau
    if (sa.head) {
      double hp, hd;
      pn_head(pm, pc, tau, hp, hd);
      dphi += hp;
      ddphi += hd;
    }
    Chirp cs;
    cs.kappa = cn.kappa - ddphi * T / (2.0 * kPi);   // dphi/dt = -dphi/dtau
    cs.phase = cn.phase + dphi;
    cs.amp = cn.amp * exp(sa.c_amp * y2);
    cs.beta = cn.beta * pow(cs.kappa / cn.kappa, 11.0 / 3.0);
    cs.dres = (11.0 / 24.0) * cs.beta * cs.beta / cs.kappa;
    double* w = tab + r;
    w[0] = cs.kappa;
    w[ps] = cs.phase;
    w[2 * ps] = cs.amp;
    w[3 * ps] = cs.beta;
    w[4 * ps] = cs.dres;
    // judge term: A_PN^2 exp(i dphi) sinc(dkappa) per SFT row
    const Chirp cp = pn35_chirp(tau, pm.nu, pm.inv5Mnu, pm.Mt, pm.nu25, phic, T, pc);
    const double dk = cs.kappa - cp.kappa;
    const double snc = fabs(dk) < 1e-8 ? 1.0 - kPi * kPi * dk * dk / 6.0 : sin(kPi * dk) / (kPi * dk);
    const double wt = cp.amp * cp.amp * (double)n_act;
    double sd, cd;
    sincos(cs.phase - cp.phase, &sd, &cd);
    sr += wt * cd * snc;
    si += wt * sd * snc;
    sw += wt;
  }
  const double mm = sw > 0.0 ? 1.0 - sqrt(sr * sr + si * si) / sw : 0.0;
  if (mismatch) mismatch[m] = mm;
  const bool fallback = !(mm <= sa.judge_tol);
  xflags[m] = fallback ? kFlagSurrogateFallback : 0u;
  if (!fallback) return;
  for (int g = 0; g < n_groups; ++g) {
    int n_act = 0;
    for (int d = 0; d < SFT_GROUP_MAX; ++d) {
      const int r = g_rows[g * SFT_GROUP_MAX + d];
      n_act += (r >= 0 && r >= lo && r <= hi) ? 1 : 0;
    }
    const double tau = tc - g_tmid[g];
    if (n_act == 0 || !(tau > 0.0)) continue;
    const Chirp cp = pn35_chirp(tau, pm.nu, pm.inv5Mnu, pm.Mt, pm.nu25, phic, T, pc);
    double* w = tab + (int64_t)g * nb + m;
    w[0] = cp.kappa;
    w[ps] = cp.phase;
    w[2 * ps] = cp.amp;
    w[3 * ps] = cp.beta;
    w[4 * ps] = cp.dres;
  }
}

extern "C" sft_status sft_surrogate_targets(const sft_surrogate* s, const double* mc, const double* q,
                                            const double* tau, int64_t n, double tsun, float* u, float* y,
                                            void* hip_stream)
{
  if (!s || !mc || !q || !tau || !u || !y) return fail(SFT_E_INVALID, "sft_surrogate_targets: null argument");
  if (n < 0) return fail(SFT_E_INVALID, "sft_surrogate_targets: negative n");
  if (!(tsun > 0.0)) return fail(SFT_E_INVALID, "sft_surrogate_targets: tsun must be positive");
  if (n == 0) return SFT_OK;
  hipLaunchKernelGGL(sur_targets_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)hip_stream,
                     sur_args(s, tsun), mc, q, tau, n, u, y);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SFT_OK : fail(SFT_E_DEVICE, "sft_surrogate_targets: %s", hipGetErrorString(e));
}

// Templates per surrogate batch: about 2^23 network evaluations (one per template and
// timestamp group), which bounds the batch workspace near 1 GiB.
static int64_t sur_batch(int64_t n, int32_t n_groups)
{
  int64_t b = ((int64_t)1 << 23) / std::max(1, n_groups);
  b = std::max<int64_t>(256, b / 256 * 256);
  return std::min(b, n);
}

// Scan with the surrogate waveform, batch by batch: network inputs, FP64 network
// evaluation (values and d/du_tau), surrogate chirps + judge -> chirp table, then the
// table-driven scan of the batch.
static sft_status surrogate_scan(const sft_data* d, const sft_bank* bank, int64_t n, const sft_opts* o, sft_out* out,
                                 hipStream_t st)
{
  const sft_surrogate* sur = o->surrogate;
  const SurArgs sa = sur_args(sur, o->tsun);
  const int64_t B = sur_batch(n, d->n_groups);
  const int64_t R = B * d->n_groups;
  const int64_t chunk = std::min<int64_t>(R, 1 << 16);
  // workspace: U [R][3], Y, dY [R][2], table [5][R], xflags [B], network scratch, scan workspace
  Prepared P0;
  sft_status s = prepare_scan(d, bank, B, o, d->tune, P0, WF_TABLE, nullptr, nullptr);
  if (s != SFT_OK) return s;
  const size_t off_y = (size_t)R * 3 * sizeof(double);
  const size_t off_dy = off_y + (size_t)R * 2 * sizeof(double);
  const size_t off_tab = off_dy + (size_t)R * 2 * sizeof(double);
  const size_t off_xf = off_tab + (size_t)R * 5 * sizeof(double);
  const size_t off_nn = (off_xf + (size_t)B * sizeof(uint32_t) + 255) / 256 * 256;
  const size_t off_scan = (off_nn + mlp_infer_scratch_bytes(sur->d.hidden, chunk) + 255) / 256 * 256;
  size_t scan_ws = P0.ws_bytes;
  for (int64_t m0 = 0; m0 < n; m0 += B) {   // the last batch may have a different shape
    const int64_t nb = std::min(B, n - m0);
    Prepared Pt;
    if ((s = prepare_scan(d, bank, nb, o, d->tune, Pt, WF_TABLE, nullptr, nullptr)) != SFT_OK) return s;
    scan_ws = std::max(scan_ws, Pt.ws_bytes);
  }
  char* ws = nullptr;
  HIP_OR_FAIL(hipMallocAsync((void**)&ws, off_scan + scan_ws, st));
  double* U = (double*)ws;
  double* Y = (double*)(ws + off_y);
  double* dY = (double*)(ws + off_dy);
  double* tab = (double*)(ws + off_tab);
  uint32_t* xf = (uint32_t*)(ws + off_xf);
  hipError_t e = hipSuccess;
  for (int64_t m0 = 0; m0 < n && e == hipSuccess && s == SFT_OK; m0 += B) {
    const int64_t nb = std::min(B, n - m0);
    const int64_t rows = nb * d->n_groups;
    sft_bank b = *bank;
    b.mc += m0;
    b.t_c += m0;
    if (b.q) b.q += m0;
    if (b.phi_c) b.phi_c += m0;
    if (b.a_first) b.a_first += m0;
    if (b.a_last) b.a_last += m0;
    sft_out ob = *out;
    ob.zp += 2 * m0;
    ob.zx += 2 * m0;
    ob.hhp += m0;
    ob.hhx += m0;
    ob.rho += m0;
    ob.flags += m0;
    if (ob.mismatch) ob.mismatch += m0;
    hipLaunchKernelGGL(sur_inputs_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, sa, b.mc, b.q, b.t_c,
                       d->g_tmid, nb, d->n_groups, U);
    if ((e = hipGetLastError()) != hipSuccess) break;
    if ((e = mlp_infer(sur, U, rows, Y, dY, ws + off_nn, chunk, st)) != hipSuccess) break;
    hipLaunchKernelGGL(sur_post_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, sa, b.mc, b.q, b.t_c,
                       b.phi_c, b.a_first, b.a_last, d->g_tmid, d->g_rows, nb, d->n_groups, d->T, Y, dY, tab, xf,
                       ob.mismatch);
    if ((e = hipGetLastError()) != hipSuccess) break;
    Prepared P;
    if ((s = prepare_scan(d, &b, nb, o, d->tune, P, WF_TABLE, tab, xf)) != SFT_OK) break;
    e = enqueue_scan(P, ws + off_scan, &ob, st, m0 == 0);
  }
  hipError_t e2 = hipFreeAsync(ws, st);
  if (s != SFT_OK) return s;
  if (e != hipSuccess) return fail(SFT_E_DEVICE, "scan (surrogate): %s", hipGetErrorString(e));
  if (e2 != hipSuccess) return fail(SFT_E_DEVICE, "scan (surrogate): hipFreeAsync: %s", hipGetErrorString(e2));
  return SFT_OK;
}

extern "C" sft_status sft_template_bank_scan(const sft_data* d, const sft_bank* bank, int64_t n, const sft_opts* o,
                                             sft_out* out, void* hip_stream)
{
  sft_status s = validate_scan(d, o);
  if (s != SFT_OK) return s;
  if ((s = validate_io(bank, n, out)) != SFT_OK || n == 0) return s;
  hipStream_t st = (hipStream_t)hip_stream;
  if (o->waveform == SFT_WF_SURROGATE) return surrogate_scan(d, bank, n, o, out, st);
  Prepared P;
  if ((s = prepare_scan(d, bank, n, o, d->tune, P)) != SFT_OK) return s;
  void* ws = nullptr;
  HIP_OR_FAIL(hipMallocAsync(&ws, P.ws_bytes, st));
  hipError_t e = enqueue_scan(P, ws, out, st, true);
  hipError_t e2 = hipFreeAsync(ws, st);
  if (e != hipSuccess) return fail(SFT_E_DEVICE, "scan: launch failed: %s", hipGetErrorString(e));
  if (e2 != hipSuccess) return fail(SFT_E_DEVICE, "scan: hipFreeAsync: %s", hipGetErrorString(e2));
  return SFT_OK;
}

// ---------------------------------------------------------------------------- tuning
extern "C" sft_status sft_get_tuning(const sft_data* d, sft_tuning* t)
{
  if (!d || !t) return fail(SFT_E_INVALID, "sft_get_tuning: null argument");
  *t = d->tune;
  return SFT_OK;
}

extern "C" sft_status sft_set_tuning(sft_data* d, const sft_tuning* t)
{
  if (!d) return fail(SFT_E_INVALID, "sft_set_tuning: null data");
  sft_status s = validate_tuning(t);
  if (s != SFT_OK) return s;
  d->tune = *t;
  d->tune.reserved = 0;
  return SFT_OK;
}

extern "C" sft_status sft_autotune(sft_data* d, const sft_bank* bank, int64_t n, const sft_opts* o, sft_out* out,
                                   void* hip_stream, int32_t reps, sft_tuning* best, float* best_ms)
{
  sft_status s = validate_scan(d, o);
  if (s != SFT_OK) return s;
  if ((s = validate_io(bank, n, out)) != SFT_OK) return s;
  if (n == 0) return fail(SFT_E_INVALID, "sft_autotune: needs at least one template");
  if (o->waveform == SFT_WF_SURROGATE)
    return fail(SFT_E_UNSUPPORTED, "sft_autotune: tune with the Newtonian or 3.5PN waveform");
  if (reps < 1 || reps > 100) return fail(SFT_E_RANGE, "sft_autotune: reps must be in [1, 100]");
  hipStream_t st = (hipStream_t)hip_stream;
  std::vector<sft_tuning> cand;
  const int blocks[] = {64, 128, 256};
  const int nchunks[] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64};
  for (int b : blocks)
    for (int nc : nchunks) {
      if (nc > d->n_groups) continue;
      for (int pers = 0; pers < 2; ++pers) {
        sft_tuning t{};
        t.block = b;
        t.chunk_groups = (d->n_groups + nc - 1) / nc;
        t.persistent = pers;
        cand.push_back(t);
      }
    }
  std::vector<Prepared> preps(cand.size());
  size_t ws_max = 0;
  for (size_t i = 0; i < cand.size(); ++i) {
    if ((s = prepare_scan(d, bank, n, o, cand[i], preps[i])) != SFT_OK) return s;
    ws_max = std::max(ws_max, preps[i].ws_bytes);
  }
  void* ws = nullptr;
  HIP_OR_FAIL(hipMallocAsync(&ws, ws_max, st));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float bms = 3.4e38f;
  size_t bi = 0;
  for (size_t i = 0; i < cand.size() && e == hipSuccess; ++i) {
    e = enqueue_scan(preps[i], ws, out, st, false);   // warm-up
    if (e != hipSuccess) break;
    if ((e = hipEventRecord(e0, st)) != hipSuccess) break;
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = enqueue_scan(preps[i], ws, out, st, false);
    if (e != hipSuccess) break;
    if ((e = hipEventRecord(e1, st)) != hipSuccess) break;
    if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
    float ms = 0.f;
    if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
    ms /= (float)reps;
    if (ms < bms) {
      bms = ms;
      bi = i;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  hipError_t e2 = hipFreeAsync(ws, st);
  if (e != hipSuccess) return fail(SFT_E_DEVICE, "sft_autotune: %s", hipGetErrorString(e));
  if (e2 != hipSuccess) return fail(SFT_E_DEVICE, "sft_autotune: hipFreeAsync: %s", hipGetErrorString(e2));
  d->tune = cand[bi];
  if (best) *best = cand[bi];
  if (best_ms) *best_ms = bms;
  return SFT_OK;
}

// ---------------------------------------------------------------------------- graph plans
struct sft_plan {
  Prepared P;
  void* ws;
  sft_out out;
  hipGraph_t graph;
  hipGraphExec_t exec;
};

extern "C" void sft_plan_destroy(sft_plan* p)
{
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->ws) (void)hipFree(p->ws);
  delete p;
}

extern "C" sft_status sft_plan_create(const sft_data* d, const sft_bank* bank, int64_t n, const sft_opts* o,
                                      sft_out* out, sft_plan** plan)
{
  if (!plan) return fail(SFT_E_INVALID, "sft_plan_create: null plan pointer");
  *plan = nullptr;
  sft_status s = validate_scan(d, o);
  if (s != SFT_OK) return s;
  if ((s = validate_io(bank, n, out)) != SFT_OK) return s;
  if (n == 0) return fail(SFT_E_INVALID, "sft_plan_create: needs at least one template");
  if (o->waveform == SFT_WF_SURROGATE)
    return fail(SFT_E_UNSUPPORTED, "sft_plan_create: the surrogate waveform is not captured into graphs");
  sft_plan* p = new sft_plan();
  p->ws = nullptr;
  p->graph = nullptr;
  p->exec = nullptr;
  p->out = *out;
  if ((s = prepare_scan(d, bank, n, o, d->tune, p->P)) != SFT_OK) {
    delete p;
    return s;
  }
  hipError_t e = hipMalloc(&p->ws, p->P.ws_bytes);
  if (e != hipSuccess) {
    sft_plan_destroy(p);
    return fail(e == hipErrorOutOfMemory ? SFT_E_NOMEM : SFT_E_DEVICE, "sft_plan_create: hipMalloc: %s", hipGetErrorString(e));
  }
  hipStream_t cs = nullptr;
  e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e == hipSuccess) {
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t el = enqueue_scan(p->P, p->ws, &p->out, cs, false);
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(cs, &g);
      p->graph = g;
      if (el != hipSuccess) e = el;
    }
    (void)hipStreamDestroy(cs);
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    sft_plan_destroy(p);
    return fail(SFT_E_DEVICE, "sft_plan_create: graph capture: %s", hipGetErrorString(e));
  }
  *plan = p;
  return SFT_OK;
}

extern "C" sft_status sft_plan_launch(sft_plan* p, void* hip_stream)
{
  if (!p) return fail(SFT_E_INVALID, "sft_plan_launch: null plan");
  hipError_t e = hipGraphLaunch(p->exec, (hipStream_t)hip_stream);
  if (e != hipSuccess) return fail(SFT_E_DEVICE, "sft_plan_launch: %s", hipGetErrorString(e));
  return SFT_OK;
}

extern "C" sft_status sft_inner_product(const sft_data* d, double mc, double q, double t_c, double phi_c,
                                        int32_t a_first, int32_t a_last, const sft_opts* o, double zp[2],
                                        double zx[2], double* hhp, double* hhx, double* rho, uint32_t* flags)
{
  sft_status s = validate_scan(d, o);
  if (s != SFT_OK) return s;
  // one device block: 4 doubles in + 2 ints in, 7 doubles + 1 flag out
  struct Blk {
    double mc, q, tc, phic;
    int32_t af, al;
    double zp[2], zx[2], hhp, hhx, rho;
    uint32_t fl;
  };
  Blk h{};
  h.mc = mc;
  h.q = q;
  h.tc = t_c;
  h.phic = phi_c;
  h.af = a_first;
  h.al = a_last;
  Blk* dv = nullptr;
  HIP_OR_FAIL(hipMalloc(&dv, sizeof(Blk)));
  hipError_t e = hipMemcpy(dv, &h, sizeof(Blk), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(dv);
    return fail(SFT_E_DEVICE, "sft_inner_product: %s", hipGetErrorString(e));
  }
  sft_bank b{&dv->mc, &dv->q, &dv->tc, &dv->phic, &dv->af, &dv->al};
  sft_out ou{dv->zp, dv->zx, &dv->hhp, &dv->hhx, &dv->rho, &dv->fl};
  s = sft_template_bank_scan(d, &b, 1, o, &ou, nullptr);
  if (s == SFT_OK) {
    e = hipMemcpy(&h, dv, sizeof(Blk), hipMemcpyDeviceToHost);  // waits for the default stream
    if (e != hipSuccess) s = fail(SFT_E_DEVICE, "sft_inner_product: %s", hipGetErrorString(e));
  }
  (void)hipFree(dv);
  if (s != SFT_OK) return s;
  if (zp) { zp[0] = h.zp[0]; zp[1] = h.zp[1]; }
  if (zx) { zx[0] = h.zx[0]; zx[1] = h.zx[1]; }
  if (hhp) *hhp = h.hhp;
  if (hhx) *hhx = h.hhx;
  if (rho) *rho = h.rho;
  if (flags) *flags = h.fl;
  return SFT_OK;
}
