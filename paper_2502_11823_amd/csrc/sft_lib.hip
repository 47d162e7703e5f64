// sft_lib.hip -- libsft.so: C ABI (include/sft.h) and gfx950 kernels for the
// short-Fourier-transform inner product of Tenorio & Gerosa (arXiv:2502.11823).
//
// Kernels
//   load_kernel     : per-SFT whitening d~ = 2 x~ / S (Sec. III.B), conjugation,
//                     DC/Nyquist mirroring (footnote of Sec. III.C), conversion to the
//                     storage precision, PSD masking.  Once per dataset.
//   scan_kernel     : (sft_scan.h, instantiated in scan_*.hip) one template per lane,
//                     one SFT chunk per work item; writes one partial per
//                     (template, chunk).
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
#include "sft_scan_args.h"
#include "sft_sort.h"

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
  double* g_eph;          // [n_groups][9] detector r/c, v/c, a/c at the group's midpoint (Doppler), or null;
                          // set, every group holds one row
  double* row_tmid;       // [n_sft] midpoint t_start + T/2 of each row (bank ordering)
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

// The device part of loading: raw bins dx [n_sft][n_bins][2] and PSD dp [n_sft][n_bins] (FP64,
// device) are whitened, converted and packed by load_kernel; the timestamp groups are built
// from the host start times.  dx and dp stay owned by the caller.
static sft_status load_device(const sft_data_desc* d, const double* t_start, const double* dx, const double* dp,
                              const double* fplus, const double* fcross, hipStream_t st, sft_data** out)
{
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
  hipError_t e = hipSuccess;
  if ((e = hipMalloc(&h->bins, ne * bin_sz)) != hipSuccess || (e = hipMalloc(&h->psd, nb * ps_sz)) != hipSuccess ||
      (e = hipMalloc(&h->fp, d->n_sft * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&h->fx, d->n_sft * sizeof(double))) != hipSuccess) {
    sft_free_data(h);
    return fail(e == hipErrorOutOfMemory ? SFT_E_NOMEM : SFT_E_DEVICE, "sft_load_data: hipMalloc: %s", hipGetErrorString(e));
  }
  do {
    if (fplus) e = hipMemcpyAsync(h->fp, fplus, d->n_sft * sizeof(double), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) break;
    if (fcross) e = hipMemcpyAsync(h->fx, fcross, d->n_sft * sizeof(double), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) break;
    if (!fplus || !fcross) {
      // defaults F+ = 1, Fx = 0 staged from the host
      std::vector<double> tmp(d->n_sft);
      if (!fplus) {
        for (int i = 0; i < d->n_sft; i++) tmp[i] = 1.0;
        e = hipMemcpy(h->fp, tmp.data(), d->n_sft * sizeof(double), hipMemcpyHostToDevice);
      }
      if (e == hipSuccess && !fcross) {
        for (int i = 0; i < d->n_sft; i++) tmp[i] = 0.0;
        e = hipMemcpy(h->fx, tmp.data(), d->n_sft * sizeof(double), hipMemcpyHostToDevice);
      }
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
      std::vector<double> rmid(d->n_sft);
      for (int32_t r = 0; r < d->n_sft; ++r) rmid[r] = t_start[r] + 0.5 * h->T;
      if ((e = hipMalloc(&h->row_tmid, rmid.size() * sizeof(double))) != hipSuccess) break;
      if ((e = hipMemcpyAsync(h->row_tmid, rmid.data(), rmid.size() * sizeof(double), hipMemcpyHostToDevice, st)) != hipSuccess) break;
      if ((e = hipMalloc(&h->g_tmid, tmid.size() * sizeof(double))) != hipSuccess) break;
      if ((e = hipMalloc(&h->g_rows, grows.size() * sizeof(int32_t))) != hipSuccess) break;
      if ((e = hipMemcpyAsync(h->g_tmid, tmid.data(), tmid.size() * sizeof(double), hipMemcpyHostToDevice, st)) != hipSuccess) break;
      if ((e = hipMemcpyAsync(h->g_rows, grows.data(), grows.size() * sizeof(int32_t), hipMemcpyHostToDevice, st)) != hipSuccess) break;
      e = hipStreamSynchronize(st);   // the host vectors go out of scope here
    }
  } while (0);
  if (e != hipSuccess) {
    sft_free_data(h);
    return fail(SFT_E_DEVICE, "sft_load_data: %s", hipGetErrorString(e));
  }
  *out = h;
  return SFT_OK;
}

static sft_status validate_desc(const sft_data_desc* d)
{
  if (d->n_sft < 1 || d->n_samples < 2 || (d->n_samples & 1) || !(d->t_sft > 0.0) || d->reserved != 0)
    return fail(SFT_E_INVALID, "sft_load_data: bad descriptor (n_sft=%d n=%d T=%g)", d->n_sft, d->n_samples, d->t_sft);
  if (d->n_sft >= (1 << 24)) return fail(SFT_E_RANGE, "sft_load_data: n_sft=%d, at most 2^24 - 1 SFT rows", d->n_sft);
  if (d->k_lo < 0 || d->n_bins < 1 || d->k_lo + d->n_bins - 1 > d->n_samples / 2)
    return fail(SFT_E_INVALID, "sft_load_data: band [%d, %d) outside [0, n/2]", d->k_lo, d->k_lo + d->n_bins);
  if (d->storage != SFT_STORE_F64 && d->storage != SFT_STORE_F32 && d->storage != SFT_STORE_BF16)
    return fail(SFT_E_INVALID, "sft_load_data: unknown storage %d", d->storage);
  return SFT_OK;
}

extern "C" sft_status sft_load_data(const sft_data_desc* d, const double* t_start, const double* x_bins,
                                    const double* psd, const double* fplus, const double* fcross,
                                    void* hip_stream, sft_data** out)
{
  if (!d || !t_start || !x_bins || !psd || !out) return fail(SFT_E_INVALID, "sft_load_data: null argument");
  *out = nullptr;
  sft_status s = validate_desc(d);
  if (s != SFT_OK) return s;
  hipStream_t st = (hipStream_t)hip_stream;
  size_t nb = (size_t)d->n_sft * d->n_bins;
  double *dx = nullptr, *dp = nullptr;
  hipError_t e = hipMalloc(&dx, nb * 2 * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&dp, nb * sizeof(double));
  if (e == hipSuccess) e = hipMemcpyAsync(dx, x_bins, nb * 2 * sizeof(double), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(dp, psd, nb * sizeof(double), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) s = load_device(d, t_start, dx, dp, fplus, fcross, st, out);   // synchronises st
  if (dx) (void)hipFree(dx);
  if (dp) (void)hipFree(dp);
  if (e != hipSuccess)
    return fail(e == hipErrorOutOfMemory ? SFT_E_NOMEM : SFT_E_DEVICE, "sft_load_data: %s", hipGetErrorString(e));
  return s;
}

// rows of the kept segments: dx[r] = bins[src[r]], dp[r] = psd[src[r]]
__global__ void gather_rows_kernel(const double* __restrict__ bins, const double* __restrict__ psd,
                                   const int32_t* __restrict__ src, int32_t n_rows, int32_t n_bins,
                                   double* __restrict__ dx, double* __restrict__ dp)
{
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n_rows * n_bins) return;
  const int64_t r = i / n_bins, k = i - r * n_bins;
  const int64_t s = (int64_t)src[r] * n_bins + k;
  dx[2 * i] = bins[2 * s];
  dx[2 * i + 1] = bins[2 * s + 1];
  dp[i] = psd[s];
}

extern "C" sft_status sft_load_strain(const sft_strain_desc* sd, const double* x, const double* fplus,
                                      const double* fcross, void* hip_stream, sft_data** out, int32_t* n_rows)
{
  if (!sd || !x || !out) return fail(SFT_E_INVALID, "sft_load_strain: null argument");
  *out = nullptr;
  if (sd->n_samples < 16 || sd->n_total < sd->n_samples || sd->n_det < 1)
    return fail(SFT_E_INVALID, "sft_load_strain: bad descriptor");
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t n_seg = sd->n_total / sd->n_samples;
  const int64_t n_all = n_seg * sd->n_det;
  const size_t nb = (size_t)n_all * sd->n_bins;
  double *bins = nullptr, *psd = nullptr, *dx = nullptr, *dp = nullptr;
  int32_t *keep = nullptr, *src = nullptr;
  sft_status s = SFT_OK;
  hipError_t e = hipMalloc(&bins, nb * 2 * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&psd, nb * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&keep, (size_t)n_all * sizeof(int32_t));
  std::vector<int32_t> hk(n_all);
  if (e == hipSuccess) s = sft_make_sfts(sd, x, bins, psd, keep, hip_stream);
  if (e == hipSuccess && s == SFT_OK) {
    e = hipMemcpyAsync(hk.data(), keep, hk.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  std::vector<int32_t> rows;
  std::vector<double> t_start, fp, fx;
  if (e == hipSuccess && s == SFT_OK) {
    const double T = sd->dt * sd->n_samples;
    for (int64_t a = 0; a < n_all; ++a) {
      if (!hk[a]) continue;
      rows.push_back((int32_t)a);
      t_start.push_back(sd->t0 + (double)(a % n_seg) * T);
      fp.push_back(fplus ? fplus[a] : 1.0);
      fx.push_back(fcross ? fcross[a] : 0.0);
    }
    if (rows.empty()) s = fail(SFT_E_INVALID, "sft_load_strain: every segment is a gap");
  }
  if (e == hipSuccess && s == SFT_OK) {
    const size_t nr = rows.size() * (size_t)sd->n_bins;
    e = hipMalloc(&dx, nr * 2 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&dp, nr * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&src, rows.size() * sizeof(int32_t));
    if (e == hipSuccess) e = hipMemcpyAsync(src, rows.data(), rows.size() * sizeof(int32_t), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, st, bins, psd, src,
                         (int32_t)rows.size(), sd->n_bins, dx, dp);
      e = hipGetLastError();
    }
    if (e == hipSuccess) {
      sft_data_desc dd{};
      dd.n_sft = (int32_t)rows.size();
      dd.n_samples = sd->n_samples;
      dd.t_sft = sd->dt * sd->n_samples;
      dd.k_lo = sd->k_lo;
      dd.n_bins = sd->n_bins;
      dd.storage = sd->storage;
      s = validate_desc(&dd);
      if (s == SFT_OK) s = load_device(&dd, t_start.data(), dx, dp, fp.data(), fx.data(), st, out);   // synchronises st
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  for (void* p : {(void*)bins, (void*)psd, (void*)keep, (void*)dx, (void*)dp, (void*)src})
    if (p) (void)hipFree(p);
  if (e != hipSuccess) {
    if (*out) {
      sft_free_data(*out);
      *out = nullptr;
    }
    return fail(e == hipErrorOutOfMemory ? SFT_E_NOMEM : SFT_E_DEVICE, "sft_load_strain: %s", hipGetErrorString(e));
  }
  if (s == SFT_OK && n_rows) *n_rows = (int32_t)rows.size();
  return s;
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
  if (h->g_eph) (void)hipFree(h->g_eph);
  if (h->row_tmid) (void)hipFree(h->row_tmid);
  delete h;
}

// Doppler (Sec. III.B): detector positions per SFT row.  Rows of one start time (detectors at
// different places) no longer share the waveform, so every row becomes its own timestamp group,
// in the same time order.
extern "C" sft_status sft_set_ephemeris(sft_data* h, const double* eph, void* hip_stream)
{
  if (!h || !eph) return fail(SFT_E_INVALID, "sft_set_ephemeris: null argument");
  for (int64_t i = 0; i < (int64_t)h->n_sft * 9; ++i)
    if (!std::isfinite(eph[i])) return fail(SFT_E_INVALID, "sft_set_ephemeris: non-finite entry %lld", (long long)i);
  hipStream_t st = (hipStream_t)hip_stream;
  std::vector<double> tmid(h->n_groups);
  std::vector<int32_t> grows((size_t)h->n_groups * SFT_GROUP_MAX);
  hipError_t e = hipMemcpyAsync(tmid.data(), h->g_tmid, tmid.size() * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(grows.data(), h->g_rows, grows.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(SFT_E_DEVICE, "sft_set_ephemeris: %s", hipGetErrorString(e));
  std::vector<double> nt, ne;
  std::vector<int32_t> nr;
  for (int32_t g = 0; g < h->n_groups; ++g)
    for (int d = 0; d < SFT_GROUP_MAX; ++d) {
      const int32_t r = grows[(size_t)g * SFT_GROUP_MAX + d];
      if (r < 0) continue;
      nt.push_back(tmid[g]);
      nr.push_back(r);
      for (int q = 1; q < SFT_GROUP_MAX; ++q) nr.push_back(-1);
      for (int q = 0; q < 9; ++q) ne.push_back(eph[(size_t)r * 9 + q]);
    }
  double *d_t = nullptr, *d_e = nullptr;
  int32_t* d_r = nullptr;
  if ((e = hipMalloc(&d_t, nt.size() * sizeof(double))) == hipSuccess &&
      (e = hipMalloc(&d_e, ne.size() * sizeof(double))) == hipSuccess &&
      (e = hipMalloc(&d_r, nr.size() * sizeof(int32_t))) == hipSuccess &&
      (e = hipMemcpyAsync(d_t, nt.data(), nt.size() * sizeof(double), hipMemcpyHostToDevice, st)) == hipSuccess &&
      (e = hipMemcpyAsync(d_e, ne.data(), ne.size() * sizeof(double), hipMemcpyHostToDevice, st)) == hipSuccess &&
      (e = hipMemcpyAsync(d_r, nr.data(), nr.size() * sizeof(int32_t), hipMemcpyHostToDevice, st)) == hipSuccess)
    e = hipStreamSynchronize(st);   // the host vectors go out of scope here
  if (e != hipSuccess) {
    if (d_t) (void)hipFree(d_t);
    if (d_e) (void)hipFree(d_e);
    if (d_r) (void)hipFree(d_r);
    return fail(e == hipErrorOutOfMemory ? SFT_E_NOMEM : SFT_E_DEVICE, "sft_set_ephemeris: %s", hipGetErrorString(e));
  }
  (void)hipFree(h->g_tmid);
  (void)hipFree(h->g_rows);
  if (h->g_eph) (void)hipFree(h->g_eph);
  h->g_tmid = d_t;
  h->g_rows = d_r;
  h->g_eph = d_e;
  h->n_groups = (int32_t)nt.size();
  h->nd = 1;
  return SFT_OK;
}

extern "C" void sft_default_opts(sft_opts* o)
{
  if (!o) return;
  o->K = 8;
  o->kernel = SFT_KERNEL_AUTO;
  o->precision = SFT_PREC_FP32_KAHAN;
  o->waveform = SFT_WF_NEWTON;
  o->t_ref = SFT_REF_MID;
  o->beta_switch = 1e-7;
  o->a_plus = 1.0;
  o->a_cross = 0.0;
  o->tsun = 4.925490947641267e-6;
  o->delta_max = 0.0;
  o->surrogate = nullptr;
}

// ============================================================================ scan (host side)
// Resolvability threshold of the four amplitudes of the F-statistic: M is inverted when
// det [[A, C], [C, B]] >= kFstatEps A B, i.e. when the weighted response vectors (a_alpha) and
// (b_alpha) are at least asin(sqrt(kFstatEps)) ~ 5.7 degrees from parallel; below it only the
// dominant pattern is kept (the template is flagged FSTAT_DEGENERATE).
static constexpr double kFstatEps = 1e-2;

// 2F = x.M^{-1}.x (Sec. II.B) for x = (Re z+, Re zx, Im z+, Im zx) and the block-diagonal
// norm matrix with blocks [[A, C], [C, B]] (A = hh+, B = hhx, C = hh+x), by the closed-form
// inverse of the 2x2 block; nearly parallel patterns keep the largest eigenvector u of the
// block only: 2F = ((u.x_cos)^2 + (u.x_sin)^2) / lambda_max.
__device__ inline double fstat_2f(double x0, double x1, double x2, double x3, double A, double B, double C,
                                  bool& degenerate)
{
  degenerate = false;
  if (!(A > 0.0) && !(B > 0.0)) return 0.0;
  const double D = A * B - C * C;
  if (D >= kFstatEps * A * B && D > 0.0)
    return (B * (x0 * x0 + x2 * x2) + A * (x1 * x1 + x3 * x3) - 2.0 * C * (x0 * x1 + x2 * x3)) / D;
  degenerate = true;
  const double lam = 0.5 * (A + B) + hypot(0.5 * (A - B), C);
  if (!(lam > 0.0)) return 0.0;
  // eigenvector from the better-conditioned row of (N - lam I) u = 0
  double u0, u1;
  if (A >= B) {
    u0 = lam - B;
    u1 = C;
  } else {
    u0 = C;
    u1 = lam - A;
  }
  const double un = hypot(u0, u1);
  u0 /= un;
  u1 /= un;
  const double pc = u0 * x0 + u1 * x1, ps = u0 * x2 + u1 * x3;
  return (pc * pc + ps * ps) / lam;
}

// Per template: the partials of the chunks in chunk order (FP64), rho (Eq. det_short), the
// flags, and with nacc = 7 the cross norm and the F-statistic.  m is the template's position
// in the scanned order; its results go to position perm[m] of the outputs (perm null: m).
__global__ __launch_bounds__(256) void finalize_kernel(const double* __restrict__ part, const uint32_t* __restrict__ pflags,
                                                       int64_t n, int32_t n_chunks, int32_t nacc, double a_plus,
                                                       double a_cross, double* __restrict__ zp, double* __restrict__ zx,
                                                       double* __restrict__ hhp, double* __restrict__ hhx,
                                                       double* __restrict__ rho, uint32_t* __restrict__ flags,
                                                       const uint32_t* __restrict__ xflags, double* __restrict__ hhpx,
                                                       double* __restrict__ twoF, const int32_t* __restrict__ perm,
                                                       int32_t* __restrict__ n_used)
{
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  const int64_t w = perm ? (int64_t)perm[m] : m;
  double v[7] = {0, 0, 0, 0, 0, 0, 0};
  uint32_t fl = 0;
  int64_t used = 0;
  for (int c = 0; c < n_chunks; ++c) {
    const double* p = part + (int64_t)c * nacc * n + m;
#pragma unroll
    for (int q = 0; q < 6; ++q) v[q] += p[q * n];
    if (nacc == 7) v[6] += p[6 * n];
    const uint32_t pf = pflags[(int64_t)c * n + m];
    fl |= pf & ((1u << kUsedShift) - 1u);
    used += pf >> kUsedShift;
  }
  if (n_used) n_used[w] = (int32_t)used;
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
  if (nacc == 7) {
    bool deg = false;
    const double f2 = fstat_2f(v[0], v[2], v[1], v[3], v[4], v[5], v[6], deg);
    if (deg) fl |= SFT_FLAG_FSTAT_DEGENERATE;
    fin = fin && isfinite(v[6]) && isfinite(f2);
    if (hhpx) hhpx[w] = v[6];
    if (twoF) twoF[w] = f2;
  }
  if (!fin) fl |= kFlagNonfinite;
  if (xflags) fl |= xflags[m];
  zp[2 * w] = v[0];
  zp[2 * w + 1] = v[1];
  zx[2 * w] = v[2];
  zx[2 * w + 1] = v[3];
  hhp[w] = v[4];
  hhx[w] = v[5];
  rho[w] = r;
  flags[w] = fl;
}

// wf: WF_NEWTON, WF_PN35 or WF_TABLE (the surrogate path); fs: the F-statistic form
static ScanFn pick_kernel(const sft_data* d, const sft_opts* o, int wf, bool fs, bool dop)
{
  const int kern = o->kernel == SFT_KERNEL_DIRICHLET ? KERN_DIRICHLET : KERN_FRESNEL;
  if (dop) return scan_pick_doppler(o->precision, fs ? 1 : 0, kern, o->K);
  if (o->t_ref == SFT_REF_START) return scan_pick_start(d->storage, o->precision, wf, kern, d->nd, fs ? 1 : 0);
  if (fs) return scan_pick_fstat(o->precision, kern, o->K, d->nd);
  if (o->precision == SFT_PREC_FP64) return scan_pick_f64(wf, kern, o->K, d->nd);
  if (d->storage == SFT_STORE_F32) {
    const bool kahan = o->precision == SFT_PREC_FP32_KAHAN;
    switch (wf) {
    case WF_PN35: return kahan ? scan_pick_f32k_pn35(kern, o->K, d->nd) : scan_pick_f32n_pn35(kern, o->K, d->nd);
    case WF_TABLE: return kahan ? scan_pick_f32k_table(kern, o->K, d->nd) : scan_pick_f32n_table(kern, o->K, d->nd);
    default: return kahan ? scan_pick_f32k_newton(kern, o->K, d->nd) : scan_pick_f32n_newton(kern, o->K, d->nd);
    }
  }
  return scan_pick_bf16(o->precision, kern, o->K, d->nd);
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
  if (o->t_ref != SFT_REF_MID && o->t_ref != SFT_REF_START)
    return fail(SFT_E_INVALID, "scan: unknown reference time %d", o->t_ref);
  if (o->t_ref == SFT_REF_START && o->waveform == SFT_WF_SURROGATE)
    return fail(SFT_E_UNSUPPORTED, "scan: the surrogate waveform is evaluated at the SFT midpoints only");
  if (o->precision == SFT_PREC_FP64) {
    if (d->storage != SFT_STORE_F64) return fail(SFT_E_UNSUPPORTED, "scan: FP64 precision needs F64 storage");
  } else if (o->precision == SFT_PREC_FP32_KAHAN || o->precision == SFT_PREC_FP32_NAIVE) {
    if (d->storage == SFT_STORE_F64) return fail(SFT_E_UNSUPPORTED, "scan: FP32 precision needs F32 or BF16 storage");
  } else {
    return fail(SFT_E_INVALID, "scan: unknown precision %d", o->precision);
  }
  return SFT_OK;
}

// The F-statistic form (out->twoF set) exists for the Newtonian waveform with FP32-Kahan sums
// on F32 data or FP64 sums on F64 data.
static sft_status validate_fstat(const sft_data* d, const sft_opts* o, const sft_out* out)
{
  if (!out || !out->twoF) return SFT_OK;
  if (o->waveform != SFT_WF_NEWTON)
    return fail(SFT_E_UNSUPPORTED, "scan: the F-statistic is computed with the Newtonian waveform only");
  if (!((o->precision == SFT_PREC_FP32_KAHAN && d->storage == SFT_STORE_F32) || o->precision == SFT_PREC_FP64))
    return fail(SFT_E_UNSUPPORTED, "scan: the F-statistic needs FP32-Kahan sums on F32 data or FP64 sums");
  return SFT_OK;
}

// The Doppler form (bank->sky set) needs the data's ephemeris, the Newtonian waveform and
// FP32-Kahan sums on F32 data or FP64 sums on F64 data.
static sft_status validate_doppler(const sft_data* d, const sft_opts* o, const sft_bank* bank)
{
  if (!bank || !bank->sky) return SFT_OK;
  if (!d->g_eph) return fail(SFT_E_INVALID, "scan: bank.sky given but the data have no ephemeris (sft_set_ephemeris)");
  if (o->t_ref != SFT_REF_MID)
    return fail(SFT_E_UNSUPPORTED, "scan: the Doppler form uses the midpoint reference (its ephemeris is at the midpoints)");
  if (o->waveform != SFT_WF_NEWTON)
    return fail(SFT_E_UNSUPPORTED, "scan: the Doppler form is computed with the Newtonian waveform only");
  if (!((o->precision == SFT_PREC_FP32_KAHAN && d->storage == SFT_STORE_F32) || o->precision == SFT_PREC_FP64))
    return fail(SFT_E_UNSUPPORTED, "scan: the Doppler form needs FP32-Kahan sums on F32 data or FP64 sums");
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
  if (t->order != SFT_ORDER_GIVEN && t->order != SFT_ORDER_TRACK)
    return fail(SFT_E_RANGE, "tuning: order must be SFT_ORDER_GIVEN or SFT_ORDER_TRACK (got %d)", t->order);
  return SFT_OK;
}

// A scan prepared for launch: arguments, launch shape and workspace layout.
struct Prepared {
  ScanArgs a;
  ScanFn fn;
  const uint32_t* xflags;  // extra per-template flags ORed in by the finalize kernel (or null)
  const int32_t* perm;     // output position of each scanned template (or null: the given order)
  dim3 grid, block;
  int32_t nacc;            // partial sums per template and chunk: 6, or 7 in the F-statistic form
  size_t part_bytes, flag_bytes, counter_off, ws_bytes;
  int64_t n;
  double a_plus, a_cross;
};

static void bind_bank(ScanArgs& a, const sft_bank& b)
{
  a.mc = b.mc;
  a.q = b.q;
  a.t_c = b.t_c;
  a.phi_c = b.phi_c;
  a.a_first = b.a_first;
  a.a_last = b.a_last;
  a.sky = b.sky;
}

static sft_status prepare_scan(const sft_data* d, const sft_bank* bank, int64_t n, const sft_opts* o,
                               const sft_tuning& t, Prepared& P, bool fs, int wf = -1, const double* wtab = nullptr,
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
  bind_bank(a, *bank);
  a.g_eph = d->g_eph;
  a.n_tmpl = n;
  a.wtab = wtab;
  P.xflags = xflags;
  P.perm = nullptr;
  P.fn = pick_kernel(d, o, wf >= 0 ? wf : o->waveform, fs, bank->sky != nullptr);
  P.nacc = fs ? 7 : 6;
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
  P.part_bytes = (size_t)a.n_chunks * P.nacc * n * sizeof(double);
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
                     a.n_chunks, P.nacc, P.a_plus, P.a_cross, out->zp, out->zx, out->hhp, out->hhx, out->rho,
                     out->flags, P.xflags, P.nacc == 7 ? out->hhpx : nullptr, P.nacc == 7 ? out->twoF : nullptr,
                     P.perm, out->n_used);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------- bank order
// Workspace of SFT_ORDER_TRACK: the permutation, the sort's keys, indices and temporary
// storage, and the bank gathered into the sorted order.  Offsets are 256-byte aligned.
struct BankOrder {
  int64_t n = 0;
  size_t temp_bytes = 0, bytes = 0;
  size_t o_perm = 0, o_ka = 0, o_kb = 0, o_idx = 0, o_temp = 0;
  size_t o_mc = 0, o_q = 0, o_tc = 0, o_phi = 0, o_af = 0, o_al = 0, o_sky = 0;
  sft_bank given{};
  sft_bank sorted{};
  char* base = nullptr;
  int32_t* perm = nullptr;
};

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

static sft_status order_layout(const sft_bank* bank, int64_t n, BankOrder& B)
{
  B.n = n;
  B.given = *bank;
  hipError_t e = sort_temp_bytes(n, &B.temp_bytes);
  if (e != hipSuccess) return fail(SFT_E_DEVICE, "scan (track order): radix sort size: %s", hipGetErrorString(e));
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align256(off + bytes);
    return at;
  };
  const size_t u = (size_t)n;
  B.o_perm = take(u * sizeof(int32_t));
  B.o_ka = take(u * sizeof(uint64_t));
  B.o_kb = take(u * sizeof(uint64_t));
  B.o_idx = take(u * sizeof(int32_t));
  B.o_temp = take(B.temp_bytes);
  B.o_mc = take(u * sizeof(double));
  B.o_tc = take(u * sizeof(double));
  if (bank->q) B.o_q = take(u * sizeof(double));
  if (bank->phi_c) B.o_phi = take(u * sizeof(double));
  if (bank->a_first) B.o_af = take(u * sizeof(int32_t));
  if (bank->a_last) B.o_al = take(u * sizeof(int32_t));
  if (bank->sky) B.o_sky = take(3 * u * sizeof(double));
  B.bytes = off;
  return SFT_OK;
}

static void order_bind(BankOrder& B, void* base)
{
  char* c = (char*)base;
  B.base = c;
  B.perm = (int32_t*)(c + B.o_perm);
  B.sorted = sft_bank{};
  B.sorted.mc = (const double*)(c + B.o_mc);
  B.sorted.t_c = (const double*)(c + B.o_tc);
  if (B.given.q) B.sorted.q = (const double*)(c + B.o_q);
  if (B.given.phi_c) B.sorted.phi_c = (const double*)(c + B.o_phi);
  if (B.given.a_first) B.sorted.a_first = (const int32_t*)(c + B.o_af);
  if (B.given.a_last) B.sorted.a_last = (const int32_t*)(c + B.o_al);
  if (B.given.sky) B.sorted.sky = (const double*)(c + B.o_sky);
}

// the order of the given bank (keys, radix sort) into B.perm
static hipError_t order_sort(const sft_data* d, const sft_opts* o, BankOrder& B, hipStream_t st)
{
  SortKeyArgs k;
  k.mc = B.given.mc;
  k.t_c = B.given.t_c;
  k.a_first = B.given.a_first;
  k.a_last = B.given.a_last;
  k.row_tmid = d->row_tmid;
  k.n_sft = d->n_sft;
  k.T = d->T;
  k.tsun = o->tsun;
  k.n = B.n;
  return sort_by_track(k, B.base + B.o_temp, B.temp_bytes, (uint64_t*)(B.base + B.o_ka), (uint64_t*)(B.base + B.o_kb),
                       (int32_t*)(B.base + B.o_idx), B.perm, st);
}

// the given bank's arrays gathered into the order B.perm
static hipError_t order_gather(const BankOrder& B, hipStream_t st)
{
  const sft_bank& g = B.given;
  const sft_bank& s = B.sorted;
  hipError_t e = gather_f64(g.mc, B.perm, B.n, 1, (double*)s.mc, st);
  if (e == hipSuccess) e = gather_f64(g.t_c, B.perm, B.n, 1, (double*)s.t_c, st);
  if (e == hipSuccess && g.q) e = gather_f64(g.q, B.perm, B.n, 1, (double*)s.q, st);
  if (e == hipSuccess && g.phi_c) e = gather_f64(g.phi_c, B.perm, B.n, 1, (double*)s.phi_c, st);
  if (e == hipSuccess && g.a_first) e = gather_i32(g.a_first, B.perm, B.n, (int32_t*)s.a_first, st);
  if (e == hipSuccess && g.a_last) e = gather_i32(g.a_last, B.perm, B.n, (int32_t*)s.a_last, st);
  if (e == hipSuccess && g.sky) e = gather_f64(g.sky, B.perm, B.n, 3, (double*)s.sky, st);
  return e;
}

// scan P over the bank in the order B (bound to its workspace): gather, scan, finalize with perm
static hipError_t enqueue_ordered(Prepared& P, BankOrder& B, void* ws, sft_out* out, hipStream_t st, bool timed)
{
  hipError_t e = order_gather(B, st);
  if (e != hipSuccess) return e;
  bind_bank(P.a, B.sorted);
  P.perm = B.perm;
  return enqueue_scan(P, ws, out, st, timed);
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

// S_r(kappa) of SFT row r, linearly interpolated between the stored PSD bins floor(kappa) and
// floor(kappa) + 1 (the interpolation of the norm); 0 when either bin is outside the stored
// band or masked (stored as 0).
template <typename PS>
__device__ inline double psd_at(const PS* __restrict__ psd, int r, double kappa, int32_t k_lo, int32_t n_bins)
{
  const double kf = floor(kappa);
  const double i0 = kf - (double)k_lo;
  if (!(i0 >= 0.0 && i0 + 1.0 < (double)n_bins)) return 0.0;
  const PS* p = psd + (int64_t)r * n_bins + (int64_t)i0;
  const double S0 = (double)p[0], S1 = (double)p[1];
  if (!(S0 > 0.0) || !(S1 > 0.0)) return 0.0;
  const double w = kappa - kf;
  return (1.0 - w) * S0 + w * S1;
}

// One lane per template of the batch: the surrogate chirp of every group the template
// uses (Newtonian chirp plus the network's corrections), the judge against the 3.5PN
// chirp, and the chirp table the scan reads (the 3.5PN chirps for a rejected template).
// The judge's weight of SFT row r is A_PN^2 T / S_r(f_PN) (the row's share of <h,h>); rows
// whose PSD is masked or outside the stored band at f_PN carry no weight.
template <typename PS>
__global__ __launch_bounds__(256) void sur_post_kernel(SurArgs sa, const double* __restrict__ mc,
                                                       const double* __restrict__ q, const double* __restrict__ t_c,
                                                       const double* __restrict__ phi_c, const int32_t* __restrict__ a_first,
                                                       const int32_t* __restrict__ a_last,
                                                       const double* __restrict__ g_tmid, const int32_t* __restrict__ g_rows,
                                                       int64_t nb, int32_t n_groups, double T,
                                                       const double* __restrict__ Y, const double* __restrict__ dY,
                                                       double* __restrict__ tab, uint32_t* __restrict__ xflags,
                                                       double* __restrict__ mismatch, const PS* __restrict__ psd,
                                                       int32_t k_lo, int32_t n_bins)
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
    // judge term: A_PN^2 T / S_r(f_PN) exp(i dphi) sinc(dkappa), summed over the group's rows
    const Chirp cp = pn35_chirp(tau, pm.nu, pm.inv5Mnu, pm.Mt, pm.nu25, phic, T, pc);
    const double dk = cs.kappa - cp.kappa;
    const double snc = fabs(dk) < 1e-8 ? 1.0 - kPi * kPi * dk * dk / 6.0 : sin(kPi * dk) / (kPi * dk);
    double inv_s = 0.0;
    for (int d = 0; d < SFT_GROUP_MAX; ++d) {
      const int rr = g_rows[g * SFT_GROUP_MAX + d];
      if (rr < 0 || rr < lo || rr > hi) continue;
      const double S = psd_at(psd, rr, cp.kappa, k_lo, n_bins);
      if (S > 0.0) inv_s += 1.0 / S;
    }
    const double wt = cp.amp * cp.amp * T * inv_s;
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
  sft_status s = prepare_scan(d, bank, B, o, d->tune, P0, false, WF_TABLE, nullptr, nullptr);
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
    if ((s = prepare_scan(d, bank, nb, o, d->tune, Pt, false, WF_TABLE, nullptr, nullptr)) != SFT_OK) return s;
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
    if (ob.n_used) ob.n_used += m0;
    hipLaunchKernelGGL(sur_inputs_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, sa, b.mc, b.q, b.t_c,
                       d->g_tmid, nb, d->n_groups, U);
    if ((e = hipGetLastError()) != hipSuccess) break;
    if ((e = mlp_infer(sur, U, rows, Y, dY, ws + off_nn, chunk, st)) != hipSuccess) break;
    if (d->storage == SFT_STORE_F64)
      hipLaunchKernelGGL(sur_post_kernel<double>, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, sa, b.mc, b.q,
                         b.t_c, b.phi_c, b.a_first, b.a_last, d->g_tmid, d->g_rows, nb, d->n_groups, d->T, Y, dY, tab,
                         xf, ob.mismatch, (const double*)d->psd, d->k_lo, d->n_bins);
    else
      hipLaunchKernelGGL(sur_post_kernel<float>, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, sa, b.mc, b.q,
                         b.t_c, b.phi_c, b.a_first, b.a_last, d->g_tmid, d->g_rows, nb, d->n_groups, d->T, Y, dY, tab,
                         xf, ob.mismatch, (const float*)d->psd, d->k_lo, d->n_bins);
    if ((e = hipGetLastError()) != hipSuccess) break;
    Prepared P;
    if ((s = prepare_scan(d, &b, nb, o, d->tune, P, false, WF_TABLE, tab, xf)) != SFT_OK) break;
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
  if ((s = validate_io(bank, n, out)) != SFT_OK || (s = validate_fstat(d, o, out)) != SFT_OK ||
      (s = validate_doppler(d, o, bank)) != SFT_OK || n == 0) return s;
  hipStream_t st = (hipStream_t)hip_stream;
  if (o->waveform == SFT_WF_SURROGATE) return surrogate_scan(d, bank, n, o, out, st);
  Prepared P;
  if ((s = prepare_scan(d, bank, n, o, d->tune, P, out->twoF != nullptr)) != SFT_OK) return s;
  const bool track = d->tune.order == SFT_ORDER_TRACK && n > 1;
  BankOrder B;
  if (track && (s = order_layout(bank, n, B)) != SFT_OK) return s;
  void* ws = nullptr;
  HIP_OR_FAIL(hipMallocAsync(&ws, P.ws_bytes + (track ? B.bytes : 0), st));
  hipError_t e;
  if (track) {
    order_bind(B, (char*)ws + P.ws_bytes);
    e = order_sort(d, o, B, st);
    if (e == hipSuccess) e = enqueue_ordered(P, B, ws, out, st, true);
  } else {
    e = enqueue_scan(P, ws, out, st, true);
  }
  hipError_t e2 = hipFreeAsync(ws, st);
  if (e != hipSuccess) return fail(SFT_E_DEVICE, "scan: launch failed: %s", hipGetErrorString(e));
  if (e2 != hipSuccess) return fail(SFT_E_DEVICE, "scan: hipFreeAsync: %s", hipGetErrorString(e2));
  return SFT_OK;
}

// ---------------------------------------------------------------------------- allocation-free scan
// Workspace of sft_template_bank_scan_noalloc: one file-scope array per GPU, held until the
// process ends.  In host code `scratch` only names the symbol; its address on a device comes
// from hipGetSymbolAddress with that device current (each GPU has its own copy), resolved once
// per device and kept in g_scratch_ptr.  Only that address is ever handed to kernels.
static __device__ __align__(256) unsigned char scratch[SFT_NOALLOC_SCRATCH_BYTES];
static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static sft_status scratch_address(int dev, void** out)
{
  if (dev < 0 || dev >= kMaxDevices) return fail(SFT_E_RANGE, "scan (no-alloc): device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SFT_E_DEVICE, "scan (no-alloc): hipGetSymbolAddress: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SFT_OK;
}

extern "C" sft_status sft_template_bank_scan_noalloc(const sft_data* d, const sft_bank* bank, int64_t n,
                                                     const sft_opts* o, sft_out* out, void* hip_stream)
{
  sft_status s = validate_scan(d, o);
  if (s != SFT_OK) return s;
  if ((s = validate_io(bank, n, out)) != SFT_OK || (s = validate_fstat(d, o, out)) != SFT_OK ||
      (s = validate_doppler(d, o, bank)) != SFT_OK || n == 0) return s;
  if (o->waveform == SFT_WF_SURROGATE)
    return fail(SFT_E_UNSUPPORTED, "scan (no-alloc): the surrogate waveform needs its batch workspace");
  const bool fs = out->twoF != nullptr;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != d->device)
    return fail(SFT_E_INVALID, "scan (no-alloc): the data live on device %d, not on the current device", d->device);
  // the handle's launch shape, with fewer (larger) chunks when its partial sums would not fit
  sft_tuning t = d->tune;
  Prepared P;
  if ((s = prepare_scan(d, bank, n, o, t, P, fs)) != SFT_OK) return s;
  if (P.ws_bytes > SFT_NOALLOC_SCRATCH_BYTES) {
    const size_t per_chunk = (P.part_bytes + P.flag_bytes) / (size_t)P.a.n_chunks;   // bytes per chunk
    const size_t room = SFT_NOALLOC_SCRATCH_BYTES - 512;   // counter slot and alignment
    const int64_t nc_max = (int64_t)(room / per_chunk);
    if (nc_max < 1)
      return fail(SFT_E_RANGE, "scan (no-alloc): %lld templates need %zu bytes of partial sums, more than the %u-byte scratch",
                  (long long)n, per_chunk, (unsigned)SFT_NOALLOC_SCRATCH_BYTES);
    if (t.block == 0 && t.chunk_groups == 0 && t.persistent == 0) t.persistent = 1;   // keep the automatic grid
    t.chunk_groups = (int32_t)((d->n_groups + nc_max - 1) / nc_max);
    if ((s = prepare_scan(d, bank, n, o, t, P, fs)) != SFT_OK) return s;
    if (P.ws_bytes > SFT_NOALLOC_SCRATCH_BYTES)
      return fail(SFT_E_RANGE, "scan (no-alloc): workspace of %zu bytes exceeds the scratch", P.ws_bytes);
  }
  void* ws = nullptr;
  if ((s = scratch_address(dev, &ws)) != SFT_OK) return s;
  hipError_t e = enqueue_scan(P, ws, out, (hipStream_t)hip_stream, false);
  if (e != hipSuccess) return fail(SFT_E_DEVICE, "scan (no-alloc): launch failed: %s", hipGetErrorString(e));
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
  return SFT_OK;
}

extern "C" sft_status sft_autotune(sft_data* d, const sft_bank* bank, int64_t n, const sft_opts* o, sft_out* out,
                                   void* hip_stream, int32_t reps, sft_tuning* best, float* best_ms)
{
  sft_status s = validate_scan(d, o);
  if (s != SFT_OK) return s;
  if ((s = validate_io(bank, n, out)) != SFT_OK || (s = validate_fstat(d, o, out)) != SFT_OK ||
      (s = validate_doppler(d, o, bank)) != SFT_OK) return s;
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
    if ((s = prepare_scan(d, bank, n, o, cand[i], preps[i], out->twoF != nullptr)) != SFT_OK) return s;
    ws_max = std::max(ws_max, preps[i].ws_bytes);
  }
  void* ws = nullptr;
  HIP_OR_FAIL(hipMallocAsync(&ws, ws_max, st));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  // mean time of reps launches of candidate i after one warm-up launch
  auto time_cand = [&](size_t i, float& ms) -> hipError_t {
    hipError_t r = enqueue_scan(preps[i], ws, out, st, false);
    if (r == hipSuccess) r = hipEventRecord(e0, st);
    for (int k = 0; k < reps && r == hipSuccess; ++k) r = enqueue_scan(preps[i], ws, out, st, false);
    if (r == hipSuccess) r = hipEventRecord(e1, st);
    if (r == hipSuccess) r = hipEventSynchronize(e1);
    if (r == hipSuccess) r = hipEventElapsedTime(&ms, e0, e1);
    ms /= (float)reps;
    return r;
  };
  std::vector<float> t1(cand.size(), 3.4e38f);
  float bms = 3.4e38f;
  size_t bi = 0;
  for (size_t i = 0; i < cand.size() && e == hipSuccess; ++i) {
    e = time_cand(i, t1[i]);
    if (e == hipSuccess && t1[i] < bms) {
      bms = t1[i];
      bi = i;
    }
  }
  // Candidates within 2% of the best are timed again, in turn, twice: near-equal shapes are
  // then told apart by their best repeated time rather than by the noise of one pass.
  std::vector<size_t> close;
  for (size_t i = 0; i < cand.size(); ++i)
    if (t1[i] <= 1.02f * bms) close.push_back(i);
  if (e == hipSuccess && close.size() > 1) {
    std::vector<float> t2(cand.size(), 3.4e38f);
    for (int pass = 0; pass < 2 && e == hipSuccess; ++pass)
      for (size_t i : close) {
        float ms = 0.f;
        if ((e = time_cand(i, ms)) != hipSuccess) break;
        t2[i] = std::min(t2[i], ms);
      }
    if (e == hipSuccess) {
      bms = 3.4e38f;
      for (size_t i : close)
        if (t2[i] < bms) {
          bms = t2[i];
          bi = i;
        }
    }
  }
  hipError_t e2 = hipFreeAsync(ws, st);
  ws = nullptr;
  // the fastest tuning again with the bank sorted by track (the sort timed with it)
  sft_tuning bt = cand[bi];
  BankOrder B;
  if (e == hipSuccess && e2 == hipSuccess && n > 1) {
    if ((s = order_layout(bank, n, B)) != SFT_OK) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return s;
    }
    Prepared P = preps[bi];
    e = hipMallocAsync(&ws, P.ws_bytes + B.bytes, st);
    if (e == hipSuccess) {
      order_bind(B, (char*)ws + P.ws_bytes);
      hipError_t el = order_sort(d, o, B, st);
      if (el == hipSuccess) el = enqueue_ordered(P, B, ws, out, st, false);   // warm-up
      if (el == hipSuccess) el = hipEventRecord(e0, st);
      for (int r = 0; r < reps && el == hipSuccess; ++r) {
        el = order_sort(d, o, B, st);
        if (el == hipSuccess) el = enqueue_ordered(P, B, ws, out, st, false);
      }
      if (el == hipSuccess) el = hipEventRecord(e1, st);
      if (el == hipSuccess) el = hipEventSynchronize(e1);
      float ms = 0.f;
      if (el == hipSuccess) el = hipEventElapsedTime(&ms, e0, e1);
      if (el == hipSuccess && ms / (float)reps < bms) {
        bms = ms / (float)reps;
        bt.order = SFT_ORDER_TRACK;
      } else if (el == hipSuccess) {
        el = enqueue_scan(preps[bi], ws, out, st, false);   // outputs of the kept tuning
      }
      e = el;
      e2 = hipFreeAsync(ws, st);
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(SFT_E_DEVICE, "sft_autotune: %s", hipGetErrorString(e));
  if (e2 != hipSuccess) return fail(SFT_E_DEVICE, "sft_autotune: hipFreeAsync: %s", hipGetErrorString(e2));
  d->tune = bt;
  if (best) *best = bt;
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
  BankOrder B;   // with SFT_ORDER_TRACK: the order fixed at creation (B.perm) and the gathered bank
  bool track;
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
  if ((s = validate_io(bank, n, out)) != SFT_OK || (s = validate_fstat(d, o, out)) != SFT_OK ||
      (s = validate_doppler(d, o, bank)) != SFT_OK) return s;
  if (n == 0) return fail(SFT_E_INVALID, "sft_plan_create: needs at least one template");
  if (o->waveform == SFT_WF_SURROGATE)
    return fail(SFT_E_UNSUPPORTED, "sft_plan_create: the surrogate waveform is not captured into graphs");
  sft_plan* p = new sft_plan();
  p->ws = nullptr;
  p->graph = nullptr;
  p->exec = nullptr;
  p->out = *out;
  if ((s = prepare_scan(d, bank, n, o, d->tune, p->P, out->twoF != nullptr)) != SFT_OK) {
    delete p;
    return s;
  }
  p->track = d->tune.order == SFT_ORDER_TRACK && n > 1;
  if (p->track && (s = order_layout(bank, n, p->B)) != SFT_OK) {
    delete p;
    return s;
  }
  hipError_t e = hipMalloc(&p->ws, p->P.ws_bytes + (p->track ? p->B.bytes : 0));
  if (e != hipSuccess) {
    sft_plan_destroy(p);
    return fail(e == hipErrorOutOfMemory ? SFT_E_NOMEM : SFT_E_DEVICE, "sft_plan_create: hipMalloc: %s", hipGetErrorString(e));
  }
  hipStream_t cs = nullptr;
  e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e == hipSuccess && p->track) {
    // the order of the bank's contents now (work queued on other streams finished first);
    // the radix sort stays outside the graph
    order_bind(p->B, (char*)p->ws + p->P.ws_bytes);
    e = hipDeviceSynchronize();
    if (e == hipSuccess) e = order_sort(d, o, p->B, cs);
    if (e == hipSuccess) e = hipStreamSynchronize(cs);
  }
  if (e == hipSuccess) {
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t el = p->track ? enqueue_ordered(p->P, p->B, p->ws, &p->out, cs, false)
                               : enqueue_scan(p->P, p->ws, &p->out, cs, false);
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(cs, &g);
      p->graph = g;
      if (el != hipSuccess) e = el;
    }
  }
  if (cs) (void)hipStreamDestroy(cs);
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
