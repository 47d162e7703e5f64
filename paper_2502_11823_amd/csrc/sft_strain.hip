// sft_strain.hip -- SFTs of raw strain series on the device (Sec. III.B segmentation,
// Eq. d_SFT) with the per-SFT noise PSD estimate (bias-corrected running median of the SFT's
// own periodogram), gaps detected as segments holding a non-finite sample.
//
// strain_sft_kernel: one workgroup per segment of n = 2M samples.  The real series is taken as
// M complex points z[m] = x[2m] + i x[2m+1], loaded in bit-reversed order into LDS and
// transformed in place by log2(M) radix-2 decimation-in-time stages (FP64); the n/2 + 1 bins of
// the real transform follow from Z[k] and conj(Z[M - k]):
//   X[k] = (Z[k] + conj(Z[M-k])) / 2 - i e^{-2 pi i k / n} (Z[k] - conj(Z[M-k])) / 2.
// The band bins are written as dt X[k]; the PSD of band bin k is 2 median(P) / (T B) over the
// block of N = 2w+1 periodogram values P[j] = |dt X[j]|^2 centred on k (shifted at the ends of
// [0, n/2]), with B the mean of the middle order statistic of N unit exponentials.  The median
// is the sorted block's middle element (ties broken by bin): found by a wavefront-wide sort of
// the union of 64 neighbouring blocks (half widths w <= 32), or by rank counting per bin.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/sft.h"

sft_status sft_set_error(sft_status st, const char* msg);

namespace {

constexpr int kStrainBlock = 256;

__device__ inline double2 cmul(double2 a, double2 b)
{
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}

__device__ inline double pw(const double2* X, int j)
{
  const double2 v = X[j];
  return fma(v.x, v.x, v.y * v.y);
}

// Median of each lane's block by a wavefront-wide sort: the 64 lanes of a wavefront take 64
// consecutive band bins, whose blocks of 2w+1 periodogram values lie in a union of at most
// 64 + 2w <= 128 bins.  The union's (value, bin) pairs are sorted once per wavefront by a
// bitonic network in the wavefront's LDS slot (one compare-exchange per lane and stage), then
// every lane walks the sorted list and stops at the (w+1)-th entry that falls in its block:
// the block's middle element in (value, bin) order, as a sort of the block itself gives.
constexpr int kSortN = 128;
constexpr int kMaxSortW = (kSortN - 64) / 2;   // w <= 32

__device__ inline void wave_sync()
{
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline bool pair_less(double va, int ia, double vb, int ib)
{
  return va < vb || (va == vb && ia < ib);
}

__global__ __launch_bounds__(kStrainBlock) void strain_sft_kernel(
    const double* __restrict__ x, int64_t n_total, int32_t n_seg, int32_t logM, double dt, int32_t w, double psd_scale,
    int32_t k_lo, int32_t n_bins, int32_t staged, double s_white, const double2* __restrict__ tw,
    const double2* __restrict__ rtw, double* __restrict__ bins, double* __restrict__ psd, int32_t* __restrict__ keep)
{
  // LDS: buf[M + 1] complex; with staged = 1 a region of M + 1 doubles after it, holding the
  // twiddles during the transform and the periodogram afterwards
  extern __shared__ double2 buf[];
  __shared__ int s_bad;
  __shared__ double s_val[kStrainBlock / 64][kSortN];
  __shared__ int s_idx[kStrainBlock / 64][kSortN];
  const int M = 1 << logM;
  double* U = reinterpret_cast<double*>(buf + M + 1);
  double2* tws = reinterpret_cast<double2*>(U);
  const int row = blockIdx.x;
  const int det = row / n_seg, seg = row - det * n_seg;
  const double* xs = x + (int64_t)det * n_total + (int64_t)seg * 2 * M;
  const int tid = threadIdx.x;
  if (tid == 0) s_bad = 0;
  __syncthreads();
  bool bad = false;
  // z[m] = x[2m] + i x[2m+1]: one 16-byte load per point where the segment is 16-byte aligned
  if ((reinterpret_cast<uintptr_t>(xs) & 15) == 0) {
    const double2* xs2 = reinterpret_cast<const double2*>(xs);
    for (int m = tid; m < M; m += blockDim.x) {
      const double2 z = xs2[m];
      bad = bad || !isfinite(z.x) || !isfinite(z.y);
      buf[(int)(__brev((unsigned)m) >> (32 - logM))] = z;
    }
  } else {
    for (int m = tid; m < M; m += blockDim.x) {
      const double re = xs[2 * m], im = xs[2 * m + 1];
      bad = bad || !isfinite(re) || !isfinite(im);
      buf[(int)(__brev((unsigned)m) >> (32 - logM))] = make_double2(re, im);
    }
  }
  if (staged)
    for (int j = tid; j < M / 2; j += blockDim.x) tws[j] = tw[j];
  if (bad) s_bad = 1;
  __syncthreads();
  double* bo = bins + (int64_t)row * 2 * n_bins;
  double* po = psd + (int64_t)row * n_bins;
  if (s_bad) {
    for (int i = tid; i < n_bins; i += blockDim.x) {
      bo[2 * i] = 0.0;
      bo[2 * i + 1] = 0.0;
      po[i] = 0.0;
    }
    if (tid == 0) keep[row] = 0;
    return;
  }
  // radix-2 stages; tw[j] = e^{-2 pi i j / M}, j < M / 2
  const double2* twp = staged ? tws : tw;
  for (int s = 1; s <= logM; ++s) {
    const int half = 1 << (s - 1);
    const int tstride = M >> s;
    for (int b = tid; b < M / 2; b += blockDim.x) {
      const int k = b & (half - 1);
      const int i = ((b >> (s - 1)) << s) + k;
      const double2 u = buf[i];
      const double2 v = cmul(buf[i + half], twp[k * tstride]);
      buf[i] = make_double2(u.x + v.x, u.y + v.y);
      buf[i + half] = make_double2(u.x - v.x, u.y - v.y);
    }
    __syncthreads();
  }
  // real-transform bins, in place, pair (k, M - k) per thread; rtw[k] = e^{-2 pi i k / n}, k <= M/2
  for (int k = tid; k <= M / 2; k += blockDim.x) {
    const int kk = (M - k) & (M - 1);  // M - k, with Z[M] = Z[0]
    const double2 a = buf[k], b = buf[kk];
    // X[k]
    const double2 e = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));   // (Z[k] + conj Z[M-k]) / 2
    const double2 o = make_double2(0.5 * (a.x - b.x), 0.5 * (a.y + b.y));   // (Z[k] - conj Z[M-k]) / 2
    const double2 ro = cmul(rtw[k], o);
    const double2 Xk = make_double2(e.x + ro.y, e.y - ro.x);                // e - i ro
    // X[M - k] from the same pair with the roles exchanged: e' = conj(e), o' = -conj(o),
    // e^{-2 pi i (M-k)/n} = -conj(e^{-2 pi i k / n})
    const double2 rc = make_double2(-rtw[k].x, rtw[k].y);
    const double2 o2 = make_double2(-o.x, o.y);
    const double2 ro2 = cmul(rc, o2);
    const double2 Xm = make_double2(e.x + ro2.y, -e.y - ro2.x);
    if (k == 0) {
      buf[0] = Xk;
      buf[M] = Xm;   // Nyquist bin
    } else if (2 * k == M) {
      buf[k] = Xk;   // the pair's two members coincide
    } else {
      buf[k] = Xk;
      buf[M - k] = Xm;
    }
  }
  __syncthreads();
  if (staged) {
    // the periodogram, over the twiddles (the transform is done)
    for (int j = tid; j <= M; j += blockDim.x) U[j] = pw(buf, j);
    __syncthreads();
  }
  for (int i = tid; i < n_bins; i += blockDim.x) {
    const double2 v = buf[k_lo + i];
    bo[2 * i] = dt * v.x;
    bo[2 * i + 1] = dt * v.y;
  }
  auto P = [&](int j) { return staged ? U[j] : pw(buf, j); };
  const int N = 2 * w + 1;
  if (s_white > 0.0) {
    // a known white PSD: no estimate
    for (int i = tid; i < n_bins; i += blockDim.x) po[i] = s_white;
  } else if (w <= kMaxSortW) {
    const int lane = tid & 63, wv = tid >> 6;
    double* sv = s_val[wv];
    int* si = s_idx[wv];
    // every wavefront walks its chunks of 64 band bins (wave-uniform loop)
    for (int c0 = wv * 64; c0 < n_bins; c0 += blockDim.x) {
      const int kb = k_lo + c0;
      int u0 = kb - w;                          // the union of the chunk's blocks: [u0, u0 + L)
      u0 = u0 < 0 ? 0 : u0;
      u0 = u0 + 2 * w > M ? M - 2 * w : u0;
      int u1 = kb + 63 - w;
      u1 = u1 < 0 ? 0 : u1;
      u1 = u1 + 2 * w > M ? M - 2 * w : u1;
      const int L = u1 + N - u0;                // <= 64 + 2w <= kSortN
      for (int q = lane; q < kSortN; q += 64) {
        sv[q] = q < L ? P(u0 + q) : INFINITY;
        si[q] = q < L ? u0 + q : 0x7fffffff;
      }
      wave_sync();
      // bitonic sort of the kSortN pairs: lane l compare-exchanges one pair per stage
      for (int size = 2; size <= kSortN; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
          const int q = 2 * lane - (lane & (stride - 1));   // lower index of lane's pair
          const int r = q + stride;
          const bool up = (q & size) == 0;
          const double vq = sv[q], vr = sv[r];
          const int iq = si[q], ir = si[r];
          const bool swap = up ? pair_less(vr, ir, vq, iq) : pair_less(vq, iq, vr, ir);
          wave_sync();
          if (swap) {
            sv[q] = vr;
            si[q] = ir;
            sv[r] = vq;
            si[r] = iq;
          }
          wave_sync();
        }
      }
      // every lane counts, along the sorted list, the entries inside its own block; its median
      // is the entry at which that count reaches w + 1.  The list is read as broadcasts in a
      // wave-uniform loop without an early exit, so the reads pipeline.
      const int i = c0 + lane;
      const int k = k_lo + i;
      int s0 = k - w;
      s0 = s0 < 0 ? 0 : s0;
      s0 = s0 + 2 * w > M ? M - 2 * w : s0;
      int cnt = 0;
      double med = 0.0;
#pragma unroll 8
      for (int q = 0; q < L; ++q) {
        const int j = si[q];
        const bool in = j >= s0 && j < s0 + N;
        med = (in && cnt == w) ? sv[q] : med;
        cnt += in ? 1 : 0;
      }
      if (i < n_bins) po[i] = psd_scale * (dt * dt) * med;
      wave_sync();
    }
  } else {
    // wide blocks: rank counting per bin (ties broken by position)
    for (int i = tid; i < n_bins; i += blockDim.x) {
      const int k = k_lo + i;
      int s0 = k - w;
      s0 = s0 < 0 ? 0 : s0;
      s0 = s0 + 2 * w > M ? M - 2 * w : s0;
      double med = 0.0;
      for (int a = 0; a < N; ++a) {
        const double pa = P(s0 + a);
        int rank = 0;
        for (int b = 0; b < N; ++b) {
          const double pb = P(s0 + b);
          rank += (pb < pa || (pb == pa && b < a)) ? 1 : 0;
        }
        if (rank == w) {
          med = pa;
          break;
        }
      }
      po[i] = psd_scale * (dt * dt) * med;
    }
  }
  if (tid == 0) keep[row] = 1;
}

// Segments whose length n is not a power of two: the band bins by their defining sum
// X[k] = sum_j x_j e^{-2 pi i j k / n} (Eq. d_SFT), one bin per thread, the segment in LDS (read
// as a broadcast), the twiddle advanced by the rotation e^{-2 pi i k / n} and re-anchored from
// the exact table W[m] = e^{-2 pi i m / n} every kAnchor samples (rounding drift <= kAnchor eps).
// The PSD is the given white level (no estimate).
constexpr int kAnchor = 256;

__global__ __launch_bounds__(kStrainBlock) void strain_dft_kernel(
    const double* __restrict__ x, int64_t n_total, int32_t n_seg, int32_t n, double dt, double s_white,
    int32_t k_lo, int32_t n_bins, const double2* __restrict__ W, double* __restrict__ bins, double* __restrict__ psd,
    int32_t* __restrict__ keep)
{
  extern __shared__ double xl[];   // the segment, n values
  __shared__ int s_bad;
  const int row = blockIdx.x;
  const int det = row / n_seg, seg = row - det * n_seg;
  const double* xs = x + (int64_t)det * n_total + (int64_t)seg * n;
  const int tid = threadIdx.x;
  if (tid == 0) s_bad = 0;
  __syncthreads();
  bool bad = false;
  for (int j = tid; j < n; j += blockDim.x) {
    const double v = xs[j];
    bad = bad || !isfinite(v);
    xl[j] = v;
  }
  if (bad) s_bad = 1;
  __syncthreads();
  double* bo = bins + (int64_t)row * 2 * n_bins;
  double* po = psd + (int64_t)row * n_bins;
  if (s_bad) {
    for (int i = tid; i < n_bins; i += blockDim.x) {
      bo[2 * i] = 0.0;
      bo[2 * i + 1] = 0.0;
      po[i] = 0.0;
    }
    if (tid == 0) keep[row] = 0;
    return;
  }
  for (int i = tid; i < n_bins; i += blockDim.x) {
    const int k = k_lo + i;
    const double2 r = W[k % n];
    const int step = (int)(((int64_t)kAnchor * k) % n);
    double re = 0.0, im = 0.0;
    int idx = 0;   // (j0 k) mod n
    for (int j0 = 0; j0 < n; j0 += kAnchor) {
      double2 wv = W[idx];
      const int j1 = j0 + kAnchor < n ? j0 + kAnchor : n;
      for (int j = j0; j < j1; ++j) {
        const double xj = xl[j];
        re = fma(xj, wv.x, re);
        im = fma(xj, wv.y, im);
        wv = cmul(wv, r);
      }
      idx += step;
      idx = idx >= n ? idx - n : idx;
    }
    bo[2 * i] = dt * re;
    bo[2 * i + 1] = dt * im;
    po[i] = s_white;
  }
  if (tid == 0) keep[row] = 1;
}

}  // namespace

static sft_status strain_fail(sft_status st, const char* msg) { return sft_set_error(st, msg); }

extern "C" sft_status sft_make_sfts(const sft_strain_desc* d, const double* x, double* bins, double* psd, int32_t* keep,
                                    void* hip_stream)
{
  if (!d || !x || !bins || !psd || !keep) return strain_fail(SFT_E_INVALID, "sft_make_sfts: null argument");
  const int n = d->n_samples;
  const bool pow2 = (n & (n - 1)) == 0;
  if (n < 16 || n > 16384 || (n & 1))
    return strain_fail(SFT_E_UNSUPPORTED, "sft_make_sfts: n_samples must be even and in [16, 16384]");
  if (!pow2 && !(d->s_white > 0.0))
    return strain_fail(SFT_E_UNSUPPORTED, "sft_make_sfts: the PSD estimate needs n a power of two (else give s_white)");
  if (d->n_det < 1 || d->n_total < n || !(d->dt > 0.0) || !(d->s_white >= 0.0))
    return strain_fail(SFT_E_INVALID, "sft_make_sfts: bad descriptor");
  const int M = n / 2;
  if (d->k_lo < 0 || d->n_bins < 1 || d->k_lo + d->n_bins - 1 > M)
    return strain_fail(SFT_E_INVALID, "sft_make_sfts: band outside [0, n/2]");
  if (!(d->s_white > 0.0) && (d->psd_w < 0 || 2 * d->psd_w + 1 > M + 1))
    return strain_fail(SFT_E_INVALID, "sft_make_sfts: running-median block wider than the spectrum");
  const int64_t n_seg = d->n_total / n;
  if (n_seg * d->n_det > INT32_MAX) return strain_fail(SFT_E_RANGE, "sft_make_sfts: too many segments");
  hipStream_t st = (hipStream_t)hip_stream;
  const long double pi = 3.141592653589793238462643383279502884L;
  if (!pow2) {
    std::vector<double2> W(n);
    for (int m = 0; m < n; ++m) {
      const long double a = -2.0L * pi * (long double)m / (long double)n;
      W[m] = make_double2((double)cosl(a), (double)sinl(a));
    }
    double2* d_W = nullptr;
    hipError_t e = hipMallocAsync((void**)&d_W, n * sizeof(double2), st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_W, W.data(), n * sizeof(double2), hipMemcpyHostToDevice, st);
    const size_t lds = (size_t)n * sizeof(double);
    if (e == hipSuccess && lds > 65536)
      e = hipFuncSetAttribute((const void*)strain_dft_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess && n_seg > 0) {
      hipLaunchKernelGGL(strain_dft_kernel, dim3((unsigned)(n_seg * d->n_det)), dim3(kStrainBlock), lds, st, x,
                         d->n_total, (int32_t)n_seg, n, d->dt, d->s_white, d->k_lo, d->n_bins, d_W, bins, psd, keep);
      e = hipGetLastError();
    }
    hipError_t e2 = hipStreamSynchronize(st);   // W is read by the upload
    if (d_W) (void)hipFreeAsync(d_W, st);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) return strain_fail(SFT_E_DEVICE, hipGetErrorString(e));
    return SFT_OK;
  }
  int logM = 0;
  while ((1 << logM) < M) ++logM;
  // twiddles in long double, rounded once
  std::vector<double2> tw(M / 2 > 0 ? M / 2 : 1), rtw(M / 2 + 1);
  for (int j = 0; j < M / 2; ++j) {
    const long double a = -2.0L * pi * (long double)j / (long double)M;
    tw[j] = make_double2((double)cosl(a), (double)sinl(a));
  }
  for (int k = 0; k <= M / 2; ++k) {
    const long double a = -2.0L * pi * (long double)k / (long double)n;
    rtw[k] = make_double2((double)cosl(a), (double)sinl(a));
  }
  double B = 0.0;
  for (int i = 0; i <= d->psd_w; ++i) B += 1.0 / (double)(2 * d->psd_w + 1 - i);
  const double T = d->dt * n;
  const double psd_scale = 2.0 / (T * B);
  double2 *d_tw = nullptr, *d_rtw = nullptr;
  hipError_t e = hipMallocAsync((void**)&d_tw, tw.size() * sizeof(double2), st);
  if (e == hipSuccess) e = hipMallocAsync((void**)&d_rtw, rtw.size() * sizeof(double2), st);
  if (e == hipSuccess) e = hipMemcpyAsync(d_tw, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(d_rtw, rtw.data(), rtw.size() * sizeof(double2), hipMemcpyHostToDevice, st);
  // the twiddles and the periodogram are staged in LDS beside the spectrum when both fit
  const int staged = M <= 4096 ? 1 : 0;
  const size_t lds = (size_t)(M + 1) * (sizeof(double2) + (staged ? sizeof(double) : 0));
  if (e == hipSuccess && lds > 65536)
    e = hipFuncSetAttribute((const void*)strain_sft_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess && n_seg > 0) {
    hipLaunchKernelGGL(strain_sft_kernel, dim3((unsigned)(n_seg * d->n_det)), dim3(kStrainBlock), lds, st, x,
                       d->n_total, (int32_t)n_seg, logM, d->dt, d->psd_w, psd_scale, d->k_lo, d->n_bins, staged,
                       d->s_white, d_tw, d_rtw, bins, psd, keep);
    e = hipGetLastError();
  }
  // the twiddle uploads read host vectors: finish before they go out of scope
  hipError_t e2 = hipStreamSynchronize(st);
  if (d_tw) (void)hipFreeAsync(d_tw, st);
  if (d_rtw) (void)hipFreeAsync(d_rtw, st);
  if (e == hipSuccess) e = e2;
  if (e != hipSuccess) return strain_fail(SFT_E_DEVICE, hipGetErrorString(e));
  return SFT_OK;
}
