// sft_strain.hip -- SFTs of raw strain series on the device (Sec. III.B segmentation,
// Eq. d_SFT) with the per-SFT noise PSD estimate (bias-corrected running median of the SFT's
// own periodogram), gaps detected as segments holding a non-finite sample.
//
// strain_sft_kernel: one workgroup per segment of n = 2M samples.  The real series is taken as
// M complex points z[m] = x[2m] + i x[2m+1], loaded in natural order into LDS and transformed
// in place by radix-8 decimation-in-frequency passes (FP64); the n/2 + 1 bins of the real
// transform follow from Z[k] and conj(Z[M - k]):
//   X[k] = (Z[k] + conj(Z[M-k])) / 2 - i e^{-2 pi i k / n} (Z[k] - conj(Z[M-k])) / 2.
// The band bins are written as dt X[k]; the PSD of band bin k is 2 median(P) / (T B) over the
// block of N = 2w+1 periodogram values P[j] = |dt X[j]|^2 centred on k (shifted at the ends of
// [0, n/2]), with B the mean of the middle order statistic of N unit exponentials.  The median
// is the sorted block's middle element (ties broken by bin): found by a wavefront-wide sort of
// the union of 64 neighbouring blocks (half widths w <= 32), or by rank counting per bin.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/sft.h"

sft_status sft_set_error(sft_status st, const char* msg);

namespace {

constexpr int kStrainBlock = 256;

__device__ inline double2 cmul(double2 a, double2 b)
{
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}

// Median of each lane's block by a wavefront-wide sort: the 64 lanes of a wavefront take 64
// consecutive band bins, whose blocks of 2w+1 periodogram values lie in a union of at most
// 64 + 2w <= 128 bins.  The union's (value, bin) pairs are sorted once per wavefront by a
// bitonic network held in registers (two pairs per lane, the partner of each compare-exchange
// fetched across lanes; the 28 stages unrolled and free of branches) and stored in the
// wavefront's LDS slot; every lane then finds the (w+1)-th entry of the sorted list that falls in
// its block (a binary search over prefix masks of the list's bins): the block's middle element in
// (value, bin) order, as a sort of the block itself gives.
constexpr int kSortN = 128;
constexpr int kMaxSortW = (kSortN - 64) / 2;   // w <= 32
// LDS bytes of the sort slots of a workgroup: per wavefront the kSortN sorted values, then for
// every position of the sorted list the 128-bit mask of the union bins (relative to the union's
// first bin) that it and the entries before it hold
constexpr int kSortBytes = kStrainBlock / 64 * kSortN * (int)(sizeof(double) + sizeof(uint4));

__device__ inline void wave_sync()
{
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline bool pair_less(double va, int ia, double vb, int ib)
{
  return (va < vb) | ((va == vb) & (ia < ib));   // no short circuit: selects, not branches
}

// The 32-bit value of lane (lane ^ S) of the wavefront: quad permutes for S = 1, 2, a half-row
// mirror then a quad reversal for S = 4 ((i ^ 7) ^ 3 = i ^ 4 within each 8 lanes), a rotation
// by 8 within each row of 16 for S = 8 (all on the vector ALU); a swizzle in xor mode within 32
// lanes for S = 16 and a backward permute for S = 32.
template <int S>
__device__ inline int lane_xor(int v, int lane)
{
  if constexpr (S == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
  else if constexpr (S == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
  else if constexpr (S == 4) {
    const int t = __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false);   // row_half_mirror
    return __builtin_amdgcn_mov_dpp(t, 0x1B, 0xF, 0xF, false);           // quad_perm [3,2,1,0]
  } else if constexpr (S == 8) return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false);   // row_ror:8
  else if constexpr (S == 16) return __builtin_amdgcn_ds_swizzle(v, 0x401F);   // and 0x1f, xor 0x10
  else return __builtin_amdgcn_ds_bpermute((lane ^ 32) << 2, v);
}

template <int S>
__device__ inline void xchg_pair(double v, int i, int lane, double& pv, int& pi)
{
  const long long b = __double_as_longlong(v);
  const int lo = lane_xor<S>((int)(b & 0xffffffffll), lane);
  const int hi = lane_xor<S>((int)(b >> 32), lane);
  pv = __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
  pi = lane_xor<S>(i, lane);
}

// One compare-exchange stage of the bitonic network on kSortN = 128 (value, bin) pairs held two
// per lane: element `lane` in (a, ia), element `lane + 64` in (b, ib).  Stride 64 pairs the two
// elements of a lane; smaller strides pair an element with the same one of lane ^ STRIDE, and
// the lower member of the pair keeps the smaller (up) or the larger (down) of the two.
template <int SIZE, int STRIDE>
__device__ inline void bitonic_stage(double& a, int& ia, double& b, int& ib, int lane)
{
  if constexpr (STRIDE == 64) {
    // SIZE = 128: every pair ascending
    const bool sw = pair_less(b, ib, a, ia);
    const double ta = a;
    const int tia = ia;
    a = sw ? b : a;
    ia = sw ? ib : ia;
    b = sw ? ta : b;
    ib = sw ? tia : ib;
  } else {
    const bool lower = (lane & STRIDE) == 0;
    const int qlo = lane & ~STRIDE;
    double pa, pb;
    int pia, pib;
    xchg_pair<STRIDE>(a, ia, lane, pa, pia);
    xchg_pair<STRIDE>(b, ib, lane, pb, pib);
    // keep the smaller of the pair when this lane holds the lower member of an ascending pair
    // or the upper member of a descending one
    const bool mina = lower == ((qlo & SIZE) == 0);
    const bool minb = lower == (((qlo + 64) & SIZE) == 0);
    const bool ta = mina ? pair_less(pa, pia, a, ia) : pair_less(a, ia, pa, pia);
    const bool tb = minb ? pair_less(pb, pib, b, ib) : pair_less(b, ib, pb, pib);
    a = ta ? pa : a;
    ia = ta ? pia : ia;
    b = tb ? pb : b;
    ib = tb ? pib : ib;
  }
}

// Inclusive OR-scan of a 32-bit word over the 64 lanes: shifts by 1, 2, 4, 8 within each row of
// 16 lanes (zero shifted in), then the last lane of rows 0 and 2 into rows 1 and 3, and lane 31
// into rows 2 and 3.
__device__ inline uint32_t wave_or_scan(uint32_t x)
{
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true);    // row_shr:1
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true);    // row_shr:2
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true);    // row_shr:4
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, true);    // row_shr:8
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);   // row_bcast:15
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);   // row_bcast:31
  return x;
}

template <int SIZE, int STRIDE>
__device__ inline void bitonic_from(double& a, int& ia, double& b, int& ib, int lane)
{
  bitonic_stage<SIZE, STRIDE>(a, ia, b, ib, lane);
  if constexpr (STRIDE > 1) bitonic_from<SIZE, STRIDE / 2>(a, ia, b, ib, lane);
  else if constexpr (SIZE < kSortN) bitonic_from<SIZE * 2, SIZE>(a, ia, b, ib, lane);
}

// Transform of the M = 2^LOGM complex points in LDS (natural order in, digit-reversed out), as
// in-place decimation-in-frequency passes of radix 8 (and one of radix 2 or 4 for the leftover
// bits).  Before pass i the data are M / L independent sub-transforms of length L = M / 8^i,
// each contiguous; with L = R L', the work item (g, n1) of sub-transform g reads its R points
// n1 + L' n2, forms their R-point DFT in registers, multiplies output k2 by W_L^{n1 k2} and
// writes it back to the position it read point n2 = k2 from: sub-transform g R + k2, of length
// L', holds the outputs R k1 + k2 of sub-transform g (its k1-th output after the later passes).
// So X[k] ends at position pos(k), the digits of k (radix 8 from the least significant end)
// in reverse order.
template <int LOGM>
struct FftShape {
  static constexpr int M = 1 << LOGM;
  static constexpr int NP = (LOGM + 2) / 3;                              // passes
  static constexpr int lr(int i) { return i < LOGM / 3 ? 3 : LOGM % 3; }  // log2 of pass i's radix
};

// LDS slot of point i: the 16 points of an aligned run (one pass over the 64 banks, 16 bytes
// each) are permuted by an XOR of higher index bits, so that the strided accesses of the later
// passes and the digit-reversed reads of the unfolding spread over the banks (a model of the
// 16-lane groups of a 16-byte LDS read puts their mean conflict degree at ~1.3 instead of ~4.3
// for M = 2048).  A bijection on each run, the identity for M <= 16.
__device__ inline int swz(int i) { return i ^ (((i >> 4) ^ (i >> 7) ^ (i >> 8)) & 15); }

template <int LOGM>
__device__ inline int fft_pos(int k)
{
  int p = 0;
#pragma unroll
  for (int i = 0; i < FftShape<LOGM>::NP; ++i) {
    const int l = FftShape<LOGM>::lr(i);
    p |= ((k >> (3 * i)) & ((1 << l) - 1)) << (LOGM - 3 * i - l);
  }
  return p;
}

// in-place R-point DFT, v[k] <- sum_n v[n] e^{-2 pi i n k / R}, R = 2, 4 or 8
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 mul_mi(double2 a) { return make_double2(a.y, -a.x); }   // times -i

__device__ inline void dft4(double2& u0, double2& u1, double2& u2, double2& u3)
{
  const double2 c0 = cadd(u0, u2), c1 = csub(u0, u2), c2 = cadd(u1, u3), c3 = mul_mi(csub(u1, u3));
  u0 = cadd(c0, c2);
  u1 = cadd(c1, c3);
  u2 = csub(c0, c2);
  u3 = csub(c1, c3);
}

template <int R>
__device__ inline void dft_small(double2* v)
{
  if constexpr (R == 2) {
    const double2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    dft4(v[0], v[1], v[2], v[3]);
  } else {
    // radix-2 split: even outputs from a_n = v_n + v_{n+4}, odd ones from
    // b_n = (v_n - v_{n+4}) e^{-2 pi i n / 8}, each by a 4-point DFT
    constexpr double c = 0.70710678118654752440;
    double2 a[4], b[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      a[n] = cadd(v[n], v[n + 4]);
      b[n] = csub(v[n], v[n + 4]);
    }
    b[1] = make_double2(c * (b[1].x + b[1].y), c * (b[1].y - b[1].x));
    b[2] = mul_mi(b[2]);
    b[3] = make_double2(c * (b[3].y - b[3].x), -c * (b[3].x + b[3].y));
    dft4(a[0], a[1], a[2], a[3]);
    dft4(b[0], b[1], b[2], b[3]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[2 * k] = a[k];
      v[2 * k + 1] = b[k];
    }
  }
}

template <int LOGM, int I>
__device__ inline void fft_pass(double2* buf, const double2* __restrict__ tw, int tid)
{
  constexpr int M = 1 << LOGM;
  constexpr int LR = FftShape<LOGM>::lr(I), R = 1 << LR;
  constexpr int LOGL = LOGM - 3 * I, L = 1 << LOGL, LP = L >> LR;
#pragma unroll
  for (int t0 = 0; t0 < M / R; t0 += kStrainBlock) {
    const int t = t0 + tid;
    if (M / R % kStrainBlock == 0 || t < M / R) {
      const int g = t >> (LOGL - LR), n1 = t & (LP - 1);
      const int base = g * L + n1;
      // W_L^{n1 k2} = W_M^{(M / L) n1 k2}; tw holds W_M^j for j < M / 2, W_M^{j + M/2} = -W_M^j.
      // The twiddle loads are issued first, so that their latency overlaps the LDS reads and
      // the R-point DFT.
      double2 wv[R];
      if constexpr (LP > 1) {
#pragma unroll
        for (int k2 = 1; k2 < R; ++k2) wv[k2] = tw[((n1 * k2) << (LOGM - LOGL)) & (M / 2 - 1)];
      }
      double2 v[R];
#pragma unroll
      for (int n2 = 0; n2 < R; ++n2) v[n2] = buf[swz(base + LP * n2)];
      dft_small<R>(v);
      if constexpr (LP > 1) {
#pragma unroll
        for (int k2 = 1; k2 < R; ++k2) {
          const double sg = (((n1 * k2) << (LOGM - LOGL)) & (M / 2)) ? -1.0 : 1.0;
          v[k2] = cmul(v[k2], make_double2(sg * wv[k2].x, sg * wv[k2].y));
        }
      }
#pragma unroll
      for (int k2 = 0; k2 < R; ++k2) buf[swz(base + LP * k2)] = v[k2];
    }
  }
  __syncthreads();
  if constexpr (I + 1 < FftShape<LOGM>::NP) fft_pass<LOGM, I + 1>(buf, tw, tid);
}

// One workgroup per segment of n = 2M samples.  LDS: the M complex points (buf), then, once the
// spectrum is in registers, the M + 1 periodogram values over it, the median's sort slots at
// byte sort_off and one gap flag per wavefront at byte flag_off.  A segment with a non-finite
// sample is transformed like any other (the values are discarded) and its gap is found after
// the transform, so that no LDS word has to stay reserved through it.
template <int LOGM>
__global__ __launch_bounds__(kStrainBlock) void strain_sft_kernel(
    const double* __restrict__ x, int64_t n_total, int32_t n_seg, double dt, int32_t w, double psd_scale,
    int32_t k_lo, int32_t n_bins, double s_white, const double2* __restrict__ tw, const double2* __restrict__ rtw,
    double* __restrict__ bins, double* __restrict__ psd, int32_t* __restrict__ keep, int32_t sort_off,
    int32_t flag_off)
{
  constexpr int M = 1 << LOGM;
  extern __shared__ double2 buf[];
  double* U = reinterpret_cast<double*>(buf);   // the periodogram, after the transform
  const int row = blockIdx.x;
  const int det = row / n_seg, seg = row - det * n_seg;
  const double* xs = x + (int64_t)det * n_total + (int64_t)seg * 2 * M;
  const int tid = threadIdx.x;
  bool bad = false;
  // z[m] = x[2m] + i x[2m+1] (one 16-byte load per point where the segment is 16-byte
  // aligned), in batches of up to 8 points per thread whose loads are all issued before the
  // first is used
  {
    constexpr int NL = (M + kStrainBlock - 1) / kStrainBlock, NB = NL < 8 ? NL : 8;
    const bool al = (reinterpret_cast<uintptr_t>(xs) & 15) == 0;
    const double2* xs2 = reinterpret_cast<const double2*>(xs);
#pragma unroll
    for (int r0 = 0; r0 < NL; r0 += NB) {
      double2 z[NB];
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        const int m = tid + (r0 + r) * kStrainBlock;
        if (M % kStrainBlock == 0 || m < M) z[r] = al ? xs2[m] : make_double2(xs[2 * m], xs[2 * m + 1]);
      }
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        const int m = tid + (r0 + r) * kStrainBlock;
        if (M % kStrainBlock == 0 || m < M) {
          bad |= !(isfinite(z[r].x) && isfinite(z[r].y));
          buf[swz(m)] = z[r];
        }
      }
    }
  }
  __syncthreads();
  double* bo = bins + (int64_t)row * 2 * n_bins;
  double* po = psd + (int64_t)row * n_bins;
  fft_pass<LOGM, 0>(buf, tw, tid);
  // real-transform bins, pair (k, M - k) per work item; rtw[k] = e^{-2 pi i k / n}, k <= M/2.
  // The band bins go out as dt X[k]; the periodogram |X[k]|^2 stays in registers until every
  // item has read the spectrum, then overlays it in LDS.
  constexpr int NPAIR = (M / 2 + kStrainBlock) / kStrainBlock;   // ceil((M/2 + 1) / block)
  double pk[NPAIR], pm[NPAIR];
  double2 rtk[NPAIR];
#pragma unroll
  for (int r = 0; r < NPAIR; ++r) {
    const int k = tid + r * kStrainBlock;
    rtk[r] = rtw[k <= M / 2 ? k : M / 2];   // all issued before the first is used
  }
#pragma unroll
  for (int r = 0; r < NPAIR; ++r) {
    const int k = tid + r * kStrainBlock;
    pk[r] = pm[r] = 0.0;
    if (k <= M / 2) {
      const int kk = (M - k) & (M - 1);  // M - k, with Z[M] = Z[0]
      const double2 a = buf[swz(fft_pos<LOGM>(k))], b = buf[swz(fft_pos<LOGM>(kk))];
      const double2 e = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));   // (Z[k] + conj Z[M-k]) / 2
      const double2 o = make_double2(0.5 * (a.x - b.x), 0.5 * (a.y + b.y));   // (Z[k] - conj Z[M-k]) / 2
      const double2 rt = rtk[r];
      const double2 ro = cmul(rt, o);
      const double2 Xk = make_double2(e.x + ro.y, e.y - ro.x);                // e - i ro
      // X[M - k] from the same pair with the roles exchanged: e' = conj(e), o' = -conj(o),
      // e^{-2 pi i (M-k)/n} = -conj(e^{-2 pi i k / n})
      const double2 ro2 = cmul(make_double2(-rt.x, rt.y), make_double2(-o.x, o.y));
      const double2 Xm = make_double2(e.x + ro2.y, -e.y - ro2.x);
      const int im = M - k - k_lo;   // band index of X[M - k] (the Nyquist bin for k = 0)
      if (k - k_lo >= 0 && k - k_lo < n_bins) {
        bo[2 * (k - k_lo)] = dt * Xk.x;
        bo[2 * (k - k_lo) + 1] = dt * Xk.y;
      }
      if (2 * k != M && im >= 0 && im < n_bins) {
        bo[2 * im] = dt * Xm.x;
        bo[2 * im + 1] = dt * Xm.y;
      }
      pk[r] = fma(Xk.x, Xk.x, Xk.y * Xk.y);
      pm[r] = fma(Xm.x, Xm.x, Xm.y * Xm.y);
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < NPAIR; ++r) {
    const int k = tid + r * kStrainBlock;
    if (k <= M / 2) {
      U[k] = pk[r];
      if (2 * k != M) U[M - k] = pm[r];
    }
  }
  int* gap = reinterpret_cast<int*>(reinterpret_cast<char*>(buf) + flag_off);
  const bool wave_bad = __ballot(bad) != 0;
  if ((tid & 63) == 0) gap[tid >> 6] = wave_bad ? 1 : 0;
  __syncthreads();
  bool seg_bad = false;
#pragma unroll
  for (int v = 0; v < kStrainBlock / 64; ++v) seg_bad = seg_bad || gap[v] != 0;
  if (seg_bad) {
    // a gap: zeros over the band bins this thread wrote above (same addresses, same thread, so
    // the zeros land last), a zero PSD and keep = 0
#pragma unroll
    for (int r = 0; r < NPAIR; ++r) {
      const int k = tid + r * kStrainBlock;
      if (k <= M / 2) {
        const int im = M - k - k_lo;
        if (k - k_lo >= 0 && k - k_lo < n_bins) {
          bo[2 * (k - k_lo)] = 0.0;
          bo[2 * (k - k_lo) + 1] = 0.0;
        }
        if (2 * k != M && im >= 0 && im < n_bins) {
          bo[2 * im] = 0.0;
          bo[2 * im + 1] = 0.0;
        }
      }
    }
    for (int i = tid; i < n_bins; i += kStrainBlock) po[i] = 0.0;
    if (tid == 0) keep[row] = 0;
    return;
  }
  auto P = [&](int j) { return U[j]; };
  const int N = 2 * w + 1;
  if (s_white > 0.0) {
    // a known white PSD: no estimate
    for (int i = tid; i < n_bins; i += blockDim.x) po[i] = s_white;
  } else if (w <= kMaxSortW) {
    const int lane = tid & 63, wv = tid >> 6;
    double* sv = reinterpret_cast<double*>(reinterpret_cast<char*>(buf) + sort_off) + wv * kSortN;
    uint4* pm = reinterpret_cast<uint4*>(reinterpret_cast<char*>(buf) + sort_off + (kStrainBlock / 64) * kSortN * 8) +
                wv * kSortN;
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
      // the kSortN pairs sorted in registers (two per lane), then stored in sorted order
      double a = lane < L ? P(u0 + lane) : INFINITY, b = lane + 64 < L ? P(u0 + lane + 64) : INFINITY;
      int ia = lane < L ? lane : 0x7fffffff, ib = lane + 64 < L ? lane + 64 : 0x7fffffff;
      bitonic_from<2, 1>(a, ia, b, ib, lane);
      // prefix masks of the sorted list: bit j of pm[q] is set when union bin j is one of the
      // entries 0..q (an OR-scan of one-hot masks over the lanes, the second half of the list
      // on top of the first; the pads set no bit)
      uint32_t sa[4], sb[4];
#pragma unroll
      for (int wd = 0; wd < 4; ++wd) {
        sa[wd] = wave_or_scan((ia >> 5) == wd ? 1u << (ia & 31) : 0u);
        const uint32_t t = (uint32_t)__builtin_amdgcn_readlane((int)sa[wd], 63);
        sb[wd] = wave_or_scan((ib >> 5) == wd ? 1u << (ib & 31) : 0u) | t;
      }
      sv[lane] = a;
      sv[lane + 64] = b;
      pm[lane] = make_uint4(sa[0], sa[1], sa[2], sa[3]);
      pm[lane + 64] = make_uint4(sb[0], sb[1], sb[2], sb[3]);
      wave_sync();
      // The count of a lane's block entries among the sorted entries 0..q is the popcount of
      // pm[q] under the block's mask and grows with q; the block's median is the entry at which
      // it reaches w + 1: the smallest such q, by a binary search (7 steps over kSortN).
      const int i = c0 + lane;
      const int k = k_lo + i;
      int s0 = k - w;
      s0 = s0 < 0 ? 0 : s0;
      s0 = s0 + 2 * w > M ? M - 2 * w : s0;
      const int s0r = s0 - u0;   // the block's first bin in the union
      uint32_t wm[4];
#pragma unroll
      for (int wd = 0; wd < 4; ++wd) {
        const int lo = min(max(s0r - 32 * wd, 0), 32), hi = min(max(s0r + N - 32 * wd, 0), 32);
        wm[wd] = (uint32_t)(((1ull << hi) - 1ull) & ~((1ull << lo) - 1ull));
      }
      int qlo = 0, qhi = kSortN - 1;
#pragma unroll
      for (int it = 0; it < 7; ++it) {
        const int mid = (qlo + qhi) >> 1;
        const uint4 p = pm[mid];
        const int c = __builtin_popcount(p.x & wm[0]) + __builtin_popcount(p.y & wm[1]) +
                      __builtin_popcount(p.z & wm[2]) + __builtin_popcount(p.w & wm[3]);
        if (c >= w + 1) qhi = mid;
        else qlo = mid + 1;
      }
      const int mq = qlo;
      const double med = sv[mq];
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

// Twiddle tables of a segment length n, in long double rounded once to FP64: for n a power of
// two, tw[j] = e^{-2 pi i j / M} (j < M/2, M = n/2) and rtw[k] = e^{-2 pi i k / n} (k <= M/2);
// otherwise W[m] = e^{-2 pi i m / n} (m < n).  Built on a device's first call for n and kept
// there until the process ends (tens of KB per length), so that later calls only launch.
struct TwTables {
  double2* tw = nullptr;
  double2* rtw = nullptr;
  double2* W = nullptr;
};

static hipError_t upload(const std::vector<double2>& h, double2** d)
{
  hipError_t e = hipMalloc((void**)d, h.size() * sizeof(double2));
  if (e == hipSuccess) e = hipMemcpy(*d, h.data(), h.size() * sizeof(double2), hipMemcpyHostToDevice);
  if (e != hipSuccess && *d) {
    (void)hipFree(*d);
    *d = nullptr;
  }
  return e;
}

static hipError_t twiddle_tables(int n, TwTables& out)
{
  static std::mutex mu;
  static std::map<std::pair<int, int>, TwTables> cache;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  const auto it = cache.find({dev, n});
  if (it != cache.end()) {
    out = it->second;
    return hipSuccess;
  }
  const long double pi = 3.141592653589793238462643383279502884L;
  TwTables t;
  if ((n & (n - 1)) != 0) {
    std::vector<double2> W(n);
    for (int m = 0; m < n; ++m) {
      const long double a = -2.0L * pi * (long double)m / (long double)n;
      W[m] = make_double2((double)cosl(a), (double)sinl(a));
    }
    e = upload(W, &t.W);
  } else {
    const int M = n / 2;
    std::vector<double2> tw(M / 2 > 0 ? M / 2 : 1), rtw(M / 2 + 1);
    for (int j = 0; j < M / 2; ++j) {
      const long double a = -2.0L * pi * (long double)j / (long double)M;
      tw[j] = make_double2((double)cosl(a), (double)sinl(a));
    }
    for (int k = 0; k <= M / 2; ++k) {
      const long double a = -2.0L * pi * (long double)k / (long double)n;
      rtw[k] = make_double2((double)cosl(a), (double)sinl(a));
    }
    e = upload(tw, &t.tw);
    if (e == hipSuccess) e = upload(rtw, &t.rtw);
    if (e != hipSuccess && t.tw) (void)hipFree(t.tw);
  }
  if (e != hipSuccess) return e;
  cache[{dev, n}] = t;
  out = t;
  return hipSuccess;
}

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
  TwTables tt;
  hipError_t e = twiddle_tables(n, tt);
  if (e != hipSuccess) return strain_fail(SFT_E_DEVICE, hipGetErrorString(e));
  if (!pow2) {
    const size_t lds = (size_t)n * sizeof(double);
    if (lds > 65536)
      e = hipFuncSetAttribute((const void*)strain_dft_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess && n_seg > 0) {
      hipLaunchKernelGGL(strain_dft_kernel, dim3((unsigned)(n_seg * d->n_det)), dim3(kStrainBlock), lds, st, x,
                         d->n_total, (int32_t)n_seg, n, d->dt, d->s_white, d->k_lo, d->n_bins, tt.W, bins, psd, keep);
      e = hipGetLastError();
    }
    if (e != hipSuccess) return strain_fail(SFT_E_DEVICE, hipGetErrorString(e));
    return SFT_OK;
  }
  int logM = 0;
  while ((1 << logM) < M) ++logM;
  double2* d_tw = tt.tw;
  double2* d_rtw = tt.rtw;
  double B = 0.0;
  for (int i = 0; i <= d->psd_w; ++i) B += 1.0 / (double)(2 * d->psd_w + 1 - i);
  const double T = d->dt * n;
  const double psd_scale = 2.0 / (T * B);
  // LDS: the M complex points; the periodogram (M + 1 values), the median's sort slots and the
  // gap flags (each 16-byte aligned after the previous) overlay them once the transform is done
  size_t lds = (size_t)M * sizeof(double2);
  int32_t sort_off = 0;
  int32_t flag_off = (int32_t)(((size_t)(M + 1) * sizeof(double) + 15) / 16 * 16);
  if (!(d->s_white > 0.0) && d->psd_w <= kMaxSortW) {
    sort_off = flag_off;
    flag_off = sort_off + kSortBytes;
  }
  if ((size_t)flag_off + 16 > lds) lds = (size_t)flag_off + 16;
  const void* kern = nullptr;
  switch (logM) {
    case 3: kern = (const void*)strain_sft_kernel<3>; break;
    case 4: kern = (const void*)strain_sft_kernel<4>; break;
    case 5: kern = (const void*)strain_sft_kernel<5>; break;
    case 6: kern = (const void*)strain_sft_kernel<6>; break;
    case 7: kern = (const void*)strain_sft_kernel<7>; break;
    case 8: kern = (const void*)strain_sft_kernel<8>; break;
    case 9: kern = (const void*)strain_sft_kernel<9>; break;
    case 10: kern = (const void*)strain_sft_kernel<10>; break;
    case 11: kern = (const void*)strain_sft_kernel<11>; break;
    case 12: kern = (const void*)strain_sft_kernel<12>; break;
    case 13: kern = (const void*)strain_sft_kernel<13>; break;
    default: break;
  }
  if (e == hipSuccess && !kern) e = hipErrorInvalidValue;   // n in [16, 16384] was checked above
  if (e == hipSuccess && lds > 65536) e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess && n_seg > 0) {
    int32_t a_nseg = (int32_t)n_seg, a_w = d->psd_w, a_klo = d->k_lo, a_nbins = d->n_bins;
    int64_t a_ntot = d->n_total;
    double a_dt = d->dt, a_scale = psd_scale, a_white = d->s_white;
    void* args[] = {(void*)&x, &a_ntot, &a_nseg, &a_dt, &a_w, &a_scale, &a_klo, &a_nbins, &a_white,
                    &d_tw, &d_rtw, &bins, &psd, &keep, &sort_off, &flag_off};
    e = hipLaunchKernel(kern, dim3((unsigned)(n_seg * d->n_det)), dim3(kStrainBlock), args, lds, st);
  }
  if (e != hipSuccess) return strain_fail(SFT_E_DEVICE, hipGetErrorString(e));
  return SFT_OK;
}
