// sft_sort.hip -- order of a template bank by its track, on the device.
//
// The scan gives one template to each lane and stages, per wavefront, the union of the lanes'
// bin windows in LDS; that is cheap only when the lanes' tracks f(t) nearly coincide.  A bank
// handed over in any order is sorted here by the key
//   (first SFT row of the template) << 32 | FP32 bits of f(t*) T,
// f the leading-order frequency (the chirp of Sec. II.A) at the midpoint t* of the template's
// SFT range: templates of one range together, neighbours in frequency next to each other.
// Positive FP32 values order like their bit patterns; a template already past coalescence at
// t* gets the largest key.  The keys are sorted with their indices by rocPRIM's stable radix
// sort, and the bank arrays are gathered into that order.  Only the speed of a scan depends on
// the order: the finalize kernel writes every template's results back to its given position.
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>

#include <cstdint>

#include "sft_sort.h"

namespace {

constexpr double kPiSort = 3.14159265358979323846;

__global__ __launch_bounds__(256) void track_key_kernel(SortKeyArgs a, uint64_t* __restrict__ key,
                                                        int32_t* __restrict__ idx)
{
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= a.n) return;
  const int last = a.n_sft - 1;
  int lo = a.a_first ? a.a_first[m] : 0;
  int hi = a.a_last ? a.a_last[m] : last;
  lo = lo < 0 ? 0 : (lo > last ? last : lo);
  hi = hi < lo ? lo : (hi > last ? last : hi);
  const double t = 0.5 * (a.row_tmid[lo] + a.row_tmid[hi]);
  const double tau = a.t_c[m] - t;
  const double M = a.mc[m] * a.tsun;
  float kap = 3.0e38f;
  if (tau > 0.0 && M > 0.0) {
    const double f = pow(5.0 * M / tau, 0.375) / (8.0 * kPiSort * M);
    const float v = (float)(f * a.T);
    if (v >= 0.0f && v < 3.0e38f) kap = v;
  }
  key[m] = ((uint64_t)(uint32_t)lo << 32) | (uint64_t)__float_as_uint(kap);
  idx[m] = (int32_t)m;
}

template <typename T>
__global__ __launch_bounds__(256) void gather_kernel(const T* __restrict__ src, const int32_t* __restrict__ perm,
                                                     int64_t n, int32_t width, T* __restrict__ dst)
{
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * width) return;
  const int64_t r = i / width;
  dst[i] = src[(int64_t)perm[r] * width + (i - r * width)];
}

}  // namespace

hipError_t sort_temp_bytes(int64_t n, size_t* bytes)
{
  *bytes = 0;
  return rocprim::radix_sort_pairs(nullptr, *bytes, (uint64_t*)nullptr, (uint64_t*)nullptr, (int32_t*)nullptr,
                                   (int32_t*)nullptr, (size_t)n, 0, 64);
}

hipError_t sort_by_track(const SortKeyArgs& a, void* temp, size_t temp_bytes, uint64_t* key_a, uint64_t* key_b,
                         int32_t* idx_a, int32_t* perm, hipStream_t st)
{
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(track_key_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st, a, key_a, idx_a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  size_t tb = temp_bytes;
  return rocprim::radix_sort_pairs(temp, tb, key_a, key_b, idx_a, perm, (size_t)a.n, 0, 64, st);
}

hipError_t gather_f64(const double* src, const int32_t* perm, int64_t n, int32_t width, double* dst, hipStream_t st)
{
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_kernel<double>, dim3((unsigned)((n * width + 255) / 256)), dim3(256), 0, st, src, perm, n,
                     width, dst);
  return hipGetLastError();
}

hipError_t gather_i32(const int32_t* src, const int32_t* perm, int64_t n, int32_t* dst, hipStream_t st)
{
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_kernel<int32_t>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, perm, n, 1,
                     dst);
  return hipGetLastError();
}
