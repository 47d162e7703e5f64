// sft_sort.h -- order of a template bank by its track on the device (sft_sort.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

struct SortKeyArgs {
  const double* mc;
  const double* t_c;
  const int32_t* a_first;  // may be null (row 0)
  const int32_t* a_last;   // may be null (the last row)
  const double* row_tmid;  // [n_sft] midpoint time of each SFT row
  int32_t n_sft;
  double T, tsun;
  int64_t n;
};

// Bytes of temporary storage the radix sort of n keys needs.
hipError_t sort_temp_bytes(int64_t n, size_t* bytes);
// perm[i] = index of the template that goes to position i; key_a, key_b, idx_a ([n] each) and
// temp (sort_temp_bytes) are scratch.  Stable: templates of equal keys keep their given order.
hipError_t sort_by_track(const SortKeyArgs& a, void* temp, size_t temp_bytes, uint64_t* key_a, uint64_t* key_b,
                         int32_t* idx_a, int32_t* perm, hipStream_t st);
// dst[i * width + c] = src[perm[i] * width + c] for i < n, c < width
hipError_t gather_f64(const double* src, const int32_t* perm, int64_t n, int32_t width, double* dst, hipStream_t st);
hipError_t gather_i32(const int32_t* src, const int32_t* perm, int64_t n, int32_t* dst, hipStream_t st);
