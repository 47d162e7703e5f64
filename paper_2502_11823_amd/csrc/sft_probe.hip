// sft_probe.hip -- issue-rate probe of the vector ALU.  The scan kernel's roofline counts FP32
// lane-operation slots against the nominal FP32 vector peak, which assumes the packed FP32
// instructions (two FP32 operations per lane and instruction); this library leaves those off, so
// the rate that plain wave64 instructions actually sustain on the part is the practical ceiling.
// Each lane runs 16 independent chains of one instruction for a fixed number of iterations,
// over a grid that fills every CU several times; the rate is in wave-instructions per second.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/sft.h"

sft_status sft_set_error(sft_status st, const char* msg);

namespace {

constexpr int kProbeBlocks = 2048;   // 8 workgroups of 256 per CU
constexpr int kProbeThreads = 256;
constexpr int kProbeIters = 4096;
constexpr int kChains = 16;

template <int OP>
__global__ __launch_bounds__(kProbeThreads) void probe_kernel(float* __restrict__ out, int iters, float seed)
{
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  if constexpr (OP == SFT_PROBE_FMA_F64) {
    double x[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) x[i] = (double)seed + 0.001 * (threadIdx.x + i);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int i = 0; i < kChains; ++i) x[i] = fma(x[i], 0.999, 0.0001);
    }
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += x[i];
    out[tid] = (float)s;
  } else if constexpr (OP == SFT_PROBE_FMA_F32_INT32) {
    // half the chains FP32 FMAs, half 32-bit xorshift steps (a shift and an xor each): one
    // FP32 instruction per two integer instructions, as a mixed instruction stream
    float x[kChains / 2];
    uint32_t y[kChains / 2];
#pragma unroll
    for (int i = 0; i < kChains / 2; ++i) {
      x[i] = seed + 0.001f * (threadIdx.x + i);
      y[i] = 0x9e3779b9u * (uint32_t)(tid + i + 1);
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int i = 0; i < kChains / 2; ++i) {
        x[i] = fmaf(x[i], 0.999f, 0.0001f);
        y[i] ^= y[i] << 5;
      }
    }
    float s = 0.f;
    uint32_t h = 0;
#pragma unroll
    for (int i = 0; i < kChains / 2; ++i) {
      s += x[i];
      h ^= y[i];
    }
    out[tid] = s + (float)h;   // every bit of every chain reaches the output
  } else {
    float x[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) x[i] = seed + 0.001f * (threadIdx.x + i);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int i = 0; i < kChains; ++i) {
        if constexpr (OP == SFT_PROBE_FMA_F32) x[i] = fmaf(x[i], 0.999f, 0.0001f);
        else x[i] = __builtin_amdgcn_rcpf(x[i]);
      }
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += x[i];
    out[tid] = s;
  }
}

hipError_t launch_probe(int op, float* out, hipStream_t st)
{
  const dim3 g(kProbeBlocks), b(kProbeThreads);
  switch (op) {
    case SFT_PROBE_FMA_F32: hipLaunchKernelGGL(probe_kernel<SFT_PROBE_FMA_F32>, g, b, 0, st, out, kProbeIters, 1.0f); break;
    case SFT_PROBE_RCP_F32: hipLaunchKernelGGL(probe_kernel<SFT_PROBE_RCP_F32>, g, b, 0, st, out, kProbeIters, 1.0f); break;
    case SFT_PROBE_FMA_F64: hipLaunchKernelGGL(probe_kernel<SFT_PROBE_FMA_F64>, g, b, 0, st, out, kProbeIters, 1.0f); break;
    default: hipLaunchKernelGGL(probe_kernel<SFT_PROBE_FMA_F32_INT32>, g, b, 0, st, out, kProbeIters, 1.0f); break;
  }
  return hipGetLastError();
}

}  // namespace

extern "C" sft_status sft_probe_issue_rate(int32_t op, double* instr_per_s, void* hip_stream)
{
  if (!instr_per_s) return sft_set_error(SFT_E_INVALID, "sft_probe_issue_rate: null argument");
  if (op < SFT_PROBE_FMA_F32 || op > SFT_PROBE_FMA_F32_INT32)
    return sft_set_error(SFT_E_INVALID, "sft_probe_issue_rate: unknown probe");
  hipStream_t st = (hipStream_t)hip_stream;
  float* out = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipMalloc((void**)&out, (size_t)kProbeBlocks * kProbeThreads * sizeof(float));
  if (e == hipSuccess) e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  for (int w = 0; w < 3 && e == hipSuccess; ++w) e = launch_probe(op, out, st);   // warm-up (clocks, code object)
  float best = 0.f;
  for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
    e = hipEventRecord(a, st);
    if (e == hipSuccess) e = launch_probe(op, out, st);
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (e == hipSuccess && (rep == 0 || ms < best)) best = ms;
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (out) (void)hipFree(out);
  if (e != hipSuccess) return sft_set_error(SFT_E_DEVICE, hipGetErrorString(e));
  const int per_iter = op == SFT_PROBE_FMA_F32_INT32 ? kChains / 2 * 3 : kChains;   // VALU per lane and iteration
  const double instr = (double)kProbeBlocks * (kProbeThreads / 64) * kProbeIters * per_iter;
  *instr_per_s = best > 0.f ? instr / (best * 1e-3) : 0.0;
  return SFT_OK;
}
