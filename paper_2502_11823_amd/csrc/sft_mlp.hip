// sft_mlp.hip -- the learned surrogate's network on gfx950: training (FP32 forward,
// backward, Adam, epoch shuffling) and inference (forward pass with the forward-mode
// derivative along the ln(tau) input: fused FP64 or BF16 matrix-core kernels, or a
// layer-by-layer path), built from tiled GEMM kernels and small element-wise kernels.
//
// GEMM: C[M][N] = op(A)[M][K] op(B)[K][N] for a 64 x 64 tile per 256-thread workgroup,
// K staged through LDS in steps of 16; FP32 (training) on the matrix cores, FP64 (the
// layer-by-layer inference of odd widths) with 4 x 4 vector FMAs per thread.  A grid
// z-dimension splits K into slices written to separate C planes (summed by a reduction
// kernel), which gives the weight gradients (K = batch) enough workgroups.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "sft_mlp.h"

// ---------------------------------------------------------------------------- geometry
MlpLayer mlp_layer(int hidden, int layers, int l)
{
  MlpLayer L;
  int64_t off = 0;
  for (int i = 0; i <= l; ++i) {
    const int n_in = i == 0 ? 3 : hidden;
    const int n_out = i == layers ? 2 : hidden;
    if (i == l) {
      L.n_in = n_in;
      L.n_out = n_out;
      L.w_off = off;
      L.b_off = off + (int64_t)n_in * n_out;
    }
    off += (int64_t)n_in * n_out + n_out;
  }
  return L;
}

int64_t mlp_param_count(int hidden, int layers)
{
  const MlpLayer L = mlp_layer(hidden, layers, layers);
  return L.b_off + L.n_out;
}

// ---------------------------------------------------------------------------- GEMM
template <typename T, bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_kernel(int M, int N, int K, const T* __restrict__ A, int lda,
                                                   const T* __restrict__ B, int ldb, T* __restrict__ C, int ldc,
                                                   int k_slice, int64_t c_plane)
{
  __shared__ T As[16][64 + 1];
  __shared__ T Bs[16][64 + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int kb = blockIdx.z * k_slice;
  const int ke = min(K, kb + k_slice);
  T acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = (T)0;
  for (int k0 = kb; k0 < ke; k0 += 16) {
    for (int e = threadIdx.x; e < 1024; e += 256) {
      int ii, kk;
      if (TA) { ii = e & 63; kk = e >> 6; } else { ii = e >> 4; kk = e & 15; }
      const int gi = i0 + ii, gk = k0 + kk;
      T v = (T)0;
      if (gi < M && gk < ke) v = TA ? A[(int64_t)gk * lda + gi] : A[(int64_t)gi * lda + gk];
      As[kk][ii] = v;
    }
    for (int e = threadIdx.x; e < 1024; e += 256) {
      int jj, kk;
      if (TB) { jj = e >> 4; kk = e & 15; } else { jj = e & 63; kk = e >> 6; }
      const int gj = j0 + jj, gk = k0 + kk;
      T v = (T)0;
      if (gj < N && gk < ke) v = TB ? B[(int64_t)gj * ldb + gk] : B[(int64_t)gk * ldb + gj];
      Bs[kk][jj] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      T a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = As[kk][ty + 16 * r];
#pragma unroll
      for (int c = 0; c < 4; ++c) b[c] = Bs[kk][tx + 16 * c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = fma(a[r], b[c], acc[r][c]);
    }
    __syncthreads();
  }
  // thread (tx, ty) owns rows ty + 16 r and columns tx + 16 c of the tile, so that a
  // wavefront's LDS reads and global stores touch consecutive addresses
  T* Cp = C + (int64_t)blockIdx.z * c_plane;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int gi = i0 + ty + 16 * r;
    if (gi >= M) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int gj = j0 + tx + 16 * c;
      if (gj < N) Cp[(int64_t)gi * ldc + gj] = acc[r][c];
    }
  }
}

// FP32 GEMM on the matrix cores (v_mfma_f32_16x16x4f32): the same tile, staging and K slices
// as gemm_kernel, each wavefront computing a 32 x 32 quarter of the 64 x 64 tile as 2 x 2
// blocks of 16 x 16.  Operand layouts (checked with an in-bounds probe): A[i][k] in lane
// i + 16 k, B[k][j] in lane j + 16 k, D[i][j] in lane j + 16 (i / 4), element i % 4.
// Epilogues of the training passes (EPI):
//   kEpiPlain   C = op(A) op(B);
//   kEpiBiasAct forward layer: z = C + bias[j] stored in C (the pre-activation), SiLU(z) in out2;
//   kEpiActBack input gradient of the layer below: C = (op(A) op(B)) * SiLU'(Zb) with Zb = in2
//               (that layer's pre-activations, ld = ldc);
//   kEpiColSum  weight gradient with the bias gradient: the workgroups of the first row tile
//               also sum the columns of B over their K slice into row M of their C plane
//               (the plane holds (M + 1) rows: W then b, as the parameters are packed).
typedef float flt4m __attribute__((ext_vector_type(4)));
enum { kEpiPlain = 0, kEpiBiasAct = 1, kEpiActBack = 2, kEpiColSum = 3 };

__device__ inline float sigm_f(float z) { return 1.0f / (1.0f + expf(-z)); }

template <bool TA, bool TB, int EPI = kEpiPlain>
__global__ __launch_bounds__(256) void gemm_mfma_kernel(int M, int N, int K, const float* __restrict__ A, int lda,
                                                        const float* __restrict__ B, int ldb, float* __restrict__ C,
                                                        int ldc, int k_slice, int64_t c_plane,
                                                        const float* __restrict__ in2 = nullptr,
                                                        float* __restrict__ out2 = nullptr)
{
  __shared__ float As[16][64 + 4];
  __shared__ float Bs[16][64 + 4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wi = 32 * (wave >> 1), wj = 32 * (wave & 1);   // the wavefront's quarter of the tile
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int kb = blockIdx.z * k_slice;
  const int ke = min(K, kb + k_slice);
  flt4m acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = flt4m{0.0f, 0.0f, 0.0f, 0.0f};
  const bool csum = EPI == kEpiColSum && blockIdx.y == 0;
  float colsum = 0.0f;   // thread t < 64: column j0 + t of B over this K slice
  for (int k0 = kb; k0 < ke; k0 += 16) {
    for (int e = threadIdx.x; e < 1024; e += 256) {
      int ii, kk;
      if (TA) { ii = e & 63; kk = e >> 6; } else { ii = e >> 4; kk = e & 15; }
      const int gi = i0 + ii, gk = k0 + kk;
      float v = 0.0f;
      if (gi < M && gk < ke) v = TA ? A[(int64_t)gk * lda + gi] : A[(int64_t)gi * lda + gk];
      As[kk][ii] = v;
    }
    for (int e = threadIdx.x; e < 1024; e += 256) {
      int jj, kk;
      if (TB) { jj = e >> 4; kk = e & 15; } else { jj = e & 63; kk = e >> 6; }
      const int gj = j0 + jj, gk = k0 + kk;
      float v = 0.0f;
      if (gj < N && gk < ke) v = TB ? B[(int64_t)gj * ldb + gk] : B[(int64_t)gk * ldb + gj];
      Bs[kk][jj] = v;
    }
    __syncthreads();
    if (csum && threadIdx.x < 64) {
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) colsum += Bs[kk][threadIdx.x];
    }
#pragma unroll
    for (int k4 = 0; k4 < 16; k4 += 4) {
      const float a0 = As[k4 + lk][wi + li], a1 = As[k4 + lk][wi + 16 + li];
      const float b0 = Bs[k4 + lk][wj + li], b1 = Bs[k4 + lk][wj + 16 + li];
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  float* Cp = C + (int64_t)blockIdx.z * c_plane;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int gj = j0 + wj + 16 * b + li;
      if (gj >= N) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = i0 + wi + 16 * a + 4 * lk + v;
        if (gi >= M) continue;
        const int64_t o = (int64_t)gi * ldc + gj;
        float c = acc[a][b][v];
        if constexpr (EPI == kEpiBiasAct) {
          c += in2[gj];
          out2[o] = c * sigm_f(c);
        } else if constexpr (EPI == kEpiActBack) {
          const float z = in2[o];
          const float sg = sigm_f(z);
          c *= sg * (1.0f + z * (1.0f - sg));
        }
        Cp[o] = c;
      }
    }
  if (csum && threadIdx.x < 64 && j0 + (int)threadIdx.x < N) Cp[(int64_t)M * ldc + j0 + threadIdx.x] = colsum;
}

// the training passes' fused GEMMs (epilogues above), one K slice except kEpiColSum
template <bool TA, bool TB, int EPI>
static hipError_t gemm_epi(int M, int N, int K, const float* A, int lda, const float* B, int ldb, float* C, int ldc,
                           int splits, int64_t c_plane, const float* in2, float* out2, hipStream_t st)
{
  const int k_slice = ((K + splits - 1) / splits + 15) / 16 * 16;
  const int z = (K + k_slice - 1) / k_slice;
  dim3 grid((N + 63) / 64, (M + 63) / 64, z);
  hipLaunchKernelGGL((gemm_mfma_kernel<TA, TB, EPI>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc, k_slice,
                     c_plane, in2, out2);
  return hipGetLastError();
}

// C = op(A) op(B) with k split into `splits` planes of C (plane stride c_plane); FP32 on the
// matrix cores, FP64 on the vector units
static hipError_t gemm(bool ta, bool tb, int M, int N, int K, const float* A, int lda, const float* B, int ldb,
                       float* C, int ldc, int splits, int64_t c_plane, hipStream_t st)
{
  const int k_slice = ((K + splits - 1) / splits + 15) / 16 * 16;
  const int z = (K + k_slice - 1) / k_slice;
  dim3 grid((N + 63) / 64, (M + 63) / 64, z);
  if (!ta && !tb) hipLaunchKernelGGL((gemm_mfma_kernel<false, false>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc, k_slice, c_plane);
  else if (ta && !tb) hipLaunchKernelGGL((gemm_mfma_kernel<true, false>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc, k_slice, c_plane);
  else if (!ta && tb) hipLaunchKernelGGL((gemm_mfma_kernel<false, true>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc, k_slice, c_plane);
  else hipLaunchKernelGGL((gemm_mfma_kernel<true, true>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc, k_slice, c_plane);
  return hipGetLastError();
}

template <typename T>
static hipError_t gemm(bool ta, bool tb, int M, int N, int K, const T* A, int lda, const T* B, int ldb, T* C, int ldc,
                       int splits, int64_t c_plane, hipStream_t st)
{
  const int k_slice = ((K + splits - 1) / splits + 15) / 16 * 16;
  const int z = (K + k_slice - 1) / k_slice;
  dim3 grid((N + 63) / 64, (M + 63) / 64, z);
  if (!ta && !tb) hipLaunchKernelGGL((gemm_kernel<T, false, false>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc, k_slice, c_plane);
  else if (ta && !tb) hipLaunchKernelGGL((gemm_kernel<T, true, false>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc, k_slice, c_plane);
  else if (!ta && tb) hipLaunchKernelGGL((gemm_kernel<T, false, true>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc, k_slice, c_plane);
  else hipLaunchKernelGGL((gemm_kernel<T, true, true>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc, k_slice, c_plane);
  return hipGetLastError();
}

// number of K slices actually used by gemm() for a requested split count
static int gemm_planes(int K, int splits)
{
  const int k_slice = ((K + splits - 1) / splits + 15) / 16 * 16;
  return (K + k_slice - 1) / k_slice;
}

// ---------------------------------------------------------------------------- element-wise
template <typename T>
__device__ inline T sigm(T z) { return (T)1 / ((T)1 + exp(-z)); }

// output layer: Y = Z + b, residual r = Y - T, loss partials per block, G = 2 r / batch
__global__ void out_loss_kernel(const float* __restrict__ Z, const float* __restrict__ b, const float* __restrict__ Tg,
                                int64_t rows, float inv_b2, float* __restrict__ G, double* __restrict__ part)
{
  __shared__ double red[256];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double sq = 0.0;
  if (i < rows * 2) {
    const float y = Z[i] + b[i & 1];
    const float r = y - Tg[i];
    G[i] = r * inv_b2;
    sq = (double)r * (double)r;
  }
  red[threadIdx.x] = sq;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void sum_parts_kernel(const double* __restrict__ part, int n, double scale, float* __restrict__ out)
{
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (float)(red[0] * scale);
}

// Sum of the K-slice planes of a weight gradient, in a fixed order: a workgroup takes 64
// consecutive elements, its four wavefronts a quarter of the planes each (summed in plane
// order, their loads in flight together), then the four partial sums in wavefront order.
__global__ __launch_bounds__(256) void sum_planes_kernel(const float* __restrict__ src, int planes, int64_t count,
                                                         float* __restrict__ dst)
{
  __shared__ float part[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  const int p0 = wv * planes / 4, p1 = (wv + 1) * planes / 4;
  float s = 0.f;
  if (i < count) {
#pragma unroll 16
    for (int p = p0; p < p1; ++p) s += src[(int64_t)p * count + i];
  }
  part[wv][lane] = s;
  __syncthreads();
  if (wv == 0 && i < count) dst[i] = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1,
                            float* __restrict__ m2, int64_t count, float lr, float b1, float b2, float eps, float c1,
                            float c2)
{
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.f - b1) * gi;
  const float v = b2 * m2[i] + (1.f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = v;
  p[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// inference epilogue on [2R][n] (rows 0..R-1 values, R..2R-1 tangents):
// value h = SiLU(z + b), tangent t = SiLU'(z + b) zt
__global__ void act_tangent_kernel(double* __restrict__ Z, const double* __restrict__ b, int64_t R, int n)
{
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R * n) return;
  const double z = Z[i] + b[i % n];
  const double s = sigm(z);
  Z[i] = z * s;
  Z[R * n + i] *= s * (1.0 + z * (1.0 - s));
}

// inference input rows: [U; e3] for the value and tangent passes
__global__ void infer_input_kernel(const double* __restrict__ U, int64_t R, double* __restrict__ H)
{
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R * 3) return;
  H[i] = U[i];
  H[R * 3 + i] = (i % 3 == 2) ? 1.0 : 0.0;
}

__global__ void infer_output_kernel(const double* __restrict__ Z, const double* __restrict__ b, int64_t R,
                                    double* __restrict__ Y, double* __restrict__ dY)
{
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R * 2) return;
  Y[i] = Z[i] + b[i & 1];
  dY[i] = Z[R * 2 + i];
}

static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

// ---------------------------------------------------------------------------- fused inference
// The whole network for 16 rows per wavefront (64 rows per workgroup), activations kept in
// registers.  Hidden layers run on the FP64 matrix cores (v_mfma_f64_16x16x4f64) in
// transposed form, D = W^T A: M = output units (16 per tile), N = the wavefront's 16 rows,
// K = input units.  Operand layouts: A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k, and
// D[i][j] in lane j + 16 (i % 4), element i / 4.  So lane l (row j = l % 16, group
// g = l / 16) holds in its accumulators the units 16 m + g + 4 v (v = 0..3) of row j, and
// those are exactly the B-operand values it must supply in the next layer when the K slots
// of step s are the units 16 (s / 4) + g + 4 (s % 4) (a permutation of K, applied to the
// weight operand too), so
// activations pass from layer to layer without a transpose.  Value and tangent rows share
// each weight fragment (two MFMAs per fragment).  Each hidden layer's weights are staged in
// LDS once per workgroup.  The first layer (K = 3) and the output layer (2 units) use plain
// FMAs, the latter with a reduction over the four lane groups.
typedef double dbl4 __attribute__((ext_vector_type(4)));

// SiLU and its derivative times the tangent, FP64.  The sigmoid's reciprocal is the
// hardware FP64 estimate refined by two Newton steps (within an ulp of the quotient); the
// exponent is capped so that 1 + e^-z stays finite.
__device__ inline void silu_tangent(double z, double zt, double& h, double& t)
{
  const double d = 1.0 + exp(fmin(-z, 700.0));
  double s = __builtin_amdgcn_rcp(d);
  s = fma(s, fma(-d, s, 1.0), s);
  s = fma(s, fma(-d, s, 1.0), s);
  h = z * s;
  t = s * (1.0 + z * (1.0 - s)) * zt;
}

template <int NT>
__global__ __launch_bounds__(256) void mlp_fused_kernel(const double* __restrict__ U, int64_t n,
                                                        const double* __restrict__ par, int layers,
                                                        double* __restrict__ Y, double* __restrict__ dY)
{
  constexpr int H = 16 * NT;
  __shared__ double wl[H * H];   // the current hidden layer's W [H][H]
  const int lane = threadIdx.x & 63;
  const int j = lane & 15, g = lane >> 4;
  const int64_t r = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16 + j;
  const bool valid = r < n;
  double u0 = 0.0, u1 = 0.0, u2 = 0.0;
  if (valid) {
    u0 = U[3 * r];
    u1 = U[3 * r + 1];
    u2 = U[3 * r + 2];
  }
  double av[NT][4], at[NT][4];
  {
    const double* W = par;           // [3][H]
    const double* b = par + 3 * H;   // [H]
#pragma unroll
    for (int m = 0; m < NT; ++m)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int u = 16 * m + g + 4 * v;
        const double z = fma(W[2 * H + u], u2, fma(W[H + u], u1, fma(W[u], u0, b[u])));
        silu_tangent(z, W[2 * H + u], av[m][v], at[m][v]);
      }
  }
  int64_t off = 4 * H;
  for (int l = 1; l < layers; ++l) {
    const double* W = par + off;     // [H][H]
    const double* b = W + H * H;     // [H]
    __syncthreads();                 // every wavefront is done with the previous layer's weights
    // direct global -> LDS copies (16 bytes per lane; a wavefront fills 1 KiB at the
    // wave-uniform LDS base, lane i at base + 16 i), no registers in between
    constexpr int PER = (H * H + 511) / 512;
#pragma unroll
    for (int c = 0; c < PER; ++c) {
      const int i = 2 * threadIdx.x + 512 * c;
      if (i < H * H)
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(W + i),
                                         (__attribute__((address_space(3))) void*)(wl + 512 * c + 128 * (threadIdx.x >> 6)),
                                         16, 0, 0);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    double nv[NT][4], nt[NT][4];
#pragma unroll
    for (int mo = 0; mo < NT; ++mo) {
      dbl4 cv = {0.0, 0.0, 0.0, 0.0}, ct = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 4 * NT; ++s) {
        const int kin = 16 * (s >> 2) + g + 4 * (s & 3);
        const double a = wl[kin * H + 16 * mo + j];
        cv = __builtin_amdgcn_mfma_f64_16x16x4f64(a, av[s >> 2][s & 3], cv, 0, 0, 0);
        ct = __builtin_amdgcn_mfma_f64_16x16x4f64(a, at[s >> 2][s & 3], ct, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) silu_tangent(cv[v] + b[16 * mo + g + 4 * v], ct[v], nv[mo][v], nt[mo][v]);
    }
#pragma unroll
    for (int m = 0; m < NT; ++m)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        av[m][v] = nv[m][v];
        at[m][v] = nt[m][v];
      }
    off += (int64_t)H * H + H;
  }
  const double* W = par + off;   // [H][2]
  const double* b = W + 2 * H;
  double y0 = 0.0, y1 = 0.0, t0 = 0.0, t1 = 0.0;
#pragma unroll
  for (int m = 0; m < NT; ++m)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int u = 16 * m + g + 4 * v;
      y0 = fma(W[2 * u], av[m][v], y0);
      y1 = fma(W[2 * u + 1], av[m][v], y1);
      t0 = fma(W[2 * u], at[m][v], t0);
      t1 = fma(W[2 * u + 1], at[m][v], t1);
    }
  y0 += __shfl_xor(y0, 16);
  y1 += __shfl_xor(y1, 16);
  t0 += __shfl_xor(t0, 16);
  t1 += __shfl_xor(t1, 16);
  y0 += __shfl_xor(y0, 32);
  y1 += __shfl_xor(y1, 32);
  t0 += __shfl_xor(t0, 32);
  t1 += __shfl_xor(t1, 32);
  if (g == 0 && valid) {
    Y[2 * r] = y0 + b[0];
    Y[2 * r + 1] = y1 + b[1];
    dY[2 * r] = t0;
    dY[2 * r + 1] = t1;
  }
}

static bool mlp_fused_ok(int hidden) { return hidden % 16 == 0 && hidden >= 16 && hidden <= 128; }

static hipError_t mlp_fused(const sft_surrogate* s, const double* U, int64_t n, double* Y, double* dY, hipStream_t st)
{
  const dim3 grid((unsigned)((n + 63) / 64)), block(256);
  const int L = s->d.layers;
  switch (s->d.hidden / 16) {
  case 1: hipLaunchKernelGGL(mlp_fused_kernel<1>, grid, block, 0, st, U, n, s->par_inf, L, Y, dY); break;
  case 2: hipLaunchKernelGGL(mlp_fused_kernel<2>, grid, block, 0, st, U, n, s->par_inf, L, Y, dY); break;
  case 3: hipLaunchKernelGGL(mlp_fused_kernel<3>, grid, block, 0, st, U, n, s->par_inf, L, Y, dY); break;
  case 4: hipLaunchKernelGGL(mlp_fused_kernel<4>, grid, block, 0, st, U, n, s->par_inf, L, Y, dY); break;
  case 5: hipLaunchKernelGGL(mlp_fused_kernel<5>, grid, block, 0, st, U, n, s->par_inf, L, Y, dY); break;
  case 6: hipLaunchKernelGGL(mlp_fused_kernel<6>, grid, block, 0, st, U, n, s->par_inf, L, Y, dY); break;
  case 7: hipLaunchKernelGGL(mlp_fused_kernel<7>, grid, block, 0, st, U, n, s->par_inf, L, Y, dY); break;
  default: hipLaunchKernelGGL(mlp_fused_kernel<8>, grid, block, 0, st, U, n, s->par_inf, L, Y, dY); break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------- BF16 fused inference
// The same network for 16 rows per wavefront on the BF16 matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation), activations in FP32 registers.  Operand
// layouts of that instruction: A[i][k] in lane i + 16 (k / 8), element k % 8; B[k][j] in lane
// j + 16 (k / 8), element k % 8; D[i][j] in lane j + 16 (i / 4), element i % 4.  Lane l (row
// j = l % 16, group g = l / 16) therefore holds the units 16 m + 4 g + v (v = 0..3) of row j,
// and as its B operand of K step s it supplies the units 32 s + 16 (e / 4) + 4 g + e % 4
// (element e = 0..7), which it already holds (tiles 2 s and 2 s + 1).  The weight fragments
// are packed in that permuted K order whenever the parameters change (pack_bf16_kernel), one
// 16-byte fragment per lane, hi and lo parts: fragment index
// (((layer - 1) NT + mo) S + s) 2 + part, times 64, plus the lane.
// SPLIT: every operand x is the sum of two BF16 numbers hi = bf16(x), lo = bf16(x - hi) (16
// significant bits) and each product takes three MFMAs, hi.hi + lo.hi + hi.lo (lo.lo is below
// 2^-16 relative).  Without SPLIT: one MFMA of the rounded operands.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float flt4 __attribute__((ext_vector_type(4)));

static bool mlp_bf16_ok(int hidden) { return hidden % 32 == 0 && hidden >= 32 && hidden <= 128; }

// fragments of one hidden-to-hidden layer (16 bytes each)
static int64_t bf16_frags_per_layer(int hidden) { return (int64_t)(hidden / 16) * (hidden / 32) * 2 * 64; }

__global__ __launch_bounds__(256) void pack_bf16_kernel(const float* __restrict__ par, int H, int layers,
                                                        bf16x8* __restrict__ frag)
{
  const int NT = H / 16, S = H / 32;
  const int64_t nf = (int64_t)(layers - 1) * NT * S * 2 * 64;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nf) return;
  int64_t f = t;
  const int lane = (int)(f % 64);
  f /= 64;
  const int part = (int)(f % 2);
  f /= 2;
  const int s = (int)(f % S);
  f /= S;
  const int mo = (int)(f % NT);
  const int l = 1 + (int)(f / NT);
  const float* W = par + 4 * (int64_t)H + (int64_t)(l - 1) * (H * H + H);   // [H][H], input-major
  const int i = lane & 15, g = lane >> 4;
  bf16x8 v;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int kin = 32 * s + 16 * (e >> 2) + 4 * g + (e & 3);
    const float w = W[(int64_t)kin * H + 16 * mo + i];
    const __bf16 hi = (__bf16)w;
    v[e] = part ? (__bf16)(w - (float)hi) : hi;
  }
  frag[t] = v;
}

// SiLU and its derivative times the tangent, FP32: reciprocal from the hardware estimate and
// one Newton step; the exponent is capped so that 1 + e^-z stays finite.
__device__ inline void silu_tangent_f32(float z, float zt, float& h, float& t)
{
  const float d = 1.0f + __expf(fminf(-z, 80.0f));
  float s = __builtin_amdgcn_rcpf(d);
  s = fmaf(s, fmaf(-d, s, 1.0f), s);
  h = z * s;
  t = s * (1.0f + z * (1.0f - s)) * zt;
}

// RT row tiles of 16 per wavefront (16 RT rows): each weight fragment read from LDS serves RT
// tiles, and the fragments staged per workgroup serve 64 RT rows.  With split operands the
// fragments are double buffered: layer l + 1's are loaded into LDS while layer l runs (the
// layer's biases are read into registers before that prefetch is issued, so that waiting for
// them does not wait for it).  The plain kernel keeps one buffer (its registers leave room for
// two wavefronts per SIMD, which 128 KiB of LDS per workgroup would not).
template <int NT, bool SPLIT, int RT>
__global__ __launch_bounds__(256) void mlp_bf16_kernel(const double* __restrict__ U, int64_t n,
                                                       const float* __restrict__ par,
                                                       const bf16x8* __restrict__ frag, int layers,
                                                       double* __restrict__ Y, double* __restrict__ dY)
{
  constexpr int H = 16 * NT, S = H / 32;
  constexpr int NF = NT * S * 2 * 64;   // fragments of one layer (a multiple of 256)
  constexpr bool DB = SPLIT;
  __shared__ bf16x8 wl2[(DB ? 2 : 1) * NF];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, g = lane >> 4;
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + wave) * 16 * RT + j;   // row of tile t: r0 + 16 t
  // direct global -> LDS copies of a layer's fragments: a wavefront fills 1 KiB at its
  // wave-uniform base, lane i at base + 16 i
  auto stage = [&](const bf16x8* F, bf16x8* dst) {
#pragma unroll
    for (int c = 0; c < NF / 256; ++c)
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(F + 256 * c + threadIdx.x),
                                       (__attribute__((address_space(3))) void*)(dst + 256 * c + 64 * wave), 16, 0, 0);
  };
  if (DB && layers > 1) stage(frag, wl2);   // layer 1, behind the first layer's work
  float av[RT][NT][4], at[RT][NT][4];
  {
    const float* W = par;           // [3][H]
    const float* b = par + 3 * H;   // [H]
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const int64_t r = r0 + 16 * t;
      float u0 = 0.0f, u1 = 0.0f, u2 = 0.0f;
      if (r < n) {
        u0 = (float)U[3 * r];
        u1 = (float)U[3 * r + 1];
        u2 = (float)U[3 * r + 2];
      }
#pragma unroll
      for (int m = 0; m < NT; ++m)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int u = 16 * m + 4 * g + v;
          const float z = fmaf(W[2 * H + u], u2, fmaf(W[H + u], u1, fmaf(W[u], u0, b[u])));
          silu_tangent_f32(z, W[2 * H + u], av[t][m][v], at[t][m][v]);
        }
    }
  }
  int64_t off = 4 * H;
  for (int l = 1; l < layers; ++l) {
    // double buffer: this layer's fragments are in buffer (l - 1) % 2, and every wavefront is
    // done with layer l - 1, whose buffer takes layer l + 1.  Single buffer: every wavefront is
    // done with layer l - 1, and this layer's fragments are loaded now.
    if constexpr (DB) __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const bf16x8* wl = wl2 + (DB ? ((l - 1) & 1) * NF : 0);
    float bl[NT][4];
#pragma unroll
    for (int mo = 0; mo < NT; ++mo)
#pragma unroll
      for (int v = 0; v < 4; ++v) bl[mo][v] = par[off + H * H + 16 * mo + 4 * g + v];
    if constexpr (DB) {
      if (l + 1 < layers) stage(frag + (int64_t)l * NF, wl2 + (l & 1) * NF);
    } else {
      stage(frag + (int64_t)(l - 1) * NF, wl2);
    }
    // meanwhile the B operands of every K step: this lane's activations in the permuted order
    bf16x8 bvh[RT][S], bvl[RT][S], bth[RT][S], btl[RT][S];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int s = 0; s < S; ++s)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float x = av[t][2 * s + (e >> 2)][e & 3], y = at[t][2 * s + (e >> 2)][e & 3];
          const __bf16 xh = (__bf16)x, yh = (__bf16)y;
          bvh[t][s][e] = xh;
          bth[t][s][e] = yh;
          if constexpr (SPLIT) {
            bvl[t][s][e] = (__bf16)(x - (float)xh);
            btl[t][s][e] = (__bf16)(y - (float)yh);
          }
        }
    if constexpr (!DB) {
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
#pragma unroll
    for (int mo = 0; mo < NT; ++mo) {
      flt4 cv[RT], ct[RT];
#pragma unroll
      for (int t = 0; t < RT; ++t) cv[t] = ct[t] = flt4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const bf16x8 ah = wl[((mo * S + s) * 2) * 64 + lane];
#pragma unroll
        for (int t = 0; t < RT; ++t) {
          cv[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bvh[t][s], cv[t], 0, 0, 0);
          ct[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bth[t][s], ct[t], 0, 0, 0);
        }
        if constexpr (SPLIT) {
          const bf16x8 al = wl[((mo * S + s) * 2 + 1) * 64 + lane];
#pragma unroll
          for (int t = 0; t < RT; ++t) {
            cv[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bvh[t][s], cv[t], 0, 0, 0);
            cv[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bvl[t][s], cv[t], 0, 0, 0);
            ct[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bth[t][s], ct[t], 0, 0, 0);
            ct[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, btl[t][s], ct[t], 0, 0, 0);
          }
        }
      }
      // the B operands hold this layer's inputs: the outputs may overwrite av, at
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          silu_tangent_f32(cv[t][v] + bl[mo][v], ct[t][v], av[t][mo][v], at[t][mo][v]);
    }
    off += (int64_t)H * H + H;
  }
  const float* W = par + off;   // [H][2]
  const float* b = W + 2 * H;
#pragma unroll
  for (int t = 0; t < RT; ++t) {
    float y0 = 0.0f, y1 = 0.0f, t0 = 0.0f, t1 = 0.0f;
#pragma unroll
    for (int m = 0; m < NT; ++m)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int u = 16 * m + 4 * g + v;
        y0 = fmaf(W[2 * u], av[t][m][v], y0);
        y1 = fmaf(W[2 * u + 1], av[t][m][v], y1);
        t0 = fmaf(W[2 * u], at[t][m][v], t0);
        t1 = fmaf(W[2 * u + 1], at[t][m][v], t1);
      }
    y0 += __shfl_xor(y0, 16);
    y1 += __shfl_xor(y1, 16);
    t0 += __shfl_xor(t0, 16);
    t1 += __shfl_xor(t1, 16);
    y0 += __shfl_xor(y0, 32);
    y1 += __shfl_xor(y1, 32);
    t0 += __shfl_xor(t0, 32);
    t1 += __shfl_xor(t1, 32);
    const int64_t r = r0 + 16 * t;
    if (g == 0 && r < n) {
      Y[2 * r] = (double)(y0 + b[0]);
      Y[2 * r + 1] = (double)(y1 + b[1]);
      dY[2 * r] = (double)t0;
      dY[2 * r + 1] = (double)t1;
    }
  }
}

// rows per wavefront of the BF16 kernel: 16 * MLP_BF16_RT
#ifndef MLP_BF16_RT
#define MLP_BF16_RT 2
#endif

template <bool SPLIT>
static hipError_t mlp_bf16_launch(const sft_surrogate* s, const double* U, int64_t n, double* Y, double* dY,
                                  hipStream_t st)
{
  constexpr int RT = MLP_BF16_RT;
  const dim3 grid((unsigned)((n + 64 * RT - 1) / (64 * RT))), block(256);
  const int L = s->d.layers;
  const bf16x8* F = (const bf16x8*)s->frag;
  switch (s->d.hidden / 32) {
  case 1: hipLaunchKernelGGL((mlp_bf16_kernel<2, SPLIT, RT>), grid, block, 0, st, U, n, s->par, F, L, Y, dY); break;
  case 2: hipLaunchKernelGGL((mlp_bf16_kernel<4, SPLIT, RT>), grid, block, 0, st, U, n, s->par, F, L, Y, dY); break;
  case 3: hipLaunchKernelGGL((mlp_bf16_kernel<6, SPLIT, RT>), grid, block, 0, st, U, n, s->par, F, L, Y, dY); break;
  default: hipLaunchKernelGGL((mlp_bf16_kernel<8, SPLIT, RT>), grid, block, 0, st, U, n, s->par, F, L, Y, dY); break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------- inference
size_t mlp_infer_scratch_bytes(int hidden, int64_t chunk)
{
  if (mlp_fused_ok(hidden)) return 256;
  return 2 * (size_t)(2 * chunk) * (size_t)std::max(hidden, 3) * sizeof(double) + 256;
}

hipError_t mlp_infer(const sft_surrogate* s, const double* U, int64_t n, double* Y, double* dY, void* scratch,
                     int64_t chunk, hipStream_t st)
{
  const int H = s->d.hidden, L = s->d.layers;
  if (s->d.inference == SFT_INFER_BF16X3) return n > 0 ? mlp_bf16_launch<true>(s, U, n, Y, dY, st) : hipSuccess;
  if (s->d.inference == SFT_INFER_BF16) return n > 0 ? mlp_bf16_launch<false>(s, U, n, Y, dY, st) : hipSuccess;
  if (mlp_fused_ok(H)) return n > 0 ? mlp_fused(s, U, n, Y, dY, st) : hipSuccess;
  double* b0 = (double*)scratch;
  double* b1 = b0 + (size_t)(2 * chunk) * std::max(H, 3);
  for (int64_t r0 = 0; r0 < n; r0 += chunk) {
    const int64_t R = std::min(chunk, n - r0);
    hipLaunchKernelGGL(infer_input_kernel, dim3(nblk(R * 3)), dim3(256), 0, st, U + r0 * 3, R, b0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    double* hin = b0;
    double* z = b1;
    for (int l = 0; l <= L; ++l) {
      const MlpLayer ly = mlp_layer(H, L, l);
      e = gemm<double>(false, false, (int)(2 * R), ly.n_out, ly.n_in, hin, ly.n_in, s->par_inf + ly.w_off, ly.n_out,
                       z, ly.n_out, 1, 0, st);
      if (e != hipSuccess) return e;
      if (l < L) {
        hipLaunchKernelGGL(act_tangent_kernel, dim3(nblk(R * ly.n_out)), dim3(256), 0, st, z, s->par_inf + ly.b_off,
                           R, ly.n_out);
      } else {
        hipLaunchKernelGGL(infer_output_kernel, dim3(nblk(R * 2)), dim3(256), 0, st, z, s->par_inf + ly.b_off, R,
                           Y + r0 * 2, dY + r0 * 2);
      }
      if ((e = hipGetLastError()) != hipSuccess) return e;
      std::swap(hin, z);
    }
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------- training
struct TrainBuf {
  float* Z;      // [L+1][B][H] pre-activations (layer l at l*B*H); the output layer's [B][2] at L*B*H
  float* Hs;     // [L+1][B][H] layer inputs: Hs[0] = U ([B][3]), Hs[l] = SiLU(Z[l-1])
  float* G;      // [B][H] gradient buffer
  float* G2;     // [B][H]
  float* plane;  // [splits][H][H] split-K partial weight gradients
  double* part;  // loss partials
  int splits;
};

static size_t train_bytes(int H, int L, int64_t B, int splits)
{
  size_t f = (size_t)(L + 1) * B * H * 2 + (size_t)B * H * 2 + (size_t)splits * (H + 1) * H;
  return f * sizeof(float) + (size_t)nblk(B * 2) * sizeof(double) + 1024;
}

static void train_layout(void* ws, int H, int L, int64_t B, int splits, TrainBuf& t)
{
  float* f = (float*)ws;
  t.Z = f;
  f += (size_t)(L + 1) * B * H;
  t.Hs = f;
  f += (size_t)(L + 1) * B * H;
  t.G = f;
  f += (size_t)B * H;
  t.G2 = f;
  f += (size_t)B * H;
  t.plane = f;
  f += (size_t)splits * (H + 1) * H;
  t.part = (double*)(((uintptr_t)f + 255) / 256 * 256);
  t.splits = splits;
}

// loss (mean over the batch of the summed squared residuals) and its gradient into s->grad.
// Forward: each hidden layer's GEMM adds the bias and applies SiLU in its epilogue (keeping the
// pre-activations Z for the backward pass).  Backward, layer l from the output down, with G =
// dL/dZ_l: the weight-gradient GEMM Hl^T G in K slices, whose first row tile also sums the
// columns of G (the bias gradient) into the row after W of each slice; the slices are summed in
// fixed order straight into W and b of the gradient (packed W then b); and the input-gradient
// GEMM G W^T with SiLU'(Z_{l-1}) in its epilogue gives dL/dZ_{l-1}.
static hipError_t loss_grad(sft_surrogate* s, const float* U, const float* Tg, int64_t B, float* loss, TrainBuf& t,
                            hipStream_t st)
{
  const int H = s->d.hidden, L = s->d.layers;
  hipError_t e;
  // forward
  const float* hin = U;
  for (int l = 0; l <= L; ++l) {
    const MlpLayer ly = mlp_layer(H, L, l);
    float* Z = t.Z + (size_t)l * B * H;
    if (l < L) {
      float* Hn = t.Hs + (size_t)(l + 1) * B * H;
      if ((e = gemm_epi<false, false, kEpiBiasAct>((int)B, ly.n_out, ly.n_in, hin, ly.n_in, s->par + ly.w_off,
                                                    ly.n_out, Z, ly.n_out, 1, 0, s->par + ly.b_off, Hn, st)) !=
          hipSuccess)
        return e;
      hin = Hn;
    } else {
      if ((e = gemm(false, false, (int)B, ly.n_out, ly.n_in, hin, ly.n_in, s->par + ly.w_off, ly.n_out, Z, ly.n_out,
                    1, 0, st)) != hipSuccess)
        return e;
      hipLaunchKernelGGL(out_loss_kernel, dim3(nblk(B * 2)), dim3(256), 0, st, Z, s->par + ly.b_off, Tg, B,
                         2.0f / (float)B, t.G, t.part);
      hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(256), 0, st, t.part, (int)nblk(B * 2), 1.0 / (double)B, loss);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  // backward: t.G holds dL/dY = dL/dZ_L [B][2]
  float* G = t.G;
  float* Gn = t.G2;
  for (int l = L; l >= 0; --l) {
    const MlpLayer ly = mlp_layer(H, L, l);
    const float* Hl = l == 0 ? U : t.Hs + (size_t)l * B * H;
    // dW = Hl^T G and db = column sums of G, per K slice ((n_in + 1) x n_out planes)
    const int planes = gemm_planes((int)B, t.splits);
    const int64_t pc = (int64_t)(ly.n_in + 1) * ly.n_out;
    if ((e = gemm_epi<true, false, kEpiColSum>(ly.n_in, ly.n_out, (int)B, Hl, ly.n_in, G, ly.n_out, t.plane,
                                                ly.n_out, t.splits, pc, nullptr, nullptr, st)) != hipSuccess)
      return e;
    hipLaunchKernelGGL(sum_planes_kernel, dim3((unsigned)((pc + 63) / 64)), dim3(256), 0, st, t.plane, planes, pc,
                       s->grad + ly.w_off);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (l > 0) {
      // dL/dZ_{l-1} = (G W^T) * SiLU'(Z_{l-1})
      if ((e = gemm_epi<false, true, kEpiActBack>((int)B, ly.n_in, ly.n_out, G, ly.n_out, s->par + ly.w_off,
                                                   ly.n_out, Gn, ly.n_in, 1, 0, t.Z + (size_t)(l - 1) * B * H,
                                                   nullptr, st)) != hipSuccess)
        return e;
      std::swap(G, Gn);
    }
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------- epoch shuffling
// A keyed bijection of [0, 2^(2h)): a four-round Feistel network on the two h-bit halves with
// the 32-bit integer hash "lowbias32" (C. Wellons' published finaliser) as round function.
// Cycle walking (apply again while the image is >= n) restricts it to a bijection of [0, n);
// with 2^(2h) < 4 n a walk takes fewer than 4 steps on average and always ends, since the
// cycle through x < n returns to x.
__device__ inline uint32_t hash32(uint32_t x)
{
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

__device__ inline uint32_t feistel(uint32_t x, int h, uint32_t key)
{
  const uint32_t mask = (1u << h) - 1u;
  uint32_t L = x >> h, R = x & mask;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const uint32_t t = L ^ (hash32(R ^ (key + 0x9e3779b9u * (uint32_t)(r + 1))) & mask);
    L = R;
    R = t;
  }
  return (L << h) | R;
}

// the rows first .. first + B - 1 of the shuffled order, copied into the batch buffers
__global__ __launch_bounds__(256) void gather_batch_kernel(const float* __restrict__ u, const float* __restrict__ y,
                                                           uint32_t n, int64_t first, int64_t B, int h, uint32_t key,
                                                           float* __restrict__ ub, float* __restrict__ yb)
{
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= B) return;
  uint32_t x = (uint32_t)(first + r);
  do {
    x = feistel(x, h, key);
  } while (x >= n);
  ub[3 * r] = u[3 * (int64_t)x];
  ub[3 * r + 1] = u[3 * (int64_t)x + 1];
  ub[3 * r + 2] = u[3 * (int64_t)x + 2];
  yb[2 * r] = y[2 * (int64_t)x];
  yb[2 * r + 1] = y[2 * (int64_t)x + 1];
}

// ---------------------------------------------------------------------------- C ABI
static sft_status mlp_fail(sft_status st, const char* msg, hipError_t e = hipSuccess)
{
  char buf[320];
  snprintf(buf, sizeof(buf), "%s%s%s", msg, e != hipSuccess ? ": " : "", e != hipSuccess ? hipGetErrorString(e) : "");
  return sft_set_error(st, buf);
}

// inference copy: FP64 values of the FP32 parameters, optionally rounded to BF16
// (round to nearest even on the upper 16 bits)
__global__ void inference_copy_kernel(const float* __restrict__ p, double* __restrict__ q, int64_t n, int bf16)
{
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float v = p[i];
  if (bf16) {
    uint32_t u = __float_as_uint(v);
    u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
    v = __uint_as_float(u);
  }
  q[i] = (double)v;
}

static hipError_t refresh_inference_copy(sft_surrogate* s, hipStream_t st)
{
  hipLaunchKernelGGL(inference_copy_kernel, dim3(nblk(s->P)), dim3(256), 0, st, s->par, s->par_inf, s->P,
                     s->d.inference == SFT_INFER_FP64_BF16W ? 1 : 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !s->frag) return e;
  const int64_t nf = (int64_t)(s->d.layers - 1) * bf16_frags_per_layer(s->d.hidden);
  hipLaunchKernelGGL(pack_bf16_kernel, dim3(nblk(nf)), dim3(256), 0, st, s->par, s->d.hidden, s->d.layers,
                     (bf16x8*)s->frag);
  return hipGetLastError();
}

extern "C" int64_t sft_surrogate_param_count(int32_t hidden, int32_t layers)
{
  if (hidden < 1 || layers < 1) return 0;
  return mlp_param_count(hidden, layers);
}

extern "C" void sft_surrogate_free(sft_surrogate* s)
{
  if (!s) return;
  if (s->par) (void)hipFree(s->par);
  if (s->grad) (void)hipFree(s->grad);
  if (s->mom1) (void)hipFree(s->mom1);
  if (s->mom2) (void)hipFree(s->mom2);
  if (s->par_inf) (void)hipFree(s->par_inf);
  if (s->frag) (void)hipFree(s->frag);
  delete s;
}

extern "C" sft_status sft_surrogate_create(const sft_surrogate_desc* d, const float* params, sft_surrogate** out)
{
  if (!d || !params || !out) return mlp_fail(SFT_E_INVALID, "sft_surrogate_create: null argument");
  *out = nullptr;
  if (d->hidden < 8 || d->hidden > 256 || d->layers < 1 || d->layers > 8)
    return mlp_fail(SFT_E_RANGE, "sft_surrogate_create: hidden must be in [8, 256], layers in [1, 8]");
  if (!(d->mc_hi > d->mc_lo) || !(d->q_hi > d->q_lo) || !(d->lt_hi > d->lt_lo) || !(d->c_phi != 0.0) ||
      !(d->c_amp != 0.0) || !(d->judge_tol >= 0.0))
    return mlp_fail(SFT_E_INVALID, "sft_surrogate_create: bad ranges or scales");
  if (d->inference < SFT_INFER_FP64 || d->inference > SFT_INFER_BF16)
    return mlp_fail(SFT_E_INVALID, "sft_surrogate_create: unknown inference mode");
  const bool bf16 = d->inference == SFT_INFER_BF16X3 || d->inference == SFT_INFER_BF16;
  if (bf16 && !mlp_bf16_ok(d->hidden))
    return mlp_fail(SFT_E_UNSUPPORTED, "sft_surrogate_create: BF16 inference needs hidden = 32, 64, 96 or 128");
  sft_surrogate* s = new sft_surrogate();
  std::memset(s, 0, sizeof(*s));
  s->d = *d;
  s->P = mlp_param_count(d->hidden, d->layers);
  hipError_t e = hipGetDevice(&s->device);
  if (e == hipSuccess) e = hipMalloc(&s->par, s->P * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&s->grad, s->P * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&s->mom1, s->P * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&s->mom2, s->P * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&s->par_inf, s->P * sizeof(double));
  if (e == hipSuccess && bf16 && d->layers > 1)
    e = hipMalloc(&s->frag, (size_t)(d->layers - 1) * bf16_frags_per_layer(d->hidden) * sizeof(bf16x8));
  if (e == hipSuccess) e = hipMemcpy(s->par, params, s->P * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(s->grad, 0, s->P * sizeof(float));
  if (e == hipSuccess) e = hipMemset(s->mom1, 0, s->P * sizeof(float));
  if (e == hipSuccess) e = hipMemset(s->mom2, 0, s->P * sizeof(float));
  if (e == hipSuccess) e = refresh_inference_copy(s, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    sft_surrogate_free(s);
    return mlp_fail(e == hipErrorOutOfMemory ? SFT_E_NOMEM : SFT_E_DEVICE, "sft_surrogate_create", e);
  }
  *out = s;
  return SFT_OK;
}

extern "C" sft_status sft_surrogate_get_params(const sft_surrogate* s, float* params)
{
  if (!s || !params) return mlp_fail(SFT_E_INVALID, "sft_surrogate_get_params: null argument");
  hipError_t e = hipMemcpy(params, s->par, s->P * sizeof(float), hipMemcpyDeviceToHost);
  return e == hipSuccess ? SFT_OK : mlp_fail(SFT_E_DEVICE, "sft_surrogate_get_params", e);
}

extern "C" sft_status sft_surrogate_loss_grad(sft_surrogate* s, const float* u, const float* y, int64_t n, float* loss,
                                              float* grad, void* hip_stream)
{
  if (!s || !u || !y || !loss) return mlp_fail(SFT_E_INVALID, "sft_surrogate_loss_grad: null argument");
  if (n < 1 || n > (1 << 21)) return mlp_fail(SFT_E_RANGE, "sft_surrogate_loss_grad: n outside [1, 2^21]");
  hipStream_t st = (hipStream_t)hip_stream;
  const int splits = (int)std::min<int64_t>(64, std::max<int64_t>(1, n / 64));
  void* ws = nullptr;
  hipError_t e = hipMallocAsync(&ws, train_bytes(s->d.hidden, s->d.layers, n, splits), st);
  if (e != hipSuccess) return mlp_fail(SFT_E_NOMEM, "sft_surrogate_loss_grad", e);
  TrainBuf t;
  train_layout(ws, s->d.hidden, s->d.layers, n, splits, t);
  e = loss_grad(s, u, y, n, loss, t, st);
  if (e == hipSuccess && grad) e = hipMemcpyAsync(grad, s->grad, s->P * sizeof(float), hipMemcpyDeviceToDevice, st);
  hipError_t e2 = hipFreeAsync(ws, st);
  if (e != hipSuccess) return mlp_fail(SFT_E_DEVICE, "sft_surrogate_loss_grad", e);
  if (e2 != hipSuccess) return mlp_fail(SFT_E_DEVICE, "sft_surrogate_loss_grad: free", e2);
  return SFT_OK;
}

extern "C" sft_status sft_surrogate_adam(sft_surrogate* s, float lr, void* hip_stream)
{
  if (!s) return mlp_fail(SFT_E_INVALID, "sft_surrogate_adam: null argument");
  hipStream_t st = (hipStream_t)hip_stream;
  s->step += 1;
  const float c1 = 1.0f - powf(0.9f, (float)s->step), c2 = 1.0f - powf(0.999f, (float)s->step);
  hipLaunchKernelGGL(adam_kernel, dim3(nblk(s->P)), dim3(256), 0, st, s->par, s->grad, s->mom1, s->mom2, s->P, lr, 0.9f,
                     0.999f, 1e-8f, c1, c2);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = refresh_inference_copy(s, st);
  return e == hipSuccess ? SFT_OK : mlp_fail(SFT_E_DEVICE, "sft_surrogate_adam", e);
}

extern "C" sft_status sft_surrogate_train(sft_surrogate* s, const float* u, const float* y, int64_t n, int32_t batch,
                                          int32_t epochs, float lr, float lr_min, void* hip_stream, float* epoch_loss)
{
  if (!s || !u || !y) return mlp_fail(SFT_E_INVALID, "sft_surrogate_train: null argument");
  if (batch < 16 || batch > (1 << 20) || n < batch || epochs < 1 || n > ((int64_t)1 << 31))
    return mlp_fail(SFT_E_RANGE, "sft_surrogate_train: need 16 <= batch <= n <= 2^31 and epochs >= 1");
  hipStream_t st = (hipStream_t)hip_stream;
  const int splits = std::min(64, std::max(1, batch / 64));   // K slices of the weight-gradient GEMMs
  const int64_t steps = n / batch;
  int h = 1;   // half width of the shuffling bijection: 2^(2h) >= n
  while (((int64_t)1 << (2 * h)) < n) ++h;
  const size_t tb = train_bytes(s->d.hidden, s->d.layers, batch, splits);
  void* ws = nullptr;
  float* dloss = nullptr;
  hipError_t e = hipMallocAsync(&ws, tb + steps * sizeof(float) + (size_t)batch * 5 * sizeof(float) + 256, st);
  if (e != hipSuccess) return mlp_fail(SFT_E_NOMEM, "sft_surrogate_train", e);
  TrainBuf t;
  train_layout(ws, s->d.hidden, s->d.layers, batch, splits, t);
  dloss = (float*)((char*)ws + tb);
  float* ub = (float*)((char*)ws + (tb + steps * sizeof(float) + 255) / 256 * 256);   // [batch][3]
  float* yb = ub + (size_t)batch * 3;                                                  // [batch][2]
  std::vector<float> hl(steps);
  const double total = (double)epochs * steps;
  int64_t it = 0;
  for (int ep = 0; ep < epochs && e == hipSuccess; ++ep) {
    const uint32_t key = 0x243f6a88u * (uint32_t)(ep + 1) ^ (uint32_t)s->step * 0x85a308d3u;
    for (int64_t k = 0; k < steps && e == hipSuccess; ++k, ++it) {
      // cosine learning-rate schedule from lr to lr_min
      const float lrt = lr_min + 0.5f * (lr - lr_min) * (1.0f + (float)cos(M_PI * (double)it / total));
      hipLaunchKernelGGL(gather_batch_kernel, dim3(nblk(batch)), dim3(256), 0, st, u, y, (uint32_t)n, k * batch,
                         (int64_t)batch, h, key, ub, yb);
      if ((e = hipGetLastError()) != hipSuccess) break;
      e = loss_grad(s, ub, yb, batch, dloss + k, t, st);
      if (e != hipSuccess) break;
      s->step += 1;
      const float c1 = 1.0f - powf(0.9f, (float)s->step), c2 = 1.0f - powf(0.999f, (float)s->step);
      hipLaunchKernelGGL(adam_kernel, dim3(nblk(s->P)), dim3(256), 0, st, s->par, s->grad, s->mom1, s->mom2, s->P, lrt,
                         0.9f, 0.999f, 1e-8f, c1, c2);
      e = hipGetLastError();
    }
    if (e == hipSuccess && epoch_loss) {
      e = hipMemcpyAsync(hl.data(), dloss, steps * sizeof(float), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      double m = 0.0;
      for (float v : hl) m += v;
      epoch_loss[ep] = (float)(m / (double)steps);
    }
  }
  if (e == hipSuccess) e = refresh_inference_copy(s, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  hipError_t e2 = hipFreeAsync(ws, st);
  if (e != hipSuccess) return mlp_fail(SFT_E_DEVICE, "sft_surrogate_train", e);
  if (e2 != hipSuccess) return mlp_fail(SFT_E_DEVICE, "sft_surrogate_train: free", e2);
  return SFT_OK;
}

extern "C" sft_status sft_surrogate_infer(const sft_surrogate* s, const double* u, int64_t n, double* y, double* dy,
                                          void* hip_stream)
{
  if (!s) return mlp_fail(SFT_E_INVALID, "sft_surrogate_infer: null network");
  if (n < 0) return mlp_fail(SFT_E_INVALID, "sft_surrogate_infer: negative n");
  if (n == 0) return SFT_OK;
  if (!u || !y || !dy) return mlp_fail(SFT_E_INVALID, "sft_surrogate_infer: null argument");
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t chunk = std::min<int64_t>(n, 1 << 16);
  void* ws = nullptr;
  hipError_t e = hipMallocAsync(&ws, mlp_infer_scratch_bytes(s->d.hidden, chunk), st);
  if (e != hipSuccess) return mlp_fail(SFT_E_NOMEM, "sft_surrogate_infer", e);
  e = mlp_infer(s, u, n, y, dy, ws, chunk, st);
  hipError_t e2 = hipFreeAsync(ws, st);
  if (e != hipSuccess) return mlp_fail(SFT_E_DEVICE, "sft_surrogate_infer", e);
  if (e2 != hipSuccess) return mlp_fail(SFT_E_DEVICE, "sft_surrogate_infer: free", e2);
  return SFT_OK;
}
