// sft_device.h -- device arithmetic of the SFT inner product on gfx950.
//
// Per (template, SFT) the scan evaluates the leading-order chirp at the SFT
// midpoint in FP64, reduces its phase mod 2 pi in FP64, splits the frequency into
// a window centre k0 and an offset delta in FP64, and then forms the 2K+1 kernel
// weights and the contraction with the data bins in FP32 (or FP64).
//
// Kernel weights.  With x = delta - j the offset of bin k0 + j, the midpoint
// kernel is F(x, beta) = int_{-1/2}^{1/2} exp(i(2 pi x s + pi beta s^2)) ds
// (continuum form of Eq. fresnel_og about the SFT midpoint).  Data bins are used
// without the (-1)^k midpoint factor; it is applied as (-1)^{k0} once per SFT,
// so the weights used are H_j = (-1)^j F(delta - j, beta):
//   Dirichlet (beta = 0, App. B):  H_j = sin(pi delta) / (pi (delta - j)).
//   Fresnel (beta > 0, Sec. III.C, completed square):
//     H_j = e(p-) E- - e(p+) E+  [+ (-1)^j (1+i) exp(-i pi x^2/beta) / sqrt(2 beta)
//                                  when p- < 0 <= p+, the stationary point inside]
//   with p-+ = x -+ beta/2 (the endpoint frequencies in bins), E-+ = exp(i(-+pi delta
//   + pi beta/4)) and e(p) = sgn(p) G(sqrt(2/beta) |p|) / sqrt(2 beta), where G is
//   the Fresnel auxiliary function (E(v) = (1+i)/2 - G(v) exp(i pi v^2/2)).
//   G comes from a piecewise polynomial on [0, 4.5) (fresnel_table.h) and from its
//   asymptotic series in w = 1/(pi v^2) = beta / (2 pi p^2) above, where
//   e(p) = (w (1 - 15 w^2 + 945 w^4 - 135135 w^6) + i (1 - 3 w^2 + 105 w^4 - 10395 w^6)) / (2 pi p).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fresnel_table.h"

namespace sftk {

constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double kTwoPiHi = 6.283185307179586232;       // nearest double to 2 pi
constexpr double kTwoPiLo = 2.4492935982947064e-16;     // 2 pi - kTwoPiHi
constexpr double kInvTwoPi = 0.15915494309189533577;
constexpr float kPiF = 3.14159265358979323846f;
constexpr float kInvPiF = 0.318309886183790671538f;
constexpr float kInvTwoPiF = 0.159154943091895335769f;

enum : uint32_t {
  kFlagOOB = 1u,
  kFlagTau = 2u,
  kFlagTaylor = 4u,
  kFlagNonfinite = 8u,
  kFlagEmpty = 64u
};

// ---------------------------------------------------------------- storage types
struct bf16x2 { uint16_t re, im; };

__host__ __device__ inline float bf16_to_f32(uint16_t h)
{
  union { uint32_t u; float f; } c;
  c.u = ((uint32_t)h) << 16;
  return c.f;
}

__host__ __device__ inline uint16_t f32_to_bf16(float f)
{
  union { uint32_t u; float f; } c;
  c.f = f;
  if ((c.u & 0x7f800000u) == 0x7f800000u && (c.u & 0x007fffffu)) return (uint16_t)((c.u >> 16) | 0x40u);
  uint32_t r = c.u + 0x7fffu + ((c.u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(r >> 16);
}

template <typename Bin> struct BinIO;
template <> struct BinIO<double2> {
  using R = double;
  __device__ static inline void load(const double2* p, double& re, double& im) { double2 v = *p; re = v.x; im = v.y; }
};
template <> struct BinIO<float2> {
  using R = float;
  __device__ static inline void load(const float2* p, float& re, float& im) { float2 v = *p; re = v.x; im = v.y; }
};
template <> struct BinIO<bf16x2> {
  using R = float;
  __device__ static inline void load(const bf16x2* p, float& re, float& im)
  {
    uint32_t v = *reinterpret_cast<const uint32_t*>(p);
    re = bf16_to_f32((uint16_t)(v & 0xffffu));
    im = bf16_to_f32((uint16_t)(v >> 16));
  }
};

// ---------------------------------------------------------------- waveform
// Leading-order chirp at time t for a template with tau = t_c - t > 0.
// With y = tau / (5 M) and s = y^(-1/8) (= 2 v, v the PN velocity parameter):
//   f = s^3 / (8 pi M)  -> kappa = f T = s^3 * cf,  cf = T / (8 pi M)
//   phi = phi_c - 2 y^(5/8) = phi_c - 2 y s^3
//   A = (pi M f)^(2/3) = s^2 / 4
//   fdot = (3/8) f / tau, fddot = (33/64) f / tau^2, 1/tau = s^8 / (5 M).
// s starts from an FP32 estimate and takes two division-free Newton steps on
// y s^8 = 1 (s <- s + s (1 - y s^8) / 8), which reach full FP64 accuracy.
struct Chirp {
  double kappa;  // f T (bins)
  double phase;  // GW phase (rad), unreduced
  double amp;    // A
  double beta;   // fdot T^2 (bins)
  double dres;   // fddot T^3 / 8 (bins): Taylor residual about the midpoint (Eq. max_tsft)
};

__device__ inline Chirp newton_chirp(double tau, double inv5M, double cf, double phi_c, double T)
{
  double y = tau * inv5M;
  float yf = (float)y;
  // FP32 estimate from the hardware log2/exp2 (about 1 ulp); the Newton steps fix the rest
  double s = (double)__builtin_amdgcn_exp2f(-0.125f * __builtin_amdgcn_logf(yf));
  for (int it = 0; it < 2; ++it) {
    double s2 = s * s, s4 = s2 * s2, s8 = s4 * s4;
    s = fma(s * 0.125, fma(-y, s8, 1.0), s);
  }
  double s2 = s * s, s3 = s2 * s, s8 = (s2 * s2) * (s2 * s2);
  double itau = s8 * inv5M;
  Chirp c;
  c.kappa = s3 * cf;
  c.phase = fma(-2.0 * y, s3, phi_c);
  c.amp = 0.25 * s2;
  c.beta = 0.375 * c.kappa * T * itau;
  c.dres = (33.0 / 512.0) * c.kappa * T * T * itau * itau;
  return c;
}

// phi mod 2 pi in [-pi, pi] (two-constant Cody-Waite reduction in FP64)
__device__ inline double reduce_2pi(double phi)
{
  double n = rint(phi * kInvTwoPi);
  double r = fma(-n, kTwoPiHi, phi);
  return fma(-n, kTwoPiLo, r);
}

constexpr double kTwoOverPi = 0.63661977236758134308;
constexpr double kPiO2Hi = 1.5707963267948966192;     // nearest double to pi/2
constexpr double kPiO2Lo = 6.123233995736766036e-17;  // pi/2 - kPiO2Hi

// (sin phi, cos phi) in FP32 for an unreduced FP64 phase: phi = n pi/2 + r with
// |r| <= pi/4 by a two-constant Cody-Waite reduction in FP64, then the Maclaurin
// series of sin and cos on [-pi/4, pi/4] in FP32 (truncation < 1e-11), and the
// quadrant n mod 4 applied by swapping and negating.
__device__ inline void phasor(double phi, float& s, float& c)
{
  const double n = rint(phi * kTwoOverPi);
  double r = fma(-n, kPiO2Hi, phi);
  r = fma(-n, kPiO2Lo, r);
  const float x = (float)r;
  const float x2 = x * x;
  const float sp = x * fmaf(x2, fmaf(x2, fmaf(x2, fmaf(x2, fmaf(x2, -2.50521084e-8f, 2.75573192e-6f),
                                                          -1.98412698e-4f), 8.33333333e-3f), -1.66666667e-1f), 1.0f);
  const float cp = fmaf(x2, fmaf(x2, fmaf(x2, fmaf(x2, fmaf(x2, fmaf(x2, 2.08767570e-9f, -2.75573192e-7f),
                                                              2.48015873e-5f), -1.38888889e-3f), 4.16666667e-2f), -0.5f), 1.0f);
  const int q = (int)((long long)n & 3);
  const float s0 = (q & 1) ? cp : sp;
  const float c0 = (q & 1) ? sp : cp;
  s = (q & 2) ? -s0 : s0;
  c = ((q + 1) & 2) ? -c0 : c0;
}

// ---------------------------------------------------------------- Fresnel endpoint term
// 2 pi e(p) = 2 pi sgn(p) G(sqrt(2/beta)|p|) / sqrt(2 beta) as (re, im).  In the
// asymptotic range (v >= 4.5) with r = 1/p and w = beta r^2 / (2 pi):
//   2 pi e(p) = r w gs(w^2) + i r fs(w^2),
//   fs = 1 - 3 W + 105 W^2 - 10395 W^3,  gs = 1 - 15 W + 945 W^2 - 135135 W^3,  W = w^2.
// Below, G(v) from the LDS table (interval width 1/2, Horner in v - centre), scaled
// by tsc = 2 pi / sqrt(2 beta).  bq = beta / (2 pi).
__device__ inline float2 fres_endpoint2(float p, float bq, float sq2ob, float tsc, const float2* tab)
{
  const float v = fabsf(p) * sq2ob;
  if (v >= SFT_G_VASYM) {
    const float r = __builtin_amdgcn_rcpf(p);
    const float w = bq * (r * r);
    const float W = w * w;
    const float fs = fmaf(W, fmaf(W, fmaf(W, -10395.0f, 105.0f), -3.0f), 1.0f);
    const float gs = fmaf(W, fmaf(W, fmaf(W, -135135.0f, 945.0f), -15.0f), 1.0f);
    return make_float2((r * w) * gs, r * fs);
  }
  int i = (int)(v * (1.0f / SFT_G_WIDTH));
  i = i < SFT_G_NINT - 1 ? i : SFT_G_NINT - 1;
  i = i > 0 ? i : 0;
  const float u = v - ((float)i + 0.5f) * SFT_G_WIDTH;
  const float2* cc = tab + i * (SFT_G_DEG + 1);
  float gr = cc[SFT_G_DEG].x, gi = cc[SFT_G_DEG].y;
#pragma unroll
  for (int k = SFT_G_DEG - 1; k >= 0; --k) {
    gr = fmaf(gr, u, cc[k].x);
    gi = fmaf(gi, u, cc[k].y);
  }
  const float sc = p < 0.0f ? -tsc : tsc;
  return make_float2(gr * sc, gi * sc);
}

}  // namespace sftk
