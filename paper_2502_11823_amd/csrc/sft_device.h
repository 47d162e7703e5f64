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
constexpr float kFourPiSqF = 39.4784176043574344753f;   // 4 pi^2

enum : uint32_t {
  kFlagOOB = 1u,
  kFlagTau = 2u,
  kFlagTaylor = 4u,
  kFlagNonfinite = 8u,
  kFlagSurrogateFallback = 32u,
  kFlagEmpty = 64u
};
// The per-chunk flag words of the scan carry, above the flag bits, the count of SFT rows that
// entered the template's sum in that chunk (rows in its range with tau > 0).
constexpr int kUsedShift = 8;

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

// 3.5PN closed-form inspiral in Theta = nu (t_c - t) / (5 M), M the total mass [s] (the
// time-domain post-Newtonian phase and frequency series of the PN literature; Blanchet,
// Living Rev. Relativ. 17 (2014) 2).  With s = Theta^(-1/8) and L = ln Theta:
//   GW phase  phi = phi_c - (2/nu) Theta s^3 [1 + sum_k p_k s^k]        (Theta^(5/8) = Theta s^3)
//   X = 4 x = s^2 [1 + sum_k q_k s^k],  x = (M omega)^(2/3),  f = x^(3/2) / (pi M)
// k = 2..7; p_5 = c5 L, p_6 = c6 + d6 L, q_6 = e6 + g6 L.  d/dTheta of c(L) Theta^p is
// Theta^(p-1) (p c + c'), c' = dc/dL; 1/Theta = s^8.  Amplitude
//   A = nu^(2/5) x (1 + x(-107/42 + 55 nu/42) + 2 pi x^(3/2) + x^2(-2173/1512 - 1069 nu/216 + 2047 nu^2/1512)).
struct PNCoef {
  double p2, p3, p4, c5, p6, d6, p7;   // phase series
  double q2, q3, q4, q5, e6, g6, q7;   // x series
  double a2, a4;                        // amplitude 1PN and 2PN factors
};

__device__ inline PNCoef pn_coefficients(double nu)
{
  const double pi = kPi, pi2 = kPi * kPi, euler = 0.57721566490153286061, ln256 = 5.5451774444795624753;
  const double n2 = nu * nu, n3 = n2 * nu;
  PNCoef c;
  c.p2 = 3715.0 / 8064.0 + 55.0 / 96.0 * nu;
  c.p3 = -0.75 * pi;
  c.p4 = 9275495.0 / 14450688.0 + 284875.0 / 258048.0 * nu + 1855.0 / 2048.0 * n2;
  c.c5 = (-38645.0 / 172032.0 + 65.0 / 2048.0 * nu) * pi;
  c.d6 = 107.0 / 448.0;
  c.p6 = 831032450749357.0 / 57682522275840.0 - 53.0 / 40.0 * pi2 - 107.0 / 56.0 * euler
         + (-126510089885.0 / 4161798144.0 + 2255.0 / 2048.0 * pi2) * nu + 154565.0 / 1835008.0 * n2
         - 1179625.0 / 1769472.0 * n3 - c.d6 * ln256;
  c.p7 = (188516689.0 / 173408256.0 + 488825.0 / 516096.0 * nu - 141769.0 / 516096.0 * n2) * pi;
  c.q2 = 743.0 / 4032.0 + 11.0 / 48.0 * nu;
  c.q3 = -0.2 * pi;
  c.q4 = 19583.0 / 254016.0 + 24401.0 / 193536.0 * nu + 31.0 / 288.0 * n2;
  c.q5 = (-11891.0 / 53760.0 + 109.0 / 1920.0 * nu) * pi;
  c.g6 = -107.0 / 3360.0;
  c.e6 = -10052469856691.0 / 6008596070400.0 + pi2 / 6.0 + 107.0 / 420.0 * euler
         + (3147553127.0 / 780337152.0 - 451.0 / 3072.0 * pi2) * nu - 15211.0 / 442368.0 * n2
         + 25565.0 / 1327104.0 * n3 - c.g6 * ln256;
  c.q7 = (-113868647.0 / 433520640.0 - 31821.0 / 143360.0 * nu + 294941.0 / 3870720.0 * n2) * pi;
  c.a2 = -107.0 / 42.0 + 55.0 / 42.0 * nu;
  c.a4 = -2173.0 / 1512.0 - 1069.0 / 216.0 * nu + 2047.0 / 1512.0 * n2;
  return c;
}

// 3.5PN chirp at tau > 0; inv5Mnu = nu / (5 M), Mt = M [s], nu25 = nu^(2/5).
__device__ inline Chirp pn35_chirp(double tau, double nu, double inv5Mnu, double Mt, double nu25,
                                   double phi_c, double T, const PNCoef& c)
{
  const double th = tau * inv5Mnu;
  const float thf = (float)th;
  double s = (double)__builtin_amdgcn_exp2f(-0.125f * __builtin_amdgcn_logf(thf));
  for (int it = 0; it < 2; ++it) {
    const double s2 = s * s, s4 = s2 * s2, s8 = s4 * s4;
    s = fma(s * 0.125, fma(-th, s8, 1.0), s);
  }
  const double L = log(th);
  const double s2 = s * s, s3 = s2 * s, s4 = s2 * s2, s5 = s4 * s, s6 = s4 * s2, s7 = s6 * s, s8 = s4 * s4;
  // phase bracket
  const double p5 = c.c5 * L, p6 = fma(c.d6, L, c.p6);
  const double Pb = 1.0 + c.p2 * s2 + c.p3 * s3 + c.p4 * s4 + p5 * s5 + p6 * s6 + c.p7 * s7;
  // x bracket, terms q_k(L) s^(2+k) with powers p_k = -1/4 - k/8
  const double q6 = fma(c.g6, L, c.e6);
  const double t0 = s2, t2 = c.q2 * s4, t3 = c.q3 * s5, t4 = c.q4 * s6, t5 = c.q5 * s7, t6 = q6 * s8, t7 = c.q7 * s8 * s;
  const double X = t0 + t2 + t3 + t4 + t5 + t6 + t7;
  // dX/dTheta = s^8 sum_k (p_k term_k + g6 s^8 [k = 6]);  d2X/dTheta2 = s^16 sum_k ((p_k-1)(p_k term_k + b_k) + p_k b_k)
  const double g6s = c.g6 * s8;
  const double e0 = -0.25 * t0, e2 = -0.5 * t2, e3 = -0.625 * t3, e4 = -0.75 * t4, e5 = -0.875 * t5,
               e6 = -1.0 * t6 + g6s, e7 = -1.125 * t7;
  const double dX = s8 * (e0 + e2 + e3 + e4 + e5 + e6 + e7);
  const double d2X = s8 * s8 * (-1.25 * e0 - 1.5 * e2 - 1.625 * e3 - 1.75 * e4 - 1.875 * e5
                                + (-2.0 * e6 - g6s) - 2.125 * e7);
  const double x = 0.25 * X, dx = 0.25 * dX, d2x = 0.25 * d2X;
  const double sx = sqrt(x);
  const double ipm = 1.0 / (kPi * Mt);
  const double dth = -inv5Mnu;
  Chirp ch;
  const double f = x * sx * ipm;
  ch.kappa = f * T;
  ch.phase = fma(-2.0 / nu * th * s3, Pb, phi_c);
  ch.amp = nu25 * x * (1.0 + x * (c.a2 + x * c.a4) + 2.0 * kPi * x * sx);
  const double fdot = 1.5 * sx * dx * dth * ipm;
  const double fddot = (0.75 / sx * dx * dx + 1.5 * sx * d2x) * dth * dth * ipm;
  ch.beta = fdot * T * T;
  ch.dres = 0.125 * fddot * T * T * T;
  return ch;
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
// Below, G(v) from the LDS table (SFT_G_NINT intervals of width SFT_G_WIDTH, Horner of degree
// SFT_G_DEG in v - centre), scaled
// by tsc = 2 pi / sqrt(2 beta).  bq = beta / (2 pi).
// The asymptotic form alone, with the series cut after NW powers of W.  Relative to |e|,
// the first dropped term is below 1e-8 for v = |p| sqrt(2/beta) of at least
//   NW = 3: SFT_G_VASYM (4.5),  NW = 1: SFT_VASYM_W1,  NW = 0: SFT_VASYM_W0
// (w = 1 / (pi v^2), W = w^2; the dropped terms 2027025 W^4, 105 W^2 and 3 W).
#define SFT_VASYM_W1 11.0f
#define SFT_VASYM_W0 76.0f
template <int NW>
__device__ inline float2 fres_endpoint_asym(float p, float bq)
{
  const float r = __builtin_amdgcn_rcpf(p);
  const float w = bq * (r * r);
  if constexpr (NW == 0) {
    return make_float2(r * w, r);
  } else {
    const float W = w * w;
    float fs, gs;
    if constexpr (NW == 3) {
      fs = fmaf(W, fmaf(W, fmaf(W, -10395.0f, 105.0f), -3.0f), 1.0f);
      gs = fmaf(W, fmaf(W, fmaf(W, -135135.0f, 945.0f), -15.0f), 1.0f);
    } else {
      static_assert(NW == 1, "series cut after 0, 1 or 3 powers of W");
      fs = fmaf(W, -3.0f, 1.0f);
      gs = fmaf(W, -15.0f, 1.0f);
    }
    return make_float2((r * w) * gs, r * fs);
  }
}

// PRE: read the interval's coefficients before the Horner steps, so that their LDS reads are in
// flight together (the one-row kernels, where the table bins are many; the multi-row kernels keep
// the interleaved reads, which need fewer registers)
template <bool PRE = false>
__device__ inline float2 fres_endpoint2(float p, float bq, float sq2ob, float tsc, const float2* tab)
{
  const float v = fabsf(p) * sq2ob;
  if (v >= SFT_G_VASYM) return fres_endpoint_asym<3>(p, bq);
  int i = (int)(v * (1.0f / SFT_G_WIDTH));
  i = i < SFT_G_NINT - 1 ? i : SFT_G_NINT - 1;
  i = i > 0 ? i : 0;
  const float u = v - ((float)i + 0.5f) * SFT_G_WIDTH;
  const float2* cc = tab + i * (SFT_G_DEG + 1);
  float gr, gi;
  if constexpr (PRE) {
    float2 c[SFT_G_DEG + 1];
#pragma unroll
    for (int k = 0; k <= SFT_G_DEG; ++k) c[k] = cc[k];
    gr = c[SFT_G_DEG].x;
    gi = c[SFT_G_DEG].y;
#pragma unroll
    for (int k = SFT_G_DEG - 1; k >= 0; --k) {
      gr = fmaf(gr, u, c[k].x);
      gi = fmaf(gi, u, c[k].y);
    }
  } else {
    gr = cc[SFT_G_DEG].x;
    gi = cc[SFT_G_DEG].y;
#pragma unroll
    for (int k = SFT_G_DEG - 1; k >= 0; --k) {
      gr = fmaf(gr, u, cc[k].x);
      gi = fmaf(gi, u, cc[k].y);
    }
  }
  const float sc = p < 0.0f ? -tsc : tsc;
  return make_float2(gr * sc, gi * sc);
}

// ---------------------------------------------------------------- FP64 Fresnel auxiliary function
// G(v) = exp(-i pi v^2 / 2) int_v^inf exp(i pi t^2 / 2) dt for v >= 0, in FP64, for the FP64
// Fresnel weights.  v <= 2: from the power series of E(v) = int_0^v exp(i pi t^2 / 2) dt =
// sum_n (i pi / 2)^n v^(2n+1) / (n! (2n+1)), G = ((1+i)/2 - E(v)) exp(-i pi v^2 / 2) (the
// largest term is below 90 at v = 2: ~3e-15 absolute).  v > 2: G = (1+i)/2 erfcx(z) with
// z = (1 - i) sqrt(pi) v / 2 (erfcx(z) = exp(z^2) erfc(z)), erfcx from the continued fraction
// sqrt(pi) erfcx(z) = 1 / (z + (1/2) / (z + 1 / (z + (3/2) / (z + ...)))) (valid for Re z > 0),
// evaluated bottom-up from a depth that reaches ~1e-15 relative: 60 terms at v = 2, 40 from
// 2.5, 30 from 3, 20 from 4, 10 from 6.
__device__ inline double2 fresnel_aux64(double v)
{
  if (v <= 2.0) {
    const double v2 = v * v;
    const double f0 = 0.5 * kPi * v2;
    double tr = v, ti = 0.0;   // (i pi / 2)^n v^(2n+1) / n!
    double er = v, ei = 0.0;
    for (int n = 1; n < 64; ++n) {
      const double f = f0 / (double)n;
      const double nr = -ti * f, ni = tr * f;
      tr = nr;
      ti = ni;
      const double inv = 1.0 / (double)(2 * n + 1);
      er = fma(tr, inv, er);
      ei = fma(ti, inv, ei);
      if (fabs(tr) + fabs(ti) < 1e-17 * (fabs(er) + fabs(ei))) break;
    }
    double s, c;
    sincos(f0, &s, &c);
    const double ar = 0.5 - er, ai = 0.5 - ei;   // ((1+i)/2 - E) (c - i s)
    return make_double2(ar * c + ai * s, ai * c - ar * s);
  }
  const double zr = 0.88622692545275801365 * v, zi = -zr;   // sqrt(pi) / 2 = 0.886...
  const int N = v < 2.5 ? 60 : v < 3.0 ? 40 : v < 4.0 ? 30 : v < 6.0 ? 20 : 10;
  double tr = 0.0, ti = 0.0;
  for (int n = N; n >= 1; --n) {
    const double dr = zr + tr, di = zi + ti;
    const double q = (0.5 * (double)n) / (dr * dr + di * di);
    tr = dr * q;
    ti = -di * q;
  }
  const double dr = zr + tr, di = zi + ti;
  const double q = 0.56418958354775628695 / (dr * dr + di * di);   // 1 / sqrt(pi)
  const double xr = dr * q, xi = -di * q;                          // erfcx(z)
  return make_double2(0.5 * (xr - xi), 0.5 * (xr + xi));           // (1+i)/2 erfcx(z)
}

// ---------------------------------------------------------------- central bin, small drift
// For |x| <= SFT_SERIES_DELTA and |beta| <= SFT_SERIES_BETA the kernel
//   F(x, beta) = int_{-1/2}^{1/2} exp(i (2 pi x s + pi beta s^2)) ds
// is summed directly as sum_{n <= 3} (i pi beta)^n / n! M_2n(x), with the real moments
//   M_2n(x) = int s^2n cos(2 pi x s) ds = 4^-n sum_k (-1)^k (pi x)^2k / ((2k)! (2n + 2k + 1))
// (k <= 3; the dropped terms in beta and x together are below 6e-9 relative).  There the two
// endpoint terms of the central bin grow as min(1 / (2 pi |x|), 0.7 / sqrt(2 beta)) and
// cancel to a weight near 1, which would amplify their FP32 rounding up to tenfold at
// beta ~ 0.005; the series has no such cancellation.  Beyond those bounds the amplification
// stays below ~2.5 and the endpoint form is kept.
#define SFT_SERIES_BETA 0.04f
#define SFT_SERIES_DELTA 0.125f
__device__ inline float2 fres_central_series(float x, float beta)
{
  constexpr float c[4][4] = {
    {1.000000000e+00f, -1.666666667e-01f, 8.333333333e-03f, -1.984126984e-04f},
    {8.333333333e-02f, -2.500000000e-02f, 1.488095238e-03f, -3.858024691e-05f},
    {1.250000000e-02f, -4.464285714e-03f, 2.893518519e-04f, -7.891414141e-06f},
    {2.232142857e-03f, -8.680555556e-04f, 5.918560606e-05f, -1.669337607e-06f}};
  const float px = kPiF * x;
  const float u = px * px;
  const float pb = kPiF * beta;
  // M0 + i pi beta M2 - (pi beta)^2 / 2 M4 - i (pi beta)^3 / 6 M6, as two Horner chains in u
  // whose coefficients take the beta terms on the fly (few live registers)
  const float h4 = -0.5f * pb * pb, h6 = pb * pb * (-1.0f / 6.0f);
  float re = fmaf(h4, c[2][3], c[0][3]), im = fmaf(h6, c[3][3], c[1][3]);
#pragma unroll
  for (int k = 2; k >= 0; --k) {
    re = fmaf(re, u, fmaf(h4, c[2][k], c[0][k]));
    im = fmaf(im, u, fmaf(h6, c[3][k], c[1][k]));
  }
  return make_float2(re, pb * im);
}

}  // namespace sftk
