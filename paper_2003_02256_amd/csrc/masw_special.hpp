// Special functions of the per-layer terms, for the argument ranges the
// kernels use, in FP64 and FP32.  Written from the mathematics:
//
//  * reciprocal and reciprocal square root: the hardware estimate
//    (v_rcp / v_rsq, within 2^-21 relative in FP64) and, in FP64, one
//    third-order correction: with e the estimate's residual (1 - d r, or
//    1 - x y^2), 1/d = r (1 + e + e^2 + ...) and 1/sqrt(x) = y (1 + e/2 +
//    3e^2/8 + ...), so keeping the terms through e^2 leaves an error of order
//    e^3, far below the rounding; FP32 uses the estimates as they are (within
//    1 ulp);
//  * expm1(-y), y >= 0: Cody and Waite's additive range reduction
//    y = n ln2 + r with ln2 split in two parts (the high part has enough
//    trailing zero bits that n * hi is exact), |r| <= ln2/2, a polynomial for
//    expm1 on that interval, and expm1(-y) = 2^-n expm1(-r) + (2^-n - 1);
//  * sin^2(x) and sin(x) cos(x), x >= 0: Cody and Waite reduction by pi/2
//    (pi/2 in three parts), |r| <= pi/4, polynomials for sin and cos on that
//    interval, and the quadrant parity (sin^2 x = sin^2 r or cos^2 r,
//    sin x cos x = +- sin r cos r).
//
// The polynomials keep the first Taylor terms exact (expm1 z = z + z^2/2 +
// z^3 w(z), sin r = r + r^3 q(r^2), cos r = 1 - r^2/2 + r^4 v(r^2)) and
// take w, q and v from Chebyshev interpolation on the reduced interval
// (near-minimax), of the lowest degree that keeps the evaluated result
// within about 2 units of the last place: w of degree 9 (FP64) or 3 (FP32),
// q and v of degree 5 (FP64) or 2 (FP32).  Every step is an explicit fused
// multiply-add, so the rounding is fixed by the source.
#pragma once
#include <hip/hip_runtime.h>

namespace masw {
namespace special {

// ln 2 = kLn2Hi + kLn2Lo; kLn2Hi has 11 trailing zero significand bits (FP64)
constexpr double kLn2Hi = 0.6931471805598903;      // 0x3fe62e42fefa3800
constexpr double kLn2Lo = 5.497923018708371e-14;
constexpr double kInvLn2 = 1.4426950408889634;
// pi/2 = kPio2_1 + kPio2_2 + kPio2_3 (each the double nearest to the remainder)
constexpr double kPio2_1 = 1.5707963267948966;
constexpr double kPio2_2 = 6.123233995736766e-17;
constexpr double kPio2_3 = -1.4973849048591698e-33;
constexpr double kTwoOverPi = 0.6366197723675814;

// FP32 splits: kLn2HiF has 8 trailing zero significand bits
constexpr float kLn2HiF = 0.693145751953125f;
constexpr float kLn2LoF = 1.428606765330187e-06f;
constexpr float kInvLn2F = 1.44269504f;
constexpr float kPio2_1F = 1.5707963705062866f;
constexpr float kPio2_2F = -4.371138828673793e-08f;
constexpr float kPio2_3F = -1.7151245100058819e-15f;
constexpr float kTwoOverPiF = 0.63661977f;

// Polynomial coefficients, highest degree first (Chebyshev interpolants of
// w(z) = (expm1 z - z - z^2/2)/z^3 on |z| <= ln2/2, q(u) = (sin r/r - 1)/u
// and v(u) = ((cos r - 1)/u + 1/2)/u on 0 <= u = r^2 <= (pi/4)^2).
constexpr double kExpm1W[10] = {2.091122972975856e-09, 2.5100375832561234e-08, 2.755728298405588e-07,
                                2.7557268480310024e-06, 2.4801587317135164e-05, 0.00019841269863040545,
                                0.0013888888888886554, 0.008333333333330065, 0.041666666666666664,
                                0.16666666666666669};
constexpr double kSinQ[6] = {1.5918129294866608e-10, -2.5051131845003624e-08, 2.755731610255244e-06,
                             -0.00019841269836758574, 0.008333333333330948, -0.16666666666666666};
constexpr double kCosV[6] = {-1.1382632425521717e-11, 2.08761462684032e-09, -2.7557317271729793e-07,
                             2.480158729876569e-05, -0.0013888888888887398, 0.041666666666666664};
constexpr float kExpm1WF[4] = {0.001391871366649866f, 0.008357199840247631f, 0.04166662320494652f,
                               0.16666631400585175f};
constexpr float kSinQF[3] = {-0.00019587890710681677f, 0.008332747966051102f, -0.166666641831398f};
constexpr float kCosVF[3] = {2.454794230288826e-05f, -0.001388830249197781f, 0.0416666641831398f};

// ------------------------------------------------------------------- FP64 --
// One Horner step p * x + c as a three-operand v_fma_f64.  FP64 coefficients
// that do not fit in SGPRs are kept in VGPRs across the layer loop; written
// as __builtin_fma, such a step is compiled into a copy of c followed by an
// accumulating v_fmac_f64, two VALU slots instead of one.
__device__ __forceinline__ double horner(double p, double x, double c) {
  double d;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(p), "v"(x), "v"(c));
  return d;
}

__device__ __forceinline__ double rcp(double d) {
  const double r = __builtin_amdgcn_rcp(d);
  const double e = __builtin_fma(-d, r, 1.0);           // 1 - d r
  return __builtin_fma(r, __builtin_fma(e, e, e), r);   // r (1 + e + e^2)
}

// 1/sqrt(x) for a positive normal x.
__device__ __forceinline__ double rsqrt(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = __builtin_fma(-(x * y), y, 1.0);     // 1 - x y^2
  return __builtin_fma(y * e, __builtin_fma(e, 0.375, 0.5), y);  // y (1 + e/2 + 3e^2/8)
}

// expm1(-y) for finite y >= 0.
__device__ __forceinline__ double expm1_neg(double y) {
  const double m = __builtin_rint(y * -kInvLn2);  // -n
  double r = __builtin_fma(m, kLn2Hi, y);
  r = __builtin_fma(m, kLn2Lo, r);
  const double z = -r;
  double w = kExpm1W[0];
#pragma unroll
  for (int k = 1; k < 10; ++k) w = __builtin_fma(w, z, kExpm1W[k]);
  const double p = __builtin_fma(__builtin_fma(w, z, 0.5), z, 1.0);
  const double em = z * p;                          // expm1(-r)
  const double s = __builtin_ldexp(1.0, int(m));    // 2^-n (0 once it underflows)
  return __builtin_fma(s, em, s - 1.0);
}

// sin^2(x) and sin(x) cos(x) for 0 <= x < 2^20.
__device__ __forceinline__ void sin2_sincos(double x, double* s2, double* sc) {
  const double k = __builtin_rint(x * kTwoOverPi);
  double r = __builtin_fma(-k, kPio2_1, x);
  r = __builtin_fma(-k, kPio2_2, r);
  r = __builtin_fma(-k, kPio2_3, r);
  const double r2 = r * r;
  double q = kSinQ[0];
#pragma unroll
  for (int j = 1; j < 6; ++j) q = horner(q, r2, kSinQ[j]);
  const double sn = __builtin_fma(r * r2, q, r);    // sin r
  double v = kCosV[0];
#pragma unroll
  for (int j = 1; j < 6; ++j) v = horner(v, r2, kCosV[j]);
  const double cs = __builtin_fma(__builtin_fma(v, r2, -0.5), r2, 1.0);  // cos r
  const bool odd = (int(k) & 1) != 0;
  *s2 = odd ? cs * cs : sn * sn;
  *sc = odd ? -(sn * cs) : sn * cs;
}

// ------------------------------------------------------------------- FP32 --
__device__ __forceinline__ float rcp(float d) { return __builtin_amdgcn_rcpf(d); }

__device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }

__device__ __forceinline__ float expm1_neg(float y) {
  const float m = __builtin_rintf(y * -kInvLn2F);  // -n
  float r = __builtin_fmaf(m, kLn2HiF, y);
  r = __builtin_fmaf(m, kLn2LoF, r);
  const float z = -r;
  float w = kExpm1WF[0];
#pragma unroll
  for (int k = 1; k < 4; ++k) w = __builtin_fmaf(w, z, kExpm1WF[k]);
  const float p = __builtin_fmaf(__builtin_fmaf(w, z, 0.5f), z, 1.0f);
  const float em = z * p;
  const float s = __builtin_ldexpf(1.0f, int(m));
  return __builtin_fmaf(s, em, s - 1.0f);
}

__device__ __forceinline__ void sin2_sincos(float x, float* s2, float* sc) {
  const float k = __builtin_rintf(x * kTwoOverPiF);
  float r = __builtin_fmaf(-k, kPio2_1F, x);
  r = __builtin_fmaf(-k, kPio2_2F, r);
  r = __builtin_fmaf(-k, kPio2_3F, r);
  const float r2 = r * r;
  float q = kSinQF[0];
  q = __builtin_fmaf(q, r2, kSinQF[1]);
  q = __builtin_fmaf(q, r2, kSinQF[2]);
  const float sn = __builtin_fmaf(r * r2, q, r);
  float v = kCosVF[0];
  v = __builtin_fmaf(v, r2, kCosVF[1]);
  v = __builtin_fmaf(v, r2, kCosVF[2]);
  const float cs = __builtin_fmaf(__builtin_fmaf(v, r2, -0.5f), r2, 1.0f);
  const bool odd = (int(k) & 1) != 0;
  *s2 = odd ? cs * cs : sn * sn;
  *sc = odd ? -(sn * cs) : sn * cs;
}

}  // namespace special
}  // namespace masw
