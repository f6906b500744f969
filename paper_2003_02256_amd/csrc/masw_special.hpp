// Special functions of the per-layer terms, for the argument ranges the
// kernels use, in FP64 and FP32.  Written from the mathematics:
//
//  * reciprocal and reciprocal square root: the hardware estimate
//    (v_rcp / v_rsq; about 2^-23 relative in FP64) refined by Newton's
//    iteration, two steps in FP64 (error squares per step), none in FP32
//    (the FP32 estimates are already within 1 ulp);
//  * expm1(-y), y >= 0: Cody and Waite's additive range reduction
//    y = n ln2 + r with ln2 split in two parts (the high part has enough
//    trailing zero bits that n * hi is exact), |r| <= ln2/2, the Taylor
//    series of expm1 at 0, and expm1(-y) = 2^-n expm1(-r) + (2^-n - 1);
//  * sin^2(x) and sin(x) cos(x), x >= 0: Cody and Waite reduction by pi/2
//    (pi/2 in three parts), |r| <= pi/4, the Taylor series of sin and cos,
//    and the quadrant parity (sin^2 x = sin^2 r or cos^2 r,
//    sin x cos x = +- sin r cos r).
//
// Taylor degrees are the smallest whose first omitted term is below half an
// ulp over the reduced range: expm1 to z^13/13! (FP64) or z^8/8! (FP32); sin
// to r^15/15! (r^9/9!); cos to r^16/16! (r^10/10!).  Every step is an explicit
// fused multiply-add, so the rounding is fixed by the source.
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

// 1/k!, correctly rounded
constexpr double kInvFact[19] = {
    1.0, 1.0, 0.5, 0.16666666666666666, 0.041666666666666664, 0.008333333333333333,
    0.001388888888888889, 0.0001984126984126984, 2.48015873015873e-05, 2.7557319223985893e-06,
    2.755731922398589e-07, 2.505210838544172e-08, 2.08767569878681e-09, 1.6059043836821613e-10,
    1.1470745597729725e-11, 7.647163731819816e-13, 4.779477332387385e-14, 2.8114572543455206e-15,
    1.5619206968586225e-16};

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
  double r = __builtin_amdgcn_rcp(d);
  double e = __builtin_fma(-d, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-d, r, 1.0);
  return __builtin_fma(r, e, r);
}

// 1/sqrt(x) for a positive normal x.
__device__ __forceinline__ double rsqrt(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  double e = __builtin_fma(-hx * y, y, 0.5);  // (1 - x y^2) / 2
  y = __builtin_fma(y, e, y);
  e = __builtin_fma(-hx * y, y, 0.5);
  return __builtin_fma(y, e, y);
}

// expm1(-y) for finite y >= 0.
__device__ __forceinline__ double expm1_neg(double y) {
  const double n = __builtin_rint(y * kInvLn2);
  double r = __builtin_fma(-n, kLn2Hi, y);
  r = __builtin_fma(-n, kLn2Lo, r);
  const double z = -r;
  double p = kInvFact[13];
#pragma unroll
  for (int k = 12; k >= 1; --k) p = __builtin_fma(p, z, kInvFact[k]);
  const double em = z * p;                          // expm1(-r)
  const double s = __builtin_ldexp(1.0, -int(n));   // 2^-n (0 once it underflows)
  return __builtin_fma(s, em, s - 1.0);
}

// sin^2(x) and sin(x) cos(x) for 0 <= x < 2^20.
__device__ __forceinline__ void sin2_sincos(double x, double* s2, double* sc) {
  const double k = __builtin_rint(x * kTwoOverPi);
  double r = __builtin_fma(-k, kPio2_1, x);
  r = __builtin_fma(-k, kPio2_2, r);
  r = __builtin_fma(-k, kPio2_3, r);
  const double r2 = r * r;
  double ps = -kInvFact[15];
  ps = horner(ps, r2, kInvFact[13]);
  ps = horner(ps, r2, -kInvFact[11]);
  ps = horner(ps, r2, kInvFact[9]);
  ps = horner(ps, r2, -kInvFact[7]);
  ps = horner(ps, r2, kInvFact[5]);
  ps = horner(ps, r2, -kInvFact[3]);
  ps = __builtin_fma(ps, r2, 1.0);
  const double sn = r * ps;                         // sin r
  double pc = kInvFact[16];
  pc = horner(pc, r2, -kInvFact[14]);
  pc = horner(pc, r2, kInvFact[12]);
  pc = horner(pc, r2, -kInvFact[10]);
  pc = horner(pc, r2, kInvFact[8]);
  pc = horner(pc, r2, -kInvFact[6]);
  pc = horner(pc, r2, kInvFact[4]);
  pc = __builtin_fma(pc, r2, -0.5);
  const double cs = __builtin_fma(pc, r2, 1.0);     // cos r
  const bool odd = (int(k) & 1) != 0;
  *s2 = odd ? cs * cs : sn * sn;
  *sc = odd ? -(sn * cs) : sn * cs;
}

// ------------------------------------------------------------------- FP32 --
__device__ __forceinline__ float rcp(float d) { return __builtin_amdgcn_rcpf(d); }

__device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }

__device__ __forceinline__ float expm1_neg(float y) {
  const float n = __builtin_rintf(y * kInvLn2F);
  float r = __builtin_fmaf(-n, kLn2HiF, y);
  r = __builtin_fmaf(-n, kLn2LoF, r);
  const float z = -r;
  float p = float(kInvFact[8]);
#pragma unroll
  for (int k = 7; k >= 1; --k) p = __builtin_fmaf(p, z, float(kInvFact[k]));
  const float em = z * p;
  const float s = __builtin_ldexpf(1.0f, -int(n));
  return __builtin_fmaf(s, em, s - 1.0f);
}

__device__ __forceinline__ void sin2_sincos(float x, float* s2, float* sc) {
  const float k = __builtin_rintf(x * kTwoOverPiF);
  float r = __builtin_fmaf(-k, kPio2_1F, x);
  r = __builtin_fmaf(-k, kPio2_2F, r);
  r = __builtin_fmaf(-k, kPio2_3F, r);
  const float r2 = r * r;
  float ps = float(kInvFact[9]);
  ps = __builtin_fmaf(ps, r2, -float(kInvFact[7]));
  ps = __builtin_fmaf(ps, r2, float(kInvFact[5]));
  ps = __builtin_fmaf(ps, r2, -float(kInvFact[3]));
  ps = __builtin_fmaf(ps, r2, 1.0f);
  const float sn = r * ps;
  float pc = -float(kInvFact[10]);
  pc = __builtin_fmaf(pc, r2, float(kInvFact[8]));
  pc = __builtin_fmaf(pc, r2, -float(kInvFact[6]));
  pc = __builtin_fmaf(pc, r2, float(kInvFact[4]));
  pc = __builtin_fmaf(pc, r2, -float(kInvFact[2]));
  const float cs = __builtin_fmaf(pc, r2, 1.0f);
  const bool odd = (int(k) & 1) != 0;
  *s2 = odd ? cs * cs : sn * sn;
  *sc = odd ? -(sn * cs) : sn * cs;
}

}  // namespace special
}  // namespace masw
