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
//    sin x cos x = +- sin r cos r);
//  * for |z| <= 1, ch(z) = (cosh sqrt(z) - 1)/z = sum_n z^n/(2n+2)! and
//    shc(z) = sinh(sqrt z)/sqrt(z) = sum_n z^n/(2n+1)!: both are entire
//    functions of z, real for z of either sign (for z = -y^2 they are
//    (1 - cos y)/y^2 and sin(y)/y), so one polynomial pair serves both
//    sides of z = 0 with no square root and no range reduction.
//
// The polynomials keep the first Taylor terms exact (expm1 z = z + z^2/2 +
// z^3 w(z), sin r = r + r^3 q(r^2), cos r = 1 - r^2/2 + r^4 v(r^2),
// ch z = 1/2 + z A(z), shc z = 1 + z B(z)) and take w, q, v, A and B from
// Chebyshev interpolation on the reduced interval (near-minimax), of the
// lowest degree that keeps the evaluated result within about 2 units of the
// last place: w of degree 9 (FP64) or 3 (FP32), q and v of degree 5 (FP64)
// or 2 (FP32), A and B of degree 7 (FP64) or 3 (FP32).  Every step is an
// explicit fused multiply-add, so the rounding is fixed by the source.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

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
// A(z) = (ch z - 1/2)/z and B(z) = (shc z - 1)/z on |z| <= 1.
constexpr double kChA[8] = {1.5619384905095966e-16, 4.77955953918308e-14, 1.147074559661762e-11,
                            2.0876756982730167e-09, 2.7557319223985915e-07, 2.4801587301587403e-05,
                            0.001388888888888889,   0.041666666666666664};
constexpr double kShcB[8] = {2.811496400404939e-15,  7.647328145588498e-13,  1.6059043834374984e-10,
                             2.5052108375165837e-08, 2.755731922398594e-06,  0.00019841269841270047,
                             0.008333333333333333,   0.16666666666666666};
constexpr float kExpm1WF[4] = {0.001391871366649866f, 0.008357199840247631f, 0.04166662320494652f,
                               0.16666631400585175f};
constexpr float kSinQF[3] = {-0.00019587890710681677f, 0.008332747966051102f, -0.166666641831398f};
constexpr float kCosVF[3] = {2.454794230288826e-05f, -0.001388830249197781f, 0.0416666641831398f};
constexpr float kChAF[4] = {2.7558465376387176e-07f, 2.4803675842122175e-05f, 0.0013888889225199819f,
                            0.0416666679084301f};
constexpr float kShcBF[4] = {2.7558924102777382e-06f, 0.00019843774498440325f, 0.008333333767950535f,
                             0.1666666567325592f};

// ------------------------------------------------------------------- FP64 --
// Where the FP64 polynomial coefficients live.  Held in VGPRs (hoisted out
// of the layer loop by the compiler), a coefficient costs two VGPRs in every
// wavefront; materialised in an SGPR pair by two scalar moves where it is
// used, it costs two scalar instructions per use, which issue beside other
// wavefronts' vector instructions but take issue slots from a wavefront that
// runs alone on its SIMD.  The layer loop uses more FP64 coefficients than
// fit in SGPRs beside its other uniform values, so the choice is made per
// polynomial and per translation unit (MASW_COEFF_POLICY, before including
// this header):
//   0 (default): the small-argument series, used by about two thirds of the
//                potential evaluations, in VGPRs; the others in SGPRs;
//   1: all in SGPRs (kernels held to few VGPRs);
//   2: all in VGPRs (kernels that run one wavefront per SIMD).
// The arithmetic is the same in every case (the same FMA, product and sum
// instructions in the same order), so the results are bitwise equal.
#ifndef MASW_COEFF_POLICY
#define MASW_COEFF_POLICY 0
#endif
enum class Coef { Sgpr, Vgpr };
constexpr Coef kCoefSeries = MASW_COEFF_POLICY == 1 ? Coef::Sgpr : Coef::Vgpr;
constexpr Coef kCoefOther = MASW_COEFF_POLICY == 2 ? Coef::Vgpr : Coef::Sgpr;

// The FP64 constant with bit pattern B: in a VGPR pair of the compiler's
// choosing, or in an SGPR pair written where it is used (volatile: the
// compiler cannot hoist it out of the loop).
template <uint64_t B, Coef P>
__device__ __forceinline__ double kconst() {
  if constexpr (P == Coef::Vgpr) {
    return __builtin_bit_cast(double, B);
  } else {
    uint32_t lo, hi;
    asm volatile("s_mov_b32 %0, %1" : "=s"(lo) : "i"(int32_t(uint32_t(B))));
    asm volatile("s_mov_b32 %0, %1" : "=s"(hi) : "i"(int32_t(uint32_t(B >> 32))));
    return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
  }
}

// p * x + c as one three-operand v_fma_f64 (written as __builtin_fma with c
// in a VGPR, the step would become a copy of c and an accumulating
// v_fmac_f64).
template <Coef P>
__device__ __forceinline__ double fma_sc(double p, double x, double c) {
  double d;
  if constexpr (P == Coef::Vgpr)
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(p), "v"(x), "v"(c));
  else
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(p), "v"(x), "s"(c));
  return d;
}

// x * c0 + c1 as one v_fma_f64.  With both constants in SGPRs (one VALU
// instruction can read only one SGPR pair) c1 is first copied to a VGPR
// pair by one v_mov_b64, so the two placements round alike.
template <Coef P>
__device__ __forceinline__ double fma_cc(double x, double c0, double c1) {
  double d;
  if constexpr (P == Coef::Vgpr) {
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(x), "v"(c0), "v"(c1));
  } else {
    double v1;
    asm("v_mov_b64 %0, %1" : "=v"(v1) : "s"(c1));
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(x), "s"(c0), "v"(v1));
  }
  return d;
}

// Horner's rule for the polynomial C[0] z^(D-1) + ... + C[D-1] (highest
// degree first), one FMA per step; each coefficient after the first two is
// materialised one step ahead of the FMA that reads it.
template <const double* C, int J, int D, Coef P>
__device__ __forceinline__ double horner_k(double p, double z, double cj) {
  if constexpr (J + 1 == D) {
    return fma_sc<P>(p, z, cj);
  } else {
    const double cn = kconst<__builtin_bit_cast(uint64_t, C[J + 1]), P>();
    return horner_k<C, J + 1, D, P>(fma_sc<P>(p, z, cj), z, cn);
  }
}

template <const double* C, int D, Coef P>
__device__ __forceinline__ double poly_k(double z) {
  const double c0 = kconst<__builtin_bit_cast(uint64_t, C[0]), P>();
  const double c1 = kconst<__builtin_bit_cast(uint64_t, C[1]), P>();
  const double c2 = kconst<__builtin_bit_cast(uint64_t, C[2]), P>();
  return horner_k<C, 2, D, P>(fma_cc<P>(z, c0, c1), z, c2);
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
  const double w = poly_k<kExpm1W, 10, kCoefOther>(z);
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
  const double q = poly_k<kSinQ, 6, kCoefOther>(r2);
  const double sn = __builtin_fma(r * r2, q, r);    // sin r
  const double v = poly_k<kCosV, 6, kCoefOther>(r2);
  const double cs = __builtin_fma(__builtin_fma(v, r2, -0.5), r2, 1.0);  // cos r
  const bool odd = (int(k) & 1) != 0;
  *s2 = odd ? cs * cs : sn * sn;
  *sc = odd ? -(sn * cs) : sn * cs;
}

// ch(z) = (cosh sqrt(z) - 1)/z and shc(z) = sinh(sqrt z)/sqrt(z) for |z| <= 1.
__device__ __forceinline__ void ch_shc(double z, double* ch, double* shc) {
  const double a = poly_k<kChA, 8, kCoefSeries>(z);
  const double b = poly_k<kShcB, 8, kCoefSeries>(z);
  *ch = __builtin_fma(a, z, 0.5);
  *shc = __builtin_fma(b, z, 1.0);
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

__device__ __forceinline__ void ch_shc(float z, float* ch, float* shc) {
  float a = kChAF[0], b = kShcBF[0];
#pragma unroll
  for (int j = 1; j < 4; ++j) {
    a = __builtin_fmaf(a, z, kChAF[j]);
    b = __builtin_fmaf(b, z, kShcBF[j]);
  }
  *ch = __builtin_fmaf(a, z, 0.5f);
  *shc = __builtin_fmaf(b, z, 1.0f);
}

}  // namespace special
}  // namespace masw
