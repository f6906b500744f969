// Per-lane determinant sign of the layered stiffness matrix K(k, c).
//
// The global matrix (size 2(N+1), symmetric, heptadiagonal; Section 2.1 and
// Section 3.1) is block tridiagonal in 2x2 blocks.  Layer j's 4x4 element
// matrix [[P_j, Q_j], [Q_j^T, R_j]] adds P_j to diagonal block j, R_j to block
// j+1 and Q_j to the off-diagonal block (j, j+1); the half-space's 2x2 matrix
// adds to block N.  The determinant is the product of the determinants of the
// block pivots of an unpivoted block LDL^T elimination,
//     S_0 = A_0,   S_{j+1} = A_{j+1} - Q_j^T S_j^{-1} Q_j,   det K = prod det S_j,
// which is the O(N) banded elimination that the paper runs instead of a dense
// LU (Section 2.3, Section 3.1), carried out here in registers while the
// element matrices are formed, so the matrix is never stored.  Only the sign
// is needed by the search, so only the sign of each det S_j is kept (the
// magnitude overflows FP64 beyond a few tens of layers).
//
// Entries are divided by k mu_ref (mu_ref = the half-space's rho beta^2), and
// the hyperbolic functions of a potential with large t Re sqrt(x) (t = k h)
// are multiplied by E = exp(-t Re sqrt(x)); both are positive factors that
// cancel in f * numerator / denominator, so every entry is computed with no
// overflow at any k h, and the result is real for every real c below the
// half-space's S velocity.  With q = sqrt(|x|) for x = r^2 = 1 - c^2/alpha^2
// or x = s^2 = 1 - c^2/beta^2, and z = t^2 x:
//     |z| <= 1:  E = 1,          a = cosh(tq) - 1 = z ch(z),   Sh = t shc(z),       R = x Sh
//     z > 1:     E = exp(-t q),  a = E (cosh tq - 1),          Sh = E sinh(tq)/q,   R = E q sinh(tq)
//     z < -1:    E = 1,          a = cos tq - 1,               Sh = sin(tq)/q,      R = -q sin(tq)
// where ch and shc are the entire functions (cosh sqrt(z) - 1)/z and
// sinh(sqrt z)/sqrt(z) (cos and sin for z < 0; masw_special.hpp).  The first
// row covers c = alpha or c = beta (x = 0, the removable 0/0: a = 0, Sh = t,
// R = 0) and about two thirds of the layer evaluations of the workloads, with
// one polynomial pair and no square root, exponential or range reduction.
// a and Sh are formed from that series, from expm1 or from the half-angle
// sin/cos, so that the long-wavelength cancellation 1 - cosh cosh is never
// computed as a difference of O(1) terms.
// Divisions are reciprocals refined to about 1 ulp (masw_special.hpp): only the
// sign of the determinant is used, and a last-bit difference in a quotient is
// far below the rounding of the elimination itself.
#pragma once
#include <hip/hip_runtime.h>

#include "masw_internal.hpp"
#include "masw_special.hpp"

namespace masw {

// ---------------------------------------------------------------- helpers --
template <typename T>
__device__ __forceinline__ T fma_(T a, T b, T c) {
  return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float fma_(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}

template <typename T>
__device__ __forceinline__ T sqrt_(T x) {
  return __builtin_sqrt(x);
}
template <>
__device__ __forceinline__ float sqrt_(float x) {
  return __builtin_sqrtf(x);
}

// The four functions of one potential (see the file comment).  For |z| > 1
// one reciprocal square root gives both q and 1/q, and the half-angle form
// cos(tq) - 1 = -2 sin^2(tq/2), sin(tq) = 2 sin(tq/2) cos(tq/2) keeps the
// trigonometric side accurate where tq is near a multiple of 2 pi.
template <typename T>
struct Terms {
  T E, a, Sh, R;
};

template <typename T>
__device__ __forceinline__ Terms<T> potential_terms(T x, T t, T t2) {
  Terms<T> o;
  const T z = t2 * x;  // (t q)^2, with the sign of x
  if (__builtin_fabs(z) <= T(1)) {
    T ch, shc;
    special::ch_shc(z, &ch, &shc);
    o.E = T(1);
    o.a = z * ch;
    o.Sh = t * shc;
    o.R = x * o.Sh;
  } else if (x < T(0)) {
    const T iq = special::rsqrt(-x);
    const T q = -x * iq;
    T s2, sc;
    special::sin2_sincos(T(0.5) * t * q, &s2, &sc);
    const T sn = T(2) * sc;                      // sin(tq)
    o.E = T(1);
    o.a = T(-2) * s2;                            // cos(tq) - 1
    o.Sh = sn * iq;
    o.R = -q * sn;
  } else {
    const T iq = special::rsqrt(x);
    const T q = x * iq;
    const T m = special::expm1_neg(t * q);       // E - 1
    const T half_sh = T(-0.5) * m * (T(2) + m);  // E sinh(tq) = (1 - E^2) / 2
    o.E = T(1) + m;
    o.a = T(0.5) * m * m;                        // E cosh - E = (1 - E)^2 / 2
    o.Sh = half_sh * iq;
    o.R = half_sh * q;
  }
  return o;
}

// Six distinct entries of one layer's scaled element matrix
//     [[k11,  k12,  k13,  k14],
//      [k12,  k22, -k14,  k24],
//      [k13, -k14,  k11, -k12],
//      [k14,  k24, -k12,  k22]]  / (k mu_ref)
// and gD = E_r E_s D, whose sign is the sign of the layer's denominator D.
// The coupling entries k13, k14, k24 are also kept without the factor F
// (q13 = k13 / F, ...): the block elimination takes F^2 into the reciprocal
// of its pivot's determinant instead (schur_layer), one product fewer per
// layer; kernels that need the entries themselves read k13, k14, k24.
template <typename T>
struct LayerK {
  T k11, k12, k13, k14, k22, k24, gD;
  T F, q13, q14, q24;
};

template <typename T>
__device__ __forceinline__ LayerK<T> layer_entries(T c2, T t, T ia2, T ib2, T rh, T mh) {
  const T xr = T(1) - c2 * ia2;  // r^2
  const T xs = T(1) - c2 * ib2;  // s^2
  const T t2 = t * t;
  const Terms<T> P = potential_terms(xr, t, t2);
  const Terms<T> S = potential_terms(xs, t, t2);
  const T Cr = P.E + P.a;        // E_r cosh(t r)
  const T Cs = S.E + S.a;
  const T u = P.E * S.a + P.a * S.E + P.a * S.a;  // E_r E_s (C_r C_s - 1)
  LayerK<T> o;
  o.gD = T(-2) * u + P.Sh * S.Sh + P.R * S.R;
  const T F = rh * c2 * special::rcp(o.gD);  // f / (k mu_ref), E factors cancelled
  o.F = F;
  o.k11 = F * (Cr * S.Sh - P.R * Cs);
  // F (u - R_r R_s) - mh (1 + s^2), with mh folded into the two FMAs
  o.k12 = fma_(-mh, xs, fma_(F, u - P.R * S.R, -mh));
  o.q13 = P.R * S.E - S.Sh * P.E;
  o.q14 = S.a * P.E - P.a * S.E;
  o.q24 = S.R * P.E - P.Sh * S.E;
  o.k13 = F * o.q13;
  o.k14 = F * o.q14;
  o.k22 = F * (P.Sh * Cs - S.R * Cr);
  o.k24 = F * o.q24;
  return o;
}

// Symmetric 2x2 block (s11, s12; s12, s22).
template <typename T>
struct Block2 {
  T s11, s12, s22;
};

// One layer of the block elimination.  On entry S holds the part of diagonal
// block j built so far (R_{j-1} - Q_{j-1}^T S_{j-1}^{-1} Q_{j-1}, or 0 for j = 0).
// Adds P_j to complete S_j, returns det S_j, and leaves R_j - Q_j^T S_j^{-1} Q_j
// (the start of block j+1) in S.
template <typename T>
__device__ __forceinline__ T schur_layer(Block2<T>& S, const LayerK<T>& K) {
  const T s11 = S.s11 + K.k11;
  const T s12 = S.s12 + K.k12;
  const T s22 = S.s22 + K.k22;
  const T d = s11 * s22 - s12 * s12;
  // Q_j = F [[q13, q14], [-q14, q24]];  W = adj(S_j) Q_j / F;  M = Q_j^T W / F,
  // so that Q_j^T S_j^{-1} Q_j = M F^2 / d
  const T g = K.F * (K.F * special::rcp(d));
  const T q11 = K.q13, q12 = K.q14, q21 = -K.q14, q22 = K.q24;
  const T w11 = s22 * q11 - s12 * q21;
  const T w12 = s22 * q12 - s12 * q22;
  const T w21 = s11 * q21 - s12 * q11;
  const T w22 = s11 * q22 - s12 * q12;
  const T m11 = q11 * w11 + q21 * w21;
  const T m12 = q11 * w12 + q21 * w22;
  const T m22 = q12 * w12 + q22 * w22;
  S.s11 = K.k11 - m11 * g;
  S.s12 = -K.k12 - m12 * g;
  S.s22 = K.k22 - m22 * g;
  return d;
}

// Real and imaginary parts of det S_N, S_N = S + H with H the scaled
// half-space matrix
//     h11 = mh r (1 - s^2)/(1 - r s),  h22 = mh s (1 - s^2)/(1 - r s),
//     h12 = mh ((1 - s^2)/(1 - r s) - 2),
// where r and s are taken on the principal branch from their real squares
// (x < 0 gives +i sqrt(-x)).  H is complex only above the half-space's S
// velocity; below it a real-only form is taken (no complex products, r and s
// from the refined reciprocal square root).  With a_out, *a_out receives Re
// of the (1,1) entry of S_N.
template <typename T>
__device__ __forceinline__ void halfspace_det(const Block2<T>& S, T c2, T ia2, T ib2, T mh,
                                              T* re, T* im, T* a_out = nullptr) {
  const T xr = T(1) - c2 * ia2;
  const T xs = T(1) - c2 * ib2;
  if (xs > T(0)) {
    // Below the half-space's S velocity (then also below its P velocity):
    // r, s and H are real, and so is det S_N.  The choice is per lane, so a
    // grid point's value does not depend on the wavefront that evaluates it.
    const T qr = xr * special::rsqrt(xr);
    const T qs = xs * special::rsqrt(xs);
    const T mz = mh * (c2 * ib2) * special::rcp(T(1) - qr * qs);  // mh (1 - s^2) / (1 - r s)
    const T ar = S.s11 + mz * qr;
    const T br = S.s22 + mz * qs;
    const T er = S.s12 + (mz - T(2) * mh);
    *re = ar * br - er * er;
    *im = T(0);
    if (a_out) *a_out = ar;
    return;
  }
  const T qr = sqrt_<T>(xr < T(0) ? -xr : xr);  // may be exactly 0 (c = alpha)
  const T qs = sqrt_<T>(xs < T(0) ? -xs : xs);
  const T rr = xr >= T(0) ? qr : T(0), ri = xr >= T(0) ? T(0) : qr;
  const T sr = xs >= T(0) ? qs : T(0), si = xs >= T(0) ? T(0) : qs;
  const T dr = T(1) - (rr * sr - ri * si);  // 1 - r s
  const T di = -(rr * si + ri * sr);
  const T inv = special::rcp(dr * dr + di * di);
  const T zr = dr * inv, zi = -di * inv;    // 1 / (1 - r s)
  const T mu = mh * (c2 * ib2);             // mh (1 - s^2)
  const T h11r = mu * (rr * zr - ri * zi), h11i = mu * (rr * zi + ri * zr);
  const T h22r = mu * (sr * zr - si * zi), h22i = mu * (sr * zi + si * zr);
  const T h12r = mu * zr - T(2) * mh, h12i = mu * zi;
  const T ar = S.s11 + h11r, ai = h11i;
  const T br = S.s22 + h22r, bi = h22i;
  const T er = S.s12 + h12r, ei = h12i;
  *re = ar * br - ai * bi - (er * er - ei * ei);
  *im = ar * bi + ai * br - T(2) * er * ei;
  if (a_out) *a_out = ar;
}

// Layer records are read-only for a whole launch and uniform across a
// wavefront; reading them through the constant address space lets the
// compiler use scalar loads into SGPRs, which VALU instructions take as
// operands without occupying vector registers.  A fused small launch keeps
// its records in LDS (a workgroup writes them itself): those are read as
// LDS, since a scalar load of an LDS address would read global memory at a
// meaningless address.  The compiler knows each pointer's address space
// after inlining, so the test costs nothing at run time.  The loops over
// layers read each record one layer ahead (the record after the last layer
// is the half-space's), so that the load's latency overlaps the previous
// layer's arithmetic: a wavefront alone on its SIMD otherwise waits for it
// at every layer.
template <typename T>
using ConstRec = const __attribute__((address_space(4))) LayerRec<T>;

// A pointer read from memory (a serving slot's records) is declared not to
// point into LDS, so that load_rec's address-space test folds at compile
// time.
template <typename T>
__device__ __forceinline__ const T* as_global(const T* p) {
  __builtin_assume(!__builtin_amdgcn_is_shared((const __attribute__((address_space(0))) void*)(p)));
  return p;
}

template <typename T>
__device__ __forceinline__ LayerRec<T> load_rec(const LayerRec<T>* L, int j) {
  LayerRec<T> r;
  if (__builtin_amdgcn_is_shared((const __attribute__((address_space(0))) void*)(L))) {
    const LayerRec<T>& q = L[j];
    r.ia2 = q.ia2;
    r.ib2 = q.ib2;
    r.rh = q.rh;
    r.mh = q.mh;
    r.h = q.h;
    r.aux = q.aux;
  } else {
    ConstRec<T>* p = (ConstRec<T>*)(L) + j;  // address-space cast (generic -> constant)
    r.ia2 = p->ia2;
    r.ib2 = p->ib2;
    r.rh = p->rh;
    r.mh = p->mh;
    r.h = p->h;
    r.aux = p->aux;
  }
  r.zb = r.pad2 = T(0);
  return r;
}

__device__ __forceinline__ int sign_code(bool negative, double v) {
  if (v != v) return kNaNSign;
  const int s = (v > 0.0) - (v < 0.0);
  return negative ? -s : s;
}

// sign(Re det K(k, c)) in {-1, 0, +1}, or kNaNSign.  L points at the model's
// N layer records followed by its half-space record (uniform across the
// wavefront).  With kMask, *dmask receives bit (j mod 64) xor-folded for
// every layer whose denominator D_j is negative.
template <typename T, bool kMask>
__device__ __forceinline__ int det_sign(T c, T k, const LayerRec<T>* __restrict__ L, int N,
                                        uint64_t* dmask) {
  const T c2 = c * c;
  Block2<T> S{T(0), T(0), T(0)};
  bool neg = false;
  uint64_t mask = 0;
  LayerRec<T> nxt = load_rec<T>(L, 0);
  for (int j = 0; j < N; ++j) {
    const LayerRec<T> rec = nxt;
    nxt = load_rec<T>(L, j + 1);  // one layer ahead; after the last layer, the half-space
    const LayerK<T> K = layer_entries<T>(c2, k * rec.h, rec.ia2, rec.ib2, rec.rh, rec.mh);
    if (kMask) mask ^= uint64_t(K.gD < T(0)) << (j & 63);
    const T d = schur_layer<T>(S, K);
    neg ^= (d < T(0));
  }
  const LayerRec<T> hs = nxt;
  T re, im;
  halfspace_det<T>(S, c2, hs.ia2, hs.ib2, hs.mh, &re, &im);
  if (kMask) *dmask = mask;
  return sign_code(neg, double(re));
}

// As det_sign<T, true>, also returning Re det K of the scaled matrix as
// *mant * 2^*expo (mant in [0.5, 1) in magnitude, or 0 / NaN), with no
// overflow at any N.  Used to place refinement points.
__device__ __forceinline__ int det_sign_value(double c, double k, const LayerRec<double>* __restrict__ L, int N,
                                              uint64_t* dmask, double* mant, int* expo) {
  const double c2 = c * c;
  Block2<double> S{0.0, 0.0, 0.0};
  bool neg = false;
  uint64_t mask = 0;
  double m = 1.0;
  int e = 0;
  LayerRec<double> nxt = load_rec<double>(L, 0);
  for (int j = 0; j < N; ++j) {
    const LayerRec<double> rec = nxt;
    nxt = load_rec<double>(L, j + 1);
    const LayerK<double> K = layer_entries<double>(c2, k * rec.h, rec.ia2, rec.ib2, rec.rh, rec.mh);
    mask ^= uint64_t(K.gD < 0.0) << (j & 63);
    const double d = schur_layer<double>(S, K);
    neg ^= (d < 0.0);
    int ex;
    m = __builtin_frexp(m * d, &ex);
    e += ex;
  }
  const LayerRec<double> hs = nxt;
  double re, im;
  halfspace_det<double>(S, c2, hs.ia2, hs.ib2, hs.mh, &re, &im);
  *dmask = mask;
  int ex;
  *mant = __builtin_frexp(m * re, &ex);
  *expo = e + ex;
  return sign_code(neg, re);
}

// As det_sign, also returning in *odd whether an odd number of the layer
// denominators D_j are negative.  That parity flips where c crosses a pole of
// det K (one D_j changes sign there).
template <typename T>
__device__ __forceinline__ int det_sign_parity(T c, T k, const LayerRec<T>* __restrict__ L, int N, int* odd) {
  const T c2 = c * c;
  Block2<T> S{T(0), T(0), T(0)};
  bool neg = false, par = false;
  LayerRec<T> nxt = load_rec<T>(L, 0);
  for (int j = 0; j < N; ++j) {
    const LayerRec<T> rec = nxt;
    nxt = load_rec<T>(L, j + 1);
    const LayerK<T> K = layer_entries<T>(c2, k * rec.h, rec.ia2, rec.ib2, rec.rh, rec.mh);
    par ^= (K.gD < T(0));
    const T d = schur_layer<T>(S, K);
    neg ^= (d < T(0));
  }
  const LayerRec<T> hs = nxt;
  T re, im;
  halfspace_det<T>(S, c2, hs.ia2, hs.ib2, hs.mh, &re, &im);
  *odd = par ? 1 : 0;
  return sign_code(neg, double(re));
}

// As det_sign, also returning ln|det K| of the unscaled matrix:
// sum_j ln|det S_j| + ln|det S_N| + 2(N+1) ln(k mu_ref).
template <typename T>
__device__ __forceinline__ int det_sign_logabs(T c, T k, const LayerRec<T>* __restrict__ L, int N,
                                               double mu_ref, double k64, double* logabs) {
  const T c2 = c * c;
  Block2<T> S{T(0), T(0), T(0)};
  bool neg = false;
  double acc = 0.0;
  LayerRec<T> nxt = load_rec<T>(L, 0);
  for (int j = 0; j < N; ++j) {
    const LayerRec<T> rec = nxt;
    nxt = load_rec<T>(L, j + 1);
    const LayerK<T> K = layer_entries<T>(c2, k * rec.h, rec.ia2, rec.ib2, rec.rh, rec.mh);
    const T d = schur_layer<T>(S, K);
    neg ^= (d < T(0));
    acc += ::log(::fabs(double(d)));
  }
  const LayerRec<T> hs = nxt;
  T re, im;
  halfspace_det<T>(S, c2, hs.ia2, hs.ib2, hs.mh, &re, &im);
  acc += ::log(::hypot(double(re), double(im)));
  *logabs = acc + 2.0 * double(N + 1) * ::log(k64 * mu_ref);
  return sign_code(neg, double(re));
}

}  // namespace masw
