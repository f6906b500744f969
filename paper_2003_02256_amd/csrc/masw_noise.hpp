// FP64 noise band of one grid point below the half-space's S velocity (the
// test of MASW_CHECK_NOISE; the full description is in masw_noise.hip), for
// the batch check kernel and for served requests in the tick kernel.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "masw_internal.hpp"
#include "masw_math.hpp"

namespace masw {
namespace noise {

constexpr int kBisect = 44;  // B 2^-44: far finer than the factor the band test needs

// Negative eigenvalues of the symmetric 2x2 [[a, b], [b, d]].
__device__ __forceinline__ int neg2(double a, double b, double d) {
  const double det = a * d - b * b;
  if (det < 0.0) return 1;
  if (det > 0.0) return a < 0.0 ? 2 : 0;
  return (a + d < 0.0) ? 1 : 0;
}

// The half-space's scaled 2x2 block (real below its S velocity).
__device__ __forceinline__ void halfspace_block(double c2, const LayerRec<double>& hs, double* h11, double* h12,
                                                double* h22) {
  const double rr = __builtin_sqrt(1.0 - c2 * hs.ia2);
  const double sr = __builtin_sqrt(1.0 - c2 * hs.ib2);
  const double z = 1.0 / (1.0 - rr * sr);
  const double mu = hs.mh * (c2 * hs.ib2);
  *h11 = mu * rr * z;
  *h22 = mu * sr * z;
  *h12 = mu * z - 2.0 * hs.mh;
}

// ||K||_inf of the scaled matrix at c.
__device__ inline double row_norm(double c, double k, const LayerRec<double>* L, int N) {
  const double c2 = c * c;
  double p11 = 0.0, p12 = 0.0, p22 = 0.0, p13 = 0.0, p14 = 0.0, p24 = 0.0;  // layer j-1
  double B = 0.0;
  for (int j = 0; j < N; ++j) {
    const LayerRec<double> rec = load_rec<double>(L, j);
    const LayerK<double> K = layer_entries<double>(c2, k * rec.h, rec.ia2, rec.ib2, rec.rh, rec.mh);
    // diagonal block j = R_{j-1} + P_j, R = [[k11, -k12], [-k12, k22]]
    const double a00 = p11 + K.k11, a01 = -p12 + K.k12, a11 = p22 + K.k22;
    const double r0 = __builtin_fabs(a00) + __builtin_fabs(a01) + __builtin_fabs(p13) + __builtin_fabs(p14) +
                      __builtin_fabs(K.k13) + __builtin_fabs(K.k14);
    const double r1 = __builtin_fabs(a01) + __builtin_fabs(a11) + __builtin_fabs(p14) + __builtin_fabs(p24) +
                      __builtin_fabs(K.k14) + __builtin_fabs(K.k24);
    B = __builtin_fmax(B, __builtin_fmax(r0, r1));
    p11 = K.k11; p12 = K.k12; p22 = K.k22; p13 = K.k13; p14 = K.k14; p24 = K.k24;
  }
  double h11, h12, h22;
  halfspace_block(c2, load_rec<double>(L, N), &h11, &h12, &h22);
  const double a00 = p11 + h11, a01 = -p12 + h12, a11 = p22 + h22;
  const double r0 = __builtin_fabs(a00) + __builtin_fabs(a01) + __builtin_fabs(p13) + __builtin_fabs(p14);
  const double r1 = __builtin_fabs(a01) + __builtin_fabs(a11) + __builtin_fabs(p14) + __builtin_fabs(p24);
  return __builtin_fmax(B, __builtin_fmax(r0, r1));
}

// Eigenvalues of K below x0 and below x1 (counts[0], counts[1]); false if a
// pivot is not finite.
__device__ inline bool count_below(double c, double k, const LayerRec<double>* L, int N, double x0, double x1,
                            int counts[2]) {
  const double c2 = c * c;
  const double x[2] = {x0, x1};
  double s11[2] = {0.0, 0.0}, s12[2] = {0.0, 0.0}, s22[2] = {0.0, 0.0};
  int neg[2] = {0, 0};
  bool finite = true;
  for (int j = 0; j < N; ++j) {
    const LayerRec<double> rec = load_rec<double>(L, j);
    const LayerK<double> K = layer_entries<double>(c2, k * rec.h, rec.ia2, rec.ib2, rec.rh, rec.mh);
    const double q11 = K.k13, q12 = K.k14, q21 = -K.k14, q22 = K.k24;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      // pivot j = carried part + P_j - x I
      const double a = s11[i] + K.k11 - x[i], b = s12[i] + K.k12, d = s22[i] + K.k22 - x[i];
      neg[i] += neg2(a, b, d);
      const double det = a * d - b * b;
      finite = finite && (__builtin_fabs(det) < __builtin_inf()) && det != 0.0;
      const double id = 1.0 / det;
      // next carried part: R_j - Q_j^T pivot^-1 Q_j
      const double w11 = d * q11 - b * q21, w12 = d * q12 - b * q22;
      const double w21 = a * q21 - b * q11, w22 = a * q22 - b * q12;
      s11[i] = K.k11 - (q11 * w11 + q21 * w21) * id;
      s12[i] = -K.k12 - (q11 * w12 + q21 * w22) * id;
      s22[i] = K.k22 - (q12 * w12 + q22 * w22) * id;
    }
  }
  double h11, h12, h22;
  halfspace_block(c2, load_rec<double>(L, N), &h11, &h12, &h22);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double a = s11[i] + h11 - x[i], b = s12[i] + h12, d = s22[i] + h22 - x[i];
    finite = finite && (__builtin_fabs(a * d - b * b) < __builtin_inf());
    counts[i] = neg[i] + neg2(a, b, d);
  }
  return finite;
}

__device__ inline bool in_band(double c, double k, const LayerRec<double>* L, int N, double threshold) {
  const int n = 2 * (N + 1);
  const double T = threshold * 9007199254740992.0 / double(n);  // 2^53
  const double B = row_norm(c, k, L, N);
  if (!(B < __builtin_inf()) || !(B > 0.0)) return true;
  int cnt[2];
  if (!count_below(c, k, L, N, B / T, -B / T, cnt)) return true;
  if (cnt[0] == cnt[1]) return false;  // no eigenvalue in [-B/T, B/T)
  // extreme eigenvalues by bisection: lo_top < lambda_max <= hi_top, and
  // lo_bot < lambda_min <= hi_bot
  double lo_top = -B, hi_top = B, lo_bot = -B, hi_bot = B;
  for (int it = 0; it < kBisect; ++it) {
    const double mt = 0.5 * (lo_top + hi_top), mb = 0.5 * (lo_bot + hi_bot);
    if (!count_below(c, k, L, N, mt, mb, cnt)) return true;
    if (cnt[0] == n) hi_top = mt; else lo_top = mt;  // all eigenvalues below mt
    if (cnt[1] >= 1) hi_bot = mb; else lo_bot = mb;  // some eigenvalue below mb
  }
  const double amax = __builtin_fmax(__builtin_fabs(hi_top), __builtin_fabs(lo_bot));
  const double s = amax / T;
  if (!count_below(c, k, L, N, s, -s, cnt)) return true;
  return cnt[0] != cnt[1];
}

}  // namespace noise
}  // namespace masw
