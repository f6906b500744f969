// Pick output shared by the grid sweep and the inertia search: the first
// sign change among a wavefront's lanes, the FP64 multisection of a pick's
// bracket, and the per-wavelength outputs (Algorithm 1's C_t, with the
// refined root that the paper does not compute).
#pragma once
#include <hip/hip_runtime.h>

#include "masw_internal.hpp"
#include "masw_math.hpp"

namespace masw {

// Output slots of one item.
struct ItemOut {
  double* ct;
  int32_t* idx;
  int32_t* status;
  double* cref;  // may be null
  int refine;
  double refine_rel;  // refinement bracket width / c_hi
};

// Outputs of a wavelength without a pick; `writer` is the one thread that
// stores them.
__device__ __forceinline__ void write_no_pick(const ItemOut& o, int status, bool writer) {
  if (writer) {
    *o.idx = -1;
    *o.status = status;
    *o.ct = __builtin_nan("");
    if (o.cref) *o.cref = __builtin_nan("");
  }
}

// First sign change among the 64 lanes of one wavefront, lane l holding
// consecutive position l; lane 0 has no predecessor.  Every wavefront that
// calls it with the same signs gets the same answer, with no LDS or barrier.
// Returns the uniform lane of the first change or -1; *sig_at / *prev_at
// receive the signs at the change and *last the sign of lane 63.
__device__ __forceinline__ int wave_first_change(int sg, int* sig_at, int* prev_at, int* last) {
  const int lane = threadIdx.x & 63;
  const int prev = __shfl_up(sg, 1, 64);
  const bool change = (lane > 0) && (sg != kNoSign) && (prev != kNoSign) && (sg != prev);
  const unsigned long long mask = __ballot(change);
  *last = __shfl(sg, 63, 64);
  if (!mask) return -1;
  const int f = __ffsll((long long)mask) - 1;
  *sig_at = __shfl(sg, f, 64);
  *prev_at = __shfl(prev, f, 64);
  return f;
}

// Status, refined root and outputs of the pick at grid index `found`, whose
// determinant signs are sig_f there and prev_f at found - 1.  Run by one whole
// wavefront; its lane 0 stores the outputs.  FP64 multisection of
// [c[found-1], c[found]], 64 increasing points per round, one per lane, lanes
// 0 and 63 at the bracket's ends; the new bracket is the first sign change.
// A uniform round (63 equal parts) is followed by at most one window round:
// from the determinant's values at the ends of the new bracket, linear
// interpolation of det K (or of 1/det K, when a layer denominator changes
// sign in the grid step: a pole) estimates the root, and lanes 1..62 are
// placed 0.9 tol apart around the estimate, so one window round ends the
// refinement whenever the estimate is within about 30 tol of the root.
// Otherwise it still narrows the bracket, and a uniform round follows.  The
// first round also yields the layer-denominator sign masks at the two grid
// points (pole flag).  Returns the determinant evaluations made.
__device__ __forceinline__ unsigned long long refine_and_write(const ItemOut& o, const double* c64, double k64,
                                                               const LayerRec64* L64, int N, int found, int sig_f,
                                                               int prev_f) {
  const int lane = threadIdx.x & 63;
  unsigned long long evals = 0;
  int status = MASW_STATUS_FOUND;
  if (sig_f == kNaNSign || prev_f == kNaNSign) status = MASW_STATUS_NAN;
  double c_ref = __builtin_nan("");
  if (status == MASW_STATUS_FOUND) {
    double lo = c64[found - 1], hi = c64[found];
    const double tol = o.refine_rel * hi;
    const double step = 0.9 * tol;  // window spacing
    bool pole = false, have_est = false;
    double est = 0.0;
    for (int k = 0; k < 48; ++k) {
      const double w = hi - lo;
      const bool window = have_est && 62.0 * step < w;
      double c;
      if (window) {
        const double a = __builtin_fmin(__builtin_fmax(est - 30.5 * step, lo + 0.5 * step), hi - 61.5 * step);
        c = (lane == 0) ? lo : (lane == 63) ? hi : a + double(lane - 1) * step;
      } else {
        c = (lane == 63) ? hi : lo + w * (double(lane) / 63.0);
      }
      uint64_t dm = 0;
      double mant;
      int expo;
      const int sg = det_sign_value(c, k64, L64, N, &dm, &mant, &expo);
      if (k == 0 && __shfl(dm, 0, 64) != __shfl(dm, 63, 64)) {
        status |= MASW_FLAG_POLE;
        pole = true;
      }
      int s_c = 0, p_c = 0, unused;
      const int f = wave_first_change(sg, &s_c, &p_c, &unused);
      evals += 64ull;
      if (f < 0 || s_c == kNaNSign || p_c == kNaNSign) break;
      lo = __shfl(c, f - 1, 64);
      hi = __shfl(c, f, 64);
      if (!o.refine || hi - lo <= tol) break;
      // root estimate from the values at the new bracket's ends, after a
      // uniform round only
      have_est = false;
      if (!window) {
        const double ma = __shfl(mant, f - 1, 64), mb = __shfl(mant, f, 64);
        const int ea = __shfl(expo, f - 1, 64), eb = __shfl(expo, f, 64);
        if (ma * mb < 0.0) {  // finite, nonzero, opposite signs
          // q = v_b / v_a for a zero, v_a / v_b for a pole; q < 0 and the
          // estimate is lo + (hi - lo) / (1 - q)
          const int de = max(-1000, min(1000, pole ? ea - eb : eb - ea));
          const double q = __builtin_ldexp(pole ? ma / mb : mb / ma, de);
          const double t = 1.0 / (1.0 - q);
          if (t > 0.0 && t < 1.0) {
            est = lo + (hi - lo) * t;
            have_est = true;
          }
        }
      }
    }
    if (o.refine) c_ref = 0.5 * (lo + hi);
  }
  if (lane == 0) {
    *o.idx = found;
    *o.status = status;
    *o.ct = c64[found];
    if (o.cref) *o.cref = c_ref;
  }
  return evals;
}

}  // namespace masw
