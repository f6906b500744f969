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
// [c[found-1], c[found]]: 64 points per round, both ends included, one per
// lane; the new bracket is the first sign change.  The first round also
// yields the layer-denominator sign masks at the two grid points (pole flag).
// Returns the determinant evaluations made.
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
    for (int k = 0; k < 24; ++k) {
      const double w = hi - lo;
      const double c = (lane == 63) ? hi : lo + w * (double(lane) / 63.0);
      uint64_t dm = 0;
      const int sg = det_sign<double, true>(c, k64, L64, N, &dm);
      if (k == 0 && __shfl(dm, 0, 64) != __shfl(dm, 63, 64)) status |= MASW_FLAG_POLE;
      int s_c = 0, p_c = 0, unused;
      const int f = wave_first_change(sg, &s_c, &p_c, &unused);
      evals += 64ull;
      if (f < 0 || s_c == kNaNSign || p_c == kNaNSign) break;
      const double nhi = (f == 63) ? hi : lo + w * (double(f) / 63.0);
      const double nlo = lo + w * (double(f - 1) / 63.0);
      lo = nlo;
      hi = nhi;
      if (!o.refine || hi - lo <= tol) break;
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
