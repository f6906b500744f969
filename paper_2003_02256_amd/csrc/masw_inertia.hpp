// First sign change of det K by inertia counts (opt-in: MASW_SEARCH_INERTIA).
//
// Algorithm 1 walks the c grid and stops at the first grid point where
// sign(det K) differs from the previous one.  Below the half-space's S
// velocity K is real symmetric, and sign(det K) = (-1)^s with s(c) the number
// of negative eigenvalues of K(c), so the pick is the first grid point where
// the parity of s differs from its parity at c_test[0].  s is not monotone in
// c, but it is one of two monotone counts (the Wittrick-Williams theorem,
// Wittrick and Williams 1971, for the exact dynamic stiffness of a
// conservative system, here with wavenumber k fixed and frequency kc rising):
//     J(c) = s(c) + P(c) = the number of modes with phase velocity below c,
//     P(c) = sum_j P_j(c), P_j = modes of layer j with both faces fixed
//            (the poles of det K, where D_j changes sign) below c.
// E = J + P = s + 2P is non-decreasing, and s changes only where E does, so
// the first change of sign(det K) along the grid is found by a search on E
// instead of a walk (search() below):
//   0. Prediction (when the picks of neighbouring wavelengths predict this
//      one): counts at c_test[0], before a 62-point window around the
//      prediction and in it; equal counts before the window prove no change
//      there, and the window's first differing count is the change of E.
//   1. Sampling: det K's sign at c_test[0] and 63 spread grid points; the
//      first sampled sign that differs bounds the pick from above, so the
//      counts stay at velocities near it (a layer needs more sublayers, see
//      below, the further c lies above its beta).
//   2. Counts: multisection of (a, b] (E(a) = E_a known) by the 64 lanes of
//      a wavefront, each counting E at one spread grid point; the first lane
//      whose count differs from E_a gives the next (a, b], until one grid
//      step is left.
//   3. At that grid point the sign is the parity of E.  If it differs from
//      the sign at c_test[0] that is the pick.  Otherwise (a mode and a pole
//      in one grid step, or two modes) the search goes on from there.
//   4. A grid point at or above the half-space's S velocity (K complex) or
//      one where an elimination is not finite counts as a change of E.  If
//      the search stops at such a point with the sign unchanged, the rest of
//      the grid is walked as in Algorithm 1.
// No grid point below the pick is skipped unless the counts at its ends
// prove that sign(det K) is constant there, so the pick is the walk's, up to
// rounding of the counts (the FP64 noise band).  Sign changes between two
// counted points that cancel in E cannot happen; a determinant that is
// exactly zero or not finite at a grid point that is not counted is not seen.
//
// P_j from the layer alone.  For a field u(z) e^{ikx} that vanishes on both
// faces of a layer, the strain energy is the integral of
// (lambda + mu)|div u|^2 + mu (k^2 |u|^2 + |u'|^2) (the cross terms
// integrate to zero), and Wirtinger's inequality bounds the integral of
// |u'|^2 below by (pi/h)^2 times that of |u|^2.  So every fixed-face mode has
// rho omega^2 >= mu (k^2 + (pi/h)^2), i.e. c^2 > beta^2 (1 + (pi/(kh))^2),
// and P_j(c) = 0 when k h sqrt(c^2/beta^2 - 1) <= pi.  Otherwise the layer is
// cut into m = floor(k h sqrt(c^2/beta^2 - 1)/pi) + 1 equal sublayers, none
// of which has such a mode below c, and the theorem applied to the layer with
// both faces fixed gives P_j = the number of negative eigenvalues of the
// stiffness of the m - 1 interior interfaces: the same unpivoted 2x2-block
// elimination, m - 1 pivots of one sublayer's element matrix.
//
// Each count costs one elimination of K plus, per layer above that bound,
// one more element matrix and m - 1 pivots, against Algorithm 1's one
// elimination per grid point up to the pick.  One wavefront per wavelength.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "masw.h"
#include "masw_internal.hpp"
#include "masw_math.hpp"
#include "masw_pick.hpp"

namespace masw {
namespace inertia {

constexpr int kEvent = 0x7fffffff;      // count of a point that ends the search on E
constexpr double kMaxSub = 4096.0;      // sublayers of one layer before a point counts as kEvent
constexpr double kInvPi = 0.318309886183790671537767526745028724;

// Work of one wavefront.  evals, entries and pivots are per lane (each lane
// counts its own points); the rest are uniform across the wavefront.
struct Tally {
  unsigned long long evals = 0, entries = 0, pivots = 0, scan = 0, check = 0, refine = 0, useful = 0;
  // handoff: a walk (below) is not run but handed back to the caller as
  // kResume, with the grid index it would start from and its carried sign
  bool handoff = false;
  int resume = 0, resume_carry = 0;
};

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Negative eigenvalues of a symmetric 2x2 pivot with (1,1) entry a and
// determinant d != 0.
__device__ __forceinline__ int neg_eigs(double a, double d) { return d < 0.0 ? 1 : (a < 0.0 ? 2 : 0); }

__device__ __forceinline__ bool usable(double d) { return d != 0.0 && __builtin_fabs(d) < __builtin_inf(); }

// P_j(c) of one layer (its modes with both faces fixed below c), added to
// *P: zero by the energy bound when k h sqrt(c^2/beta^2 - 1) <= pi, else the
// negative eigenvalues of the m - 1 interior interfaces of m equal
// sublayers.  Clears *ok where a pivot is zero or not finite, or where the
// layer would need more than kMaxSub sublayers.  Returns the sublayer pivots
// eliminated (0 when the bound settles it).
__device__ __forceinline__ unsigned layer_poles(double c2, double kh, const LayerRec<double>& rec, int* P,
                                                bool* ok) {
  const double x = c2 * rec.ib2 - 1.0;
  if (!(x > 0.0)) return 0u;
  const double q = kh * __builtin_sqrt(x) * kInvPi;
  if (!(q >= 1.0)) return 0u;
  if (!(q < kMaxSub)) {
    *ok = false;
    return 0u;
  }
  const int m = int(q) + 1;
  const LayerK<double> Ks = layer_entries<double>(c2, kh / double(m), rec.ia2, rec.ib2, rec.rh, rec.mh);
  Block2<double> R{Ks.k11, -Ks.k12, Ks.k22};  // the first sublayer's share of interface 1
  for (int i = 1; i < m; ++i) {
    const double a2 = R.s11 + Ks.k11;
    const double d2 = schur_layer<double>(R, Ks);
    *ok = *ok && usable(d2);
    *P += neg_eigs(a2, d2);
  }
  return unsigned(m);
}

// E(c) = s(c) + 2 P(c), or kEvent (c at or above the half-space's S velocity,
// a zero or non-finite pivot, or a layer that would need more than kMaxSub
// sublayers).  The work is added to t if `tally`.
__device__ __forceinline__ int count_E(double c, double k, const LayerRec64* __restrict__ L, int N, Tally& t, bool tally) {
  const double c2 = c * c;
  const LayerRec<double> hs = load_rec<double>(L, N);
  if (!(c2 * hs.ib2 < 1.0)) return kEvent;
  unsigned long long entries = unsigned(N), pivots = unsigned(N + 1);
  Block2<double> S{0.0, 0.0, 0.0};
  int s = 0, P = 0;
  bool ok = true;
  LayerRec<double> nxt = load_rec<double>(L, 0);
  for (int j = 0; j < N; ++j) {
    const LayerRec<double> rec = nxt;
    nxt = load_rec<double>(L, j + 1);  // one layer ahead
    const double kh = k * rec.h;
    const LayerK<double> K = layer_entries<double>(c2, kh, rec.ia2, rec.ib2, rec.rh, rec.mh);
    const double a = S.s11 + K.k11;
    const double d = schur_layer<double>(S, K);
    ok = ok && usable(d);
    s += neg_eigs(a, d);
    const unsigned m = layer_poles(c2, kh, rec, &P, &ok);
    if (m) {
      ++entries;
      pivots += (unsigned long long)(m - 1);
    }
  }
  double re, im, ar;
  halfspace_det<double>(S, c2, hs.ia2, hs.ib2, hs.mh, &re, &im, &ar);
  ok = ok && usable(re);
  s += neg_eigs(ar, re);
  if (tally) {
    ++t.evals;
    t.entries += entries;
    t.pivots += pivots;
  }
  return ok ? s + 2 * P : kEvent;
}

// The split path's FP64 check of one grid point: det_sign_parity<double>'s
// sign code and pole parity from the same elimination, and in *E the
// inertia of its pivots, s(c), or kEvent where a pivot is zero or not finite
// or c is at or above the half-space's S velocity.  E(c) = s(c) when
// *poles_bounded (every layer's P_j is zero by the energy bound); otherwise
// count_E gives E(c).  Tallying s costs a few operations per layer; the
// sublayers of P_j are left to count_E, which needs them rarely.
__device__ __forceinline__ int det_sign_inertia(double c, double k, const LayerRec64* __restrict__ L, int N,
                                                int* odd, int* E, bool* poles_bounded) {
  const double c2 = c * c;
  Block2<double> S{0.0, 0.0, 0.0};
  bool neg = false, par = false, ok = true, bounded = true;
  int s = 0;
  LayerRec<double> nxt = load_rec<double>(L, 0);
  for (int j = 0; j < N; ++j) {
    const LayerRec<double> rec = nxt;
    nxt = load_rec<double>(L, j + 1);  // one layer ahead; after the last layer, the half-space
    const double kh = k * rec.h;
    const LayerK<double> K = layer_entries<double>(c2, kh, rec.ia2, rec.ib2, rec.rh, rec.mh);
    par ^= (K.gD < 0.0);
    const double a = S.s11 + K.k11;
    const double d = schur_layer<double>(S, K);
    neg ^= (d < 0.0);
    ok = ok && usable(d);
    s += neg_eigs(a, d);
    // P_j = 0 when k h sqrt(c^2/beta^2 - 1) < pi (layer_poles' bound), tested
    // with a margin below pi^2 so that layer_poles' own rounding agrees
    const double x = c2 * rec.ib2 - 1.0;
    bounded = bounded && !(x > 0.0 && kh * kh * x >= 9.86);
  }
  const LayerRec<double> hs = nxt;
  double re, im, ar;
  halfspace_det<double>(S, c2, hs.ia2, hs.ib2, hs.mh, &re, &im, &ar);
  ok = ok && usable(re) && (c2 * hs.ib2 < 1.0);
  s += neg_eigs(ar, re);
  *odd = par ? 1 : 0;
  *E = ok ? s : kEvent;
  *poles_bounded = bounded;
  return sign_code(neg, re);
}

// P(c) = sum_j P_j(c) of all layers, by layer_poles, in a loop of its own
// (the split path's rare full counts: the pivots' inertia comes from
// det_sign_inertia, and keeping the sublayers out of that elimination keeps
// its registers down).  Clears *ok as layer_poles does.
__device__ __forceinline__ int poles_below(double c, double k, const LayerRec64* __restrict__ L, int N, bool* ok) {
  const double c2 = c * c;
  int P = 0;
  LayerRec<double> nxt = load_rec<double>(L, 0);
  for (int j = 0; j < N; ++j) {
    const LayerRec<double> rec = nxt;
    nxt = load_rec<double>(L, j + 1);
    layer_poles(c2, k * rec.h, rec, &P, ok);
  }
  return P;
}

// E(c) as count_E gives it, from det_sign_inertia and poles_below.
__device__ __forceinline__ int count_E_split(double c, double k, const LayerRec64* __restrict__ L, int N) {
  int odd, E;
  bool bounded;
  det_sign_inertia(c, k, L, N, &odd, &E, &bounded);
  if (E == kEvent || bounded) return E;
  bool ok = true;
  const int P = poles_below(c, k, L, N, &ok);
  return ok ? E + 2 * P : kEvent;
}

constexpr int kResume = -3;  // a walk handed back to the caller (Tally::handoff)

// Algorithm 1's walk from grid index `start`, whose predecessor has sign
// `carry`, one grid point per lane.  Returns the index of the first change
// (-1 if none) and its signs, or kResume with t.handoff.
__device__ inline int walk(const double* c64, int n_c, double k, const LayerRec64* L, int N, int start,
                           int carry, int* sig_f, int* prev_f, Tally& t) {
  if (t.handoff) {
    t.resume = start;
    t.resume_carry = carry;
    return kResume;
  }
  const int lane = threadIdx.x & 63;
  for (int base = start; base < n_c; base += 64) {
    const int i = base + lane;
    const int sg = (i < n_c) ? det_sign<double, false>(c64[i], k, L, N, nullptr) : kNoSign;
    const int up = __shfl_up(sg, 1, 64);
    const int prev = (lane == 0) ? carry : up;
    const bool change = (sg != kNoSign) && (prev != kNoSign) && (sg != prev);
    const unsigned long long mask = __ballot(change);
    t.scan += (unsigned long long)min(64, n_c - base);
    if (mask) {
      const int f = __ffsll((long long)mask) - 1;
      *sig_f = __shfl(sg, f, 64);
      *prev_f = __shfl(prev, f, 64);
      return base + f;
    }
    carry = __shfl(sg, 63, 64);
  }
  return -1;
}

// Sign code of a point whose count E is finite: E = s + 2P has the parity of
// s, and sign(det K) = (-1)^s there (no zero or non-finite pivot).
__device__ __forceinline__ int parity_sign(int E) { return (E & 1) ? -1 : 1; }

// Spread points of (lo, hi] for the lanes (of `lanes`) from `first` on:
// every point if they fit, else lanes - first points whose last is hi.
// *valid is false for a lane without a point.
__device__ __forceinline__ int spread(int lo, int hi, int lane, int first, bool* valid, int lanes = 64) {
  const int n = hi - lo, k = lane - first, n_lanes = lanes - first;
  if (n <= n_lanes) {
    *valid = k >= 0 && k < n;
    return lo + 1 + k;
  }
  *valid = k >= 0;
  return lo + int((int64_t(n) * (k + 1)) / n_lanes);
}

// First counted point after lo whose count differs from E_a, over (lo, hi]
// with the 64 lanes; false if none.  On success (lo, hi] is narrowed to
// (point before it, it] and E_hi is its count.
__device__ __forceinline__ bool narrow_once(const double* c64, double k, const LayerRec64* L, int N, int E_a,
                                            int* lo, int* hi, int* E_hi, Tally& t) {
  const int lane = threadIdx.x & 63;
  bool valid;
  const int p = spread(*lo, *hi, lane, 0, &valid);
  const int E = valid ? count_E(c64[p], k, L, N, t, true) : E_a;
  const unsigned long long mask = __ballot(valid && E != E_a);
  if (!mask) return false;
  const int f = __ffsll((long long)mask) - 1;
  const int p_f = __shfl(p, f, 64);
  *lo = (f == 0) ? *lo : __shfl(p, f - 1, 64);
  *hi = p_f;
  *E_hi = __shfl(E, f, 64);
  return true;
}

// A bracket of the search: (lo, hi] holds the first change of E after lo,
// E(lo) = E_a, E(hi) = E_hi; the first change of sign(det K) after the start
// is at or before `bound`.
struct Bracket {
  int lo, hi, E_a, E_hi, bound;
};
constexpr int kLocated = -2;

// Round B.  The first change of sign(det K) after a (sign sig0 on [0, a]) is
// in (a, pf], pb the sampled point before pf.  Counts at a (lane 0; E_a if
// `known`), at pb (lane 1) and at 62 points of (pb, pf].  Returns kLocated
// with *br set, or the pick (-1: none) with its signs.
__device__ inline int from_sampled_bound(const double* c64, int n_c, double k, const LayerRec64* L, int N, int a,
                                         bool known, int E_a, int sig0, int pb, int pf, Bracket* br, int* sig_f,
                                         int* prev_f, Tally& t) {
  const int lane = threadIdx.x & 63;
  bool vb;
  const int pbk = (lane == 0) ? a : (lane == 1 ? pb : spread(pb, pf, lane, 2, &vb));
  if (lane < 2) vb = true;
  const int E = (lane == 0 && known) ? E_a : (vb ? count_E(c64[pbk], k, L, N, t, lane != 1 || pb != a) : 0);
  if (!known) {
    E_a = __shfl(E, 0, 64);
    if (E_a == kEvent) return walk(c64, n_c, k, L, N, a + 1, sig0, sig_f, prev_f, t);
  }
  const int E_b = __shfl(E, 1, 64);
  br->E_a = E_a;
  br->bound = pf;
  if (E_b != E_a) {
    br->lo = a;  // a change of E before the sampled point before the bound
    br->hi = pb;
    br->E_hi = E_b;
    return kLocated;
  }
  const unsigned long long mb = __ballot(lane >= 2 && vb && E != E_a);
  if (!mb) return walk(c64, n_c, k, L, N, pb + 1, sig0, sig_f, prev_f, t);
  const int f2 = __ffsll((long long)mb) - 1;
  br->hi = __shfl(pbk, f2, 64);
  br->lo = __shfl(pbk, f2 - 1, 64);
  br->E_hi = __shfl(E, f2, 64);
  return kLocated;
}

// From a bracket to the pick: narrowing to one grid step, the sign there
// (the parity of E), and the search after a change of E that leaves the
// sign unchanged (a mode and a pole, or two modes, in one step).  Returns the
// pick (-1: none) with its signs.
__device__ inline int finish(const double* c64, int n_c, double k, const LayerRec64* L, int N, int sig0, Bracket br,
                             int* sig_f, int* prev_f, Tally& t) {
  const int n = n_c - 1;
  int lo = br.lo, hi = br.hi, E_a = br.E_a, E_hi = br.E_hi;
  const int bound = br.bound;
  for (;;) {
    // hi's count differed before and is deterministic, so narrowing always
    // succeeds; walking from lo + 1 (predecessor sign sig0) is the fallback
    // that needs no such argument
    while (hi > lo + 1)
      if (!narrow_once(c64, k, L, N, E_a, &lo, &hi, &E_hi, t))
        return walk(c64, n_c, k, L, N, lo + 1, sig0, sig_f, prev_f, t);
    int sg;
    if (E_hi == kEvent) {
      sg = det_sign<double, false>(c64[hi], k, L, N, nullptr);
      ++t.check;
    } else {
      sg = parity_sign(E_hi);
    }
    if (sg != sig0) {
      *sig_f = sg;
      *prev_f = sig0;
      return hi;
    }
    if (E_hi == kEvent) return walk(c64, n_c, k, L, N, hi + 1, sig0, sig_f, prev_f, t);
    E_a = E_hi;
    lo = hi;
    hi = bound;
    if (hi <= lo || !narrow_once(c64, k, L, N, E_a, &lo, &hi, &E_hi, t)) {
      // with bound < n the sampled sign proves a change in (lo, bound]
      if (bound < n) return walk(c64, n_c, k, L, N, lo + 1, sig0, sig_f, prev_f, t);
      return -1;
    }
  }
}

// The pick of one wavelength (-1: none), with the determinant signs at it and
// at its predecessor.  pred >= 1 predicts the pick (from the previous
// wavelengths of the same model), or is -1.
//   P. With a prediction: counts at c_test[0] (lane 0), at the grid point w0
//      before a window of 62 consecutive grid points around the prediction
//      (lane 1), and at the window's points.  E(w0) = E(c_test[0]) proves no
//      change of E up to w0, and the first window point whose count differs
//      is then the first change of E.  If E changes before w0 the counts
//      narrow (0, w0]; if it changes in neither, the search goes on after
//      the window (A, B).
//   A. Determinant signs at the start point (lane 0) and 63 spread grid
//      points after it.  A sampled sign that differs from the start's bounds
//      the pick from above, so the counts that follow stay at velocities
//      near it, where a layer needs few sublayers (their number grows with
//      c).
//   B. Counts at the start point, at the sampled point before that bound,
//      and at 62 points between the two sampled points; then narrowing on E.
// With no sampled sign different (no change, or an even number of changes
// between samples), the counts search the rest of the grid.
__device__ inline int search(const double* c64, int n_c, double k, const LayerRec64* L, int N, int pred,
                             int* sig_f, int* prev_f, Tally& t) {
  const int lane = threadIdx.x & 63;
  const int n = n_c - 1;
  int a = 0;         // no change of sign(det K) in [0, a]
  int E_a = 0;       // E(a), once known
  int sig0 = 0;      // sign(det K) on [0, a], once known
  bool known = false;
  bool located = false;  // (lo, hi] holds the first change of E after lo
  int bound = n, lo = 0, hi = 0, E_hi = 0;
  if (pred >= 1 && n >= 64) {
    // P
    const int w0 = max(0, min(pred - 32, n - 62));
    const int p = (lane == 0) ? 0 : w0 + lane - 1;  // lanes 2..63: w0 + 1 .. w0 + 62 <= n
    const int E = count_E(c64[p], k, L, N, t, lane != 1 || w0 > 0);
    E_a = __shfl(E, 0, 64);
    if (E_a == kEvent) {
      sig0 = det_sign<double, false>(c64[0], k, L, N, nullptr);
      ++t.check;
      return walk(c64, n_c, k, L, N, 1, sig0, sig_f, prev_f, t);
    }
    sig0 = parity_sign(E_a);
    known = true;
    const int E_w = __shfl(E, 1, 64);
    if (E_w != E_a) {  // a change of E in (0, w0]
      hi = w0;
      E_hi = E_w;
      located = true;
    } else {
      const unsigned long long m = __ballot(lane >= 2 && E != E_a);
      if (m) {
        const int f = __ffsll((long long)m) - 1;
        hi = __shfl(p, f, 64);
        lo = __shfl(p, f - 1, 64);
        E_hi = __shfl(E, f, 64);
        located = true;
      } else {
        a = w0 + 62;  // no change up to the window's end
      }
    }
  }
  if (!located) {
    // A
    bool va;
    const int pa = (lane == 0) ? a : spread(a, n, lane, 1, &va);
    if (lane == 0) va = true;
    const int sa =
        (lane == 0 && known) ? sig0 : (va ? det_sign<double, false>(c64[pa], k, L, N, nullptr) : kNoSign);
    t.check += (unsigned long long)((known ? 0 : 1) + min(63, n - a));
    if (!known) {
      sig0 = __shfl(sa, 0, 64);
      if (sig0 != 1 && sig0 != -1) return walk(c64, n_c, k, L, N, 1, sig0, sig_f, prev_f, t);
    }
    const unsigned long long ma = __ballot(lane > 0 && va && sa != sig0);
    if (ma) {
      // B: the first change of sign(det K) after a is in (a, p_f]
      const int f = __ffsll((long long)ma) - 1;
      const int pf = __shfl(pa, f, 64), pb = __shfl(pa, f - 1, 64);
      Bracket br;
      const int r = from_sampled_bound(c64, n_c, k, L, N, a, known, E_a, sig0, pb, pf, &br, sig_f, prev_f, t);
      if (r != kLocated) return r;
      lo = br.lo;
      hi = br.hi;
      E_a = br.E_a;
      E_hi = br.E_hi;
      bound = br.bound;
    } else {
      // no sampled sign differs: counts over the rest of the grid
      bool v0;
      const int p0 = (lane == 0) ? a : spread(a, n, lane, 1, &v0);
      if (lane == 0) v0 = true;
      const int E0 = (lane == 0 && known) ? E_a : (v0 ? count_E(c64[p0], k, L, N, t, true) : 0);
      if (!known) {
        E_a = __shfl(E0, 0, 64);
        if (E_a == kEvent) return walk(c64, n_c, k, L, N, a + 1, sig0, sig_f, prev_f, t);
      }
      const unsigned long long m0 = __ballot(lane > 0 && v0 && E0 != E_a);
      if (!m0) return -1;  // no change of E after a: sign(det K) is constant
      const int f = __ffsll((long long)m0) - 1;
      hi = __shfl(p0, f, 64);
      lo = __shfl(p0, f - 1, 64);
      E_hi = __shfl(E0, f, 64);
    }
  }
  return finish(c64, n_c, k, L, N, sig0, Bracket{lo, hi, E_a, E_hi, bound}, sig_f, prev_f, t);
}

}  // namespace inertia
}  // namespace masw
