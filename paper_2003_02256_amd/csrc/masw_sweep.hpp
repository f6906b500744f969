// The persistent early-exit sweep of Algorithm 1 (FP64, or FP32 with FP64
// re-check), shared by the batch launch and the serving tick: items,
// rounds, shared sweeps, the split path's certificate, refinement and
// outputs.  A header so that the FP64 and the split batch kernels are built
// in translation units of their own, each with the placement of FP64
// polynomial coefficients that suits it (MASW_COEFF_POLICY,
// masw_special.hpp): masw_kernels.hip instantiates the FP64 kernels and the
// serving tick, masw_sweep_split.hip the split kernels.
//
// Work decomposition.  An item is one (model, wavelength).  A workgroup of G
// wavefronts takes one item at a time from a global atomic queue ordered
// longest-expected-first, and walks the c grid in rounds of G*64 consecutive
// velocities, one velocity per lane.  Each round ends with a wavefront ballot
// of "my sign differs from my predecessor's" and a cross-wavefront minimum in
// LDS, so the first sign change is known after the round and the item stops
// (Algorithm 1's early exit; the paper's GPU design evaluated every (lambda, c)
// instead, Section 2.3).  G is chosen by the host: 1 when there are many more
// items than wavefront slots, up to 16 when a few deep items must fill the chip.
// When items are few, the deepest of them would still finish long after the
// rest: those items run as shared sweeps, whose rounds any workgroup that
// finds the queue empty may claim and evaluate, while the owning workgroup
// resolves the rounds in grid order.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "masw_inertia.hpp"
#include "masw_internal.hpp"
#include "masw_math.hpp"
#include "masw_pick.hpp"

namespace masw {

// ------------------------------------------------------------ utilities --
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// First sign change in one round of G*64 consecutive positions, one per
// thread (position = round base + threadIdx.x).  `prev0` is the sign of the
// position before the round (kNoSign if none).  A position whose predecessor
// has no sign never counts as a change.  Returns the uniform offset in the
// round of the first change, or -1; *carry receives the last thread's sign.
// *sig_at / *prev_at receive the signs at the change (for NaN reporting).
template <int G>
__device__ __forceinline__ int round_first_change(int sg, int prev0, int* s_last, int* s_first,
                                                  int* s_pair, int* carry, int* sig_at,
                                                  int* prev_at) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int up = __shfl_up(sg, 1, 64);
  if (lane == 63) s_last[wave] = sg;
  __syncthreads();
  const int prev = (lane == 0) ? (wave == 0 ? prev0 : s_last[wave - 1]) : up;
  const bool change = (sg != kNoSign) && (prev != kNoSign) && (sg != prev);
  const unsigned long long mask = __ballot(change);
  if (lane == 0) s_first[wave] = mask ? (__ffsll((long long)mask) - 1) : 64;
  __syncthreads();
  int first = -1;
#pragma unroll
  for (int w = 0; w < G; ++w) {
    const int f = s_first[w];
    if (first < 0 && f < 64) first = w * 64 + f;
  }
  if (first >= 0 && (int)threadIdx.x == first) {
    s_pair[0] = sg;
    s_pair[1] = prev;
  }
  *carry = s_last[G - 1];
  __syncthreads();
  if (first >= 0) {
    *sig_at = s_pair[0];
    *prev_at = s_pair[1];
  }
  __syncthreads();
  return first;
}

// Sweep code of a grid point in the FP32 sweep: the determinant's sign code,
// plus 4 when an odd number of layer denominators are negative.  The parity
// flips where c crosses a pole of det K, so a pole crossing is a candidate
// for the FP64 check even where FP32 gets the determinant's sign wrong next to
// the pole (a zero and a pole within a grid step or two, on both sides of
// which FP32 would otherwise see the same sign).
__device__ __forceinline__ int sweep_code32(float c, float k, const LayerRec32* L, int N) {
  int odd;
  const int sg = det_sign_parity<float>(c, k, L, N, &odd);
  return sg + 4 * odd;
}

// The determinant's sign code of a sweep code (kNoSign stays kNoSign).
__device__ __forceinline__ int code_sign(int code) { return (code == kNoSign || code < 3) ? code : code - 4; }

// --------------------------------------------------------------- sweep --
enum { kModeFP64 = 0, kModeSplit = 1 };

template <int G>
struct SweepShared {
  int item;
  int last[G];
  int first[G];
  int pair[2];
  int check[8];
  int coop[6];
};

struct WorkCount {
  unsigned long long sweep = 0, check = 0, refine = 0, useful = 0, helper = 0;
};

// Everything uniform about one item.
struct ItemRef {
  int N, n_c;
  int n_real;  // leading grid points below the half-space's S velocity (the FP32 sweep's extent)
  double k64;
  const double* c64;
  const float* c32;
  const LayerRec64* L64;
  const LayerRec32* L32;
};

// Extent of a sweep in precision T: the whole grid in FP64; in FP32 the
// points below the half-space's S velocity, where inertia counts certify it.
// FP32 grid point i: the staged copy, or (c32 null: a fused launch) the FP64
// value rounded here, which is the value the staging stores.
__device__ __forceinline__ float c32_at(const ItemRef& r, int i) { return r.c32 ? r.c32[i] : float(r.c64[i]); }

template <typename T>
__device__ __forceinline__ int sweep_len(const ItemRef& r) {
  return sizeof(T) == 8 ? r.n_c : r.n_real;
}

template <int G>
__device__ __forceinline__ void write_missing(const ItemOut& o, int status) {
  write_no_pick(o, status, threadIdx.x == 0);
}

// ------------------------------------------------- shared (cooperative) sweep --
// Cross-workgroup state lives in HBM and is read and written with
// agent-scope atomics only: the L2 caches of the XCDs are not coherent with
// each other for plain accesses.
__device__ __forceinline__ int ld_agent(int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(int32_t* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_agent(uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int kCoopStall = -2;          // a shared sweep gave up waiting (never expected)
constexpr int kCoopMaxPolls = 1 << 20;  // polls of one round summary (~2 s) before giving up
constexpr int kJoinIdle = 32;           // fruitless searches before a joining workgroup leaves

// Summary of one evaluated round, published as a single 64-bit word so that
// no ordering between stores is needed: bit 63 set once published, bits
// 32..47 the first change inside the round plus one (0: none), bytes 0..3
// the sign codes at the round's first and last positions, at the change and
// just before it.
struct RoundSum {
  int s0, sl, sa, pa, f;
};

__device__ __forceinline__ uint64_t pack_round(int s0, int sl, int sa, int pa, int f) {
  return (1ull << 63) | (uint64_t(uint32_t(f + 1) & 0xffffu) << 32) | (uint64_t(uint8_t(pa)) << 24) |
         (uint64_t(uint8_t(sa)) << 16) | (uint64_t(uint8_t(sl)) << 8) | uint64_t(uint8_t(s0));
}

__device__ __forceinline__ RoundSum unpack_round(uint64_t w) {
  RoundSum u;
  u.s0 = int8_t(w & 0xff);
  u.sl = int8_t((w >> 8) & 0xff);
  u.sa = int8_t((w >> 16) & 0xff);
  u.pa = int8_t((w >> 24) & 0xff);
  u.f = int((w >> 32) & 0xffff) - 1;
  return u;
}

// Where one workgroup's shared sweep keeps its state (ci null: not shared).
struct CoopRef {
  CoopItem* ci;
  uint64_t* sum;     // the item's round summaries
  int32_t* active;   // this workgroup's slot in the list of open shared sweeps
  int item;          // queue position
};
constexpr CoopRef kNoCoop{nullptr, nullptr, nullptr, 0};

// Round rd of an item: positions rd*P .. rd*P+P-1, the first one with no
// predecessor.  Returns the first change inside the round (uniform); *sl is
// the sign at the last position (uniform), *sa/*pa the signs at the change
// and before it, and thread 0's *s0 the sign at the first position.
template <typename T, int G>
__device__ __forceinline__ int eval_round(const ItemRef& r, int rd, SweepShared<G>& sh, int* s0, int* sl,
                                          int* sa, int* pa) {
  constexpr int P = 64 * G;
  const int i = rd * P + int(threadIdx.x);
  int sg = kNoSign;
  if (i < sweep_len<T>(r)) {
    if constexpr (sizeof(T) == 8)
      sg = det_sign<double, false>(r.c64[i], r.k64, r.L64, r.N, nullptr);
    else
      sg = sweep_code32(c32_at(r, i), float(r.k64), r.L32, r.N);
  }
  *s0 = sg;
  return round_first_change<G>(sg, kNoSign, sh.last, sh.first, sh.pair, sl, sa, pa);
}

// The owner's side of a shared sweep over the whole grid: the same first
// change, and the same signs at it, as a sweep by this workgroup alone
// (Algorithm 1's scan), while workgroups that join may evaluate any of the
// rounds.  Thread 0 claims rounds one ahead (the claim's latency overlaps the
// round), applies each round's summary in grid order with the carried sign
// of the previous round, and waits only when it has no round of its own left.
// Returns the change's position, -1 if the grid has none, or kCoopStall.
template <typename T, int G>
__device__ int coop_sweep(const ItemRef& r, const CoopRef& co, SweepShared<G>& sh, WorkCount& wc,
                          Counters* cnt, int* sig, int* prev) {
  constexpr int P = 64 * G;
  const int tid = threadIdx.x;
  const int n_sw = sweep_len<T>(r);
  const int n_rounds = (n_sw + P - 1) / P;
  int claim = 0, resolved = 0, carry = kNoSign, found = -1, fs = 0, fp = 0;
  int stop = 0x7fffffff;
  bool done = false;
  if (tid == 0) {
    st_agent(&co.ci->rounds, n_rounds);
    st_agent(co.active, co.item);
    claim = atomicAdd(&co.ci->next, 1);
  }
  for (;;) {
    if (tid == 0) {
      sh.coop[0] = claim;
      sh.coop[1] = stop;
    }
    __syncthreads();
    const int rd = sh.coop[0];
    const bool eval = rd < n_rounds && rd <= sh.coop[1];
    __syncthreads();
    int nclaim = 0x7fffffff, nstop = stop;
    if (eval) {
      if (tid == 0) {
        nclaim = atomicAdd(&co.ci->next, 1);
        nstop = ld_agent(&co.ci->stop);
      }
      int s0, sl, sa = 0, pa = 0;
      const int f = eval_round<T, G>(r, rd, sh, &s0, &sl, &sa, &pa);
      wc.sweep += (unsigned long long)min(P, n_sw - rd * P);
      if (tid == 0) {
        if (f >= 0) {
          atomicMin(&co.ci->stop, rd);
          stop = min(stop, rd);
        }
        if (rd == resolved) {  // next in grid order: apply it here
          if (rd > 0 && carry != kNoSign && s0 != kNoSign && s0 != carry) {
            found = rd * P, fs = s0, fp = carry, done = true;
          } else if (f >= 0) {
            found = rd * P + f, fs = sa, fp = pa, done = true;
          } else {
            carry = sl;
            ++resolved;
          }
        } else {
          st_agent(&co.sum[rd], pack_round(s0, sl, sa, pa, f));
        }
      }
    } else if (tid == 0) {
      nstop = ld_agent(&co.ci->stop);
    }
    if (tid == 0) {
      stop = min(stop, nstop);
      const int bound = stop >= n_rounds ? n_rounds : stop + 1;
      // Rounds below the owner's next claim that are not resolved yet were
      // claimed by joining workgroups (or published above).
      while (!done && resolved < bound && resolved < nclaim) {
        uint64_t w = ld_agent(&co.sum[resolved]);
        if (!(w >> 63)) {
          if (nclaim < bound) break;  // evaluate the own next round first
          // Bounded wait; after any stall in the launch, no further waiting.
          const int max_polls = ld_agent(reinterpret_cast<int32_t*>(&cnt->coop_stall)) ? 0 : kCoopMaxPolls;
          int polls = 0;
          while (!((w = ld_agent(&co.sum[resolved])) >> 63) && polls < max_polls) {
            ++polls;
            __builtin_amdgcn_s_sleep(2);
          }
          if (!(w >> 63)) {
            atomicAdd(&cnt->coop_stall, 1u);
            found = kCoopStall, done = true;
            break;
          }
        }
        const RoundSum u = unpack_round(w);
        const int q = resolved;
        if (q > 0 && carry != kNoSign && u.s0 != kNoSign && u.s0 != carry) {
          found = q * P, fs = u.s0, fp = carry, done = true;
        } else if (u.f >= 0) {
          found = q * P + u.f, fs = u.sa, fp = u.pa, done = true;
        } else {
          carry = u.sl;
          ++resolved;
        }
      }
      if (!done && resolved >= n_rounds) done = true;  // no change in the grid
      if (!done && nclaim >= bound && resolved >= bound) {
        // bound < n_rounds means round `stop` holds a change, which the loop
        // above must have found; anything else is a broken invariant.
        atomicAdd(&cnt->coop_stall, 1u);
        found = kCoopStall, done = true;
      }
      if (done) {
        st_agent(&co.ci->stop, -1);  // close: joining workgroups stop claiming
        st_agent(&co.ci->rounds, -1);
        st_agent(co.active, -1);
      } else {
        st_agent(&co.ci->resolved, resolved);
      }
      sh.coop[2] = done ? 1 : 0;
      sh.coop[3] = found;
      sh.coop[4] = fs;
      sh.coop[5] = fp;
      claim = nclaim;
    }
    __syncthreads();
    if (sh.coop[2]) {
      found = sh.coop[3];
      *sig = sh.coop[4];
      *prev = sh.coop[5];
      __syncthreads();
      return found;
    }
  }
}

// Advance one item by at most `budget` sweep rounds of G*64 positions.  When
// the first sign change is known (after the FP64 re-check for the split
// path), refine it in FP64 and write the outputs through wavefront 0, then
// return true.  If the budget runs out first, save where the sweep stands
// in `st` and return false; resuming from `st` gives the same result as an
// uninterrupted run, whatever G the resumed call uses.
//
// The split path trusts FP32 signs only where FP64 certifies them.  It
// sweeps in FP32 only below the half-space's S velocity, where K is real
// symmetric and the inertia count E(c) = s + 2P of the inertia search exists
// (s: negative eigenvalues of K; P: poles below c).  E is non-decreasing in
// c and changes at every zero and every pole of det K, so equal counts at
// two points prove that sign(det K) is constant between them.  Every FP32
// candidate (a change of the sign, or of the parity of negative layer
// denominators) is re-checked in FP64 on a 64-point window, and the stretch
// FP32 passed over before the window, from the segment's origin (the grid
// start, or the last FP64-checked point), is certified by E at the window's
// first point: E = 0 there proves it at once (E is non-negative and
// non-decreasing); otherwise E at the origin must be equal.  The same
// certificate covers the stretch before the end of the FP32 sweep when FP32
// sees no change.  A failed certificate sends the item back to an FP64 walk
// from the segment's origin; the grid above the half-space's S velocity is
// walked in FP64.  So the split pick is Algorithm 1's pick in FP64 (up to
// the noise band of the FP64 signs and counts).
template <int MODE, int G>
__device__ bool run_item(const ItemRef& r, ItemState& st, int budget, SweepShared<G>& sh, WorkCount& wc,
                         const ItemOut& o, const CoopRef& co, Counters* cnt) {
  constexpr int P = 64 * G;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int n_c = r.n_c;
  int found = -1, sig_f = 0, prev_f = 0;
  int start = st.start, carry = st.carry, rounds = 0;
  bool fp64 = (MODE == kModeFP64) || st.fp64;

  if (!fp64 && r.n_real <= 0) {  // the whole grid at or above the half-space's S velocity
    fp64 = true;
    st.fp64 = 1;
  }
  if (!fp64) {
    const float k32 = float(r.k64);
    const int n32 = r.n_real;
    int seg_start = st.seg_start, seg_carry = st.seg_carry;
    bool shared = co.ci != nullptr;  // the first FP32 pass is a shared sweep
    for (;;) {
      // FP32 sweep for a candidate, from `start` (inside the segment that
      // began at seg_start, whose predecessor's FP64 sign is seg_carry).
      int cand = -1;
      if (shared) {
        shared = false;
        int s_c = 0, p_c = 0;
        cand = coop_sweep<float, G>(r, co, sh, wc, cnt, &s_c, &p_c);
        if (cand == kCoopStall) {
          st.done = 1;
          write_missing<G>(o, MASW_STATUS_INVALID);
          return true;
        }
      } else {
        for (int base = start; base < n32; base += P) {
          if (rounds == budget) {
            st.start = base;
            st.carry = carry;
            st.seg_start = seg_start;
            st.seg_carry = seg_carry;
            return false;
          }
          ++rounds;
          const int i = base + tid;
          const int sg = (i < n32) ? sweep_code32(c32_at(r, i), k32, r.L32, r.N) : kNoSign;
          int s_c, p_c;
          const int f = round_first_change<G>(sg, carry, sh.last, sh.first, sh.pair, &carry, &s_c, &p_c);
          wc.sweep += (unsigned long long)min(P, n32 - base);
          if (f >= 0) {
            cand = base + f;
            break;
          }
        }
      }
      // FP64 check by wavefront 0 while the others wait: the 64 positions
      // ws-1 .. ws+62 around a candidate (48 before it, 15 after), or, when
      // FP32 saw no change up to the end of its sweep, the last position it
      // swept (lane 0).  Lane 0 also counts E at ws - 1 when the segment's
      // origin lies before it.  The positions do not depend on the group
      // size, so neither does the outcome.
      const bool at_end = cand < 0;
      const int ws = at_end ? n32 : max(1, cand - 48);
      const int origin = (seg_carry == kNoSign) ? 0 : seg_start - 1;
      const bool certify = ws - 1 > origin;
      if (wave == 0) {
        const int i = ws - 1 + lane;
        int sg = kNoSign, odd = 0, E = 0;
        bool bounded = true;
        if (at_end ? lane == 0 : i < n_c) sg = inertia::det_sign_inertia(r.c64[i], r.k64, r.L64, r.N, &odd, &E, &bounded);
        int last, s_c = 0, p_c = 0;
        const int f = at_end ? -1 : wave_first_change(sg, &s_c, &p_c, &last);
        if (lane == 63) sh.check[6] = (sg == kNoSign) ? kNoSign : sg + 4 * odd;  // sweep code of the window's end
        if (lane == 0) {
          sh.check[0] = f;
          sh.check[1] = at_end ? kNoSign : last;
          sh.check[2] = s_c;
          sh.check[3] = p_c;
          sh.check[4] = sg;  // FP64 sign at ws - 1
          sh.check[5] = E;  // inertia of the pivots at ws - 1 (E there if `bounded`)
          sh.check[7] = bounded ? 1 : 0;
        }
      }
      __syncthreads();
      const int f = sh.check[0];
      const int last = sh.check[1];
      const int first64 = sh.check[4];
      int E_p = sh.check[5];
      const bool bounded = sh.check[7] != 0;
      const int last_code = sh.check[6];
      sig_f = sh.check[2];
      prev_f = sh.check[3];
      __syncthreads();
      wc.check += at_end ? 1ull : (unsigned long long)min(64, n_c - (ws - 1));
      bool ok = seg_carry == kNoSign || first64 == seg_carry;
      if (ok && certify && !(bounded && E_p == 0)) {
        // Rare: a layer whose poles need counting at ws - 1, or a change of E
        // before it (one FP32 did not see, or changes that cancel within one
        // grid step).  The full counts at ws - 1 and at the origin, by
        // thread 0.
        if (tid == 0) {
          int e = E_p;
          if (e != inertia::kEvent && !bounded) {
            bool pok = true;
            const int P = inertia::poles_below(r.c64[ws - 1], r.k64, r.L64, r.N, &pok);
            e = pok ? e + 2 * P : inertia::kEvent;
          }
          if (e != 0 && e != inertia::kEvent)
            e = (inertia::count_E_split(r.c64[origin], r.k64, r.L64, r.N) == e) ? 0 : inertia::kEvent;
          sh.check[5] = e;
        }
        __syncthreads();
        E_p = sh.check[5];
        __syncthreads();
        ok = E_p == 0;
        wc.check += 1ull;
      }
      if (!ok) {
        // FP32 may have missed a change in [seg_start, ws - 1]: continue in FP64.
        fp64 = true;
        st.fp64 = 1;
        start = seg_start;
        carry = seg_carry;
        break;
      }
      if (at_end) {
        // no change below n32; the rest of the grid, at or above the
        // half-space's S velocity, is walked in FP64
        if (n32 < n_c) {
          fp64 = true;
          st.fp64 = 1;
          start = n32;
          carry = first64;
        }
        break;
      }
      if (f >= 0) {
        found = ws - 1 + f;
        break;
      }
      // Rejected: a new segment begins after the window, from the FP64 sign
      // of its last position.  A window that reached the end of the grid
      // leaves nothing to search; one that reached n32 leaves an FP64 walk.
      start = ws + 63;
      if (start >= n_c) break;
      seg_carry = last;
      carry = last_code;
      seg_start = start;
      if (start >= n32) {
        fp64 = true;
        st.fp64 = 1;
        carry = last;
        break;
      }
    }
  }
  if (fp64 && MODE == kModeFP64 && co.ci) {
    found = coop_sweep<double, G>(r, co, sh, wc, cnt, &sig_f, &prev_f);
    if (found == kCoopStall) {
      st.done = 1;
      write_missing<G>(o, MASW_STATUS_INVALID);
      return true;
    }
  } else if (fp64) {
    for (int base = start; base < n_c; base += P) {
      if (rounds == budget) {
        st.start = base;
        st.carry = carry;
        return false;
      }
      ++rounds;
      const int i = base + tid;
      const int sg = (i < n_c) ? det_sign<double, false>(r.c64[i], r.k64, r.L64, r.N, nullptr) : kNoSign;
      const int f = round_first_change<G>(sg, carry, sh.last, sh.first, sh.pair, &carry, &sig_f, &prev_f);
      wc.sweep += (unsigned long long)min(P, n_c - base);
      if (f >= 0) {
        found = base + f;
        break;
      }
    }
  }
  st.done = 1;

  if (found < 0) {
    write_missing<G>(o, MASW_STATUS_NOT_FOUND);
    wc.useful += (unsigned long long)n_c;
    return true;
  }
  wc.useful += (unsigned long long)(found + 1);

  // Refinement and output by wavefront 0 alone; the others go on to the
  // next barrier.  One wavefront at a time on a SIMD finishes these few
  // rounds sooner than the whole group sharing the SIMDs would.
  if (wave == 0) wc.refine += refine_and_write(o, r.c64, r.k64, r.L64, r.N, found, sig_f, prev_f);
  return true;
}

// A workgroup's work counts at its end: into its own row of wg (the host
// sums the rows), or with atomics on the counters (serving ticks).
__device__ __forceinline__ void flush_counts(Counters* c, unsigned long long* wg, const WorkCount& wc) {
  if (threadIdx.x != 0) return;
  if (wg) {  // this workgroup's row
    unsigned long long* row = wg + size_t(blockIdx.x) * kWgCounts;
    row[0] = wc.sweep;
    row[1] = wc.check;
    row[2] = wc.refine;
    row[3] = wc.useful;
    row[4] = wc.helper;
    row[5] = row[6] = row[7] = 0ull;
    return;
  }
  atomicAdd(&c->sweep, wc.sweep);
  atomicAdd(&c->check, wc.check);
  atomicAdd(&c->refine, wc.refine);
  atomicAdd(&c->useful, wc.useful);
  if (wc.helper) atomicAdd(&c->helper, wc.helper);
}

// The uniform description of the item at queue position `it`; *g_out is its
// wavelength and *m_out (if given) its model.
__device__ __forceinline__ ItemRef item_ref(const SweepArgs& a, int it, int* g_out, int* m_out = nullptr) {
  const int g = uniform(a.order[it]);
  const int m = uniform(a.lam_model[g]);
  if (m_out) *m_out = m;
  const ModelDesc d = a.models[m];
  ItemRef r;
  r.N = uniform(d.n_layers);
  r.n_c = uniform(d.n_c);
  r.n_real = uniform(d.n_real);
  r.k64 = a.lam_k[g];
  r.c64 = a.c64 + uniform(d.c_base);
  r.c32 = a.c32 + uniform(d.c_base);
  r.L64 = a.layers64 + uniform(d.layer_base);
  r.L32 = a.layers32 + uniform(d.layer_base);
  *g_out = g;
  return r;
}

// A workgroup that finds the queue empty joins the shared sweeps still open:
// wavefront 0 looks through the owners' slots (starting at its own, so that
// joiners spread out) for the sweep with the fewest rounds in flight beyond
// its owner's resolution, and the workgroup claims and evaluates rounds of it
// until it runs more than coop_window rounds ahead or the sweep has seen a
// change.  It leaves when no shared sweep is open, or after kJoinIdle
// searches that found nothing to join.
template <int MODE, int G>
__device__ void join_sweeps(const SweepArgs& a, SweepShared<G>& sh, WorkCount& wc) {
  using T = typename std::conditional<MODE == kModeFP64, double, float>::type;
  constexpr int P = 64 * G;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nb = gridDim.x;
  int idle = 0;
  for (;;) {
    if (wave == 0) {
      int best = -1;
      bool open = false;
      for (int k = 0; k < nb && best < 0; k += 64) {
        int key = 0x7fffffff;  // (rounds in flight << 24) | item, for the helpable ones
        bool op = false;
        if (k + lane < nb) {
          const int it = ld_agent(&a.coop_active[(int(blockIdx.x) + k + lane) % nb]);
          if (it >= 0 && it < a.n_coop) {
            CoopItem* ci = a.coop + it;
            const int rounds = ld_agent(&ci->rounds);
            const int next = ld_agent(&ci->next);
            const int stop = ld_agent(&ci->stop);
            const int res = ld_agent(&ci->resolved);
            if (rounds > 0) {
              op = true;
              const int bound = stop >= rounds ? rounds : stop + 1;
              if (next < bound && next - res < a.coop_window) key = (max(next - res, 0) << 24) | it;
            }
          }
        }
        for (int off = 32; off > 0; off >>= 1) key = min(key, __shfl_xor(key, off, 64));
        open = open || (__ballot(op) != 0ull);
        if (key != 0x7fffffff) best = key & 0xffffff;
      }
      if (lane == 0) {
        sh.coop[0] = best;
        sh.coop[1] = open ? 1 : 0;
      }
    }
    __syncthreads();
    const int item = sh.coop[0];
    const bool open = sh.coop[1] != 0;
    __syncthreads();
    if (item < 0) {
      if (!open || ++idle > kJoinIdle) return;
      __builtin_amdgcn_s_sleep(127);
      continue;
    }
    idle = 0;
    int g;
    const ItemRef r = item_ref(a, item, &g);
    CoopItem* ci = a.coop + item;
    uint64_t* sum = a.coop_sum + size_t(item) * size_t(a.coop_stride);
    for (;;) {
      if (tid == 0) {
        const int rd = atomicAdd(&ci->next, 1);
        const int rounds = ld_agent(&ci->rounds);
        const int stop = ld_agent(&ci->stop);
        sh.coop[0] = rd;
        sh.coop[1] = (rounds > 0 && rd < rounds && rd <= stop) ? 1 : 0;
        sh.coop[2] = ld_agent(&ci->resolved);
      }
      __syncthreads();
      const int rd = sh.coop[0];
      const bool go = sh.coop[1] != 0;
      const int res = sh.coop[2];
      __syncthreads();
      if (!go) break;
      int s0, sl, sa = 0, pa = 0;
      const int f = eval_round<T, G>(r, rd, sh, &s0, &sl, &sa, &pa);
      const unsigned long long n = (unsigned long long)min(P, sweep_len<T>(r) - rd * P);
      wc.sweep += n;
      wc.helper += n;
      if (tid == 0) {
        st_agent(&sum[rd], pack_round(s0, sl, sa, pa, f));
        if (f >= 0) atomicMin(&ci->stop, rd);
      }
      if (f >= 0 || rd + 1 - res >= a.coop_window) break;
    }
  }
}

// Algorithm 2 fused into the batch launch: after an item's outputs are
// written, the workgroup counts the item off its model, and the workgroup
// that finishes the model's last wavelength reduces the model's misfit,
// mean_i |C_t,i - C_e,i| / C_e,i, in the order of misfit_kernel (256 partial
// sums, each over a stride of 256 wavelengths, then a fixed tree), so the
// result equals the separate launch's bit for bit.  Agent-scope fences order
// each item's plain output stores before its count (release) and the last
// workgroup's reads after it (acquire): the XCDs' L2 caches are not coherent
// with each other otherwise.
template <int G>
__device__ void model_finished(const SweepArgs& a, int m, SweepShared<G>& sh, double* s_mis) {
  constexpr int P = 64 * G;
  __syncthreads();  // wavefront 0 has written the item's outputs
  if (threadIdx.x == 0) {
    __threadfence();
    sh.coop[0] = atomicSub(a.model_left + m, 1);
  }
  __syncthreads();
  const bool last = sh.coop[0] == 1;
  __syncthreads();
  if (!last) return;
  __threadfence();
  const int lo = a.lambda_off[m], hi = a.lambda_off[m + 1];
  for (int v = threadIdx.x; v < 256; v += P) {
    double acc = 0.0;
    for (int i = lo + v; i < hi; i += 256) acc += ::fabs(a.out_ct[i] - a.c_e[i]) / a.c_e[i];
    s_mis[v] = acc;
  }
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    for (int v = threadIdx.x; v < w; v += P) s_mis[v] += s_mis[v + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.misfit[m] = s_mis[0] / double(hi - lo);
  __syncthreads();
}

// Batch launch: a persistent grid pulls items from the ordered queue and runs
// each to completion; items at queue positions below n_coop run as shared
// sweeps that workgroups with an empty queue join.  MISFIT: Algorithm 2 fused
// (model_finished), an instantiation of its own so that the plain sweeps
// keep their register allocation; it is held to 128 VGPRs (4 wavefronts per
// SIMD, as the plain FP64 sweeps), spilling a little outside the layer loop.
// The plain split sweeps are held to 96 VGPRs (5 wavefronts per SIMD), which
// their FP32 loop fits without spilling.
template <int MODE, int G, bool MISFIT>
__global__ __launch_bounds__(64 * G) __attribute__((amdgpu_waves_per_eu(MISFIT ? 4 : (MODE == kModeSplit ? 5 : 1))))
void sweep_kernel(SweepArgs a) {
  __shared__ SweepShared<G> sh;
  __shared__ double s_mis[MISFIT ? 256 : 1];  // fused misfit reduction
  WorkCount wc;
  constexpr int P = 64 * G;
  stamp_start(a.tstamp, 1);
  // Queue positions below gridDim.x (the launch has at most one workgroup
  // per item) are taken by workgroup index, the rest from the atomic queue:
  // a launch with no more items than workgroups makes no claim at all.
  for (int claim = 0;; ++claim) {
    int it = int(blockIdx.x);
    if (claim > 0) {
      if (int(gridDim.x) >= a.n_items) break;
      if (threadIdx.x == 0) {
        const uint32_t q = gridDim.x + atomicAdd(&a.counters->queue_head, 1u);
        sh.item = q >= uint32_t(a.n_items) ? a.n_items : int(q);
      }
      __syncthreads();
      it = uniform(sh.item);
      __syncthreads();
    }
    if (it >= a.n_items) break;

    int g, m;
    const ItemRef r = item_ref(a, it, &g, &m);
    const ItemOut o{a.out_ct + g, a.out_idx + g, a.out_status + g, a.out_cref ? a.out_cref + g : nullptr,
                    a.refine, a.refine_rel};
    if (!(r.k64 == r.k64)) {  // invalid model, grid or wavelength
      write_missing<G>(o, MASW_STATUS_INVALID);
      if constexpr (MISFIT) model_finished<G>(a, m, sh, s_mis);
      continue;
    }
    // Deeper items (earlier queue positions) take issue precedence over the
    // other workgroup on the same compute unit, shortening the launch's
    // critical path; the total work is unchanged.
    if (it < a.prio_hi) __builtin_amdgcn_s_setprio(2);
    else if (it < a.prio_mid) __builtin_amdgcn_s_setprio(1);
    else __builtin_amdgcn_s_setprio(0);
    CoopRef co{nullptr, nullptr, nullptr, it};
    if (it < a.n_coop && (r.n_c + P - 1) / P <= a.coop_stride) {
      co.ci = a.coop + it;
      co.sum = a.coop_sum + size_t(it) * size_t(a.coop_stride);
      co.active = a.coop_active + blockIdx.x;
    }
    ItemState st = item_state_init();
    run_item<MODE, G>(r, st, 0x7fffffff, sh, wc, o, co, a.counters);
    if constexpr (MISFIT) model_finished<G>(a, m, sh, s_mis);
  }
  __builtin_amdgcn_s_setprio(0);
  if (a.n_coop > 0) join_sweeps<MODE, G>(a, sh, wc);
  flush_counts(a.counters, a.wg_counts, wc);
  stamp_end(a.tstamp);
}


// A small single-model launch with the staging folded in (SweepArgs::fused):
// the workgroup of index w takes wavelength w.  It checks the raw model (as
// the staging does), writes the layer records into its LDS, checks the grid
// and counts its points below the half-space's S velocity, and computes k,
// all with the staging's arithmetic, so outputs equal those of the staged
// launch bit for bit.  A kernel of its own: its records are read from LDS,
// while the staged kernels read theirs with scalar loads.
template <int MODE>
__global__ __launch_bounds__(64 * kFusedG) void fused_sweep_kernel(SweepArgs a) {
  constexpr int G = kFusedG;
  __shared__ SweepShared<G> sh;
  __shared__ int s_below;
  extern __shared__ __attribute__((aligned(64))) unsigned char fused_lds[];
  const int N = a.fused_N, n_c = a.f_n_c, tid = threadIdx.x;
  LayerRec64* L64 = reinterpret_cast<LayerRec64*>(fused_lds);
  LayerRec32* L32 = reinterpret_cast<LayerRec32*>(fused_lds + sizeof(LayerRec64) * size_t(N + 1));
  stamp_start(a.tstamp, 0, 1);  // the job is this one launch
  if (tid == 0) s_below = 0;
  // the model: checks and records (build_model's)
  const double be_hs = a.f_beta[N];
  const double mu_ref = a.f_rho[N] * be_hs * be_hs;
  bool lok = (N >= 0) && (N <= kFusedMaxLayers);
  for (int j = tid; j <= N; j += 64 * G) {
    const double al = a.f_alpha[j], be = a.f_beta[j], rh = a.f_rho[j];
    const bool finite = (al < __builtin_inf()) && (rh < __builtin_inf());
    bool ok = finite && (be > 0.0) && (al > be) && (rh > 0.0);
    const double h = (j < N) ? a.f_h[j] : 0.0;
    if (j < N) ok = ok && (h > 0.0) && (h < __builtin_inf());
    lok = lok && ok;
    LayerRec64 r;
    r.ia2 = 1.0 / (al * al);
    r.ib2 = 1.0 / (be * be);
    r.rh = rh / mu_ref;
    r.mh = rh * be * be / mu_ref;
    r.h = h;
    r.aux = (j == N) ? mu_ref : 0.0;
    r.zb = 0.0;  // only the batch staging's work order reads it
    r.pad2 = 0.0;
    L64[j] = r;
    LayerRec32 q;
    q.ia2 = float(r.ia2);
    q.ib2 = float(r.ib2);
    q.rh = float(r.rh);
    q.mh = float(r.mh);
    q.h = float(r.h);
    q.aux = float(mu_ref);
    q.zb = 0.0f;
    q.pad2 = 0.0f;
    L32[j] = q;
  }
  // the grid: finite, > 0, strictly increasing (the staging's checks), and
  // its points below beta_hs in the arithmetic of build_model's search
  const double ib2 = 1.0 / (be_hs * be_hs);
  bool gok = true;
  int below = 0;
  for (int i = tid; i < n_c; i += 64 * G) {
    const double c = a.f_c[i];
    bool ok = (c > 0.0) && (c < __builtin_inf());
    if (i + 1 < n_c) ok = ok && (c < a.f_c[i + 1]);
    gok = gok && ok;
    below += (c * c * ib2 < 1.0) ? 1 : 0;
  }
  const int bad = __syncthreads_or((lok && gok) ? 0 : 1);
  for (int o = 32; o > 0; o >>= 1) below += __shfl_xor(below, o, 64);
  if ((tid & 63) == 0 && below) atomicAdd(&s_below, below);
  __syncthreads();
  const int n_real = s_below;
  const int g = int(blockIdx.x);
  const double lam = a.f_lambda[g];
  const bool ok = !bad && (lam > 0.0) && (lam < __builtin_inf());
  ItemRef r;
  r.N = bad ? 0 : N;
  r.n_c = n_c;
  r.n_real = bad ? 0 : n_real;
  r.k64 = ok ? (2.0 * M_PI / lam) : __builtin_nan("");
  r.c64 = a.f_c;
  r.c32 = nullptr;  // rounded from c64 where read
  r.L64 = L64;
  r.L32 = L32;
  const ItemOut o{a.out_ct + g, a.out_idx + g, a.out_status + g, a.out_cref ? a.out_cref + g : nullptr, a.refine,
                  a.refine_rel};
  WorkCount wc;
  if (!ok) {
    write_missing<G>(o, MASW_STATUS_INVALID);
  } else {
    ItemState st = item_state_init();
    run_item<MODE, G>(r, st, 0x7fffffff, sh, wc, o, kNoCoop, a.counters);
  }
  flush_counts(a.counters, a.wg_counts, wc);
  stamp_end(a.tstamp);
}

// Dynamic LDS of a fused launch: the model's FP64 and FP32 records.
inline size_t fused_lds_bytes(int N) { return (sizeof(LayerRec64) + sizeof(LayerRec32)) * size_t(N + 1); }

// The split kernels (masw_sweep_split.hip): sweep_kernel<kModeSplit, G,
// misfit> for G in 1, 2, 4, 8, 16, or null; fused_sweep_kernel<kModeSplit>.
const void* split_sweep_symbol(int G, bool misfit);
const void* split_fused_symbol();

}  // namespace masw
