// HIP kernels for gfx950: staging/precompute, work ordering, the persistent
// early-exit sweep (FP64, or FP32 with FP64 re-check), FP64 root refinement,
// and the full-grid sign map.
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
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
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

// ------------------------------------------------------------- staging --
// Validation and per-layer records of model m by one wavefront, one layer
// per lane.  With a.layer_off == nullptr the batch is a single model of
// single_N layers and single_W wavelengths.
__device__ void build_model(const PrepArgs& a, int m, int single_N, int single_W) {
  const int lane = threadIdx.x & 63;
  const int lo = a.layer_off ? a.layer_off[m] : 0;
  const int hi = a.layer_off ? a.layer_off[m + 1] : single_N;
  const int N = hi - lo;
  const int rec0 = lo + m;  // records and alpha/beta/rho entries of model m
  bool ok = (N >= 0) && (N <= MASW_MAX_LAYERS);
  if (ok) {
    bool lok = true;
    for (int j = lane; j <= N; j += 64) {
      const double al = a.alpha[rec0 + j], be = a.beta[rec0 + j], rh = a.rho[rec0 + j];
      const bool finite = (al < __builtin_inf()) && (rh < __builtin_inf());
      lok = lok && finite && (be > 0.0) && (al > be) && (rh > 0.0);
      if (j < N) {
        const double h = a.h[lo + j];
        lok = lok && (h > 0.0) && (h < __builtin_inf());
      }
    }
    ok = __ballot(!lok) == 0ull;
  }
  // Grid points below the half-space's S velocity: the first c with
  // c^2 / beta_hs^2 >= 1, in the arithmetic of the inertia count's test (the
  // grid rises; a grid that does not fails its own checks).  A 64-way search
  // by the wavefront: each round tests 64 evenly spaced points of [lo, hi),
  // whose outcomes form a prefix, and keeps the gap after the last point
  // below; two or three dependent loads for the usual grids instead of a
  // binary search's ten to fifteen.
  int n_real = 0;
  if (ok) {
    const double be = a.beta[rec0 + N];
    const double ib2 = 1.0 / (be * be);
    int lo = 0, hi = a.n_c;  // n_real in [lo, hi]
    while (lo < hi) {
      const int step = (hi - lo + 63) / 64;
      const int i = lo + lane * step;
      bool below = false;
      if (i < hi) {
        const double c = a.c_in[i];
        below = c * c * ib2 < 1.0;
      }
      const int t = __popcll(__ballot(below));
      if (t == 0) {
        hi = lo;
      } else {
        const int last = lo + (t - 1) * step;
        hi = min(hi, last + step);
        lo = last + 1;
      }
    }
    n_real = lo;
  }
  if (lane == 0) {
    ModelDesc d;
    d.n_layers = ok ? N : 0;
    d.layer_base = rec0;
    d.c_base = 0;
    d.n_c = a.n_c;
    d.lam_base = a.lambda_off ? a.lambda_off[m] : 0;
    d.n_lam = a.lambda_off ? (a.lambda_off[m + 1] - a.lambda_off[m]) : single_W;
    d.valid = ok ? 1 : 0;
    d.n_real = n_real;
    a.models[m] = d;
    if (a.model_left) {
      a.model_left[m] = d.n_lam;
      if (d.n_lam == 0) a.misfit[m] = __builtin_nan("");
    }
  }
  if (!ok) return;
  const double mu_ref = a.rho[rec0 + N] * a.beta[rec0 + N] * a.beta[rec0 + N];
  double z0 = 0.0;  // depth of the top of this 64-layer chunk
  for (int j0 = 0; j0 <= N; j0 += 64) {
    const int j = j0 + lane;
    // depth of each layer's bottom: inclusive prefix sum over the chunk
    double z = (j < N) ? a.h[lo + j] : 0.0;
    for (int off = 1; off < 64; off <<= 1) {
      const double up = __shfl_up(z, off, 64);
      if (lane >= off) z += up;
    }
    z += z0;
    z0 = __shfl(z, 63, 64);
    if (j > N) continue;
    const double al = a.alpha[rec0 + j], be = a.beta[rec0 + j], rh = a.rho[rec0 + j];
    LayerRec64 r;
    r.ia2 = 1.0 / (al * al);
    r.ib2 = 1.0 / (be * be);
    r.rh = rh / mu_ref;
    r.mh = rh * be * be / mu_ref;
    r.h = (j < N) ? a.h[lo + j] : 0.0;
    r.aux = (j == N) ? mu_ref : 0.0;
    r.zb = z;
    r.pad2 = 0.0;
    a.layers64[rec0 + j] = r;
    LayerRec32 q;
    q.ia2 = float(r.ia2);
    q.ib2 = float(r.ib2);
    q.rh = float(r.rh);
    q.mh = float(r.mh);
    q.h = float(r.h);
    q.aux = float(mu_ref);
    q.zb = float(z);
    q.pad2 = 0.0f;
    a.layers32[rec0 + j] = q;
  }
}

// The front of the staging, one launch:
//  * blocks [0, nb_grid): grid checks (finite, > 0, strictly increasing) and
//    the FP32 copy; each block writes its own flag, so nothing needs clearing
//    first;
//  * the next nb_models blocks: validation and layer records, one wavefront
//    per model;
//  * the last nb_clear blocks: the counters and the shared-sweep state.
__global__ __launch_bounds__(kPrepThreads) void prep_front_kernel(PrepArgs a, CoopInitArgs ci, int nb_grid,
                                                                  int nb_models, int nb_clear, int single_N,
                                                                  int single_W) {
  const int b = blockIdx.x;
  if (b < nb_grid) {
    const int i = b * kPrepThreads + int(threadIdx.x);
    int bad = 0;
    if (i < a.n_c) {
      const double c = a.c_in[i];
      if (a.c64 != a.c_in) a.c64[i] = c;
      a.c32[i] = float(c);
      bool ok = (c > 0.0) && (c < __builtin_inf());
      if (i + 1 < a.n_c) ok = ok && (c < a.c_in[i + 1]);
      bad = ok ? 0 : 1;
    }
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) a.grid_flags[b] = bad ? 1u : 0u;
    return;
  }
  if (b < nb_grid + nb_models) {
    const int m = (b - nb_grid) * (kPrepThreads / 64) + int(threadIdx.x >> 6);
    if (m < a.n_models) build_model(a, m, single_N, single_W);
    return;
  }
  const size_t t = size_t(b - nb_grid - nb_models) * kPrepThreads + threadIdx.x;
  const size_t stride = size_t(nb_clear) * kPrepThreads;
  uint32_t* cw = reinterpret_cast<uint32_t*>(a.counters);
  for (size_t i = t; i < sizeof(Counters) / sizeof(uint32_t); i += stride) cw[i] = 0u;
  for (size_t i = t; i < size_t(ci.n_coop); i += stride) ci.coop[i] = CoopItem{0, 0x7fffffff, 0, 0};
  for (size_t i = t; i < ci.n_sum; i += stride) ci.coop_sum[i] = 0ull;
  for (size_t i = t; i < size_t(ci.n_active); i += stride) ci.coop_active[i] = -1;
}

// One thread per wavelength: k, its model, and the work-order key.  The
// expected search depth is the grid index of 0.9 beta at depth lambda/3 (a
// Rayleigh wave samples roughly the top third of a wavelength); the cost is
// that depth times N+1.  Longer wavelengths see faster material and search
// deeper (Section 3.2's observation behind the modular partition), so the key
// orders them first.  The key only orders the work, so the grid index is
// interpolated between kBuckets grid samples staged in LDS.  A launch of one
// block (at most kLamBlock wavelengths) also finishes the counting sort in
// LDS; otherwise the histogram goes to the counters for order_scan_kernel and
// order_scatter_kernel.
struct LambdaShared {
  uint32_t hist[kBuckets];
  uint32_t scan[kBuckets];
  double c[kBuckets];
};

// The wavelength part of the staging for the wavelengths of this block;
// `bad` is the grid's validity (uniform).  LDS arrays in `ls`.
__device__ void stage_lambdas(const PrepArgs& a, int bad, LambdaShared& ls) {
  uint32_t* s_hist = ls.hist;
  uint32_t* s_scan = ls.scan;
  double* s_c = ls.c;
  const int t = threadIdx.x;
  const int ns = min(kBuckets, a.n_c);  // grid samples: c at index (s * (n_c - 1)) / (ns - 1)
  for (int i = t; i < kBuckets; i += blockDim.x) {
    s_hist[i] = 0u;
    if (i < ns) s_c[i] = a.c64[ns > 1 ? int((int64_t(i) * (a.n_c - 1)) / (ns - 1)) : 0];
  }
  __syncthreads();
  if (blockIdx.x == 0 && t == 0) a.counters->grid_bad = bad ? 1u : 0u;
  const int g = blockIdx.x * blockDim.x + t;
  int key = 0;
  uint32_t rank = 0;
  if (g < a.n_lam) {
    int m = 0;
    if (a.lambda_off) {  // last m with lambda_off[m] <= g
      int lo = 0, hi = a.n_models;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (a.lambda_off[mid] <= g) lo = mid; else hi = mid;
      }
      m = lo;
    }
    const double lam = a.lambda[g];
    const ModelDesc d = a.models[m];
    const bool ok = !bad && d.valid && (lam > 0.0) && (lam < __builtin_inf());
    a.lam_model[g] = m;
    a.lam_k[g] = ok ? (2.0 * M_PI / lam) : __builtin_nan("");
    key = kBuckets - 1;
    if (ok) {
      const LayerRec64* L = a.layers64 + d.layer_base;
      int lo = 0, hi = d.n_layers;  // first layer whose bottom reaches lambda / 3
      const double z3 = lam * (1.0 / 3.0);
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (L[mid].zb < z3) lo = mid + 1; else hi = mid;
      }
      const double c_est = 0.9 / ::sqrt(L[lo].ib2);
      double pos = 0.0;  // interpolated grid index of c_est
      if (ns > 1 && c_est > s_c[0]) {
        int sl = 0, sh = ns - 1;  // last sample below c_est
        while (sh - sl > 1) {
          const int mid = (sl + sh) >> 1;
          if (s_c[mid] < c_est) sl = mid; else sh = mid;
        }
        const double step = double(a.n_c - 1) / double(ns - 1);
        const double span = s_c[sl + 1] - s_c[sl];
        const double f = span > 0.0 ? min(1.0, (c_est - s_c[sl]) / span) : 0.0;
        pos = (double(sl) + f) * step;
      }
      const double cost = double(d.n_layers + 1) * (pos + 64.0);
      const int bk = min(kBuckets - 1, max(0, int(8.0 * ::log2(cost))));
      key = kBuckets - 1 - bk;
    }
    a.lam_bucket[g] = uint8_t(key);
    rank = atomicAdd(&s_hist[key], 1u);
  }
  __syncthreads();
  if (gridDim.x > 1) {
    for (int i = t; i < kBuckets; i += blockDim.x)
      if (s_hist[i]) atomicAdd(&a.counters->hist[i], s_hist[i]);
    return;
  }
  // one block: exclusive prefix sum of the histogram, then the scatter
  if (t < kBuckets) s_scan[t] = s_hist[t];
  __syncthreads();
  for (int off = 1; off < kBuckets; off <<= 1) {
    const uint32_t v = (t < kBuckets && t >= off) ? s_scan[t - off] : 0u;
    __syncthreads();
    if (t < kBuckets) s_scan[t] += v;
    __syncthreads();
  }
  if (g < a.n_lam) a.order[s_scan[key] - s_hist[key] + rank] = g;
}

__global__ __launch_bounds__(kLamBlock) void prep_lambda_kernel(PrepArgs a, int nb_grid) {
  __shared__ LambdaShared ls;
  int bad = 0;
  for (int i = threadIdx.x; i < nb_grid; i += blockDim.x) bad |= int(a.grid_flags[i]);
  bad = __syncthreads_or(bad);
  stage_lambdas(a, bad, ls);
}

// The whole staging of a small job in one block (one launch instead of
// two): grid checks and the FP32 copy, the models' records (one wavefront
// per model), the counters and shared-sweep state, then the wavelengths.
// For jobs of at most kLamBlock wavelengths, kSmallModels models and
// kSmallGrid grid points.
constexpr int kSmallModels = kLamBlock / 64;
constexpr int kSmallGrid = 16 * kLamBlock;

__global__ __launch_bounds__(kLamBlock) void prep_small_kernel(PrepArgs a, CoopInitArgs ci, int single_N,
                                                               int single_W) {
  __shared__ LambdaShared ls;
  const int t = threadIdx.x;
  int bad = 0;
  for (int i = t; i < a.n_c; i += kLamBlock) {
    const double c = a.c_in[i];
    if (a.c64 != a.c_in) a.c64[i] = c;
    a.c32[i] = float(c);
    bool ok = (c > 0.0) && (c < __builtin_inf());
    if (i + 1 < a.n_c) ok = ok && (c < a.c_in[i + 1]);
    bad |= ok ? 0 : 1;
  }
  for (int m = t >> 6; m < a.n_models; m += kLamBlock / 64) build_model(a, m, single_N, single_W);
  uint32_t* cw = reinterpret_cast<uint32_t*>(a.counters);
  for (int i = t; i < int(sizeof(Counters) / sizeof(uint32_t)); i += kLamBlock) cw[i] = 0u;
  for (int i = t; i < ci.n_coop; i += kLamBlock) ci.coop[i] = CoopItem{0, 0x7fffffff, 0, 0};
  for (uint64_t i = t; i < ci.n_sum; i += kLamBlock) ci.coop_sum[i] = 0ull;
  for (int i = t; i < ci.n_active; i += kLamBlock) ci.coop_active[i] = -1;
  bad = __syncthreads_or(bad);  // also: records, grid copy and counters are written
  stage_lambdas(a, bad, ls);
}

// Exclusive prefix sum of the histogram, in place (one block of kBuckets).
__global__ void order_scan_kernel(Counters* c) {
  __shared__ uint32_t s[kBuckets];
  const int t = threadIdx.x;
  s[t] = c->hist[t];
  __syncthreads();
  for (int off = 1; off < kBuckets; off <<= 1) {
    const uint32_t v = (t >= off) ? s[t - off] : 0u;
    __syncthreads();
    s[t] += v;
    __syncthreads();
  }
  c->hist[t] = s[t] - c->hist[t];
}

// Scatter wavelengths into their buckets (order inside a bucket is free).
__global__ void order_scatter_kernel(PrepArgs a) {
  __shared__ uint32_t s_cnt[kBuckets];
  __shared__ uint32_t s_base[kBuckets];
  for (int i = threadIdx.x; i < kBuckets; i += blockDim.x) s_cnt[i] = 0u;
  __syncthreads();
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  int key = 0;
  uint32_t rank = 0;
  if (g < a.n_lam) {
    key = a.lam_bucket[g];
    rank = atomicAdd(&s_cnt[key], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kBuckets; i += blockDim.x)
    s_base[i] = s_cnt[i] ? atomicAdd(&a.counters->hist[i], s_cnt[i]) : 0u;
  __syncthreads();
  if (g < a.n_lam) a.order[s_base[key] + rank] = g;
}

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
      sg = sweep_code32(r.c32[i], float(r.k64), r.L32, r.N);
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
          const int sg = (i < n32) ? sweep_code32(r.c32[i], k32, r.L32, r.N) : kNoSign;
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

template <int G>
__device__ __forceinline__ void flush_counts(Counters* c, const WorkCount& wc) {
  if (threadIdx.x == 0) {
    atomicAdd(&c->sweep, wc.sweep);
    atomicAdd(&c->check, wc.check);
    atomicAdd(&c->refine, wc.refine);
    atomicAdd(&c->useful, wc.useful);
    if (wc.helper) atomicAdd(&c->helper, wc.helper);
  }
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
// SIMD, as the plain sweeps), spilling a little outside the layer loop.
template <int MODE, int G, bool MISFIT>
__global__ __launch_bounds__(64 * G) __attribute__((amdgpu_waves_per_eu(MISFIT ? 4 : 1)))
void sweep_kernel(SweepArgs a) {
  __shared__ SweepShared<G> sh;
  __shared__ double s_mis[MISFIT ? 256 : 1];  // fused misfit reduction
  WorkCount wc;
  constexpr int P = 64 * G;
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
  flush_counts<G>(a.counters, wc);
}


// ------------------------------------------------------------- serving --
// Precompute of newly admitted requests.  Block (b, y) moves chunk y of
// request b's raw inputs from the staging copy into the request's pool block,
// with the FP32 copy of the grid part; block (b, 0) also checks the model and
// writes its layer records, the k values and the item states.  The host has
// already checked every value at submit, so an invalid model here (never
// expected) only marks its wavelengths invalid.
constexpr int kAdmitChunk = 1024;

__global__ __launch_bounds__(kAdmitChunk) void admit_kernel(const AdmitList* __restrict__ list,
                                                            int32_t* slot_remaining) {
  const int b = blockIdx.x;
  if (b >= list->n) return;
  const SlotDesc d = list->desc[b];
  const double* __restrict__ src = list->src[b];
  const int N = d.N, W = d.W, n_c = d.n_c;
  const int c_off = N + 3 * (N + 1) + W;
  const int i = int(blockIdx.y) * kAdmitChunk + int(threadIdx.x);
  if (i < c_off + n_c) {
    const double v = src[i];
    const_cast<double*>(d.raw)[i] = v;
    if (i >= c_off) d.c32[i - c_off] = float(v);
  }
  if (blockIdx.y != 0) return;
  const double* h = src;
  const double* alpha = h + N;
  const double* beta = alpha + (N + 1);
  const double* rho = beta + (N + 1);
  const double* lam = rho + (N + 1);
  int bad = (N < 0 || N > MASW_MAX_LAYERS) ? 1 : 0;
  for (int j = threadIdx.x; !bad && j <= N; j += blockDim.x) {
    const double al = alpha[j], be = beta[j], rh = rho[j];
    bool ok = (al < __builtin_inf()) && (rh < __builtin_inf()) && (be > 0.0) && (al > be) && (rh > 0.0);
    if (j < N) ok = ok && (h[j] > 0.0) && (h[j] < __builtin_inf());
    bad |= ok ? 0 : 1;
  }
  const bool valid = __syncthreads_or(bad) == 0;
  const double mu_ref = valid ? rho[N] * beta[N] * beta[N] : 0.0;
  if (valid) {
    for (int j = threadIdx.x; j <= N; j += blockDim.x) {
      const double al = alpha[j], be = beta[j], rh = rho[j];
      LayerRec64 r;
      r.ia2 = 1.0 / (al * al);
      r.ib2 = 1.0 / (be * be);
      r.rh = rh / mu_ref;
      r.mh = rh * be * be / mu_ref;
      r.h = (j < N) ? h[j] : 0.0;
      r.aux = (j == N) ? mu_ref : 0.0;
      r.zb = r.pad2 = 0.0;
      d.L64[j] = r;
      LayerRec32 q;
      q.ia2 = float(r.ia2);
      q.ib2 = float(r.ib2);
      q.rh = float(r.rh);
      q.mh = float(r.mh);
      q.h = float(r.h);
      q.aux = float(mu_ref);
      q.zb = q.pad2 = 0.0f;
      d.L32[j] = q;
    }
  }
  for (int w = threadIdx.x; w < W; w += blockDim.x) {
    const double l = lam[w];
    const bool ok = valid && (l > 0.0) && (l < __builtin_inf());
    d.lam_k[w] = ok ? (2.0 * M_PI / l) : __builtin_nan("");
    d.state[w] = item_state_init();
  }
  if (threadIdx.x == 0) slot_remaining[list->slot[b]] = W;
}

// One FP64 item of a serving tick by the inertia-count search: the sampling
// round of the search on all G wavefronts (64 G grid points: c_test[0] and
// 64 G - 1 spread points), then the counts, the sign at the change and the
// refinement on wavefront 0.  The sampled bound leaves a bracket of about
// n_c / (64 G) grid points, which one round of counts resolves.  The other
// wavefronts wait at the barrier.  Where the search would fall back to
// walking, the item is handed to the walking path instead (all G wavefronts,
// at most `budget` rounds per tick, resumed in later ticks), so that no item
// holds a tick for a long walk.  Returns true once the outputs are written;
// they equal the walk's.
template <int G>
__device__ bool inertia_tick_item(const ItemRef& r, ItemState& st, int budget, SweepShared<G>& sh, WorkCount& wc,
                                  const ItemOut& o, Counters* cnt) {
  if (!st.fp64) {
    constexpr int P = 64 * G;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = r.n_c - 1;
    bool va = true;
    const int pa = (tid == 0) ? 0 : inertia::spread(0, n, tid, 1, &va, P);
    if (tid == 0) va = true;
    const int sa = va ? det_sign<double, false>(r.c64[pa], r.k64, r.L64, r.N, nullptr) : kNoSign;
    if (tid == 0) sh.check[0] = sa;
    __syncthreads();
    const int sig0 = sh.check[0];
    const unsigned long long m = __ballot(tid > 0 && va && sa != sig0);
    if (lane == 0) sh.first[wave] = m ? wave * 64 + (__ffsll((long long)m) - 1) : P;
    __syncthreads();
    if (wave == 0) {
      int f = P;
#pragma unroll
      for (int w = 0; w < G; ++w) f = min(f, sh.first[w]);
      inertia::Tally t;
      t.handoff = true;  // a walk continues below, G wavefronts wide and within the tick's budget
      t.check = (unsigned long long)min(P, r.n_c);
      int sig_f = 0, prev_f = 0, found;
      if (sig0 != 1 && sig0 != -1) {
        found = inertia::walk(r.c64, r.n_c, r.k64, r.L64, r.N, 1, sig0, &sig_f, &prev_f, t);
      } else if (f == P) {
        // no sampled sign differs: the one-wavefront search from the start
        found = inertia::search(r.c64, r.n_c, r.k64, r.L64, r.N, -1, &sig_f, &prev_f, t);
      } else {
        bool v;
        const int pf = inertia::spread(0, n, f, 1, &v, P);
        const int pb = (f == 1) ? 0 : inertia::spread(0, n, f - 1, 1, &v, P);
        inertia::Bracket br;
        found = inertia::from_sampled_bound(r.c64, r.n_c, r.k64, r.L64, r.N, 0, false, 0, sig0, pb, pf, &br,
                                            &sig_f, &prev_f, t);
        if (found == inertia::kLocated)
          found = inertia::finish(r.c64, r.n_c, r.k64, r.L64, r.N, sig0, br, &sig_f, &prev_f, t);
      }
      wc.sweep += t.scan;
      wc.check += t.check;
      if (found == inertia::kResume) {
        if (lane == 0) {
          sh.check[1] = t.resume;
          sh.check[2] = t.resume_carry;
        }
      } else {
        if (found < 0) {
          write_no_pick(o, MASW_STATUS_NOT_FOUND, lane == 0);
          wc.useful += (unsigned long long)r.n_c;
        } else {
          wc.useful += (unsigned long long)(found + 1);
          wc.refine += refine_and_write(o, r.c64, r.k64, r.L64, r.N, found, sig_f, prev_f);
        }
        if (lane == 0) sh.check[1] = -1;
      }
    }
    __syncthreads();
    const int resume = sh.check[1], carry = sh.check[2];
    __syncthreads();
    if (resume < 0) {
      st.done = 1;
      return true;
    }
    // the search handed back a walk (after an unusable count, or a first
    // sign that is not +-1): the walking path takes the item from there
    st.start = resume;
    st.carry = carry;
    st.fp64 = 1;
  }
  return run_item<kModeFP64, G>(r, st, budget, sh, wc, o, kNoCoop, cnt);
}

// One serving tick: every unfinished item of every active request advances by
// at most desc->budget sweep rounds (then its re-check and refinement if its
// change was found).  The last item of a request to finish raises the
// request's completion flag in pinned host memory.
// With G = 8 the kernel is held to 128 VGPRs (4 wavefronts per SIMD), so two
// workgroups fit on a CU, as for the batch sweep.  INERTIA (a server started
// with search_inertia) runs FP64 items with the inertia-count search instead
// of walking them; it needs more registers, so it is an instantiation of its
// own and the walking ticks keep their allocation.
template <int G, bool INERTIA>
__global__ __launch_bounds__(64 * G) __attribute__((amdgpu_waves_per_eu((G >= 8 && !INERTIA) ? 4 : 1)))
void tick_kernel(TickArgs a) {
  __shared__ SweepShared<G> sh;
  WorkCount wc;
  const TickDesc* __restrict__ D = a.desc;
  const int n_units = D->n_units;
  const int n_active = D->n_active;
  const int budget = D->budget;
  const uint32_t base = D->base;
  for (;;) {
    // every workgroup ends with exactly one claim at or beyond n_units
    if (threadIdx.x == 0) sh.item = int(atomicAdd(&a.counters->queue_head, 1u) - base);
    __syncthreads();
    const int u = uniform(sh.item);
    __syncthreads();
    if (u >= n_units) break;
    int lo = 0, hi = n_active;  // last active slot with prefix <= u
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (D->prefix[mid] <= u) lo = mid; else hi = mid;
    }
    const int slot = uniform(D->active[lo]);
    const int j = u - D->prefix[lo];
    const SlotDesc& sd = D->slot[slot];
    ItemState st = sd.state[j];
    if (st.done) continue;
    ItemRef r;
    r.N = uniform(sd.N);
    r.n_c = uniform(sd.n_c);
    r.n_real = uniform(sd.n_real);
    r.k64 = sd.lam_k[j];
    r.c64 = sd.raw + (r.N + 3 * (r.N + 1) + sd.W);
    r.c32 = sd.c32;
    r.L64 = sd.L64;
    r.L32 = sd.L32;
    const int og = sd.out_base + j;
    const ItemOut o{a.out_ct + og, a.out_idx + og, a.out_status + og, a.out_cref + og,
                    (a.refine && !(sd.flags & MASW_NO_REFINE)) ? 1 : 0, a.refine_rel};
    bool done;
    if (!(r.k64 == r.k64)) {
      write_missing<G>(o, MASW_STATUS_INVALID);
      st.done = 1;
      done = true;
    } else if (sd.prec == MASW_PREC_SPLIT) {
      done = run_item<kModeSplit, G>(r, st, budget, sh, wc, o, kNoCoop, a.counters);
    } else if (INERTIA) {
      done = inertia_tick_item<G>(r, st, budget, sh, wc, o, a.counters);
    } else {
      done = run_item<kModeFP64, G>(r, st, budget, sh, wc, o, kNoCoop, a.counters);
    }
    if (threadIdx.x == 0) {
      sd.state[j] = st;
      if (done) {
        __threadfence_system();
        if (atomicSub(&a.slot_remaining[slot], 1) == 1) a.host_done[slot] = 1;
      }
    }
    __syncthreads();  // wavefront 0's outputs are written before the next item is fetched
  }
  flush_counts<G>(a.counters, wc);
  // The last workgroup to leave tells the host, through pinned memory, that
  // the tick is over: the host waits on this word instead of the stream.
  // Every workgroup's outputs are released (system scope) before its count.
  if (threadIdx.x == 0) {
    __threadfence_system();
    const uint32_t left = atomicAdd(&a.counters->tick_exit, 1u) + 1u - D->exit_base;
    if (left == gridDim.x) {
      __threadfence_system();
      __hip_atomic_store(a.host_tick, D->seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

// -------------------------------------------------------------- misfit --
// Algorithm 2 per model: one workgroup of 256 threads per model; each thread
// sums a strided subset in order, then a fixed-order tree in LDS.
__global__ __launch_bounds__(256) void misfit_kernel(int n_models, const int32_t* __restrict__ lambda_off,
                                                     const double* __restrict__ c_t,
                                                     const double* __restrict__ c_e, double* __restrict__ out) {
  __shared__ double s[256];
  const int m = blockIdx.x;
  if (m >= n_models) return;
  const int lo = lambda_off[m], hi = lambda_off[m + 1];
  double acc = 0.0;
  for (int i = lo + threadIdx.x; i < hi; i += blockDim.x) acc += ::fabs(c_t[i] - c_e[i]) / c_e[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[m] = (hi > lo) ? s[0] / double(hi - lo) : __builtin_nan("");
}

hipError_t launch_misfit(int n_models, const int32_t* lambda_off, const double* c_t, const double* c_e,
                         double* out, hipStream_t st) {
  if (n_models <= 0) return hipSuccess;
  hipLaunchKernelGGL(misfit_kernel, dim3(n_models), dim3(256), 0, st, n_models, lambda_off, c_t, c_e, out);
  return hipGetLastError();
}

// ------------------------------------------------------------ sign map --
// Every (wavelength, grid point) of model 0, no early exit: blockIdx.y is
// the wavelength, x covers the grid.
template <typename T>
__global__ __launch_bounds__(256) void sign_map_kernel(SignMapArgs a) {
  const int w = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n_c) return;
  const ModelDesc d = a.models[0];
  const double k64 = a.lam_k[w];
  const size_t o = size_t(w) * size_t(a.n_c) + size_t(i);
  if (!(k64 == k64)) {
    a.sigma[o] = int8_t(kNaNSign);
    if (a.logabs) a.logabs[o] = __builtin_nan("");
    return;
  }
  const int N = uniform(d.n_layers);
  const double c = a.c64[d.c_base + i];
  int sg;
  if constexpr (sizeof(T) == 8) {
    const LayerRec64* L = a.layers64 + uniform(d.layer_base);
    if (a.logabs) {
      double la;
      sg = det_sign_logabs<double>(c, k64, L, N, L[N].aux, k64, &la);
      a.logabs[o] = la;
    } else {
      sg = det_sign<double, false>(c, k64, L, N, nullptr);
    }
  } else {
    const LayerRec32* L = a.layers32 + uniform(d.layer_base);
    const LayerRec64* L64 = a.layers64 + uniform(d.layer_base);
    if (a.logabs) {
      double la;
      sg = det_sign_logabs<float>(float(c), float(k64), L, N, L64[N].aux, k64, &la);
      a.logabs[o] = la;
    } else {
      sg = det_sign<float, false>(float(c), float(k64), L, N, nullptr);
    }
  }
  a.sigma[o] = int8_t(sg);
}

// ------------------------------------------------------- no-alloc scratch --
// Workspace of masw_dispersion_curve_noalloc: one static array per device
// (each device that loads the library holds its own copy until the process
// ends).  Host code never uses the array's name as an address: masw_create
// looks up each device's copy once, with that device current, and the entry
// point hands the kernels that address in their argument structs.
constexpr int kMaxScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[MASW_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void* g_scratch[kMaxScratchDevices] = {};

hipError_t setup_scratch(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e == hipSuccess) g_scratch[device] = p;
  return e;
}

void* scratch_of(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch[device];
}

// --------------------------------------------------------- host launchers --
template <int MODE, bool MISFIT>
static const void* sweep_symbol_mode(int G) {
  switch (G) {
    case 1: return reinterpret_cast<const void*>(&sweep_kernel<MODE, 1, MISFIT>);
    case 2: return reinterpret_cast<const void*>(&sweep_kernel<MODE, 2, MISFIT>);
    case 4: return reinterpret_cast<const void*>(&sweep_kernel<MODE, 4, MISFIT>);
    case 8: return reinterpret_cast<const void*>(&sweep_kernel<MODE, 8, MISFIT>);
    case 16: return reinterpret_cast<const void*>(&sweep_kernel<MODE, 16, MISFIT>);
  }
  return nullptr;
}

static const void* sweep_symbol(int mode, int G, bool misfit = false) {
  if (misfit) return mode == kModeFP64 ? sweep_symbol_mode<kModeFP64, true>(G) : sweep_symbol_mode<kModeSplit, true>(G);
  return mode == kModeFP64 ? sweep_symbol_mode<kModeFP64, false>(G) : sweep_symbol_mode<kModeSplit, false>(G);
}

int sweep_blocks_per_cu(int mode, int G) {
  const void* f = sweep_symbol(mode, G);
  if (!f) return 0;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, 64 * G, 0) != hipSuccess) return 0;
  return n;
}

hipError_t launch_sweep(int mode, int G, int blocks, hipStream_t s, const SweepArgs& a) {
  const void* f = sweep_symbol(mode, G, a.misfit != nullptr);
  if (!f) return hipErrorInvalidValue;
  void* args[] = {const_cast<SweepArgs*>(&a)};
  return hipLaunchKernel(f, dim3(blocks), dim3(64 * G), args, 0, s);
}

hipError_t launch_prep(const PrepArgs& a, const CoopInitArgs& ci, int single_N, int single_W, hipStream_t s) {
  const uint64_t n_clear_small = std::max<uint64_t>(ci.n_sum, uint64_t(std::max(ci.n_coop, ci.n_active)));
  if (a.n_lam <= kLamBlock && a.n_models <= kSmallModels && a.n_c <= kSmallGrid && n_clear_small <= kSmallGrid) {
    hipLaunchKernelGGL(prep_small_kernel, dim3(1), dim3(kLamBlock), 0, s, a, ci, single_N, single_W);
    return hipGetLastError();
  }
  const int nb_grid = (a.n_c + kPrepThreads - 1) / kPrepThreads;
  const int nb_models = (a.n_models + kPrepThreads / 64 - 1) / (kPrepThreads / 64);
  const uint64_t n_clear = std::max<uint64_t>(ci.n_sum, uint64_t(std::max(ci.n_coop, ci.n_active)));
  const int nb_clear = int(std::max<uint64_t>(1, std::min<uint64_t>(512, (n_clear + kPrepThreads - 1) / kPrepThreads)));
  hipLaunchKernelGGL(prep_front_kernel, dim3(nb_grid + nb_models + nb_clear), dim3(kPrepThreads), 0, s, a, ci,
                     nb_grid, nb_models, nb_clear, single_N, single_W);
  if (a.n_lam > 0) {
    if (a.n_lam <= kLamBlock) {
      hipLaunchKernelGGL(prep_lambda_kernel, dim3(1), dim3(kLamBlock), 0, s, a, nb_grid);
    } else {
      const int nb = (a.n_lam + kPrepThreads - 1) / kPrepThreads;
      hipLaunchKernelGGL(prep_lambda_kernel, dim3(nb), dim3(kPrepThreads), 0, s, a, nb_grid);
      hipLaunchKernelGGL(order_scan_kernel, dim3(1), dim3(kBuckets), 0, s, a.counters);
      hipLaunchKernelGGL(order_scatter_kernel, dim3(nb), dim3(kPrepThreads), 0, s, a);
    }
  }
  return hipGetLastError();
}

static const void* tick_symbol(int G, bool inertia) {
  switch (G) {
    case 1: return inertia ? reinterpret_cast<const void*>(&tick_kernel<1, true>)
                           : reinterpret_cast<const void*>(&tick_kernel<1, false>);
    case 2: return inertia ? reinterpret_cast<const void*>(&tick_kernel<2, true>)
                           : reinterpret_cast<const void*>(&tick_kernel<2, false>);
    case 4: return inertia ? reinterpret_cast<const void*>(&tick_kernel<4, true>)
                           : reinterpret_cast<const void*>(&tick_kernel<4, false>);
    case 8: return inertia ? reinterpret_cast<const void*>(&tick_kernel<8, true>)
                           : reinterpret_cast<const void*>(&tick_kernel<8, false>);
  }
  return nullptr;
}

int tick_blocks_per_cu(int G, bool inertia) {
  const void* f = tick_symbol(G, inertia);
  int n = 0;
  if (!f || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, 64 * G, 0) != hipSuccess) return 0;
  return n;
}

hipError_t launch_admit(const AdmitList* list_dev, int n, int max_raw, int32_t* slot_remaining, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int chunks = std::max(1, (max_raw + kAdmitChunk - 1) / kAdmitChunk);
  hipLaunchKernelGGL(admit_kernel, dim3(n, chunks), dim3(kAdmitChunk), 0, s, list_dev, slot_remaining);
  return hipGetLastError();
}

hipError_t launch_tick(int G, int blocks, hipStream_t s, const TickArgs& a) {
  const void* f = tick_symbol(G, a.inertia != 0);
  if (!f) return hipErrorInvalidValue;
  void* args[] = {const_cast<TickArgs*>(&a)};
  return hipLaunchKernel(f, dim3(blocks), dim3(64 * G), args, 0, s);
}

hipError_t launch_sign_map(bool fp32, const SignMapArgs& a, hipStream_t s) {
  if (a.n_lam == 0 || a.n_c == 0) return hipSuccess;
  const dim3 grid((a.n_c + 255) / 256, a.n_lam);
  if (fp32)
    hipLaunchKernelGGL(sign_map_kernel<float>, grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(sign_map_kernel<double>, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace masw
