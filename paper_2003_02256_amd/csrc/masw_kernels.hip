// HIP kernels for gfx950: staging/precompute, work ordering, the FP64 batch
// sweep kernels (the sweep itself is in masw_sweep.hpp; the split kernels
// are built in masw_sweep_split.hip), the serving tick, the misfit and the
// full-grid sign map, and the host launchers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "masw_inertia.hpp"
#include "masw_internal.hpp"
#include "masw_math.hpp"
#include "masw_pick.hpp"
#include "masw_sweep.hpp"

namespace masw {

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
  stamp_start(a.tstamp, 0);
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
  stamp_start(a.tstamp, 0);
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
    r.L64 = as_global(sd.L64);
    r.L32 = as_global(sd.L32);
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
  // (the work counts of ticks are not reported: no atomics on a shared
  // counter line at every tick's end)
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
  if (mode != kModeFP64) return split_sweep_symbol(G, misfit);
  return misfit ? sweep_symbol_mode<kModeFP64, true>(G) : sweep_symbol_mode<kModeFP64, false>(G);
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

hipError_t launch_fused(int mode, int blocks, hipStream_t s, const SweepArgs& a) {
  const void* f = mode == kModeFP64 ? reinterpret_cast<const void*>(&fused_sweep_kernel<kModeFP64>)
                                    : split_fused_symbol();
  if (!f || a.fused_N < 0 || a.fused_N > kFusedMaxLayers) return hipErrorInvalidValue;
  void* args[] = {const_cast<SweepArgs*>(&a)};
  return hipLaunchKernel(f, dim3(blocks), dim3(64 * kFusedG), args, unsigned(fused_lds_bytes(a.fused_N)), s);
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
