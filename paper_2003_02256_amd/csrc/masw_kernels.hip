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
#include <hip/hip_runtime.h>

#include "masw_internal.hpp"
#include "masw_math.hpp"

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

// ------------------------------------------------------------- staging --
__global__ void zero_counters_kernel(Counters* c) {
  uint32_t* p = reinterpret_cast<uint32_t*>(c);
  const int n = sizeof(Counters) / sizeof(uint32_t);
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

// Grid checks (strictly increasing, finite, > 0) and the FP32 copy of the grid.
__global__ void prep_grid_kernel(const double* __restrict__ c_in, int n_c, double* __restrict__ c64,
                                 float* __restrict__ c32, Counters* counters) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_c) return;
  const double c = c_in[i];
  if (c64 != c_in) c64[i] = c;
  c32[i] = float(c);
  bool ok = (c > 0.0) && (c < __builtin_inf());
  if (i + 1 < n_c) ok = ok && (c < c_in[i + 1]);
  if (!ok) atomicOr(&counters->grid_bad, 1u);
}

// One thread per model: validation and the per-layer coefficient records.
// With a.layer_off == nullptr the batch is a single model of
// single_N layers and single_W wavelengths.
__global__ void prep_models_kernel(PrepArgs a, int single_N, int single_W) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= a.n_models) return;
  const int lo = a.layer_off ? a.layer_off[m] : 0;
  const int hi = a.layer_off ? a.layer_off[m + 1] : single_N;
  const int N = hi - lo;
  const int rec0 = lo + m;  // records and alpha/beta/rho entries of model m
  bool ok = (N >= 0) && (N <= MASW_MAX_LAYERS) && (a.counters->grid_bad == 0u);
  if (ok) {
    for (int j = 0; j <= N; ++j) {
      const double al = a.alpha[rec0 + j], be = a.beta[rec0 + j], rh = a.rho[rec0 + j];
      const bool finite = (al < __builtin_inf()) && (rh < __builtin_inf());
      ok = ok && finite && (be > 0.0) && (al > be) && (rh > 0.0);
      if (j < N) {
        const double h = a.h[lo + j];
        ok = ok && (h > 0.0) && (h < __builtin_inf());
      }
    }
  }
  ModelDesc d;
  d.n_layers = ok ? N : 0;
  d.layer_base = rec0;
  d.c_base = 0;
  d.n_c = a.n_c;
  d.lam_base = a.lambda_off ? a.lambda_off[m] : 0;
  d.n_lam = a.lambda_off ? (a.lambda_off[m + 1] - a.lambda_off[m]) : single_W;
  d.valid = ok ? 1 : 0;
  d.pad = 0;
  a.models[m] = d;
  if (!ok) return;
  const double mu_ref = a.rho[rec0 + N] * a.beta[rec0 + N] * a.beta[rec0 + N];
  for (int j = 0; j <= N; ++j) {
    const double al = a.alpha[rec0 + j], be = a.beta[rec0 + j], rh = a.rho[rec0 + j];
    LayerRec64 r;
    r.ia2 = 1.0 / (al * al);
    r.ib2 = 1.0 / (be * be);
    r.rh = rh / mu_ref;
    r.mh = rh * be * be / mu_ref;
    r.h = (j < N) ? a.h[lo + j] : 0.0;
    r.aux = (j == N) ? mu_ref : 0.0;
    r.pad1 = r.pad2 = 0.0;
    a.layers64[rec0 + j] = r;
    LayerRec32 s;
    s.ia2 = float(r.ia2);
    s.ib2 = float(r.ib2);
    s.rh = float(r.rh);
    s.mh = float(r.mh);
    s.h = float(r.h);
    s.aux = float(mu_ref);
    s.pad1 = s.pad2 = 0.0f;
    a.layers32[rec0 + j] = s;
  }
}

// One thread per wavelength: k, its model, and the work-order key.  The
// expected search depth is the grid index of 0.9 beta at depth lambda/3 (a
// Rayleigh wave samples roughly the top third of a wavelength); the cost is
// that depth times N+1.  Longer wavelengths see faster material and search
// deeper (Section 3.2's observation behind the modular partition), so the key
// orders them first.
__global__ void prep_lambda_kernel(PrepArgs a) {
  __shared__ uint32_t s_hist[kBuckets];
  for (int i = threadIdx.x; i < kBuckets; i += blockDim.x) s_hist[i] = 0u;
  __syncthreads();
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
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
    const bool ok = d.valid && (lam > 0.0) && (lam < __builtin_inf());
    a.lam_model[g] = m;
    a.lam_k[g] = ok ? (2.0 * M_PI / lam) : __builtin_nan("");
    int key = kBuckets - 1;
    if (ok) {
      const LayerRec64* L = a.layers64 + d.layer_base;
      double z = 0.0, beta = 0.0;
      int j = 0;
      for (; j < d.n_layers; ++j) {
        z += L[j].h;
        if (z >= lam * (1.0 / 3.0)) break;
      }
      beta = 1.0 / ::sqrt(L[j].ib2);
      const double c_est = 0.9 * beta;
      int lo = 0, hi = d.n_c;  // first index with c >= c_est
      const double* c = a.c64 + d.c_base;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (c[mid] < c_est) lo = mid + 1; else hi = mid;
      }
      const double cost = double(d.n_layers + 1) * double(lo + 64);
      const int b = min(kBuckets - 1, max(0, int(8.0 * ::log2(cost))));
      key = kBuckets - 1 - b;
    }
    a.lam_bucket[g] = uint8_t(key);
    atomicAdd(&s_hist[key], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kBuckets; i += blockDim.x)
    if (s_hist[i]) atomicAdd(&a.counters->hist[i], s_hist[i]);
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

template <int MODE, int G>
__global__ __launch_bounds__(64 * G) void sweep_kernel(SweepArgs a) {
  constexpr int P = 64 * G;  // positions per round
  __shared__ int s_item;
  __shared__ int s_last[G];
  __shared__ int s_first[G];
  __shared__ int s_pair[2];
  __shared__ int s_check[4];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  unsigned long long n_sweep = 0, n_check = 0, n_refine = 0, n_useful = 0;

  for (;;) {
    if (tid == 0) s_item = (int)atomicAdd(&a.counters->queue_head, 1u);
    __syncthreads();
    const int it = uniform(s_item);
    __syncthreads();
    if (it >= a.n_items) break;

    const int g = uniform(a.order[it]);
    const int m = uniform(a.lam_model[g]);
    const ModelDesc d = a.models[m];
    const int N = uniform(d.n_layers);
    const int n_c = uniform(d.n_c);
    const double k64 = a.lam_k[g];
    const double* __restrict__ c64 = a.c64 + uniform(d.c_base);
    const float* __restrict__ c32 = a.c32 + uniform(d.c_base);
    const LayerRec64* __restrict__ L64 = a.layers64 + uniform(d.layer_base);
    const LayerRec32* __restrict__ L32 = a.layers32 + uniform(d.layer_base);

    if (!(k64 == k64)) {  // invalid model, grid or wavelength
      if (tid == 0) {
        a.out_idx[g] = -1;
        a.out_status[g] = MASW_STATUS_INVALID;
        a.out_ct[g] = __builtin_nan("");
        if (a.out_cref) a.out_cref[g] = __builtin_nan("");
      }
      continue;
    }

    int found = -1, sig_f = 0, prev_f = 0, carry = kNoSign;
    if (MODE == kModeFP64) {
      for (int base = 0; base < n_c; base += P) {
        const int i = base + tid;
        const int sg = (i < n_c) ? det_sign<double, false>(c64[i], k64, L64, N, nullptr) : kNoSign;
        const int f = round_first_change<G>(sg, carry, s_last, s_first, s_pair, &carry, &sig_f, &prev_f);
        n_sweep += (unsigned long long)min(P, n_c - base);
        if (f >= 0) {
          found = base + f;
          break;
        }
      }
    } else {
      const float k32 = float(k64);
      int start = 0;
      while (start < n_c && found < 0) {
        // FP32 sweep from `start` for a candidate change.
        int cand = -1;
        for (int base = start; base < n_c; base += P) {
          const int i = base + tid;
          const int sg = (i < n_c) ? det_sign<float, false>(c32[i], k32, L32, N, nullptr) : kNoSign;
          int s_c, p_c;
          const int f = round_first_change<G>(sg, carry, s_last, s_first, s_pair, &carry, &s_c, &p_c);
          n_sweep += (unsigned long long)min(P, n_c - base);
          if (f >= 0) {
            cand = base + f;
            break;
          }
        }
        if (cand < 0) break;
        // FP64 re-check of the 64 positions ws-1 .. ws+62 around the
        // candidate (48 before it, 15 after), one per lane of wavefront 0;
        // the other wavefronts wait.  The window does not depend on the
        // group size, so neither does the outcome.
        const int ws = max(1, cand - 48);
        if (wave == 0) {
          const int i = ws - 1 + lane;
          const int sg = (i < n_c) ? det_sign<double, false>(c64[i], k64, L64, N, nullptr) : kNoSign;
          int last, s_c = 0, p_c = 0;
          const int f = wave_first_change(sg, &s_c, &p_c, &last);
          if (lane == 0) {
            s_check[0] = f;
            s_check[1] = last;
            s_check[2] = s_c;
            s_check[3] = p_c;
          }
        }
        __syncthreads();
        const int f = s_check[0];
        const int last = s_check[1];
        sig_f = s_check[2];
        prev_f = s_check[3];
        __syncthreads();
        n_check += (unsigned long long)min(64, n_c - (ws - 1));
        if (f >= 0) {
          found = ws - 1 + f;
        } else {
          // Rejected: resume the FP32 sweep after the checked window,
          // carrying the FP64 sign of its last position.
          start = ws + 63;
          carry = last;
        }
      }
    }

    if (found < 0) {
      if (tid == 0) {
        a.out_idx[g] = -1;
        a.out_status[g] = MASW_STATUS_NOT_FOUND;
        a.out_ct[g] = __builtin_nan("");
        if (a.out_cref) a.out_cref[g] = __builtin_nan("");
      }
      n_useful += (unsigned long long)n_c;
      continue;
    }
    n_useful += (unsigned long long)(found + 1);

    // Refinement and output by wavefront 0 alone; the others go on to the
    // next item's queue barrier.  One wavefront at a time on a SIMD finishes
    // these few rounds sooner than the whole group sharing the SIMDs would.
    if (wave == 0) {
      int status = MASW_STATUS_FOUND;
      if (sig_f == kNaNSign || prev_f == kNaNSign) status = MASW_STATUS_NAN;
      double c_ref = __builtin_nan("");
      if (status == MASW_STATUS_FOUND) {
        // FP64 multisection of [c[found-1], c[found]]: 64 points per round,
        // both ends included, one per lane; the new bracket is the first
        // sign change.  The first round also yields the layer-denominator
        // sign masks at the two grid points (pole flag).
        double lo = c64[found - 1], hi = c64[found];
        const double tol = kRefineRel * hi;
        for (int r = 0; r < 24; ++r) {
          const double w = hi - lo;
          const double c = (lane == 63) ? hi : lo + w * (double(lane) / 63.0);
          uint64_t dm = 0;
          const int sg = det_sign<double, true>(c, k64, L64, N, &dm);
          if (r == 0 && __shfl(dm, 0, 64) != __shfl(dm, 63, 64)) status |= MASW_FLAG_POLE;
          int s_c = 0, p_c = 0, unused;
          const int f = wave_first_change(sg, &s_c, &p_c, &unused);
          n_refine += 64ull;
          if (f < 0 || s_c == kNaNSign || p_c == kNaNSign) break;
          const double nhi = (f == 63) ? hi : lo + w * (double(f) / 63.0);
          const double nlo = lo + w * (double(f - 1) / 63.0);
          lo = nlo;
          hi = nhi;
          if (!a.refine || hi - lo <= tol) break;
        }
        if (a.refine) c_ref = 0.5 * (lo + hi);
      }
      if (tid == 0) {
        a.out_idx[g] = found;
        a.out_status[g] = status;
        a.out_ct[g] = c64[found];
        if (a.out_cref) a.out_cref[g] = c_ref;
      }
    }
  }
  if (tid == 0) {
    atomicAdd(&a.counters->sweep, n_sweep);
    atomicAdd(&a.counters->check, n_check);
    atomicAdd(&a.counters->refine, n_refine);
    atomicAdd(&a.counters->useful, n_useful);
  }
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

// --------------------------------------------------------- host launchers --
template <int MODE>
static const void* sweep_symbol_mode(int G) {
  switch (G) {
    case 1: return reinterpret_cast<const void*>(&sweep_kernel<MODE, 1>);
    case 2: return reinterpret_cast<const void*>(&sweep_kernel<MODE, 2>);
    case 4: return reinterpret_cast<const void*>(&sweep_kernel<MODE, 4>);
    case 8: return reinterpret_cast<const void*>(&sweep_kernel<MODE, 8>);
    case 16: return reinterpret_cast<const void*>(&sweep_kernel<MODE, 16>);
  }
  return nullptr;
}

static const void* sweep_symbol(int mode, int G) {
  return mode == kModeFP64 ? sweep_symbol_mode<kModeFP64>(G) : sweep_symbol_mode<kModeSplit>(G);
}

int sweep_blocks_per_cu(int mode, int G) {
  const void* f = sweep_symbol(mode, G);
  if (!f) return 0;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, 64 * G, 0) != hipSuccess) return 0;
  return n;
}

hipError_t launch_sweep(int mode, int G, int blocks, hipStream_t s, const SweepArgs& a) {
  const void* f = sweep_symbol(mode, G);
  if (!f) return hipErrorInvalidValue;
  void* args[] = {const_cast<SweepArgs*>(&a)};
  return hipLaunchKernel(f, dim3(blocks), dim3(64 * G), args, 0, s);
}

hipError_t launch_prep(const PrepArgs& a, int single_N, int single_W, hipStream_t s) {
  hipLaunchKernelGGL(zero_counters_kernel, dim3(1), dim3(256), 0, s, a.counters);
  hipLaunchKernelGGL(prep_grid_kernel, dim3((a.n_c + 255) / 256), dim3(256), 0, s, a.c_in, a.n_c,
                     a.c64, a.c32, a.counters);
  hipLaunchKernelGGL(prep_models_kernel, dim3((a.n_models + 127) / 128), dim3(128), 0, s, a,
                     single_N, single_W);
  if (a.n_lam > 0) {
    const int nb = (a.n_lam + 255) / 256;
    hipLaunchKernelGGL(prep_lambda_kernel, dim3(nb), dim3(256), 0, s, a);
    hipLaunchKernelGGL(order_scan_kernel, dim3(1), dim3(kBuckets), 0, s, a.counters);
    hipLaunchKernelGGL(order_scatter_kernel, dim3(nb), dim3(256), 0, s, a);
  }
  return hipGetLastError();
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
