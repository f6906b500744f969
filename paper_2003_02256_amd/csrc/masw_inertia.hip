// The inertia-count search as a launch of its own (MASW_SEARCH_INERTIA on the
// curve and batch calls); the search itself is in masw_inertia.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "masw.h"
#include "masw_host.hpp"
#include "masw_inertia.hpp"
#include "masw_internal.hpp"

namespace masw {
namespace {

using inertia::Tally;
using inertia::wave_sum;

constexpr int kInertiaWaves = 4;  // wavefronts (wavelengths) per workgroup

// One wavelength: search, refinement and outputs.  Returns the pick (-1: none).
__device__ int run_wavelength(const SweepArgs& a, int g, int pred, Tally& t) {
  const int lane = threadIdx.x & 63;
  const int m = __builtin_amdgcn_readfirstlane(a.lam_model[g]);
  const ModelDesc d = a.models[m];
  const ItemOut o{a.out_ct + g, a.out_idx + g, a.out_status + g, a.out_cref ? a.out_cref + g : nullptr, a.refine,
                  a.refine_rel};
  const double k = a.lam_k[g];
  const int n_c = __builtin_amdgcn_readfirstlane(d.n_c);
  if (!(k == k)) {  // invalid model, grid or wavelength
    write_no_pick(o, MASW_STATUS_INVALID, lane == 0);
    return -1;
  }
  const int N = __builtin_amdgcn_readfirstlane(d.n_layers);
  const double* c64 = a.c64 + __builtin_amdgcn_readfirstlane(d.c_base);
  const LayerRec64* L = a.layers64 + __builtin_amdgcn_readfirstlane(d.layer_base);
  int sig_f = 0, prev_f = 0;
  const int found = inertia::search(c64, n_c, k, L, N, pred, &sig_f, &prev_f, t);
  if (found < 0) {
    write_no_pick(o, MASW_STATUS_NOT_FOUND, lane == 0);
    t.useful += (unsigned long long)n_c;
  } else {
    t.useful += (unsigned long long)(found + 1);
    t.refine += refine_and_write(o, c64, k, L, N, found, sig_f, prev_f);
  }
  return found;
}

// Persistent grid; counters stay in registers until the end.  With
// chunk = 1 (wavelengths no more than a few per wavefront) wavefront w of W
// takes wavelengths w, w + W, ...  Otherwise each wavefront claims runs of
// `chunk` consecutive wavelengths from an atomic queue, and within a run the
// picks of the previous wavelengths of the same model predict the next pick
// (round P of search()).  Three wavefronts per SIMD (at most 168 VGPRs,
// with a few spilled) ran the 4096-model batch 6% faster than the two that
// the unconstrained 173 VGPRs allow.
__global__ __launch_bounds__(64 * kInertiaWaves) __attribute__((amdgpu_waves_per_eu(3))) void inertia_kernel(
    SweepArgs a, int chunk) {
  __shared__ unsigned long long s_cnt[kInertiaWaves][7];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  Tally t;
  if (chunk <= 1) {
    const int W = gridDim.x * kInertiaWaves;
    for (int g = blockIdx.x * kInertiaWaves + wave; g < a.n_items; g += W) run_wavelength(a, g, -1, t);
  } else {
    for (;;) {
      unsigned q = 0;
      if (lane == 0) q = atomicAdd(&a.counters->queue_head, 1u);
      const int64_t first = int64_t(__shfl(q, 0, 64)) * chunk;
      if (first >= a.n_items) break;
      const int last = int(std::min<int64_t>(first + chunk, a.n_items));
      int model = -1, p1 = -1, p2 = -1;  // the last two picks of `model` in this run
      for (int g = int(first); g < last; ++g) {
        const int m = __builtin_amdgcn_readfirstlane(a.lam_model[g]);
        if (m != model) {
          model = m;
          p1 = p2 = -1;
        }
        const int pred = p1 < 1 ? -1 : (p2 < 1 ? p1 : max(1, 2 * p1 - p2));
        const int found = run_wavelength(a, g, pred, t);
        p2 = found < 0 ? -1 : p1;
        p1 = found;
      }
    }
  }
  const unsigned long long evals = wave_sum(t.evals), entries = wave_sum(t.entries), pivots = wave_sum(t.pivots);
  if (lane == 0) {
    s_cnt[wave][0] = evals;
    s_cnt[wave][1] = entries;
    s_cnt[wave][2] = pivots;
    s_cnt[wave][3] = t.scan;
    s_cnt[wave][4] = t.check;
    s_cnt[wave][5] = t.refine;
    s_cnt[wave][6] = t.useful;
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    unsigned long long sum = 0;
    for (int w = 0; w < kInertiaWaves; ++w) sum += s_cnt[w][threadIdx.x];
    Counters* c = a.counters;
    unsigned long long* dst[7] = {&c->inertia_evals, &c->inertia_entries, &c->inertia_pivots, &c->sweep,
                                  &c->check,         &c->refine,          &c->useful};
    if (sum) atomicAdd(dst[threadIdx.x], sum);
  }
}

}  // namespace

hipError_t launch_inertia(const SweepArgs& a, int cus, hipStream_t s, int* blocks_out) {
  *blocks_out = 0;
  if (a.n_items <= 0) return hipSuccess;
  static const int per_cu = [] {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(inertia_kernel),
                                                     64 * kInertiaWaves, 0) != hipSuccess || n < 1)
      n = 1;
    return n;
  }();
  const int64_t need = (int64_t(a.n_items) + kInertiaWaves - 1) / kInertiaWaves;
  const int64_t blocks = std::min<int64_t>(need, int64_t(cus) * per_cu);
  *blocks_out = int(blocks);
  // runs of consecutive wavelengths only when each wavefront gets many
  // (a run is searched in sequence), at most 16 so that runs balance
  const int64_t waves = blocks * kInertiaWaves;
  const int chunk = int(std::max<int64_t>(1, std::min<int64_t>(16, int64_t(a.n_items) / (4 * waves))));
  hipLaunchKernelGGL(inertia_kernel, dim3(unsigned(blocks)), dim3(64 * kInertiaWaves), 0, s, a, chunk);
  return hipGetLastError();
}

}  // namespace masw
