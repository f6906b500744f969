// The inertia-count search as a launch of its own (MASW_SEARCH_INERTIA on the
// curve and batch calls): the kernel, compiled by two translation units.
// masw_inertia.hip builds the variant for many wavelengths per SIMD (FP64
// polynomial coefficients materialised in SGPRs where used, four wavefronts
// per SIMD: MASW_COEFF_POLICY 1); masw_inertia_lone.hip builds the variant
// for launches of at most one wavefront per SIMD, with every coefficient in
// VGPRs (MASW_COEFF_POLICY 2), where scalar moves would take issue slots from
// the lone wavefront's vector instructions.  The search itself is in masw_inertia.hpp; both variants
// compute bitwise the same results.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "masw.h"
#include "masw_host.hpp"
#include "masw_inertia.hpp"
#include "masw_internal.hpp"

#if MASW_COEFF_POLICY == 2
#define MASW_INERTIA_KERNEL inertia_lone_kernel
#define MASW_INERTIA_WAVES_PER_EU 1
#else
#define MASW_INERTIA_KERNEL inertia_kernel
#define MASW_INERTIA_WAVES_PER_EU 4
#endif

namespace masw {
namespace {

using inertia::Tally;
using inertia::wave_sum;

constexpr int kInertiaWaves = 4;  // wavefronts (wavelengths) per workgroup

// One wavelength: search, refinement and outputs.  Returns the pick (-1: none).
__device__ __forceinline__ int run_wavelength(const SweepArgs& a, int g, int pred, Tally& t) {
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
// (round P of search()).  The variant for many wavelengths is held to four
// wavefronts per SIMD (at most 128 VGPRs; it spills some values outside its
// hot loops), which ran the 4096-model batch 2.7% faster than three
// wavefronts (153 VGPRs, no spill); with the earlier coefficient placement,
// three wavefronts had run it 6% faster than the two of an unconstrained
// allocation.  The variant for launches of at most one wavefront per SIMD is
// not held, and takes its polynomial coefficients from VGPRs
// (masw_special.hpp).
__global__ __launch_bounds__(64 * kInertiaWaves) __attribute__((amdgpu_waves_per_eu(MASW_INERTIA_WAVES_PER_EU)))
void MASW_INERTIA_KERNEL(SweepArgs a, int chunk) {
  __shared__ unsigned long long s_cnt[kInertiaWaves][7];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  stamp_start(a.tstamp, 1);
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
  if (threadIdx.x < 8) {  // this workgroup's row of a.wg_counts (see SweepArgs)
    unsigned long long sum = 0;
    if (threadIdx.x < 7)
      for (int w = 0; w < kInertiaWaves; ++w) sum += s_cnt[w][threadIdx.x];
    constexpr int kCol[8] = {5, 6, 7, 0, 1, 2, 3, 4};  // s_cnt order to the row's
    if (a.wg_counts) {
      a.wg_counts[size_t(blockIdx.x) * kWgCounts + kCol[threadIdx.x]] = sum;
    } else if (sum) {
      Counters* c = a.counters;
      unsigned long long* dst[8] = {&c->inertia_evals, &c->inertia_entries, &c->inertia_pivots, &c->sweep,
                                    &c->check,         &c->refine,          &c->useful,          &c->helper};
      atomicAdd(dst[threadIdx.x], sum);
    }
  }
  stamp_end(a.tstamp);
}

}  // namespace

// The lone-wavefront variant's launch (masw_inertia_lone.hip).
hipError_t launch_inertia_lone(const SweepArgs& a, unsigned blocks, int chunk, hipStream_t s);

}  // namespace masw
