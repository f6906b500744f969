// FP64 noise band of each pick's bracket (opt-in: MASW_CHECK_NOISE).
//
// The sweep decides a pick by the sign of det K at the two grid points of its
// bracket.  A grid point c is in the FP64 noise band when the first-order
// relative error bound of an FP64 determinant, cond_2(K(c)) 2(N+1) 2^-53,
// reaches a threshold (masw_opts.noise_threshold, 1e-2 by default); a pick
// with a bracket point in the band may differ from an exact computation's,
// and MASW_FLAG_NOISE marks it.
//
// Below the half-space's S velocity K(c) is real symmetric, so cond_2 is
// max|lambda| / min|lambda| over its eigenvalues, and c is in the band iff K
// has an eigenvalue in [-s, s], s = max|lambda| / T,
// T = threshold 2^53 / (2(N+1)).
// The number of eigenvalues of K below x is the number of negative
// eigenvalues of the 2x2 block pivots of the block LDL^T elimination of
// K - x I (Sylvester's law of inertia), so the eigenvalues in an interval are
// counted with two eliminations, each of the same O(N) recurrence as the
// determinant's.
//  1. B = ||K||_inf >= max|lambda|.  No eigenvalue in [-B/T, B/T] (two
//     eliminations) means no eigenvalue in [-s, s]: not in the band.  This
//     settles almost every point.
//  2. Otherwise the extreme eigenvalues are bisected with the same counts to
//     get max|lambda|, and the eigenvalues in [-s, s] are counted.
// Above the half-space's S velocity K is complex and no point is tested.
// A non-finite pivot marks the point as in the band.
//
// Two lanes per wavelength, one per bracket end; the wavelength is flagged if
// either end is in the band.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "masw.h"
#include "masw_host.hpp"
#include "masw_internal.hpp"
#include "masw_math.hpp"
#include "masw_noise.hpp"

namespace masw {
namespace {

constexpr int kNoiseThreads = 256;
using noise::in_band;

struct NoiseArgsDev {
  const ModelDesc* models;
  const LayerRec64* layers64;
  const double* c64;
  const double* lam_k;
  const int32_t* lam_model;
  const int32_t* idx;
  int32_t* status;
  int64_t n_lam;
  double threshold;
};

__global__ __launch_bounds__(kNoiseThreads) void noise_kernel(NoiseArgsDev a) {
  const int64_t t = int64_t(blockIdx.x) * kNoiseThreads + threadIdx.x;
  const int64_t g = t >> 1;  // wavelength
  const int end = int(t & 1);  // 0: c[idx-1], 1: c[idx]
  const bool active = g < a.n_lam;
  int status = 0;
  bool band = false;
  if (active) {
    status = a.status[g];
    const int i = a.idx[g];
    if ((status & 0xFF) == MASW_STATUS_FOUND && i >= 1) {
      const ModelDesc d = a.models[a.lam_model[g]];
      if (d.valid && i < d.n_c) {
        const LayerRec64* L = a.layers64 + d.layer_base;
        const double c = a.c64[d.c_base + i - 1 + end];
        if (c * c * L[d.n_layers].ib2 < 1.0) band = in_band(c, a.lam_k[g], L, d.n_layers, a.threshold);
      }
    }
  }
  const int other = __shfl_xor(int(band), 1, 64);  // the other end, next lane
  if (active && end == 0 && (band || other)) a.status[g] = status | MASW_FLAG_NOISE;
}

// Served requests with MASW_CHECK_NOISE, after the tick that finished
// them: block b takes request b of the list, two threads per wavelength as
// above.  The picks and statuses are the request's outputs in pinned host
// memory; the grid is the request's staged copy in its pool block.
__global__ __launch_bounds__(kNoiseThreads) void serve_noise_kernel(ServeNoiseList list, const int32_t* out_idx,
                                                                   int32_t* out_status, double threshold) {
  const SlotDesc& d = list.slot[blockIdx.x];
  const double* c64 = d.raw + (d.N + 3 * (d.N + 1) + d.W);
  for (int t = threadIdx.x; t < 2 * d.W; t += kNoiseThreads) {
    const int g = t >> 1, end = t & 1;
    const int o = d.out_base + g;
    const int status = out_status[o];
    const int i = out_idx[o];
    bool band = false;
    if ((status & 0xFF) == MASW_STATUS_FOUND && i >= 1 && i < d.n_c) {
      const double c = c64[i - 1 + end];
      const LayerRec64* L = as_global(d.L64);
      if (c * c * L[d.N].ib2 < 1.0) band = in_band(c, d.lam_k[g], L, d.N, threshold);
    }
    const int other = __shfl_xor(int(band), 1, 64);
    if (end == 0 && (band || other)) out_status[o] = status | MASW_FLAG_NOISE;
  }
}

}  // namespace

hipError_t launch_noise_check(const ModelDesc* models, const LayerRec64* layers64, const double* c64,
                              const double* lam_k, const int32_t* lam_model, const int32_t* idx,
                              int32_t* status, int64_t n_lam, double threshold, hipStream_t s) {
  if (n_lam <= 0) return hipSuccess;
  NoiseArgsDev a{models, layers64, c64, lam_k, lam_model, idx, status, n_lam, threshold};
  const int64_t blocks = (2 * n_lam + kNoiseThreads - 1) / kNoiseThreads;
  hipLaunchKernelGGL(noise_kernel, dim3(unsigned(blocks)), dim3(kNoiseThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_serve_noise(const ServeNoiseList& list, const int32_t* out_idx, int32_t* out_status,
                              double threshold, hipStream_t s) {
  if (list.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(serve_noise_kernel, dim3(unsigned(list.n)), dim3(kNoiseThreads), 0, s, list, out_idx,
                     out_status, threshold);
  return hipGetLastError();
}

}  // namespace masw
