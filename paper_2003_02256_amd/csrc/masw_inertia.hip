// The inertia-count search as a launch of its own: the variant for many
// wavelengths per SIMD, and the choice between the two variants
// (masw_inertia_kernel.hpp).
#define MASW_COEFF_POLICY 1
#include "masw_inertia_kernel.hpp"

namespace masw {

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
  if (waves <= 4 * int64_t(cus)) return launch_inertia_lone(a, unsigned(blocks), chunk, s);  // one per SIMD
  hipLaunchKernelGGL(inertia_kernel, dim3(unsigned(blocks)), dim3(64 * kInertiaWaves), 0, s, a, chunk);
  return hipGetLastError();
}

}  // namespace masw
