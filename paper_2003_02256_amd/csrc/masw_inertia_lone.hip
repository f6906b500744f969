// The inertia-count search kernel for launches of at most one wavefront per
// SIMD, with its polynomial coefficients in VGPRs (masw_inertia_kernel.hpp).
#define MASW_COEFF_POLICY 2
#include "masw_inertia_kernel.hpp"

namespace masw {

hipError_t launch_inertia_lone(const SweepArgs& a, unsigned blocks, int chunk, hipStream_t s) {
  hipLaunchKernelGGL(inertia_lone_kernel, dim3(blocks), dim3(64 * kInertiaWaves), 0, s, a, chunk);
  return hipGetLastError();
}

}  // namespace masw
