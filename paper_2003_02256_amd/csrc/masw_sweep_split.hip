// The split path's batch sweep kernels (FP32 sweep, FP64 re-check and
// refinement; masw_sweep.hpp), in a translation unit of their own: every
// FP64 polynomial coefficient is materialised in SGPRs where it is used
// (MASW_COEFF_POLICY 1), which keeps these kernels, whose FP32 sweep needs
// few VGPRs, at four to five wavefronts per SIMD.
#define MASW_COEFF_POLICY 1
#include "masw_sweep.hpp"

namespace masw {

template <bool MISFIT>
static const void* split_symbol(int G) {
  switch (G) {
    case 1: return reinterpret_cast<const void*>(&sweep_kernel<kModeSplit, 1, MISFIT>);
    case 2: return reinterpret_cast<const void*>(&sweep_kernel<kModeSplit, 2, MISFIT>);
    case 4: return reinterpret_cast<const void*>(&sweep_kernel<kModeSplit, 4, MISFIT>);
    case 8: return reinterpret_cast<const void*>(&sweep_kernel<kModeSplit, 8, MISFIT>);
    case 16: return reinterpret_cast<const void*>(&sweep_kernel<kModeSplit, 16, MISFIT>);
  }
  return nullptr;
}

const void* split_sweep_symbol(int G, bool misfit) {
  return misfit ? split_symbol<true>(G) : split_symbol<false>(G);
}

const void* split_fused_symbol() { return reinterpret_cast<const void*>(&fused_sweep_kernel<kModeSplit>); }

}  // namespace masw
