// Test-only probe: evaluates the device special functions of the sweep
// (paper_2003_02256_amd/csrc/masw_special.hpp) on arrays, so that
// tests/test_gpu_special.py can compare them with high-precision references
// over their whole argument ranges.  Built beside the tests by
// paper_2003_02256_amd/build.py; not part of libmasw.so.
#include <hip/hip_runtime.h>

#include "masw_special.hpp"

namespace {

enum { kExpm1Neg = 0, kSin2Sincos = 1, kRcp = 2, kRsqrt = 3, kRcpSeed = 4, kRsqrtSeed = 5, kChShc = 6 };

template <typename T>
__global__ void probe_kernel(int kind, const double* __restrict__ x, double* __restrict__ y0,
                             double* __restrict__ y1, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T v = T(x[i]);
  double a = 0.0, b = 0.0;
  if (kind == kExpm1Neg) {
    a = double(masw::special::expm1_neg(v));
  } else if (kind == kSin2Sincos) {
    T s2, sc;
    masw::special::sin2_sincos(v, &s2, &sc);
    a = double(s2);
    b = double(sc);
  } else if (kind == kChShc) {
    T ch, shc;
    masw::special::ch_shc(v, &ch, &shc);
    a = double(ch);
    b = double(shc);
  } else if (kind == kRcp) {
    a = double(masw::special::rcp(v));
  } else if (kind == kRsqrt) {
    a = double(masw::special::rsqrt(v));
  } else if (kind == kRcpSeed) {  // the hardware estimates the refinements start from
    if constexpr (sizeof(T) == 8) a = __builtin_amdgcn_rcp(v); else a = double(__builtin_amdgcn_rcpf(v));
  } else if (kind == kRsqrtSeed) {
    if constexpr (sizeof(T) == 8) a = __builtin_amdgcn_rsq(v); else a = double(__builtin_amdgcn_rsqf(v));
  }
  y0[i] = a;
  y1[i] = b;
}

}  // namespace

// Host arrays in and out: x[n] -> y0[n], y1[n] (y1 is sin x cos x for
// kind 1, sinh(sqrt x)/sqrt(x) for kind 6 (y0: (cosh sqrt(x) - 1)/x), else 0;
// kinds 4 and 5 are the raw hardware reciprocal and reciprocal square root
// estimates).  fp32 != 0 evaluates the FP32 variant on float(x).
// Returns 0 or a hipError_t code.
extern "C" int probe_special(int fp32, int kind, const double* x, double* y0, double* y1, int n) {
  if (n <= 0) return 0;
  const size_t bytes = size_t(n) * sizeof(double);
  double *dx = nullptr, *d0 = nullptr, *d1 = nullptr;
  hipError_t e = hipMalloc(&dx, bytes);
  if (e == hipSuccess) e = hipMalloc(&d0, bytes);
  if (e == hipSuccess) e = hipMalloc(&d1, bytes);
  if (e == hipSuccess) e = hipMemcpy(dx, x, bytes, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    const dim3 grid((n + 255) / 256), block(256);
    if (fp32)
      hipLaunchKernelGGL(probe_kernel<float>, grid, block, 0, 0, kind, dx, d0, d1, n);
    else
      hipLaunchKernelGGL(probe_kernel<double>, grid, block, 0, 0, kind, dx, d0, d1, n);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpy(y0, d0, bytes, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(y1, d1, bytes, hipMemcpyDeviceToHost);
  if (dx) (void)hipFree(dx);
  if (d0) (void)hipFree(d0);
  if (d1) (void)hipFree(d1);
  return int(e);
}
