// Zero/pole classification of determinant sign changes with an independent
// secular function.
//
// sign(det K) of the stiffness formulation (Section 2.1) changes at the zeros
// of the dispersion function and at the poles where some layer denominator
// D_j changes sign.  This kernel evaluates the dispersion function in a
// formulation with no denominators, the Haskell-Thomson propagator of the
// P-SV equations of motion, and shares no arithmetic with the stiffness path.
//
// State and system.  For v = (u_x, -i u_z, tau_xz / (k mu_ref),
// -i tau_zz / (k mu_ref)) and zeta = k z (z down), a layer obeys
// dv/dzeta = A v with a real 4x4 matrix A (entries in `system_matrix` below)
// whose eigenvalues are +-r, +-s (u = r^2 = 1 - c^2/alpha^2,
// w = s^2 = 1 - c^2/beta^2); mu_ref is the half-space's rho beta^2.
//
// Propagator.  A^2 has the two eigenvalues u and w, so every even function of
// A is a first-degree polynomial in A^2 and every odd one is A times such a
// polynomial (Cayley-Hamilton).  With U = t^2 u, W = t^2 w and the divided
// differences of the entire functions cosh(t sqrt(z)) and
// sinh(t sqrt(z)) / sqrt(z) at z = u, w:
//     exp(-A t) = cosh(A t) - sinh(A t) = a0 I + a1 A^2 - b0 A - b1 A^3,
//     a1 = t^2 sum_{n>=1} h_{n-1} / (2n)!,   a0 = 1 - U W sum_{n>=2} h_{n-2} / (2n)!,
//     b1 = t^3 sum_{n>=1} h_{n-1} / (2n+1)!, b0 = t (1 - U W sum_{n>=2} h_{n-2} / (2n+1)!),
// where h_n = sum_{i=0}^{n} U^i W^(n-i) (h_0 = 1, h_n = U h_{n-1} + W^n).
// Nothing here divides by u - w, and every quantity is real for real c on
// either side of alpha and beta.  Steps satisfy t max(|u|, |w|)^(1/2) <= 1,
// so |U|, |W| <= 1 and twelve terms reach the FP64 rounding.
//
// Secular function.  The half-space's solutions decaying with depth (c below
// its beta) are P = (1, r, -2r, g - 2) and SV = (s, 1, g - 2, -2s),
// g = c^2/beta^2.  The pair is carried up across every layer by exp(-A k h)
// in equal steps of at most one unit of k dz max(|r|, |s|), and after each
// step replaced by a nearly orthonormal basis of its span with the same
// orientation (Gram-Schmidt: both columns divided by positive numbers).  At
// the surface F = the determinant of its two traction rows, which vanishes
// exactly at the modes; the positive factors dropped by the
// orthonormalisation leave its sign and zeros unchanged.
//
// Work split.  One wavefront per wavelength, four per workgroup.  Lane l
// evaluates F at point l
// of 64 equally spaced points of the bracket: a different sign at the two
// ends is a mode, and the first lane whose sign differs from the lower end's
// gives the next bracket, 63 times narrower (multisection), until it is no
// wider than 1e-12 c_test[idx].  Control flow is uniform across the wavefront
// (ballots and shuffles); each lane's layer loop runs its own step count.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "masw.h"
#include "masw_host.hpp"

namespace masw {
namespace {

constexpr int kClassifyWaves = 4;           // wavefronts (wavelengths) per workgroup
constexpr int kMaxStepsPerLayer = 1 << 16;  // beyond this a layer is not crossed
constexpr int kMaxRounds = 8;               // 63^8 > 2e14
constexpr int kTerms = 12;                  // series terms, |U|, |W| <= 1
constexpr double kRootTol = 1e-12;

// The doubles nearest to 1/m!, m = 0 .. 2 kTerms + 1.
__constant__ double kInvFact[2 * kTerms + 2] = {
    1.0, 1.0, 0.5, 0.16666666666666666, 0.041666666666666664,
    0.008333333333333333, 0.001388888888888889, 0.0001984126984126984, 2.48015873015873e-05, 2.7557319223985893e-06,
    2.755731922398589e-07, 2.505210838544172e-08, 2.08767569878681e-09, 1.6059043836821613e-10, 1.1470745597729725e-11,
    7.647163731819816e-13, 4.779477332387385e-14, 2.8114572543455206e-15, 1.5619206968586225e-16, 8.22063524662433e-18,
    4.110317623312165e-19, 1.9572941063391263e-20, 8.896791392450574e-22, 3.868170170630684e-23, 1.6117375710961184e-24,
    6.446950284384474e-26};

struct ClassifyArgsDev {
  const int32_t* layer_off;
  const double* h;
  const double* alpha;
  const double* beta;
  const double* rho;
  const int32_t* lambda_off;
  const double* lambda;
  const double* c;
  const int32_t* idx;
  int32_t* cls;
  double* c_sec;
  unsigned long long* counters;  // [3]: evaluations, layers crossed, steps
  int64_t n_lam;
  int32_t n_models;
  int32_t n_c;
};

__device__ __forceinline__ bool finite_pos(double v) { return v > 0.0 && v < __builtin_inf(); }

// The six entries of A other than the constants A[0,1] = 1, A[3,2] = -1 (see
// the file comment for the state; every other entry is 0), from the layer's
// M = rho alpha^2, mu = rho beta^2, their reciprocals, rho c^2 and 1/mu_ref.
struct SysMat {
  double a02, a10, a13, a20, a23, a31;
};

__device__ __forceinline__ SysMat system_matrix(double M, double mu, double iM, double imu, double rc2,
                                              double mu_ref, double i_ref) {
  const double lam = M - 2.0 * mu;
  SysMat o;
  o.a02 = mu_ref * imu;
  o.a10 = -lam * iM;
  o.a13 = mu_ref * iM;
  o.a20 = (4.0 * mu * (lam + mu) * iM - rc2) * i_ref;
  o.a23 = lam * iM;
  o.a31 = -rc2 * i_ref;
  return o;
}

// exp(-A t) for one step (file comment), given u = r^2, w = s^2, row-major.
// A couples E = (u_x, tau_zz) only with O = (u_z, tau_xz): in that order
// A = [[0, X], [Y, 0]] with X = [[1, a02], [a31, -1]], Y = [[a10, a13],
// [a20, a23]], so A^2 = diag(XY, YX) and A^3 = [[0, XYX], [YXY, 0]], and
// exp(-A t) = [[a0 I + a1 XY, -(b0 X + b1 XYX)], [-(b0 Y + b1 YXY), a0 I + a1 YX]].
__device__ __forceinline__ void step_propagator(const SysMat& m, double u, double w, double t, double P[16]) {
  const double U = t * t * u, W = t * t * w;
  double sc1 = 0.0, ss1 = 0.0, sc0 = 0.0, ss0 = 0.0;
  double h_prev = 0.0, h_cur = 1.0, Wp = 1.0;  // h_{n-2}, h_{n-1}
#pragma unroll
  for (int n = 1; n <= kTerms; ++n) {
    sc1 = __builtin_fma(h_cur, kInvFact[2 * n], sc1);
    ss1 = __builtin_fma(h_cur, kInvFact[2 * n + 1], ss1);
    if (n >= 2) {
      sc0 = __builtin_fma(h_prev, kInvFact[2 * n], sc0);
      ss0 = __builtin_fma(h_prev, kInvFact[2 * n + 1], ss0);
    }
    Wp *= W;
    const double h_next = __builtin_fma(U, h_cur, Wp);
    h_prev = h_cur;
    h_cur = h_next;
  }
  const double UW = U * W;
  const double a1 = t * t * sc1;
  const double a0 = 1.0 - UW * sc0;
  const double b1 = t * t * t * ss1;
  const double b0 = t * (1.0 - UW * ss0);
  // XY and YX (rows/columns in E and O order)
  const double xy00 = __builtin_fma(m.a02, m.a20, m.a10), xy01 = __builtin_fma(m.a02, m.a23, m.a13);
  const double xy10 = __builtin_fma(m.a31, m.a10, -m.a20), xy11 = __builtin_fma(m.a31, m.a13, -m.a23);
  const double yx00 = __builtin_fma(m.a13, m.a31, m.a10), yx01 = __builtin_fma(m.a10, m.a02, -m.a13);
  const double yx10 = __builtin_fma(m.a23, m.a31, m.a20), yx11 = __builtin_fma(m.a20, m.a02, -m.a23);
  // XYX = (XY) X and YXY = (YX) Y
  const double xyx00 = __builtin_fma(xy01, m.a31, xy00), xyx01 = __builtin_fma(xy00, m.a02, -xy01);
  const double xyx10 = __builtin_fma(xy11, m.a31, xy10), xyx11 = __builtin_fma(xy10, m.a02, -xy11);
  const double yxy00 = __builtin_fma(yx01, m.a20, yx00 * m.a10), yxy01 = __builtin_fma(yx01, m.a23, yx00 * m.a13);
  const double yxy10 = __builtin_fma(yx11, m.a20, yx10 * m.a10), yxy11 = __builtin_fma(yx11, m.a23, yx10 * m.a13);
  // state index of E = (0, 3) and O = (1, 2)
  P[0 * 4 + 0] = __builtin_fma(a1, xy00, a0);
  P[0 * 4 + 3] = a1 * xy01;
  P[3 * 4 + 0] = a1 * xy10;
  P[3 * 4 + 3] = __builtin_fma(a1, xy11, a0);
  P[1 * 4 + 1] = __builtin_fma(a1, yx00, a0);
  P[1 * 4 + 2] = a1 * yx01;
  P[2 * 4 + 1] = a1 * yx10;
  P[2 * 4 + 2] = __builtin_fma(a1, yx11, a0);
  P[0 * 4 + 1] = -__builtin_fma(b1, xyx00, b0);
  P[0 * 4 + 2] = -__builtin_fma(b1, xyx01, b0 * m.a02);
  P[3 * 4 + 1] = -__builtin_fma(b1, xyx10, b0 * m.a31);
  P[3 * 4 + 2] = -__builtin_fma(b1, xyx11, -b0);
  P[1 * 4 + 0] = -__builtin_fma(b1, yxy00, b0 * m.a10);
  P[1 * 4 + 3] = -__builtin_fma(b1, yxy01, b0 * m.a13);
  P[2 * 4 + 0] = -__builtin_fma(b1, yxy10, b0 * m.a20);
  P[2 * 4 + 3] = -__builtin_fma(b1, yxy11, b0 * m.a23);
}

// Replace the columns (x, y) by a nearly orthonormal basis of their span
// with the same orientation: x divided by about its norm, then y less its
// component along x and divided by about its norm.  Only the span, the
// orientation (both divisors positive) and a well-conditioned basis matter to
// the sign and the zeros of F, so the hardware reciprocal square root
// (relative error below 2^-21) serves as the divisor without refinement.
__device__ __forceinline__ void orthonormalize(double x[4], double y[4]) {
  const double ix = __builtin_amdgcn_rsq(x[0] * x[0] + x[1] * x[1] + x[2] * x[2] + x[3] * x[3]);
#pragma unroll
  for (int i = 0; i < 4; ++i) x[i] *= ix;
  const double d = x[0] * y[0] + x[1] * y[1] + x[2] * y[2] + x[3] * y[3];
#pragma unroll
  for (int i = 0; i < 4; ++i) y[i] = __builtin_fma(-d, x[i], y[i]);
  const double iy = __builtin_amdgcn_rsq(y[0] * y[0] + y[1] * y[1] + y[2] * y[2] + y[3] * y[3]);
#pragma unroll
  for (int i = 0; i < 4; ++i) y[i] *= iy;
}

// F(c) for wavenumber k and a model of N layers over a half-space (values at
// index N); c below the half-space's beta.  NaN if a layer needs more than
// kMaxStepsPerLayer steps.
__device__ double secular(double c, double k, const double* __restrict__ h, const double* __restrict__ al,
                          const double* __restrict__ be, const double* __restrict__ rh, int N,
                          unsigned* steps_taken) {
  const double c2 = c * c;
  const double mu_ref = rh[N] * be[N] * be[N];
  const double i_ref = 1.0 / mu_ref;
  const double g = c2 / (be[N] * be[N]);
  const double r = __builtin_sqrt(1.0 - c2 / (al[N] * al[N]));
  const double s = __builtin_sqrt(1.0 - g);
  double x[4] = {1.0, r, -2.0 * r, g - 2.0};
  double y[4] = {s, 1.0, g - 2.0, -2.0 * s};
  orthonormalize(x, y);
  for (int j = N - 1; j >= 0; --j) {
    const double a = al[j], b = be[j], rho = rh[j];
    const double M = rho * a * a, mu = rho * b * b;
    const double iM = 1.0 / M, imu = 1.0 / mu;
    const double rc2 = rho * c2;
    const double u = 1.0 - rc2 * iM;   // 1 - c^2/alpha^2
    const double w = 1.0 - rc2 * imu;  // 1 - c^2/beta^2
    const double q = __builtin_sqrt(__builtin_fmax(__builtin_fabs(u), __builtin_fabs(w)));
    const double kh = k * h[j];
    const double need = __builtin_ceil(kh * q);
    if (!(need <= double(kMaxStepsPerLayer))) return __builtin_nan("");
    const int steps = need < 1.0 ? 1 : int(need);
    *steps_taken += unsigned(steps);
    double P[16];
    step_propagator(system_matrix(M, mu, iM, imu, rc2, mu_ref, i_ref), u, w, kh / double(steps), P);
    for (int st = 0; st < steps; ++st) {
      double nx[4], ny[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        nx[i] = P[i * 4 + 0] * x[0] + P[i * 4 + 1] * x[1] + P[i * 4 + 2] * x[2] + P[i * 4 + 3] * x[3];
        ny[i] = P[i * 4 + 0] * y[0] + P[i * 4 + 1] * y[1] + P[i * 4 + 2] * y[2] + P[i * 4 + 3] * y[3];
      }
      orthonormalize(nx, ny);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        x[i] = nx[i];
        y[i] = ny[i];
      }
    }
  }
  return x[2] * y[3] - y[2] * x[3];
}

__device__ __forceinline__ int sgn(double v) { return int(v > 0.0) - int(v < 0.0); }

// Workgroups are dispatched to the eight XCDs round-robin (block b on XCD
// b mod 8), and each XCD has its own L2.  Within every run of 8 kXcdRun
// dispatched blocks, the blocks are renumbered so that each XCD takes kXcdRun
// consecutive block numbers: neighbouring wavelengths, which share a model's
// records and the output cache lines, stay in one L2, while the runs keep
// every XCD's share of the models mixed.  Blocks past the last whole run keep
// their numbers.  The renumbering is a bijection of [0, nb), so it changes no
// result.
constexpr unsigned kXcds = 8;
constexpr unsigned kXcdRun = 16;

__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
  constexpr unsigned span = kXcds * kXcdRun;
  if (b >= nb / span * span) return b;
  const unsigned base = b / span * span, w = b % span;
  return base + (w % kXcds) * kXcdRun + w / kXcds;
}

// Class and root of wavelength wl, by one whole wavefront.  Returns the
// multisection rounds run (uniform across the wavefront); *steps gets this
// lane's propagator steps and *n_layers the model's layer count.
__device__ int classify_one(const ClassifyArgsDev& a, int64_t wl, int lane, int* cls_out, double* root_out,
                            unsigned* steps_out, int* n_layers) {
  // model of wavelength wl: lambda_off[m] <= wl < lambda_off[m + 1]
  int m_lo = 0, m_hi = a.n_models;
  while (m_hi - m_lo > 1) {
    const int mid = (m_lo + m_hi) >> 1;
    if (int64_t(a.lambda_off[mid]) <= wl) m_lo = mid; else m_hi = mid;
  }
  const int m = m_lo;
  const int N = a.layer_off[m + 1] - a.layer_off[m];
  const double* h = a.h + a.layer_off[m];
  const int64_t r0 = int64_t(a.layer_off[m]) + m;
  const double* al = a.alpha + r0;
  const double* be = a.beta + r0;
  const double* rh = a.rho + r0;
  const int i = a.idx[wl];

  int cls;
  double root = __builtin_nan("");
  unsigned steps = 0;  // propagator steps of this lane
  int rounds = 0;
  if (i < 1 || i >= a.n_c) {
    cls = MASW_PICK_NONE;
  } else {
    // device validation of the model, the wavelength and the bracket
    bool bad = (N < 0 || N > MASW_MAX_LAYERS);
    for (int j = lane; !bad && j <= N; j += 64) {
      const double aj = al[j], bj = be[j], rj = rh[j];
      bool ok = finite_pos(aj) && finite_pos(bj) && finite_pos(rj) && aj > bj;
      if (j < N) ok = ok && finite_pos(h[j]);
      bad = !ok;
    }
    const double lam = a.lambda[wl];
    const double c_lo0 = a.c[i - 1], c_hi0 = a.c[i];
    bad = bad || !finite_pos(lam) || !finite_pos(c_lo0) || !finite_pos(c_hi0) || !(c_hi0 > c_lo0);
    if (__ballot(bad) != 0ull) {
      cls = MASW_PICK_INVALID;
    } else if (c_hi0 >= be[N]) {
      cls = MASW_PICK_LEAKY;
    } else {
      const double k = 2.0 * 3.14159265358979323846 / lam;
      const double tol = kRootTol * c_hi0;
      double lo = c_lo0, hi = c_hi0;
      int s_lo = 0;
      cls = MASW_PICK_MODE;
      for (int round = 0; round < kMaxRounds; ++round) {
        const double cl = lane == 63 ? hi : __builtin_fma(hi - lo, double(lane) * (1.0 / 63.0), lo);
        const double F = secular(cl, k, h, al, be, rh, N, &steps);
        ++rounds;
        const bool nan = !(F == F) || !(__builtin_fabs(F) < __builtin_inf());
        if (__ballot(nan) != 0ull) {
          cls = MASW_PICK_UNRESOLVED;
          break;
        }
        const int sg = sgn(F);
        if (round == 0) {
          s_lo = __shfl(sg, 0, 64);
          if (__shfl(sg, 63, 64) == s_lo) {
            cls = MASW_PICK_POLE;
            break;
          }
        }
        // first point whose sign differs from the lower end's (lane 63 does)
        const uint64_t diff = __ballot(lane >= 1 && sg != s_lo);
        const int l = __builtin_ctzll(diff);
        lo = __shfl(cl, l - 1, 64);
        hi = __shfl(cl, l, 64);
        if (hi - lo <= tol) break;
      }
      if (cls == MASW_PICK_MODE) root = 0.5 * (lo + hi);
    }
  }
  *cls_out = cls;
  *root_out = root;
  *steps_out = steps;
  *n_layers = N;
  return rounds;
}

__global__ __launch_bounds__(64 * kClassifyWaves) void classify_kernel(ClassifyArgsDev a) {
  __shared__ unsigned long long s_cnt[kClassifyWaves][3];
  const int lane = int(threadIdx.x) & 63;
  const int wave = int(threadIdx.x) >> 6;
  const unsigned vb = xcd_block(blockIdx.x, gridDim.x);
  const int64_t wl = int64_t(vb) * kClassifyWaves + wave;
  unsigned long long n_eval = 0, n_layer = 0, n_step = 0;
  if (wl < a.n_lam) {  // uniform across the wavefront
    int cls, N;
    double root;
    unsigned steps;
    const int rounds = classify_one(a, wl, lane, &cls, &root, &steps, &N);
    n_step = steps;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) n_step += __shfl_xor(n_step, off, 64);
    n_eval = 64ull * unsigned(rounds);
    n_layer = n_eval * unsigned(N);
    if (lane == 0) {
      a.cls[wl] = cls;
      if (a.c_sec) a.c_sec[wl] = root;
    }
  }
  // work counters: summed over the workgroup in LDS, one atomic per counter
  // and workgroup (device-scope atomics bypass the L2, so each costs a
  // memory write)
  if (lane == 0) {
    s_cnt[wave][0] = n_eval;
    s_cnt[wave][1] = n_layer;
    s_cnt[wave][2] = n_step;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    unsigned long long sum = 0;
#pragma unroll
    for (int w = 0; w < kClassifyWaves; ++w) sum += s_cnt[w][threadIdx.x];
    if (sum) atomicAdd(&a.counters[threadIdx.x], sum);
  }
}

__global__ void clear_counters_kernel(unsigned long long* c) {
  if (threadIdx.x < 3) c[threadIdx.x] = 0ull;
}

}  // namespace

hipError_t launch_classify(const ClassifyArgs& in, hipStream_t s) {
  if (in.n_lam <= 0) return hipSuccess;
  if (!in.counters) return hipErrorInvalidValue;
  ClassifyArgsDev a;
  a.layer_off = in.layer_off;
  a.h = in.h;
  a.alpha = in.alpha;
  a.beta = in.beta;
  a.rho = in.rho;
  a.lambda_off = in.lambda_off;
  a.lambda = in.lambda;
  a.c = in.c;
  a.idx = in.idx;
  a.cls = in.cls;
  a.c_sec = in.c_sec;
  a.n_lam = in.n_lam;
  a.n_models = in.n_models;
  a.n_c = in.n_c;
  a.counters = reinterpret_cast<unsigned long long*>(in.counters);
  // a kernel, not a memset, clears the counters, so a caller may capture the call
  hipLaunchKernelGGL(clear_counters_kernel, dim3(1), dim3(64), 0, s, a.counters);
  const int64_t blocks = (in.n_lam + kClassifyWaves - 1) / kClassifyWaves;
  hipLaunchKernelGGL(classify_kernel, dim3(unsigned(blocks)), dim3(64 * kClassifyWaves), 0, s, a);
  return hipGetLastError();
}

}  // namespace masw
