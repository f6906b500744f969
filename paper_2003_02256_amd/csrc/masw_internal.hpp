// Device-memory layout shared by the HIP kernels and the host runtime.
//
// HBM layout of one launch (all arrays in the context's arena):
//   ModelDesc     models[n_models]        32 B each
//   LayerRec64    layers64[R]             64 B each, R = sum_m (N_m + 1)
//   LayerRec32    layers32[R]             32 B each (FP32 copy for the sweep)
//   double/float  c64[], c32[]            test-velocity grids
//   double        lam_k[L]                k = 2 pi / lambda per wavelength
//   int32         lam_model[L]            model of each wavelength
//   int32         order[L]                work items, longest-expected-first
//   counters                              queue head, work counters, histogram
// Per-layer records hold only what the determinant needs, already divided
// by mu_ref = rho_hs beta_hs^2 so that the scaled matrix K / (k mu_ref)
// depends on k only through t = k h.
#pragma once
#include <stdint.h>

#include "masw.h"

namespace masw {

constexpr int kNoSign = 0x7f;        // "no predecessor" marker in the sign scan
constexpr int kNaNSign = 2;          // sign code of a NaN determinant
constexpr int kBuckets = 256;        // work-order buckets
constexpr double kRefineRel = 1e-9;  // refinement bracket width / c_hi

template <typename T>
struct alignas(8 * sizeof(T)) LayerRec {
  T ia2;  // 1 / alpha^2
  T ib2;  // 1 / beta^2
  T rh;   // rho / mu_ref
  T mh;   // mu / mu_ref
  T h;    // thickness (0 for the half-space record)
  T aux;   // half-space record: mu_ref (Pa); 0 otherwise
  T pad1, pad2;
};
using LayerRec64 = LayerRec<double>;
using LayerRec32 = LayerRec<float>;

struct alignas(32) ModelDesc {
  int32_t n_layers;    // N
  int32_t layer_base;  // first record of this model (N layers, then half-space)
  int32_t c_base;      // first grid point in the grid pool
  int32_t n_c;         // grid points
  int32_t lam_base;    // first wavelength (flattened index)
  int32_t n_lam;       // wavelengths
  int32_t valid;       // 1 if the model and its grid passed validation
  int32_t pad;
};

// Counters written by the kernels (one block in the arena, zeroed per call).
struct alignas(64) Counters {
  uint32_t queue_head;        // next work item
  uint32_t grid_bad;          // nonzero if the c grid failed validation
  uint32_t pad0[14];
  unsigned long long useful;  // sum of idx + 1
  unsigned long long sweep;   // sweep evaluations
  unsigned long long check;   // FP64 re-check evaluations
  unsigned long long refine;  // refinement evaluations
  uint32_t hist[kBuckets];    // work-order histogram, then bucket offsets
};

struct SweepArgs {
  const ModelDesc* models;
  const LayerRec64* layers64;
  const LayerRec32* layers32;
  const double* c64;
  const float* c32;
  const double* lam_k;
  const int32_t* lam_model;
  const int32_t* order;
  int32_t n_items;
  int32_t refine;  // 1 = compute c_ref
  Counters* counters;
  double* out_ct;
  int32_t* out_idx;
  int32_t* out_status;
  double* out_cref;  // may be null
};

struct PrepArgs {
  // raw flattened inputs (device)
  int32_t n_models;
  const int32_t* layer_off;
  const double* h;
  const double* alpha;
  const double* beta;
  const double* rho;
  const int32_t* lambda_off;
  const double* lambda;
  const double* c_in;  // shared grid [n_c]
  int32_t n_c;
  // outputs
  ModelDesc* models;
  LayerRec64* layers64;
  LayerRec32* layers32;
  double* c64;
  float* c32;
  double* lam_k;
  int32_t* lam_model;
  uint8_t* lam_bucket;
  int32_t* order;
  int32_t n_lam;
  Counters* counters;
};

struct SignMapArgs {
  const ModelDesc* models;
  const LayerRec64* layers64;
  const LayerRec32* layers32;
  const double* c64;
  const double* lam_k;
  int32_t n_lam;
  int32_t n_c;
  int8_t* sigma;
  double* logabs;  // may be null
};

}  // namespace masw
