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
constexpr double kRefineRel = 1e-9;  // default refinement bracket width / c_hi
constexpr int kPrepThreads = 256;    // threads per staging block
constexpr int kLamBlock = 1024;      // wavelengths sorted by one staging block

template <typename T>
struct alignas(8 * sizeof(T)) LayerRec {
  T ia2;  // 1 / alpha^2
  T ib2;  // 1 / beta^2
  T rh;   // rho / mu_ref
  T mh;   // mu / mu_ref
  T h;    // thickness (0 for the half-space record)
  T aux;   // half-space record: mu_ref (Pa); 0 otherwise
  T zb;    // depth of the layer's bottom (m), for the work-order key of the
           // batch staging; 0 in served requests, which are not reordered
  T pad2;
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
  int32_t n_real;      // grid points c with c^2 / beta_hs^2 < 1 (K real, inertia counts exist): the
                       // leading part of the grid, where the split path sweeps in FP32
};

// Counters written by the kernels (one block in the arena, zeroed per call).
struct alignas(64) Counters {
  uint32_t queue_head;        // next work item
  uint32_t grid_bad;          // nonzero if the c grid failed validation
  uint32_t coop_stall;        // cooperative waits that reached their bound
  uint32_t tick_exit;         // serving: workgroups that have left their tick (never cleared)
  uint32_t pad0[12];
  unsigned long long useful;  // sum of idx + 1
  unsigned long long sweep;   // sweep evaluations
  unsigned long long check;   // FP64 re-check evaluations
  unsigned long long refine;  // refinement evaluations
  unsigned long long helper;  // sweep evaluations done by joining workgroups
  unsigned long long inertia_evals;    // inertia counts (MASW_SEARCH_INERTIA)
  unsigned long long inertia_entries;  // layer and sublayer element matrices formed by them
  unsigned long long inertia_pivots;   // 2x2 block pivots eliminated by them
  uint32_t hist[kBuckets];    // work-order histogram, then bucket offsets
};

// Shared sweep of one work item that idle workgroups may join (queue
// positions below SweepArgs::n_coop).  The item's grid is cut into rounds of
// 64 G positions; every workgroup on the item claims rounds from `next`,
// evaluates them and publishes one summary word per round, and the owning
// workgroup resolves the summaries in grid order, so the pick does not depend
// on who evaluated which round.  All fields are accessed with agent-scope
// atomics.
struct alignas(16) CoopItem {
  int32_t next;      // next round to claim
  int32_t stop;      // rounds after this one are not needed (INT32_MAX until a change is seen; -1 when closed)
  int32_t resolved;  // rounds resolved in grid order by the owner
  int32_t rounds;    // rounds in the sweep; 0 before the owner starts, -1 after the shared sweep ends
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
  double refine_rel;  // refinement bracket width / c_hi
  Counters* counters;
  double* out_ct;
  int32_t* out_idx;
  int32_t* out_status;
  double* out_cref;  // may be null
  // Cooperative tail: items at queue positions < n_coop may be joined by
  // workgroups that find the queue empty.
  int32_t n_coop;
  int32_t coop_stride;   // summary words per item (rounds of the longest sweep)
  CoopItem* coop;        // [n_coop]
  uint64_t* coop_sum;    // [n_coop * coop_stride] round summaries, 0 = not yet published
  int32_t* coop_active;  // [gridDim.x] item each workgroup owns in its shared sweep, or -1
  int32_t coop_window;   // rounds a joining workgroup may run ahead of the owner's resolution
  // Issue priority of a workgroup's wavefronts while it runs queue position
  // it: 2 for it < prio_hi, 1 for it < prio_mid, else 0 (0 = all off).
  int32_t prio_hi;
  int32_t prio_mid;
  // Algorithm 2 fused into the launch (misfit null: off): the workgroup that
  // finishes a model's last wavelength reduces the model's misfit.
  const double* c_e;          // [n_lam] experimental velocities
  double* misfit;             // [n_models]
  int32_t* model_left;        // [n_models] wavelengths not finished (set by the staging)
  const int32_t* lambda_off;  // [n_models + 1]
  // Work counts of each workgroup, [gridDim.x][kWgCounts] (plain stores; the
  // host sums them for masw_get_stats): one atomic add per workgroup and
  // counter on a shared cache line serialises at the end of a launch.
  unsigned long long* wg_counts;
  // A small single-model launch with the staging folded in (fused != 0, one
  // item per workgroup, the item of workgroup w is wavelength w): each
  // workgroup checks the raw model and grid itself, builds the model's layer
  // records in its LDS and takes k from its wavelength, so no staging launch
  // runs before the sweep.  Raw device inputs, as masw_model and the curve
  // call take them; models, layers64/32, c32, lam_k, lam_model and order are
  // unused.
  int32_t fused;
  int32_t fused_N;  // layers of the model (at most kFusedMaxLayers)
  const double* f_h;
  const double* f_alpha;
  const double* f_beta;
  const double* f_rho;
  const double* f_lambda;
  const double* f_c;
  int32_t f_n_c;
  // Launch timing (null: not timed): see stamp_start / stamp_end.
  unsigned long long* tstamp;
};
constexpr int kFusedG = 8;              // wavefronts per workgroup of a fused launch
constexpr int kFusedMaxLayers = 64;     // layers of a model that a fused launch stages in LDS
constexpr int kFusedMaxGrid = 16384;    // grid points that each workgroup of a fused launch checks
constexpr int kWgCounts = 8;  // sweep, check, refine, useful, helper, inertia evals, entries, pivots
constexpr int kMaxWgRows = 65536;  // workgroup rows reserved for wg_counts (above any launch's grid)

// Zero-state of the cooperative arrays (one launch before the sweep).
struct CoopInitArgs {
  CoopItem* coop;
  int32_t n_coop;
  uint64_t* coop_sum;
  uint64_t n_sum;
  int32_t* coop_active;
  int32_t n_active;
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
  uint32_t* grid_flags;  // [ceil(n_c / kPrepThreads)] 1 where a block of the grid failed its checks
  int32_t* model_left;   // fused misfit: [n_models] set to each model's wavelength count (else null)
  double* misfit;        // fused misfit: [n_models], NaN written here for a model with no wavelength
  unsigned long long* tstamp;  // launch timing of the job (null: not timed): its start
};

// Launch timing from the GPU's constant-rate real-time counter
// (s_memrealtime, the device's wall-clock rate), without host events: a
// timed job's slot holds [0] the start of its first kernel, [1] the start
// of its sweep (or inertia) kernel and [2] the end of that kernel's last
// workgroup.  Workgroup 0 of a launch is dispatched first, so its start
// stands for the launch's; the end is the largest of every workgroup's end
// (an atomic maximum, which needs no reset between uses of a slot since the
// counter only grows).
// (With j >= 0 the same reading goes to slot words i and j.)
__device__ __forceinline__ void stamp_start(unsigned long long* ts, int i, int j = -1) {
  if (ts && blockIdx.x == 0 && threadIdx.x == 0) {
    const unsigned long long t = __builtin_amdgcn_s_memrealtime();
    ts[i] = t;
    if (j >= 0) ts[j] = t;
  }
}
__device__ __forceinline__ void stamp_end(unsigned long long* ts) {
  if (ts && threadIdx.x == 0) atomicMax(ts + 2, (unsigned long long)__builtin_amdgcn_s_memrealtime());
}

// Where one item's search stands.  The batch kernels keep it in registers;
// the serving tick kernel keeps it in HBM between ticks.
struct ItemState {
  int32_t start;      // first grid position of the next sweep round
  int32_t carry;      // sign at start - 1 (kNoSign before the first round)
  int32_t seg_start;  // split path: where the current FP32 segment began
  int32_t seg_carry;  // split path: FP64 sign at seg_start - 1 (kNoSign at the grid start)
  int32_t done;       // 1 once the outputs are written
  int32_t fp64;       // split path: 1 once it fell back to the FP64 sweep
  int32_t pad[2];
};

__host__ __device__ inline ItemState item_state_init() { return ItemState{0, kNoSign, 0, kNoSign, 0, 0, {0, 0}}; }

// ------------------------------------------------------------- serving --
constexpr int kMaxSlots = 256;     // requests resident on the device at once
constexpr int kMaxAdmit = 64;      // requests admitted per tick

// One resident request (slot).  Pointers address the request's own region of
// the serving pool; outputs go to pinned host memory at out_base.
struct alignas(64) SlotDesc {
  const double* raw;        // staged inputs: h[N], alpha, beta, rho[N+1], lambda[W], c[n_c]
  LayerRec64* L64;          // [N+1]
  LayerRec32* L32;          // [N+1]
  float* c32;               // [n_c]
  double* lam_k;            // [W]
  ItemState* state;         // [W]
  int32_t N, W, n_c, prec;  // prec: MASW_PREC_*
  int32_t out_base;         // first output index (slot * w_max)
  int32_t n_real;           // as ModelDesc::n_real, computed by the host at submit
  uint32_t flags;           // the request's MASW_CHECK_NOISE / MASW_NO_REFINE
  int32_t pad;
};

// Per-tick descriptor, written by the host into pinned memory and copied to
// the device by the captured graph.
struct TickDesc {
  int32_t n_active;              // active slots in this tick
  int32_t n_units;               // sum of their W
  int32_t budget;                // sweep rounds per item per tick
  uint32_t base;                 // queue counter at the start of this tick: the
                                 // counter is never cleared, each tick takes
                                 // exactly n_units + (workgroups) from it
  int32_t active[kMaxSlots];     // slot ids
  int32_t prefix[kMaxSlots + 1]; // prefix sums of W over `active`
  uint32_t exit_base;            // Counters::tick_exit at the start of this tick
  uint32_t seq;                  // this tick's number, written to TickArgs::host_tick at its end
  int32_t pad2;
  SlotDesc slot[kMaxSlots];
};

// Requests admitted in one tick.  The list and the requests' raw inputs
// travel in one host-to-device copy; src[b] is where request b's raw inputs
// (h, alpha, beta, rho, lambda, c) landed, and the admit kernel moves them
// into the request's pool block (desc[b].raw).
struct AdmitList {
  int32_t n;
  int32_t slot[kMaxAdmit];
  SlotDesc desc[kMaxAdmit];
  const double* src[kMaxAdmit];
};

// Finished requests with MASW_CHECK_NOISE whose picks the serve-noise
// kernel tests after a tick (kernel argument, by value).
constexpr int kNoiseList = 16;
struct ServeNoiseList {
  int32_t n;
  SlotDesc slot[kNoiseList];
};

struct TickArgs {
  const TickDesc* desc;      // device copy
  int32_t* slot_remaining;   // [kMaxSlots] items not finished
  Counters* counters;
  int32_t refine;
  int32_t inertia;           // 1: FP64 items use the inertia-count search
  double refine_rel;         // refinement bracket width / c_hi
  // outputs in pinned host memory (device-accessible)
  double* out_ct;
  int32_t* out_idx;
  int32_t* out_status;
  double* out_cref;
  int32_t* host_done;        // [kMaxSlots] set to 1 when a slot's last item finishes
  uint32_t* host_tick;       // pinned: the number of the last tick whose workgroups have all left
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
