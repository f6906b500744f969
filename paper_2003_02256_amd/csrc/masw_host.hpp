// Host-side declarations shared by the runtime (masw_runtime.hip) and the
// serving loop (masw_server.hip): the context, error reporting, and the
// kernel launchers defined next to the kernels (masw_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <mutex>
#include <string>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "masw.h"
#include "masw_internal.hpp"

namespace masw {
// A named roctx range over a scope (shown by rocprofv3 --marker-trace; a
// cheap no-op without a profiler).
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

int sweep_blocks_per_cu(int mode, int G);
int tick_blocks_per_cu(int G, bool inertia);
hipError_t launch_sweep(int mode, int G, int blocks, hipStream_t s, const SweepArgs& a);
// A fused small launch (SweepArgs::fused): `blocks` workgroups of kFusedG
// wavefronts, one wavelength each.
hipError_t launch_fused(int mode, int blocks, hipStream_t s, const SweepArgs& a);
// The inertia-count search (masw_inertia.hip), one wavefront per wavelength.
hipError_t launch_inertia(const SweepArgs& a, int cus, hipStream_t s, int* blocks_out);
hipError_t launch_prep(const PrepArgs& a, const CoopInitArgs& ci, int single_N, int single_W, hipStream_t s);
hipError_t launch_sign_map(bool fp32, const SignMapArgs& a, hipStream_t s);
hipError_t launch_admit(const AdmitList* list_dev, int n, int max_raw, int32_t* slot_remaining, hipStream_t s);
hipError_t launch_tick(int G, int blocks, hipStream_t s, const TickArgs& a);
hipError_t launch_misfit(int n_models, const int32_t* lambda_off, const double* c_t, const double* c_e,
                         double* out, hipStream_t s);

// Device arrays of a zero/pole classification (masw_classify.hip), laid out
// as masw_batch plus the bracket indices and the two outputs.
struct ClassifyArgs {
  int32_t n_models = 0;
  const int32_t* layer_off = nullptr;
  const double* h = nullptr;
  const double* alpha = nullptr;
  const double* beta = nullptr;
  const double* rho = nullptr;
  const int32_t* lambda_off = nullptr;
  const double* lambda = nullptr;
  const double* c = nullptr;
  int32_t n_c = 0;
  const int32_t* idx = nullptr;
  int32_t* cls = nullptr;
  double* c_sec = nullptr;  // may be null
  int64_t n_lam = 0;
  uint64_t* counters = nullptr;  // [3]: evaluations, layers crossed, steps (cleared by the launch)
};
hipError_t launch_classify(const ClassifyArgs& a, hipStream_t s);
// FP64 noise-band flag of the picks of finished served requests
// (masw_noise.hip), after their tick.
hipError_t launch_serve_noise(const ServeNoiseList& list, const int32_t* out_idx, int32_t* out_status,
                              double threshold, hipStream_t s);
// FP64 noise-band flag of every pick (masw_noise.hip), after the sweep.
hipError_t launch_noise_check(const ModelDesc* models, const LayerRec64* layers64, const double* c64,
                              const double* lam_k, const int32_t* lam_model, const int32_t* idx,
                              int32_t* status, int64_t n_lam, double threshold, hipStream_t s);

// The no-alloc entry point's static scratch array (masw_kernels.hip): looks
// up its address on `device`, which must be current, once; then returns it
// (nullptr before the lookup).
hipError_t setup_scratch(int device);
void* scratch_of(int device);

// Records `msg` as the calling thread's last error and returns `code`.
int fail(int code, const std::string& msg);

// Host-side argument checks (host pointers); MASW_OK or MASW_EINVAL via fail().
int check_model_values(int32_t N, const double* h, const double* alpha, const double* beta,
                       const double* rho, const char* what);
int check_grid(const double* c, int32_t n_c, bool values);
int check_lambda(const double* lam, int32_t n, bool values);

struct Server;  // masw_server.hip
void server_destroy(Server* s);
}  // namespace masw

#define MASW_HIP(call)                                                                     \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return ::masw::fail(MASW_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct masw_ctx {
  int device = -1;
  hipStream_t last_stream = nullptr;  // stream of the last synchronous call (may be the null stream)
  bool last_valid = false;
  // per-workgroup work counts of the last timed sweep or inertia launch
  unsigned long long* wg_counts = nullptr;
  int wg_rows = 0;
  bool last_fused = false;  // the last timed launch staged inside the sweep (SweepArgs::fused)
  bool fused_small = true;  // small single-curve launches fuse the staging (MASW_FUSED_SMALL=0: never)
  char* arena = nullptr;
  size_t arena_size = 0;          // whole HBM budget
  size_t sync_size = 0;           // front part used by the synchronous calls
  int cus = 0;
  int blocks_per_cu[2][5] = {};   // [mode][log2 G], G = 1..16
  // options (masw_set_opts); the environment variables named below set their
  // initial values, for tuning
  double refine_rel = masw::kRefineRel;  // c_ref bracket width / c_test[idx]
  double noise_threshold = 1e-2;   // MASW_CHECK_NOISE band
  int forced_waves = 0;            // MASW_WAVES_PER_ITEM; 0 = chosen per launch
  bool shared_sweeps = true;       // MASW_SHARED_SWEEPS=0 turns shared sweeps off
  int shared_window = 8;           // MASW_SHARED_WINDOW: joiners' look-ahead in rounds
  bool first_item_priority = true;  // each workgroup's first item at issue priority 2
  int prio_hi = -1, prio_mid = -1;  // MASW_PRIO=hi,mid: issue priority by queue position
                                    // (-1: the launch's workgroup count, i.e. each one's first item)
  std::mutex mu;
  masw_stats last = {};
  bool stats_pending = false;
  masw::Counters* counters = nullptr;  // arena offset 0
  // Timing of the last kTimingSlots synchronous calls: each call's kernels
  // write the GPU's real-time counter into its slot of tring (device memory,
  // kTimingSlots x kStampWords; see stamp_start), so that back-to-back calls
  // are timed with no host event and no synchronisation per call.  The
  // pending slots are read back together (one copy after the stream has
  // drained) when the ring comes round to a pending slot, or when the
  // timing or the stats are read.
  // With timing_events (masw_opts) a slot's call records HIP events instead
  // (start, sweep start, sweep end; the fused launch has no sweep start).
  struct TimingSlot {
    bool pending = false;
    bool events = false;
    bool fused = false;
    hipEvent_t ev[3] = {};
    float sweep_ms = 0.f, total_ms = 0.f;
  };
  static constexpr int kTimingSlots = 256;
  static constexpr int kStampWords = 4;  // start, sweep start, end, unused
  TimingSlot tslot[kTimingSlots];
  unsigned long long* tring = nullptr;                  // device
  unsigned long long tring_host[kTimingSlots * kStampWords] = {};
  int rtc_khz = 0;  // real-time counter rate (hipDeviceAttributeWallClockRate)
  bool timing_events = false;  // masw_opts::timing_events (slot events created on first use)
  int tslot_next = 0;
  int tslot_last = -1;
  masw_timing timing = {};
  masw::Server* server = nullptr; // serving loop, if started
  // The last masw_classify_picks call: its work counters (in the arena) and
  // HIP events around its kernel, read by masw_get_stats.
  hipEvent_t cls_ev[2] = {};
  uint64_t* cls_counters = nullptr;
  bool cls_pending = false;
};
