// Host runtime behind masw.h: context, HBM arena, argument validation,
// staging of host inputs, launch configuration and the C ABI.
//
// The context allocates its whole HBM budget once (masw_create) and carves
// every call's workspace from it with a bump allocator, so no call allocates
// device memory.  A request whose workspace exceeds the budget fails with
// MASW_ENOMEM before any work is queued.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "masw.h"
#include "masw_host.hpp"
#include "masw_internal.hpp"

using namespace masw;

// ------------------------------------------------------------ errors --
static thread_local std::string g_last_error;

int masw::fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

// ------------------------------------------------------- validation --
static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Host-side checks of one model's values (host pointers only).
int masw::check_model_values(int32_t N, const double* h, const double* alpha, const double* beta,
                       const double* rho, const char* what) {
  if (N < 0 || N > MASW_MAX_LAYERS)
    return fail(MASW_EINVAL, std::string(what) + ": n_layers out of range [0, MASW_MAX_LAYERS]");
  if ((N > 0 && !h) || !alpha || !beta || !rho)
    return fail(MASW_EINVAL, std::string(what) + ": null model array");
  for (int j = 0; j < N; ++j)
    if (!finite_pos(h[j])) return fail(MASW_EINVAL, std::string(what) + ": h must be finite and > 0");
  for (int j = 0; j <= N; ++j) {
    if (!finite_pos(beta[j]) || !finite_pos(alpha[j]) || !finite_pos(rho[j]))
      return fail(MASW_EINVAL, std::string(what) + ": alpha, beta, rho must be finite and > 0");
    if (!(alpha[j] > beta[j]))
      return fail(MASW_EINVAL, std::string(what) + ": alpha must exceed beta in every layer");
  }
  return MASW_OK;
}

int masw::check_grid(const double* c, int32_t n_c, bool values) {
  if (n_c < 2) return fail(MASW_EINVAL, "c_test: n_c must be >= 2");
  if (!c) return fail(MASW_EINVAL, "c_test: null pointer");
  if (!values) return MASW_OK;
  for (int i = 0; i < n_c; ++i) {
    if (!finite_pos(c[i])) return fail(MASW_EINVAL, "c_test: values must be finite and > 0");
    if (i > 0 && !(c[i] > c[i - 1])) return fail(MASW_EINVAL, "c_test: must be strictly increasing");
  }
  return MASW_OK;
}

int masw::check_lambda(const double* lam, int32_t n, bool values) {
  if (n < 0) return fail(MASW_EINVAL, "lambda: n_lambda must be >= 0");
  if (n > 0 && !lam) return fail(MASW_EINVAL, "lambda: null pointer");
  if (!values) return MASW_OK;
  for (int i = 0; i < n; ++i)
    if (!finite_pos(lam[i])) return fail(MASW_EINVAL, "lambda: values must be finite and > 0");
  return MASW_OK;
}

namespace {

constexpr size_t kAlign = 256;
constexpr int64_t kMinSharedRounds = 4;  // shared sweeps only on grids of more rounds than this

// Every synchronous call reuses the front of the arena.  A call on a stream
// other than the previous call's first waits for that stream, so the previous
// call's kernels are done with the memory.
hipError_t claim_arena(masw_ctx* ctx, hipStream_t s) {
  if (ctx->last_valid && ctx->last_stream != s) return hipStreamSynchronize(ctx->last_stream);
  return hipSuccess;
}

struct Bump {
  char* base;
  size_t cap;
  size_t off;
  template <typename T>
  T* take(size_t n) {
    off = (off + kAlign - 1) & ~(kAlign - 1);
    T* p = reinterpret_cast<T*>(base + off);
    off += n * sizeof(T);
    return p;
  }
  bool ok() const { return off <= cap; }
};

// Flattened view of the inputs, host or device, with sizes.
struct Inputs {
  int32_t n_models = 0;
  const int32_t* layer_off = nullptr;  // nullptr: single model
  int32_t single_N = 0;
  int32_t single_W = 0;
  const double* h = nullptr;
  const double* alpha = nullptr;
  const double* beta = nullptr;
  const double* rho = nullptr;
  const int32_t* lambda_off = nullptr;
  const double* lambda = nullptr;
  const double* c = nullptr;
  int32_t n_c = 0;
  int64_t n_layers_total = 0;  // sum N_m
  int64_t n_lam = 0;           // sum W_m
  const double* c_e = nullptr;  // fused misfit (batch only): experimental curve, [n_lam]
  double* misfit = nullptr;     // fused misfit: [n_models] (null: no misfit)
};

// Blocks of the grid check, one flag each.
size_t grid_blocks(int64_t n_c) { return size_t((n_c + kPrepThreads - 1) / kPrepThreads); }

// Rows of per-workgroup work counts a launch may write: one per workgroup,
// and a launch has at most one workgroup per wavelength.
size_t wg_rows(const Inputs& in) {
  return size_t(std::min<int64_t>(std::max<int64_t>(in.n_lam, 1), kMaxWgRows));
}

// Total device bytes of one call's workspace.

size_t workspace_bytes(const Inputs& in, bool stage_inputs, bool stage_outputs) {
  Bump b{nullptr, ~size_t(0), 0};
  const size_t R = size_t(in.n_layers_total + in.n_models);
  b.take<Counters>(1);
  b.take<uint32_t>(grid_blocks(in.n_c));
  b.take<ModelDesc>(size_t(in.n_models));
  b.take<LayerRec64>(R);
  b.take<LayerRec32>(R);
  if (stage_inputs) b.take<double>(size_t(in.n_c));  // device pointers: the grid is read in place
  b.take<float>(size_t(in.n_c));
  b.take<double>(size_t(in.n_lam));
  b.take<int32_t>(size_t(in.n_lam));
  b.take<uint8_t>(size_t(in.n_lam));
  b.take<int32_t>(size_t(in.n_lam));
  if (stage_inputs) {
    b.take<int32_t>(size_t(in.n_models) + 1);
    b.take<int32_t>(size_t(in.n_models) + 1);
    b.take<double>(size_t(in.n_layers_total));
    b.take<double>(R * 3);
    b.take<double>(size_t(in.n_lam));
  }
  if (stage_outputs) {
    b.take<double>(size_t(in.n_lam) * 2);
    b.take<int32_t>(size_t(in.n_lam) * 2);
  }
  if (in.misfit) {
    b.take<int32_t>(size_t(in.n_models));
    if (stage_inputs) {
      b.take<double>(size_t(in.n_lam));
      b.take<double>(size_t(in.n_models));
    }
  }
  b.take<unsigned long long>(wg_rows(in) * kWgCounts);
  return b.off + kAlign;
}

int log2_of(int g) { return g <= 1 ? 0 : g <= 2 ? 1 : g <= 4 ? 2 : g <= 8 ? 3 : 4; }

// Wavefronts per item.  Items run to an early exit whose depth varies by two
// orders of magnitude across wavelengths, so a launch with few items is
// bounded by its deepest item: give each item as many wavefronts as keeps
// every item queued at most about four times over the resident slots, and one
// wavefront per item when items outnumber slots.  G stays small enough that
// two groups fit on a compute unit, so that one group's single-wavefront FP64
// re-check and refinement overlap the other group's sweep.  The persistent
// grid then pulls items longest-expected-first until the queue is empty.
// The FP64 walk takes half that G when it lets every item start at once in a
// workgroup of its own (no item queued behind another), which the rule's G
// does not: measured 3% faster at 1000 fine-scale wavelengths, where 8
// wavefronts per item left two items per workgroup.  The split path keeps
// the rule's G, whose second workgroup per CU overlaps each item's
// single-wavefront FP64 re-check.
int pick_waves_per_item(masw_ctx* ctx, int mode, int64_t n_items, int* blocks) {
  int G = 1;
  if (ctx->forced_waves) {
    G = ctx->forced_waves;
  } else {
    for (int lg = 4; lg >= 0; --lg) {
      const int g = 1 << lg;
      const int bpc = ctx->blocks_per_cu[mode][lg];
      const int64_t slots = int64_t(ctx->cus) * bpc * g;
      if (bpc >= 2 && n_items * g <= 4 * slots) {
        G = g;
        break;
      }
    }
    if (mode == 0 && G >= 2) {
      const int lg = log2_of(G);
      const int64_t fit = int64_t(ctx->cus) * ctx->blocks_per_cu[mode][lg];
      const int64_t fit_half = int64_t(ctx->cus) * ctx->blocks_per_cu[mode][lg - 1];
      if (n_items > fit && n_items <= fit_half) G /= 2;
    }
  }
  const int64_t max_blocks = int64_t(ctx->cus) * std::max(1, ctx->blocks_per_cu[mode][log2_of(G)]);
  *blocks = int(std::max<int64_t>(1, std::min<int64_t>(n_items, max_blocks)));
  return G;
}

// Waits for a timed call's last event and adds its durations to the sums.
// Resolves every pending timing slot into the running sums, oldest first:
// a slot timed by the real-time counter from one read-back of the ring
// (their calls ran on last_stream, or on a stream that claim_arena has since
// drained), a slot timed by events from its events.
hipError_t resolve_timing(masw_ctx* ctx) {
  bool stamps = false;
  for (const auto& T : ctx->tslot) stamps = stamps || (T.pending && !T.events);
  if (stamps) {
    hipError_t e = hipMemcpyAsync(ctx->tring_host, ctx->tring, sizeof(ctx->tring_host), hipMemcpyDeviceToHost,
                                  ctx->last_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->last_stream);
    if (e != hipSuccess) return e;
  }
  const double per_ms = double(ctx->rtc_khz);  // counter ticks per millisecond
  masw_timing& t = ctx->timing;
  for (int k = 0; k < masw_ctx::kTimingSlots; ++k) {
    const int i = (ctx->tslot_next + k) % masw_ctx::kTimingSlots;
    masw_ctx::TimingSlot& T = ctx->tslot[i];
    if (!T.pending) continue;
    if (T.events) {
      hipError_t e = hipEventSynchronize(T.ev[2]);
      if (e == hipSuccess) e = hipEventElapsedTime(&T.total_ms, T.ev[0], T.ev[2]);
      if (e == hipSuccess && !T.fused) e = hipEventElapsedTime(&T.sweep_ms, T.ev[1], T.ev[2]);
      if (e != hipSuccess) return e;
      if (T.fused) T.sweep_ms = T.total_ms;  // one launch: the sweep with its staging
    } else {
      const unsigned long long* w = ctx->tring_host + size_t(i) * masw_ctx::kStampWords;
      T.total_ms = w[2] > w[0] ? float(double(w[2] - w[0]) / per_ms) : 0.f;
      T.sweep_ms = w[2] > w[1] ? float(double(w[2] - w[1]) / per_ms) : 0.f;
    }
    T.pending = false;
    t.sweep_ms_min = t.launches ? std::min(t.sweep_ms_min, T.sweep_ms) : T.sweep_ms;
    t.sweep_ms_max = t.launches ? std::max(t.sweep_ms_max, T.sweep_ms) : T.sweep_ms;
    t.sweep_ms_sum += T.sweep_ms;
    t.total_ms_sum += T.total_ms;
    ++t.launches;
  }
  return hipSuccess;
}

// Where a call's workspace lives: the context's arena (timed, with work
// counters for masw_get_stats), or the static scratch array of the no-alloc
// entry point (device pointers only; no arena claim, no events, no stats).
struct Workspace {
  char* base;
  size_t cap;
  bool noalloc;
};

// Shared body of the curve and batch calls.
int run_curves(masw_ctx* ctx, const Inputs& in, masw_precision prec, uint32_t flags, void* stream,
               const masw_outputs* out, const Workspace& ws) {
  const bool dev = (flags & MASW_DEVICE_PTRS) != 0;
  hipStream_t s = static_cast<hipStream_t>(stream);  // NULL: the default stream
  const size_t need = workspace_bytes(in, !dev, !dev);
  if (need > ws.cap)
    return fail(MASW_ENOMEM, "request needs " + std::to_string(need) + " B of device memory, " +
                                 (ws.noalloc ? "the no-alloc scratch holds " : "budget is ") +
                                 std::to_string(ws.cap) + " B");
  MASW_HIP(hipSetDevice(ctx->device));
  if (!ws.noalloc) MASW_HIP(claim_arena(ctx, s));

  Bump b{ws.base, ws.cap, 0};
  const size_t R = size_t(in.n_layers_total + in.n_models);
  PrepArgs p{};
  p.counters = b.take<Counters>(1);
  p.grid_flags = b.take<uint32_t>(grid_blocks(in.n_c));
  p.models = b.take<ModelDesc>(size_t(in.n_models));
  p.layers64 = b.take<LayerRec64>(R);
  p.layers32 = b.take<LayerRec32>(R);
  double* c_copy = dev ? nullptr : b.take<double>(size_t(in.n_c));
  p.c32 = b.take<float>(size_t(in.n_c));
  p.lam_k = b.take<double>(size_t(in.n_lam));
  p.lam_model = b.take<int32_t>(size_t(in.n_lam));
  p.lam_bucket = b.take<uint8_t>(size_t(in.n_lam));
  p.order = b.take<int32_t>(size_t(in.n_lam));
  p.n_models = in.n_models;
  p.n_c = in.n_c;
  p.n_lam = int32_t(in.n_lam);

  SweepArgs sw{};
  if (dev) {
    p.layer_off = in.layer_off;
    p.lambda_off = in.lambda_off;
    p.h = in.h;
    p.alpha = in.alpha;
    p.beta = in.beta;
    p.rho = in.rho;
    p.lambda = in.lambda;
    p.c_in = in.c;
    p.c64 = const_cast<double*>(in.c);  // the grid is read in place
    sw.out_ct = out->c_t;
    sw.out_idx = out->idx;
    sw.out_status = out->status;
    sw.out_cref = out->c_ref;
  } else {
    int32_t* loff = nullptr;
    int32_t* woff = nullptr;
    if (in.layer_off) {
      loff = b.take<int32_t>(size_t(in.n_models) + 1);
      woff = b.take<int32_t>(size_t(in.n_models) + 1);
    } else {
      b.take<int32_t>(size_t(in.n_models) + 1);
      b.take<int32_t>(size_t(in.n_models) + 1);
    }
    double* hh = b.take<double>(size_t(in.n_layers_total));
    double* abr = b.take<double>(R * 3);
    double* ll = b.take<double>(size_t(in.n_lam));
    if (loff) {
      MASW_HIP(hipMemcpyAsync(loff, in.layer_off, sizeof(int32_t) * (in.n_models + 1), hipMemcpyHostToDevice, s));
      MASW_HIP(hipMemcpyAsync(woff, in.lambda_off, sizeof(int32_t) * (in.n_models + 1), hipMemcpyHostToDevice, s));
    }
    if (in.n_layers_total)
      MASW_HIP(hipMemcpyAsync(hh, in.h, sizeof(double) * in.n_layers_total, hipMemcpyHostToDevice, s));
    MASW_HIP(hipMemcpyAsync(abr, in.alpha, sizeof(double) * R, hipMemcpyHostToDevice, s));
    MASW_HIP(hipMemcpyAsync(abr + R, in.beta, sizeof(double) * R, hipMemcpyHostToDevice, s));
    MASW_HIP(hipMemcpyAsync(abr + 2 * R, in.rho, sizeof(double) * R, hipMemcpyHostToDevice, s));
    if (in.n_lam) MASW_HIP(hipMemcpyAsync(ll, in.lambda, sizeof(double) * in.n_lam, hipMemcpyHostToDevice, s));
    MASW_HIP(hipMemcpyAsync(c_copy, in.c, sizeof(double) * in.n_c, hipMemcpyHostToDevice, s));
    p.layer_off = loff;
    p.lambda_off = woff;
    p.h = hh;
    p.alpha = abr;
    p.beta = abr + R;
    p.rho = abr + 2 * R;
    p.lambda = ll;
    p.c_in = c_copy;
    p.c64 = c_copy;
    sw.out_ct = b.take<double>(size_t(in.n_lam));
    sw.out_cref = b.take<double>(size_t(in.n_lam));
    sw.out_idx = b.take<int32_t>(size_t(in.n_lam));
    sw.out_status = b.take<int32_t>(size_t(in.n_lam));
  }
  // fused misfit: per-model countdown, and the staged C_e and misfit
  const double* c_e_dev = nullptr;
  double* misfit_dev = nullptr;
  if (in.misfit) {
    p.model_left = b.take<int32_t>(size_t(in.n_models));
    if (dev) {
      c_e_dev = in.c_e;
      misfit_dev = in.misfit;
    } else {
      double* ce = b.take<double>(size_t(in.n_lam));
      misfit_dev = b.take<double>(size_t(in.n_models));
      if (in.n_lam) MASW_HIP(hipMemcpyAsync(ce, in.c_e, sizeof(double) * in.n_lam, hipMemcpyHostToDevice, s));
      c_e_dev = ce;
    }
    p.misfit = misfit_dev;
  }
  sw.wg_counts = b.take<unsigned long long>(wg_rows(in) * kWgCounts);
  if (!b.ok()) return fail(MASW_ENOMEM, "workspace exceeds the HBM budget");

  const bool inertia = (flags & MASW_SEARCH_INERTIA) != 0;
  // a split call on a grid that two rounds of a small launch cover runs as
  // the FP64 walk (include/masw.h, MASW_PREC_SPLIT)
  const bool split_as_fp64 = prec == MASW_PREC_SPLIT && int64_t(in.n_c) < int64_t(MASW_SPLIT_MIN_GRID);
  const int mode = (prec == MASW_PREC_SPLIT && !split_as_fp64) ? 1 : 0;
  int blocks = 1;
  const int G = inertia ? 1 : pick_waves_per_item(ctx, mode, in.n_lam, &blocks);

  // Shared sweeps when items are few enough that the deepest ones decide the
  // launch time: every item, with one summary word per round of its grid,
  // if that fits in what is left of the budget.  Not on grids of a few
  // rounds, where a joining workgroup could take at most one round and the
  // claims and summaries only add latency.
  CoopInitArgs ci{};
  const int64_t stride = (int64_t(in.n_c) + 64 * G - 1) / (64 * G);
  if (!inertia && ctx->shared_sweeps && blocks > 1 && in.n_lam > 0 && in.n_lam <= 4 * int64_t(blocks) &&
      stride > kMinSharedRounds) {
    const size_t save = b.off;
    ci.n_coop = int32_t(in.n_lam);
    ci.coop = b.take<CoopItem>(size_t(ci.n_coop));
    ci.n_sum = uint64_t(ci.n_coop) * uint64_t(stride);
    ci.coop_sum = b.take<uint64_t>(ci.n_sum);
    ci.n_active = blocks;
    ci.coop_active = b.take<int32_t>(size_t(blocks));
    if (!b.ok()) {
      b.off = save;
      ci = CoopInitArgs{};
    }
  }

  // A small single-curve launch stages inside the sweep kernel
  // (SweepArgs::fused): one launch instead of a staging launch and a sweep,
  // on grids short enough that no shared sweep would run.
  const bool fused = ctx->fused_small && !inertia && !in.misfit && !(flags & MASW_CHECK_NOISE) && !in.layer_off &&
                     in.n_models == 1 && in.n_lam > 0 && in.n_lam <= kLamBlock && in.single_N <= kFusedMaxLayers &&
                     int64_t(in.n_c) <= int64_t(kMinSharedRounds) * 64 * kFusedG &&
                     (ctx->forced_waves == 0 || ctx->forced_waves == kFusedG);
  if (fused) {
    ci = CoopInitArgs{};
    blocks = int(in.n_lam);
    sw.fused = 1;
    sw.fused_N = in.single_N;
    sw.f_h = p.h;
    sw.f_alpha = p.alpha;
    sw.f_beta = p.beta;
    sw.f_rho = p.rho;
    sw.f_lambda = p.lambda;
    sw.f_c = p.c_in;
    sw.f_n_c = in.n_c;
  }

  // timed (a slot of the stamp ring) unless no-alloc or without a sweep
  masw_ctx::TimingSlot* T = nullptr;
  const int ts = ctx->tslot_next;
  if (!ws.noalloc && in.n_lam > 0) {
    T = &ctx->tslot[ts];
    if (T->pending) MASW_HIP(resolve_timing(ctx));
    ctx->tslot_next = (ts + 1) % masw_ctx::kTimingSlots;
    T->events = ctx->timing_events;
    T->fused = fused;
    if (T->events) {
      MASW_HIP(hipEventRecord(T->ev[0], s));
    } else {
      p.tstamp = ctx->tring + size_t(ts) * masw_ctx::kStampWords;
      sw.tstamp = p.tstamp;
    }
  }
  if (!fused) MASW_HIP(launch_prep(p, ci, in.single_N, in.single_W, s));

  sw.n_coop = ci.n_coop;
  sw.coop_stride = int32_t(stride);
  sw.coop = ci.coop;
  sw.coop_sum = ci.coop_sum;
  sw.coop_active = ci.coop_active;
  sw.coop_window = ctx->shared_window;
  // A workgroup's first item comes from the deep end of the queue: it takes
  // issue precedence over items claimed later on the same compute unit.
  sw.prio_hi = !ctx->first_item_priority ? 0 : ctx->prio_hi >= 0 ? ctx->prio_hi : blocks;
  sw.prio_mid = !ctx->first_item_priority ? 0 : ctx->prio_mid >= 0 ? ctx->prio_mid : blocks;
  sw.models = p.models;
  sw.layers64 = p.layers64;
  sw.layers32 = p.layers32;
  sw.c64 = p.c64;
  sw.c32 = p.c32;
  sw.lam_k = p.lam_k;
  sw.lam_model = p.lam_model;
  sw.order = p.order;
  sw.n_items = int32_t(in.n_lam);
  sw.refine = (flags & MASW_NO_REFINE) ? 0 : 1;
  sw.refine_rel = ctx->refine_rel;
  sw.counters = p.counters;
  if (in.misfit && !inertia) {  // the inertia search takes a separate misfit launch below
    sw.c_e = c_e_dev;
    sw.misfit = misfit_dev;
    sw.model_left = p.model_left;
    sw.lambda_off = p.lambda_off;
  }
  if (T && T->events && !fused) MASW_HIP(hipEventRecord(T->ev[1], s));
  if (fused)
    MASW_HIP(launch_fused(mode, blocks, s, sw));
  else if (in.n_lam > 0)
    MASW_HIP(inertia ? launch_inertia(sw, ctx->cus, s, &blocks) : launch_sweep(mode, G, blocks, s, sw));
  if (T && T->events) MASW_HIP(hipEventRecord(T->ev[2], s));
  if (in.misfit && inertia)
    MASW_HIP(launch_misfit(in.n_models, p.lambda_off, sw.out_ct, c_e_dev, misfit_dev, s));
  // optional diagnostic after the timed sweep: the FP64 noise band of each
  // pick's bracket
  if ((flags & MASW_CHECK_NOISE) && in.n_lam > 0)
    MASW_HIP(launch_noise_check(p.models, p.layers64, p.c64, p.lam_k, p.lam_model, sw.out_idx, sw.out_status,
                                in.n_lam, ctx->noise_threshold, s));
  if (ws.noalloc) return MASW_OK;
  if (T) T->pending = true;
  ctx->tslot_last = T ? ts : -1;
  ctx->last = masw_stats{};
  ctx->last.n_lambda = uint64_t(in.n_lam);
  ctx->last.waves_per_item = fused ? kFusedG : G;
  ctx->last_fused = fused;
  ctx->last.fused_staging = fused ? 1 : 0;
  ctx->last.split_as_fp64 = split_as_fp64 ? 1 : 0;
  ctx->last.workgroups = in.n_lam > 0 ? blocks : 0;
  ctx->wg_counts = sw.wg_counts;
  ctx->wg_rows = in.n_lam > 0 ? blocks : 0;
  ctx->last.shared_items = ci.n_coop;
  ctx->stats_pending = true;
  ctx->cls_pending = false;
  ctx->last_stream = s;
  ctx->last_valid = true;

  if (!dev) {
    const size_t W = size_t(in.n_lam);
    if (W) {
      MASW_HIP(hipMemcpyAsync(out->c_t, sw.out_ct, sizeof(double) * W, hipMemcpyDeviceToHost, s));
      MASW_HIP(hipMemcpyAsync(out->idx, sw.out_idx, sizeof(int32_t) * W, hipMemcpyDeviceToHost, s));
      MASW_HIP(hipMemcpyAsync(out->status, sw.out_status, sizeof(int32_t) * W, hipMemcpyDeviceToHost, s));
      if (out->c_ref)
        MASW_HIP(hipMemcpyAsync(out->c_ref, sw.out_cref, sizeof(double) * W, hipMemcpyDeviceToHost, s));
    }
    if (in.misfit)
      MASW_HIP(hipMemcpyAsync(in.misfit, misfit_dev, sizeof(double) * in.n_models, hipMemcpyDeviceToHost, s));
    MASW_HIP(hipStreamSynchronize(s));
  }
  return MASW_OK;
}

int check_common(masw_ctx* ctx, masw_precision prec, uint32_t flags) {
  if (prec != MASW_PREC_FP64 && prec != MASW_PREC_SPLIT) return fail(MASW_EINVAL, "prec: unknown precision");
  if (flags & ~(MASW_DEVICE_PTRS | MASW_NO_REFINE | MASW_CHECK_NOISE | MASW_SEARCH_INERTIA))
    return fail(MASW_EINVAL, "flags: unknown bits");
  if ((flags & MASW_SEARCH_INERTIA) && prec != MASW_PREC_FP64)
    return fail(MASW_EINVAL, "flags: MASW_SEARCH_INERTIA needs MASW_PREC_FP64");
  if (!ctx) return fail(MASW_EINVAL, "ctx: null context");
  return MASW_OK;
}

}  // namespace

// ================================================================ C ABI ==
extern "C" {

const char* masw_version(void) { return "maswx 0.1.0 (gfx950)"; }

const char* masw_last_error(void) { return g_last_error.c_str(); }

const char* masw_strerror(int code) {
  switch (code) {
    case MASW_OK: return "success";
    case MASW_EINVAL: return "invalid argument";
    case MASW_ENOMEM: return "request exceeds the HBM budget";
    case MASW_EBUSY: return "busy / not ready";
    case MASW_EDEVICE: return "HIP device error";
    case MASW_ETIMEOUT: return "timed out";
    case MASW_ENOENT: return "unknown ticket";
    default: return "unknown error code";
  }
}

int masw_create(int device, size_t hbm_budget_bytes, masw_ctx** out) {
  if (!out) return fail(MASW_EINVAL, "out: null pointer");
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return fail(MASW_EDEVICE, "no HIP device present");
  if (device < 0 || device >= n) return fail(MASW_EDEVICE, "device index out of range");
  const size_t budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t(256) << 20);
  masw_ctx* ctx = new masw_ctx();
  ctx->device = device;
  auto cleanup = [&](int code, const std::string& msg) {
    if (ctx->arena) (void)hipFree(ctx->arena);
    if (ctx->tring) (void)hipFree(ctx->tring);
    for (auto& e : ctx->cls_ev)
      if (e) (void)hipEventDestroy(e);
    delete ctx;
    return fail(code, msg);
  };
  if (hipSetDevice(device) != hipSuccess) return cleanup(MASW_EDEVICE, "hipSetDevice failed");
  if (setup_scratch(device) != hipSuccess)
    return cleanup(MASW_EDEVICE, "cannot look up the no-alloc scratch array on this device");
  if (hipDeviceGetAttribute(&ctx->cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    return cleanup(MASW_EDEVICE, "cannot query compute units");
  if (hipDeviceGetAttribute(&ctx->rtc_khz, hipDeviceAttributeWallClockRate, device) != hipSuccess ||
      ctx->rtc_khz <= 0)
    return cleanup(MASW_EDEVICE, "cannot query the real-time counter rate");
  if (hipMalloc(&ctx->tring, sizeof(ctx->tring_host)) != hipSuccess ||
      hipMemset(ctx->tring, 0, sizeof(ctx->tring_host)) != hipSuccess)
    return cleanup(MASW_ENOMEM, "cannot allocate the timing slots");
  // The classification's events only time its launch (outputs reach the
  // host through their own copies and synchronisations): a device-scope
  // release spares each of them a system-scope cache writeback.
  for (auto& e : ctx->cls_ev)
    if (hipEventCreateWithFlags(&e, hipEventReleaseToDevice) != hipSuccess)
      return cleanup(MASW_EDEVICE, "hipEventCreate failed");
  if (hipMalloc(&ctx->arena, budget) != hipSuccess) return cleanup(MASW_ENOMEM, "cannot allocate the HBM budget");
  ctx->arena_size = budget;
  ctx->sync_size = budget;
  ctx->counters = reinterpret_cast<Counters*>(ctx->arena);
  for (int mode = 0; mode < 2; ++mode)
    for (int lg = 0; lg < 5; ++lg) ctx->blocks_per_cu[mode][lg] = sweep_blocks_per_cu(mode, 1 << lg);
  if (const char* f = std::getenv("MASW_WAVES_PER_ITEM")) {
    const int g = std::atoi(f);
    if (g == 1 || g == 2 || g == 4 || g == 8 || g == 16) ctx->forced_waves = g;
  }
  if (const char* f = std::getenv("MASW_SHARED_SWEEPS")) ctx->shared_sweeps = std::atoi(f) != 0;
  if (const char* f = std::getenv("MASW_FUSED_SMALL")) ctx->fused_small = std::atoi(f) != 0;
  if (const char* f = std::getenv("MASW_PRIO")) {
    // "hi,mid" queue positions (tuning; "0,0" = off)
    int hi = 0, mid = 0;
    if (std::sscanf(f, "%d,%d", &hi, &mid) == 2 && hi >= 0 && mid >= hi) {
      ctx->prio_hi = hi;
      ctx->prio_mid = mid;
    }
  }
  if (const char* f = std::getenv("MASW_SHARED_WINDOW")) {
    const int w = std::atoi(f);
    if (w >= 1 && w <= 1024) ctx->shared_window = w;
  }

  *out = ctx;
  return MASW_OK;
}

void masw_destroy(masw_ctx* ctx) {
  if (!ctx) return;
  if (ctx->server) {
    server_destroy(ctx->server);
    ctx->server = nullptr;
  }
  (void)hipSetDevice(ctx->device);
  if (ctx->last_valid) (void)hipStreamSynchronize(ctx->last_stream);
  if (ctx->arena) (void)hipFree(ctx->arena);
  if (ctx->tring) (void)hipFree(ctx->tring);
  for (auto& t : ctx->tslot)
    for (auto& e : t.ev)
      if (e) (void)hipEventDestroy(e);
  for (auto& e : ctx->cls_ev)
    if (e) (void)hipEventDestroy(e);
  delete ctx;
}

int masw_dispersion_curve(masw_ctx* ctx, const double* c_test, int32_t n_c, const double* lambda,
                          int32_t n_lambda, const masw_model* model, masw_precision prec, uint32_t flags,
                          void* stream, double* C_t, int32_t* idx, int32_t* status, double* c_ref) {
  TraceRange trace("masw_dispersion_curve");
  const bool dev = (flags & MASW_DEVICE_PTRS) != 0;
  int rc;
  if (!model) return fail(MASW_EINVAL, "model: null pointer");
  if ((rc = check_grid(c_test, n_c, !dev))) return rc;
  if ((rc = check_lambda(lambda, n_lambda, !dev))) return rc;
  if (dev) {
    if (model->n_layers < 0 || model->n_layers > MASW_MAX_LAYERS)
      return fail(MASW_EINVAL, "model: n_layers out of range [0, MASW_MAX_LAYERS]");
    if ((model->n_layers > 0 && !model->h) || !model->alpha || !model->beta || !model->rho)
      return fail(MASW_EINVAL, "model: null model array");
  } else if ((rc = check_model_values(model->n_layers, model->h, model->alpha, model->beta, model->rho,
                                      "model"))) {
    return rc;
  }
  if (n_lambda > 0 && (!C_t || !idx || !status)) return fail(MASW_EINVAL, "outputs: C_t, idx, status required");
  if ((rc = check_common(ctx, prec, flags))) return rc;
  std::lock_guard<std::mutex> lock(ctx->mu);
  Inputs in;
  in.n_models = 1;
  in.single_N = model->n_layers;
  in.single_W = n_lambda;
  in.h = model->h;
  in.alpha = model->alpha;
  in.beta = model->beta;
  in.rho = model->rho;
  in.lambda = lambda;
  in.c = c_test;
  in.n_c = n_c;
  in.n_layers_total = model->n_layers;
  in.n_lam = n_lambda;
  masw_outputs o{C_t, idx, status, c_ref};
  return run_curves(ctx, in, prec, flags, stream, &o, Workspace{ctx->arena, ctx->sync_size, false});
}

int masw_dispersion_curve_noalloc(masw_ctx* ctx, const double* c_test, int32_t n_c, const double* lambda,
                                  int32_t n_lambda, const masw_model* model, masw_precision prec, uint32_t flags,
                                  void* stream, double* C_t, int32_t* idx, int32_t* status, double* c_ref) {
  TraceRange trace("masw_dispersion_curve_noalloc");
  int rc;
  if (!(flags & MASW_DEVICE_PTRS)) return fail(MASW_EINVAL, "flags: MASW_DEVICE_PTRS is required");
  if (!model) return fail(MASW_EINVAL, "model: null pointer");
  if ((rc = check_grid(c_test, n_c, false))) return rc;
  if ((rc = check_lambda(lambda, n_lambda, false))) return rc;
  if (model->n_layers < 0 || model->n_layers > MASW_MAX_LAYERS)
    return fail(MASW_EINVAL, "model: n_layers out of range [0, MASW_MAX_LAYERS]");
  if ((model->n_layers > 0 && !model->h) || !model->alpha || !model->beta || !model->rho)
    return fail(MASW_EINVAL, "model: null model array");
  if (n_lambda > 0 && (!C_t || !idx || !status)) return fail(MASW_EINVAL, "outputs: C_t, idx, status required");
  if ((rc = check_common(ctx, prec, flags))) return rc;
  void* sp = scratch_of(ctx->device);
  if (!sp) return fail(MASW_EDEVICE, "the no-alloc scratch array is not set up on this device");
  std::lock_guard<std::mutex> lock(ctx->mu);
  Inputs in;
  in.n_models = 1;
  in.single_N = model->n_layers;
  in.single_W = n_lambda;
  in.h = model->h;
  in.alpha = model->alpha;
  in.beta = model->beta;
  in.rho = model->rho;
  in.lambda = lambda;
  in.c = c_test;
  in.n_c = n_c;
  in.n_layers_total = model->n_layers;
  in.n_lam = n_lambda;
  masw_outputs o{C_t, idx, status, c_ref};
  return run_curves(ctx, in, prec, flags, stream, &o,
                    Workspace{static_cast<char*>(sp), size_t(MASW_NOALLOC_SCRATCH_BYTES), true});
}

// Shared body of masw_dispersion_batch and masw_dispersion_batch_misfit
// (C_e, misfit null for the former).
static int batch_impl(masw_ctx* ctx, const double* c_test, int32_t n_c, const masw_batch* batch,
                      masw_precision prec, uint32_t flags, void* stream, const masw_outputs* out,
                      const double* C_e, double* misfit) {
  const bool dev = (flags & MASW_DEVICE_PTRS) != 0;
  int rc;
  if (!batch) return fail(MASW_EINVAL, "batch: null pointer");
  if (!out) return fail(MASW_EINVAL, "out: null pointer");
  if ((rc = check_grid(c_test, n_c, !dev))) return rc;
  if (batch->n_models < 1) return fail(MASW_EINVAL, "batch: n_models must be >= 1");
  if (!batch->layer_off || !batch->lambda_off || !batch->alpha || !batch->beta || !batch->rho || !batch->lambda)
    return fail(MASW_EINVAL, "batch: null array");
  // Sizes come from the offset arrays, which are read on the host (for
  // device pointers they are copied back; they are n_models + 1 ints).
  std::vector<int32_t> loff(size_t(batch->n_models) + 1), woff(size_t(batch->n_models) + 1);
  if (dev) {
    if ((rc = check_common(ctx, prec, flags))) return rc;
    MASW_HIP(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);  // NULL: the default stream
    MASW_HIP(hipMemcpyAsync(loff.data(), batch->layer_off, sizeof(int32_t) * loff.size(), hipMemcpyDeviceToHost, s));
    MASW_HIP(hipMemcpyAsync(woff.data(), batch->lambda_off, sizeof(int32_t) * woff.size(), hipMemcpyDeviceToHost, s));
    MASW_HIP(hipStreamSynchronize(s));
  } else {
    std::memcpy(loff.data(), batch->layer_off, sizeof(int32_t) * loff.size());
    std::memcpy(woff.data(), batch->lambda_off, sizeof(int32_t) * woff.size());
  }
  if (loff[0] != 0 || woff[0] != 0) return fail(MASW_EINVAL, "batch: offsets must start at 0");
  for (int m = 0; m < batch->n_models; ++m) {
    const int32_t N = loff[m + 1] - loff[m];
    if (N < 0 || N > MASW_MAX_LAYERS) return fail(MASW_EINVAL, "batch: layer_off must be non-decreasing, N <= MASW_MAX_LAYERS");
    if (woff[m + 1] < woff[m]) return fail(MASW_EINVAL, "batch: lambda_off must be non-decreasing");
  }
  const int64_t L = loff[batch->n_models];
  const int64_t W = woff[batch->n_models];
  if (L > 0 && !batch->h) return fail(MASW_EINVAL, "batch: null h");
  if (W > 0 && (!out->c_t || !out->idx || !out->status)) return fail(MASW_EINVAL, "outputs: C_t, idx, status required");
  if (!dev) {
    for (int m = 0; m < batch->n_models; ++m) {
      const int32_t N = loff[m + 1] - loff[m];
      const int64_t r0 = int64_t(loff[m]) + m;
      if ((rc = check_model_values(N, batch->h + loff[m], batch->alpha + r0, batch->beta + r0, batch->rho + r0,
                                   ("batch model " + std::to_string(m)).c_str())))
        return rc;
    }
    if ((rc = check_lambda(batch->lambda, int32_t(W), true))) return rc;
    if (misfit)
      for (int64_t i = 0; i < W; ++i)
        if (!(std::isfinite(C_e[i]) && C_e[i] > 0.0)) return fail(MASW_EINVAL, "C_e must be finite and > 0");
    if ((rc = check_common(ctx, prec, flags))) return rc;
  }
  std::lock_guard<std::mutex> lock(ctx->mu);
  Inputs in;
  in.n_models = batch->n_models;
  in.layer_off = batch->layer_off;
  in.lambda_off = batch->lambda_off;
  in.h = batch->h;
  in.alpha = batch->alpha;
  in.beta = batch->beta;
  in.rho = batch->rho;
  in.lambda = batch->lambda;
  in.c = c_test;
  in.n_c = n_c;
  in.n_layers_total = L;
  in.n_lam = W;
  in.c_e = C_e;
  in.misfit = misfit;
  return run_curves(ctx, in, prec, flags, stream, out, Workspace{ctx->arena, ctx->sync_size, false});
}

int masw_dispersion_batch(masw_ctx* ctx, const double* c_test, int32_t n_c, const masw_batch* batch,
                          masw_precision prec, uint32_t flags, void* stream, const masw_outputs* out) {
  TraceRange trace("masw_dispersion_batch");
  return batch_impl(ctx, c_test, n_c, batch, prec, flags, stream, out, nullptr, nullptr);
}

int masw_dispersion_batch_misfit(masw_ctx* ctx, const double* c_test, int32_t n_c, const masw_batch* batch,
                                 masw_precision prec, uint32_t flags, void* stream, const masw_outputs* out,
                                 const double* C_e, double* misfit) {
  TraceRange trace("masw_dispersion_batch_misfit");
  if (!C_e || !misfit) return fail(MASW_EINVAL, "C_e, misfit: null array");
  return batch_impl(ctx, c_test, n_c, batch, prec, flags, stream, out, C_e, misfit);
}

int masw_sign_map(masw_ctx* ctx, const double* c_test, int32_t n_c, const double* lambda, int32_t n_lambda,
                  const masw_model* model, masw_precision prec, uint32_t flags, void* stream, int8_t* sigma,
                  double* log_abs_det) {
  TraceRange trace("masw_sign_map");
  const bool dev = (flags & MASW_DEVICE_PTRS) != 0;
  int rc;
  if (!model) return fail(MASW_EINVAL, "model: null pointer");
  if ((rc = check_grid(c_test, n_c, !dev))) return rc;
  if ((rc = check_lambda(lambda, n_lambda, !dev))) return rc;
  if (!dev && (rc = check_model_values(model->n_layers, model->h, model->alpha, model->beta, model->rho, "model")))
    return rc;
  if (n_lambda > 0 && !sigma) return fail(MASW_EINVAL, "sigma: null pointer");
  if ((rc = check_common(ctx, prec, flags))) return rc;
  std::lock_guard<std::mutex> lock(ctx->mu);
  hipStream_t s = static_cast<hipStream_t>(stream);  // NULL: the default stream
  Inputs in;
  in.n_models = 1;
  in.single_N = model->n_layers;
  in.single_W = n_lambda;
  in.n_c = n_c;
  in.n_layers_total = model->n_layers;
  in.n_lam = n_lambda;
  const size_t cells = size_t(n_lambda) * size_t(n_c);
  size_t need = workspace_bytes(in, !dev, false);
  if (!dev) need += cells * (sizeof(int8_t) + sizeof(double)) + 2 * kAlign;
  if (need > ctx->sync_size) return fail(MASW_ENOMEM, "sign map exceeds the HBM budget");
  MASW_HIP(hipSetDevice(ctx->device));
  MASW_HIP(claim_arena(ctx, s));
  Bump b{ctx->arena, ctx->sync_size, 0};
  const size_t R = size_t(model->n_layers + 1);
  PrepArgs p{};
  p.counters = b.take<Counters>(1);
  p.grid_flags = b.take<uint32_t>(grid_blocks(n_c));
  p.models = b.take<ModelDesc>(1);
  p.layers64 = b.take<LayerRec64>(R);
  p.layers32 = b.take<LayerRec32>(R);
  double* c_copy = b.take<double>(size_t(n_c));
  p.c32 = b.take<float>(size_t(n_c));
  p.lam_k = b.take<double>(size_t(n_lambda));
  p.lam_model = b.take<int32_t>(size_t(n_lambda));
  p.lam_bucket = b.take<uint8_t>(size_t(n_lambda));
  p.order = b.take<int32_t>(size_t(n_lambda));
  p.n_models = 1;
  p.n_c = n_c;
  p.n_lam = n_lambda;
  int8_t* sig_dst = sigma;
  double* log_dst = log_abs_det;
  if (dev) {
    p.h = model->h; p.alpha = model->alpha; p.beta = model->beta; p.rho = model->rho;
    p.lambda = lambda; p.c_in = c_test; p.c64 = const_cast<double*>(c_test);
  } else {
    b.take<int32_t>(2); b.take<int32_t>(2);
    double* hh = b.take<double>(size_t(model->n_layers));
    double* abr = b.take<double>(R * 3);
    double* ll = b.take<double>(size_t(n_lambda));
    if (model->n_layers) MASW_HIP(hipMemcpyAsync(hh, model->h, sizeof(double) * model->n_layers, hipMemcpyHostToDevice, s));
    MASW_HIP(hipMemcpyAsync(abr, model->alpha, sizeof(double) * R, hipMemcpyHostToDevice, s));
    MASW_HIP(hipMemcpyAsync(abr + R, model->beta, sizeof(double) * R, hipMemcpyHostToDevice, s));
    MASW_HIP(hipMemcpyAsync(abr + 2 * R, model->rho, sizeof(double) * R, hipMemcpyHostToDevice, s));
    if (n_lambda) MASW_HIP(hipMemcpyAsync(ll, lambda, sizeof(double) * n_lambda, hipMemcpyHostToDevice, s));
    MASW_HIP(hipMemcpyAsync(c_copy, c_test, sizeof(double) * n_c, hipMemcpyHostToDevice, s));
    p.h = hh; p.alpha = abr; p.beta = abr + R; p.rho = abr + 2 * R; p.lambda = ll; p.c_in = c_copy; p.c64 = c_copy;
    sig_dst = b.take<int8_t>(cells);
    log_dst = log_abs_det ? b.take<double>(cells) : nullptr;
  }
  if (!b.ok()) return fail(MASW_ENOMEM, "sign map exceeds the HBM budget");
  MASW_HIP(launch_prep(p, CoopInitArgs{}, model->n_layers, n_lambda, s));
  SignMapArgs a{};
  a.models = p.models;
  a.layers64 = p.layers64;
  a.layers32 = p.layers32;
  a.c64 = p.c64;
  a.lam_k = p.lam_k;
  a.n_lam = n_lambda;
  a.n_c = n_c;
  a.sigma = sig_dst;
  a.logabs = log_dst;
  MASW_HIP(launch_sign_map(prec == MASW_PREC_SPLIT, a, s));
  ctx->stats_pending = false;
  ctx->cls_pending = false;
  ctx->last = masw_stats{};
  ctx->last_stream = s;
  ctx->last_valid = true;
  if (!dev) {
    if (cells) {
      MASW_HIP(hipMemcpyAsync(sigma, sig_dst, cells, hipMemcpyDeviceToHost, s));
      if (log_abs_det) MASW_HIP(hipMemcpyAsync(log_abs_det, log_dst, cells * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    MASW_HIP(hipStreamSynchronize(s));
  }
  return MASW_OK;
}

int masw_misfit(masw_ctx* ctx, int32_t n_models, const int32_t* lambda_off, const double* C_t, const double* C_e,
                uint32_t flags, void* stream, double* misfit) {
  TraceRange trace("masw_misfit");
  const bool dev = (flags & MASW_DEVICE_PTRS) != 0;
  if (n_models < 0) return fail(MASW_EINVAL, "n_models must be >= 0");
  if (n_models > 0 && (!lambda_off || !C_t || !C_e || !misfit)) return fail(MASW_EINVAL, "misfit: null array");
  if (flags & ~MASW_DEVICE_PTRS) return fail(MASW_EINVAL, "flags: unknown bits");
  std::vector<int32_t> off;
  if (!dev && n_models > 0) {
    off.assign(lambda_off, lambda_off + n_models + 1);
    if (off[0] != 0) return fail(MASW_EINVAL, "lambda_off must start at 0");
    for (int m = 0; m < n_models; ++m)
      if (off[m + 1] < off[m]) return fail(MASW_EINVAL, "lambda_off must be non-decreasing");
    for (int i = 0; i < off[n_models]; ++i)
      if (!(std::isfinite(C_e[i]) && C_e[i] > 0.0)) return fail(MASW_EINVAL, "C_e must be finite and > 0");
  }
  if (!ctx) return fail(MASW_EINVAL, "ctx: null context");
  if (n_models == 0) return MASW_OK;
  std::lock_guard<std::mutex> lock(ctx->mu);
  MASW_HIP(hipSetDevice(ctx->device));
  hipStream_t s = static_cast<hipStream_t>(stream);  // NULL: the default stream
  if (dev) {
    // reads and writes only caller memory: no arena claim
    MASW_HIP(launch_misfit(n_models, lambda_off, C_t, C_e, misfit, s));
    ctx->last_stream = s;
    ctx->last_valid = true;
    return MASW_OK;
  }
  const size_t W = size_t(off[n_models]);
  MASW_HIP(claim_arena(ctx, s));
  Bump b{ctx->arena, ctx->sync_size, 0};
  b.take<Counters>(1);  // keep the counters block of the last call intact
  int32_t* d_off = b.take<int32_t>(size_t(n_models) + 1);
  double* d_ct = b.take<double>(W);
  double* d_ce = b.take<double>(W);
  double* d_out = b.take<double>(size_t(n_models));
  if (!b.ok()) return fail(MASW_ENOMEM, "misfit exceeds the HBM budget");
  MASW_HIP(hipMemcpyAsync(d_off, off.data(), sizeof(int32_t) * (n_models + 1), hipMemcpyHostToDevice, s));
  if (W) {
    MASW_HIP(hipMemcpyAsync(d_ct, C_t, sizeof(double) * W, hipMemcpyHostToDevice, s));
    MASW_HIP(hipMemcpyAsync(d_ce, C_e, sizeof(double) * W, hipMemcpyHostToDevice, s));
  }
  MASW_HIP(launch_misfit(n_models, d_off, d_ct, d_ce, d_out, s));
  MASW_HIP(hipMemcpyAsync(misfit, d_out, sizeof(double) * n_models, hipMemcpyDeviceToHost, s));
  MASW_HIP(hipStreamSynchronize(s));
  ctx->last_stream = s;
  ctx->last_valid = true;
  return MASW_OK;
}

int masw_classify_picks(masw_ctx* ctx, const double* c_test, int32_t n_c, const masw_batch* batch,
                        const int32_t* idx, uint32_t flags, void* stream, int32_t* pick_class, double* c_sec) {
  TraceRange trace("masw_classify_picks");
  const bool dev = (flags & MASW_DEVICE_PTRS) != 0;
  int rc;
  if (flags & ~MASW_DEVICE_PTRS) return fail(MASW_EINVAL, "flags: unknown bits");
  if (dev && !ctx) return fail(MASW_EINVAL, "ctx: null context");
  if (!batch) return fail(MASW_EINVAL, "batch: null pointer");
  if ((rc = check_grid(c_test, n_c, !dev))) return rc;
  if (batch->n_models < 1) return fail(MASW_EINVAL, "batch: n_models must be >= 1");
  if (!batch->layer_off || !batch->lambda_off || !batch->alpha || !batch->beta || !batch->rho || !batch->lambda)
    return fail(MASW_EINVAL, "batch: null array");
  const size_t n_off = size_t(batch->n_models) + 1;
  std::vector<int32_t> loff(n_off), woff(n_off);
  hipStream_t s = static_cast<hipStream_t>(stream);  // NULL: the default stream
  if (dev) {
    MASW_HIP(hipSetDevice(ctx->device));
    MASW_HIP(hipMemcpyAsync(loff.data(), batch->layer_off, sizeof(int32_t) * n_off, hipMemcpyDeviceToHost, s));
    MASW_HIP(hipMemcpyAsync(woff.data(), batch->lambda_off, sizeof(int32_t) * n_off, hipMemcpyDeviceToHost, s));
    MASW_HIP(hipStreamSynchronize(s));
  } else {
    std::memcpy(loff.data(), batch->layer_off, sizeof(int32_t) * n_off);
    std::memcpy(woff.data(), batch->lambda_off, sizeof(int32_t) * n_off);
  }
  if (loff[0] != 0 || woff[0] != 0) return fail(MASW_EINVAL, "batch: offsets must start at 0");
  for (int m = 0; m < batch->n_models; ++m) {
    const int32_t N = loff[m + 1] - loff[m];
    if (N < 0 || N > MASW_MAX_LAYERS) return fail(MASW_EINVAL, "batch: layer_off must be non-decreasing, N <= MASW_MAX_LAYERS");
    if (woff[m + 1] < woff[m]) return fail(MASW_EINVAL, "batch: lambda_off must be non-decreasing");
  }
  const int64_t L = loff[batch->n_models];
  const int64_t W = woff[batch->n_models];
  const int64_t R = L + batch->n_models;  // alpha/beta/rho entries
  if (L > 0 && !batch->h) return fail(MASW_EINVAL, "batch: null h");
  if (W > 0 && (!idx || !pick_class)) return fail(MASW_EINVAL, "idx and pick_class required");
  if (!dev) {
    for (int m = 0; m < batch->n_models; ++m) {
      const int32_t N = loff[m + 1] - loff[m];
      const int64_t r0 = int64_t(loff[m]) + m;
      if ((rc = check_model_values(N, batch->h + loff[m], batch->alpha + r0, batch->beta + r0, batch->rho + r0,
                                   ("batch model " + std::to_string(m)).c_str())))
        return rc;
    }
    if ((rc = check_lambda(batch->lambda, int32_t(W), true))) return rc;
  }
  if (!ctx) return fail(MASW_EINVAL, "ctx: null context");
  if (W == 0) return MASW_OK;
  std::lock_guard<std::mutex> lock(ctx->mu);
  MASW_HIP(hipSetDevice(ctx->device));
  MASW_HIP(claim_arena(ctx, s));
  Bump b{ctx->arena, ctx->sync_size, 0};
  b.take<Counters>(1);  // keep the counters block of the last call intact
  ClassifyArgs a;
  a.n_models = batch->n_models;
  a.n_c = n_c;
  a.n_lam = W;
  a.counters = b.take<uint64_t>(3);
  ctx->stats_pending = false;
  ctx->cls_pending = false;
  if (dev) {
    a.layer_off = batch->layer_off; a.h = batch->h; a.alpha = batch->alpha; a.beta = batch->beta;
    a.rho = batch->rho; a.lambda_off = batch->lambda_off; a.lambda = batch->lambda; a.c = c_test;
    a.idx = idx; a.cls = pick_class; a.c_sec = c_sec;
    MASW_HIP(hipEventRecord(ctx->cls_ev[0], s));
    MASW_HIP(launch_classify(a, s));
    MASW_HIP(hipEventRecord(ctx->cls_ev[1], s));
    ctx->cls_counters = a.counters;
    ctx->cls_pending = true;
    ctx->last_stream = s;
    ctx->last_valid = true;
    return MASW_OK;
  }
  int32_t* d_loff = b.take<int32_t>(n_off);
  int32_t* d_woff = b.take<int32_t>(n_off);
  double* d_h = b.take<double>(size_t(L));
  double* d_abr = b.take<double>(size_t(R) * 3);
  double* d_lam = b.take<double>(size_t(W));
  double* d_c = b.take<double>(size_t(n_c));
  int32_t* d_idx = b.take<int32_t>(size_t(W));
  int32_t* d_cls = b.take<int32_t>(size_t(W));
  double* d_sec = b.take<double>(size_t(W));
  if (!b.ok()) return fail(MASW_ENOMEM, "classification exceeds the HBM budget");
  MASW_HIP(hipMemcpyAsync(d_loff, loff.data(), sizeof(int32_t) * n_off, hipMemcpyHostToDevice, s));
  MASW_HIP(hipMemcpyAsync(d_woff, woff.data(), sizeof(int32_t) * n_off, hipMemcpyHostToDevice, s));
  if (L) MASW_HIP(hipMemcpyAsync(d_h, batch->h, sizeof(double) * L, hipMemcpyHostToDevice, s));
  MASW_HIP(hipMemcpyAsync(d_abr, batch->alpha, sizeof(double) * R, hipMemcpyHostToDevice, s));
  MASW_HIP(hipMemcpyAsync(d_abr + R, batch->beta, sizeof(double) * R, hipMemcpyHostToDevice, s));
  MASW_HIP(hipMemcpyAsync(d_abr + 2 * R, batch->rho, sizeof(double) * R, hipMemcpyHostToDevice, s));
  MASW_HIP(hipMemcpyAsync(d_lam, batch->lambda, sizeof(double) * W, hipMemcpyHostToDevice, s));
  MASW_HIP(hipMemcpyAsync(d_c, c_test, sizeof(double) * n_c, hipMemcpyHostToDevice, s));
  MASW_HIP(hipMemcpyAsync(d_idx, idx, sizeof(int32_t) * W, hipMemcpyHostToDevice, s));
  a.layer_off = d_loff; a.h = d_h; a.alpha = d_abr; a.beta = d_abr + R; a.rho = d_abr + 2 * R;
  a.lambda_off = d_woff; a.lambda = d_lam; a.c = d_c; a.idx = d_idx; a.cls = d_cls; a.c_sec = d_sec;
  MASW_HIP(hipEventRecord(ctx->cls_ev[0], s));
  MASW_HIP(launch_classify(a, s));
  MASW_HIP(hipEventRecord(ctx->cls_ev[1], s));
  ctx->cls_counters = a.counters;
  ctx->cls_pending = true;
  MASW_HIP(hipMemcpyAsync(pick_class, d_cls, sizeof(int32_t) * W, hipMemcpyDeviceToHost, s));
  if (c_sec) MASW_HIP(hipMemcpyAsync(c_sec, d_sec, sizeof(double) * W, hipMemcpyDeviceToHost, s));
  MASW_HIP(hipStreamSynchronize(s));
  ctx->last_stream = s;
  ctx->last_valid = true;
  return MASW_OK;
}

int masw_set_opts(masw_ctx* ctx, const masw_opts* opts) {
  masw_opts o{};
  if (opts) o = *opts;
  const double tol = o.refine_rel_tol == 0.0 ? kRefineRel : o.refine_rel_tol;
  const double thr = o.noise_threshold == 0.0 ? 1e-2 : o.noise_threshold;
  if (!(tol >= 1e-15 && tol <= 1e-3)) return fail(MASW_EINVAL, "opts: refine_rel_tol out of [1e-15, 1e-3]");
  if (!(thr > 0.0 && thr <= 1.0)) return fail(MASW_EINVAL, "opts: noise_threshold out of (0, 1]");
  const int g = o.waves_per_item;
  if (!(g == 0 || g == 1 || g == 2 || g == 4 || g == 8 || g == 16))
    return fail(MASW_EINVAL, "opts: waves_per_item must be 0, 1, 2, 4, 8 or 16");
  if (!(o.shared_window == -1 || (o.shared_window >= 0 && o.shared_window <= 1024)))
    return fail(MASW_EINVAL, "opts: shared_window must be -1 or in [0, 1024]");
  if (!(o.first_item_priority == 0 || o.first_item_priority == -1))
    return fail(MASW_EINVAL, "opts: first_item_priority must be 0 or -1");
  if (!(o.timing_events == 0 || o.timing_events == 1)) return fail(MASW_EINVAL, "opts: timing_events must be 0 or 1");
  if (!ctx) return fail(MASW_EINVAL, "ctx: null context");
  std::lock_guard<std::mutex> lock(ctx->mu);
  if (o.timing_events && !ctx->tslot[0].ev[0]) {
    // the slots' events, on first use (device-scope release: they only time
    // launches, so they need no system-scope cache writeback)
    MASW_HIP(hipSetDevice(ctx->device));
    for (auto& t : ctx->tslot)
      for (auto& e : t.ev)
        if (!e) MASW_HIP(hipEventCreateWithFlags(&e, hipEventReleaseToDevice));
  }
  ctx->timing_events = o.timing_events == 1;
  ctx->refine_rel = tol;
  ctx->noise_threshold = thr;
  ctx->forced_waves = g;
  ctx->shared_sweeps = o.shared_window != -1;
  ctx->shared_window = o.shared_window > 0 ? o.shared_window : 8;
  ctx->first_item_priority = o.first_item_priority == 0;
  return MASW_OK;
}

int masw_get_opts(masw_ctx* ctx, masw_opts* out) {
  if (!ctx || !out) return fail(MASW_EINVAL, "null argument");
  std::lock_guard<std::mutex> lock(ctx->mu);
  masw_opts o{};
  o.refine_rel_tol = ctx->refine_rel;
  o.noise_threshold = ctx->noise_threshold;
  o.waves_per_item = ctx->forced_waves;
  o.shared_window = ctx->shared_sweeps ? ctx->shared_window : -1;
  o.first_item_priority = ctx->first_item_priority ? 0 : -1;
  o.timing_events = ctx->timing_events ? 1 : 0;
  *out = o;
  return MASW_OK;
}

int masw_get_stats(masw_ctx* ctx, masw_stats* out) {
  if (!ctx || !out) return fail(MASW_EINVAL, "null argument");
  std::lock_guard<std::mutex> lock(ctx->mu);
  if (ctx->cls_pending) {
    MASW_HIP(hipSetDevice(ctx->device));
    MASW_HIP(hipEventSynchronize(ctx->cls_ev[1]));
    uint64_t c[3];
    MASW_HIP(hipMemcpy(c, ctx->cls_counters, sizeof(c), hipMemcpyDeviceToHost));
    float ms = 0.f;
    MASW_HIP(hipEventElapsedTime(&ms, ctx->cls_ev[0], ctx->cls_ev[1]));
    ctx->last = masw_stats{};
    ctx->last.classify_evals = c[0];
    ctx->last.classify_layers = c[1];
    ctx->last.classify_steps = c[2];
    ctx->last.sweep_ms = ms;
    ctx->last.total_ms = ms;
    ctx->cls_pending = false;
  }
  if (ctx->stats_pending) {
    MASW_HIP(hipSetDevice(ctx->device));
    if (ctx->last_valid) MASW_HIP(hipStreamSynchronize(ctx->last_stream));
    Counters c{};  // a fused launch has no staging, which is what clears the counters
    if (!ctx->last_fused) MASW_HIP(hipMemcpy(&c, ctx->counters, sizeof(Counters), hipMemcpyDeviceToHost));
    ctx->last.useful_evals = c.useful;
    ctx->last.sweep_evals = c.sweep;
    ctx->last.check_evals = c.check;
    ctx->last.refine_evals = c.refine;
    ctx->last.helper_evals = c.helper;
    ctx->last.inertia_evals = c.inertia_evals;
    ctx->last.inertia_entries = c.inertia_entries;
    ctx->last.inertia_pivots = c.inertia_pivots;
    ctx->last.shared_stalls = c.coop_stall;
    if (ctx->wg_rows > 0) {  // the launch's per-workgroup rows (SweepArgs::wg_counts)
      std::vector<unsigned long long> rows(size_t(ctx->wg_rows) * kWgCounts);
      MASW_HIP(hipMemcpy(rows.data(), ctx->wg_counts, rows.size() * sizeof(unsigned long long),
                         hipMemcpyDeviceToHost));
      unsigned long long sum[kWgCounts] = {};
      for (size_t i = 0; i < rows.size(); ++i) sum[i % kWgCounts] += rows[i];
      ctx->last.sweep_evals += sum[0];
      ctx->last.check_evals += sum[1];
      ctx->last.refine_evals += sum[2];
      ctx->last.useful_evals += sum[3];
      ctx->last.helper_evals += sum[4];
      ctx->last.inertia_evals += sum[5];
      ctx->last.inertia_entries += sum[6];
      ctx->last.inertia_pivots += sum[7];
    }
    if (ctx->tslot_last >= 0) {
      masw_ctx::TimingSlot& T = ctx->tslot[ctx->tslot_last];
      if (T.pending) MASW_HIP(resolve_timing(ctx));
      ctx->last.sweep_ms = T.sweep_ms;
      ctx->last.total_ms = T.total_ms;
    }
    ctx->stats_pending = false;
  }
  *out = ctx->last;
  return MASW_OK;
}

int masw_get_timing(masw_ctx* ctx, int reset, masw_timing* out) {
  if (!ctx || !out) return fail(MASW_EINVAL, "null argument");
  std::lock_guard<std::mutex> lock(ctx->mu);
  MASW_HIP(hipSetDevice(ctx->device));
  MASW_HIP(resolve_timing(ctx));
  *out = ctx->timing;
  if (reset) ctx->timing = masw_timing{};
  return MASW_OK;
}

}  // extern "C"
