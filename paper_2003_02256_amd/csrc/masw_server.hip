// Serving loop: continuous batching of dispersion-curve requests on one GPU.
//
// masw_submit checks and copies a request and queues it.  A driver thread
// repeats ticks:
//   1. admission: while a slot is free and the request's device footprint
//      fits the serving pool (a first-fit allocator over the context's HBM
//      budget), pack its raw inputs into pinned staging behind the tick's
//      admit list; one H2D copy moves both, and the admit kernel moves each
//      request's inputs into its pool block and writes its layer records, k
//      values, FP32 grid and item states on the device;
//   2. one replay of a captured hipGraph (copy of the tick descriptor, the
//      tick kernel), chosen among four graphs by the number of wavefronts per
//      wavelength; the descriptor carries the tick's start value of the
//      queue counter, which is never cleared;
//   3. harvest: requests whose last wavelength finished in this tick (a flag
//      the kernel writes to pinned memory) have their results, already in
//      pinned memory, copied out; their slot and memory are released.
// Every wavelength advances at most rounds_per_tick sweep rounds per tick
// and keeps its search state in HBM, so requests arriving while others run
// are admitted at the next tick and share the GPU with them.
#include <hip/hip_runtime.h>
#include <time.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "masw.h"
#include "masw_host.hpp"
#include "masw_internal.hpp"

namespace masw {
namespace {

uint64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return uint64_t(ts.tv_sec) * 1000000000ull + uint64_t(ts.tv_nsec);
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over [0, size) with coalescing of freed blocks.
class PoolAlloc {
 public:
  void reset(size_t size) {
    free_.clear();
    free_[0] = size;
  }
  bool alloc(size_t n, size_t* off) {
    n = align_up(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      *off = it->first;
      const size_t rest = it->second - n, next = it->first + n;
      free_.erase(it);
      if (rest) free_[next] = rest;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = align_up(n);
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;
};

struct Request {
  uint64_t ticket = 0;
  int prec = 0;
  int N = 0, W = 0, n_c = 0;
  int n_real = 0;           // grid points below the half-space's S velocity
  uint32_t flags = 0;       // MASW_CHECK_NOISE, MASW_NO_REFINE
  std::vector<double> raw;  // h[N], alpha, beta, rho [N+1], lambda[W], c[n_c]
  std::vector<double> ct, cref;
  std::vector<int32_t> idx, status;
  int slot = -1;
  bool done = false;
  size_t pool_off = 0, pool_bytes = 0;
  masw_request_info info{};
};

// Offsets of a request's parts inside its pool block.
struct Layout {
  size_t raw, l64, l32, c32, lamk, state, total;
};

Layout layout_of(int N, int W, int n_c) {
  Layout L;
  size_t o = 0;
  L.raw = o;
  o = align_up(o + sizeof(double) * (size_t(N) + 3 * size_t(N + 1) + size_t(W) + size_t(n_c)));
  L.l64 = o;
  o = align_up(o + sizeof(LayerRec64) * size_t(N + 1));
  L.l32 = o;
  o = align_up(o + sizeof(LayerRec32) * size_t(N + 1));
  L.c32 = o;
  o = align_up(o + sizeof(float) * size_t(n_c));
  L.lamk = o;
  o = align_up(o + sizeof(double) * size_t(W));
  L.state = o;
  o = align_up(o + sizeof(ItemState) * size_t(W));
  L.total = o;
  return L;
}

}  // namespace

struct Server {
  masw_ctx* ctx = nullptr;
  masw_server_opts opt{};
  hipStream_t stream = nullptr;
  // device memory (tail of the context arena)
  char* region = nullptr;
  size_t region_size = 0;
  char* pool = nullptr;
  size_t pool_size = 0;
  TickDesc* desc_dev = nullptr;
  AdmitList* admit_dev = nullptr;   // head of the device staging area
  int32_t* remaining_dev = nullptr;
  Counters* counters_dev = nullptr;
  // pinned host memory
  TickDesc* desc_host = nullptr;
  AdmitList* admit_host = nullptr;  // head of the pinned staging area
  double* out_ct = nullptr;
  double* out_cref = nullptr;
  int32_t* out_idx = nullptr;
  int32_t* out_status = nullptr;
  int32_t* host_done = nullptr;
  uint32_t* host_tick = nullptr;    // the kernel's end-of-tick word (TickArgs::host_tick)
  int32_t* out_idx_dev = nullptr;   // device views of out_idx, out_status
  int32_t* out_status_dev = nullptr;
  double noise_threshold = 1e-2;    // MASW_CHECK_NOISE band of served requests
  char* staging = nullptr;          // pinned: admit list, then raw inputs
  char* staging_dev = nullptr;      // device copy of the same
  size_t staging_size = 0;
  // one captured tick per G = 1, 2, 4, 8
  hipGraph_t graph[4] = {};
  hipGraphExec_t exec[4] = {};
  int bpc[4] = {};
  int blocks[4] = {};
  uint32_t queue_base = 0;  // value of the tick queue counter at the next tick
  uint32_t exit_base = 0;   // value of Counters::tick_exit at the next tick
  uint32_t tick_seq = 0;    // number of the last tick launched
  // host state
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_watch;
  std::thread driver, watchdog;
  uint64_t tick_start_ns = 0;  // start of the tick in flight, 0 if none
  bool stop = false;
  bool stop_watch = false;
  bool failed = false;
  std::atomic<bool> failed_flag{false};  // `failed`, readable without mu (the tick wait)
  std::string fail_msg;
  std::deque<Request*> pending;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> requests;
  Request* slot_req[kMaxSlots] = {};
  int resident = 0;
  PoolAlloc alloc;
  uint64_t next_ticket = 1;
  masw_server_stats stats{};

  int pick_graph(int units) const;
  void run();
  void watch();
  void fail_all(const std::string& msg);  // with mu held
  void release_all();
  hipError_t check_noise_of_finished();  // driver thread, after a tick
};

void Server::fail_all(const std::string& msg) {
  failed = true;
  failed_flag.store(true, std::memory_order_release);
  fail_msg = msg;
  for (auto& kv : requests) kv.second->done = true;
  cv_done.notify_all();
}

// Watchdog: fails the server when a tick has been in flight longer than
// opt.tick_timeout_us, so that waiters return instead of blocking on a tick
// that does not come back.  The driver also checks each finished tick's
// duration itself.
void Server::watch() {
  const uint64_t limit_ns = uint64_t(opt.tick_timeout_us) * 1000ull;
  const auto period = std::chrono::microseconds(std::clamp<int64_t>(opt.tick_timeout_us / 2, 1000, 100000));
  std::unique_lock<std::mutex> lk(mu);
  while (!stop_watch) {
    if (!failed && tick_start_ns != 0 && now_ns() - tick_start_ns > limit_ns)
      fail_all("serving watchdog: a tick ran longer than tick_timeout_us");
    cv_watch.wait_for(lk, period);
  }
}

int Server::pick_graph(int units) const {
  for (int gi = 3; gi > 0; --gi) {
    const int G = 1 << gi;
    if (bpc[gi] >= 2 && int64_t(units) * G <= 4 * int64_t(ctx->cus) * bpc[gi] * G) return gi;
  }
  return 0;
}

void Server::run() {
  (void)hipSetDevice(ctx->device);
  roctxNameOsThread("masw serving driver");
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_work.wait(lk, [&] { return stop || !pending.empty() || resident > 0; });
    if (stop && pending.empty() && resident == 0) break;

    // 1. admission
    int n_admit = 0, max_raw = 0;
    size_t staged = align_up(sizeof(AdmitList));
    bool waited = false;
    while (!pending.empty() && n_admit < kMaxAdmit && resident < kMaxSlots) {
      Request* r = pending.front();
      const Layout L = layout_of(r->N, r->W, r->n_c);
      const size_t raw_bytes = r->raw.size() * sizeof(double);
      if (staged + align_up(raw_bytes) > staging_size) break;
      size_t off = 0;
      if (!alloc.alloc(L.total, &off)) {
        waited = true;
        break;
      }
      int slot = 0;
      while (slot_req[slot]) ++slot;
      pending.pop_front();
      r->slot = slot;
      r->pool_off = off;
      r->pool_bytes = L.total;
      r->info.admit_ns = now_ns();
      slot_req[slot] = r;
      ++resident;
      host_done[slot] = 0;
      std::memcpy(staging + staged, r->raw.data(), raw_bytes);
      char* base = pool + off;
      SlotDesc d{};
      d.raw = reinterpret_cast<const double*>(base + L.raw);
      d.L64 = reinterpret_cast<LayerRec64*>(base + L.l64);
      d.L32 = reinterpret_cast<LayerRec32*>(base + L.l32);
      d.c32 = reinterpret_cast<float*>(base + L.c32);
      d.lam_k = reinterpret_cast<double*>(base + L.lamk);
      d.state = reinterpret_cast<ItemState*>(base + L.state);
      d.N = r->N;
      d.W = r->W;
      d.n_c = r->n_c;
      d.prec = r->prec;
      d.n_real = r->n_real;
      d.flags = r->flags;
      d.out_base = slot * opt.max_lambda;
      desc_host->slot[slot] = d;
      admit_host->slot[n_admit] = slot;
      admit_host->desc[n_admit] = d;
      admit_host->src[n_admit] = reinterpret_cast<const double*>(staging_dev + staged);
      max_raw = std::max(max_raw, int(r->raw.size()));
      staged += align_up(raw_bytes);
      ++n_admit;
    }
    if (waited) ++stats.admit_waits;
    admit_host->n = n_admit;

    // tick descriptor: every resident request
    int n_active = 0, units = 0;
    for (int s = 0; s < kMaxSlots; ++s) {
      if (!slot_req[s]) continue;
      desc_host->active[n_active] = s;
      desc_host->prefix[n_active] = units;
      units += slot_req[s]->W;
      ++n_active;
    }
    desc_host->prefix[n_active] = units;
    desc_host->n_active = n_active;
    desc_host->n_units = units;
    desc_host->budget = opt.rounds_per_tick;
    desc_host->base = queue_base;
    desc_host->exit_base = exit_base;
    desc_host->seq = ++tick_seq;
    const int gi = units > 0 ? pick_graph(units) : 0;
    stats.resident = uint32_t(resident);
    stats.max_resident = std::max(stats.max_resident, uint32_t(resident));
    const uint64_t t0 = now_ns();
    tick_start_ns = t0;
    lk.unlock();

    // 2. device work, in stream order
    hipError_t e = hipSuccess;
    roctxRangePushA("masw_tick");
    if (n_admit > 0) e = hipMemcpyAsync(staging_dev, staging, staged, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && n_admit > 0) e = launch_admit(admit_dev, n_admit, max_raw, remaining_dev, stream);
    if (e == hipSuccess && units > 0) {
      e = hipGraphLaunch(exec[gi], stream);
      queue_base += uint32_t(units) + uint32_t(blocks[gi]);  // one final claim per workgroup
      exit_base += uint32_t(blocks[gi]);
    }
    if (e == hipSuccess && units > 0) {
      // the tick kernel's last workgroup writes the tick's number to pinned
      // memory; spinning on it returns sooner than a stream synchronisation.
      // The watchdog ends the wait by failing the server.
      while (__atomic_load_n(host_tick, __ATOMIC_ACQUIRE) != tick_seq &&
             !failed_flag.load(std::memory_order_acquire))
        __builtin_ia32_pause();
      const hipError_t q = hipStreamQuery(stream);  // an error of the tick's work, if any
      if (q != hipSuccess && q != hipErrorNotReady) e = q;
    } else if (e == hipSuccess) {
      e = hipStreamSynchronize(stream);
    }
    if (e == hipSuccess) e = check_noise_of_finished();
    roctxRangePop();
    const uint64_t t1 = now_ns();

    // 3. harvest
    lk.lock();
    tick_start_ns = 0;
    stats.busy_ms += double(t1 - t0) * 1e-6;
    if (e != hipSuccess) {
      fail_all(std::string("serving tick: ") + hipGetErrorString(e));
      break;
    }
    if (!failed && t1 - t0 > uint64_t(opt.tick_timeout_us) * 1000ull)
      fail_all("serving watchdog: a tick ran longer than tick_timeout_us");
    if (failed) break;
    ++stats.ticks;
    for (int s = 0; s < kMaxSlots; ++s) {
      Request* r = slot_req[s];
      if (!r) continue;
      ++r->info.ticks;
      if (!host_done[s]) continue;
      const size_t o = size_t(s) * size_t(opt.max_lambda);
      std::memcpy(r->ct.data(), out_ct + o, sizeof(double) * r->W);
      std::memcpy(r->cref.data(), out_cref + o, sizeof(double) * r->W);
      std::memcpy(r->idx.data(), out_idx + o, sizeof(int32_t) * r->W);
      std::memcpy(r->status.data(), out_status + o, sizeof(int32_t) * r->W);
      r->done = true;
      r->info.done_ns = now_ns();
      alloc.release(r->pool_off, r->pool_bytes);
      slot_req[s] = nullptr;
      --resident;
      ++stats.completed;
    }
    cv_done.notify_all();
  }
}

// The noise band of the picks of requests with MASW_CHECK_NOISE that the
// tick just finished, before their results are harvested: one launch per 16
// such requests, then one synchronisation.
hipError_t Server::check_noise_of_finished() {
  ServeNoiseList list{};
  bool launched = false;
  hipError_t e = hipSuccess;
  for (int s = 0; s < kMaxSlots && e == hipSuccess; ++s) {
    const Request* r = slot_req[s];
    if (!r || !host_done[s] || !(r->flags & MASW_CHECK_NOISE)) continue;
    list.slot[list.n++] = desc_host->slot[s];
    if (list.n == kNoiseList) {
      e = launch_serve_noise(list, out_idx_dev, out_status_dev, noise_threshold, stream);
      launched = true;
      list.n = 0;
    }
  }
  if (e == hipSuccess && list.n > 0) {
    e = launch_serve_noise(list, out_idx_dev, out_status_dev, noise_threshold, stream);
    launched = true;
  }
  if (e == hipSuccess && launched) e = hipStreamSynchronize(stream);
  return e;
}

void Server::release_all() {
  for (auto& g : exec)
    if (g) (void)hipGraphExecDestroy(g);
  for (auto& g : graph)
    if (g) (void)hipGraphDestroy(g);
  if (stream) (void)hipStreamDestroy(stream);
  for (void* p : {static_cast<void*>(desc_host), static_cast<void*>(out_ct),
                  static_cast<void*>(out_cref), static_cast<void*>(out_idx), static_cast<void*>(out_status),
                  static_cast<void*>(host_done), static_cast<void*>(host_tick), static_cast<void*>(staging)})
    if (p) (void)hipHostFree(p);
}

void server_destroy(Server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->driver.joinable()) s->driver.join();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop_watch = true;
  }
  s->cv_watch.notify_all();
  if (s->watchdog.joinable()) s->watchdog.join();
  (void)hipSetDevice(s->ctx->device);
  s->ctx->sync_size = s->ctx->arena_size;
  s->release_all();
  delete s;
}

}  // namespace masw

using namespace masw;

extern "C" {

int masw_server_start(masw_ctx* ctx, const masw_server_opts* opts) {
  if (!ctx) return fail(MASW_EINVAL, "ctx: null context");
  masw_server_opts o{};
  if (opts) o = *opts;
  if (o.max_layers == 0) o.max_layers = 64;
  if (o.max_lambda == 0) o.max_lambda = 512;
  if (o.max_grid == 0) o.max_grid = 32768;
  if (o.rounds_per_tick == 0) o.rounds_per_tick = 16;
  if (o.tick_timeout_us == 0) o.tick_timeout_us = 10000000;
  if (o.max_layers < 0 || o.max_layers > MASW_MAX_LAYERS || o.max_lambda < 1 || o.max_grid < 2 ||
      o.rounds_per_tick < 1 || o.tick_timeout_us < 0 || (o.search_inertia != 0 && o.search_inertia != 1) ||
      o.reserved != 0)
    return fail(MASW_EINVAL, "server opts: out of range");
  std::lock_guard<std::mutex> lock(ctx->mu);
  if (ctx->server) return fail(MASW_EBUSY, "server already running");
  if (o.pool_bytes == 0) o.pool_bytes = ctx->arena_size / 2;
  // staging: the admit list, then room for a few of the largest requests' raw inputs
  const size_t staging_size =
      align_up(sizeof(AdmitList)) +
      align_up(sizeof(double) * (size_t(4) * (o.max_layers + 1) + o.max_lambda + o.max_grid)) * 8;
  const size_t fixed = align_up(sizeof(TickDesc)) + staging_size +
                       align_up(sizeof(int32_t) * kMaxSlots) + align_up(sizeof(Counters));
  const size_t region = align_up(o.pool_bytes) + fixed;
  if (region + (size_t(16) << 20) > ctx->arena_size)
    return fail(MASW_ENOMEM, "serving pool leaves less than 16 MiB of the budget for synchronous calls");
  MASW_HIP(hipSetDevice(ctx->device));
  if (ctx->last_valid) MASW_HIP(hipStreamSynchronize(ctx->last_stream));  // no call still uses the tail

  Server* s = new Server();
  s->ctx = ctx;
  s->opt = o;
  s->region_size = region;
  s->region = ctx->arena + ((ctx->arena_size - region) & ~(kAlign - 1));
  char* p = s->region;
  s->desc_dev = reinterpret_cast<TickDesc*>(p);
  p += align_up(sizeof(TickDesc));
  s->staging_dev = p;
  s->admit_dev = reinterpret_cast<AdmitList*>(p);
  p += staging_size;
  s->remaining_dev = reinterpret_cast<int32_t*>(p);
  p += align_up(sizeof(int32_t) * kMaxSlots);
  s->counters_dev = reinterpret_cast<Counters*>(p);
  p += align_up(sizeof(Counters));
  s->pool = p;
  s->pool_size = align_up(o.pool_bytes);
  s->alloc.reset(s->pool_size);

  auto bail = [&](const std::string& msg) {
    s->release_all();
    delete s;
    return fail(MASW_EDEVICE, msg);
  };
  const size_t n_out = size_t(kMaxSlots) * size_t(o.max_lambda);
  // room to stage a few of the largest requests per tick
  s->staging_size = staging_size;
  if (hipHostMalloc(reinterpret_cast<void**>(&s->desc_host), sizeof(TickDesc), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&s->out_ct), sizeof(double) * n_out, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&s->out_cref), sizeof(double) * n_out, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&s->out_idx), sizeof(int32_t) * n_out, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&s->out_status), sizeof(int32_t) * n_out, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&s->host_done), sizeof(int32_t) * kMaxSlots, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&s->host_tick), sizeof(uint32_t), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&s->staging), s->staging_size, hipHostMallocDefault) != hipSuccess)
    return bail("hipHostMalloc failed for the serving buffers");
  std::memset(s->desc_host, 0, sizeof(TickDesc));
  s->admit_host = reinterpret_cast<AdmitList*>(s->staging);
  std::memset(s->admit_host, 0, sizeof(AdmitList));
  std::memset(s->host_done, 0, sizeof(int32_t) * kMaxSlots);
  *s->host_tick = 0;
  if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess)
    return bail("hipStreamCreate failed");
  // the tick counters start at zero once; ticks never clear them (TickDesc::base)
  if (hipMemsetAsync(s->counters_dev, 0, sizeof(Counters), s->stream) != hipSuccess ||
      hipStreamSynchronize(s->stream) != hipSuccess)
    return bail("clearing the tick counters failed");

  TickArgs ta{};
  ta.desc = s->desc_dev;
  ta.slot_remaining = s->remaining_dev;
  ta.counters = s->counters_dev;
  ta.refine = 1;
  ta.inertia = o.search_inertia;
  ta.refine_rel = ctx->refine_rel;
  s->noise_threshold = ctx->noise_threshold;
  void* dp = nullptr;
  if (hipHostGetDevicePointer(&dp, s->out_ct, 0) != hipSuccess) return bail("hipHostGetDevicePointer failed");
  ta.out_ct = static_cast<double*>(dp);
  if (hipHostGetDevicePointer(&dp, s->out_cref, 0) != hipSuccess) return bail("hipHostGetDevicePointer failed");
  ta.out_cref = static_cast<double*>(dp);
  if (hipHostGetDevicePointer(&dp, s->out_idx, 0) != hipSuccess) return bail("hipHostGetDevicePointer failed");
  ta.out_idx = static_cast<int32_t*>(dp);
  s->out_idx_dev = ta.out_idx;
  if (hipHostGetDevicePointer(&dp, s->out_status, 0) != hipSuccess) return bail("hipHostGetDevicePointer failed");
  ta.out_status = static_cast<int32_t*>(dp);
  s->out_status_dev = ta.out_status;
  if (hipHostGetDevicePointer(&dp, s->host_done, 0) != hipSuccess) return bail("hipHostGetDevicePointer failed");
  ta.host_done = static_cast<int32_t*>(dp);
  if (hipHostGetDevicePointer(&dp, s->host_tick, 0) != hipSuccess) return bail("hipHostGetDevicePointer failed");
  ta.host_tick = static_cast<uint32_t*>(dp);
  for (int gi = 0; gi < 4; ++gi) {
    const int G = 1 << gi;
    s->bpc[gi] = tick_blocks_per_cu(G, o.search_inertia != 0);
    const int blocks = ctx->cus * std::max(1, s->bpc[gi]);
    s->blocks[gi] = blocks;
    if (hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return bail("hipStreamBeginCapture failed");
    hipError_t e = hipMemcpyAsync(s->desc_dev, s->desc_host, sizeof(TickDesc), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = launch_tick(G, blocks, s->stream, ta);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(s->stream, &g);
    s->graph[gi] = g;
    if (e != hipSuccess || e2 != hipSuccess) return bail("capturing the tick graph failed");
    if (hipGraphInstantiate(&s->exec[gi], g, nullptr, nullptr, 0) != hipSuccess)
      return bail("hipGraphInstantiate failed");
  }
  // One empty replay of each graph (no units: every workgroup makes its one
  // final claim and exits), so that no served tick pays a first launch.
  for (int gi = 0; gi < 4; ++gi) {
    s->desc_host->base = s->queue_base;
    if (hipGraphLaunch(s->exec[gi], s->stream) != hipSuccess || hipStreamSynchronize(s->stream) != hipSuccess)
      return bail("warming the tick graphs failed");
    s->queue_base += uint32_t(s->blocks[gi]);
    s->exit_base += uint32_t(s->blocks[gi]);
    s->desc_host->exit_base = s->exit_base;
  }
  s->stats.pool_bytes = s->pool_size;
  ctx->sync_size = (ctx->arena_size - region) & ~(kAlign - 1);
  s->driver = std::thread([s] { s->run(); });
  s->watchdog = std::thread([s] { s->watch(); });
  ctx->server = s;
  return MASW_OK;
}

int masw_server_stop(masw_ctx* ctx) {
  if (!ctx) return fail(MASW_EINVAL, "ctx: null context");
  std::lock_guard<std::mutex> lock(ctx->mu);
  if (!ctx->server) return fail(MASW_EBUSY, "server not running");
  server_destroy(ctx->server);
  ctx->server = nullptr;
  return MASW_OK;
}

int masw_submit(masw_ctx* ctx, const double* c_test, int32_t n_c, const double* lambda, int32_t n_lambda,
                const masw_model* model, masw_precision prec, uint32_t flags, uint64_t* ticket) {
  int rc;
  if (!model) return fail(MASW_EINVAL, "model: null pointer");
  if (!ticket) return fail(MASW_EINVAL, "ticket: null pointer");
  if ((rc = check_grid(c_test, n_c, true))) return rc;
  if ((rc = check_lambda(lambda, n_lambda, true))) return rc;
  if ((rc = check_model_values(model->n_layers, model->h, model->alpha, model->beta, model->rho, "model")))
    return rc;
  if (prec != MASW_PREC_FP64 && prec != MASW_PREC_SPLIT) return fail(MASW_EINVAL, "prec: unknown precision");
  if (flags & ~(MASW_CHECK_NOISE | MASW_NO_REFINE))
    return fail(MASW_EINVAL, "flags: a request takes only MASW_CHECK_NOISE and MASW_NO_REFINE");
  if (!ctx) return fail(MASW_EINVAL, "ctx: null context");
  Server* s = ctx->server;
  if (!s) return fail(MASW_EBUSY, "server not running");
  const int N = model->n_layers;
  if (N > s->opt.max_layers || n_lambda > s->opt.max_lambda || n_c > s->opt.max_grid)
    return fail(MASW_EINVAL, "request exceeds the server's max_layers / max_lambda / max_grid");
  if (layout_of(N, n_lambda, n_c).total > s->pool_size)
    return fail(MASW_ENOMEM, "request can never fit the serving pool");
  auto r = std::make_unique<Request>();
  r->prec = prec;
  r->flags = flags;
  r->N = N;
  r->W = n_lambda;
  r->n_c = n_c;
  {
    // first grid point with c^2 / beta_hs^2 >= 1, in the arithmetic of the
    // device's inertia-count test (the grid rises, checked above)
    const double be = model->beta[N];
    const double ib2 = 1.0 / (be * be);
    int lo = 0, hi = n_c;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      const double c = c_test[mid];
      if (c * c * ib2 < 1.0) lo = mid + 1; else hi = mid;
    }
    r->n_real = lo;
  }
  r->raw.reserve(size_t(N) + 3 * size_t(N + 1) + size_t(n_lambda) + size_t(n_c));
  r->raw.insert(r->raw.end(), model->h, model->h + N);
  r->raw.insert(r->raw.end(), model->alpha, model->alpha + N + 1);
  r->raw.insert(r->raw.end(), model->beta, model->beta + N + 1);
  r->raw.insert(r->raw.end(), model->rho, model->rho + N + 1);
  r->raw.insert(r->raw.end(), lambda, lambda + n_lambda);
  r->raw.insert(r->raw.end(), c_test, c_test + n_c);
  r->ct.assign(n_lambda, 0.0);
  r->cref.assign(n_lambda, 0.0);
  r->idx.assign(n_lambda, 0);
  r->status.assign(n_lambda, 0);
  r->info.submit_ns = now_ns();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->failed) return fail(MASW_EDEVICE, s->fail_msg);
    r->ticket = s->next_ticket++;
    *ticket = r->ticket;
    ++s->stats.submitted;
    if (n_lambda == 0) {  // nothing to compute
      r->done = true;
      r->info.admit_ns = r->info.done_ns = r->info.submit_ns;
      ++s->stats.completed;
    } else {
      s->pending.push_back(r.get());
    }
    s->requests.emplace(r->ticket, std::move(r));
  }
  s->cv_work.notify_one();
  return MASW_OK;
}

static int collect(Server* s, std::unique_lock<std::mutex>& lk, uint64_t ticket, double* C_t, int32_t* idx,
                   int32_t* status, double* c_ref, masw_request_info* info) {
  auto it = s->requests.find(ticket);
  if (it == s->requests.end()) return fail(MASW_ENOENT, "unknown or already collected ticket");
  Request* r = it->second.get();
  if (s->failed) return fail(MASW_EDEVICE, s->fail_msg);
  if (!r->done) return MASW_EBUSY;
  const size_t W = size_t(r->W);
  if (W && (!C_t || !idx || !status)) return fail(MASW_EINVAL, "outputs: C_t, idx, status required");
  if (W) {
    std::memcpy(C_t, r->ct.data(), sizeof(double) * W);
    std::memcpy(idx, r->idx.data(), sizeof(int32_t) * W);
    std::memcpy(status, r->status.data(), sizeof(int32_t) * W);
    if (c_ref) std::memcpy(c_ref, r->cref.data(), sizeof(double) * W);
  }
  if (info) *info = r->info;
  s->requests.erase(it);
  (void)lk;
  return MASW_OK;
}

int masw_poll(masw_ctx* ctx, uint64_t ticket, double* C_t, int32_t* idx, int32_t* status, double* c_ref,
              masw_request_info* info) {
  if (!ctx) return fail(MASW_EINVAL, "ctx: null context");
  Server* s = ctx->server;
  if (!s) return fail(MASW_EBUSY, "server not running");
  std::unique_lock<std::mutex> lk(s->mu);
  return collect(s, lk, ticket, C_t, idx, status, c_ref, info);
}

int masw_wait(masw_ctx* ctx, uint64_t ticket, int64_t timeout_us, double* C_t, int32_t* idx, int32_t* status,
              double* c_ref, masw_request_info* info) {
  if (!ctx) return fail(MASW_EINVAL, "ctx: null context");
  Server* s = ctx->server;
  if (!s) return fail(MASW_EBUSY, "server not running");
  std::unique_lock<std::mutex> lk(s->mu);
  auto ready = [&] {
    auto it = s->requests.find(ticket);
    return s->failed || it == s->requests.end() || it->second->done;
  };
  if (timeout_us < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
    return fail(MASW_ETIMEOUT, "request not finished within the timeout");
  }
  return collect(s, lk, ticket, C_t, idx, status, c_ref, info);
}

int masw_server_get_stats(masw_ctx* ctx, masw_server_stats* out) {
  if (!ctx || !out) return fail(MASW_EINVAL, "null argument");
  Server* s = ctx->server;
  if (!s) return fail(MASW_EBUSY, "server not running");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  return MASW_OK;
}

}  // extern "C"
