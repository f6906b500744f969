/*
 * masw.h -- C ABI of the MI355X dispersion-curve library.
 *
 * The library computes theoretical Rayleigh-wave dispersion curves of layered
 * elastic models: for every wavelength lambda (k = 2 pi / lambda) and every
 * test phase velocity c of an ascending grid, the sign of the determinant of
 * the layered stiffness matrix, and the first grid velocity at which that sign
 * changes (the paper's Algorithm 1, Section 2.1).  It adds an FP64 refinement
 * of the root inside the bracketing grid interval.
 *
 * Units: lambda and h in m, alpha (P velocity), beta (S velocity) and c in
 * m/s, rho in kg/m^3.
 *
 * Pointers.  Array arguments are HOST pointers unless `flags` contains
 * MASW_DEVICE_PTRS; then every array argument (inputs and outputs) is a HIP
 * device pointer, read and written in stream order on `stream`.  The caller
 * owns every buffer.  The library copies host inputs into its own device
 * memory before it returns and keeps no caller pointer after the call,
 * except that with MASW_DEVICE_PTRS the kernels may still run on `stream`
 * after the call returns (synchronise `stream` before reading outputs or
 * reusing inputs).  `stream` is a hipStream_t; NULL is the device's default
 * (null) stream, as everywhere in HIP, so device-pointer work issued on the
 * default stream by the caller is ordered with the library's.
 *
 * Errors.  Every function returning int returns MASW_OK (0) or a negative
 * MASW_E* code; nothing aborts or throws across the ABI.  Argument checks
 * (sizes, finiteness, ordering, physical bounds) run on the host before any
 * HIP call for host pointers.  With MASW_DEVICE_PTRS the values are checked
 * on the device and a failing model reports MASW_STATUS_INVALID in the
 * per-wavelength status.  masw_last_error() describes the last failure of the
 * calling thread.
 *
 * Threads.  Calls on one context are serialised by an internal mutex, so a
 * context may be shared by threads.  While a server runs, masw_submit,
 * masw_poll, masw_wait and masw_server_get_stats may be called from any
 * number of threads at once (a waiting thread does not block submitters).
 * masw_server_stop and masw_destroy must not overlap any other call on
 * the context.
 */
#ifndef MASW_H
#define MASW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes -- */
enum {
    MASW_OK = 0,
    MASW_EINVAL = -1,   /* an argument failed validation                      */
    MASW_ENOMEM = -2,   /* the request does not fit the context's HBM budget  */
    MASW_EBUSY = -3,    /* serving: result not ready / no free slot           */
    MASW_EDEVICE = -4,  /* a HIP call failed or no device is present          */
    MASW_ETIMEOUT = -5, /* serving: wait timed out                            */
    MASW_ENOENT = -6    /* serving: unknown ticket                            */
};

/* Per-wavelength status (low byte) and flag bits. */
enum {
    MASW_STATUS_FOUND = 0,      /* a sign change was found at idx              */
    MASW_STATUS_NOT_FOUND = 1,  /* no sign change in c_test: idx = -1, C_t NaN */
    MASW_STATUS_INVALID = 2,    /* the model or grid failed device validation  */
    MASW_STATUS_NAN = 3,        /* a determinant evaluated to NaN at idx       */
    MASW_FLAG_POLE = 0x100,     /* some layer denominator D_j changes sign
                                   between c_test[idx-1] and c_test[idx]: the
                                   change is a pole of det K, not a zero      */
    MASW_FLAG_NOISE = 0x200     /* with MASW_CHECK_NOISE: c_test[idx-1] or
                                   c_test[idx] lies in the FP64 noise band,
                                   cond_2(K) 2(N+1) 2^-53 >= 1e-2, so the pick
                                   may differ from an exact computation's.
                                   Tested only below the half-space's S
                                   velocity, where K is real symmetric and
                                   cond_2 follows from eigenvalue counts
                                   (Sylvester's law of inertia on the block
                                   elimination)                               */
};

/* Arithmetic of the search.
 * MASW_PREC_FP64:  every determinant sign in FP64.
 * MASW_PREC_SPLIT: the c-grid sweep in FP32 below the half-space's S
 *                  velocity; each FP32 candidate is re-checked in FP64 over a
 *                  window of grid points around it, the stretch FP32 passed
 *                  over is certified by FP64 inertia counts (equal
 *                  Wittrick-Williams counts at its ends prove no zero and no
 *                  pole of det K in it, otherwise it is walked in FP64), the
 *                  grid at or above the half-space's S velocity is walked in
 *                  FP64, and the refinement is FP64.  So idx is Algorithm 1's
 *                  FP64 pick, as with MASW_PREC_FP64, outside the FP64 noise
 *                  band.  A curve or batch call whose grid has fewer than
 *                  MASW_SPLIT_MIN_GRID points runs as MASW_PREC_FP64 (two
 *                  rounds of a small launch's sweep cover such a grid, so
 *                  the FP32 sweep saves none of them, and its FP64 re-check
 *                  window would add one); masw_stats.split_as_fp64 says so. */
enum { MASW_PREC_FP64 = 0, MASW_PREC_SPLIT = 1 };
#define MASW_SPLIT_MIN_GRID 1025
/* A plain integer, not the enum type, so that any value a caller passes is
 * well defined on both sides of the ABI; others are rejected (MASW_EINVAL). */
typedef int32_t masw_precision;

/* Flags. */
#define MASW_DEVICE_PTRS 0x1u  /* array arguments are device pointers        */
#define MASW_NO_REFINE   0x2u  /* skip the root refinement (c_ref = NaN)     */
#define MASW_CHECK_NOISE 0x4u  /* masw_dispersion_curve / _batch: test each
                                  pick's bracket for the FP64 noise band and
                                  set MASW_FLAG_NOISE (an extra kernel after
                                  the sweep; not in its timing)               */
#define MASW_SEARCH_INERTIA 0x8u /* masw_dispersion_curve / _batch, FP64
                                  only: find each pick by a search on
                                  inertia counts instead of walking the grid
                                  (Algorithm 1's early-exit scan).  Below the
                                  half-space's S velocity K is real symmetric
                                  and sign(det K) = (-1)^(negative eigenvalues);
                                  that count plus twice the number of
                                  fixed-face layer modes below c does not
                                  decrease along c (Wittrick-Williams), so the
                                  grid points whose counts prove the sign
                                  constant are skipped.  Same outputs as the
                                  walk outside the FP64 noise band; grid points
                                  at or above that velocity are walked.
                                  MASW_PREC_SPLIT with it: MASW_EINVAL        */

/* Limits. */
#define MASW_MAX_LAYERS 1024   /* finite layers per model                    */

typedef struct masw_ctx masw_ctx;

/* One model: n_layers finite layers over a half-space (n_layers = 0 is a
 * homogeneous half-space).  h has n_layers entries (> 0); alpha, beta, rho
 * have n_layers + 1 entries, the last for the half-space, with
 * alpha > beta > 0 and rho > 0, all finite. */
typedef struct {
    int32_t n_layers;
    const double *h;
    const double *alpha;
    const double *beta;
    const double *rho;
} masw_model;

/* A batch of models of uneven sizes, flattened.
 * Model m has N_m = layer_off[m+1] - layer_off[m] layers; its h entries are
 * h[layer_off[m] .. layer_off[m+1]-1] and its alpha/beta/rho entries are at
 * [layer_off[m] + m .. layer_off[m+1] + m] (N_m + 1 values, half-space last).
 * Its wavelengths are lambda[lambda_off[m] .. lambda_off[m+1]-1].  Outputs
 * are indexed by the flattened wavelength index.  layer_off and lambda_off
 * are non-decreasing with layer_off[0] = lambda_off[0] = 0. */
typedef struct {
    int32_t n_models;
    const int32_t *layer_off;   /* [n_models + 1] */
    const double *h;            /* [layer_off[n_models]] */
    const double *alpha;        /* [layer_off[n_models] + n_models] */
    const double *beta;         /* [layer_off[n_models] + n_models] */
    const double *rho;          /* [layer_off[n_models] + n_models] */
    const int32_t *lambda_off;  /* [n_models + 1] */
    const double *lambda;       /* [lambda_off[n_models]] */
} masw_batch;

/* Per-wavelength results, each an array of the number of wavelengths.
 * c_t = c_test[idx] (the upper end of the bracketing grid interval, as in
 * Algorithm 1), idx = grid index (-1 if none), status = MASW_STATUS_* |
 * flags, c_ref = FP64 root inside [c_test[idx-1], c_test[idx]] to a bracket
 * width of refine_rel_tol c_test[idx] (masw_opts; 1e-9 by default), or NaN if
 * not found or MASW_NO_REFINE.  c_ref may be NULL. */
typedef struct {
    double *c_t;
    int32_t *idx;
    int32_t *status;
    double *c_ref;
} masw_outputs;

/* Work counters of the last completed call on a context. */
typedef struct {
    uint64_t useful_evals;  /* sum over wavelengths of idx + 1 (n_c if none)    */
    uint64_t sweep_evals;   /* determinant signs evaluated by the grid sweep   */
    uint64_t check_evals;   /* FP64 re-check evaluations (split precision)     */
    uint64_t refine_evals;  /* FP64 refinement evaluations                     */
    uint64_t n_lambda;      /* wavelengths processed                           */
    int32_t waves_per_item; /* wavefronts that cooperated on one wavelength    */
    int32_t workgroups;     /* persistent workgroups launched                  */
    float sweep_ms;         /* device time of the sweep/re-check/refine kernel,
                               from the GPU's real-time counter (masw_timing)  */
    float total_ms;         /* device time of staging + ordering + sweep       */
    int32_t shared_items;   /* wavelengths run as shared sweeps, which workgroups
                               that run out of queued work join                */
    uint32_t shared_stalls; /* shared sweeps abandoned after waiting too long
                               for a joined round (always 0 unless the device
                               misbehaves; such wavelengths get
                               MASW_STATUS_INVALID)                            */
    uint64_t helper_evals;  /* of sweep_evals, those done by joining workgroups */
    /* After masw_classify_picks (the fields above are then 0, except
     * sweep_ms = total_ms = the classification kernel's device time): */
    uint64_t classify_evals;  /* secular-function evaluations (one per lane and
                                 multisection round, 64 per round)            */
    uint64_t classify_layers; /* layers crossed by those evaluations           */
    uint64_t classify_steps;  /* propagator steps taken by those evaluations   */
    /* With MASW_SEARCH_INERTIA (sweep_evals then counts the grid points
     * walked, check_evals the determinant signs at the changes of the count): */
    uint64_t inertia_evals;   /* inertia counts evaluated                      */
    uint64_t inertia_entries; /* layer and sublayer element matrices formed    */
    uint64_t inertia_pivots;  /* 2x2 block pivots eliminated                   */
    int32_t fused_staging;    /* 1: a small single-curve launch that staged its
                                 model, grid and wavelengths inside the sweep
                                 kernel (one launch; sweep_ms = total_ms)      */
    int32_t split_as_fp64;    /* 1: a MASW_PREC_SPLIT call on a grid of at most
                                 MASW_SPLIT_MIN_GRID - 1 points, run as the
                                 FP64 walk (see MASW_PREC_SPLIT)              */
} masw_stats;

/* Options of a context.  A zero field keeps its default, so a
 * zero-initialised struct (or NULL) gives the defaults. */
typedef struct {
    double refine_rel_tol;    /* c_ref bracket width / c_test[idx], in
                                 [1e-15, 1e-3] (0 = 1e-9)                      */
    double noise_threshold;   /* MASW_CHECK_NOISE: a grid point is in the band
                                 when cond_2(K) 2(N+1) 2^-53 >= this, in
                                 (0, 1] (0 = 1e-2)                            */
    int32_t waves_per_item;   /* wavefronts per wavelength in a sweep launch:
                                 1, 2, 4, 8 or 16 (0 = chosen per launch)     */
    int32_t shared_window;    /* rounds a workgroup with an empty queue may
                                 evaluate ahead in a shared sweep, 1..1024
                                 (0 = 8; -1 = no shared sweeps)               */
    int32_t first_item_priority; /* 0 = each workgroup's first (deepest) item
                                 runs at wave issue priority 2; -1 = off      */
    int32_t timing_events;    /* 1 = time each call with HIP events around its
                                 kernels (the launches' exact bounds, as a
                                 profiler sees them; each event costs some
                                 5 us of host time); 0 = from the GPU's
                                 real-time counter (masw_get_timing)          */
} masw_opts;

/* Set the options of ctx (NULL = defaults).  They apply to later calls; a
 * server takes refine_rel_tol when it starts.  MASW_EINVAL on a value out of
 * range (nothing is changed then). */
int masw_set_opts(masw_ctx *ctx, const masw_opts *opts);

/* The options in effect, with defaults filled in. */
int masw_get_opts(masw_ctx *ctx, masw_opts *out);

/* Create a context on HIP device `device` that may hold up to
 * `hbm_budget_bytes` of device memory (0 = 256 MiB).  The budget is
 * allocated once, here.  Returns MASW_EDEVICE if no such device exists. */
int masw_create(int device, size_t hbm_budget_bytes, masw_ctx **out);

/* Wait for outstanding work, free the context's memory and streams.  NULL is
 * ignored. */
void masw_destroy(masw_ctx *ctx);

/* Dispersion curve of one model (Algorithm 1 plus refinement).
 * c_test: [n_c], strictly increasing, finite, > 0, n_c >= 2.
 * lambda: [n_lambda], finite, > 0 (n_lambda = 0 does nothing).
 * Outputs C_t, idx, status, c_ref (c_ref may be NULL): [n_lambda].
 * Synchronous for host pointers; stream-ordered with MASW_DEVICE_PTRS. */
int masw_dispersion_curve(masw_ctx *ctx, const double *c_test, int32_t n_c,
                          const double *lambda, int32_t n_lambda,
                          const masw_model *model, masw_precision prec,
                          uint32_t flags, void *stream,
                          double *C_t, int32_t *idx, int32_t *status,
                          double *c_ref);

/* masw_dispersion_curve without allocation, for callers that cannot call
 * hipMalloc: code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation.  Same arguments, meaning and outputs as
 * masw_dispersion_curve, with every array a device pointer in stream order
 * (MASW_DEVICE_PTRS is required; MASW_EINVAL otherwise).  The call's device
 * workspace (layer records, the FP32 grid, k and the work order per
 * wavelength, counters, shared-sweep state) lives in a static device array
 * of the library, MASW_NOALLOC_SCRATCH_BYTES on each device that loads the
 * library (held until the process ends), instead of the context's arena; the
 * call allocates nothing, synchronises nothing and records no events.  The
 * context supplies its device and options only; masw_create set the array up
 * on that device.
 * Limit: a request whose workspace exceeds MASW_NOALLOC_SCRATCH_BYTES (about
 * 4 B per grid point, 17 B per wavelength and 96 B per layer, plus, when
 * they fit, 8 B per round of 64 G grid points per wavelength for shared
 * sweeps) fails with MASW_ENOMEM before anything is queued.
 * Sharing: every call on one device uses that device's one array, which
 * keeps the last call's contents (the call's first kernel clears what must
 * start at zero).  Calls whose work overlaps on the device (other streams,
 * threads or contexts) race on it: the caller orders them.  These calls are
 * not counted by masw_get_stats or masw_get_timing. */
#define MASW_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int masw_dispersion_curve_noalloc(masw_ctx *ctx, const double *c_test, int32_t n_c,
                                  const double *lambda, int32_t n_lambda,
                                  const masw_model *model, masw_precision prec,
                                  uint32_t flags, void *stream, double *C_t,
                                  int32_t *idx, int32_t *status, double *c_ref);

/* Dispersion curves of a batch of models sharing one c grid, in one
 * persistent launch whose work queue hands out (model, wavelength) items
 * longest-expected-first.  Same rules as masw_dispersion_curve. */
int masw_dispersion_batch(masw_ctx *ctx, const double *c_test, int32_t n_c,
                          const masw_batch *batch, masw_precision prec,
                          uint32_t flags, void *stream,
                          const masw_outputs *out);

/* One step of inversion chains (Algorithm 2 over a batch): the batch's
 * curves, as masw_dispersion_batch, and the misfit of every model,
 * misfit[m] = mean over its wavelengths i of |C_t,i - C_e,i| / C_e,i, as
 * masw_misfit computes it (bit for bit), in the same persistent launch: the
 * workgroup that finishes a model's last wavelength reduces the model's
 * misfit.  C_e: [total wavelengths], laid out as batch->lambda, finite and
 * > 0 (checked on the host for host pointers); misfit: [n_models] (NaN for a
 * model without wavelengths, or with a wavelength without a pick).  With
 * MASW_SEARCH_INERTIA the misfit is a second launch after the search.  Same
 * rules as masw_dispersion_batch otherwise. */
int masw_dispersion_batch_misfit(masw_ctx *ctx, const double *c_test, int32_t n_c,
                                 const masw_batch *batch, masw_precision prec,
                                 uint32_t flags, void *stream, const masw_outputs *out,
                                 const double *C_e, double *misfit);

/* Full sign map of one model: for every wavelength w and grid point i, with
 * no early exit, sigma[w * n_c + i] = sign(Re det K) in {-1, 0, +1} (2 if the
 * determinant is NaN) and, if log_abs_det is not NULL,
 * log_abs_det[w * n_c + i] = natural log of |det K| (the unscaled matrix).
 * This is the GPU counterpart of evaluating every stiffness matrix of the
 * (wavelength, velocity) grid (Section 2.3).  MASW_PREC_FP64 or
 * MASW_PREC_SPLIT (the latter evaluates in FP32). */
int masw_sign_map(masw_ctx *ctx, const double *c_test, int32_t n_c,
                  const double *lambda, int32_t n_lambda,
                  const masw_model *model, masw_precision prec,
                  uint32_t flags, void *stream,
                  int8_t *sigma, double *log_abs_det);

/* ------------------------------------------------------------- serving -- */
/* A serving loop takes requests (one model each, as masw_dispersion_curve)
 * as they arrive and batches them continuously: a driver thread admits
 * queued requests while a slot is free and their device memory fits the
 * serving pool (HBM-budget admission), and every tick replays one captured
 * hipGraph that advances every unfinished wavelength of every resident
 * request by a bounded number of sweep rounds, keeping each wavelength's
 * search state in HBM between ticks.  A request admitted while others are
 * in flight joins the next tick; its results are the same as from
 * masw_dispersion_curve, bit for bit.  Inputs are host pointers, copied at
 * submit; results are delivered by masw_poll / masw_wait. */
typedef struct {
    int32_t max_layers;      /* per request, <= MASW_MAX_LAYERS (0 = 64)          */
    int32_t max_lambda;      /* wavelengths per request (0 = 512)                 */
    int32_t max_grid;        /* c values per request (0 = 32768)                  */
    int32_t rounds_per_tick; /* sweep rounds per wavelength per tick (0 = 16)     */
    size_t pool_bytes;       /* device memory for resident requests, taken from
                                the context's budget (0 = half of it)            */
    int64_t tick_timeout_us; /* watchdog: a tick (admission + graph replay) that
                                runs longer fails the server: pending and later
                                calls return MASW_EDEVICE, and the server must be
                                stopped and started again (0 = 10 s)             */
    int32_t search_inertia;  /* 1: FP64 requests find their picks with the
                                inertia-count search (as MASW_SEARCH_INERTIA),
                                each within one tick: the tick's wavefronts
                                sample det K's sign, one wavefront finishes;
                                where the search falls back to walking (grid
                                points at or above the half-space's S
                                velocity), the walk proceeds rounds_per_tick
                                rounds per tick like a walking request's;
                                0: they walk.  Split requests always walk.
                                Other values: MASW_EINVAL                       */
    int32_t reserved;        /* must be 0                                         */
} masw_server_opts;

/* Timing of one request (CLOCK_MONOTONIC ns) and the ticks it took part in. */
typedef struct {
    uint64_t submit_ns;
    uint64_t admit_ns;
    uint64_t done_ns;
    uint32_t ticks;
    uint32_t reserved;
} masw_request_info;

typedef struct {
    uint64_t ticks;           /* graph replays                                  */
    uint64_t submitted;
    uint64_t completed;
    uint64_t admit_waits;     /* ticks in which a queued request did not fit    */
    uint32_t max_resident;    /* most requests resident at once                 */
    uint32_t resident;        /* requests resident now                          */
    uint64_t pool_bytes;
    double busy_ms;           /* host time spent in ticks (launch to completion) */
} masw_server_stats;

/* Start the serving loop on ctx (opts may be NULL).  MASW_EBUSY if it is
 * already running, MASW_ENOMEM if the pool does not fit the budget.  While
 * it runs, synchronous calls on ctx use the rest of the budget. */
int masw_server_start(masw_ctx *ctx, const masw_server_opts *opts);

/* Finish every submitted request, then stop the loop and release the pool.
 * Results not yet collected are discarded.  No other call on ctx may be in
 * progress (in particular no masw_wait). */
int masw_server_stop(masw_ctx *ctx);

/* Queue one request.  Arguments as masw_dispersion_curve with host pointers;
 * they are checked and copied before the call returns.  flags: 0, or any of
 * MASW_CHECK_NOISE (each pick's bracket is tested for the FP64 noise band
 * when the pick is made, and MASW_FLAG_NOISE set in its status, as for the
 * synchronous calls) and MASW_NO_REFINE (c_ref = NaN); other bits are
 * MASW_EINVAL.  MASW_EINVAL on a bad argument or one above the server's
 * limits, MASW_ENOMEM if the request could never fit the pool, MASW_EBUSY if
 * the loop is not running.  *ticket identifies the request. */
int masw_submit(masw_ctx *ctx, const double *c_test, int32_t n_c, const double *lambda,
                int32_t n_lambda, const masw_model *model, masw_precision prec,
                uint32_t flags, uint64_t *ticket);

/* If the request is finished, copy its results (arrays of its n_lambda;
 * c_ref and info may be NULL) and forget the ticket: MASW_OK.  MASW_EBUSY if
 * it is not finished, MASW_ENOENT if the ticket is unknown or was collected. */
int masw_poll(masw_ctx *ctx, uint64_t ticket, double *C_t, int32_t *idx, int32_t *status,
              double *c_ref, masw_request_info *info);

/* As masw_poll, waiting up to timeout_us microseconds (< 0: no limit);
 * MASW_ETIMEOUT if the request is still not finished. */
int masw_wait(masw_ctx *ctx, uint64_t ticket, int64_t timeout_us, double *C_t, int32_t *idx,
              int32_t *status, double *c_ref, masw_request_info *info);

int masw_server_get_stats(masw_ctx *ctx, masw_server_stats *out);

/* Misfit of each model's theoretical curve against an experimental curve
 * (Algorithm 2, Section 2.1): for model m with l_m wavelengths,
 *     misfit[m] = (1/l_m) * sum_i |C_t[i] - C_e[i]| / C_e[i]
 * over its wavelengths i (lambda_off as in masw_batch).  A NaN C_t (no sign
 * change found) makes that model's misfit NaN; a model with no wavelengths
 * gets NaN.  C_t, C_e: [lambda_off[n_models]]; C_e finite and > 0;
 * misfit: [n_models].  The sum is a fixed-order tree, so the result does
 * not depend on the launch. */
int masw_misfit(masw_ctx *ctx, int32_t n_models, const int32_t *lambda_off,
                const double *C_t, const double *C_e, uint32_t flags, void *stream,
                double *misfit);

/* ------------------------------------------------ zero/pole classification --
 * Algorithm 1 (Section 2.1) reports the first grid interval where
 * sign(det K) changes.  det K of the stiffness formulation is the dispersion
 * function divided by the layer denominators D_j, so a change can be a zero
 * (a surface-wave mode) or a pole (a resonance of one layer with both faces
 * fixed; MASW_FLAG_POLE marks it from the D_j).  masw_classify_picks decides
 * which with an independent formulation that has no denominators: the
 * Haskell-Thomson propagator of the P-SV equations of motion.  The
 * half-space's two solutions that decay with depth are carried up to the
 * surface, and F(c) = the determinant of their two tractions there vanishes
 * exactly at the modes.  Each layer is crossed in steps of at most one unit
 * of k dz max(|r|, |s|) (r^2 = 1 - c^2/alpha^2, s^2 = 1 - c^2/beta^2), with
 * the pair re-orthonormalised after each step; that divides F by a positive
 * factor, so its sign and zeros are unchanged. */
enum {
    MASW_PICK_MODE = 0,       /* F changes sign between c_test[idx-1] and
                                 c_test[idx] (a zero counts as a sign)        */
    MASW_PICK_POLE = 1,       /* F has the same sign at both ends: no mode in
                                 the bracket, so a sign change of det K there
                                 is a pole                                    */
    MASW_PICK_LEAKY = 2,      /* c_test[idx] >= the half-space's beta: F is
                                 not real there; not classified               */
    MASW_PICK_NONE = 3,       /* idx < 1 or idx >= n_c: no bracket (takes
                                 precedence over the other classes)           */
    MASW_PICK_UNRESOLVED = 4, /* a layer needs more than 65536 steps
                                 (k h max(|r|, |s|) > 65536), or F is not
                                 finite                                       */
    MASW_PICK_INVALID = 5     /* the model, wavelength or bracket failed
                                 device validation                            */
};

/* Classify the sign change at grid index idx[w] of every wavelength w of a
 * batch (layout as masw_dispersion_batch; idx is typically that call's idx
 * output, or any index whose bracket holds a sign change of a sign map).
 * pick_class[w] = MASW_PICK_*.  c_sec[w] = for MASW_PICK_MODE, the root of F
 * in the bracket (multisection to a bracket no wider than
 * 1e-12 c_test[idx[w]], midpoint), else NaN; c_sec may be NULL.
 * c_test: [n_c] as masw_dispersion_curve.  idx, pick_class: int32
 * [lambda_off[n_models]]; c_sec: double [lambda_off[n_models]].  Host
 * pointers are validated (models, wavelengths, grid) and the call is
 * synchronous; with MASW_DEVICE_PTRS every array is a device pointer, the
 * call is stream-ordered after reading the two offset arrays, and invalid
 * values give MASW_PICK_INVALID.  Only MASW_DEVICE_PTRS is accepted in
 * flags. */
int masw_classify_picks(masw_ctx *ctx, const double *c_test, int32_t n_c,
                        const masw_batch *batch, const int32_t *idx,
                        uint32_t flags, void *stream,
                        int32_t *pick_class, double *c_sec);

/* Counters of the last completed call on ctx (for MASW_DEVICE_PTRS calls,
 * after the stream has been synchronised; this function synchronises). */
int masw_get_stats(masw_ctx *ctx, masw_stats *out);

/* Device time of the masw_dispersion_curve / masw_dispersion_batch calls
 * made on ctx since the timing was last reset (calls with n_lambda > 0), from
 * the GPU's constant-rate real-time counter, which each call's kernels read
 * at the start of its first kernel, the start of its sweep and the end of
 * the sweep's last workgroup (no host event and no synchronisation between
 * calls is needed to time them; the dispatch latency before a kernel's
 * first workgroup starts is not counted).  Waits for those calls to finish.  With reset != 0 the sums start
 * again from zero after being returned.  Calls on other contexts, sign maps
 * and served requests are not counted. */
typedef struct {
    uint64_t launches;    /* calls timed                                        */
    double sweep_ms_sum;  /* sum of their sweep-kernel durations (ms)           */
    double total_ms_sum;  /* sum of their staging + ordering + sweep durations  */
    float sweep_ms_min;   /* shortest and longest sweep-kernel duration (ms);   */
    float sweep_ms_max;   /* 0 when launches == 0                               */
} masw_timing;
int masw_get_timing(masw_ctx *ctx, int reset, masw_timing *out);

/* Static text for an error code. */
const char *masw_strerror(int code);

/* Description of the calling thread's last error ("" if none). */
const char *masw_last_error(void);

/* Library version string. */
const char *masw_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MASW_H */
