#!/usr/bin/env python3
"""Throughput benchmark of the dispersion-curve hot path on one MI355X.

A step is one whole dispersion-curve job through the C ABI: staging and
precompute, work ordering, the early-exit sweep with its FP64 refinement, and
the results in HBM.  Inputs are resident in HBM before timing starts.

Default workload: the batch of 4096 seeded models of uneven sizes (N 3-30,
50-500 wavelengths log-spaced 1-80 m each, about 1.1 M wavelengths; c 50-1000
m/s at 0.05 m/s, 19,001 values; about 15% with a low-velocity layer), one
persistent launch per job.  Headline: the plain FP64 path.  The split path
(FP32 sweep + FP64 re-check and inertia-count certificate + FP64 refinement)
and the FP64 inertia-count search are timed on the same inputs and reported
beside it.  Legs of the default run:
  * fine_scale: the 20-layer model, 1000 wavelengths log-spaced 1-100 m,
    c 50-1200 m/s at 0.01 m/s (115,001 values), the same three paths;
  * serving: a short replay of the 2000 req/s trace, p50/p99 latency of the
    split and plain-FP64 servers;
  * two_layer_vs_oracle (with the CPU leg): the two-layer case's picks and
    refined roots against the oracle, split and FP64;
  * cpu_baseline: the oracle on a bounded sample of the batch.

Headline unit: useful determinant evaluations per second, the sum over
wavelengths of (pick index + 1), the work Algorithm 1 needs whatever the
implementation.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
                       [--workload batch|fine_scale|two_layer|serving|uniform|chains|classify]
                       [--no-cpu-baseline] [--no-legs]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "det evals/s + dispersion curves/s vs plain FP64 at 1e-6 rel; p50/p99 latency"
FP64_PEAK_TFLOPS = 78.6    # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
FP32_PEAK_TFLOPS = 157.3   # published, packed FP32 (packed math is not used here)


def flops_per_eval(n_layers: float) -> float:
    """Algorithmic FP operations of one determinant sign (add/sub/mul = 1,
    a fused multiply-add = 2, each sqrt/division/expm1/sincos = 1):
    per layer 101 (element entries 67 incl. k h, block elimination 34), plus 48
    for the half-space block and the final complex 2x2 determinant."""
    return 101.0 * n_layers + 48.0


def inertia_flops(evals: int, entries: int, pivots: int) -> float:
    """Algorithmic FP operations of the inertia counts of a launch, from its
    work counters (the rules of flops_per_eval): 67 per element matrix formed
    (a layer's or a sublayer's), 34 per 2x2 block pivot eliminated, and 48 for
    the half-space block of each count in place of its pivot."""
    return 67.0 * entries + 34.0 * (pivots - evals) + 48.0 * evals


def classify_flops(evals: int, layers: int, steps: int) -> float:
    """Algorithmic FP operations of a zero/pole classification launch, from its
    work counters (same counting rules as flops_per_eval, a shared
    subexpression once, a reciprocal square root 1): per secular-function
    evaluation 61 (the sample point 4, c^2, mu_ref and its reciprocal 4, the
    half-space pair 11, its orthonormalisation 39, the traction minor 3); per
    layer crossed 238 (M, mu, their reciprocals, rho c^2, r^2, s^2 and the
    step count and length 15, the system matrix 13, the step propagator's
    series and coefficients 140, the 2x2 block products XY, YX, XYX, YXY 36,
    its assembly 34); per propagator step 95 (the 4x4 by 4x2 product 56, the
    orthonormalisation 39)."""
    return 61.0 * evals + 238.0 * layers + 95.0 * steps


# HBM bytes per launch of the dominant kernel, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs each scaled by the same counter's reading for a plain copy of
# known size (FETCH x 2.000, WRITE x 1.000); see profiles/.  Keyed by the hash
# of the kernel sources the counters were taken on (KERNEL_SOURCES for the
# sweep, INERTIA_SOURCES for the inertia search, CLASSIFY_SOURCES for the
# classification), the workload and the
# launch, so a changed kernel reports null until it is measured again.
MEASURED_TRAFFIC = {
    ("4e502a09f3d5959a", "fine_scale_N20_1000lam_115001c", "sweep_kernel<FP64,G=4>"):
        8170.61 * 1024 * 2.000 + 4899.36 * 1024 * 1.000,
    ("4e502a09f3d5959a", "batch_4096models_19001c", "sweep_kernel<FP64,G=1>"):
        267238.81 * 1024 * 2.000 + 147567.77 * 1024 * 1.000,
    ("31a58e2a8353c3d3", "fine_scale_N20_1000lam_115001c", "inertia_lone_kernel"):
        902.00 * 1024 * 2.000 + 50.80 * 1024 * 1.000,
    ("31a58e2a8353c3d3", "batch_4096models_19001c", "inertia_kernel"):
        55078.56 * 1024 * 2.000 + 1205151.92 * 1024 * 1.000,
    ("ef681d38c885d05d", "classify_batch_4096models_19001c", "classify_kernel"):
        14642.625 * 1024 * 2.000 + 21872.34 * 1024 * 1.000,
}

# (timed steps, warm-up steps) per workload when the command line gives none.
DEFAULT_STEPS = {"fine_scale": (200, 50), "two_layer": (200, 50), "batch": (5, 1), "uniform": (20, 3),
                 "chains": (100, 3), "classify": (5, 2)}

KERNEL_SOURCES = ["masw_internal.hpp", "masw_math.hpp", "masw_special.hpp", "masw_pick.hpp", "masw_sweep.hpp",
                  "masw_kernels.hip", "masw_sweep_split.hip"]
CLASSIFY_SOURCES = ["masw_classify.hip"]
INERTIA_SOURCES = ["masw_internal.hpp", "masw_math.hpp", "masw_special.hpp", "masw_pick.hpp", "masw_inertia.hpp",
                   "masw_inertia_kernel.hpp", "masw_inertia.hip", "masw_inertia_lone.hip"]


def kernel_source_hash(files=KERNEL_SOURCES) -> str:
    """sha256[:16] of the sources' code: comments, trailing blanks and empty
    lines removed, so that an edit of a comment keeps a measurement valid."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2003_02256_amd", "csrc", f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        lines = (re.sub(r"//.*$", "", line).rstrip() for line in text.splitlines())
        h.update("\n".join(line for line in lines if line).encode())
    return h.hexdigest()[:16]


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- workloads --
def make_workload(name: str):
    import workloads as WL
    if name == "fine_scale":
        return WL.fine_scale_case()
    if name == "two_layer":
        return WL.two_layer_case()
    if name == "batch":
        return WL.batch_case()
    raise SystemExit(f"unknown workload {name}")


class DeviceJob:
    """Inputs and outputs of one workload resident on the GPU."""

    def __init__(self, wl, torch, dev):
        import paper_2003_02256_amd as M
        self.M, self.torch, self.wl = M, torch, wl
        arrs = M.flatten_models(wl.models, wl.lambdas)
        self.arrs = [torch.as_tensor(a, device=dev) for a in arrs]
        self.c = torch.as_tensor(wl.c_test, device=dev)
        self.W = int(arrs[-1].shape[0])
        self.single = len(wl.models) == 1
        self.prepared = {}
        f64, i32 = torch.float64, torch.int32
        self.out = {p: (torch.empty(self.W, dtype=f64, device=dev), torch.empty(self.W, dtype=i32, device=dev),
                        torch.empty(self.W, dtype=i32, device=dev), torch.empty(self.W, dtype=f64, device=dev))
                    for p in (M.MASW_PREC_FP64, M.MASW_PREC_SPLIT, "inertia")}
        self.n_layers = [m.n_layers for m in wl.models]
        self.lam_model = np.repeat(np.arange(len(wl.models)), [len(l) for l in wl.lambdas])

    def run(self, ctx, prec):
        """prec: a precision, or "inertia" for the FP64 inertia-count search.
        A single curve goes through a PreparedCurve (arguments marshalled
        once), so that a small job's time is not the binding's."""
        M, a = self.M, self.arrs
        flags = M.MASW_SEARCH_INERTIA if prec == "inertia" else 0
        p = M.MASW_PREC_FP64 if prec == "inertia" else prec
        if self.single:
            key = (ctx.value, prec)
            if key not in self.prepared:
                self.prepared[key] = M.PreparedCurve(ctx, self.c, a[6], a[1], a[2], a[3], a[4], p, flags, None,
                                                     *self.out[prec])
            self.prepared[key]()
        else:
            M.masw_dispersion_batch(ctx, self.c, *a, p, flags, None, *self.out[prec])

    def results(self, prec):
        return tuple(o.cpu().numpy() for o in self.out[prec])


def time_path(job, ctx, prec, steps, warmup):
    """Two timed passes of `steps` back-to-back jobs on the library's stream,
    after `warmup` jobs.  The first runs with the library's default timing
    (the GPU's real-time counter, read by the kernels; no host event): its
    wall time per job is the path's rate.  In the second the library records
    HIP events around every launch (masw_opts.timing_events), each costing
    some 5 us of host time: the mean sweep-kernel and job device times of
    exactly those launches give the roofline.  Returns (wall, sweep_ms,
    total_ms, stats of the last job, details)."""
    torch, M = job.torch, job.M
    opts = M.masw_get_opts(ctx)  # kept (environment tuning included); only the timing source changes

    def timed(events):
        M.masw_set_opts(ctx, **{**opts, "timing_events": events})
        M.masw_get_timing(ctx, reset=True)
        t0 = time.perf_counter()
        for _ in range(steps):
            job.run(ctx, prec)
        torch.cuda.synchronize()
        w = (time.perf_counter() - t0) / steps
        tm = M.masw_get_timing(ctx, reset=True)
        if tm["launches"] != steps:
            raise RuntimeError(f"timed {tm['launches']} launches, expected {steps}")
        return w, tm["sweep_ms_sum"] / steps, tm["total_ms_sum"] / steps

    for _ in range(warmup):
        job.run(ctx, prec)
    torch.cuda.synchronize()
    wall, sweep_c, total_c = timed(0)
    wall_e, sweep_e, total_e = timed(1)
    M.masw_set_opts(ctx, **opts)               # the options as they were
    stats = M.masw_get_stats(ctx)              # counters of the last job
    details = {"ms_per_step_with_events": wall_e * 1e3, "sweep_ms_counter": sweep_c,
               "device_ms_per_step_counter": total_c}
    return wall, sweep_e, total_e, stats, details


# ------------------------------------------------------------------ serving --
def serving_trace(rate: float, warm_s: float, dur_s: float, seed: int = 55):
    """Arrival times and request arrays of the serving workload
    (workloads.serving_trace): each arrival picks one of 64 chains uniformly
    and advances it one random-walk step."""
    import workloads as WL
    times, models = WL.serving_trace(rate, warm_s + dur_s, seed)
    reqs = [(np.ascontiguousarray(m.h), np.ascontiguousarray(m.alpha), np.ascontiguousarray(m.beta),
             np.ascontiguousarray(m.rho), lam, m.n_layers) for m, lam in models]
    return times, reqs


SPIN_NS = 1_000_000  # the load generator spins for the last 1 ms before each arrival


def run_serving(M, ctx, prec, times, reqs, c, warm_s: float, search_inertia: int = 0):
    """Replay the trace against the serving loop: a submitter thread at the
    arrival times; the results are collected after the last submission (the
    library stamps each completion itself, and a collector thread running
    meanwhile would compete with the submitter for the interpreter lock).
    Latency = the library's completion timestamp - the scheduled arrival
    (CLOCK_MONOTONIC); submit_lag_us says how late the submitter reached
    masw_submit.  search_inertia: FP64 requests take the inertia-count
    search."""
    import threading
    n = len(times)
    tickets = [None] * n
    sched = [0] * n
    M.masw_server_start(ctx, search_inertia=search_inertia)
    # the submitter must keep to the arrival times: no collector pauses
    # during the replay (latency counts from the scheduled arrival)
    import gc
    gc.collect()
    gc.disable()
    t0 = time.monotonic_ns() + 50_000_000

    lag = [0] * n

    def submitter():
        # sleep to within SPIN_NS of the arrival, then spin: time.sleep alone
        # wakes tens to hundreds of microseconds late (timer slack), which
        # would count as latency of the server
        for i in range(n):
            at = t0 + int(times[i] * 1e9)
            dt = (at - SPIN_NS - time.monotonic_ns()) / 1e9
            if dt > 0:
                time.sleep(dt)
            while time.monotonic_ns() < at:
                pass
            h, a, b, r, lam, _ = reqs[i]
            sched[i] = at
            lag[i] = time.monotonic_ns() - at
            tickets[i] = M.masw_submit(ctx, c, lam, h, a, b, r, prec)

    results = [None] * n
    th = threading.Thread(target=submitter)
    th.start()
    th.join()
    for i in range(n):
        W = len(reqs[i][4])
        out = (np.empty(W), np.empty(W, np.int32), np.empty(W, np.int32), np.empty(W))
        info = M.masw_wait(ctx, tickets[i], -1, *out)
        results[i] = (info, out[1])
    gc.enable()
    stats = M.masw_server_get_stats(ctx)
    M.masw_server_stop(ctx)
    meas = [i for i in range(n) if times[i] >= warm_s]
    lat = np.array([(results[i][0]["done_ns"] - sched[i]) / 1e6 for i in meas])
    sub_lag = np.array([lag[i] / 1e3 for i in meas])
    t_first = min(sched[i] for i in meas)
    t_last = max(results[i][0]["done_ns"] for i in meas)
    span = (t_last - t_first) / 1e9
    useful = sum(int(np.where(results[i][1] >= 0, results[i][1] + 1, c.shape[0]).sum()) for i in meas)
    return {"requests": len(meas), "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max()), "curves_per_s": len(meas) / span,
            "det_evals_per_s": useful / span, "useful_evals": useful, "span_s": span,
            "ticks": stats["ticks"], "max_resident": stats["max_resident"], "admit_waits": stats["admit_waits"],
            "busy_frac": stats["busy_ms"] / (span * 1e3),
            "submit_lag_us": {"p50": float(np.percentile(sub_lag, 50)), "p99": float(np.percentile(sub_lag, 99)),
                              "max": float(sub_lag.max())}}, [r[1] for r in results]


def serving_bench(M, torch, a):
    import workloads as WL
    c = WL.serving_grid()
    warm = 1.0
    times, reqs = serving_trace(2000.0, warm, a.serve_seconds)
    log(f"serving trace: {len(times)} requests over {warm + a.serve_seconds:.0f} s")
    ctx_obj = M.Context(0, 4 << 30)
    split, idx_s = run_serving(M, ctx_obj.ctx, M.MASW_PREC_SPLIT, times, reqs, c, warm)
    log(f"split: {split}")
    fp64, idx_d = run_serving(M, ctx_obj.ctx, M.MASW_PREC_FP64, times, reqs, c, warm)
    log(f"fp64: {fp64}")
    inertia, idx_i = run_serving(M, ctx_obj.ctx, M.MASW_PREC_FP64, times, reqs, c, warm, search_inertia=1)
    log(f"fp64 with the inertia search: {inertia}")
    mism = sum(int(np.sum(x != y)) for x, y in zip(idx_s, idx_d))
    mism_i = sum(int(np.sum(x != y)) for x, y in zip(idx_i, idx_d))
    ctx_obj.close()
    n_lam = int(np.mean([len(r[4]) for r in reqs]))
    res = {
        "metric": METRIC, "value": split["det_evals_per_s"], "unit": "det evals/s", "n_gpus": 1,
        "steps": split["requests"], "warmup": int(np.sum(times < warm)), "ms_per_step": split["mean_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 sweep + f64 re-check/refine", "data": "synthetic",
        "config": {"workload": "serving_64chains_2000rps", "arrival_rate": 2000, "seconds": a.serve_seconds,
                   "n_c": int(c.shape[0]), "wavelengths_mean": n_lam},
        "p50_ms": split["p50_ms"], "p99_ms": split["p99_ms"], "curves_per_s": split["curves_per_s"],
        "split": split, "fp64": fp64, "idx_mismatch_split_vs_fp64": mism,
        "fp64_inertia": inertia, "idx_mismatch_inertia_vs_fp64": mism_i,
    }
    print(json.dumps(res), flush=True)


# ------------------------------------------------------------------ uniform --
def uniform_bench(M, torch, a):
    """The paper's uniform curves (Section 3.3): lengths 50-500 of one repeated
    wavelength, picks at 72, 238, 256 m/s, 1000 test velocities, 14x14
    matrices (N = 6).  Early exit (this library's curve) against evaluating
    every (wavelength, velocity) matrix (the sign map, as the paper's GPU
    code did)."""
    import workloads as WL
    dev = torch.device("cuda:0")
    ctx_obj = M.Context(0, 1 << 30)
    ctx = ctx_obj.ctx
    rows, tot_useful, tot_s = [], 0, 0.0
    t64 = lambda x: torch.as_tensor(np.ascontiguousarray(x, np.float64), device=dev)
    for c_pick in (72.0, 238.0, 256.0):
        for L in (50, 100, 200, 300, 400, 500):
            wl = WL.uniform_case(c_pick, L)
            m, lam, c = wl.models[0], wl.lambdas[0], wl.c_test
            args = [t64(c), t64(lam), t64(m.h), t64(m.alpha), t64(m.beta), t64(m.rho)]
            out = (torch.empty(L, dtype=torch.float64, device=dev), torch.empty(L, dtype=torch.int32, device=dev),
                   torch.empty(L, dtype=torch.int32, device=dev), torch.empty(L, dtype=torch.float64, device=dev))
            out2 = tuple(torch.empty_like(o) for o in out)
            sig = torch.empty(L * c.shape[0], dtype=torch.int8, device=dev)

            curve = M.PreparedCurve(ctx, *args, M.MASW_PREC_FP64, 0, None, *out)
            pick_only = M.PreparedCurve(ctx, *args, M.MASW_PREC_FP64, M.MASW_NO_REFINE, None, *out2)
            smap = M.PreparedSignMap(ctx, *args, M.MASW_PREC_FP64, 0, None, sig)

            res = {}
            for name, fn in (("early_exit", curve), ("early_exit_no_refine", pick_only), ("sign_map", smap)):
                for _ in range(a.warmup):
                    fn()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(a.steps):
                    fn()
                torch.cuda.synchronize()
                res[name] = (time.perf_counter() - t0) / a.steps * 1e3
            idx = out[1].cpu().numpy()
            useful = int((idx + 1).sum())
            tot_useful += useful
            tot_s += res["early_exit"] * 1e-3
            rows.append({"c_pick": c_pick, "length": L, "idx": int(idx[0]), "early_exit_ms": res["early_exit"],
                         "early_exit_no_refine_ms": res["early_exit_no_refine"],
                         "sign_map_ms": res["sign_map"], "useful_evals": useful,
                         "grid_evals": L * int(c.shape[0])})
    ctx_obj.close()
    out = {"metric": METRIC, "value": tot_useful / tot_s, "unit": "det evals/s", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": tot_s * 1e3 / len(rows), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "uniform_curves_L50-500_c72_238_256", "n_c": 1000, "layers": 6},
           "uniform": rows}
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------- cpu baseline --
def chains_bench(M, torch, a):
    """Inversion chains (paper_2003_02256_amd/inversion.py): 256 random-walk
    Metropolis chains on one synthetic site (a 15-layer base of the serving
    recipe, its split-path curve plus 0.5% noise as C_e), every step one
    batched sweep of all proposals plus one device misfit launch."""
    import workloads as WL
    from paper_2003_02256_amd import inversion as I
    base = WL.chain_bases(64, seed=5)
    site = next(b for b in base if b.model.n_layers == 15)
    c = WL.serving_grid()
    ctx_obj = M.Context(0, 2 << 30)
    ctx = ctx_obj.ctx
    ev0 = I.DeviceEvaluator(ctx, c, site.lambdas, np.ones(len(site.lambdas)))
    ct = torch.empty(len(site.lambdas), dtype=torch.float64, device=ev0.dev)
    idx = torch.empty(len(site.lambdas), dtype=torch.int32, device=ev0.dev)
    st = torch.empty_like(idx)
    t = lambda x: torch.as_tensor(np.ascontiguousarray(x, np.float64), device=ev0.dev)
    m = site.model
    M.masw_dispersion_curve(ctx, t(c), t(site.lambdas), t(m.h), t(m.alpha), t(m.beta), t(m.rho),
                            M.MASW_PREC_FP64, M.MASW_NO_REFINE, None, ct, idx, st, None)
    C_e = I.synthetic_curve(ct.cpu().numpy(), 0.005, seed=6)
    useful = [0]

    class Counting(I.DeviceEvaluator):
        def __call__(self, models):
            out = super().__call__(models)
            useful[0] += M.masw_get_stats(ctx)["useful_evals"]
            return out
    ev = Counting(ctx, c, site.lambdas, C_e)
    rng = np.random.Generator(np.random.PCG64(8))
    start = [I.perturb(rng, m, 0.1) for _ in range(256)]
    T = I.misfit_scale(C_e, float(c[1] - c[0]))
    I.run_chains(ev, start[:8], max(1, a.warmup), step=0.02, temperature=T, seed=1)  # warm-up
    useful[0] = 0
    ev.models_evaluated = 0
    M.masw_get_timing(ctx, reset=True)
    import gc
    gc.collect()
    gc.disable()  # no collector pause inside a timed run
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = I.run_chains(ev, start, a.steps, step=0.02, temperature=T, seed=9)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gc.enable()
    tm = M.masw_get_timing(ctx, reset=True)
    # the same chains with the FP64 inertia-count search: its picks are the
    # FP64 walk's, which the split path's equal on these workloads
    ev_i = I.DeviceEvaluator(ctx, c, site.lambdas, C_e, inertia=True)
    I.run_chains(ev_i, start[:8], max(1, a.warmup), step=0.02, temperature=T, seed=1)
    ev_i.models_evaluated = 0
    M.masw_get_timing(ctx, reset=True)
    gc.collect()
    gc.disable()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res_i = I.run_chains(ev_i, start, a.steps, step=0.02, temperature=T, seed=9)
    torch.cuda.synchronize()
    wall_i = time.perf_counter() - t0
    gc.enable()
    tm_i = M.masw_get_timing(ctx, reset=True)
    ctx_obj.close()
    steps = a.steps + 1  # the start models are evaluated too
    print(json.dumps({
        "metric": METRIC, "value": useful[0] / wall, "unit": "det evals/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": wall / steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 sweep + f64 re-check", "data": "synthetic",
        "config": {"workload": "inversion_chains_256x15layers", "chains": 256, "n_layers": 15,
                   "wavelengths": int(len(site.lambdas)), "n_c": int(c.shape[0])},
        "models_per_s": ev.models_evaluated / wall,
        "sweep_ms_per_step": tm["sweep_ms_sum"] / max(1, tm["launches"]),
        "acceptance": res.acceptance_rate,
        "mean_misfit_start": float(np.nanmean(res.start_misfit)),
        "mean_misfit_best": float(np.nanmean(res.best_misfit)),
        "inertia": {"ms_per_step": wall_i / steps * 1e3, "models_per_s": ev_i.models_evaluated / wall_i,
                    "sweep_ms_per_step": tm_i["sweep_ms_sum"] / max(1, tm_i["launches"]),
                    "speedup_vs_split": wall / wall_i, "acceptance": res_i.acceptance_rate,
                    "same_best_misfits": bool(np.array_equal(res_i.best_misfit, res.best_misfit,
                                                             equal_nan=True))},
    }), flush=True)


# ---------------------------------------------------------------- classify --
def _oracle_classify(args):
    from oracle import propagator as PR
    lam, c, idx, model = args
    return PR.classify(lam, c, idx, model)[0]


def classify_bench(M, torch, a):
    """Zero/pole classification (masw_classify_picks) of every pick of the
    4096-model batch: picks from one FP64 batch launch (untimed), then the
    classification launches timed back to back with device-resident inputs.
    The oracle's propagator classifies an evenly spaced sample on the host."""
    import multiprocessing as mp
    import workloads as WL
    wl = WL.batch_case()
    dev = torch.device("cuda:0")
    arrs = M.flatten_models(wl.models, wl.lambdas)
    td = [torch.as_tensor(x, device=dev) for x in arrs]
    c = torch.as_tensor(wl.c_test, device=dev)
    W = int(arrs[-1].shape[0])
    ctx_obj = M.Context(0, 2 << 30)
    ctx = ctx_obj.ctx
    ct = torch.empty(W, dtype=torch.float64, device=dev)
    idx = torch.empty(W, dtype=torch.int32, device=dev)
    st = torch.empty(W, dtype=torch.int32, device=dev)
    cref = torch.empty(W, dtype=torch.float64, device=dev)
    M.masw_dispersion_batch(ctx, c, *td, M.MASW_PREC_FP64, 0, None, ct, idx, st, cref)
    cls = torch.empty(W, dtype=torch.int32, device=dev)
    sec = torch.empty(W, dtype=torch.float64, device=dev)
    for _ in range(a.warmup):
        M.masw_classify_picks(ctx, c, *td, idx, 0, None, cls, sec)
    torch.cuda.synchronize()
    kms, wall, stats = [], 0.0, None
    for _ in range(a.steps):
        t0 = time.perf_counter()
        M.masw_classify_picks(ctx, c, *td, idx, 0, None, cls, sec)
        stats = M.masw_get_stats(ctx)            # waits for the launch
        wall += time.perf_counter() - t0
        kms.append(stats["sweep_ms"])
    kms_mean = float(np.mean(kms))
    flops = classify_flops(stats["classify_evals"], stats["classify_layers"], stats["classify_steps"])
    achieved = flops / (kms_mean * 1e-3) / 1e12
    cls_h, sec_h, cref_h = cls.cpu().numpy(), sec.cpu().numpy(), cref.cpu().numpy()
    mode = cls_h == M.MASW_PICK_MODE
    rel = np.abs(sec_h[mode] - cref_h[mode]) / cref_h[mode]
    idx_h = idx.cpu().numpy()
    ctx_obj.close()
    out = {
        "metric": METRIC, "value": W / (wall / a.steps), "unit": "classified picks/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": wall / a.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "classify_batch_4096models_19001c", "models": len(wl.models), "picks": W},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": MEASURED_TRAFFIC.get((kernel_source_hash(CLASSIFY_SOURCES),
                                                      "classify_batch_4096models_19001c", "classify_kernel")),
                     "kernel": "classify_kernel", "kernel_ms": kms_mean, "flops_per_launch": flops},
        "counts": {"mode": int(mode.sum()), "pole": int((cls_h == M.MASW_PICK_POLE).sum()),
                   "other": int((~mode & (cls_h != M.MASW_PICK_POLE)).sum())},
        "secular_evals": stats["classify_evals"], "layers_crossed": stats["classify_layers"],
        "propagator_steps": stats["classify_steps"],
        "root_rel_diff_vs_stiffness_max": float(rel.max()) if rel.size else None,
    }
    if not a.no_cpu_baseline:
        pairs = [(float(l), mi) for mi, ls in enumerate(wl.lambdas) for l in ls]
        pick = np.linspace(0, W - 1, 64).round().astype(int)
        tasks = [(pairs[i][0], wl.c_test, int(idx_h[i]), wl.models[pairs[i][1]]) for i in pick]
        workers = min(16, os.cpu_count() or 1)
        os.environ["OMP_NUM_THREADS"] = "1"
        t0 = time.perf_counter()
        with mp.get_context("fork").Pool(workers) as pool:
            want = pool.map(_oracle_classify, tasks, chunksize=1)
        cpu_wall = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": len(tasks) / cpu_wall, "unit": "classified picks/s", "cores": workers,
                               "kind": "oracle",
                               "sample": f"{len(tasks)} of {W} picks evenly spaced, {cpu_wall:.1f} s wall on "
                                         f"{workers} processes"}
        out["oracle_class_mismatches"] = int(sum(int(w != cls_h[i]) for w, i in zip(want, pick)))
    print(json.dumps(out), flush=True)


def _oracle_point(args):
    import oracle as O
    lam, c, model = args
    p = O.dispersion_point(lam, c, model, refine=True)
    return p.evals


def cpu_baseline(wl, target_s: float, workers: int):
    """The oracle (dense complex LU per determinant, FP64) on a bounded,
    evenly spaced sample of the workload's wavelengths, on `workers` host
    processes; returns useful evals/s."""
    import multiprocessing as mp
    os.environ["OMP_NUM_THREADS"] = "1"
    lam_all = [(float(l), mi) for mi, ls in enumerate(wl.lambdas) for l in ls]
    # ~45 us per 42x42 determinant on one core: size the sample to target_s of work
    per_eval_s = 45e-6 * (np.mean([m.n_layers for m in wl.models]) + 1) / 21.0
    est_depth = 0.3 * wl.c_test.shape[0]
    n = int(max(workers, min(len(lam_all), target_s / (per_eval_s * est_depth))))
    pick = np.unique(np.linspace(0, len(lam_all) - 1, n).round().astype(int))
    tasks = [(lam_all[i][0], wl.c_test, wl.models[lam_all[i][1]]) for i in pick]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        evals = pool.map(_oracle_point, tasks, chunksize=1)
    wall = time.perf_counter() - t0
    cpu = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": float(sum(evals) / wall), "unit": "useful det evals/s", "cores": workers,
            "kind": "oracle",
            "sample": f"{len(tasks)} of {len(lam_all)} wavelengths evenly spaced, {sum(evals)} useful evals, "
                      f"{wall:.1f} s wall on {workers} processes ({cpu})"}


# ---------------------------------------------------------------------- main --
def inertia_leg(wl, r64, r_i, wall64, wall_i, sweep_i, st_i, n_lay, n_curves):
    """The FP64 inertia-count search on the same inputs: its outputs against
    the FP64 walk's (bitwise), its rates in wavelengths and curves per second
    and the work it performed (inertia counts, and the determinant signs it
    evaluated), and its kernel's own roofline from its work counters: the
    inertia counts, plus the determinant signs of the sampling, refinement and
    of any walk at or above the half-space's S velocity (F(N) each, N the mean
    layer count of the wavelengths)."""
    same = all(np.array_equal(x, y, equal_nan=True) for x, y in zip(r64, r_i))
    nbar = float(np.mean(n_lay)) if len(n_lay) else 0.0
    det_evals = st_i["sweep_evals"] + st_i["check_evals"] + st_i["refine_evals"]
    flops = (inertia_flops(st_i["inertia_evals"], st_i["inertia_entries"], st_i["inertia_pivots"])
             + det_evals * flops_per_eval(nbar))
    achieved = flops / (sweep_i * 1e-3) / 1e12
    # the library runs the variant for at most one wavefront per SIMD when the
    # wavelengths, four per workgroup (one per SIMD), need no more workgroups
    # than there are CUs
    lone = st_i["workgroups"] <= st_i["cus"]
    kname = "inertia_lone_kernel" if lone else "inertia_kernel"
    return {
        "value": wl.n_lambda_total / wall_i, "unit": "wavelengths/s",
        "ms_per_step": wall_i * 1e3, "dtype": "f64", "speedup_vs_fp64_walk": wall64 / wall_i,
        "curves_per_s": n_curves / wall_i,
        "outputs_bitwise_equal_to_fp64_walk": bool(same),
        "idx_mismatch_vs_fp64": int(np.sum(r64[1] != r_i[1])),
        "performed": {"inertia_counts": st_i["inertia_evals"], "element_matrices": st_i["inertia_entries"],
                      "pivots": st_i["inertia_pivots"], "det_signs": det_evals,
                      "walked": st_i["sweep_evals"], "check": st_i["check_evals"],
                      "refine": st_i["refine_evals"]},
        "performed_counts_and_signs_per_s": (st_i["inertia_evals"] + det_evals) / wall_i,
        "kernel_ms": sweep_i,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": MEASURED_TRAFFIC.get((kernel_source_hash(INERTIA_SOURCES), wl.name, kname)),
                     "kernel": kname,
                     "kernel_ms": sweep_i, "flops_per_launch": flops},
    }


def measure_curves(M, torch, wl, steps: int, warmup: int, inertia: bool = True) -> dict:
    """One workload through masw_dispersion_curve / _batch with inputs resident
    in HBM: the plain FP64 walk (the headline rate), the split path and the
    FP64 inertia-count search on the same inputs, each timed over `steps`
    back-to-back jobs after `warmup`, and the FP64 sweep kernel's roofline
    from the library's HIP events."""
    dev = torch.device("cuda:0")
    log(f"workload {wl.name}: {len(wl.models)} model(s), {wl.n_lambda_total} wavelengths, {wl.c_test.shape[0]} c")
    job = DeviceJob(wl, torch, dev)
    ctx_obj = M.Context(0, 4 << 30)
    ctx = ctx_obj.ctx
    # first call (includes module load and first-touch of the arena) vs steady state
    t0 = time.perf_counter()
    job.run(ctx, M.MASW_PREC_FP64)
    torch.cuda.synchronize()
    first_call_ms = (time.perf_counter() - t0) * 1e3

    log(f"{wl.name}: timing the FP64 path")
    wall64, sweep64, total64, st64, x64 = time_path(job, ctx, M.MASW_PREC_FP64, steps, warmup)
    r64 = job.results(M.MASW_PREC_FP64)
    log(f"{wl.name}: timing the split path")
    wall32, sweep32, total32, st32, _ = time_path(job, ctx, M.MASW_PREC_SPLIT, steps, warmup)
    r32 = job.results(M.MASW_PREC_SPLIT)
    if inertia:
        log(f"{wl.name}: timing the inertia-count search")
        wall_i, sweep_i, total_i, st_i, _ = time_path(job, ctx, "inertia", steps, warmup)
        st_i["cus"] = torch.cuda.get_device_properties(0).multi_processor_count
        r_i = job.results("inertia")
    graph = graph_replay(M, torch, job, ctx, steps, warmup, r64) if job.single and wl.n_lambda_total <= 1024 else None
    ctx_obj.close()

    idx64, idx32 = r64[1], r32[1]
    useful = int(np.where(idx64 >= 0, idx64 + 1, wl.c_test.shape[0]).sum())
    assert useful == st64["useful_evals"], (useful, st64["useful_evals"])
    both = (idx64 == idx32) & (idx64 >= 0)
    root_rel = np.abs(r32[3][both] - r64[3][both]) / r64[3][both]

    # algorithmic flops of one FP64 launch: the evaluations the method needs
    # (every grid point up to each pick, plus the refinement) x F(N); rounds
    # evaluated past a pick, speculatively or to fill a round, are not counted
    n_lay = np.asarray(job.n_layers)[job.lam_model]
    nbar = float(np.average(n_lay, weights=np.where(idx64 >= 0, idx64 + 1, wl.c_test.shape[0])))
    performed64 = st64["sweep_evals"] + st64["check_evals"] + st64["refine_evals"]
    algorithmic64 = st64["useful_evals"] + st64["check_evals"] + st64["refine_evals"]
    flops64 = algorithmic64 * flops_per_eval(nbar)
    achieved = flops64 / (sweep64 * 1e-3) / 1e12
    algorithmic32 = st32["useful_evals"] + st32["check_evals"] + st32["refine_evals"]
    achieved32 = algorithmic32 * flops_per_eval(nbar) / (sweep32 * 1e-3) / 1e12
    n_curves = len(wl.models)
    kname = ("fused_sweep_kernel<FP64>" if st64.get("fused_staging")
             else f"sweep_kernel<FP64,G={st64['waves_per_item']}>")
    traffic = MEASURED_TRAFFIC.get((kernel_source_hash(), wl.name, kname))
    res = {
        "value": useful / wall64, "unit": "det evals/s", "ms_per_step": wall64 * 1e3, "dtype": "f64",
        "config": {"workload": wl.name, "models": n_curves, "wavelengths": wl.n_lambda_total,
                   "n_c": int(wl.c_test.shape[0]), "layers_mean": nbar, "path": "plain FP64"},
        "curves_per_s": n_curves / wall64,
        "wavelengths_per_s": wl.n_lambda_total / wall64,
        "useful_evals": useful,
        "performed_evals": performed64,
        "algorithmic_evals": algorithmic64,
        "first_call_ms": first_call_ms,
        "device_ms_per_step": total64,
        "timing": {"ms_per_step_with_events": x64["ms_per_step_with_events"],
                   "device_ms_per_step_counter": x64["device_ms_per_step_counter"],
                   "sweep_ms_counter": x64["sweep_ms_counter"],
                   "note": "ms_per_step: the library's default timing (GPU real-time counter); "
                           "device times and roofline: a second pass with HIP events per launch"},
        "split": {
            "value": useful / wall32, "unit": "det evals/s", "ms_per_step": wall32 * 1e3,
            "dtype": "f32 sweep + f64 re-check/refine", "speedup_vs_fp64": wall64 / wall32,
            "curves_per_s": n_curves / wall32, "wavelengths_per_s": wl.n_lambda_total / wall32,
            "sweep_evals": st32["sweep_evals"], "check_evals": st32["check_evals"],
            "refine_evals": st32["refine_evals"], "sweep_kernel_ms": sweep32,
            "kernel": (("fused_sweep_kernel<FP64>" if st32.get("fused_staging")
                        else f"sweep_kernel<FP64,G={st32['waves_per_item']}>") if st32.get("split_as_fp64")
                       else "fused_sweep_kernel<split>" if st32.get("fused_staging")
                       else f"sweep_kernel<split,G={st32['waves_per_item']}>"),
            "split_as_fp64": bool(st32.get("split_as_fp64")),
            "achieved_tflops_fp64_counted": achieved32,
            "idx_mismatch_vs_fp64": int(np.sum((idx64 != idx32))),
            "root_rel_err_vs_fp64_max": float(root_rel.max()) if root_rel.size else None,
            "root_rel_err_vs_fp64_mean": float(root_rel.mean()) if root_rel.size else None,
        },
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic,
                     "kernel": kname,
                     "kernel_ms": sweep64, "flops_per_launch": flops64},
    }
    if inertia:
        res["inertia"] = inertia_leg(wl, r64, r_i, wall64, wall_i, sweep_i, st_i, n_lay, n_curves)
    if graph:
        res["graph"] = graph
    return res


def graph_replay(M, torch, job, ctx, steps: int, warmup: int, r64) -> dict:
    """A small job as one captured hipGraph: the FP64 curve call without
    allocation (masw_dispersion_curve_noalloc: staging and sweep, two kernel
    nodes) captured once on a side stream and replayed back to back.  Every
    output of the last replay must equal the eager FP64 call's."""
    a = job.arrs
    W = job.W
    out = (torch.empty(W, dtype=torch.float64, device="cuda:0"), torch.empty(W, dtype=torch.int32, device="cuda:0"),
           torch.empty(W, dtype=torch.int32, device="cuda:0"), torch.empty(W, dtype=torch.float64, device="cuda:0"))
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    call = M.PreparedCurve(ctx, job.c, a[6], a[1], a[2], a[3], a[4], M.MASW_PREC_FP64, 0, side.cuda_stream, *out,
                           noalloc=True)
    with torch.cuda.stream(side):
        call()                      # eager once on the side stream
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        call()
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    same = all(np.array_equal(o.cpu().numpy(), x, equal_nan=True) for o, x in zip(out, r64))
    return {"ms_per_step": wall * 1e3, "entry": "masw_dispersion_curve_noalloc replayed as a captured hipGraph",
            "outputs_equal_eager_fp64": bool(same)}


def serving_leg(M, torch, seconds: float) -> dict:
    """A short replay of the serving trace (2000 req/s Poisson arrivals from
    64 random-walk chains, 1 s warm-up): p50/p99 latency and curves/s of the
    split path, of the plain-FP64 server and of the FP64 server with the
    inertia-count search, on the identical trace."""
    import workloads as WL
    c = WL.serving_grid()
    warm = 1.0
    times, reqs = serving_trace(2000.0, warm, seconds)
    log(f"serving leg: {len(times)} requests over {warm + seconds:.0f} s, split, FP64, FP64 inertia search")
    ctx_obj = M.Context(0, 4 << 30)
    split, idx_s = run_serving(M, ctx_obj.ctx, M.MASW_PREC_SPLIT, times, reqs, c, warm)
    fp64, idx_d = run_serving(M, ctx_obj.ctx, M.MASW_PREC_FP64, times, reqs, c, warm)
    inertia, idx_i = run_serving(M, ctx_obj.ctx, M.MASW_PREC_FP64, times, reqs, c, warm, search_inertia=1)
    ctx_obj.close()
    keep = ("requests", "p50_ms", "p99_ms", "mean_ms", "max_ms", "curves_per_s", "det_evals_per_s", "busy_frac",
            "submit_lag_us")
    return {"workload": "serving_64chains_2000rps", "seconds": seconds, "n_c": int(c.shape[0]),
            "split": {k: split[k] for k in keep}, "fp64": {k: fp64[k] for k in keep},
            "fp64_inertia": {k: inertia[k] for k in keep},
            "idx_mismatch_split_vs_fp64": sum(int(np.sum(x != y)) for x, y in zip(idx_s, idx_d)),
            "idx_mismatch_inertia_vs_fp64": sum(int(np.sum(x != y)) for x, y in zip(idx_i, idx_d))}


def _oracle_curve_points(args):
    import oracle as O
    lam, c, model = args
    p = O.dispersion_point(lam, c, model, refine=True)
    return p.idx, p.c_ref, p.evals


def two_layer_vs_oracle(M, torch, workers: int) -> dict:
    """The split path on the two-layer case (30 wavelengths, 801 velocities)
    against the oracle, per wavelength: grid-index mismatches and the root
    error |c_ref - c_ref_oracle| / c_ref_oracle (max and mean over the
    curve), with the plain FP64 path beside it.  The oracle runs on the host
    here, as part of the CPU leg."""
    import multiprocessing as mp
    import workloads as WL
    wl = WL.two_layer_case()
    m, lam, c = wl.models[0], wl.lambdas[0], wl.c_test
    ctx_obj = M.Context(0, 64 << 20)
    got = {p: ctx_obj.curve(c, lam, m, p) for p in (M.MASW_PREC_SPLIT, M.MASW_PREC_FP64)}
    ctx_obj.close()
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        want = pool.map(_oracle_curve_points, [(float(l), c, m) for l in lam], chunksize=1)
    wall = time.perf_counter() - t0
    w_idx = np.array([w[0] for w in want])
    w_ref = np.array([w[1] for w in want])
    out = {"workload": wl.name, "wavelengths": int(len(lam)), "oracle_s": wall}
    for p, name in ((M.MASW_PREC_SPLIT, "split"), (M.MASW_PREC_FP64, "fp64")):
        ct, idx, st, cr = got[p]
        ok = (idx == w_idx) & (w_idx >= 0)
        rel = np.abs(cr[ok] - w_ref[ok]) / w_ref[ok]
        out[name] = {"idx_mismatch_vs_oracle": int(np.sum(idx != w_idx)),
                     "root_rel_err_max": float(rel.max()) if rel.size else None,
                     "root_rel_err_mean": float(rel.mean()) if rel.size else None}
    return out


def host_workers() -> int:
    """Host processes for the oracle: the CPUs this process may run on,
    at most 16 (one GPU's share of the GPU machine's host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: per workload)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed warm-up steps (default: per workload)")
    ap.add_argument("--workload", default="batch",
                    choices=["fine_scale", "two_layer", "batch", "serving", "uniform", "chains", "classify"])
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="measured seconds of the serving trace")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true",
                    help="batch workload: only the headline, without the fine-scale, serving and two-layer legs")
    ap.add_argument("--serve-leg-seconds", type=float, default=2.0,
                    help="measured seconds of the serving leg of the default run")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="target CPU work of the oracle sample")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times (the reference "
                         "for scaling HBM counter readings) and exit")
    a = ap.parse_args()
    # Defaults: at least ~0.3 s of warm-up and timed work for the short jobs,
    # so that the GPU clock has left its idle state before the timed steps.
    steps, warmup = DEFAULT_STEPS.get(a.workload, (20, 3))
    a.steps = steps if a.steps is None else a.steps
    a.warmup = warmup if a.warmup is None else a.warmup
    if a.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {a.gpus} is not supported (the dispersion path has no "
              f"cross-GPU exchange; the library runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2003_02256_amd as M
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if a.calibrate_copy:
        n = a.calibrate_copy << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "copies": 3}), flush=True)
        return
    M.library()
    if a.workload == "serving":
        serving_bench(M, torch, a)
        return
    if a.workload == "uniform":
        uniform_bench(M, torch, a)
        return
    if a.workload == "chains":
        chains_bench(M, torch, a)
        return
    if a.workload == "classify":
        classify_bench(M, torch, a)
        return
    import workloads as WL
    wl = make_workload(a.workload)
    res = {"metric": METRIC}
    head = measure_curves(M, torch, wl, a.steps, a.warmup)
    res.update({"value": head.pop("value"), "unit": head.pop("unit"), "n_gpus": 1, "steps": a.steps,
                "warmup": a.warmup, "ms_per_step": head.pop("ms_per_step"), "higher_is_better": True,
                "scaling": "weak", "vs_baseline": None, "dtype": head.pop("dtype"), "data": "synthetic",
                "config": head.pop("config")})
    res.update(head)
    if a.workload == "batch" and not a.no_legs:
        # the other configurations, each a leg of its own beside the headline
        fs_steps, fs_warm = DEFAULT_STEPS["fine_scale"]
        fs = measure_curves(M, torch, WL.fine_scale_case(), fs_steps, fs_warm)
        fs["steps"], fs["warmup"] = fs_steps, fs_warm
        res["fine_scale"] = fs
        res["serving"] = serving_leg(M, torch, a.serve_leg_seconds)
    if not a.no_cpu_baseline:
        workers = host_workers()
        log(f"timing the CPU oracle on a sample ({workers} processes)")
        res["cpu_baseline"] = cpu_baseline(wl, a.cpu_seconds, workers)
        if a.workload == "batch" and not a.no_legs:
            log("the two-layer case against the oracle")
            res["two_layer_vs_oracle"] = two_layer_vs_oracle(M, torch, workers)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
