"""Python binding of the MI355X dispersion-curve library (libmasw.so).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in include/masw.h.  The functions below
carry the C names; numpy arrays are passed as host pointers and torch tensors
on a GPU as device pointers (MASW_DEVICE_PTRS is added automatically).  If the
library has not been built, importing works but every call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmasw.so")

# --------------------------------------------------------------- constants --
MASW_OK = 0
MASW_EINVAL = -1
MASW_ENOMEM = -2
MASW_EBUSY = -3
MASW_EDEVICE = -4
MASW_ETIMEOUT = -5
MASW_ENOENT = -6

MASW_STATUS_FOUND = 0
MASW_STATUS_NOT_FOUND = 1
MASW_STATUS_INVALID = 2
MASW_STATUS_NAN = 3
MASW_FLAG_POLE = 0x100
MASW_FLAG_NOISE = 0x200

MASW_PICK_MODE = 0
MASW_PICK_POLE = 1
MASW_PICK_LEAKY = 2
MASW_PICK_NONE = 3
MASW_PICK_UNRESOLVED = 4
MASW_PICK_INVALID = 5

MASW_PREC_FP64 = 0
MASW_PREC_SPLIT = 1

MASW_DEVICE_PTRS = 0x1
MASW_NO_REFINE = 0x2
MASW_CHECK_NOISE = 0x4
MASW_SEARCH_INERTIA = 0x8
MASW_MAX_LAYERS = 1024
MASW_NOALLOC_SCRATCH_BYTES = 32 << 20


class MaswError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: {detail} (code {code})")
        self.code = code


# ------------------------------------------------------------------ structs --
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


class masw_model(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int32), ("h", _dp), ("alpha", _dp),
                ("beta", _dp), ("rho", _dp)]


class masw_batch(ctypes.Structure):
    _fields_ = [("n_models", ctypes.c_int32), ("layer_off", _ip), ("h", _dp),
                ("alpha", _dp), ("beta", _dp), ("rho", _dp),
                ("lambda_off", _ip), ("lambda_", _dp)]


class masw_outputs(ctypes.Structure):
    _fields_ = [("c_t", _dp), ("idx", _ip), ("status", _ip), ("c_ref", _dp)]


class masw_stats(ctypes.Structure):
    _fields_ = [("useful_evals", ctypes.c_uint64), ("sweep_evals", ctypes.c_uint64),
                ("check_evals", ctypes.c_uint64), ("refine_evals", ctypes.c_uint64),
                ("n_lambda", ctypes.c_uint64), ("waves_per_item", ctypes.c_int32),
                ("workgroups", ctypes.c_int32), ("sweep_ms", ctypes.c_float), ("total_ms", ctypes.c_float),
                ("shared_items", ctypes.c_int32), ("shared_stalls", ctypes.c_uint32),
                ("helper_evals", ctypes.c_uint64), ("classify_evals", ctypes.c_uint64),
                ("classify_layers", ctypes.c_uint64), ("classify_steps", ctypes.c_uint64),
                ("inertia_evals", ctypes.c_uint64), ("inertia_entries", ctypes.c_uint64),
                ("inertia_pivots", ctypes.c_uint64), ("fused_staging", ctypes.c_int32),
                ("split_as_fp64", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class masw_opts(ctypes.Structure):
    _fields_ = [("refine_rel_tol", ctypes.c_double), ("noise_threshold", ctypes.c_double),
                ("waves_per_item", ctypes.c_int32), ("shared_window", ctypes.c_int32),
                ("first_item_priority", ctypes.c_int32), ("timing_events", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class masw_timing(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_uint64), ("sweep_ms_sum", ctypes.c_double),
                ("total_ms_sum", ctypes.c_double), ("sweep_ms_min", ctypes.c_float),
                ("sweep_ms_max", ctypes.c_float)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class masw_server_opts(ctypes.Structure):
    _fields_ = [("max_layers", ctypes.c_int32), ("max_lambda", ctypes.c_int32), ("max_grid", ctypes.c_int32),
                ("rounds_per_tick", ctypes.c_int32), ("pool_bytes", ctypes.c_size_t),
                ("tick_timeout_us", ctypes.c_int64), ("search_inertia", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class masw_request_info(ctypes.Structure):
    _fields_ = [("submit_ns", ctypes.c_uint64), ("admit_ns", ctypes.c_uint64), ("done_ns", ctypes.c_uint64),
                ("ticks", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class masw_server_stats(ctypes.Structure):
    _fields_ = [("ticks", ctypes.c_uint64), ("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("admit_waits", ctypes.c_uint64), ("max_resident", ctypes.c_uint32), ("resident", ctypes.c_uint32),
                ("pool_bytes", ctypes.c_uint64), ("busy_ms", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


# ------------------------------------------------------------------ loading --
_lib = None


def library() -> ctypes.CDLL:
    """The loaded libmasw.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise MaswError(MASW_EDEVICE, "libmasw.so",
                            f"not built ({LIB_PATH}); run paper_2003_02256_amd.build")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i32, u32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_size_t
        sig = {
            "masw_create": (ctypes.c_int, [ctypes.c_int, sz, ctypes.POINTER(vp)]),
            "masw_destroy": (None, [vp]),
            "masw_dispersion_curve": (ctypes.c_int, [vp, vp, i32, vp, i32, ctypes.POINTER(masw_model),
                                                     ctypes.c_int, u32, vp, vp, vp, vp, vp]),
            "masw_dispersion_curve_noalloc": (ctypes.c_int, [vp, vp, i32, vp, i32, ctypes.POINTER(masw_model),
                                                             ctypes.c_int, u32, vp, vp, vp, vp, vp]),
            "masw_dispersion_batch_misfit": (ctypes.c_int, [vp, vp, i32, ctypes.POINTER(masw_batch), ctypes.c_int,
                                                            u32, vp, ctypes.POINTER(masw_outputs), vp, vp]),
            "masw_dispersion_batch": (ctypes.c_int, [vp, vp, i32, ctypes.POINTER(masw_batch),
                                                     ctypes.c_int, u32, vp, ctypes.POINTER(masw_outputs)]),
            "masw_sign_map": (ctypes.c_int, [vp, vp, i32, vp, i32, ctypes.POINTER(masw_model),
                                             ctypes.c_int, u32, vp, vp, vp]),
            "masw_get_stats": (ctypes.c_int, [vp, ctypes.POINTER(masw_stats)]),
            "masw_get_timing": (ctypes.c_int, [vp, ctypes.c_int, ctypes.POINTER(masw_timing)]),
            "masw_set_opts": (ctypes.c_int, [vp, ctypes.POINTER(masw_opts)]),
            "masw_get_opts": (ctypes.c_int, [vp, ctypes.POINTER(masw_opts)]),
            "masw_misfit": (ctypes.c_int, [vp, i32, vp, vp, vp, u32, vp, vp]),
            "masw_classify_picks": (ctypes.c_int, [vp, vp, i32, ctypes.POINTER(masw_batch), vp, u32, vp,
                                                   vp, vp]),
            "masw_server_start": (ctypes.c_int, [vp, ctypes.POINTER(masw_server_opts)]),
            "masw_server_stop": (ctypes.c_int, [vp]),
            "masw_submit": (ctypes.c_int, [vp, vp, i32, vp, i32, ctypes.POINTER(masw_model), ctypes.c_int, u32,
                                           ctypes.POINTER(ctypes.c_uint64)]),
            "masw_poll": (ctypes.c_int, [vp, ctypes.c_uint64, vp, vp, vp, vp, ctypes.POINTER(masw_request_info)]),
            "masw_wait": (ctypes.c_int, [vp, ctypes.c_uint64, ctypes.c_int64, vp, vp, vp, vp,
                                         ctypes.POINTER(masw_request_info)]),
            "masw_server_get_stats": (ctypes.c_int, [vp, ctypes.POINTER(masw_server_stats)]),
            "masw_strerror": (ctypes.c_char_p, [ctypes.c_int]),
            "masw_last_error": (ctypes.c_char_p, []),
            "masw_version": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(rc: int, where: str) -> int:
    if rc != MASW_OK:
        lib = library()
        raise MaswError(rc, where, f"{lib.masw_strerror(rc).decode()}: {lib.masw_last_error().decode()}")
    return rc


# -------------------------------------------------------------- marshalling --
def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _ptr(x, dtype) -> Optional[int]:
    """Address of a contiguous numpy array or torch tensor of `dtype`."""
    if x is None:
        return None
    if _is_torch(x):
        import torch
        want = {np.float64: torch.float64, np.int32: torch.int32, np.int8: torch.int8}[dtype]
        if x.dtype != want or not x.is_contiguous():
            raise MaswError(MASW_EINVAL, "marshal", f"tensor must be contiguous {want}")
        return x.data_ptr()
    if not isinstance(x, np.ndarray) or x.dtype != dtype or not x.flags.c_contiguous:
        raise MaswError(MASW_EINVAL, "marshal", f"array must be a contiguous {np.dtype(dtype)} ndarray")
    return x.ctypes.data


def _device_flag(*xs) -> int:
    devs = [_is_torch(x) and x.is_cuda for x in xs if x is not None]
    if any(devs) and not all(devs):
        raise MaswError(MASW_EINVAL, "marshal", "mix of host and device buffers")
    return MASW_DEVICE_PTRS if (devs and all(devs)) else 0


def _stream(stream, device_flag: int):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    if device_flag:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return None


def _model_struct(h, alpha, beta, rho) -> masw_model:
    m = masw_model()
    m.n_layers = int(alpha.shape[0]) - 1
    m.h = ctypes.cast(_ptr(h, np.float64), _dp) if int(h.shape[0]) > 0 else ctypes.cast(None, _dp)
    m.alpha = ctypes.cast(_ptr(alpha, np.float64), _dp)
    m.beta = ctypes.cast(_ptr(beta, np.float64), _dp)
    m.rho = ctypes.cast(_ptr(rho, np.float64), _dp)
    return m


# ------------------------------------------------------------------ C names --
def masw_version() -> str:
    return library().masw_version().decode()


def masw_strerror(code: int) -> str:
    return library().masw_strerror(code).decode()


def masw_last_error() -> str:
    return library().masw_last_error().decode()


def masw_create(device: int = 0, hbm_budget_bytes: int = 0) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    _check(library().masw_create(device, hbm_budget_bytes, ctypes.byref(ctx)), "masw_create")
    return ctx


def masw_destroy(ctx) -> None:
    if ctx:
        library().masw_destroy(ctx)


def masw_dispersion_curve(ctx, c_test, lam, h, alpha, beta, rho, prec: int, flags: int,
                          stream, C_t, idx, status, c_ref=None) -> int:
    """Marshals to the C function of the same name (see include/masw.h)."""
    fl = flags | _device_flag(c_test, lam, h, alpha, beta, rho, C_t, idx, status, c_ref)
    m = _model_struct(h, alpha, beta, rho)
    return _check(library().masw_dispersion_curve(
        ctx, _ptr(c_test, np.float64), int(c_test.shape[0]), _ptr(lam, np.float64), int(lam.shape[0]),
        ctypes.byref(m), prec, fl, _stream(stream, fl & MASW_DEVICE_PTRS),
        _ptr(C_t, np.float64), _ptr(idx, np.int32), _ptr(status, np.int32), _ptr(c_ref, np.float64)),
        "masw_dispersion_curve")


def masw_dispersion_curve_noalloc(ctx, c_test, lam, h, alpha, beta, rho, prec: int, flags: int,
                                  stream, C_t, idx, status, c_ref=None) -> int:
    """Marshals to the C function of the same name (see include/masw.h):
    device tensors only, the workspace in the library's static scratch."""
    fl = flags | _device_flag(c_test, lam, h, alpha, beta, rho, C_t, idx, status, c_ref)
    m = _model_struct(h, alpha, beta, rho)
    return _check(library().masw_dispersion_curve_noalloc(
        ctx, _ptr(c_test, np.float64), int(c_test.shape[0]), _ptr(lam, np.float64), int(lam.shape[0]),
        ctypes.byref(m), prec, fl, _stream(stream, fl & MASW_DEVICE_PTRS),
        _ptr(C_t, np.float64), _ptr(idx, np.int32), _ptr(status, np.int32), _ptr(c_ref, np.float64)),
        "masw_dispersion_curve_noalloc")


def _batch_structs(layer_off, h, alpha, beta, rho, lambda_off, lam, C_t, idx, status, c_ref):
    b = masw_batch()
    b.n_models = int(layer_off.shape[0]) - 1
    b.layer_off = ctypes.cast(_ptr(layer_off, np.int32), _ip)
    b.h = ctypes.cast(_ptr(h, np.float64), _dp)
    b.alpha = ctypes.cast(_ptr(alpha, np.float64), _dp)
    b.beta = ctypes.cast(_ptr(beta, np.float64), _dp)
    b.rho = ctypes.cast(_ptr(rho, np.float64), _dp)
    b.lambda_off = ctypes.cast(_ptr(lambda_off, np.int32), _ip)
    b.lambda_ = ctypes.cast(_ptr(lam, np.float64), _dp)
    o = masw_outputs()
    o.c_t = ctypes.cast(_ptr(C_t, np.float64), _dp)
    o.idx = ctypes.cast(_ptr(idx, np.int32), _ip)
    o.status = ctypes.cast(_ptr(status, np.int32), _ip)
    o.c_ref = ctypes.cast(_ptr(c_ref, np.float64), _dp)
    return b, o


def masw_dispersion_batch(ctx, c_test, layer_off, h, alpha, beta, rho, lambda_off, lam,
                          prec: int, flags: int, stream, C_t, idx, status, c_ref=None) -> int:
    fl = flags | _device_flag(c_test, layer_off, h, alpha, beta, rho, lambda_off, lam, C_t, idx, status, c_ref)
    b, o = _batch_structs(layer_off, h, alpha, beta, rho, lambda_off, lam, C_t, idx, status, c_ref)
    return _check(library().masw_dispersion_batch(
        ctx, _ptr(c_test, np.float64), int(c_test.shape[0]), ctypes.byref(b), prec, fl,
        _stream(stream, fl & MASW_DEVICE_PTRS), ctypes.byref(o)), "masw_dispersion_batch")


def masw_dispersion_batch_misfit(ctx, c_test, layer_off, h, alpha, beta, rho, lambda_off, lam,
                                 prec: int, flags: int, stream, C_t, idx, status, c_ref, C_e, misfit) -> int:
    """Marshals to the C function of the same name (see include/masw.h)."""
    fl = flags | _device_flag(c_test, layer_off, h, alpha, beta, rho, lambda_off, lam, C_t, idx, status, c_ref,
                              C_e, misfit)
    b, o = _batch_structs(layer_off, h, alpha, beta, rho, lambda_off, lam, C_t, idx, status, c_ref)
    return _check(library().masw_dispersion_batch_misfit(
        ctx, _ptr(c_test, np.float64), int(c_test.shape[0]), ctypes.byref(b), prec, fl,
        _stream(stream, fl & MASW_DEVICE_PTRS), ctypes.byref(o), _ptr(C_e, np.float64), _ptr(misfit, np.float64)),
        "masw_dispersion_batch_misfit")


def masw_sign_map(ctx, c_test, lam, h, alpha, beta, rho, prec: int, flags: int, stream,
                  sigma, log_abs_det=None) -> int:
    fl = flags | _device_flag(c_test, lam, h, alpha, beta, rho, sigma, log_abs_det)
    m = _model_struct(h, alpha, beta, rho)
    return _check(library().masw_sign_map(
        ctx, _ptr(c_test, np.float64), int(c_test.shape[0]), _ptr(lam, np.float64), int(lam.shape[0]),
        ctypes.byref(m), prec, fl, _stream(stream, fl & MASW_DEVICE_PTRS),
        _ptr(sigma, np.int8), _ptr(log_abs_det, np.float64)), "masw_sign_map")


def masw_classify_picks(ctx, c_test, layer_off, h, alpha, beta, rho, lambda_off, lam, idx,
                        flags: int, stream, pick_class, c_sec=None) -> int:
    """Marshals to the C function (zero/pole class of the change at idx)."""
    fl = flags | _device_flag(c_test, layer_off, h, alpha, beta, rho, lambda_off, lam, idx, pick_class, c_sec)
    b = masw_batch()
    b.n_models = int(layer_off.shape[0]) - 1
    b.layer_off = ctypes.cast(_ptr(layer_off, np.int32), _ip)
    b.h = ctypes.cast(_ptr(h, np.float64), _dp)
    b.alpha = ctypes.cast(_ptr(alpha, np.float64), _dp)
    b.beta = ctypes.cast(_ptr(beta, np.float64), _dp)
    b.rho = ctypes.cast(_ptr(rho, np.float64), _dp)
    b.lambda_off = ctypes.cast(_ptr(lambda_off, np.int32), _ip)
    b.lambda_ = ctypes.cast(_ptr(lam, np.float64), _dp)
    return _check(library().masw_classify_picks(
        ctx, _ptr(c_test, np.float64), int(c_test.shape[0]), ctypes.byref(b), _ptr(idx, np.int32), fl,
        _stream(stream, fl & MASW_DEVICE_PTRS), _ptr(pick_class, np.int32), _ptr(c_sec, np.float64)),
        "masw_classify_picks")


def masw_misfit(ctx, lambda_off, C_t, C_e, flags: int, stream, misfit) -> int:
    """Marshals to the C function (Algorithm 2 per model)."""
    fl = flags | _device_flag(lambda_off, C_t, C_e, misfit)
    return _check(library().masw_misfit(ctx, int(lambda_off.shape[0]) - 1, _ptr(lambda_off, np.int32),
                                        _ptr(C_t, np.float64), _ptr(C_e, np.float64), fl,
                                        _stream(stream, fl & MASW_DEVICE_PTRS), _ptr(misfit, np.float64)),
                  "masw_misfit")


def masw_set_opts(ctx, refine_rel_tol=0.0, noise_threshold=0.0, waves_per_item=0, shared_window=0,
                  first_item_priority=0, timing_events=0) -> int:
    """Options of ctx (zero = default; see masw_opts in include/masw.h)."""
    o = masw_opts(refine_rel_tol, noise_threshold, waves_per_item, shared_window, first_item_priority,
                  timing_events)
    return _check(library().masw_set_opts(ctx, ctypes.byref(o)), "masw_set_opts")


def masw_get_opts(ctx) -> dict:
    o = masw_opts()
    _check(library().masw_get_opts(ctx, ctypes.byref(o)), "masw_get_opts")
    return o.as_dict()


def masw_get_stats(ctx) -> dict:
    s = masw_stats()
    _check(library().masw_get_stats(ctx, ctypes.byref(s)), "masw_get_stats")
    return s.as_dict()


def masw_get_timing(ctx, reset: bool = False) -> dict:
    t = masw_timing()
    _check(library().masw_get_timing(ctx, 1 if reset else 0, ctypes.byref(t)), "masw_get_timing")
    return t.as_dict()


def masw_server_start(ctx, max_layers=0, max_lambda=0, max_grid=0, rounds_per_tick=0, pool_bytes=0,
                      tick_timeout_us=0, search_inertia=0) -> int:
    o = masw_server_opts(max_layers, max_lambda, max_grid, rounds_per_tick, pool_bytes, tick_timeout_us,
                         search_inertia, 0)
    return _check(library().masw_server_start(ctx, ctypes.byref(o)), "masw_server_start")


def masw_server_stop(ctx) -> int:
    return _check(library().masw_server_stop(ctx), "masw_server_stop")


def masw_submit(ctx, c_test, lam, h, alpha, beta, rho, prec: int, flags: int = 0) -> int:
    """Host numpy arrays only (copied before returning); returns the ticket."""
    m = _model_struct(h, alpha, beta, rho)
    t = ctypes.c_uint64()
    _check(library().masw_submit(ctx, _ptr(c_test, np.float64), int(c_test.shape[0]), _ptr(lam, np.float64),
                                 int(lam.shape[0]), ctypes.byref(m), prec, flags, ctypes.byref(t)), "masw_submit")
    return t.value


def _collect(fn, ctx, ticket, extra, C_t, idx, status, c_ref):
    info = masw_request_info()
    rc = fn(ctx, ctypes.c_uint64(ticket), *extra, _ptr(C_t, np.float64), _ptr(idx, np.int32),
            _ptr(status, np.int32), _ptr(c_ref, np.float64), ctypes.byref(info))
    if rc == MASW_EBUSY:
        return None
    _check(rc, fn.__name__)
    return info.as_dict()


def masw_poll(ctx, ticket, C_t, idx, status, c_ref=None):
    """Results into the given host arrays and the request's timing dict, or
    None while the request is unfinished."""
    return _collect(library().masw_poll, ctx, ticket, (), C_t, idx, status, c_ref)


def masw_wait(ctx, ticket, timeout_us, C_t, idx, status, c_ref=None):
    return _collect(library().masw_wait, ctx, ticket, (ctypes.c_int64(int(timeout_us)),), C_t, idx, status, c_ref)


def masw_server_get_stats(ctx) -> dict:
    s = masw_server_stats()
    _check(library().masw_server_get_stats(ctx, ctypes.byref(s)), "masw_server_get_stats")
    return s.as_dict()


# ------------------------------------------------------------ convenience --
def flatten_models(models, lambdas):
    """CSR arrays (layer_off, h, alpha, beta, rho, lambda_off, lam) of a list of
    models (objects with h, alpha, beta, rho arrays) and their wavelengths."""
    n = [int(m.h.shape[0]) for m in models]
    w = [int(np.asarray(l).shape[0]) for l in lambdas]
    layer_off = np.zeros(len(models) + 1, np.int32)
    layer_off[1:] = np.cumsum(n)
    lambda_off = np.zeros(len(models) + 1, np.int32)
    lambda_off[1:] = np.cumsum(w)
    cat = lambda xs: np.ascontiguousarray(np.concatenate(xs) if xs else np.zeros(0), dtype=np.float64)
    return (layer_off, cat([m.h for m in models]), cat([m.alpha for m in models]),
            cat([m.beta for m in models]), cat([m.rho for m in models]), lambda_off,
            cat([np.asarray(l, np.float64) for l in lambdas]))


class PreparedCurve:
    """masw_dispersion_curve (or, with noalloc=True,
    masw_dispersion_curve_noalloc) with its arguments marshalled once, for
    calls repeated on the same buffers (device tensors, or host arrays): each
    call() is the bare C call.  The caller keeps the buffers alive and
    unmoved while the object is used."""

    def __init__(self, ctx, c_test, lam, h, alpha, beta, rho, prec: int, flags: int, stream,
                 C_t, idx, status, c_ref=None, noalloc: bool = False):
        fl = flags | _device_flag(c_test, lam, h, alpha, beta, rho, C_t, idx, status, c_ref)
        self._model = _model_struct(h, alpha, beta, rho)   # kept alive: the C call reads it
        self._keep = (c_test, lam, h, alpha, beta, rho, C_t, idx, status, c_ref)
        lib = library()
        self._fn = lib.masw_dispersion_curve_noalloc if noalloc else lib.masw_dispersion_curve
        self._name = "masw_dispersion_curve_noalloc" if noalloc else "masw_dispersion_curve"
        self._args = (ctx, _ptr(c_test, np.float64), int(c_test.shape[0]), _ptr(lam, np.float64),
                      int(lam.shape[0]), ctypes.byref(self._model), prec, fl,
                      _stream(stream, fl & MASW_DEVICE_PTRS), _ptr(C_t, np.float64), _ptr(idx, np.int32),
                      _ptr(status, np.int32), _ptr(c_ref, np.float64))

    def __call__(self) -> int:
        rc = self._fn(*self._args)
        return rc if rc == MASW_OK else _check(rc, self._name)


class PreparedSignMap:
    """masw_sign_map with its arguments marshalled once (see PreparedCurve)."""

    def __init__(self, ctx, c_test, lam, h, alpha, beta, rho, prec: int, flags: int, stream, sigma,
                 log_abs_det=None):
        fl = flags | _device_flag(c_test, lam, h, alpha, beta, rho, sigma, log_abs_det)
        self._model = _model_struct(h, alpha, beta, rho)
        self._keep = (c_test, lam, h, alpha, beta, rho, sigma, log_abs_det)
        self._fn = library().masw_sign_map
        self._args = (ctx, _ptr(c_test, np.float64), int(c_test.shape[0]), _ptr(lam, np.float64),
                      int(lam.shape[0]), ctypes.byref(self._model), prec, fl,
                      _stream(stream, fl & MASW_DEVICE_PTRS), _ptr(sigma, np.int8), _ptr(log_abs_det, np.float64))

    def __call__(self) -> int:
        rc = self._fn(*self._args)
        return rc if rc == MASW_OK else _check(rc, "masw_sign_map")


class Context:
    """A masw_ctx on one device, with helpers that allocate outputs."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 1 << 30):
        self.ctx = masw_create(device, hbm_budget_bytes)

    def close(self) -> None:
        masw_destroy(self.ctx)
        self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def stats(self) -> dict:
        return masw_get_stats(self.ctx)

    def curve(self, c_test, lam, model, prec=MASW_PREC_FP64, flags=0):
        """Host arrays in, host arrays out: (C_t, idx, status, c_ref)."""
        W = int(np.asarray(lam).shape[0])
        out = (np.empty(W), np.empty(W, np.int32), np.empty(W, np.int32), np.empty(W))
        f64 = lambda x: np.ascontiguousarray(x, dtype=np.float64)
        masw_dispersion_curve(self.ctx, f64(c_test), f64(lam), f64(model.h), f64(model.alpha),
                              f64(model.beta), f64(model.rho), prec, flags, None, *out)
        return out

    def batch(self, c_test, models, lambdas, prec=MASW_PREC_SPLIT, flags=0):
        """Host arrays in, host arrays out, outputs flattened over all wavelengths."""
        arrs = flatten_models(models, lambdas)
        W = int(arrs[-1].shape[0])
        out = (np.empty(W), np.empty(W, np.int32), np.empty(W, np.int32), np.empty(W))
        masw_dispersion_batch(self.ctx, np.ascontiguousarray(c_test, np.float64), *arrs, prec, flags, None, *out)
        return out

    def classify(self, c_test, models, lambdas, idx):
        """Host arrays in, host arrays out: (pick_class, c_sec), flattened over
        all wavelengths, for the bracket indices idx (flattened likewise)."""
        arrs = flatten_models(models, lambdas)
        W = int(arrs[-1].shape[0])
        cls = np.empty(W, np.int32)
        sec = np.empty(W)
        masw_classify_picks(self.ctx, np.ascontiguousarray(c_test, np.float64), *arrs,
                            np.ascontiguousarray(idx, np.int32), 0, None, cls, sec)
        return cls, sec

    def sign_map(self, c_test, lam, model, prec=MASW_PREC_FP64, want_log=True):
        W, n_c = int(np.asarray(lam).shape[0]), int(np.asarray(c_test).shape[0])
        sig = np.empty(W * n_c, np.int8)
        la = np.empty(W * n_c) if want_log else None
        f64 = lambda x: np.ascontiguousarray(x, dtype=np.float64)
        masw_sign_map(self.ctx, f64(c_test), f64(lam), f64(model.h), f64(model.alpha), f64(model.beta),
                      f64(model.rho), prec, 0, None, sig, la)
        return sig.reshape(W, n_c), (la.reshape(W, n_c) if want_log else None)
