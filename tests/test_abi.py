"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/masw.h, and rejects bad arguments on the host (before any
HIP call) with MASW_EINVAL and a message naming the failing argument."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2003_02256_amd as M
import workloads as WL

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "masw.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(masw_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(M.LIB_PATH):
        pytest.fail("libmasw.so is not built: run __graft_entry__.build()")
    return M.library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("masw_create", "masw_destroy", "masw_dispersion_curve", "masw_dispersion_batch",
                 "masw_sign_map", "masw_get_stats", "masw_strerror", "masw_last_error"):
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_strerror_and_version(lib):
    assert M.masw_strerror(M.MASW_OK) == "success"
    assert M.masw_strerror(M.MASW_EINVAL) == "invalid argument"
    assert M.masw_strerror(12345) == "unknown error code"
    assert "gfx950" in M.masw_version()


def _call_curve(c, lam, m, C=None, prec=M.MASW_PREC_FP64, flags=0, ctx=None):
    W = lam.shape[0]
    out = (np.empty(W), np.empty(W, np.int32), np.empty(W, np.int32), np.empty(W))
    mod = M._model_struct(m.h, m.alpha, m.beta, m.rho)
    rc = M.library().masw_dispersion_curve(ctx, M._ptr(c, np.float64), int(c.shape[0]), M._ptr(lam, np.float64),
                                           W, ctypes.byref(mod), prec, flags, None,
                                           *[M._ptr(o, o.dtype.type) for o in out])
    return rc, M.masw_last_error()


def _good():
    wl = WL.two_layer_case()
    return wl.c_test.copy(), wl.lambdas[0].copy(), wl.models[0].copy()


def test_valid_arguments_reach_the_context_check(lib):
    c, lam, m = _good()
    rc, msg = _call_curve(c, lam, m)
    assert rc == M.MASW_EINVAL and "ctx" in msg


@pytest.mark.parametrize("mutate,needle", [
    (lambda c, l, m: c.__setitem__(5, c[4]), "strictly increasing"),
    (lambda c, l, m: c.__setitem__(0, np.nan), "finite"),
    (lambda c, l, m: c.__setitem__(0, -1.0), "finite"),
    (lambda c, l, m: l.__setitem__(3, 0.0), "lambda"),
    (lambda c, l, m: l.__setitem__(3, np.inf), "lambda"),
    (lambda c, l, m: m.h.__setitem__(0, -2.0), "h must"),
    (lambda c, l, m: m.alpha.__setitem__(1, m.beta[1]), "alpha must exceed beta"),
    (lambda c, l, m: m.beta.__setitem__(2, np.nan), "finite"),
    (lambda c, l, m: m.rho.__setitem__(0, 0.0), "finite and > 0"),
])
def test_host_validation_rejects(lib, mutate, needle):
    c, lam, m = _good()
    mutate(c, lam, m)
    rc, msg = _call_curve(c, lam, m)
    assert rc == M.MASW_EINVAL
    assert needle in msg


def test_short_grid_rejected(lib):
    c, lam, m = _good()
    rc, msg = _call_curve(c[:1].copy(), lam, m)
    assert rc == M.MASW_EINVAL and "n_c" in msg


def test_bad_precision_and_flags(lib):
    c, lam, m = _good()
    rc, msg = _call_curve(c, lam, m, prec=7)
    assert rc == M.MASW_EINVAL and "prec" in msg
    rc, msg = _call_curve(c, lam, m, flags=0x80)
    assert rc == M.MASW_EINVAL and "flags" in msg


def test_inertia_search_needs_fp64(lib):
    c, lam, m = _good()
    rc, msg = _call_curve(c, lam, m, prec=M.MASW_PREC_SPLIT, flags=M.MASW_SEARCH_INERTIA)
    assert rc == M.MASW_EINVAL and "MASW_SEARCH_INERTIA" in msg
    rc, msg = _call_curve(c, lam, m, prec=M.MASW_PREC_FP64, flags=M.MASW_SEARCH_INERTIA)
    assert rc == M.MASW_EINVAL and "ctx" in msg      # accepted up to the context check


def test_create_without_device_reports_edevice(lib):
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except Exception:
        pass
    ctx = ctypes.c_void_p()
    rc = lib.masw_create(0, 0, ctypes.byref(ctx))
    assert rc == M.MASW_EDEVICE and not ctx.value


def test_batch_offsets_validated(lib):
    wl = WL.batch_case(n_models=3, seed=11)
    arrs = list(M.flatten_models(wl.models, wl.lambdas))
    arrs[0] = arrs[0].copy()
    arrs[0][1], arrs[0][2] = arrs[0][2], arrs[0][1]   # layer_off no longer non-decreasing
    W = arrs[-1].shape[0]
    out = (np.empty(W), np.empty(W, np.int32), np.empty(W, np.int32), np.empty(W))
    with pytest.raises(M.MaswError) as e:
        M.masw_dispersion_batch(None, wl.c_test, *arrs, M.MASW_PREC_SPLIT, 0, None, *out)
    assert e.value.code == M.MASW_EINVAL


def test_sign_map_validates_on_host(lib):
    c, lam, m = _good()
    m.alpha[0] = 10.0
    sig = np.empty(lam.shape[0] * c.shape[0], np.int8)
    with pytest.raises(M.MaswError) as e:
        M.masw_sign_map(None, c, lam, m.h, m.alpha, m.beta, m.rho, M.MASW_PREC_FP64, 0, None, sig)
    assert e.value.code == M.MASW_EINVAL and "alpha" in str(e.value)


def test_marshal_rejects_wrong_dtype(lib):
    c, lam, m = _good()
    with pytest.raises(M.MaswError):
        M._ptr(c.astype(np.float32), np.float64)


def test_serving_calls_validate_without_a_device(lib):
    c, lam, m = _good()
    mod = M._model_struct(m.h, m.alpha, m.beta, m.rho)
    t = ctypes.c_uint64()
    rc = lib.masw_submit(None, M._ptr(c, np.float64), int(c.shape[0]), M._ptr(lam, np.float64), int(lam.shape[0]),
                         ctypes.byref(mod), M.MASW_PREC_FP64, 0, ctypes.byref(t))
    assert rc == M.MASW_EINVAL and "ctx" in M.masw_last_error()
    c2 = c.copy()
    c2[3] = c2[2]
    rc = lib.masw_submit(None, M._ptr(c2, np.float64), int(c2.shape[0]), M._ptr(lam, np.float64),
                         int(lam.shape[0]), ctypes.byref(mod), M.MASW_PREC_FP64, 0, ctypes.byref(t))
    assert rc == M.MASW_EINVAL and "increasing" in M.masw_last_error()
    for bad in (M.MASW_DEVICE_PTRS, M.MASW_SEARCH_INERTIA, 0x100):
        rc = lib.masw_submit(None, M._ptr(c, np.float64), int(c.shape[0]), M._ptr(lam, np.float64),
                             int(lam.shape[0]), ctypes.byref(mod), M.MASW_PREC_FP64, bad, ctypes.byref(t))
        assert rc == M.MASW_EINVAL and "flags" in M.masw_last_error()
    assert lib.masw_server_start(None, None) == M.MASW_EINVAL
    assert lib.masw_server_stop(None) == M.MASW_EINVAL
    info = M.masw_request_info()
    assert lib.masw_poll(None, 1, None, None, None, None, ctypes.byref(info)) == M.MASW_EINVAL


def test_misfit_validates_on_host(lib):
    off = np.array([0, 2, 3], np.int32)
    ct = np.array([100.0, 200.0, 300.0])
    out = np.empty(2)
    with pytest.raises(M.MaswError) as e:
        M.masw_misfit(None, off, ct, np.array([100.0, 0.0, 300.0]), 0, None, out)
    assert e.value.code == M.MASW_EINVAL and "C_e" in str(e.value)
    with pytest.raises(M.MaswError) as e:
        M.masw_misfit(None, np.array([0, 3, 2], np.int32), ct, ct, 0, None, out)
    assert e.value.code == M.MASW_EINVAL and "non-decreasing" in str(e.value)
    with pytest.raises(M.MaswError) as e:
        M.masw_misfit(None, off, ct, ct, 0, None, out)
    assert e.value.code == M.MASW_EINVAL and "ctx" in str(e.value)


def test_timing_rejects_null_arguments(lib):
    out = M.masw_timing()
    assert lib.masw_get_timing(None, 0, ctypes.byref(out)) == M.MASW_EINVAL
    assert lib.masw_get_timing(None, 1, None) == M.MASW_EINVAL


def test_classify_validates_on_host(lib):
    wl = WL.two_layer_case()
    m, lam, c = wl.models[0], wl.lambdas[0][:3], wl.c_test
    idx = np.array([10, 20, 30], np.int32)
    cls, sec = np.empty(3, np.int32), np.empty(3)

    def call(models=(m,), lams=(lam,), grid=c, flags=0):
        arrs = M.flatten_models(list(models), list(lams))
        M.masw_classify_picks(None, grid, *arrs, idx, flags, None, cls, sec)

    bad = WL.Model(m.h.copy(), m.beta.copy(), m.beta.copy(), m.rho.copy())  # alpha == beta
    for kwargs, msg in ((dict(models=(bad,)), "alpha must exceed beta"),
                        (dict(lams=(np.array([1.0, -2.0, 3.0]),)), "lambda"),
                        (dict(grid=c[::-1].copy()), "increasing"),
                        (dict(flags=0x80), "flags"),
                        (dict(), "ctx")):
        with pytest.raises(M.MaswError) as e:
            call(**kwargs)
        assert e.value.code == M.MASW_EINVAL and msg in str(e.value), (kwargs, str(e.value))


def test_opts_validate_on_host(lib):
    for kwargs, msg in ((dict(refine_rel_tol=1e-16), "refine_rel_tol"), (dict(refine_rel_tol=0.5), "refine_rel_tol"),
                        (dict(noise_threshold=2.0), "noise_threshold"), (dict(noise_threshold=-1.0), "noise_threshold"),
                        (dict(waves_per_item=3), "waves_per_item"), (dict(shared_window=2000), "shared_window"),
                        (dict(shared_window=-2), "shared_window"), (dict(first_item_priority=1), "first_item_priority"),
                        (dict(timing_events=2), "timing_events"), (dict(), "ctx")):
        with pytest.raises(M.MaswError) as e:
            M.masw_set_opts(None, **kwargs)
        assert e.value.code == M.MASW_EINVAL and msg in str(e.value), (kwargs, str(e.value))
    out = M.masw_opts()
    assert lib.masw_get_opts(None, ctypes.byref(out)) == M.MASW_EINVAL


def test_noalloc_entry_point_validates_on_host(lib):
    # the no-alloc variant takes device pointers only, and checks sizes and
    # flags before it looks at the context
    c, lam, m = _good()
    W = lam.shape[0]
    out = (np.empty(W), np.empty(W, np.int32), np.empty(W, np.int32), np.empty(W))
    mod = M._model_struct(m.h, m.alpha, m.beta, m.rho)

    def call(flags, n_c=None, prec=M.MASW_PREC_FP64):
        rc = lib.masw_dispersion_curve_noalloc(None, M._ptr(c, np.float64), int(c.shape[0] if n_c is None else n_c),
                                               M._ptr(lam, np.float64), W, ctypes.byref(mod), prec, flags, None,
                                               *[M._ptr(o, o.dtype.type) for o in out])
        return rc, M.masw_last_error()

    rc, msg = call(0)
    assert rc == M.MASW_EINVAL and "MASW_DEVICE_PTRS" in msg
    rc, msg = call(M.MASW_DEVICE_PTRS, n_c=1)
    assert rc == M.MASW_EINVAL and "n_c" in msg
    rc, msg = call(M.MASW_DEVICE_PTRS, prec=5)
    assert rc == M.MASW_EINVAL and "prec" in msg
    rc, msg = call(M.MASW_DEVICE_PTRS | 0x40)
    assert rc == M.MASW_EINVAL and "flags" in msg
    rc, msg = call(M.MASW_DEVICE_PTRS)
    assert rc == M.MASW_EINVAL and "ctx" in msg
