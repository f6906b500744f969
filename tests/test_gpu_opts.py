"""Context options (masw_set_opts / masw_get_opts) on the device: the
refinement tolerance against the oracle's bisection to the same tolerance,
schedule options that must leave every result bitwise unchanged, the noise
threshold against the oracle's band test, and the served path taking the
context's tolerance."""
import numpy as np
import pytest

import oracle as O
import paper_2003_02256_amd as M
import workloads as WL

pytestmark = pytest.mark.gpu


@pytest.fixture
def ctx(gpu):
    c = M.Context(0, 1 << 30)
    yield c
    c.close()


def test_defaults_and_round_trip(ctx):
    assert M.masw_get_opts(ctx.ctx) == {"refine_rel_tol": 1e-9, "noise_threshold": 1e-2, "waves_per_item": 0,
                                         "shared_window": 8, "first_item_priority": 0, "timing_events": 0}
    M.masw_set_opts(ctx.ctx, refine_rel_tol=1e-12, noise_threshold=0.5, waves_per_item=4, shared_window=-1,
                    first_item_priority=-1, timing_events=1)
    assert M.masw_get_opts(ctx.ctx) == {"refine_rel_tol": 1e-12, "noise_threshold": 0.5, "waves_per_item": 4,
                                         "shared_window": -1, "first_item_priority": -1, "timing_events": 1}
    M.masw_set_opts(ctx.ctx)                      # defaults again
    assert M.masw_get_opts(ctx.ctx)["refine_rel_tol"] == 1e-9


def test_refine_tolerance_matches_the_oracle(ctx):
    wl = WL.two_layer_case()
    m, lam, c = wl.models[0], wl.lambdas[0], wl.c_test
    M.masw_set_opts(ctx.ctx, refine_rel_tol=1e-13)
    ct, idx, st, cr = ctx.curve(c, lam, m, prec=M.MASW_PREC_FP64)
    for w in range(0, len(lam), 3):
        k = 2 * np.pi / lam[w]
        want = O.bisect_root(k, float(c[idx[w] - 1]), float(c[idx[w]]), m, rel_tol=1e-13)
        assert abs(cr[w] - want) <= 2e-13 * want, (w, cr[w], want)


def test_schedule_options_leave_results_unchanged(ctx):
    wl = WL.fine_scale_case()
    m, lam, c = wl.models[0], wl.lambdas[0][::10], wl.c_test
    base = ctx.curve(c, lam, m, prec=M.MASW_PREC_FP64)
    for kw in (dict(waves_per_item=2), dict(waves_per_item=16), dict(shared_window=-1),
               dict(shared_window=1, first_item_priority=-1), dict(timing_events=1)):
        M.masw_set_opts(ctx.ctx, **kw)
        got = ctx.curve(c, lam, m, prec=M.MASW_PREC_FP64)
        for a, b in zip(base, got):
            assert np.array_equal(a, b, equal_nan=True), kw


def test_noise_threshold_reaches_the_band_test(ctx):
    wl = WL.two_layer_case()
    m, lam, c = wl.models[0], wl.lambdas[0][:6], wl.c_test
    # at threshold 1e-20 the band is cond_2 >= 1e-20 / (6 2^-53) ~ 1.5e-5: every grid point
    M.masw_set_opts(ctx.ctx, noise_threshold=1e-20)
    ct, idx, st, cr = ctx.curve(c, lam, m, prec=M.MASW_PREC_FP64, flags=M.MASW_CHECK_NOISE)
    for w in range(len(lam)):
        want = any(O.in_noise_band(lam[w], c[i], m, threshold=1e-20) for i in (idx[w] - 1, idx[w]))
        assert bool(st[w] & M.MASW_FLAG_NOISE) == want
    assert all(st & M.MASW_FLAG_NOISE)


def test_server_takes_the_tolerance_at_start(ctx):
    wl = WL.two_layer_case()
    m, lam, c = wl.models[0], wl.lambdas[0], wl.c_test
    M.masw_set_opts(ctx.ctx, refine_rel_tol=1e-12)
    want = ctx.curve(c, lam, m, prec=M.MASW_PREC_FP64)
    M.masw_server_start(ctx.ctx)
    f = lambda x: np.ascontiguousarray(x, np.float64)
    t = M.masw_submit(ctx.ctx, f(c), f(lam), f(m.h), f(m.alpha), f(m.beta), f(m.rho), M.MASW_PREC_FP64)
    W = len(lam)
    out = (np.empty(W), np.empty(W, np.int32), np.empty(W, np.int32), np.empty(W))
    M.masw_wait(ctx.ctx, t, 60_000_000, *out)
    M.masw_server_stop(ctx.ctx)
    for a, b in zip(want, out):
        assert np.array_equal(a, b)
