"""The FP64 noise-band flag (MASW_CHECK_NOISE -> MASW_FLAG_NOISE), through the
C ABI, against the oracle's definition (oracle.in_noise_band: cond_2 of the
dense matrix from an SVD, times 2(N+1) 2^-53, at least 1e-2) at the same
bracket points.

The device decides the same inequality from eigenvalue counts of the block
elimination (the matrix is real symmetric below the half-space's S
velocity), so the two agree except at points whose condition number equals
the threshold to about 12 digits.  Grids are built so that a bracket end
sits at a chosen distance from a root, from the root itself (in the band) to
1e-9 relative (outside it).
"""
import math

import numpy as np
import pytest

import oracle as O
import paper_2003_02256_amd as M
import workloads as WL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu):
    c = M.Context(0, 256 << 20)
    yield c
    c.close()


def _exact_root(lam, lo, hi, model):
    # bisection on the oracle's sign down to adjacent doubles
    return O.bisect_root(2 * math.pi / lam, lo, hi, model, rel_tol=0.0)


def _band_at(lam, c, model):
    return c < model.beta[model.n_layers] and O.in_noise_band(lam, c, model)


def _check(ctx, c_test, lam, model):
    """Device picks and flags with MASW_CHECK_NOISE against the oracle's band
    test at the device's bracket points; returns the device flags."""
    ct, idx, st, cr = ctx.curve(c_test, lam, model, prec=M.MASW_PREC_FP64, flags=M.MASW_CHECK_NOISE)
    ct0, idx0, st0, cr0 = ctx.curve(c_test, lam, model, prec=M.MASW_PREC_FP64)
    assert np.array_equal(idx, idx0)                           # the flag changes no pick
    assert np.array_equal(st & ~M.MASW_FLAG_NOISE, st0)
    flags = []
    for w in range(len(lam)):
        if idx[w] < 1:
            assert not st[w] & M.MASW_FLAG_NOISE
            flags.append(False)
            continue
        want = _band_at(lam[w], c_test[idx[w] - 1], model) or _band_at(lam[w], c_test[idx[w]], model)
        got = bool(st[w] & M.MASW_FLAG_NOISE)
        assert got == want, (w, lam[w], idx[w], got, want)
        flags.append(got)
    return flags


def test_no_flag_on_the_two_layer_case(ctx):
    wl = WL.two_layer_case()
    flags = _check(ctx, wl.c_test, wl.lambdas[0], wl.models[0])
    assert not any(flags)
    want = O.dispersion_curve(wl.lambdas[0], wl.c_test, wl.models[0], check_noise=True)
    assert not any(p.status & O.FLAG_NOISE for p in want)


@pytest.mark.parametrize("case", ["halfspace", "layered"])
def test_flag_at_and_near_a_root(ctx, case):
    if case == "halfspace":
        model = WL.Model(np.zeros(0), np.array([700.0]), np.array([400.0]), np.array([2000.0]))
        lam = 3.0
    else:
        model = WL.fine_scale_case().models[0]
        lam = 7.0
    coarse = WL.uniform_grid(50.0, 0.5, 2000)
    p = O.dispersion_point(lam, coarse, model, refine=False)
    assert p.status == O.STATUS_FOUND
    root = _exact_root(lam, float(coarse[p.idx - 1]), float(coarse[p.idx]), model)
    # grids whose point 100 sits at root (1 + d): from in the band to well outside
    seen = []
    for d in (0.0, 1e-15, 1e-14, 1e-13, 1e-12, 1e-11, 1e-9):
        c0 = root * (1.0 + d)
        c_test = c0 + 0.01 * (np.arange(300) - 100.0)
        flags = _check(ctx, c_test, np.array([lam]), model)
        seen.append(flags[0])
    print(f"{case}: flagged at relative distance 0, 1e-15 .. 1e-11, 1e-9 from the root: {seen}", flush=True)
    assert seen[0] and not seen[-1], seen       # the root itself is in the band, 1e-9 away is not


def test_served_requests_carry_the_flag(ctx):
    # requests submitted with MASW_CHECK_NOISE get the same flag as the
    # synchronous call (and MASW_NO_REFINE the same NaN roots), in a mix of
    # flagged and unflagged requests sharing ticks
    model = WL.fine_scale_case().models[0]
    lam = 7.0
    coarse = WL.uniform_grid(50.0, 0.5, 2000)
    p = O.dispersion_point(lam, coarse, model, refine=False)
    root = _exact_root(lam, float(coarse[p.idx - 1]), float(coarse[p.idx]), model)
    grids = [root * (1.0 + d) + 0.01 * (np.arange(300) - 100.0) for d in (0.0, 1e-13, 1e-9)]
    lams = np.array([lam, 5.0, 9.0])
    M.masw_server_start(ctx.ctx, rounds_per_tick=1)
    try:
        jobs = []
        for g in grids:
            for prec in (M.MASW_PREC_FP64, M.MASW_PREC_SPLIT):
                for flags in (M.MASW_CHECK_NOISE, 0, M.MASW_CHECK_NOISE | M.MASW_NO_REFINE):
                    t = M.masw_submit(ctx.ctx, g, lams, model.h, model.alpha, model.beta, model.rho, prec, flags)
                    jobs.append((t, g, prec, flags))
        got_flags = []
        for t, g, prec, flags in jobs:
            o = (np.empty(3), np.empty(3, np.int32), np.empty(3, np.int32), np.empty(3))
            M.masw_wait(ctx.ctx, t, 60_000_000, *o)
            sync = ctx.curve(g, lams, model, prec=prec, flags=flags & M.MASW_CHECK_NOISE)
            np.testing.assert_array_equal(o[1], sync[1])
            np.testing.assert_array_equal(o[2], sync[2])
            np.testing.assert_array_equal(o[0], sync[0])
            if flags & M.MASW_NO_REFINE:
                assert np.all(np.isnan(o[3]))
            else:
                np.testing.assert_array_equal(o[3], sync[3])
            if flags & M.MASW_CHECK_NOISE:
                got_flags.append(bool(o[2][0] & M.MASW_FLAG_NOISE))
            else:
                assert not np.any(o[2] & M.MASW_FLAG_NOISE)
        # the grid point at the root is in the band, 1e-9 away is not
        assert got_flags[0] and not got_flags[-1], got_flags
        with pytest.raises(M.MaswError) as e:
            M.masw_submit(ctx.ctx, grids[0], lams, model.h, model.alpha, model.beta, model.rho,
                          M.MASW_PREC_FP64, M.MASW_SEARCH_INERTIA)
        assert e.value.code == M.MASW_EINVAL
    finally:
        M.masw_server_stop(ctx.ctx)
