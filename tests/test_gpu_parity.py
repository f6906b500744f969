"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Picks must equal the oracle's grid index exactly, unless one of the bracket
points of either pick lies in the FP64 noise band (cond_2(K) 2(N+1) 2^-53 >=
1e-2); such wavelengths are counted as NOISE and reported, not compared.
Refined roots must agree to 1e-6 relative (both sides bisect to a bracket of
1e-9 c, so the observed gap is far smaller).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import paper_2003_02256_amd as M
import workloads as WL

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
REL_TOL = 1e-6


@pytest.fixture(scope="module")
def torch_dev(gpu):
    import torch
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def ctx(gpu):
    c = M.Context(0, 2 << 30)
    yield c
    c.close()


def dev_curve(torch_dev, ctx, c_test, lam, model, prec, flags=0):
    torch, dev = torch_dev
    t = lambda x: torch.as_tensor(np.ascontiguousarray(x, np.float64), device=dev)
    W = len(lam)
    out = (torch.empty(W, dtype=torch.float64, device=dev), torch.empty(W, dtype=torch.int32, device=dev),
           torch.empty(W, dtype=torch.int32, device=dev), torch.empty(W, dtype=torch.float64, device=dev))
    M.masw_dispersion_curve(ctx.ctx, t(c_test), t(lam), t(model.h), t(model.alpha), t(model.beta),
                            t(model.rho), prec, flags, None, *out)
    torch.cuda.synchronize()
    return tuple(o.cpu().numpy() for o in out)


def dev_batch(torch_dev, ctx, c_test, models, lambdas, prec, flags=0):
    torch, dev = torch_dev
    arrs = M.flatten_models(models, lambdas)
    td = [torch.as_tensor(a, device=dev) for a in arrs]
    W = int(arrs[-1].shape[0])
    out = (torch.empty(W, dtype=torch.float64, device=dev), torch.empty(W, dtype=torch.int32, device=dev),
           torch.empty(W, dtype=torch.int32, device=dev), torch.empty(W, dtype=torch.float64, device=dev))
    M.masw_dispersion_batch(ctx.ctx, torch.as_tensor(c_test, device=dev), *td, prec, flags, None, *out)
    torch.cuda.synchronize()
    return tuple(o.cpu().numpy() for o in out)


def compare(name, got, want_idx, want_status, want_cref, lambdas, c_test, model):
    """Assert parity; return (n_compared, n_noise, max_rel_root_err)."""
    ct, idx, st, cr = got
    noise, errs, bad = [], [], []
    for w in range(len(want_idx)):
        wi = int(want_idx[w])
        if idx[w] != wi:
            pts = {p for i in (int(idx[w]), wi) if i > 0 for p in (i - 1, i)}
            if any(O.in_noise_band(float(lambdas[w]), float(c_test[p]), model) for p in pts):
                noise.append(w)
            else:
                bad.append((w, int(idx[w]), wi))
            continue
        assert st[w] == want_status[w], (name, w, st[w], want_status[w])
        if wi < 0:
            assert math.isnan(ct[w]) and math.isnan(cr[w])
            continue
        assert ct[w] == c_test[wi]
        errs.append(abs(cr[w] - want_cref[w]) / want_cref[w])
    assert not bad, f"{name}: index mismatches outside the noise band (w, gpu, oracle): {bad[:10]}"
    mx = max(errs) if errs else 0.0
    print(f"{name}: {len(errs)} compared, {len(noise)} noise, max rel root err {mx:.3e}", flush=True)
    assert mx <= REL_TOL
    return len(errs), len(noise), mx


def oracle_curve(lambdas, c_test, model):
    pts = O.dispersion_curve(lambdas, c_test, model)
    return ([p.idx for p in pts], [p.status for p in pts], [p.c_ref for p in pts])


# ------------------------------------------------------------ two-layer case --
@pytest.mark.parametrize("prec", [M.MASW_PREC_FP64, M.MASW_PREC_SPLIT])
def test_two_layer_case_matches_oracle(torch_dev, ctx, prec):
    wl = WL.two_layer_case()
    m, lam, c = wl.models[0], wl.lambdas[0], wl.c_test
    got = dev_curve(torch_dev, ctx, c, lam, m, prec)
    n, n_noise, _ = compare(f"two-layer prec={prec}", got, *oracle_curve(lam, c, m), lam, c, m)
    assert n == 30 and n_noise == 0
    s = ctx.stats()
    assert s["useful_evals"] == 8951
    assert s["n_lambda"] == 30


def test_host_and_device_pointer_paths_agree(torch_dev, ctx):
    wl = WL.two_layer_case()
    m, lam, c = wl.models[0], wl.lambdas[0], wl.c_test
    for prec in (M.MASW_PREC_FP64, M.MASW_PREC_SPLIT):
        a = ctx.curve(c, lam, m, prec)
        b = dev_curve(torch_dev, ctx, c, lam, m, prec)
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)


# ------------------------------------------------------------------ sign map --
def test_sign_map_fp64_matches_dense_lu(gpu, ctx):
    wl = WL.two_layer_case()
    m, lam, c = wl.models[0], wl.lambdas[0], wl.c_test
    sig, la = ctx.sign_map(c, lam, m, M.MASW_PREC_FP64)
    osig, ola = O.sign_map(lam, c, m)
    assert np.array_equal(sig, osig)
    # away from sign changes log|det| agrees to a relative 1e-10 of det
    near = np.zeros_like(osig, bool)
    ch = np.nonzero(osig[:, 1:] != osig[:, :-1])
    for w, i in zip(*ch):
        near[w, max(0, i - 2):i + 4] = True
    d = np.abs(la - ola)[~near]
    print(f"sign map two-layer: max |d ln|det|| = {d.max():.3e}", flush=True)
    assert d.max() < 1e-9


def test_sign_map_fp64_twenty_layers(gpu, ctx):
    wl = WL.fine_scale_case()
    m = wl.models[0]
    lam = wl.lambdas[0][::100].copy()
    c = wl.c_test[::97].copy()                      # 1186 points over 50-1200 m/s
    sig, la = ctx.sign_map(c, lam, m, M.MASW_PREC_FP64)
    osig, ola = O.sign_map(lam, c, m)
    mism = np.argwhere(sig != osig)
    for w, i in mism:
        assert O.in_noise_band(float(lam[w]), float(c[i]), m), (w, i, sig[w, i], osig[w, i])
    fin = np.isfinite(ola) & (sig == osig)
    rel = np.abs(la - ola)[fin]
    print(f"sign map N=20: {len(mism)} sign mismatches (all in noise band), "
          f"median |d ln|det|| {np.median(rel):.2e}", flush=True)
    assert np.median(rel) < 1e-8


def test_sign_map_fp32_close_to_fp64(gpu, ctx):
    wl = WL.two_layer_case()
    m, lam, c = wl.models[0], wl.lambdas[0], wl.c_test
    s64, _ = ctx.sign_map(c, lam, m, M.MASW_PREC_FP64, want_log=False)
    s32, _ = ctx.sign_map(c, lam, m, M.MASW_PREC_SPLIT, want_log=False)
    bad = np.argwhere(s32 != s64)
    print(f"FP32 sign map: {len(bad)} of {s64.size} signs differ from FP64", flush=True)
    assert len(bad) <= s64.size // 1000


# ------------------------------------------------------------------ edge cases --
def test_homogeneous_halfspace_root(torch_dev, ctx):
    beta = 400.0
    m = WL.Model(np.zeros(0), np.array([math.sqrt(3) * beta]), np.array([beta]), np.array([2000.0]))
    c = WL.uniform_grid(300.0, 0.01, 10001)
    lam = np.array([0.5, 5.0, 50.0])
    cR = beta * math.sqrt(2 - 2 / math.sqrt(3))
    for prec in (M.MASW_PREC_FP64, M.MASW_PREC_SPLIT):
        ct, idx, st, cr = dev_curve(torch_dev, ctx, c, lam, m, prec)
        assert np.all(st == 0)
        assert np.all(c[idx - 1] < cR) and np.all(cR <= c[idx])
        assert np.max(np.abs(cr - cR) / cR) < 1e-8


def test_not_found_and_tiny_grids(torch_dev, ctx):
    wl = WL.two_layer_case()
    m = wl.models[0]
    lam = np.array([1.0, 40.0])
    for prec in (M.MASW_PREC_FP64, M.MASW_PREC_SPLIT):
        c = WL.uniform_grid(50.0, 0.5, 100)     # entirely below every root
        ct, idx, st, cr = dev_curve(torch_dev, ctx, c, lam, m, prec)
        assert np.all(idx == -1) and np.all(st == M.MASW_STATUS_NOT_FOUND)
        assert np.all(np.isnan(ct)) and np.all(np.isnan(cr))
        c2 = np.array([137.0, 139.0])           # n_c = 2, root of lambda = 1 inside
        ct, idx, st, cr = dev_curve(torch_dev, ctx, c2, np.array([1.0]), m, prec)
        p = O.dispersion_point(1.0, c2, m)
        assert idx[0] == p.idx == 1 and abs(cr[0] - p.c_ref) < 1e-6 * p.c_ref


@pytest.mark.parametrize("n_c", [65, 127, 129, 300, 513, 1000, 1537])
def test_ragged_grid_lengths(torch_dev, ctx, n_c):
    # grid lengths around multiples of 64 and of the multi-wavefront rounds
    wl = WL.two_layer_case()
    m = wl.models[0]
    c = WL.uniform_grid(130.0, 190.0 / n_c, n_c)
    lam = wl.lambdas[0]
    want = oracle_curve(lam, c, m)
    for prec in (M.MASW_PREC_FP64, M.MASW_PREC_SPLIT):
        compare(f"ragged n_c={n_c} prec={prec}", dev_curve(torch_dev, ctx, c, lam, m, prec), *want, lam, c, m)


def test_empty_wavelength_list(torch_dev, ctx):
    wl = WL.two_layer_case()
    got = dev_curve(torch_dev, ctx, wl.c_test, np.zeros(0), wl.models[0], M.MASW_PREC_FP64)
    assert all(g.shape == (0,) for g in got)


def test_device_side_validation_marks_invalid(torch_dev, ctx):
    wl = WL.two_layer_case()
    m = wl.models[0].copy()
    m.alpha[1] = 0.5 * m.beta[1]                  # alpha < beta: invalid
    ct, idx, st, cr = dev_curve(torch_dev, ctx, wl.c_test, wl.lambdas[0], m, M.MASW_PREC_FP64)
    assert np.all(st == M.MASW_STATUS_INVALID) and np.all(idx == -1)
    c = wl.c_test.copy()
    c[10] = c[9]                                  # grid not strictly increasing
    ct, idx, st, cr = dev_curve(torch_dev, ctx, c, wl.lambdas[0], wl.models[0], M.MASW_PREC_SPLIT)
    assert np.all(st == M.MASW_STATUS_INVALID)
    lam = wl.lambdas[0].copy()
    lam[3] = -1.0                                 # one bad wavelength only
    ct, idx, st, cr = dev_curve(torch_dev, ctx, wl.c_test, lam, wl.models[0], M.MASW_PREC_FP64)
    assert st[3] == M.MASW_STATUS_INVALID and np.all(np.delete(st, 3) == 0)


def test_split_on_short_grids_runs_the_fp64_walk(torch_dev, ctx):
    # a split call on a grid of fewer than MASW_SPLIT_MIN_GRID points runs as
    # the FP64 walk (bitwise its outputs) and says so; from that size on it
    # sweeps in FP32, with the same picks
    wl = WL.two_layer_case()
    m, lam = wl.models[0], wl.lambdas[0]
    for n, as_fp64 in ((801, 1), (1024, 1), (1025, 0), (1601, 0)):
        c = WL.uniform_grid(50.0, 400.0 / (n - 1), n)
        want = dev_curve(torch_dev, ctx, c, lam, m, M.MASW_PREC_FP64)
        assert M.masw_get_stats(ctx.ctx)["split_as_fp64"] == 0
        got = dev_curve(torch_dev, ctx, c, lam, m, M.MASW_PREC_SPLIT)
        st = M.masw_get_stats(ctx.ctx)
        assert st["split_as_fp64"] == as_fp64, n
        if as_fp64:
            for x, y in zip(got, want):
                np.testing.assert_array_equal(x, y, err_msg=f"n_c {n}")
        else:
            np.testing.assert_array_equal(got[1], want[1], err_msg=f"n_c {n}")
            assert st["check_evals"] > 0


def test_fused_small_launches_equal_staged_launches(torch_dev, ctx):
    # Small single-curve launches stage the model, grid and wavelengths inside
    # the sweep kernel (one launch); with MASW_FUSED_SMALL=0 a context stages
    # them in a launch of their own.  Outputs must be equal bit for bit, for
    # both precisions, with and without refinement, at the limits of the fused
    # launch (64 layers, 2048 grid points, 1024 wavelengths), on a bare
    # half-space, and on inputs the device checks reject.
    os.environ["MASW_FUSED_SMALL"] = "0"
    try:
        staged = M.Context(0, 1 << 30)
    finally:
        del os.environ["MASW_FUSED_SMALL"]
    rng = np.random.Generator(np.random.PCG64(31))
    wl = WL.two_layer_case()
    two, lam2, c2 = wl.models[0], wl.lambdas[0], wl.c_test
    uni = WL.uniform_case(238.0, 100)
    deep = WL.increasing_profile(rng, 64)
    c_deep = WL.uniform_grid(60.0, 0.25, 2048)
    hs = WL.Model(np.zeros(0), np.array([math.sqrt(3) * 400.0]), np.array([400.0]), np.array([2000.0]))
    bad_model = two.copy()
    bad_model.alpha[1] = 0.5 * bad_model.beta[1]
    bad_grid = c2.copy()
    bad_grid[10] = bad_grid[9]
    bad_lam = lam2.copy()
    bad_lam[3] = -1.0
    cases = [("two-layer", c2, lam2, two), ("uniform", uni.c_test, uni.lambdas[0], uni.models[0]),
             ("64 layers, 2048 points", c_deep, WL.log_spaced(1.0, 120.0, 30), deep),
             ("1024 wavelengths", WL.uniform_grid(50.0, 1.0, 400), WL.log_spaced(0.5, 60.0, 1024), two),
             ("two points, one wavelength", c2[:2], lam2[:1], two),
             ("half-space", WL.uniform_grid(300.0, 0.5, 300), np.array([1.0, 10.0]), hs),
             ("invalid model", c2, lam2, bad_model), ("invalid grid", bad_grid, lam2, two),
             ("one invalid wavelength", c2, bad_lam, two)]
    try:
        for name, c, lam, m in cases:
            for prec in (M.MASW_PREC_FP64, M.MASW_PREC_SPLIT):
                for flags in (0, M.MASW_NO_REFINE):
                    got = dev_curve(torch_dev, ctx, c, lam, m, prec, flags)
                    assert M.masw_get_stats(ctx.ctx)["fused_staging"] == 1, name
                    want = dev_curve(torch_dev, staged, c, lam, m, prec, flags)
                    assert M.masw_get_stats(staged.ctx)["fused_staging"] == 0, name
                    for x, y in zip(got, want):
                        np.testing.assert_array_equal(x, y, err_msg=f"{name} prec {prec} flags {flags}")
            print(f"fused = staged: {name}", flush=True)
        # and the fused launch's picks against the oracle on the two-layer case
        idx, st, cr = oracle_curve(lam2, c2, two)
        compare("fused two-layer", dev_curve(torch_dev, ctx, c2, lam2, two, M.MASW_PREC_SPLIT), idx, st, cr,
                lam2, c2, two)
    finally:
        staged.close()


def test_many_layers(torch_dev, ctx):
    rng = np.random.Generator(np.random.PCG64(21))
    m = WL.increasing_profile(rng, 120)
    c = WL.uniform_grid(100.0, 0.25, 1200)
    lam = np.array([1.0, 3.0, 9.0])
    want = oracle_curve(lam, c, m)
    for prec in (M.MASW_PREC_FP64, M.MASW_PREC_SPLIT):
        compare(f"N=120 prec={prec}", dev_curve(torch_dev, ctx, c, lam, m, prec), *want, lam, c, m)


def test_maximum_layer_count_identical_stack(torch_dev, ctx):
    # MASW_MAX_LAYERS identical layers on an identical half-space behave as
    # the half-space (the pinned reduction of the oracle), so every
    # wavelength has the homogeneous Rayleigh root, here at nu = 1/4.
    N = M.MASW_MAX_LAYERS
    beta = 300.0
    m = WL.Model(np.full(N, 0.25), np.full(N + 1, math.sqrt(3) * beta), np.full(N + 1, beta),
                 np.full(N + 1, 1900.0))
    c = WL.uniform_grid(200.0, 0.05, 2401)
    lam = np.array([0.5, 5.0, 60.0, 400.0])
    cR = beta * math.sqrt(2 - 2 / math.sqrt(3))
    for prec in (M.MASW_PREC_FP64, M.MASW_PREC_SPLIT):
        ct, idx, st, cr = dev_curve(torch_dev, ctx, c, lam, m, prec)
        assert np.all(st == 0), (prec, st)
        assert np.all(c[idx - 1] < cR) and np.all(cR <= c[idx]), (prec, idx)
        assert np.max(np.abs(cr - cR) / cR) < 1e-8, (prec, cr)


def test_layer_count_above_maximum_is_rejected(torch_dev, ctx):
    N = M.MASW_MAX_LAYERS + 1
    m = WL.Model(np.full(N, 1.0), np.full(N + 1, 500.0), np.full(N + 1, 300.0), np.full(N + 1, 1900.0))
    c = WL.uniform_grid(200.0, 0.5, 100)
    with pytest.raises(M.MaswError) as e:
        dev_curve(torch_dev, ctx, c, np.array([5.0]), m, M.MASW_PREC_FP64)
    assert e.value.code == M.MASW_EINVAL


def test_grid_of_two_to_the_24_points(torch_dev, ctx):
    # A 16.8 M-point grid at 1e-5 m/s, far finer than FP32 resolves near
    # 140 m/s: picks must bracket the oracle's root and the refined roots
    # agree with it; a root beyond the grid gives NOT_FOUND.
    wl = WL.two_layer_case()
    m = wl.models[0]
    c = WL.uniform_grid(50.0, 1e-5, 1 << 24)
    lam = np.array([1.0, 4.0, 40.0])
    coarse = O.dispersion_curve(lam, wl.c_test, m)
    for prec in (M.MASW_PREC_FP64, M.MASW_PREC_SPLIT):
        ct, idx, st, cr = dev_curve(torch_dev, ctx, c, lam, m, prec)
        for w, p in enumerate(coarse):
            root = p.c_ref
            if root > c[-1]:
                assert idx[w] == -1 and st[w] == O.STATUS_NOT_FOUND, (prec, w)
                continue
            assert st[w] == 0, (prec, w, st[w])
            tol = 2e-9 * root
            assert c[idx[w] - 1] < root + tol and root - tol <= c[idx[w]], (prec, w, idx[w], root)
            assert abs(cr[w] - root) <= 1e-6 * root, (prec, w, cr[w], root)
        print(f"2^24 grid prec={prec}: idx {idx.tolist()} stats {ctx.stats()}", flush=True)


def test_low_velocity_layer_models(torch_dev, ctx):
    rng = np.random.Generator(np.random.PCG64(33))
    c = WL.uniform_grid(50.0, 0.05, 8001)
    for trial in range(4):
        m = WL.increasing_profile(rng, 6)
        m.beta[2] = 0.7 * m.beta[1]
        m.alpha[2] = 2.0 * m.beta[2]
        lam = WL.log_spaced(1.0, 60.0, 12)
        want = oracle_curve(lam, c, m)
        for prec in (M.MASW_PREC_FP64, M.MASW_PREC_SPLIT):
            compare(f"inversion trial {trial} prec={prec}", dev_curve(torch_dev, ctx, c, lam, m, prec),
                    *want, lam, c, m)


def test_repeat_runs_bitwise_identical(torch_dev, ctx):
    wl = WL.fine_scale_case()
    lam = wl.lambdas[0][::10].copy()
    a = dev_curve(torch_dev, ctx, wl.c_test, lam, wl.models[0], M.MASW_PREC_SPLIT)
    b = dev_curve(torch_dev, ctx, wl.c_test, lam, wl.models[0], M.MASW_PREC_SPLIT)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


# ---------------------------------------------------- full-size fine-scale case --
def _golden(name):
    path = os.path.join(HERE, "golden", name)
    if not os.path.exists(path):
        pytest.fail(f"missing {path}: run tests/golden/make_golden.py")
    return json.load(open(path))


@pytest.mark.parametrize("prec", [M.MASW_PREC_FP64, M.MASW_PREC_SPLIT])
def test_fine_scale_full_size(torch_dev, ctx, prec):
    g = _golden("fine_scale.json")
    wl = WL.fine_scale_case()
    m, lam, c = wl.models[0], wl.lambdas[0], wl.c_test
    got = dev_curve(torch_dev, ctx, c, lam, m, prec)
    compare(f"fine-scale prec={prec}", got, g["idx"], g["status"], [float(x) for x in g["c_ref"]], lam, c, m)
    s = ctx.stats()
    useful = int(np.sum(np.asarray(g["idx"]) + 1))
    assert s["useful_evals"] == useful
    print(f"fine-scale prec={prec}: stats {s}", flush=True)


# ------------------------------------------------------------- shared sweeps --
def _context_with_env(**env):
    """A context created with tuning variables set (they are read at creation)."""
    old = {k: os.environ.get(k) for k in env}
    os.environ.update({k: str(v) for k, v in env.items()})
    try:
        return M.Context(0, 1 << 30)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


@pytest.mark.parametrize("prec", [M.MASW_PREC_FP64, M.MASW_PREC_SPLIT])
def test_shared_sweeps_equal_unshared(torch_dev, ctx, prec):
    # With 1000 items on 512 workgroups the deepest items run as shared
    # sweeps that idle workgroups join; every output must be bitwise the same
    # as when each item is swept by its own workgroup alone.
    wl = WL.fine_scale_case()
    m, lam, c = wl.models[0], wl.lambdas[0], wl.c_test
    shared = dev_curve(torch_dev, ctx, c, lam, m, prec)
    s = ctx.stats()
    print(f"shared prec={prec}: {s}", flush=True)
    assert s["shared_items"] == len(lam) and s["shared_stalls"] == 0
    assert s["helper_evals"] > 0
    plain_ctx = _context_with_env(MASW_SHARED_SWEEPS=0)
    try:
        plain = dev_curve(torch_dev, plain_ctx, c, lam, m, prec)
        sp = plain_ctx.stats()
    finally:
        plain_ctx.close()
    assert sp["shared_items"] == 0 and sp["helper_evals"] == 0
    for x, y in zip(shared, plain):
        np.testing.assert_array_equal(x, y)


def test_shared_sweeps_one_wavefront_per_item(torch_dev):
    # G = 1: rounds of 64 velocities, up to ~700 rounds per item, so joining
    # workgroups evaluate a large share of the rounds; picks must still equal
    # the oracle's and the unshared run bitwise.
    g = _golden("fine_scale.json")
    wl = WL.fine_scale_case()
    m, c = wl.models[0], wl.c_test
    sel = np.arange(0, 1000, 4)
    lam = wl.lambdas[0][sel]
    runs = []
    for shared in (1, 0):
        cx = _context_with_env(MASW_WAVES_PER_ITEM=1, MASW_SHARED_SWEEPS=shared)
        try:
            for prec in (M.MASW_PREC_FP64, M.MASW_PREC_SPLIT):
                runs.append(dev_curve(torch_dev, cx, c, lam, m, prec))
                st = cx.stats()
                print(f"G=1 shared={shared} prec={prec}: {st}", flush=True)
                assert st["waves_per_item"] == 1 and st["shared_stalls"] == 0
                assert (st["shared_items"] > 0) == bool(shared)
        finally:
            cx.close()
    want = ([g["idx"][i] for i in sel], [g["status"][i] for i in sel], [float(g["c_ref"][i]) for i in sel])
    compare("G=1 shared fp64", runs[0], *want, lam, c, m)
    compare("G=1 shared split", runs[1], *want, lam, c, m)
    for a, b in ((runs[0], runs[2]), (runs[1], runs[3])):
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("events", [0, 1])
@pytest.mark.parametrize("case", ["fused", "staged"])
def test_timing_of_back_to_back_calls(torch_dev, ctx, case, events):
    # calls issued without synchronising in between are each timed, from the
    # GPU's real-time counter or from HIP events (masw_opts.timing_events),
    # through more calls than the library has timing slots; outputs of the
    # last call are those of a single call.  The two-layer curve runs as one
    # fused launch (sweep time = job time); a 20-wavelength slice of the
    # fine-scale curve is staged before its sweep (job time > sweep time).
    if case == "fused":
        wl = WL.two_layer_case()
        m, lam, c = wl.models[0], wl.lambdas[0], wl.c_test
        n = 300
    else:
        wl = WL.fine_scale_case()
        m, lam, c = wl.models[0], wl.lambdas[0][::50], wl.c_test
        n = 270
    M.masw_set_opts(ctx.ctx, timing_events=events)
    try:
        _timing_run(torch_dev, ctx, case, c, lam, m, n, events)
    finally:
        M.masw_set_opts(ctx.ctx)  # the module's context keeps its default options


def _timing_run(torch_dev, ctx, case, c, lam, m, n, events):
    assert M.masw_get_opts(ctx.ctx)["timing_events"] == events
    want = dev_curve(torch_dev, ctx, c, lam, m, M.MASW_PREC_FP64)
    torch, dev = torch_dev
    t = lambda x: torch.as_tensor(np.ascontiguousarray(x, np.float64), device=dev)
    args = (t(c), t(lam), t(m.h), t(m.alpha), t(m.beta), t(m.rho))
    W = len(lam)
    out = (torch.empty(W, dtype=torch.float64, device=dev), torch.empty(W, dtype=torch.int32, device=dev),
           torch.empty(W, dtype=torch.int32, device=dev), torch.empty(W, dtype=torch.float64, device=dev))
    M.masw_get_timing(ctx.ctx, reset=True)
    for _ in range(n):
        M.masw_dispersion_curve(ctx.ctx, *args, M.MASW_PREC_FP64, 0, None, *out)
    st = M.masw_get_stats(ctx.ctx)
    tm = M.masw_get_timing(ctx.ctx, reset=True)
    assert tm["launches"] == n
    assert 0.0 < tm["sweep_ms_min"] <= tm["sweep_ms_max"] < 1e3
    assert tm["sweep_ms_min"] * n <= tm["sweep_ms_sum"] + 1e-9 <= tm["total_ms_sum"] + 1e-6
    assert 0.0 < st["sweep_ms"] <= st["total_ms"]
    if case == "staged":
        assert st["fused_staging"] == 0 and tm["total_ms_sum"] > tm["sweep_ms_sum"]
    else:
        assert st["fused_staging"] == 1 and abs(tm["total_ms_sum"] - tm["sweep_ms_sum"]) <= 1e-6 * n
    assert M.masw_get_timing(ctx.ctx)["launches"] == 0
    torch.cuda.synchronize()
    for x, y in zip(want, (o.cpu().numpy() for o in out)):
        np.testing.assert_array_equal(x, y)


def test_default_stream_orders_device_calls(torch_dev, ctx):
    # A NULL stream is the device's default stream: device-pointer work that
    # torch issues there (input copies, the read-back) is ordered with the
    # library's kernels, with no explicit synchronisation in between.
    torch, dev = torch_dev
    wl = WL.two_layer_case()
    m, lam, c = wl.models[0], wl.lambdas[0], wl.c_test
    want = dev_curve(torch_dev, ctx, c, lam, m, M.MASW_PREC_FP64)
    t = lambda x: torch.as_tensor(np.ascontiguousarray(x, np.float64), device=dev)
    W = len(lam)
    for rep in range(5):
        out = (torch.full((W,), -7.0, dtype=torch.float64, device=dev), torch.full((W,), -7, dtype=torch.int32, device=dev),
               torch.full((W,), -7, dtype=torch.int32, device=dev), torch.full((W,), -7.0, dtype=torch.float64, device=dev))
        M.masw_dispersion_curve(ctx.ctx, t(c), t(lam), t(m.h), t(m.alpha), t(m.beta), t(m.rho),
                                M.MASW_PREC_FP64, 0, None, *out)
        got = [o.cpu().numpy() for o in out]   # default-stream copies, no synchronize
        for x, y in zip(want, got):
            np.testing.assert_array_equal(x, y)
        arrs = M.flatten_models([m, m], [lam, lam])
        d = [torch.as_tensor(a, device=dev) for a in arrs]
        ce = torch.as_tensor(np.tile(want[0], 2), device=dev)
        mis = torch.full((2,), -7.0, dtype=torch.float64, device=dev)
        M.masw_misfit(ctx.ctx, d[5], ce, ce, 0, None, mis)
        assert mis.cpu().tolist() == [0.0, 0.0]


# ------------------------------------------------------------ batched launch --
def test_batch_sample_and_split_vs_fp64(torch_dev, ctx):
    g = _golden("batch_sample.json")
    wl = WL.batch_case()
    arrs = M.flatten_models(wl.models, wl.lambdas)
    lam_off = arrs[5]
    split = dev_batch(torch_dev, ctx, wl.c_test, wl.models, wl.lambdas, M.MASW_PREC_SPLIT)
    s_split = ctx.stats()
    fp64 = dev_batch(torch_dev, ctx, wl.c_test, wl.models, wl.lambdas, M.MASW_PREC_FP64)
    print(f"batch split stats {s_split}; fp64 stats {ctx.stats()}", flush=True)
    for entry in g["models"]:
        mi = entry["model"]
        sl = slice(int(lam_off[mi]), int(lam_off[mi + 1]))
        for name, res in (("split", split), ("fp64", fp64)):
            compare(f"batch model {mi} {name}", tuple(r[sl] for r in res), entry["idx"], entry["status"],
                    [float(x) for x in entry["c_ref"]], wl.lambdas[mi], wl.c_test, wl.models[mi])
    # every wavelength of the batch: the split path equals the FP64 path,
    # an index difference excused only in the FP64 noise band
    diff = np.nonzero(split[1] != fp64[1])[0]
    print(f"batch: {len(diff)} of {len(split[1])} split picks differ from FP64 picks", flush=True)
    for w in diff:
        mi = int(np.searchsorted(lam_off, w, side="right") - 1)
        pts = {p for i in (int(split[1][w]), int(fp64[1][w])) if i > 0 for p in (i - 1, i)}
        assert any(O.in_noise_band(float(wl.lambdas[mi][w - lam_off[mi]]), float(wl.c_test[p]), wl.models[mi])
                   for p in pts), (mi, w - lam_off[mi], split[1][w], fp64[1][w])
    same = split[1] == fp64[1]
    for x, y in zip(fp64, split):
        np.testing.assert_array_equal(y[same], x[same])


def test_batch_equals_single_model_runs(torch_dev, ctx):
    # a model's curve is the same alone and inside a batch (bitwise)
    wl = WL.batch_case(n_models=24, seed=9)
    res = dev_batch(torch_dev, ctx, wl.c_test, wl.models, wl.lambdas, M.MASW_PREC_SPLIT)
    off = 0
    for m, lam in zip(wl.models, wl.lambdas):
        alone = dev_curve(torch_dev, ctx, wl.c_test, lam, m, M.MASW_PREC_SPLIT)
        for x, y in zip(alone, res):
            np.testing.assert_array_equal(x, y[off:off + len(lam)])
        off += len(lam)


@pytest.mark.parametrize("c0,n", [(137.9170, 60001), (137.91740293 - 3e-8, 4001)])
def test_split_on_a_grid_finer_than_fp32(torch_dev, ctx, c0, n):
    # At c ~ 138 m/s one float spans about 1500 grid points of 1e-8 m/s, so
    # the FP32 sweep sees its change hundreds of points off.  On the first
    # grid the FP64 re-check windows walk it forward, or the inertia counts
    # refuse the stretch FP32 passed over and the item re-sweeps in FP64.  On
    # the second the root lies four points after the grid start and every
    # point near it rounds to one float above the root: FP32 sees no change
    # at all, and only the counts (a mode between the grid start and the end
    # of the FP32 sweep) send the item to FP64.  Either way the split pick
    # must equal the FP64 pick and the oracle's.
    wl = WL.two_layer_case()
    m = wl.models[0]
    c = WL.uniform_grid(c0, 1e-8, n)
    lam = np.array([1.0])
    want = oracle_curve(lam, c, m)
    got64 = dev_curve(torch_dev, ctx, c, lam, m, M.MASW_PREC_FP64)
    got32 = dev_curve(torch_dev, ctx, c, lam, m, M.MASW_PREC_SPLIT)
    compare("fine grid FP64", got64, *want, lam, c, m)
    compare("fine grid split", got32, *want, lam, c, m)
    for x, y in zip(got64, got32):
        np.testing.assert_array_equal(x, y)
    st = ctx.stats()
    print(f"fine grid split stats {st}", flush=True)
    assert st["check_evals"] >= 1 and st["sweep_evals"] > st["useful_evals"] + 512


def test_misfit_matches_algorithm_2(torch_dev, ctx):
    torch, dev = torch_dev
    wl = WL.batch_case(n_models=16, seed=13)
    ct, idx, st, cr = dev_batch(torch_dev, ctx, wl.c_test, wl.models, wl.lambdas, M.MASW_PREC_SPLIT)
    lam_off = M.flatten_models(wl.models, wl.lambdas)[5]
    rng = np.random.Generator(np.random.PCG64(1))
    c_e = np.where(np.isfinite(ct), ct, 300.0) * (1.0 + 0.02 * rng.standard_normal(ct.shape[0]))
    got = np.empty(16)
    M.masw_misfit(ctx.ctx, lam_off, ct, c_e, 0, None, got)
    want = np.array([O.misfit(ct[a:b], c_e[a:b]) for a, b in zip(lam_off[:-1], lam_off[1:])])
    np.testing.assert_allclose(got, want, rtol=1e-12, equal_nan=True)
    t = lambda x: torch.as_tensor(x, device=dev)
    got_d = torch.empty(16, dtype=torch.float64, device=dev)
    M.masw_misfit(ctx.ctx, t(lam_off), t(ct), t(c_e), 0, None, got_d)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got_d.cpu().numpy(), got)


@pytest.mark.parametrize("c_pick", [72.0, 238.0, 256.0])
def test_uniform_curves(torch_dev, ctx, c_pick):
    # identical layers over an identical half-space: every pick is the grid
    # point just above the closed-form Rayleigh speed, and the full sign map's
    # first change is at the same index
    wl = WL.uniform_case(c_pick, 50)
    m, lam, c = wl.models[0], wl.lambdas[0], wl.c_test
    want = int(np.searchsorted(c, c_pick))          # c[want] == c_pick
    c_root = c_pick - 0.25
    for prec in (M.MASW_PREC_FP64, M.MASW_PREC_SPLIT):
        ct, idx, st, cr = dev_curve(torch_dev, ctx, c, lam, m, prec)
        assert np.all(idx == want) and np.all(st == 0) and np.all(ct == c_pick)
        assert np.max(np.abs(cr - c_root) / c_root) < 1e-8
    sig, _ = ctx.sign_map(c, lam[:3], m, M.MASW_PREC_FP64, want_log=False)
    for row in sig:
        assert int(np.nonzero(row[1:] != row[:-1])[0][0]) + 1 == want


def test_split_catches_a_mode_next_to_a_pole(torch_dev, ctx):
    # A mode at 67.98 m/s and a pole one grid step later: FP32 takes the wrong
    # sign between them and sees no change.  The FP32 sweep also watches the
    # parity of negative layer denominators, so the pole crossing sends the
    # region to the FP64 check, and the split pick is the oracle's.
    g = _golden("split_pole_case.json")
    m = WL.Model(np.array(g["h"]), np.array(g["alpha"]), np.array(g["beta"]), np.array(g["rho"]))
    lam = np.array([g["lambda"]])
    c = WL.serving_grid()
    want_ref = float(g["c_ref"])
    for prec in (M.MASW_PREC_FP64, M.MASW_PREC_SPLIT):
        ct, idx, st, cr = dev_curve(torch_dev, ctx, c, lam, m, prec)
        assert (int(idx[0]), int(st[0])) == (g["idx"], g["status"]), (prec, idx, st)
        assert abs(cr[0] - want_ref) <= REL_TOL * want_ref
    cls, sec = ctx.classify(c, [m], [lam], idx)
    assert int(cls[0]) == g["class"] == M.MASW_PICK_MODE


def test_split_misses_match_the_oracle(torch_dev, ctx):
    # Wavelengths of the random stress configurations on which an FP32 sweep
    # with FP64 window checks alone picked a later change than Algorithm 1
    # (FP32 saw none of an even number of changes between two FP64-checked
    # points; one of them above the half-space's S velocity, where no
    # inertia count exists).  All three paths must give the oracle's pick.
    g = _golden("split_misses.json")
    for case in g["cases"]:
        wl = WL.random_stress_config(case["seed"])
        m = wl.models[case["model"]]
        lam = np.array([wl.lambdas[case["model"]][case["lambda_index"]]])
        assert lam[0] == case["lambda"]
        want = ([case["idx"]], [case["status"]], [case["c_ref"]])
        for prec, flags, name in ((M.MASW_PREC_FP64, 0, "walk"), (M.MASW_PREC_SPLIT, 0, "split"),
                                  (M.MASW_PREC_FP64, M.MASW_SEARCH_INERTIA, "inertia")):
            got = dev_curve(torch_dev, ctx, wl.c_test, lam, m, prec, flags)
            n, n_noise, _ = compare(f"split miss seed {case['seed']} {name}", got, *want, lam, wl.c_test, m)
            assert n == 1 and n_noise == 0


def test_budget_exhaustion_is_refused_before_any_work(gpu):
    # a request whose workspace exceeds the context's budget fails with
    # MASW_ENOMEM before anything is queued, and the context stays usable
    wl = WL.fine_scale_case()
    small = WL.two_layer_case()
    with M.Context(0, 1 << 20) as c:        # the fine-scale curve needs about 1.4 MB
        with pytest.raises(M.MaswError) as e:
            c.curve(wl.c_test, wl.lambdas[0], wl.models[0])
        assert e.value.code == M.MASW_ENOMEM and "budget" in str(e.value)
        got = c.curve(small.c_test, small.lambdas[0], small.models[0])
        want = [O.dispersion_point(l, small.c_test, small.models[0], refine=False).idx for l in small.lambdas[0][:5]]
        assert got[1][:5].tolist() == want


def test_random_models_match_oracle(torch_dev, ctx):
    # 12 random models outside the workloads' recipes (N 1-12, thicknesses
    # 0.2-20 m, velocities falling as well as rising with depth, Poisson
    # ratios 0.05-0.45), 5 wavelengths each on a 0.5 m/s grid: the FP64 walk,
    # the split path and the inertia search against the oracle
    rng = np.random.Generator(np.random.PCG64(707))
    c = WL.uniform_grid(40.0, 0.5, 3001)
    for trial in range(12):
        N = int(rng.integers(1, 13))
        h = np.exp(rng.uniform(np.log(0.2), np.log(20.0), size=N))
        beta = rng.uniform(80.0, 600.0, size=N + 1)
        alpha = WL.alpha_from_poisson(beta, rng.uniform(0.05, 0.45, size=N + 1))
        m = WL.Model(h, alpha, beta, rng.uniform(1500.0, 2600.0, size=N + 1))
        lam = np.sort(np.exp(rng.uniform(np.log(0.3), np.log(150.0), size=5)))
        want_idx, want_st, want_ref = oracle_curve(lam, c, m)
        for prec, flags, name in ((M.MASW_PREC_FP64, 0, "walk"), (M.MASW_PREC_SPLIT, 0, "split"),
                                  (M.MASW_PREC_FP64, M.MASW_SEARCH_INERTIA, "inertia")):
            ct, idx, st, cr = dev_curve(torch_dev, ctx, c, lam, m, prec, flags)
            for w in range(len(lam)):
                i = int(want_idx[w])
                assert (int(idx[w]), int(st[w])) == (i, want_st[w]), (trial, name, w, idx[w], i)
                if i < 1:
                    continue
                assert ct[w] == c[i]
                k = 2 * math.pi / lam[w]
                fine = O.det_sign(k, np.linspace(c[i - 1], c[i], 2001), m)
                if np.count_nonzero(fine[1:] != fine[:-1]) <= 1:
                    # one sign change in the grid step: the refined roots agree
                    assert abs(cr[w] - want_ref[w]) <= REL_TOL * want_ref[w], (trial, name, w, cr[w], want_ref[w])
                else:
                    # several changes in the step (poles and zeros closer than
                    # the grid): any of them is a valid refinement, so check
                    # that the device's root is one
                    d = 2e-9 * cr[w]
                    assert c[i - 1] <= cr[w] <= c[i]
                    assert O.det_sign(k, cr[w] - d, m)[0] != O.det_sign(k, cr[w] + d, m)[0], (trial, name, w)


@pytest.mark.parametrize("prec,flags", [(M.MASW_PREC_SPLIT, 0), (M.MASW_PREC_FP64, 0),
                                        (M.MASW_PREC_FP64, M.MASW_SEARCH_INERTIA),
                                        (M.MASW_PREC_SPLIT, M.MASW_NO_REFINE)])
def test_fused_misfit_equals_algorithm_2(torch_dev, ctx, prec, flags):
    # masw_dispersion_batch_misfit: the same curves as masw_dispersion_batch,
    # and misfits equal to masw_misfit's bit for bit and to Algorithm 2's
    # definition (the oracle's misfit) to rounding; an invalid model and one
    # without wavelengths give NaN; host and device pointers agree
    torch, dev = torch_dev
    wl = WL.batch_case(n_models=40, seed=21)
    models, lambdas = list(wl.models), [l.copy() for l in wl.lambdas]
    bad = models[5].copy()
    bad.alpha[0] = 0.5 * bad.beta[0]            # alpha < beta: the model is invalid (on the device)
    models[5] = bad
    lambdas[9] = lambdas[9][:0]                  # no wavelengths
    arrs = M.flatten_models(models, lambdas)
    W = int(arrs[-1].shape[0])
    rng = np.random.Generator(np.random.PCG64(3))
    c_e = 300.0 * (1.0 + 0.1 * rng.standard_normal(W))
    c_e = np.abs(c_e) + 50.0
    td = [torch.as_tensor(a, device=dev) for a in arrs]
    out = (torch.empty(W, dtype=torch.float64, device=dev), torch.empty(W, dtype=torch.int32, device=dev),
           torch.empty(W, dtype=torch.int32, device=dev), torch.empty(W, dtype=torch.float64, device=dev))
    mis = torch.full((len(models),), -1.0, dtype=torch.float64, device=dev)
    M.masw_dispersion_batch_misfit(ctx.ctx, torch.as_tensor(wl.c_test, device=dev), *td, prec, flags, None, *out,
                                   torch.as_tensor(c_e, device=dev), mis)
    torch.cuda.synchronize()
    got = [o.cpu().numpy() for o in out]
    fused = mis.cpu().numpy()
    ref = dev_batch(torch_dev, ctx, wl.c_test, models, lambdas, prec, flags)
    for x, y, what in zip(ref, got, ("C_t", "idx", "status", "c_ref")):
        if what == "c_ref" and flags & M.MASW_NO_REFINE:
            continue
        np.testing.assert_array_equal(y, x, err_msg=what)
    lam_off = arrs[5]
    sep = np.empty(len(models))
    M.masw_misfit(ctx.ctx, lam_off, got[0], c_e, 0, None, sep)
    np.testing.assert_array_equal(fused, sep)
    want = np.array([O.misfit(got[0][a:b], c_e[a:b]) if b > a else np.nan for a, b in zip(lam_off[:-1], lam_off[1:])])
    np.testing.assert_allclose(fused, want, rtol=1e-12, equal_nan=True)
    assert np.isnan(fused[5]) and np.isnan(fused[9]) and np.isfinite(fused[0])
    # host pointers: the invalid model is refused on the host; with it
    # replaced, the host path's misfits are those of its own curves
    hout = (np.empty(W), np.empty(W, np.int32), np.empty(W, np.int32), np.empty(W))
    hmis = np.empty(len(models))
    with pytest.raises(M.MaswError) as e:
        M.masw_dispersion_batch_misfit(ctx.ctx, wl.c_test, *arrs, prec, flags, None, *hout, c_e, hmis)
    assert e.value.code == M.MASW_EINVAL
    models[5] = wl.models[5]
    arrs = M.flatten_models(models, lambdas)
    M.masw_dispersion_batch_misfit(ctx.ctx, wl.c_test, *arrs, prec, flags, None, *hout, c_e, hmis)
    M.masw_misfit(ctx.ctx, lam_off, hout[0], c_e, 0, None, sep)
    np.testing.assert_array_equal(hmis, sep)
    keep = np.ones(W, bool)
    keep[lam_off[5]:lam_off[6]] = False
    np.testing.assert_array_equal(hout[1][keep], got[1][keep])


def check_refined_root(lam, c_lo, c_hi, model, got_ref, want_ref, what):
    """The refined root in [c_lo, c_hi]: with one sign change of the oracle's
    determinant in the step, within REL_TOL of the oracle's root; with
    several (poles and zeros closer than the grid, reading 10), any of them
    is a valid refinement, so the device's root must be one of them."""
    if abs(got_ref - want_ref) <= REL_TOL * want_ref:
        return
    k = 2 * math.pi / lam
    fine = O.det_sign(k, np.linspace(c_lo, c_hi, 2001), model)
    if np.count_nonzero(fine[1:] != fine[:-1]) <= 1:
        assert abs(got_ref - want_ref) <= REL_TOL * want_ref, (what, got_ref, want_ref)
    else:
        d = 2e-9 * got_ref
        assert c_lo <= got_ref <= c_hi, what
        assert O.det_sign(k, got_ref - d, model)[0] != O.det_sign(k, got_ref + d, model)[0], what


def test_random_sample_matches_the_oracle(torch_dev, ctx):
    # 510 wavelengths of the random stress configurations (17 per
    # configuration, spread over each), against the oracle: the FP64 walk, the
    # split path and the inertia search, each in a batch of the sampled
    # models with only the sampled wavelengths.  Index, status and C_t are
    # compared exactly (no noise-band excuse); the refined root as in
    # check_refined_root.
    g = _golden("random_sample.json")
    by_seed = {}
    for e in g["cases"]:
        by_seed.setdefault(e["seed"], []).append(e)
    n_total = 0
    for seed, cases in sorted(by_seed.items()):
        wl = WL.random_stress_config(seed)
        c = wl.c_test
        models = [wl.models[e["model"]] for e in cases]
        lambdas = [np.array([wl.lambdas[e["model"]][e["lambda_index"]]]) for e in cases]
        for prec, flags, name in ((M.MASW_PREC_FP64, 0, "walk"), (M.MASW_PREC_SPLIT, 0, "split"),
                                  (M.MASW_PREC_FP64, M.MASW_SEARCH_INERTIA, "inertia")):
            ct, idx, st, cr = dev_batch(torch_dev, ctx, c, models, lambdas, prec, flags)
            for k, e in enumerate(cases):
                what = (seed, e["model"], e["lambda_index"], name)
                assert (int(idx[k]), int(st[k])) == (e["idx"], e["status"]), (what, idx[k], st[k])
                i = e["idx"]
                if i < 1:
                    assert math.isnan(ct[k]) and math.isnan(cr[k])
                    continue
                assert ct[k] == c[i]
                check_refined_root(float(lambdas[k][0]), float(c[i - 1]), float(c[i]), models[k], float(cr[k]),
                                   float(e["c_ref"]), what)
                n_total += 1
    print(f"random sample: {n_total} (wavelength, path) pairs equal to the oracle", flush=True)


def test_noalloc_call_replays_in_a_captured_graph(torch_dev, ctx):
    # The no-alloc curve call captured once in a hipGraph (its staging and
    # sweep kernels, no allocation, no memset node) and replayed several
    # times, with other eager library work and synchronisations in between:
    # every replay's outputs equal the eager call's, for two precisions.
    torch, dev = torch_dev
    wl = WL.two_layer_case()
    other = WL.fine_scale_case()
    m, lam, c = wl.models[0], wl.lambdas[0], wl.c_test
    t = lambda x: torch.as_tensor(np.ascontiguousarray(x, np.float64), device=dev)
    args = [t(c), t(lam), t(m.h), t(m.alpha), t(m.beta), t(m.rho)]
    W = len(lam)
    for prec in (M.MASW_PREC_FP64, M.MASW_PREC_SPLIT):
        want = dev_curve(torch_dev, ctx, c, lam, m, prec)
        out = (torch.empty(W, dtype=torch.float64, device=dev), torch.empty(W, dtype=torch.int32, device=dev),
               torch.empty(W, dtype=torch.int32, device=dev), torch.empty(W, dtype=torch.float64, device=dev))
        side = torch.cuda.Stream()
        call = M.PreparedCurve(ctx.ctx, *args, prec, 0, side.cuda_stream, *out, noalloc=True)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            call()
        for rep in range(4):
            for o in out:
                o.fill_(-3)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            got = [o.cpu().numpy() for o in out]
            for x, y, what in zip(want, got, ("C_t", "idx", "status", "c_ref")):
                np.testing.assert_array_equal(y, x, err_msg=f"replay {rep} prec {prec}: {what}")
            # eager work between replays: another curve through the arena
            dev_curve(torch_dev, ctx, other.c_test, other.lambdas[0][:50], other.models[0], M.MASW_PREC_FP64)
