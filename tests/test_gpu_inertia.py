"""The inertia-count search (MASW_SEARCH_INERTIA) against the FP64 walk and
the oracle.

The search skips grid points whose inertia counts prove sign(det K)
constant, so its outputs must be the walk's: the same index and status, and,
since the refinement of a pick is the same code on the same bracket, the same
C_t and c_ref bit for bit.  Where the picks are also compared with the oracle
the bar is the parity bar (exact index outside the FP64 noise band, roots
within 1e-6 relative).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import paper_2003_02256_amd as M
import workloads as WL
from test_gpu_parity import REL_TOL, compare, dev_batch, dev_curve, oracle_curve

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
INERTIA = M.MASW_SEARCH_INERTIA
FP64 = M.MASW_PREC_FP64


@pytest.fixture(scope="module")
def torch_dev(gpu):
    import torch
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def ctx(gpu):
    c = M.Context(0, 2 << 30)
    yield c
    c.close()


def both(torch_dev, ctx, c, lam, m, name):
    walk = dev_curve(torch_dev, ctx, c, lam, m, FP64)
    got = dev_curve(torch_dev, ctx, c, lam, m, FP64, INERTIA)
    st = ctx.stats()
    for x, y, what in zip(walk, got, ("C_t", "idx", "status", "c_ref")):
        np.testing.assert_array_equal(y, x, err_msg=f"{name}: {what}")
    return got, st


def test_two_layer_case(torch_dev, ctx):
    wl = WL.two_layer_case()
    m, lam, c = wl.models[0], wl.lambdas[0], wl.c_test
    got, st = both(torch_dev, ctx, c, lam, m, "two-layer")
    compare("two-layer inertia", got, *oracle_curve(lam, c, m), lam, c, m)
    print(f"two-layer inertia stats {st}", flush=True)
    assert st["inertia_evals"] > 0 and st["useful_evals"] == 8951


@pytest.mark.parametrize("n_c", [2, 3, 65, 127, 129, 300, 513, 1537])
def test_ragged_and_tiny_grids(torch_dev, ctx, n_c):
    wl = WL.two_layer_case()
    m = wl.models[0]
    c = WL.uniform_grid(130.0, 190.0 / n_c, n_c)
    lam = wl.lambdas[0]
    got, _ = both(torch_dev, ctx, c, lam, m, f"ragged n_c={n_c}")
    want = oracle_curve(lam, c, m)
    if n_c <= 3:
        # brackets of tens of m/s hold several sign changes, and bisection and
        # multisection may refine to different ones: compare the picks only
        assert got[1].tolist() == want[0]
    else:
        compare(f"ragged n_c={n_c} inertia", got, *want, lam, c, m)


def test_not_found(torch_dev, ctx):
    wl = WL.two_layer_case()
    c = WL.uniform_grid(50.0, 0.5, 100)     # entirely below every root
    got, _ = both(torch_dev, ctx, c, np.array([1.0, 40.0]), wl.models[0], "not found")
    assert np.all(got[1] == -1) and np.all(got[2] == M.MASW_STATUS_NOT_FOUND)


def test_grid_above_the_halfspace_velocity_is_walked(torch_dev, ctx):
    # A half-space (beta 400) on a grid that starts above its Rayleigh root:
    # no count changes below beta, the search stops at the first point at or
    # above it and walks the complex determinant from there, as the walk does.
    beta = 400.0
    m = WL.Model(np.zeros(0), np.array([math.sqrt(3) * beta]), np.array([beta]), np.array([2000.0]))
    c = WL.uniform_grid(380.0, 0.05, 8001)
    lam = np.array([0.5, 5.0, 50.0])
    got, st = both(torch_dev, ctx, c, lam, m, "above beta_hs")
    print(f"above beta_hs: idx {got[1].tolist()} status {got[2].tolist()} stats {st}", flush=True)
    assert st["sweep_evals"] > 0                 # grid points walked
    # the same on a layered model whose grid starts above its half-space's S velocity
    wl = WL.two_layer_case()
    c2 = WL.uniform_grid(401.0, 0.5, 200)
    both(torch_dev, ctx, c2, wl.lambdas[0], wl.models[0], "grid above beta_hs")


def test_homogeneous_halfspace_root(torch_dev, ctx):
    beta = 400.0
    m = WL.Model(np.zeros(0), np.array([math.sqrt(3) * beta]), np.array([beta]), np.array([2000.0]))
    c = WL.uniform_grid(300.0, 0.01, 10001)
    lam = np.array([0.5, 5.0, 50.0])
    (ct, idx, st, cr), _ = both(torch_dev, ctx, c, lam, m, "half-space")
    cR = beta * math.sqrt(2 - 2 / math.sqrt(3))
    assert np.all(st == 0) and np.all(c[idx - 1] < cR) and np.all(cR <= c[idx])


def test_low_velocity_layers_and_many_layers(torch_dev, ctx):
    rng = np.random.Generator(np.random.PCG64(33))
    c = WL.uniform_grid(50.0, 0.05, 8001)
    for trial in range(4):
        m = WL.increasing_profile(rng, 6)
        m.beta[2] = 0.7 * m.beta[1]
        m.alpha[2] = 2.0 * m.beta[2]
        lam = WL.log_spaced(1.0, 60.0, 12)
        got, _ = both(torch_dev, ctx, c, lam, m, f"inversion {trial}")
        compare(f"inversion trial {trial} inertia", got, *oracle_curve(lam, c, m), lam, c, m)
    rng = np.random.Generator(np.random.PCG64(21))
    m = WL.increasing_profile(rng, 120)
    c = WL.uniform_grid(100.0, 0.25, 1200)
    lam = np.array([1.0, 3.0, 9.0])
    got, _ = both(torch_dev, ctx, c, lam, m, "N=120")
    compare("N=120 inertia", got, *oracle_curve(lam, c, m), lam, c, m)


def test_maximum_layer_count_identical_stack(torch_dev, ctx):
    N = M.MASW_MAX_LAYERS
    beta = 300.0
    m = WL.Model(np.full(N, 0.25), np.full(N + 1, math.sqrt(3) * beta), np.full(N + 1, beta),
                 np.full(N + 1, 1900.0))
    c = WL.uniform_grid(200.0, 0.05, 2401)
    both(torch_dev, ctx, c, np.array([0.5, 5.0, 60.0, 400.0]), m, "1024 layers")


def test_invalid_inputs_marked_as_the_walk_marks_them(torch_dev, ctx):
    wl = WL.two_layer_case()
    m = wl.models[0].copy()
    m.alpha[1] = 0.5 * m.beta[1]
    got, _ = both(torch_dev, ctx, wl.c_test, wl.lambdas[0], m, "invalid model")
    assert np.all(got[2] == M.MASW_STATUS_INVALID)
    lam = wl.lambdas[0].copy()
    lam[3] = -1.0
    got, _ = both(torch_dev, ctx, wl.c_test, lam, wl.models[0], "one invalid wavelength")
    assert got[2][3] == M.MASW_STATUS_INVALID


def test_mode_next_to_a_pole(torch_dev, ctx):
    # a mode and, one grid step later, a pole of det K
    g = json.load(open(os.path.join(HERE, "golden", "split_pole_case.json")))
    m = WL.Model(np.array(g["h"]), np.array(g["alpha"]), np.array(g["beta"]), np.array(g["rho"]))
    (ct, idx, st, cr), _ = both(torch_dev, ctx, WL.serving_grid(), np.array([g["lambda"]]), m, "mode next to pole")
    assert (int(idx[0]), int(st[0])) == (g["idx"], g["status"])
    assert abs(cr[0] - float(g["c_ref"])) <= REL_TOL * float(g["c_ref"])


def test_first_changes_at_poles_and_modes(torch_dev, ctx):
    # On the 20-layer model at short wavelengths grids that begin just past
    # each of the first sign changes make every kind of change the first one:
    # poles, modes, and a pole and a mode close together.
    wl = WL.fine_scale_case()
    m = wl.models[0]
    for lam in (1.0, 3.0):
        k = 2 * math.pi / lam
        c = WL.uniform_grid(50.0, 0.01, 115001)[:60001]
        sig = O.det_sign(k, c[::50], m)
        coarse = np.nonzero(sig[1:] != sig[:-1])[0][:6]
        # each grid starts past the previous change, so its first change is the next one
        for start in [0] + [(int(j) + 1) * 50 for j in coarse[:-1]]:
            cc = c[start:start + 20001]
            got, st = both(torch_dev, ctx, cc, np.array([lam]), m, f"lambda {lam} from {cc[0]:.2f}")
            p = O.dispersion_point(lam, cc, m)
            assert int(got[1][0]) == p.idx, (lam, cc[0], got[1][0], p.idx)
            # the refined root, a pole's too (interpolated through 1/det K),
            # within the refinement tolerance of the oracle's bisection
            assert abs(got[3][0] - p.c_ref) <= 2e-9 * p.c_ref, (lam, cc[0], got[3][0], p.c_ref)
            print(f"lambda {lam} from c={cc[0]:.2f}: idx {p.idx} status {int(got[2][0])} "
                  f"counts {st['inertia_evals']}", flush=True)


def _golden(name):
    path = os.path.join(HERE, "golden", name)
    if not os.path.exists(path):
        pytest.fail(f"missing {path}: run tests/golden/make_golden.py")
    return json.load(open(path))


def test_fine_scale_full_size(torch_dev, ctx):
    g = _golden("fine_scale.json")
    wl = WL.fine_scale_case()
    m, lam, c = wl.models[0], wl.lambdas[0], wl.c_test
    got, st = both(torch_dev, ctx, c, lam, m, "fine-scale")
    compare("fine-scale inertia", got, g["idx"], g["status"], [float(x) for x in g["c_ref"]], lam, c, m)
    assert st["useful_evals"] == int(np.sum(np.asarray(g["idx"]) + 1))
    print(f"fine-scale inertia stats {st}", flush=True)
    assert st["inertia_evals"] < st["useful_evals"] // 50


def test_full_batch_equals_the_walk(torch_dev, ctx):
    wl = WL.batch_case()
    walk = dev_batch(torch_dev, ctx, wl.c_test, wl.models, wl.lambdas, FP64)
    got = dev_batch(torch_dev, ctx, wl.c_test, wl.models, wl.lambdas, FP64, INERTIA)
    st = ctx.stats()
    print(f"batch inertia stats {st}", flush=True)
    diff = np.nonzero(walk[1] != got[1])[0]
    print(f"batch: {len(diff)} of {len(got[1])} inertia picks differ from the walk's: {diff[:10].tolist()}",
          flush=True)
    assert len(diff) == 0
    np.testing.assert_array_equal(got[2], walk[2])
    np.testing.assert_array_equal(got[0], walk[0])
    np.testing.assert_array_equal(got[3], walk[3])


def test_runs_with_predictions_across_models_and_invalid_items(torch_dev, ctx):
    # 200 models (about 55,000 wavelengths, so wavefronts claim runs of
    # consecutive wavelengths and predict picks within them).  Invalid
    # models and wavelengths inside runs, and wavelengths in reverse order
    # (picks that fall along the run), must not disturb the predictions'
    # effect: outputs equal the walk's bit for bit.
    wl = WL.batch_case(n_models=200, seed=11)
    models, lambdas = list(wl.models), [l.copy() for l in wl.lambdas]
    for i in (3, 50, 51, 120):
        m = models[i].copy()
        m.alpha[1] = 0.5 * m.beta[1]        # alpha < beta: invalid on the device
        models[i] = m
    for i in (7, 90):
        lambdas[i][10] = -1.0               # one invalid wavelength in the middle of a run
    for i in range(0, 200, 9):
        lambdas[i] = lambdas[i][::-1].copy()
    walk = dev_batch(torch_dev, ctx, wl.c_test, models, lambdas, FP64)
    got = dev_batch(torch_dev, ctx, wl.c_test, models, lambdas, FP64, INERTIA)
    st = ctx.stats()
    print(f"runs: {len(got[1])} wavelengths, stats {st}", flush=True)
    for x, y, what in zip(walk, got, ("C_t", "idx", "status", "c_ref")):
        np.testing.assert_array_equal(y, x, err_msg=what)
    assert np.sum(got[2] == M.MASW_STATUS_INVALID) >= 4 * 50 + 2
    assert st["check_evals"] < 64 * len(got[1]) // 2   # runs of 4 here: most wavelengths were predicted


@pytest.mark.parametrize("seed,dc,n_c,lo", [(101, 0.5, 3001, 40.0), (102, 0.05, 12001, 60.0),
                                            (103, 0.01, 40001, 90.0)])
def test_random_models_equal_the_walk(torch_dev, ctx, seed, dc, n_c, lo):
    # random models (N 1-40) and wavelengths 0.3-150 m on three grids; with
    # many wavelengths per model the wavefronts also take predicted runs.
    # Outputs equal the walk's bit for bit; an index that differs would be
    # excused only inside the FP64 noise band (none has been seen).
    rng = np.random.Generator(np.random.PCG64(seed))
    models = [WL.random_model(rng, int(rng.integers(1, 41))) for _ in range(96)]
    lambdas = [np.sort(np.exp(rng.uniform(np.log(0.3), np.log(150.0), size=int(rng.integers(20, 400)))))
               for _ in models]
    c = WL.uniform_grid(lo, dc, n_c)
    walk = dev_batch(torch_dev, ctx, c, models, lambdas, FP64)
    got = dev_batch(torch_dev, ctx, c, models, lambdas, FP64, INERTIA)
    st = ctx.stats()
    off = np.concatenate([[0], np.cumsum([len(l) for l in lambdas])])
    diff = np.nonzero(got[1] != walk[1])[0]
    for w in diff:
        mi = int(np.searchsorted(off, w, side="right") - 1)
        lam = float(lambdas[mi][w - off[mi]])
        pts = {p for i in (int(got[1][w]), int(walk[1][w])) if i > 0 for p in (i - 1, i)}
        assert any(O.in_noise_band(lam, float(c[p]), models[mi]) for p in pts), (w, got[1][w], walk[1][w])
    same = got[1] == walk[1]
    for x, y, what in zip(walk, got, ("C_t", "idx", "status", "c_ref")):
        np.testing.assert_array_equal(y[same], x[same], err_msg=what)
    print(f"random seed {seed}: {len(got[1])} wavelengths, {len(diff)} index differences (noise band), "
          f"found {int(np.sum(got[1] >= 0))}, walked {st['sweep_evals']}, counts {st['inertia_evals']}", flush=True)


def test_random_stress_thirty_configurations(torch_dev, ctx):
    # 30 configurations of 96 random models each (about 730,000 wavelengths):
    # grids of 0.5 to 0.01 m/s up to 60,000 points, wavelengths 0.2-200 m,
    # some models' wavelengths in reverse order.  Every output of the inertia
    # search and of the split path equals the walk's; an index difference
    # would be excused only in the noise band.
    total = 0
    for seed in range(1000, 1030):
        wl = WL.random_stress_config(seed)
        c, models, lambdas = wl.c_test, wl.models, wl.lambdas
        walk = dev_batch(torch_dev, ctx, c, models, lambdas, FP64)
        off = np.concatenate([[0], np.cumsum([len(l) for l in lambdas])])
        for name, got in (("inertia", dev_batch(torch_dev, ctx, c, models, lambdas, FP64, INERTIA)),
                          ("split", dev_batch(torch_dev, ctx, c, models, lambdas, M.MASW_PREC_SPLIT))):
            for w in np.nonzero(got[1] != walk[1])[0]:
                mi = int(np.searchsorted(off, w, side="right") - 1)
                pts = {p for i in (int(got[1][w]), int(walk[1][w])) if i > 0 for p in (i - 1, i)}
                assert any(O.in_noise_band(float(lambdas[mi][w - off[mi]]), float(c[p]), models[mi]) for p in pts), \
                    (name, seed, mi, w - off[mi], got[1][w], walk[1][w])
            same = got[1] == walk[1]
            for x, y, what in zip(walk, got, ("C_t", "idx", "status", "c_ref")):
                np.testing.assert_array_equal(y[same], x[same], err_msg=f"{name} seed {seed}: {what}")
        total += len(walk[1])
    print(f"random stress: {total} wavelengths over 30 configurations", flush=True)
