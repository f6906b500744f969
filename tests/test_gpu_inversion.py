"""The inversion client on the GPU: device misfits of chain models against
the oracle's Algorithm 2 misfit, and chains that reduce the misfit."""
import numpy as np
import pytest

import oracle as O
import paper_2003_02256_amd as M
from paper_2003_02256_amd import inversion as I
import workloads as WL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup(gpu):
    wl = WL.two_layer_case()
    truth, lam, c = wl.models[0], wl.lambdas[0], wl.c_test
    idx, ct, st, _ = O.curve_arrays(O.dispersion_curve(lam, c, truth, refine=False))
    assert np.all(idx >= 0)
    ctx = M.Context(0, 1 << 30)
    yield ctx, truth, lam, c, ct
    ctx.close()


@pytest.mark.parametrize("prec,inertia", [(M.MASW_PREC_FP64, False), (M.MASW_PREC_SPLIT, False),
                                          (M.MASW_PREC_FP64, True)])
def test_device_misfit_matches_oracle(setup, prec, inertia):
    ctx, truth, lam, c, C_e = setup
    ev = I.DeviceEvaluator(ctx.ctx, c, lam, C_e, prec=prec, inertia=inertia)
    assert ev([truth])[0] == 0.0  # the true model reproduces its own curve
    rng = np.random.Generator(np.random.PCG64(21))
    models = [I.perturb(rng, truth, 0.08) for _ in range(6)]
    got = ev(models)
    for m, g in zip(models, got):
        idx, ct, st, _ = O.curve_arrays(O.dispersion_curve(lam, c, m, refine=False))
        want = O.misfit(ct, C_e) if np.all(idx >= 0) else np.nan
        if np.isnan(want):
            assert np.isnan(g)
        else:
            assert g == pytest.approx(want, rel=1e-13, abs=1e-15)


def test_chains_reduce_misfit(setup):
    ctx, truth, lam, c, C_e = setup
    C_obs = I.synthetic_curve(C_e, 0.005, seed=2)
    ev = I.DeviceEvaluator(ctx.ctx, c, lam, C_obs)
    rng = np.random.Generator(np.random.PCG64(4))
    start = [I.perturb(rng, truth, 0.12) for _ in range(16)]
    T = I.misfit_scale(C_obs, float(c[1] - c[0]))
    res = I.run_chains(ev, start, 40, step=0.02, temperature=T, seed=5)
    print(f"start {np.nanmean(res.start_misfit):.4f} best {np.nanmean(res.best_misfit):.4f} "
          f"acceptance {res.acceptance_rate:.3f} models {ev.models_evaluated}", flush=True)
    assert ev.models_evaluated == 16 * 41
    assert np.nanmean(res.best_misfit) < 0.7 * np.nanmean(res.start_misfit)
    assert 0.0 < res.acceptance_rate < 1.0
    # the recorded best misfits are those of the best models, evaluated again
    np.testing.assert_array_equal(ev(res.best_models), res.best_misfit)


def test_inertia_evaluator_equals_the_walk_on_a_population(setup):
    # 64 proposals on the serving grid: the inertia search's C_t are the
    # walk's, so the misfits are equal bit for bit
    ctx, truth, lam, c, C_e = setup
    base = WL.chain_bases(8, seed=5)[3]
    rng = np.random.Generator(np.random.PCG64(4))
    models = [I.perturb(rng, base.model, 0.05) for _ in range(64)]
    grid = WL.serving_grid()
    C_obs = np.full(len(base.lambdas), 300.0)
    walk = I.DeviceEvaluator(ctx.ctx, grid, base.lambdas, C_obs, prec=M.MASW_PREC_FP64)(models)
    fast = I.DeviceEvaluator(ctx.ctx, grid, base.lambdas, C_obs, inertia=True)(models)
    np.testing.assert_array_equal(fast, walk)
