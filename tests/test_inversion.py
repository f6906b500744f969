"""Host logic of the random-walk inversion client (no GPU): proposals, the
Metropolis rule and the chain loop, driven by a stand-in evaluator."""
import math

import numpy as np
import pytest

from paper_2003_02256_amd import inversion as I
import workloads as WL


def _model():
    m = WL.two_layer_model()
    m.alpha = m.alpha * np.array([1.0, 1.2, 1.1])  # layer-specific Poisson ratios
    return m


def test_perturb_keeps_ratios_density_and_positivity():
    m = _model()
    rng = np.random.Generator(np.random.PCG64(3))
    for _ in range(200):
        p = I.perturb(rng, m, 0.3)
        np.testing.assert_allclose(p.alpha / p.beta, m.alpha / m.beta, rtol=1e-15)
        np.testing.assert_array_equal(p.rho, m.rho)
        assert np.all(p.beta >= 1.0) and np.all(p.h >= 1e-3)
        assert np.all(p.alpha > p.beta)
    a = I.perturb(np.random.Generator(np.random.PCG64(9)), m, 0.02)
    b = I.perturb(np.random.Generator(np.random.PCG64(9)), m, 0.02)
    np.testing.assert_array_equal(a.beta, b.beta)
    np.testing.assert_array_equal(a.h, b.h)


def test_metropolis_rule():
    rng = np.random.Generator(np.random.PCG64(1))
    cur = np.array([1.0, 1.0, 1.0, np.nan, np.nan])
    new = np.array([0.5, 1.0, np.nan, 2.0, np.nan])
    ok = I.metropolis_accept(rng, cur, new, 0.1)
    # better and equal misfits are taken, NaN proposals never, a NaN chain
    # moves to any finite proposal
    assert list(ok) == [True, True, False, True, False]
    # worse by T ln 2: accepted with probability 1/2
    n = 40000
    T = 0.25
    ok = I.metropolis_accept(rng, np.zeros(n), np.full(n, T * math.log(2.0)), T)
    assert abs(ok.mean() - 0.5) < 0.01
    # far worse: essentially never
    assert not I.metropolis_accept(rng, np.zeros(n), np.full(n, 50.0 * T), T).any()


def _beta_misfit(target):
    def evaluate(models):
        return np.array([float(np.mean(np.abs(m.beta - target) / target)) for m in models])
    return evaluate


def test_chains_reduce_the_misfit_and_are_reproducible():
    truth = _model()
    ev = _beta_misfit(truth.beta)
    rng = np.random.Generator(np.random.PCG64(5))
    start = [I.perturb(rng, truth, 0.15) for _ in range(12)]
    r1 = I.run_chains(ev, start, 150, step=0.02, temperature=0.002, seed=7)
    r2 = I.run_chains(ev, start, 150, step=0.02, temperature=0.002, seed=7)
    np.testing.assert_array_equal(r1.best_misfit, r2.best_misfit)
    np.testing.assert_array_equal(r1.trace, r2.trace)
    assert np.all(r1.best_misfit <= r1.start_misfit)
    assert np.mean(r1.best_misfit) < 0.5 * np.mean(r1.start_misfit)
    assert 0.0 < r1.acceptance_rate < 1.0
    # best models reproduce their recorded misfits
    np.testing.assert_allclose(ev(r1.best_models), r1.best_misfit, rtol=0, atol=0)
    # the trace starts at the start misfits and ends at the final ones
    np.testing.assert_array_equal(r1.trace[0], r1.start_misfit)
    np.testing.assert_array_equal(r1.trace[-1], r1.final_misfit)
    r3 = I.run_chains(ev, start, 150, step=0.02, temperature=0.002, seed=8)
    assert not np.array_equal(r1.trace, r3.trace)


def test_synthetic_curve_and_scale():
    ct = np.array([100.0, 200.0, 400.0])
    np.testing.assert_array_equal(I.synthetic_curve(ct, 0.0), ct)
    noisy = I.synthetic_curve(ct, 0.01, seed=3)
    assert np.all(np.abs(noisy / ct - 1.0) < 0.06)
    assert I.misfit_scale(ct, 0.5) == pytest.approx(np.mean(0.5 / ct))


def test_population_and_zero_step():
    truth = _model()
    pop = I.Population.stack([truth, truth.copy()])
    assert len(pop) == 2 and pop.h.shape == (2, 2) and pop.beta.shape == (2, 3)
    np.testing.assert_array_equal(list(pop)[1].beta, truth.beta)
    short = WL.Model(truth.h[:1], truth.alpha[:2], truth.beta[:2], truth.rho[:2])
    with pytest.raises(ValueError):
        I.Population.stack([truth, short])
    # with a zero step every proposal is the current model: always accepted,
    # nothing changes
    ev = _beta_misfit(truth.beta * 1.1)
    r = I.run_chains(ev, [truth, truth], 5, step=0.0, temperature=0.01, seed=1)
    assert r.accepted.tolist() == [5, 5]
    np.testing.assert_array_equal(r.trace, np.full((6, 2), ev([truth])[0]))
    np.testing.assert_array_equal(r.best_models[0].beta, truth.beta)
