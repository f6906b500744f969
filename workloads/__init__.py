"""Seeded synthetic inputs for the dispersion-curve workloads.

This module only draws layered earth models, wavelength lists and test-velocity
grids.  It holds none of the dispersion arithmetic (no stiffness entries, no
determinants, no search), so both the CPU oracle and the HIP path may use it
without sharing any of the method's computation.

The paper's own datasets (a 40-wavelength "variable" experimental curve and a
"uniform" curve, Section 3) are not available; these recipes stand in for them
with the paper's scales: up to ~100 wavelengths and ~1000 test velocities per
curve with N <= 10 layers typical (Section 2.1), 40-entry variable curves and
1000-wavelength uniform curves (Section 3.2), grown to the fine-scale and batched
sizes that one MI355X is sized for.

Every generator uses numpy's PCG64 with a fixed seed and a fixed draw order.
Units: thickness h and wavelength in m, velocities in m/s, density in kg/m^3.
Layer arrays: h has N entries; alpha, beta, rho have N+1 entries, the last
being the half-space.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np


@dataclass
class Model:
    """One layered model: N finite layers over a half-space."""

    h: np.ndarray      # [N]   thickness (m)
    alpha: np.ndarray  # [N+1] P-wave velocity (m/s)
    beta: np.ndarray   # [N+1] S-wave velocity (m/s)
    rho: np.ndarray    # [N+1] density (kg/m^3)

    @property
    def n_layers(self) -> int:
        return int(self.h.shape[0])

    def copy(self) -> "Model":
        return Model(self.h.copy(), self.alpha.copy(), self.beta.copy(), self.rho.copy())


@dataclass
class Workload:
    """Models with their wavelengths and one shared test-velocity grid."""

    name: str
    models: List[Model]
    lambdas: List[np.ndarray]      # per model, wavelengths (m)
    c_test: np.ndarray             # ascending test velocities (m/s), FP64
    meta: dict = field(default_factory=dict)

    @property
    def n_lambda_total(self) -> int:
        return int(sum(len(l) for l in self.lambdas))


def uniform_grid(c_min: float, dc: float, n: int) -> np.ndarray:
    """c_i = c_min + i*dc evaluated in FP64 per index (never accumulated)."""
    return c_min + dc * np.arange(n, dtype=np.float64)


def alpha_from_poisson(beta: np.ndarray, nu: np.ndarray) -> np.ndarray:
    """P velocity of an isotropic solid with S velocity beta and Poisson ratio nu."""
    return beta * np.sqrt((2.0 - 2.0 * nu) / (1.0 - 2.0 * nu))


def log_spaced(lo: float, hi: float, n: int) -> np.ndarray:
    if n == 1:
        return np.array([lo], dtype=np.float64)
    return lo * (hi / lo) ** (np.arange(n, dtype=np.float64) / (n - 1))


# --------------------------------------------------------------------------
# The two-layer model used for the small worked case.
# --------------------------------------------------------------------------
def two_layer_model() -> Model:
    beta = np.array([150.0, 250.0, 400.0])
    return Model(h=np.array([2.0, 4.0]),
                 alpha=np.sqrt(3.0) * beta,
                 beta=beta,
                 rho=np.array([1850.0, 1900.0, 2000.0]))


def two_layer_case() -> Workload:
    """2 layers over a half-space, 30 wavelengths log-spaced 1-40 m,
    c_test 50-450 m/s at 0.5 m/s (801 values)."""
    return Workload("two_layer_30lam_801c", [two_layer_model()],
                    [log_spaced(1.0, 40.0, 30)], uniform_grid(50.0, 0.5, 801))


# --------------------------------------------------------------------------
# Velocity-increasing profiles (the fine-scale and batched recipes).
# --------------------------------------------------------------------------
def increasing_profile(rng: np.random.Generator, n_layers: int,
                       poisson: bool = True,
                       rho_lo: float = 1700.0, rho_hi: float = 2200.0) -> Model:
    """Draw order: h[N], beta0, N-1 increments, nu[N+1] (or none), rho[N+1].

    beta_0 ~ U(100, 200); beta_{j+1} = beta_j + U(5, 40); half-space beta =
    last layer beta + 100.  With poisson=True alpha comes from nu ~ U(0.25, 0.4)
    per layer and for the half-space; otherwise alpha = sqrt(3) beta.
    """
    N = n_layers
    h = rng.uniform(0.5, 3.0, size=N)
    beta = np.empty(N + 1)
    beta[0] = rng.uniform(100.0, 200.0)
    inc = rng.uniform(5.0, 40.0, size=max(N - 1, 0))
    for j in range(1, N):
        beta[j] = beta[j - 1] + inc[j - 1]
    beta[N] = (beta[N - 1] if N > 0 else beta[0]) + 100.0
    if poisson:
        nu = rng.uniform(0.25, 0.4, size=N + 1)
        alpha = alpha_from_poisson(beta, nu)
    else:
        alpha = np.sqrt(3.0) * beta
    rho = rng.uniform(rho_lo, rho_hi, size=N + 1)
    return Model(h, alpha, beta, rho)


def fine_scale_case(seed: int = 2) -> Workload:
    """20 layers, 1000 wavelengths log-spaced 1-100 m, c 50-1200 m/s at 0.01
    m/s (115,001 values), plain FP64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = increasing_profile(rng, 20)
    return Workload("fine_scale_N20_1000lam_115001c", [m],
                    [log_spaced(1.0, 100.0, 1000)], uniform_grid(50.0, 0.01, 115001))


def apply_inversion(rng: np.random.Generator, m: Model, prob: float = 0.15) -> bool:
    """With probability prob, pick j ~ U{1..N-1} and make layer j slower than
    the layer above it: beta_j = beta_{j-1} * U(0.6, 0.9), alpha_j keeping
    layer j's alpha/beta ratio.  Draw order: one uniform, then j, then the
    factor (the last two only when an inversion is applied)."""
    u = rng.uniform()
    N = m.n_layers
    if u >= prob or N < 2:
        return False
    j = int(rng.integers(1, N))            # 1..N-1
    f = rng.uniform(0.6, 0.9)
    ratio = m.alpha[j] / m.beta[j]
    m.beta[j] = m.beta[j - 1] * f
    m.alpha[j] = ratio * m.beta[j]
    return True


def batch_case(n_models: int = 4096, seed: int = 4,
               n_lo: int = 3, n_hi: int = 30,
               w_lo: int = 50, w_hi: int = 500) -> Workload:
    """Batch of seeded models of uneven sizes: N ~ U{3..30}, W ~ U{50..500}
    wavelengths log-spaced 1-80 m, c 50-1000 m/s at 0.05 m/s (19,001 values),
    about 15% with one low-velocity inversion layer."""
    rng = np.random.Generator(np.random.PCG64(seed))
    models, lams, inverted = [], [], []
    for _ in range(n_models):
        N = int(rng.integers(n_lo, n_hi + 1))
        W = int(rng.integers(w_lo, w_hi + 1))
        m = increasing_profile(rng, N)
        inverted.append(apply_inversion(rng, m))
        models.append(m)
        lams.append(log_spaced(1.0, 80.0, W))
    return Workload(f"batch_{n_models}models_19001c", models, lams,
                    uniform_grid(50.0, 0.05, 19001), meta={"inverted": inverted})


# --------------------------------------------------------------------------
# "Uniform" curves: every wavelength the same, picks at a chosen velocity.
# --------------------------------------------------------------------------
RAYLEIGH_RATIO_QUARTER_POISSON = 0.9194016867619  # c_R / beta at nu = 0.25


def uniform_case(c_pick: float, length: int, lam: float = 10.0, n_layers: int = 6) -> Workload:
    """`length` identical wavelengths over n_layers identical layers on an
    identical half-space (alpha = sqrt(3) beta, rho = 2000); c_test 50-549.5
    m/s at 0.5 m/s (1000 values).  The layered model behaves as the
    half-space, so every wavelength has the same root whatever lam is; beta
    puts that root a quarter grid step below the grid point c_pick, so the
    reported velocity (the upper end of the bracket) is c_pick."""
    beta = (c_pick - 0.25) / RAYLEIGH_RATIO_QUARTER_POISSON
    N = n_layers
    m = Model(h=np.full(N, 1.0), alpha=np.full(N + 1, np.sqrt(3.0) * beta),
              beta=np.full(N + 1, beta), rho=np.full(N + 1, 2000.0))
    return Workload(f"uniform_c{c_pick:g}_L{length}", [m], [np.full(length, lam)],
                    uniform_grid(50.0, 0.5, 1000))


# --------------------------------------------------------------------------
# Random-walk chains for the serving workload.
# --------------------------------------------------------------------------
@dataclass
class Chain:
    model: Model
    lambdas: np.ndarray


def chain_bases(n_chains: int = 64, seed: int = 5) -> List[Chain]:
    """Chain start points: N ~ U{5..25}, W ~ U{30..300} wavelengths log-spaced
    1-40 m, beta as in the velocity-increasing recipe, alpha = sqrt(3) beta,
    rho ~ U(1850, 2000)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n_chains):
        N = int(rng.integers(5, 26))
        W = int(rng.integers(30, 301))
        m = increasing_profile(rng, N, poisson=False, rho_lo=1850.0, rho_hi=2000.0)
        out.append(Chain(m, log_spaced(1.0, 40.0, W)))
    return out


def chain_step(rng: np.random.Generator, m: Model, sd: float = 0.02) -> Model:
    """One random-walk step: every beta_j and h_j times (1 + N(0, sd));
    alpha = sqrt(3) beta is kept.  Draw order: beta[N+1] then h[N]."""
    out = m.copy()
    out.beta = m.beta * (1.0 + sd * rng.standard_normal(m.beta.shape[0]))
    out.h = m.h * (1.0 + sd * rng.standard_normal(m.h.shape[0]))
    out.beta = np.maximum(out.beta, 1.0)
    out.h = np.maximum(out.h, 1e-3)
    out.alpha = np.sqrt(3.0) * out.beta
    return out


def serving_grid() -> np.ndarray:
    """Per-request grid: 50-1000 m/s at 0.1 m/s (9,501 values)."""
    return uniform_grid(50.0, 0.1, 9501)


def poisson_arrivals(rate: float, duration: float, seed: int = 55) -> np.ndarray:
    """Arrival times (s) of a Poisson process with the given rate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(rate * duration * 1.5) + 16
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    return t[t < duration]


# --------------------------------------------------------------------------
# Random models outside the recipes above (stress and parity cases).
# --------------------------------------------------------------------------
def random_model(rng: np.random.Generator, n_layers: int) -> Model:
    """A layered model outside the workloads' recipes: thicknesses over two
    decades (0.2-20 m, log-uniform), S velocities U(80, 600) that may fall
    with depth (low-velocity layers, a half-space slower than some layers),
    Poisson ratios U(0.05, 0.45), densities U(1500, 2600).  Draw order:
    h[N], beta[N+1], nu[N+1], rho[N+1]."""
    N = n_layers
    h = np.exp(rng.uniform(np.log(0.2), np.log(20.0), size=N))
    beta = rng.uniform(80.0, 600.0, size=N + 1)
    nu = rng.uniform(0.05, 0.45, size=N + 1)
    alpha = alpha_from_poisson(beta, nu)
    rho = rng.uniform(1500.0, 2600.0, size=N + 1)
    return Model(h, alpha, beta, rho)


def random_stress_config(seed: int, n_models: int = 96) -> Workload:
    """One configuration of the random-model stress: a grid of 0.5, 0.1,
    0.05, 0.02 or 0.01 m/s (by seed mod 5) from U(20, 120) m/s up to
    U(600, 1500) m/s (at most 60,000 points); n_models random models with
    N ~ U{1..40}; per model U{10..499} wavelengths log-uniform in 0.2-200 m,
    sorted, and for seeds divisible by 3 every fourth model's list reversed.
    Draw order: grid start, grid end, then per model N and the model, then
    per model the wavelength count and the wavelengths."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dc = [0.5, 0.1, 0.05, 0.02, 0.01][seed % 5]
    lo = rng.uniform(20.0, 120.0)
    n_c = int(min(60000, (rng.uniform(600.0, 1500.0) - lo) / dc))
    c = uniform_grid(lo, dc, n_c)
    models = [random_model(rng, int(rng.integers(1, 41))) for _ in range(n_models)]
    lambdas = [np.sort(np.exp(rng.uniform(np.log(0.2), np.log(200.0), size=int(rng.integers(10, 500)))))
               for _ in models]
    if seed % 3 == 0:
        for l in lambdas[::4]:
            l[:] = l[::-1]
    return Workload(f"random_stress_{seed}", models, lambdas, c)


def serving_trace(rate: float, duration: float, seed: int = 55):
    """The serving workload's request stream: Poisson arrival times (s) over
    `duration` at `rate` per second, and for each arrival the model and
    wavelengths of its request.  Each arrival picks one of the 64 chains of
    chain_bases() uniformly and advances it one chain_step.  Draw order: the
    arrival times (seed), then from PCG64(seed + 1) the chain of every
    arrival, then the steps in arrival order."""
    bases = chain_bases(64, 5)
    times = poisson_arrivals(rate, duration, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    pick = rng.integers(0, len(bases), size=len(times))
    state = [b.model for b in bases]
    reqs = []
    for i in range(len(times)):
        ch = int(pick[i])
        state[ch] = chain_step(rng, state[ch])
        reqs.append((state[ch], bases[ch].lambdas))
    return times, reqs
