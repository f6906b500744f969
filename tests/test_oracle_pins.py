"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: a textbook closed form, a
first-principles derivation from the P-SV equations of motion (matrix
exponential propagators, an independent formulation), an algebraic identity,
a physical limit, or an invariance.  A dropped term, a wrong sign or index, or
a transposed block in the oracle fails at least one of them.
"""
import math

import mpmath as mp
import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
import workloads as WL


# ---------------------------------------------------------------------------
# Independent references
# ---------------------------------------------------------------------------
def rayleigh_speed(alpha, beta):
    """Rayleigh-wave speed of a homogeneous half-space: c = beta sqrt(xi), xi the
    root in (0, 1) of the rationalised Rayleigh equation
    xi^3 - 8 xi^2 + (24 - 16 b) xi - 16 (1 - b) = 0 with b = beta^2/alpha^2."""
    b = (beta / alpha) ** 2
    roots = np.roots([1.0, -8.0, 24.0 - 16.0 * b, -16.0 * (1.0 - b)])
    real = [r.real for r in roots if abs(r.imag) < 1e-12 and 0.0 < r.real < 1.0]
    assert len(real) == 1
    return beta * math.sqrt(real[0])


def psv_system(k, c, alpha, beta, rho):
    """Real first-order P-SV system v' = A v, z positive down, for the state
    (u_x, -i u_z, tau_xz, -i tau_zz) of a plane wave exp(i(k x - k c t))."""
    mu = rho * beta ** 2
    lam = rho * alpha ** 2 - 2.0 * mu
    M = lam + 2.0 * mu
    w2 = (k * c) ** 2
    A = np.zeros((4, 4))
    A[0, 1] = k
    A[0, 2] = 1.0 / mu
    A[1, 0] = -k * lam / M
    A[1, 3] = 1.0 / M
    A[2, 0] = -rho * w2 + k * k * 4.0 * mu * (lam + mu) / M
    A[2, 3] = k * lam / M
    A[3, 1] = -rho * w2
    A[3, 2] = -k
    return A


def layer_stiffness_from_propagator(k, c, h, alpha, beta, rho):
    """Loads on a layer's faces vs its face displacements, from the transfer
    matrix exp(A h): top load = -traction(0), bottom load = +traction(h)."""
    P = sla.expm(psv_system(k, c, alpha, beta, rho) * h)
    Puu, Put, Ptu, Ptt = P[:2, :2], P[:2, 2:], P[2:, :2], P[2:, 2:]
    iPut = np.linalg.inv(Put)
    return np.block([[iPut @ Puu, -iPut], [Ptu - Ptt @ iPut @ Puu, Ptt @ iPut]])


def halfspace_stiffness_from_eigvecs(k, c, alpha, beta, rho):
    """Load on a half-space's top face vs its displacement, from the two
    decaying eigen-solutions of A (valid for c < beta)."""
    ev, V = np.linalg.eig(psv_system(k, c, alpha, beta, rho))
    order = np.argsort(ev.real)[:2]
    Vd = V[:, order].real
    return -(Vd[2:, :] @ np.linalg.inv(Vd[:2, :]))


# The oracle's vertical degree of freedom has the opposite sign to the
# propagator's; the similarity diag(1, -1, ...) leaves every determinant unchanged.
FLIP4 = np.diag([1.0, -1.0, 1.0, -1.0])
FLIP2 = np.diag([1.0, -1.0])


def mp_secular(k, c, model):
    """Rayleigh secular function of a layered half-space from mpmath propagators:
    det(P_tu + H P_uu) with P the surface-to-half-space transfer matrix applied
    to traction-free surface states and H the half-space's load/displacement
    matrix.  Independent of the stiffness-matrix formulas."""
    def sysmat(alpha, beta, rho):
        k_, c_, a_, b_, r_ = map(mp.mpf, (k, c, alpha, beta, rho))
        mu = r_ * b_ ** 2
        lam = r_ * a_ ** 2 - 2 * mu
        M = lam + 2 * mu
        w2 = (k_ * c_) ** 2
        A = mp.zeros(4, 4)
        A[0, 1] = k_
        A[0, 2] = 1 / mu
        A[1, 0] = -k_ * lam / M
        A[1, 3] = 1 / M
        A[2, 0] = -r_ * w2 + k_ * k_ * 4 * mu * (lam + mu) / M
        A[2, 3] = k_ * lam / M
        A[3, 1] = -r_ * w2
        A[3, 2] = -k_
        return A
    N = model.n_layers
    P = mp.eye(4)
    for j in range(N):
        P = mp.expm(sysmat(model.alpha[j], model.beta[j], model.rho[j]) * mp.mpf(model.h[j])) * P
    ev, V = mp.eig(sysmat(model.alpha[N], model.beta[N], model.rho[N]))
    order = sorted(range(4), key=lambda i: mp.re(ev[i]))[:2]
    Vd = mp.matrix(4, 2)
    for a, i in enumerate(order):
        for r in range(4):
            Vd[r, a] = mp.re(V[r, i])
    H = -Vd[2:4, 0:2] * mp.inverse(Vd[0:2, 0:2])
    return mp.det(P[2:4, 0:2] + H * P[0:2, 0:2])


def mp_root(k, lo, hi, model, steps=34):
    f_lo = mp_secular(k, lo, model)
    lo, hi = mp.mpf(lo), mp.mpf(hi)
    for _ in range(steps):
        mid = (lo + hi) / 2
        f_mid = mp_secular(k, mid, model)
        if mp.sign(f_mid) == mp.sign(f_lo):
            lo, f_lo = mid, f_mid
        else:
            hi = mid
    return float((lo + hi) / 2)


def halfspace_model(alpha, beta, rho):
    return WL.Model(np.zeros(0), np.array([alpha]), np.array([beta]), np.array([rho]))


# ---------------------------------------------------------------------------
# P1: homogeneous half-space, closed-form Rayleigh root
# ---------------------------------------------------------------------------
def test_rayleigh_closed_form_at_quarter_poisson():
    # nu = 0.25 (alpha = sqrt(3) beta): c_R = beta sqrt(2 - 2/sqrt(3)).
    assert rayleigh_speed(math.sqrt(3.0), 1.0) == pytest.approx(math.sqrt(2 - 2 / math.sqrt(3)), rel=1e-13)
    assert math.sqrt(2 - 2 / math.sqrt(3)) == pytest.approx(0.91940168, abs=1e-8)


@pytest.mark.parametrize("beta,nu,lam", [(400.0, 0.25, 5.0), (400.0, 0.25, 0.3),
                                         (150.0, 0.33, 12.0), (250.0, 0.40, 80.0)])
def test_halfspace_root_matches_rayleigh_equation(beta, nu, lam):
    alpha = float(WL.alpha_from_poisson(np.array([beta]), np.array([nu]))[0])
    cR = rayleigh_speed(alpha, beta)
    c_test = WL.uniform_grid(0.5 * beta, 0.01, int(0.6 * beta / 0.01))
    p = O.dispersion_point(lam, c_test, halfspace_model(alpha, beta, 1900.0))
    assert p.status == O.STATUS_FOUND
    # the pick is the upper end of the grid bracket that holds the root
    assert c_test[p.idx - 1] < cR <= c_test[p.idx]
    assert p.c_t == c_test[p.idx]
    assert abs(p.c_ref - cR) / cR <= 1e-9


def test_halfspace_det_closed_form():
    # det H = -(k mu)^2 [(1 + s^2)^2 - 4 r s] / (1 - r s) for real r, s.
    k, alpha, beta, rho = 0.9, 700.0, 400.0, 2000.0
    for c in (100.0, 250.0, 380.0):
        r = math.sqrt(1 - (c / alpha) ** 2)
        s = math.sqrt(1 - (c / beta) ** 2)
        mu = rho * beta ** 2
        want = -(k * mu) ** 2 * ((1 + s * s) ** 2 - 4 * r * s) / (1 - r * s)
        got = np.linalg.det(O.halfspace_matrix(k, np.array(c), alpha, beta, rho))
        assert abs(got.imag) == 0.0
        assert got.real == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("c", [450.0, 520.0, 650.0, 800.0, 1000.0])
def test_halfspace_det_and_sign_above_beta(c):
    # Above beta s = i sqrt(c^2/beta^2 - 1) (and above alpha r = i sqrt(...)):
    # det H is complex and the search uses the sign of its real part.
    k, alpha, beta, rho = 1.3, 700.0, 400.0, 2000.0
    def psqrt(x):
        return complex(math.sqrt(x), 0.0) if x >= 0 else complex(0.0, math.sqrt(-x))
    r, s = psqrt(1 - (c / alpha) ** 2), psqrt(1 - (c / beta) ** 2)
    mu = rho * beta ** 2
    want = -(k * mu) ** 2 * ((1 + s * s) ** 2 - 4 * r * s) / (1 - r * s)
    if c < alpha:                      # beta < c < alpha: r real, s imaginary
        assert abs(want.imag) > 1e-6 * abs(want)
    got = np.linalg.det(O.halfspace_matrix(k, np.array(c), alpha, beta, rho))
    assert abs(got - want) <= 1e-12 * abs(want)
    m = halfspace_model(alpha, beta, rho)
    assert int(O.det_sign(k, c, m)[0]) == int(np.sign(want.real))


# ---------------------------------------------------------------------------
# First principles: layer and half-space matrices from the P-SV equations
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("c", [60.0, 150.0, 199.0, 260.0, 410.0, 700.0])
@pytest.mark.parametrize("lam,h", [(7.0, 3.0), (2.0, 0.7), (30.0, 1.5)])
def test_layer_matrix_matches_propagator(c, lam, h):
    # c spans c < beta, beta < c < alpha (s imaginary) and c > alpha (both imaginary)
    k = 2 * math.pi / lam
    alpha, beta, rho = 520.0, 200.0, 1900.0
    Ko = O.layer_matrix(k, np.array(c), h, alpha, beta, rho)
    assert np.all(Ko.imag == 0.0)
    Kp = FLIP4 @ layer_stiffness_from_propagator(k, c, h, alpha, beta, rho) @ FLIP4
    scale = np.max(np.abs(Kp))
    assert np.max(np.abs(Ko.real - Kp)) <= 1e-9 * scale


@pytest.mark.parametrize("c", [50.0, 200.0, 355.0])
def test_halfspace_matrix_matches_eigensolutions(c):
    k, alpha, beta, rho = 2 * math.pi / 9.0, 650.0, 360.0, 2100.0
    Ho = O.halfspace_matrix(k, np.array(c), alpha, beta, rho)
    Hp = FLIP2 @ halfspace_stiffness_from_eigvecs(k, c, alpha, beta, rho) @ FLIP2
    assert np.max(np.abs(Ho - Hp)) <= 1e-10 * np.max(np.abs(Hp))


# ---------------------------------------------------------------------------
# P2: condensing a layer onto an identical half-space gives the half-space
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("c", [80.0, 300.0, 390.0, 450.0, 760.0])
def test_condensation_identity(c):
    # c > beta (=400) makes H complex; c > alpha (=692.8) makes r imaginary too.
    k, h = 2 * math.pi / 6.0, 2.5
    alpha, beta, rho = 400.0 * math.sqrt(3.0), 400.0, 2000.0
    KL = O.layer_matrix(k, np.array(c), h, alpha, beta, rho)
    H = O.halfspace_matrix(k, np.array(c), alpha, beta, rho)
    P, Q, R = KL[:2, :2], KL[:2, 2:], KL[2:, 2:]
    cond = P - Q @ np.linalg.solve(R + H, Q.T)
    assert np.max(np.abs(cond - H)) <= 1e-9 * np.max(np.abs(H))


# ---------------------------------------------------------------------------
# P3: identical layers over an identical half-space behave as the half-space
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("lam", [1.0, 7.0, 50.0])
def test_identical_layers_reduce_to_halfspace(lam):
    beta, rho = 400.0, 2000.0
    alpha = math.sqrt(3.0) * beta
    N = 3
    m = WL.Model(np.array([2.0, 0.7, 4.0]), np.full(N + 1, alpha), np.full(N + 1, beta), np.full(N + 1, rho))
    c_test = WL.uniform_grid(300.0, 0.01, 8001)
    p = O.dispersion_point(lam, c_test, m)
    p0 = O.dispersion_point(lam, c_test, halfspace_model(alpha, beta, rho))
    assert p.idx == p0.idx
    assert abs(p.c_ref - rayleigh_speed(alpha, beta)) / p.c_ref < 1e-9


# ---------------------------------------------------------------------------
# P4 / P5: short- and long-wavelength limits of a layer over a half-space
# ---------------------------------------------------------------------------
def _layer_over_halfspace():
    beta = np.array([150.0, 400.0])
    return WL.Model(np.array([2.0]), math.sqrt(3.0) * beta, beta, np.array([1850.0, 2000.0]))


@pytest.mark.parametrize("lam", [0.05, 0.1, 0.2])
def test_short_wavelength_limit(lam):
    m = _layer_over_halfspace()
    c_top = rayleigh_speed(m.alpha[0], m.beta[0])
    p = O.dispersion_point(lam, WL.uniform_grid(100.0, 0.01, 30001), m)
    assert abs(p.c_ref - c_top) / c_top < 1e-8


def test_long_wavelength_limit_is_monotone():
    m = _layer_over_halfspace()
    c_hs = rayleigh_speed(m.alpha[1], m.beta[1])
    grid = WL.uniform_grid(100.0, 0.01, 30001)
    errs = [c_hs - O.dispersion_point(lam, grid, m).c_ref for lam in (20.0, 200.0, 2000.0, 20000.0)]
    assert all(e > 0 for e in errs)
    assert all(a > b for a, b in zip(errs, errs[1:]))
    assert errs[-1] / c_hs < 1e-3


# ---------------------------------------------------------------------------
# Roots against an independent propagator secular function (mpmath, 30 digits)
# ---------------------------------------------------------------------------
def test_roots_match_propagator_secular_function():
    mp.mp.dps = 30
    rng = np.random.Generator(np.random.PCG64(7))
    m = WL.increasing_profile(rng, 4)
    m_inv = WL.increasing_profile(rng, 3)
    m_inv.beta[1] = 0.7 * m_inv.beta[0]          # a low-velocity layer
    m_inv.alpha[1] = 1.9 * m_inv.beta[1]
    c_test = WL.uniform_grid(50.0, 0.05, 20001)
    for model, lam in ((m, 1.5), (m, 12.0), (m_inv, 4.0)):
        p = O.dispersion_point(lam, c_test, model)
        assert p.status == O.STATUS_FOUND
        k = 2 * math.pi / lam
        assert mp.sign(mp_secular(k, c_test[p.idx - 1], model)) != mp.sign(mp_secular(k, c_test[p.idx], model))
        want = mp_root(k, c_test[p.idx - 1], c_test[p.idx], model)
        assert abs(p.c_ref - want) / want < 2e-9


# ---------------------------------------------------------------------------
# P6: scaling invariances
# ---------------------------------------------------------------------------
def test_scaling_invariances():
    wl = WL.two_layer_case()
    m, lams, c = wl.models[0], wl.lambdas[0][::3], wl.c_test
    base = [O.dispersion_point(l, c, m, refine=False).idx for l in lams]
    g = 1.7
    # lengths: (h, lambda) -> g (h, lambda)
    mh = m.copy(); mh.h = g * m.h
    assert [O.dispersion_point(g * l, c, mh, refine=False).idx for l in lams] == base
    # velocities: (alpha, beta, c_test) -> g (...)
    mv = m.copy(); mv.alpha = g * m.alpha; mv.beta = g * m.beta
    assert [O.dispersion_point(l, g * c, mv, refine=False).idx for l in lams] == base
    # density: rho -> g rho multiplies det by g^(2(N+1)) > 0
    mr = m.copy(); mr.rho = g * m.rho
    assert [O.dispersion_point(l, c, mr, refine=False).idx for l in lams] == base


# ---------------------------------------------------------------------------
# P8: structure of the assembled matrix
# ---------------------------------------------------------------------------
def test_structure_symmetric_real_heptadiagonal():
    rng = np.random.Generator(np.random.PCG64(3))
    m = WL.increasing_profile(rng, 6)
    k = 2 * math.pi / 5.0
    c = np.array([60.0, 120.0, 0.99 * m.beta[-1], 1.2 * m.beta[-1]])
    K = O.stiffness_matrix(k, c, m.h, m.alpha, m.beta, m.rho)
    n = 2 * (m.n_layers + 1)
    assert K.shape == (4, n, n)
    assert np.array_equal(K, np.swapaxes(K, -1, -2))
    assert np.all(K[:3].imag == 0.0)            # c below the half-space beta
    assert np.any(K[3].imag != 0.0)             # above it the half-space block is complex
    i, j = np.indices((n, n))
    assert np.all(K[:, np.abs(i - j) > 3] == 0.0)
    assert np.any(K[:, np.abs(i - j) == 3] != 0.0)


# ---------------------------------------------------------------------------
# Removable singularities at c = beta_j on the grid
# ---------------------------------------------------------------------------
def test_removable_singularity_on_grid_is_finite_and_continuous():
    wl = WL.two_layer_case()
    m = wl.models[0]
    k = 2 * math.pi / 10.0
    for cs in (150.0, 250.0):
        assert cs in wl.c_test
        s0, _, l0 = O.det_sign_logabs(k, np.array([cs]), m)
        sl, _, ll = O.det_sign_logabs(k, np.array([cs - 1e-6, cs + 1e-6]), m)
        assert s0[0] == sl[0] == sl[1]
        assert abs(l0[0] - ll[0]) < 1e-6 and abs(l0[0] - ll[1]) < 1e-6
    # no false pick at the grid point c = 150 = beta_1 for long wavelengths
    p = O.dispersion_point(20.0, wl.c_test, m, refine=False)
    assert wl.c_test[p.idx] != 150.0


# ---------------------------------------------------------------------------
# Algorithm 1's scan semantics, and its not-found case
# ---------------------------------------------------------------------------
def test_first_change_index_semantics():
    f = O.first_change_index
    assert f([1, 1, 1, -1, -1]) == 3
    assert f([-1, -1, -1]) == -1
    assert f([1, 0, 0, -1]) == 1           # a zero determinant differs from +1
    assert f([0, 0, 1]) == 2
    assert f([1, 1], prev=-1) == 0        # carry from the previous batch
    assert f([]) == -1


def test_batched_scan_equals_whole_grid_scan():
    wl = WL.two_layer_case()
    m = wl.models[0]
    for lam in (1.0, 9.0, 40.0):
        k = 2 * math.pi / lam
        sig = O.det_sign(k, wl.c_test, m)
        d = np.nonzero(sig[1:] != sig[:-1])[0]
        want = int(d[0]) + 1
        for batch in (1, 7, 64, 1000):
            assert O.first_sign_change(k, wl.c_test, m, batch=batch)[0] == want


def test_not_found_below_root():
    wl = WL.two_layer_case()
    p = O.dispersion_point(1.0, WL.uniform_grid(50.0, 0.5, 100), wl.models[0])
    assert p.idx == -1 and p.status == O.STATUS_NOT_FOUND and math.isnan(p.c_t) and math.isnan(p.c_ref)


# ---------------------------------------------------------------------------
# Algorithm 2 (misfit) and the FP64 noise band
# ---------------------------------------------------------------------------
def test_misfit_definition():
    assert O.misfit(np.array([1.0, 2.0, 3.0]), np.array([2.0, 2.0, 4.0])) == pytest.approx((0.5 + 0.0 + 0.25) / 3)


def test_noise_band_only_at_the_root():
    beta = 400.0
    alpha = math.sqrt(3.0) * beta
    m = halfspace_model(alpha, beta, 2000.0)
    cR = rayleigh_speed(alpha, beta)
    assert O.in_noise_band(3.0, cR, m)
    assert not O.in_noise_band(3.0, cR + 0.01, m)
    assert not O.in_noise_band(3.0, cR - 0.01, m)


# P9: the FP64 noise band against 50-digit determinants.  K is rebuilt in
# mpmath from the P-SV equations of motion (transfer matrices for the layers,
# decaying eigen-solutions for the half-space; not the oracle's entry
# formulas), and its exact determinant is compared with the oracle's FP64
# determinant (dense LU) at grid points approaching a root from both sides.
def _mp_sysmat(k, c, alpha, beta, rho):
    k_, c_, a_, b_, r_ = (mp.mpf(v) for v in (k, c, alpha, beta, rho))
    mu = r_ * b_ ** 2
    lam = r_ * a_ ** 2 - 2 * mu
    M = lam + 2 * mu
    w2 = (k_ * c_) ** 2
    A = mp.zeros(4, 4)
    A[0, 1] = k_
    A[0, 2] = 1 / mu
    A[1, 0] = -k_ * lam / M
    A[1, 3] = 1 / M
    A[2, 0] = -r_ * w2 + k_ * k_ * 4 * mu * (lam + mu) / M
    A[2, 3] = k_ * lam / M
    A[3, 1] = -r_ * w2
    A[3, 2] = -k_
    return A


def mp_stiffness_det(k, c, model):
    """det K(k, c) in the working mpmath precision: each layer's stiffness
    from its transfer matrix exp(A h) (loads vs face displacements), the
    half-space's from its decaying eigen-solutions, assembled as in the
    stiffness method.  Similar to the oracle's K by sign flips of the vertical
    degrees of freedom, so the determinant is the same (c below the
    half-space's S velocity)."""
    N = model.n_layers
    n = 2 * (N + 1)
    K = mp.zeros(n, n)
    for j in range(N):
        P = mp.expm(_mp_sysmat(k, c, model.alpha[j], model.beta[j], model.rho[j]) * mp.mpf(model.h[j]))
        Puu, Put, Ptu, Ptt = P[0:2, 0:2], P[0:2, 2:4], P[2:4, 0:2], P[2:4, 2:4]
        iPut = mp.inverse(Put)
        blocks = ((iPut * Puu, -iPut), (Ptu - Ptt * iPut * Puu, Ptt * iPut))
        for bi in range(2):
            for bj in range(2):
                for a in range(2):
                    for b in range(2):
                        K[2 * j + 2 * bi + a, 2 * j + 2 * bj + b] += blocks[bi][bj][a, b]
    ev, V = mp.eig(_mp_sysmat(k, c, model.alpha[N], model.beta[N], model.rho[N]))
    order = sorted(range(4), key=lambda i: mp.re(ev[i]))[:2]
    Vd = mp.matrix(4, 2)
    for q, i in enumerate(order):
        for r in range(4):
            Vd[r, q] = mp.re(V[r, i])
    H = -(Vd[2:4, 0:2] * mp.inverse(Vd[0:2, 0:2]))
    for a in range(2):
        for b in range(2):
            K[2 * N + a, 2 * N + b] += H[a, b]
    return mp.det(K)


def _noise_cases():
    b = 400.0
    yield halfspace_model(math.sqrt(3.0) * b, b, 2000.0), 3.0
    yield halfspace_model(b * math.sqrt(1.2 / 0.2), b, 1800.0), 10.0
    m1 = WL.Model(np.array([3.0]), np.array([300.0, 700.0]), np.array([150.0, 380.0]), np.array([1800.0, 2000.0]))
    yield m1, 2.0
    yield m1, 9.0
    two = WL.two_layer_case().models[0]
    for lam in (1.0, 9.87, 40.0):
        yield two, lam
    m3 = WL.Model(np.array([1.5, 2.5, 4.0]), np.array([330.0, 480.0, 620.0, 900.0]),
                  np.array([170.0, 240.0, 330.0, 480.0]), np.array([1750.0, 1850.0, 1950.0, 2050.0]))
    for lam in (1.5, 6.0, 25.0):
        yield m3, lam


NOISE_FACTOR = 4.0   # the measured FP64 error stays below this multiple of cond_2 2(N+1) 2^-53


def test_noise_band_calibrated_against_50_digit_determinants():
    """Reading 11's band against exact determinants on N = 0..3 models, at
    grid points 10^-16.5 .. 10^-11.5 relative from a root on both sides:
      * every FP64 sign that differs from the exact sign lies in the band;
      * the FP64 determinant's relative error never exceeds NOISE_FACTOR
        times the first-order bound cond_2(K) 2(N+1) 2^-53 the band is built on;
      * calibration of the threshold: per root, R = (band half-width) /
        (half-width of the region where the measured error reaches 1e-2);
        the band is meant to cover that 1% region, so min R over the roots
        must lie in [0.25, 2], i.e. in the tightest case the band ends
        within a factor of a few of where the FP64 determinant stops being
        1%-accurate (a threshold 10 times larger or smaller moves min R by a
        factor of 10 and fails), and max R stays below 50.
    """
    mp.mp.dps = 50
    u = 2.0 ** -53
    ratios = []
    for model, lam in _noise_cases():
        k = 2.0 * math.pi / lam
        grid = np.arange(50.0, float(model.beta[-1]) - 0.01, 0.05)
        p = O.dispersion_point(lam, grid, model)
        # the exact root inside the oracle's refined bracket (width <= 1e-9 c)
        root = mp.findroot(lambda x: mp_stiffness_det(k, x, model),
                           (mp.mpf(p.c_ref) * (1 - mp.mpf(2e-9)), mp.mpf(p.c_ref) * (1 + mp.mpf(2e-9))),
                           solver="illinois", verify=False)
        lo_s = mp.sign(mp_stiffness_det(k, root * (1 - mp.mpf(10) ** -30), model))
        hi_s = mp.sign(mp_stiffness_det(k, root * (1 + mp.mpf(10) ** -30), model))
        assert lo_s != hi_s, (model.n_layers, lam)     # a simple root, located to 1e-30
        assert abs(root - p.c_ref) <= 1e-9 * p.c_ref
        w_band = w_meas = 0.0
        for e in np.arange(-16.5, -11.4, 0.25):
            for side in (-1, 1):
                c = float(root * (1 + side * mp.mpf(10) ** e))
                exact = mp_stiffness_det(k, mp.mpf(c), model)
                sig, phase, logabs = O.det_sign_logabs(k, np.array([c]), model)
                d64 = mp.mpf(float(phase[0].real)) * mp.exp(mp.mpf(float(logabs[0])))
                err = float(abs(d64 - exact) / abs(exact))
                K = O.stiffness_matrix(k, np.array([c]), model.h, model.alpha, model.beta, model.rho)[0]
                bound = float(np.linalg.cond(K) * K.shape[0] * u)
                band = O.in_noise_band(lam, c, model)
                assert err <= NOISE_FACTOR * bound, (model.n_layers, lam, e, err, bound)
                if int(sig[0]) != int(mp.sign(exact)):
                    assert band, (model.n_layers, lam, e, "FP64 sign wrong outside the band")
                if band:
                    w_band = max(w_band, 10.0 ** e)
                if err >= 1e-2:
                    w_meas = max(w_meas, 10.0 ** e)
        # beyond the sampled offsets neither the band nor the 1% region reaches
        for e in (-11.0, -9.0, -6.0):
            assert not O.in_noise_band(lam, float(root * (1 + mp.mpf(10) ** e)), model)
        assert w_band > 0.0 and w_meas > 0.0, (model.n_layers, lam)
        ratios.append(w_band / w_meas)
    assert 0.25 <= min(ratios) <= 2.0, ratios
    assert max(ratios) <= 50.0, ratios


# ---------------------------------------------------------------------------
# P10: the propagator secular function and the zero/pole classification
# (oracle/propagator.py), against the equations of motion, the Rayleigh
# function, a 30-digit propagator and the stiffness formulation
# ---------------------------------------------------------------------------
from oracle import propagator as PR  # noqa: E402


def test_propagator_system_is_the_scaled_psv_system():
    # A of the oracle = the physical system in zeta = k z with tractions
    # divided by k mu_ref: T^-1 (A_phys / k) T, T = diag(1, 1, k mu_ref, k mu_ref).
    k, c, alpha, beta, rho, mu_ref = 0.7, 180.0, 420.0, 210.0, 1850.0, 2000.0 * 450.0 ** 2
    T = np.diag([1.0, 1.0, k * mu_ref, k * mu_ref])
    want = np.linalg.inv(T) @ (psv_system(k, c, alpha, beta, rho) / k) @ T
    got = PR.system_matrix(c, alpha, beta, rho, mu_ref)
    assert np.allclose(got, want, rtol=1e-13, atol=1e-13 * np.abs(want).max())


@pytest.mark.parametrize("c", [40.0, 150.0, 299.0])
def test_propagator_decaying_pair_are_eigenvectors(c):
    alpha, beta, rho = 560.0, 300.0, 1950.0
    A = PR.system_matrix(c, alpha, beta, rho, rho * beta ** 2)
    V = PR.decaying_pair(c, alpha, beta)
    r, s = math.sqrt(1 - (c / alpha) ** 2), math.sqrt(1 - (c / beta) ** 2)
    assert np.allclose(A @ V[:, 0], -r * V[:, 0], atol=1e-13)
    assert np.allclose(A @ V[:, 1], -s * V[:, 1], atol=1e-13)


def test_propagator_halfspace_is_the_rayleigh_function():
    # N = 0: F is a positive multiple of 4 r s - (2 - g)^2, whose root is the
    # closed-form Rayleigh speed.
    alpha, beta = 700.0, 400.0
    m = halfspace_model(alpha, beta, 2000.0)
    for c in np.linspace(50.0, 399.0, 41):
        r, s, g = math.sqrt(1 - (c / alpha) ** 2), math.sqrt(1 - (c / beta) ** 2), (c / beta) ** 2
        want = np.sign(4 * r * s - (2 - g) ** 2)
        assert PR._sgn(PR.secular(1.3, c, m)) == want
    cR = rayleigh_speed(alpha, beta)
    c_test = WL.uniform_grid(300.0, 0.5, 180)
    idx = int(np.searchsorted(c_test, cR))
    cls, c_sec = PR.classify(2.0, c_test, idx, m)
    assert cls == PR.PICK_MODE
    assert abs(c_sec - cR) / cR < 1e-11


def _sign_changes(values):
    s = np.sign(np.asarray(values, np.float64))
    return [i for i in range(1, len(s)) if s[i] != s[i - 1]]


def test_propagator_zeros_match_mpmath_propagator():
    # Same brackets of sign change, and the same roots, as the 30-digit
    # propagator determinant det(P_tu + H P_uu), which uses no orthonormalisation.
    mp.mp.dps = 30
    rng = np.random.Generator(np.random.PCG64(21))
    m = WL.increasing_profile(rng, 3)
    beta_hs = float(m.beta[-1])
    for lam in (2.0, 15.0):
        k = 2 * math.pi / lam
        cs = np.linspace(0.55 * float(m.beta[0]), 0.995 * beta_hs, 90)
        ours = _sign_changes([PR.secular(k, c, m) for c in cs])
        ref = _sign_changes([float(mp_secular(k, c, m)) for c in cs])
        assert ours == ref and ours
        i = ours[0]
        cls, c_sec = PR.classify(lam, cs, i, m)
        assert cls == PR.PICK_MODE
        want = mp_root(k, cs[i - 1], cs[i], m, steps=44)
        assert abs(c_sec - want) / want < 1e-11


def test_stiffness_and_propagator_sign_relation():
    # det K = F x (positive) / prod_j D_j: sign(det K) prod sign(D_j) sign(F)
    # is one constant below the half-space's S velocity, at every wavelength,
    # including short ones where the layer propagators grow by e^(k h).
    wl = WL.fine_scale_case()
    m = wl.models[0]
    cs = wl.c_test[::1500]
    cs = cs[cs < m.beta[-1]]
    vals = set()
    for lam in (1.0, 12.0, 100.0):
        k = 2 * math.pi / lam
        sK = O.det_sign(k, cs, m)
        for c, sk in zip(cs, sK):
            sD = (-1) ** bin(O.pole_mask(k, c, m)).count("1")
            vals.add(int(sk) * sD * PR._sgn(PR.secular(k, c, m)))
    assert vals == {1}


def test_classification_separates_modes_from_poles():
    # Along a 1 m wavelength's grid the stiffness determinant changes sign at
    # modes and at layer resonances (poles).  The propagator classes every
    # change as the stiffness denominators do, and the mode roots of the two
    # formulations agree.
    wl = WL.fine_scale_case()
    m, lam = wl.models[0], 1.0
    k = 2 * math.pi / lam
    cs = WL.uniform_grid(100.0, 2.0, 150)
    changes = _sign_changes(O.det_sign(k, cs, m))[:6]
    seen = set()
    for i in changes:
        pole = O.pole_mask(k, cs[i - 1], m) != O.pole_mask(k, cs[i], m)
        cls, c_sec = PR.classify(lam, cs, i, m, rel_tol=1e-11)
        assert cls == (PR.PICK_POLE if pole else PR.PICK_MODE)
        seen.add(cls)
        if cls == PR.PICK_MODE:
            c_ref = O.bisect_root(k, float(cs[i - 1]), float(cs[i]), m, rel_tol=1e-11)
            assert abs(c_sec - c_ref) / c_ref < 1e-10
    assert seen == {PR.PICK_MODE, PR.PICK_POLE}


def test_classification_edge_cases():
    m = halfspace_model(700.0, 400.0, 2000.0)
    c_test = WL.uniform_grid(300.0, 1.0, 200)
    assert PR.classify(1.0, c_test, 0, m)[0] == PR.PICK_NONE
    assert PR.classify(1.0, c_test, -1, m)[0] == PR.PICK_NONE
    assert PR.classify(1.0, c_test, len(c_test), m)[0] == PR.PICK_NONE
    assert PR.classify(1.0, c_test, 100, m)[0] == PR.PICK_LEAKY      # c_test[100] = 400 = beta
    assert PR.classify(1.0, c_test, 10, m)[0] == PR.PICK_POLE        # no root in [309, 310]


def test_sign_relation_holds_across_a_thick_layer():
    # k h = 250 across the first layer: its P and SV solutions grow apart by
    # e^(k h (r - s)) ~ e^70 in one crossing, more than FP64 can hold, so the
    # relation holds only if each layer is crossed in short steps.
    m = WL.Model(np.array([20.0, 4.0]), np.array([380.0, 560.0, 950.0]),
                 np.array([200.0, 300.0, 500.0]), np.array([1800.0, 1900.0, 2000.0]))
    lam = 0.5
    k = 2 * math.pi / lam
    cs = np.linspace(60.0, 199.0, 40)
    sK = O.det_sign(k, cs, m)
    vals = set()
    for c, sk in zip(cs, sK):
        sD = (-1) ** bin(O.pole_mask(k, c, m)).count("1")
        vals.add(int(sk) * sD * PR._sgn(PR.secular(k, c, m)))
    assert vals == {1}


# ---------------------------------------------------------------------------
# Normal dispersion: for velocity-increasing profiles the first-mode phase
# velocity does not decrease with wavelength (Section 3.2 observes the
# curves of its data falling with decreasing wavelength)
# ---------------------------------------------------------------------------
def test_normal_dispersion_of_stored_oracle_curves():
    import json
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    fine = json.load(open(os.path.join(here, "fine_scale.json")))
    assert np.all(np.diff(np.array(fine["idx"])) >= 0)        # wavelengths ascending, picks never fall
    batch = json.load(open(os.path.join(here, "batch_sample.json")))
    inverted = WL.batch_case().meta["inverted"]
    falling = [e["model"] for e in batch["models"] if np.any(np.diff(np.array(e["idx"])) < 0)]
    # only models with a low-velocity layer may disperse inversely
    assert all(inverted[m] for m in falling)
    assert any(not inverted[e["model"]] for e in batch["models"])
