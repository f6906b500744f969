"""CPU oracle for the propagator secular function and the zero/pole
classification of a determinant sign change.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check in __graft_entry__ and
the cpu_baseline leg of bench.py may import this module.  The library's product
path never calls it and shares no code with it.

Why.  The search of Algorithm 1 (Section 2.1) reports where sign(det K)
changes along c.  det K of the stiffness formulation carries each layer's
denominator D_j (see masw_oracle's header), so it changes sign both at a zero
of the dispersion function (a surface-wave mode) and where some D_j changes
sign (a pole: a resonance of that layer with both faces fixed).  An
independent formulation of the dispersion function, with no denominators,
tells the two apart and gives a second value of the root.

What it computes.  The P-SV equations of motion of a layer, for the state
v = (u_x, -i u_z, tau_xz / (k mu_ref), -i tau_zz / (k mu_ref)) of a plane wave
exp(i k (x - c t)) and the depth variable zeta = k z (z down), are the real
first-order system dv/dzeta = A v with

    A[0,1] = 1,              A[0,2] = mu_ref / mu,
    A[1,0] = -lambda / M,    A[1,3] = mu_ref / M,
    A[2,0] = (4 mu (lambda + mu) / M - rho c^2) / mu_ref,    A[2,3] = lambda / M,
    A[3,1] = -rho c^2 / mu_ref,                              A[3,2] = -1,

(mu = rho beta^2, M = rho alpha^2, lambda = M - 2 mu; every other entry 0),
whose eigenvalues are +-r and +-s, r^2 = 1 - c^2/alpha^2, s^2 = 1 - c^2/beta^2.
mu_ref is the half-space's rho beta^2.  For c below the half-space's S
velocity, the half-space's solutions that decay with depth are spanned by

    P:  (1, r, -2 r m, (g - 2) m),   SV:  (s, 1, -(2 - g) m, -2 s m)

(r, s > 0 of the half-space, g = c^2/beta^2, m = mu / mu_ref = 1 there).
That pair of solutions, continued upward across every layer by the
propagator exp(-A k h) (continuity of displacement and traction at each
interface), must be traction-free at the surface.  So the secular function
is

    F(c) = det of the traction rows (2 and 3) of the continued pair,

which vanishes exactly at the modes.  To keep the pair numerically
independent, each layer is crossed in equal steps of at most one unit of
k dz max(|r|, |s|), and after every step the pair is replaced by an
orthonormal basis of its span with the same orientation (QR with a positive
diagonal of R).  That divides F by a positive factor, so the sign of F and
its zeros are unchanged.  Each step's matrix exponential is
scipy.linalg.expm.

Classification of the change at grid index idx (bracket [c_test[idx-1],
c_test[idx]]):

    PICK_MODE   F has different signs at the two ends (zero counts as a sign);
                c_sec = bisection of F to a bracket no wider than
                1e-12 c_test[idx], midpoint;
    PICK_POLE   F has the same sign at both ends: no mode in the bracket
                (an odd number of them would change the sign of F), so a
                sign change of det K there is a pole;
    PICK_LEAKY  c_test[idx] >= the half-space's beta: the decaying pair is
                not real there, no classification;
    PICK_NONE   idx < 1 or idx >= len(c_test) (no bracket).

Pins: tests/test_oracle_pins.py checks A against the physical P-SV system,
the pair above against A's eigenvectors, F against the Rayleigh function of a
homogeneous half-space and its closed-form root, and F's zeros and roots
against a 30-digit propagator determinant (mpmath, no orthonormalisation).
It also checks that sign(det K) prod_j sign(D_j) sign(F) is one constant
between the stiffness and propagator formulations, including across a layer
too thick to cross in one step, and that the classes agree with the stiffness
denominators' sign changes.
"""
from __future__ import annotations

import math
from typing import Tuple

import numpy as np
import scipy.linalg as sla

PICK_MODE = 0
PICK_POLE = 1
PICK_LEAKY = 2
PICK_NONE = 3


def system_matrix(c: float, alpha: float, beta: float, rho: float, mu_ref: float) -> np.ndarray:
    """A of one layer (see the module header)."""
    mu = rho * beta * beta
    M = rho * alpha * alpha
    lam = M - 2.0 * mu
    A = np.zeros((4, 4))
    A[0, 1] = 1.0
    A[0, 2] = mu_ref / mu
    A[1, 0] = -lam / M
    A[1, 3] = mu_ref / M
    A[2, 0] = (4.0 * mu * (lam + mu) / M - rho * c * c) / mu_ref
    A[2, 3] = lam / M
    A[3, 1] = -rho * c * c / mu_ref
    A[3, 2] = -1.0
    return A


def decaying_pair(c: float, alpha: float, beta: float) -> np.ndarray:
    """4 x 2: the half-space's P and SV solutions decaying with depth (c < beta)."""
    g = (c / beta) ** 2
    r = math.sqrt(1.0 - (c / alpha) ** 2)
    s = math.sqrt(1.0 - g)
    return np.array([[1.0, s], [r, 1.0], [-2.0 * r, -(2.0 - g)], [g - 2.0, -2.0 * s]])


def _orthonormal(V: np.ndarray) -> np.ndarray:
    Q, R = np.linalg.qr(V)
    return Q * np.sign(np.diag(R))


def secular(k: float, c: float, model) -> float:
    """F(c) for wavenumber k; requires c < the half-space's beta."""
    N = model.n_layers
    mu_ref = model.rho[N] * model.beta[N] ** 2
    V = _orthonormal(decaying_pair(c, model.alpha[N], model.beta[N]))
    for j in range(N - 1, -1, -1):
        a, b, rho, h = model.alpha[j], model.beta[j], model.rho[j], model.h[j]
        A = system_matrix(c, a, b, rho, mu_ref)
        q = math.sqrt(max(abs(1.0 - (c / a) ** 2), abs(1.0 - (c / b) ** 2)))
        x = k * h
        steps = max(1, math.ceil(x * q))
        P = sla.expm(-A * (x / steps))
        for _ in range(steps):
            V = _orthonormal(P @ V)
    return float(V[2, 0] * V[3, 1] - V[2, 1] * V[3, 0])


def _sgn(v: float) -> int:
    v = float(v)
    return int(v > 0.0) - int(v < 0.0)


def classify(lam: float, c_test: np.ndarray, idx: int, model, rel_tol: float = 1e-12) -> Tuple[int, float]:
    """(class, c_sec) of the sign change at grid index idx (module header)."""
    if idx < 1 or idx >= len(c_test):
        return PICK_NONE, float("nan")
    lo, hi = float(c_test[idx - 1]), float(c_test[idx])
    if hi >= model.beta[model.n_layers]:
        return PICK_LEAKY, float("nan")
    k = 2.0 * math.pi / lam
    s_lo, s_hi = _sgn(secular(k, lo, model)), _sgn(secular(k, hi, model))
    if s_lo == s_hi:
        return PICK_POLE, float("nan")
    tol = rel_tol * hi
    while hi - lo > tol:
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if _sgn(secular(k, mid, model)) == s_lo:
            lo = mid
        else:
            hi = mid
    return PICK_MODE, 0.5 * (lo + hi)
