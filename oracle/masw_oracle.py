"""CPU oracle for the theoretical Rayleigh-wave dispersion curve.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check in __graft_entry__ and
the cpu_baseline leg of bench.py may import this module.  The library's product
path never calls it and shares no code with it.

What it computes (paper: Algorithm 1 "MASW Theoretical Dispersion Curve",
Section 2.1; the stiffness matrix method the paper names there):

* For one wavelength lambda (k = 2 pi / lambda) and one test velocity c, the
  global stiffness matrix K(k, c) of N elastic layers over an elastic
  half-space, of size 2(N+1) x 2(N+1), symmetric and heptadiagonal
  (Section 2.1, Section 3.1), is assembled by adding each layer's 4x4 element
  matrix at rows/cols 2j..2j+3 and the half-space's 2x2 matrix at 2N..2N+1.
* sign(det K) is taken as the sign of the real part of the determinant, from a
  dense LU with partial pivoting (numpy.linalg.slogdet, LAPACK getrf), which
  returns the phase and log|det| and so cannot overflow.
* The dispersion velocity of lambda is V[n] for the first n >= 1 whose sign
  differs from that of V[n-1] (Algorithm 1: the while loop compares the sign
  of the previous and the current determinant).
* A refined root: bisection on the same sign over [V[n-1], V[n]] until the
  bracket is no wider than 1e-9 V[n]; the midpoint is reported.

Everything is plain FP64 (complex128 for the matrices).  The c values are
vectorised in batches only to evaluate many independent determinants per numpy
call; the scan over them is the paper's linear scan in increasing c order.

Element matrices (not printed in the paper).  With r = sqrt(1 - c^2/alpha^2),
s = sqrt(1 - c^2/beta^2) (principal branch, taken from the real argument),
C_r = cosh(k h r), S_r = sinh(k h r), and likewise for s:

  D   = 2 (1 - C_r C_s) + (1/(r s) + r s) S_r S_s,     f = k rho c^2 / D
  k11 = f (C_r S_s/s - r S_r C_s)
  k12 = f (C_r C_s - r s S_r S_s - 1) - k rho beta^2 (1 + s^2)
  k13 = f (r S_r - S_s/s)
  k14 = f (C_s - C_r)
  k22 = f (S_r C_s/r - s C_r S_s)
  k24 = f (s S_s - S_r/r)

  K_layer = [[k11, k12, k13, k14], [k12, k22, -k14, k24],
             [k13, -k14, k11, -k12], [k14, k24, -k12, k22]]

and for the half-space (mu = rho beta^2):

  h11 = k mu r (1 - s^2)/(1 - r s),  h22 = k mu s (1 - s^2)/(1 - r s),
  h12 = k mu ((1 - s^2)/(1 - r s) - 2).

The degrees of freedom per interface are the horizontal displacement and -i
times the vertical displacement, which makes every layer matrix real for real
c.  At c = alpha or c = beta (r or s = 0) the entries have removable 0/0
forms; the oracle uses the limits S_r/r -> k h, r S_r -> 0, C_r -> 1.

Pins: tests/test_oracle_pins.py checks this module against the closed-form
Rayleigh root of a homogeneous half-space, a first-principles derivation of the
layer and half-space matrices from the P-SV equations of motion, the
condensation identity, short- and long-wavelength limits, scaling
invariances, structure, and high-precision determinants.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

import numpy as np

STATUS_FOUND = 0
STATUS_NOT_FOUND = 1
FLAG_POLE = 0x100
FLAG_NOISE = 0x200


# --------------------------------------------------------------------------
# Element matrices
# --------------------------------------------------------------------------
def _principal_sqrt(x: np.ndarray) -> np.ndarray:
    """sqrt of a real argument on the principal branch: x < 0 gives +i sqrt(-x).

    Built from the real value so that no signed-zero imaginary part can pick
    the other branch."""
    x = np.asarray(x, dtype=np.float64)
    a = np.sqrt(np.abs(x))
    return np.where(x >= 0.0, a + 0.0j, 1j * a)


def _cosh_terms(kh: float, x: np.ndarray):
    """For q = sqrt(x) (principal branch) return cosh(kh q), sinh(kh q)/q and
    q sinh(kh q), with their limits kh... at x = 0."""
    q = _principal_sqrt(x)
    ch = np.cosh(kh * q)
    sh = np.sinh(kh * q)
    zero = (q == 0)
    q_safe = np.where(zero, 1.0 + 0.0j, q)
    sh_over_q = np.where(zero, kh + 0.0j, sh / q_safe)
    q_sh = np.where(zero, 0.0j, q * sh)
    return q, ch, sh_over_q, q_sh


def layer_D(k: float, c: np.ndarray, h: float, alpha: float, beta: float) -> np.ndarray:
    """The denominator D of the layer matrix (complex128; real for real c)."""
    c = np.asarray(c, dtype=np.float64)
    xr = 1.0 - (c / alpha) ** 2
    xs = 1.0 - (c / beta) ** 2
    kh = k * h
    _, Cr, Sr_r, rSr = _cosh_terms(kh, xr)
    _, Cs, Ss_s, sSs = _cosh_terms(kh, xs)
    # (1/(r s) + r s) S_r S_s = (S_r/r)(S_s/s) + (r S_r)(s S_s)
    return 2.0 * (1.0 - Cr * Cs) + Sr_r * Ss_s + rSr * sSs


def layer_matrix(k: float, c: np.ndarray, h: float, alpha: float, beta: float,
                 rho: float) -> np.ndarray:
    """4x4 layer element matrix for every c; shape (..., 4, 4) complex128."""
    c = np.asarray(c, dtype=np.float64)
    xr = 1.0 - (c / alpha) ** 2          # r^2
    xs = 1.0 - (c / beta) ** 2           # s^2
    kh = k * h
    _, Cr, Sr_r, rSr = _cosh_terms(kh, xr)
    _, Cs, Ss_s, sSs = _cosh_terms(kh, xs)
    D = 2.0 * (1.0 - Cr * Cs) + Sr_r * Ss_s + rSr * sSs
    f = k * rho * c * c / D
    k11 = f * (Cr * Ss_s - rSr * Cs)
    k12 = f * (Cr * Cs - rSr * sSs - 1.0) - k * rho * beta * beta * (1.0 + xs)
    k13 = f * (rSr - Ss_s)
    k14 = f * (Cs - Cr)
    k22 = f * (Sr_r * Cs - sSs * Cr)
    k24 = f * (sSs - Sr_r)
    K = np.empty(c.shape + (4, 4), dtype=np.complex128)
    K[..., 0, 0] = k11; K[..., 0, 1] = k12; K[..., 0, 2] = k13; K[..., 0, 3] = k14
    K[..., 1, 0] = k12; K[..., 1, 1] = k22; K[..., 1, 2] = -k14; K[..., 1, 3] = k24
    K[..., 2, 0] = k13; K[..., 2, 1] = -k14; K[..., 2, 2] = k11; K[..., 2, 3] = -k12
    K[..., 3, 0] = k14; K[..., 3, 1] = k24; K[..., 3, 2] = -k12; K[..., 3, 3] = k22
    return K


def halfspace_matrix(k: float, c: np.ndarray, alpha: float, beta: float,
                     rho: float) -> np.ndarray:
    """2x2 half-space element matrix for every c; shape (..., 2, 2) complex128.
    Complex for c > beta (s imaginary)."""
    c = np.asarray(c, dtype=np.float64)
    r = _principal_sqrt(1.0 - (c / alpha) ** 2)
    s = _principal_sqrt(1.0 - (c / beta) ** 2)
    mu = rho * beta * beta
    one_m_s2 = 1.0 - s * s
    den = 1.0 - r * s
    H = np.empty(c.shape + (2, 2), dtype=np.complex128)
    H[..., 0, 0] = k * mu * r * one_m_s2 / den
    H[..., 1, 1] = k * mu * s * one_m_s2 / den
    H[..., 0, 1] = H[..., 1, 0] = k * mu * (one_m_s2 / den - 2.0)
    return H


def stiffness_matrix(k: float, c: np.ndarray, h: Sequence[float],
                     alpha: Sequence[float], beta: Sequence[float],
                     rho: Sequence[float]) -> np.ndarray:
    """Dense global stiffness matrix, shape (..., 2(N+1), 2(N+1)) complex128."""
    c = np.asarray(c, dtype=np.float64)
    N = len(h)
    n = 2 * (N + 1)
    K = np.zeros(c.shape + (n, n), dtype=np.complex128)
    for j in range(N):
        K[..., 2 * j:2 * j + 4, 2 * j:2 * j + 4] += layer_matrix(
            k, c, h[j], alpha[j], beta[j], rho[j])
    K[..., 2 * N:2 * N + 2, 2 * N:2 * N + 2] += halfspace_matrix(
        k, c, alpha[N], beta[N], rho[N])
    return K


# --------------------------------------------------------------------------
# Determinant sign (Algorithm 1's "sign(d)")
# --------------------------------------------------------------------------
def det_sign_logabs(k: float, c: np.ndarray, model) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(sigma, phase, log|det|) with sigma = sign(Re det K) in {-1, 0, +1}.

    Raises on a non-finite matrix: a NaN is an error, never a sign."""
    K = stiffness_matrix(k, c, model.h, model.alpha, model.beta, model.rho)
    if not np.all(np.isfinite(K)):
        raise FloatingPointError("non-finite stiffness matrix entry")
    phase, logabs = np.linalg.slogdet(K)
    sigma = np.sign(phase.real).astype(np.int8)
    return sigma, phase, logabs


def det_sign(k: float, c, model) -> np.ndarray:
    return det_sign_logabs(k, np.atleast_1d(np.asarray(c, np.float64)), model)[0]


def pole_mask(k: float, c: float, model) -> int:
    """Bit j set iff the layer-j denominator D_j(c) is negative."""
    mask = 0
    for j in range(model.n_layers):
        D = layer_D(k, np.array([c]), model.h[j], model.alpha[j], model.beta[j])[0]
        if D.real < 0.0:
            mask |= 1 << j
    return mask


@dataclass
class CurvePoint:
    idx: int          # grid index of the first sign change, -1 if none
    c_t: float        # c_test[idx] (the upper end of the bracket), NaN if none
    status: int       # STATUS_* | FLAG_POLE
    c_ref: float      # refined root (bisection midpoint), NaN if none
    evals: int        # determinant evaluations used by the scan (idx+1)


def first_change_index(signs, prev=None) -> int:
    """Algorithm 1's while loop over a sequence of signs: the first position i
    whose sign differs from the sign before it (signs[i-1], or `prev` for
    i = 0).  A zero sign differs from +1 and -1.  Returns -1 if none."""
    for i, s in enumerate(signs):
        if prev is not None and s != prev:
            return i
        prev = s
    return -1


def first_sign_change(k: float, c_test: np.ndarray, model, batch: int = 512) -> Tuple[int, int]:
    """Algorithm 1's linear scan: smallest n >= 1 with sign(V[n]) != sign(V[n-1]).

    Signs are computed `batch` test velocities at a time and scanned in order.
    Returns (n, evaluations); n = -1 when no change occurs in c_test."""
    n_c = c_test.shape[0]
    prev = None
    start = 0
    while start < n_c:
        stop = min(n_c, start + batch)
        sig = det_sign(k, c_test[start:stop], model)
        i = first_change_index(sig, prev)
        if i >= 0:
            return start + i, start + i + 1
        prev = sig[-1]
        start = stop
    return -1, n_c


def bisect_root(k: float, lo: float, hi: float, model, rel_tol: float = 1e-9) -> float:
    """Bisection on sign(Re det K) over [lo, hi] (signs differ at the ends)
    until hi - lo <= rel_tol * c_hi, where c_hi is the bracket's initial upper
    end; returns the midpoint."""
    s_lo = int(det_sign(k, lo, model)[0])
    tol = rel_tol * hi
    while hi - lo > tol:
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        s_mid = int(det_sign(k, mid, model)[0])
        if s_mid == s_lo:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def dispersion_point(lam: float, c_test: np.ndarray, model, refine: bool = True,
                     check_noise: bool = False) -> CurvePoint:
    """One wavelength of Algorithm 1, plus the refined root and pole flag.
    With check_noise, FLAG_NOISE marks a pick whose bracket has a point in the
    FP64 noise band (in_noise_band), tested only below the half-space's S
    velocity, where K is real."""
    k = 2.0 * np.pi / lam
    idx, evals = first_sign_change(k, c_test, model)
    if idx < 0:
        return CurvePoint(-1, float("nan"), STATUS_NOT_FOUND, float("nan"), evals)
    status = STATUS_FOUND
    if pole_mask(k, c_test[idx - 1], model) != pole_mask(k, c_test[idx], model):
        status |= FLAG_POLE
    if check_noise:
        beta_hs = model.beta[model.n_layers]
        if any(c < beta_hs and in_noise_band(lam, c, model) for c in (c_test[idx - 1], c_test[idx])):
            status |= FLAG_NOISE
    c_ref = bisect_root(k, float(c_test[idx - 1]), float(c_test[idx]), model) if refine else float("nan")
    return CurvePoint(idx, float(c_test[idx]), status, c_ref, evals)


def dispersion_curve(lambdas: Sequence[float], c_test: np.ndarray, model,
                     refine: bool = True, check_noise: bool = False):
    """Algorithm 1 over all wavelengths; returns a list of CurvePoint."""
    c_test = np.asarray(c_test, dtype=np.float64)
    return [dispersion_point(float(l), c_test, model, refine, check_noise) for l in lambdas]


def curve_arrays(points):
    """(idx int32, c_t f64, status int32, c_ref f64) arrays from CurvePoints."""
    idx = np.array([p.idx for p in points], dtype=np.int32)
    ct = np.array([p.c_t for p in points], dtype=np.float64)
    st = np.array([p.status for p in points], dtype=np.int32)
    cr = np.array([p.c_ref for p in points], dtype=np.float64)
    return idx, ct, st, cr


# --------------------------------------------------------------------------
# Misfit (Algorithm 2)
# --------------------------------------------------------------------------
def misfit(c_t: np.ndarray, c_e: np.ndarray) -> float:
    """Average relative error (1/l) sum |C_t - C_e| / C_e (Algorithm 2)."""
    c_t = np.asarray(c_t, np.float64)
    c_e = np.asarray(c_e, np.float64)
    return float(np.sum(np.abs(c_t - c_e) / c_e) / c_t.shape[0])


# --------------------------------------------------------------------------
# FP64 noise band
# --------------------------------------------------------------------------
def in_noise_band(lam: float, c: float, model, threshold: float = 1e-2) -> bool:
    """True iff the first-order relative error bound of an FP64 determinant,
    cond_2(K) * 2(N+1) * 2^-53, reaches `threshold` at this c."""
    k = 2.0 * np.pi / lam
    K = stiffness_matrix(k, np.array([c]), model.h, model.alpha, model.beta, model.rho)[0]
    n = K.shape[0]
    return bool(np.linalg.cond(K) * n * 2.0 ** -53 >= threshold)


# --------------------------------------------------------------------------
# Full sign map (every lambda x every c, no early exit)
# --------------------------------------------------------------------------
def sign_map(lambdas: Sequence[float], c_test: np.ndarray, model):
    """sigma and log|det| for every (lambda, c): arrays of shape (W, n_c)."""
    c_test = np.asarray(c_test, dtype=np.float64)
    W = len(lambdas)
    sig = np.empty((W, c_test.shape[0]), np.int8)
    la = np.empty((W, c_test.shape[0]), np.float64)
    for w, lam in enumerate(lambdas):
        s, _, l = det_sign_logabs(2.0 * np.pi / lam, c_test, model)
        sig[w] = s
        la[w] = l
    return sig, la
