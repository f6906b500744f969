"""CPU pins of the facts the inertia-count search (MASW_SEARCH_INERTIA) rests
on, from dense matrices and plain scans, independent of both searches.

* Below the half-space's S velocity K is real symmetric and
  sign(det K) = (-1)^s, s = the number of negative eigenvalues of K
  (eigvalsh of the oracle's dense matrix against the oracle's slogdet sign).
* The fixed-face mode count of a layer, P_j(c), computed by cutting the
  layer into floor(k h sqrt(c^2/beta^2 - 1)/pi) + 1 sublayers and counting
  the negative eigenvalues of their interior interfaces, equals the number
  of sign changes of the layer's denominator D_j on a fine scan of (0, c]
  (the poles of det K), and is 0 below the Rayleigh bound.
* J = s + P (the Wittrick-Williams count of modes below c) and P are
  non-decreasing in c, so E = s + 2P is too.
"""
import math

import numpy as np
import pytest

import oracle.masw_oracle as O
import workloads as WL


def neg_count(A):
    return int((np.linalg.eigvalsh(A) < 0.0).sum())


def s_count(k, c, m):
    K = O.stiffness_matrix(k, np.array([c]), m.h, m.alpha, m.beta, m.rho)[0]
    assert np.all(K.imag == 0.0)
    return neg_count(K.real)


def sublayers(k, c, h, beta):
    x = (c / beta) ** 2 - 1.0
    return 1 if x <= 0.0 else int(k * h * math.sqrt(x) / math.pi) + 1


def P_layer(k, c, h, a, b, rho):
    """Negative eigenvalues of the interior interfaces of m equal sublayers."""
    msub = sublayers(k, c, h, b)
    if msub == 1:
        return 0
    KL = O.layer_matrix(k, np.array([c]), h / msub, a, b, rho)[0].real
    n = 2 * (msub + 1)
    G = np.zeros((n, n))
    for i in range(msub):
        G[2 * i:2 * i + 4, 2 * i:2 * i + 4] += KL
    return neg_count(G[2:-2, 2:-2])


def D_sign_changes(k, c_hi, h, a, b, n=40000):
    """Sign changes of D_j on a uniform scan of [beta/2, c_hi] (the poles below
    c_hi: none lie below beta, where D_j > 0; D_j -> 0 as c -> 0, so the scan
    starts away from 0)."""
    cs = np.linspace(0.5 * b, c_hi, n)
    D = O.layer_D(k, cs, h, a, b).real
    assert D[0] > 0.0
    sg = np.sign(D)
    return int(np.sum(sg[1:] != sg[:-1]))


CASES = [("two-layer", WL.two_layer_case, (1.0, 4.05, 40.0)),
         ("fine-scale", WL.fine_scale_case, (1.0, 5.245248678946673, 30.0))]


@pytest.mark.parametrize("name,make,lams", CASES)
def test_parity_of_negative_eigenvalues_is_the_determinant_sign(name, make, lams):
    m = make().models[0]
    bhs = m.beta[m.n_layers]
    cs = np.linspace(55.0, bhs * 0.999, 120)
    for lam in lams:
        k = 2 * math.pi / lam
        sig = O.det_sign(k, cs, m)
        for c, sg in zip(cs, sig):
            assert (-1) ** s_count(k, float(c), m) == sg, (name, lam, c)


def test_sublayer_count_equals_the_denominator_zeros():
    m = WL.fine_scale_case().models[0]
    for lam in (1.0, 3.0):
        k = 2 * math.pi / lam
        for j in (0, 3, 10):
            h, a, b, rho = m.h[j], m.alpha[j], m.beta[j], m.rho[j]
            for c in np.linspace(b * 1.01, 700.0, 7):
                want = D_sign_changes(k, float(c), h, a, b)
                assert P_layer(k, float(c), h, a, b, rho) == want, (lam, j, c, want)
                if k * h * math.sqrt((c / b) ** 2 - 1) <= math.pi:
                    assert want == 0          # the Rayleigh bound


@pytest.mark.parametrize("name,make,lams", CASES)
def test_mode_and_pole_counts_never_decrease(name, make, lams):
    m = make().models[0]
    bhs = m.beta[m.n_layers]
    cs = np.linspace(50.0, bhs * 0.9999, 400)
    for lam in lams:
        k = 2 * math.pi / lam
        prev = None
        for c in cs:
            s = s_count(k, float(c), m)
            P = sum(P_layer(k, float(c), m.h[j], m.alpha[j], m.beta[j], m.rho[j]) for j in range(m.n_layers))
            if prev is not None:
                assert s + P >= prev[0] and P >= prev[1], (name, lam, c, s, P, prev)
            prev = (s + P, P)
