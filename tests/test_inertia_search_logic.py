"""CPU check of the inertia-count search's control flow (MASW_SEARCH_INERTIA).

The rounds of the device search are re-stated here in plain Python: the
predicted window, the sampling round, the counts between the sampled points,
narrowing, the sign at a change (the parity of the count), and the walk of
Algorithm 1 where counts are not defined.  The counts come from dense
matrices (eigvalsh of the oracle's stiffness matrix, and of the interior
interfaces of equal sublayers), so this checks the search's logic against
the oracle's linear scan, independently of the GPU kernel (which the GPU
tests check against the walk and the oracle).
"""
import math

import numpy as np

import oracle.masw_oracle as O
import workloads as WL

EVENT = 1 << 31  # a count that ends the search on E (here: c at or above the half-space's S velocity)


def count_E(k, c, m):
    """E = s + 2P at c, or EVENT."""
    if c >= m.beta[m.n_layers]:
        return EVENT
    K = O.stiffness_matrix(k, np.array([c]), m.h, m.alpha, m.beta, m.rho)[0].real
    s = int((np.linalg.eigvalsh(K) < 0).sum())
    P = 0
    for j in range(m.n_layers):
        x = (c / m.beta[j]) ** 2 - 1.0
        if x <= 0.0:
            continue
        msub = int(k * m.h[j] * math.sqrt(x) / math.pi) + 1
        if msub < 2:
            continue
        KL = O.layer_matrix(k, np.array([c]), m.h[j] / msub, m.alpha[j], m.beta[j], m.rho[j])[0].real
        G = np.zeros((2 * (msub + 1), 2 * (msub + 1)))
        for i in range(msub):
            G[2 * i:2 * i + 4, 2 * i:2 * i + 4] += KL
        P += int((np.linalg.eigvalsh(G[2:-2, 2:-2]) < 0).sum())
    return s + 2 * P


def sign(k, c, m):
    return int(O.det_sign(k, c, m)[0])


def walk(k, c, m, start, carry):
    for i in range(start, len(c)):
        if sign(k, c[i], m) != carry:
            return i
    return -1


def spread(lo, hi, first, lanes=64):
    n, nl = hi - lo, lanes - first
    if n <= nl:
        return [lo + 1 + j for j in range(n)]
    return [lo + (n * (j + 1)) // nl for j in range(nl)]


def first_change(k, c, m, lo, hi, E_a):
    pts = spread(lo, hi, 0)
    Es = [count_E(k, c[p], m) for p in pts]
    f = next((i for i, E in enumerate(Es) if E != E_a), None)
    if f is None:
        return None
    return (lo if f == 0 else pts[f - 1]), pts[f], Es[f]


def search(k, c, m, pred=-1):
    """The device search's rounds; returns the pick (-1: none)."""
    n = len(c) - 1
    a, known, located, bound = 0, False, False, n
    if pred >= 1 and n >= 64:                       # P: predicted window
        w0 = max(0, min(pred - 32, n - 62))
        pts = [0, w0] + [w0 + j for j in range(1, 63)]
        Es = [count_E(k, c[p], m) for p in pts]
        E_a = Es[0]
        if E_a == EVENT:
            return walk(k, c, m, 1, sign(k, c[0], m))
        sig0, known = (-1 if E_a & 1 else 1), True
        if Es[1] != E_a:
            lo, hi, E_hi, located = 0, w0, Es[1], True
        else:
            f = next((i for i in range(2, 64) if Es[i] != E_a), None)
            if f is not None:
                lo, hi, E_hi, located = pts[f - 1], pts[f], Es[f], True
            else:
                a = w0 + 62
    if not located:
        pa = [a] + spread(a, n, 1)                  # A: sampled signs
        sa = ([sig0] if known else [sign(k, c[a], m)]) + [sign(k, c[p], m) for p in pa[1:]]
        if not known:
            sig0 = sa[0]
            if sig0 not in (1, -1):
                return walk(k, c, m, 1, sig0)
        f = next((i for i in range(1, len(pa)) if sa[i] != sig0), None)
        if f is not None:                           # B: counts between the samples
            pf, pb = pa[f], pa[f - 1]
            bound = pf
            q = [a, pb] + spread(pb, pf, 2)
            Es = [E_a if (i == 0 and known) else count_E(k, c[x], m) for i, x in enumerate(q)]
            if not known:
                E_a = Es[0]
                if E_a == EVENT:
                    return walk(k, c, m, a + 1, sig0)
            if Es[1] != E_a:
                lo, hi, E_hi = a, pb, Es[1]
            else:
                f2 = next((i for i in range(2, len(q)) if Es[i] != E_a), None)
                if f2 is None:
                    return walk(k, c, m, pb + 1, sig0)
                lo, hi, E_hi = q[f2 - 1], q[f2], Es[f2]
        else:                                       # counts over the rest of the grid
            p0 = [a] + spread(a, n, 1)
            E0 = [E_a if (i == 0 and known) else count_E(k, c[x], m) for i, x in enumerate(p0)]
            if not known:
                E_a = E0[0]
                if E_a == EVENT:
                    return walk(k, c, m, a + 1, sig0)
            f = next((i for i in range(1, len(p0)) if E0[i] != E_a), None)
            if f is None:
                return -1
            lo, hi, E_hi = p0[f - 1], p0[f], E0[f]
    while True:                                     # narrowing, the sign at the change
        while hi > lo + 1:
            r = first_change(k, c, m, lo, hi, E_a)
            if r is None:
                return walk(k, c, m, lo + 1, sig0)
            lo, hi, E_hi = r
        s = sign(k, c[hi], m) if E_hi == EVENT else (-1 if E_hi & 1 else 1)
        if s != sig0:
            return hi
        if E_hi == EVENT:
            return walk(k, c, m, hi + 1, sig0)
        E_a, lo, hi = E_hi, hi, bound
        r = first_change(k, c, m, lo, hi, E_a) if hi > lo else None
        if r is None:
            return walk(k, c, m, lo + 1, sig0) if bound < n else -1
        lo, hi, E_hi = r


def test_two_layer_case_with_and_without_predictions():
    wl = WL.two_layer_case()
    m, c = wl.models[0], wl.c_test
    p1 = p2 = -1
    for lam in wl.lambdas[0]:
        k = 2 * math.pi / lam
        want = O.first_sign_change(k, c, m)[0]
        assert search(k, c, m) == want, lam
        pred = -1 if p1 < 1 else (p1 if p2 < 1 else max(1, 2 * p1 - p2))
        assert search(k, c, m, pred) == want, (lam, pred)
        p2, p1 = p1, want


def test_poles_and_modes_first_and_grids_above_the_halfspace():
    m = WL.fine_scale_case().models[0]
    k = 2 * math.pi / 1.0
    c = WL.uniform_grid(50.0, 0.01, 115001)[:60001]
    # grids starting past a mode (126.5 m/s) and past a pole (154.0 m/s)
    for start in (7650, 10400):
        cc = c[start:start + 2001]
        assert search(k, cc, m) == O.first_sign_change(k, cc, m)[0]
    # a half-space on a grid that starts above its Rayleigh root: walked above beta
    beta = 400.0
    hs = WL.Model(np.zeros(0), np.array([math.sqrt(3) * beta]), np.array([beta]), np.array([2000.0]))
    cc = WL.uniform_grid(380.0, 0.5, 300)
    assert search(2 * math.pi / 5.0, cc, hs) == O.first_sign_change(2 * math.pi / 5.0, cc, hs)[0]
    # a prediction far off (before and after the pick) still gives the pick
    cc = c[:3001]
    want = O.first_sign_change(k, cc, m)[0]
    assert search(k, cc, m, pred=100) == want
    assert search(k, cc, m, pred=2900) == want
