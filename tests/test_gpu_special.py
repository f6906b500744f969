"""The device special functions of the sweep against high-precision references.

The probe library (tests/special_probe.hip, built with libmasw.so) runs the
exact device code of masw_special.hpp on arrays of arguments spanning the
ranges the layer loop uses; mpmath at 40 digits gives the references.
Bounds are in units of the format's unit roundoff u (2^-53 for FP64, 2^-24
for FP32):

* reciprocal: relative error <= 2u; reciprocal square root: <= 3u (the
  residual 1 - x y^2 is formed from the rounded product x y, an absolute
  error of about u that costs u/2 in the result, beside the final rounding
  and that of the reference); FP64 refines the hardware estimate, FP32 uses
  it alone;
  the FP64 hardware estimates themselves within 2^-21 relative, which the
  one-step third-order refinement needs (its error is the cube of the
  estimate's, 2^-63 at most);
* expm1(-y): relative error <= 4u (FP64) / 8u (FP32) for every y >= 0;
* sin^2 x and sin x cos x: error <= 4u |ref| + 2u (FP64) and 8u |ref| + 4u
  (FP32), i.e. relative where the value is of order one or small like x^2 or
  x near 0, absolute near the other zeros, whose position the rounded
  argument itself only fixes to about u x;
* (cosh sqrt(z) - 1)/z and sinh(sqrt z)/sqrt(z) for |z| <= 1 (cos and sin
  for z < 0): relative error <= 4u (FP64) / 8u (FP32).
"""
import ctypes
import os

import numpy as np
import pytest

mpmath = pytest.importorskip("mpmath")

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
PROBE = os.path.join(HERE, "libspecial_probe.so")
U64, U32 = 2.0 ** -53, 2.0 ** -24


@pytest.fixture(scope="module")
def probe(gpu):
    if not os.path.exists(PROBE):
        pytest.fail("tests/libspecial_probe.so is not built: run __graft_entry__.build()")
    lib = ctypes.CDLL(PROBE)
    lib.probe_special.restype = ctypes.c_int
    dp = ctypes.POINTER(ctypes.c_double)
    lib.probe_special.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, ctypes.c_int]

    def run(fp32, kind, x):
        x = np.ascontiguousarray(x, np.float64)
        y0, y1 = np.empty_like(x), np.empty_like(x)
        p = lambda a: a.ctypes.data_as(dp)
        rc = lib.probe_special(int(fp32), kind, p(x), p(y0), p(y1), int(x.shape[0]))
        assert rc == 0, f"probe failed with HIP error {rc}"
        return y0, y1
    return run


def _ref(fn, x):
    mpmath.mp.dps = 40
    return np.array([float(fn(mpmath.mpf(float(v)))) for v in x])


def _args_expm1(fp32):
    rng = np.random.default_rng(11)
    hi = 110.0 if fp32 else 800.0
    x = np.concatenate([[0.0], 10.0 ** rng.uniform(-300 if not fp32 else -30, 0, 3000),
                        rng.uniform(0, 1, 2000), rng.uniform(1, 40, 2000), rng.uniform(40, hi, 1000)])
    return x.astype(np.float32).astype(np.float64) if fp32 else x


def _args_trig(fp32):
    rng = np.random.default_rng(12)
    top = 1e4 if fp32 else float(2 ** 20)
    x = np.concatenate([[0.0], 10.0 ** rng.uniform(-300 if not fp32 else -30, 0, 2000),
                        rng.uniform(0, 10, 2000), rng.uniform(0, 1e3, 2000), rng.uniform(0, top, 2000)])
    return x.astype(np.float32).astype(np.float64) if fp32 else x


def _report(name, err, bound):
    worst = float(np.max(err / bound))
    print(f"{name}: worst error / bound = {worst:.3f}", flush=True)
    assert worst <= 1.0, name


@pytest.mark.parametrize("fp32", [0, 1])
def test_expm1_neg(probe, fp32):
    y = _args_expm1(fp32)
    got, _ = probe(fp32, 0, y)
    want = _ref(lambda v: mpmath.expm1(-v), y)
    u = U32 if fp32 else U64
    zero = want == 0.0
    assert np.all(got[zero] == 0.0)
    rel = np.abs(got[~zero] - want[~zero]) / np.abs(want[~zero])
    _report(f"expm1_neg fp32={fp32}", rel, (8 if fp32 else 4) * u)


@pytest.mark.parametrize("fp32", [0, 1])
def test_sin2_sincos(probe, fp32):
    x = _args_trig(fp32)
    s2, sc = probe(fp32, 1, x)
    want_s2 = _ref(lambda v: mpmath.sin(v) ** 2, x)
    want_sc = _ref(lambda v: mpmath.sin(v) * mpmath.cos(v), x)
    u = U32 if fp32 else U64
    k_rel, k_abs = (8, 4) if fp32 else (4, 2)
    _report(f"sin^2 fp32={fp32}", np.abs(s2 - want_s2), k_rel * u * np.abs(want_s2) + k_abs * u)
    _report(f"sin cos fp32={fp32}", np.abs(sc - want_sc), k_rel * u * np.abs(want_sc) + k_abs * u)
    # relative accuracy where the values are ~x^2 and ~x, down to where x^2
    # leaves the format's normal range
    tiny = 1e-18 if fp32 else 1e-150
    sel = (x < 1e-3) & (x > tiny)
    if np.any(sel):
        _report(f"sin^2 small x fp32={fp32}", np.abs(s2[sel] - want_s2[sel]) / want_s2[sel], k_rel * u)
        _report(f"sin cos small x fp32={fp32}", np.abs(sc[sel] - want_sc[sel]) / want_sc[sel], k_rel * u)


def _ch(v):
    # (cosh sqrt(v) - 1)/v = sum_n v^n/(2n+2)!, summed at 40 digits (the
    # closed form cancels completely for tiny |v|)
    v = mpmath.mpf(v)
    return mpmath.fsum(v ** n / mpmath.factorial(2 * n + 2) for n in range(30))


def _shc(v):
    # sinh(sqrt v)/sqrt(v) = sum_n v^n/(2n+1)!
    v = mpmath.mpf(v)
    return mpmath.fsum(v ** n / mpmath.factorial(2 * n + 1) for n in range(30))


@pytest.mark.parametrize("fp32", [0, 1])
def test_cosh_sinh_series(probe, fp32):
    """(cosh sqrt(z) - 1)/z and sinh(sqrt z)/sqrt(z) on |z| <= 1, both signs:
    relative error <= 4u (FP64) / 8u (FP32); both lie in [0.45, 1.2] there."""
    rng = np.random.default_rng(14)
    tiny = 10.0 ** rng.uniform(-30 if fp32 else -300, 0, 1000)
    z = np.concatenate([[0.0, 1.0, -1.0], rng.uniform(-1, 1, 4000), tiny, -tiny,
                        1.0 - 10.0 ** rng.uniform(-16, -1, 200), -1.0 + 10.0 ** rng.uniform(-16, -1, 200)])
    if fp32:
        z = z.astype(np.float32).astype(np.float64)
    z = z[np.abs(z) <= 1.0]
    ch, shc = probe(fp32, 6, z)
    # the series against the closed forms where those do not cancel
    mpmath.mp.dps = 40
    for v in (1.0, -1.0, 0.5, -0.5):
        r = mpmath.sqrt(abs(mpmath.mpf(v)))
        assert abs(_ch(v) - ((mpmath.cosh(r) if v > 0 else mpmath.cos(r)) - 1) / v) < 1e-35
        assert abs(_shc(v) - (mpmath.sinh(r) if v > 0 else mpmath.sin(r)) / r) < 1e-35
    u = U32 if fp32 else U64
    k = 8 if fp32 else 4
    want_ch, want_shc = _ref(_ch, z), _ref(_shc, z)
    _report(f"ch fp32={fp32}", np.abs(ch - want_ch) / want_ch, k * u)
    _report(f"shc fp32={fp32}", np.abs(shc - want_shc) / want_shc, k * u)


@pytest.mark.parametrize("fp32", [0, 1])
def test_reciprocal_and_rsqrt(probe, fp32):
    rng = np.random.default_rng(13)
    lo, hi = (-30, 30) if fp32 else (-300, 300)
    mag = 10.0 ** rng.uniform(lo, hi, 6000)
    d = np.concatenate([mag, -mag[:3000], [1.0, -1.0, 2.0, 0.5, 3.0]])
    if fp32:
        d = d.astype(np.float32).astype(np.float64)
    u = U32 if fp32 else U64
    want_r = _ref(lambda v: 1 / v, d)
    got, _ = probe(fp32, 2, d)
    _report(f"rcp fp32={fp32}", np.abs(got - want_r) / np.abs(want_r), 2 * u)
    x = np.abs(d)
    want_q = _ref(lambda v: 1 / mpmath.sqrt(v), x)
    got, _ = probe(fp32, 3, x)
    _report(f"rsqrt fp32={fp32}", np.abs(got - want_q) / np.abs(want_q), 3 * u)
    if not fp32:
        seed, _ = probe(0, 4, d)
        _report("v_rcp_f64 estimate", np.abs(seed - want_r) / np.abs(want_r), 2.0 ** -21)
        seed, _ = probe(0, 5, x)
        _report("v_rsq_f64 estimate", np.abs(seed - want_q) / np.abs(want_q), 2.0 ** -21)
