"""Parity of the zero/pole classification (masw_classify_picks, through the C
ABI) with the oracle's propagator secular function (oracle/propagator.py).

Classes must be equal.  A mode's c_sec must agree with the oracle's within
1e-9 relative (both narrow the bracket to 1e-12 c), and with the stiffness
path's refined root c_ref within 1.5e-9 (that refinement stops at a bracket of
1e-9 c).  At full size, where the oracle is too slow for every pick, two
independent formulations are compared instead: the class against the
stiffness path's pole flag (from the layer denominators), and c_sec against
c_ref.
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import propagator as PR
import paper_2003_02256_amd as M
import workloads as WL

pytestmark = pytest.mark.gpu
SEC_TOL = 1e-9
REF_TOL = 1.5e-9


@pytest.fixture(scope="module")
def ctx(gpu):
    c = M.Context(0, 2 << 30)
    yield c
    c.close()


def _expand(models, lambdas):
    """(model, lambda) of every flattened wavelength."""
    return [(m, float(l)) for m, lams in zip(models, lambdas) for l in lams]


def _check_vs_oracle(where, cls, sec, c, pairs, idx, rows):
    for w in rows:
        m, lam = pairs[w]
        want_cls, want_sec = PR.classify(lam, c, int(idx[w]), m)
        assert cls[w] == want_cls, (where, w, lam, int(idx[w]), int(cls[w]), want_cls)
        if want_cls == PR.PICK_MODE:
            assert abs(sec[w] - want_sec) <= SEC_TOL * want_sec, (where, w, sec[w], want_sec)
        else:
            assert np.isnan(sec[w]), (where, w, sec[w])


def _check_vs_stiffness(where, cls, sec, c, status, idx, c_ref, beta_hs):
    found = (status & 0xFF) == M.MASW_STATUS_FOUND
    pole = (status & M.MASW_FLAG_POLE) != 0
    leaky = found & (c[np.clip(idx, 0, len(c) - 1)] >= beta_hs)
    assert np.all(cls[~found] == M.MASW_PICK_NONE), where
    assert np.all(cls[leaky] == M.MASW_PICK_LEAKY), where
    inside = found & ~leaky
    # the propagator's class and the layer denominators agree on every pick
    assert np.all((cls[inside] == M.MASW_PICK_POLE) == pole[inside]), where
    assert np.all(np.isin(cls[inside], (M.MASW_PICK_MODE, M.MASW_PICK_POLE))), where
    mode = cls == M.MASW_PICK_MODE
    rel = np.abs(sec[mode] - c_ref[mode]) / c_ref[mode]
    assert rel.size == 0 or rel.max() <= REF_TOL, (where, rel.max())
    return int(mode.sum()), int((cls == M.MASW_PICK_POLE).sum()), int(leaky.sum())


def test_fine_scale_picks(ctx):
    wl = WL.fine_scale_case()
    m, lams, c = wl.models[0], wl.lambdas[0], wl.c_test
    C_t, idx, st, c_ref = ctx.curve(c, lams, m, prec=M.MASW_PREC_FP64)
    cls, sec = ctx.classify(c, [m], [lams], idx)
    st_cls = ctx.stats()
    # work counters: 64 evaluations per round, N = 20 layers each, at least
    # one step per layer crossed
    assert st_cls["classify_evals"] > 0 and st_cls["classify_evals"] % 64 == 0
    assert st_cls["classify_layers"] == 20 * st_cls["classify_evals"]
    assert st_cls["classify_steps"] >= st_cls["classify_layers"]
    assert st_cls["sweep_ms"] > 0.0 and st_cls["useful_evals"] == 0
    counts = _check_vs_stiffness("fine-scale", cls, sec, c, st, idx, c_ref, m.beta[-1])
    print(f"fine-scale picks: mode, pole, leaky = {counts}", flush=True)
    assert counts[0] > 0
    pairs = _expand([m], [lams])
    _check_vs_oracle("fine-scale", cls, sec, c, pairs, idx, range(0, len(lams), 111))


def test_modes_and_poles_along_a_grid(ctx):
    # later sign changes of det K at short wavelengths include layer
    # resonances (poles); every one of the first six per wavelength, from the
    # oracle's dense determinant, is classed as the oracle classes it
    wl = WL.fine_scale_case()
    m = wl.models[0]
    c = WL.uniform_grid(100.0, 2.0, 150)
    lams, idx = [], []
    for lam in (1.0, 3.0):
        s = O.det_sign(2 * math.pi / lam, c, m)
        ch = [i for i in range(1, len(s)) if s[i] != s[i - 1]][:6]
        lams += [lam] * len(ch)
        idx += ch
    lams, idx = np.array(lams), np.array(idx, np.int32)
    cls, sec = ctx.classify(c, [m], [lams], idx)
    pairs = _expand([m], [lams])
    _check_vs_oracle("grid changes", cls, sec, c, pairs, idx, range(len(lams)))
    for w, (mm, lam) in enumerate(pairs):
        k = 2 * math.pi / lam
        pole = O.pole_mask(k, c[idx[w] - 1], mm) != O.pole_mask(k, c[idx[w]], mm)
        assert (cls[w] == M.MASW_PICK_POLE) == pole
    assert set(cls.tolist()) == {M.MASW_PICK_MODE, M.MASW_PICK_POLE}


def test_batch_sample_picks(ctx):
    wl = WL.batch_case(n_models=16, seed=13)
    C_t, idx, st, c_ref = ctx.batch(wl.c_test, wl.models, wl.lambdas, prec=M.MASW_PREC_FP64)
    cls, sec = ctx.classify(wl.c_test, wl.models, wl.lambdas, idx)
    pairs = _expand(wl.models, wl.lambdas)
    beta_hs = np.array([m.beta[-1] for m, _ in pairs])
    counts = _check_vs_stiffness("batch sample", cls, sec, wl.c_test, st, idx, c_ref, beta_hs)
    print(f"batch sample picks: mode, pole, leaky = {counts}", flush=True)
    off = np.concatenate([[0], np.cumsum([len(l) for l in wl.lambdas])])
    rows = [int(off[i] + (i % 2) * (off[i + 1] - off[i] - 1)) for i in range(len(wl.models))]
    _check_vs_oracle("batch sample", cls, sec, wl.c_test, pairs, idx, rows)


def test_full_batch_against_the_stiffness_path(ctx):
    wl = WL.batch_case()
    C_t, idx, st, c_ref = ctx.batch(wl.c_test, wl.models, wl.lambdas, prec=M.MASW_PREC_FP64)
    cls, sec = ctx.classify(wl.c_test, wl.models, wl.lambdas, idx)
    beta_hs = np.repeat([m.beta[-1] for m in wl.models], [len(l) for l in wl.lambdas])
    counts = _check_vs_stiffness("full batch", cls, sec, wl.c_test, st, idx, c_ref, beta_hs)
    print(f"full batch ({len(idx)} wavelengths): mode, pole, leaky = {counts}", flush=True)


def _rayleigh_speed(alpha, beta):
    b = (beta / alpha) ** 2
    roots = np.roots([1.0, -8.0, 24.0 - 16.0 * b, -16.0 * (1.0 - b)])
    xi = [r.real for r in roots if abs(r.imag) < 1e-12 and 0.0 < r.real < 1.0][0]
    return beta * math.sqrt(xi)


def test_edge_cases(ctx):
    hs = WL.Model(np.zeros(0), np.array([700.0]), np.array([400.0]), np.array([2000.0]))
    c = WL.uniform_grid(300.0, 0.5, 203)           # 300 .. 401, crosses beta = 400
    cR = _rayleigh_speed(700.0, 400.0)
    i_root = int(np.searchsorted(c, cR))
    thick = WL.Model(np.array([2.0e5]), np.array([900.0, 1900.0]), np.array([500.0, 1000.0]),
                     np.array([1900.0, 2000.0]))
    lam = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0])   # 7: not a multiple of the wavefronts per group
    idx_hs = np.array([i_root, 0, -1, len(c), 202, i_root - 20, 1], np.int32)
    cls, sec = ctx.classify(c, [hs], [lam], idx_hs)
    assert cls.tolist() == [M.MASW_PICK_MODE, M.MASW_PICK_NONE, M.MASW_PICK_NONE, M.MASW_PICK_NONE,
                            M.MASW_PICK_LEAKY, M.MASW_PICK_POLE, M.MASW_PICK_POLE]
    assert abs(sec[0] - cR) / cR < 1e-11
    assert np.isnan(sec[1:]).all()
    st = ctx.stats()                 # a half-space has no layer to cross
    assert st["classify_evals"] > 0 and st["classify_layers"] == 0 and st["classify_steps"] == 0
    # a layer that would need more than 65536 steps is not crossed
    cls, sec = ctx.classify(c, [thick], [lam[:1]], np.array([10], np.int32))
    assert cls.tolist() == [M.MASW_PICK_UNRESOLVED] and np.isnan(sec[0])
    # an empty wavelength list is a no-op
    cls, sec = ctx.classify(c, [hs], [np.zeros(0)], np.zeros(0, np.int32))
    assert cls.shape == (0,)


def test_device_pointers_match_host_and_validate_on_device(ctx):
    import torch
    dev = torch.device("cuda:0")
    wl = WL.batch_case(n_models=3, seed=5)
    C_t, idx, st, c_ref = ctx.batch(wl.c_test, wl.models, wl.lambdas, prec=M.MASW_PREC_FP64)
    cls_h, sec_h = ctx.classify(wl.c_test, wl.models, wl.lambdas, idx)
    arrs = M.flatten_models(wl.models, wl.lambdas)
    W = int(arrs[-1].shape[0])

    def run(arrs):
        td = [torch.as_tensor(a, device=dev) for a in arrs]
        cls = torch.full((W,), -9, dtype=torch.int32, device=dev)
        sec = torch.empty(W, dtype=torch.float64, device=dev)
        M.masw_classify_picks(ctx.ctx, torch.as_tensor(wl.c_test, device=dev), *td,
                              torch.as_tensor(idx, device=dev), 0, None, cls, sec)
        torch.cuda.synchronize()
        return cls.cpu().numpy(), sec.cpu().numpy()

    cls_d, sec_d = run(arrs)
    assert np.array_equal(cls_d, cls_h)
    assert np.array_equal(np.isnan(sec_d), np.isnan(sec_h))
    ok = ~np.isnan(sec_h)
    assert np.array_equal(sec_d[ok], sec_h[ok])
    # model 1 made invalid (alpha < beta in its first layer): only its
    # wavelengths report MASW_PICK_INVALID
    bad = list(arrs)
    bad[2] = arrs[2].copy()
    r0 = int(arrs[0][1]) + 1
    bad[2][r0] = 0.5 * arrs[3][r0]
    cls_b, _ = run(bad)
    lo, hi = int(arrs[5][1]), int(arrs[5][2])
    has_bracket = idx[lo:hi] >= 1            # no bracket (NONE) takes precedence
    assert has_bracket.any()
    assert np.all(cls_b[lo:hi][has_bracket] == M.MASW_PICK_INVALID)
    assert np.all(cls_b[lo:hi][~has_bracket] == M.MASW_PICK_NONE)
    assert np.array_equal(cls_b[:lo], cls_h[:lo]) and np.array_equal(cls_b[hi:], cls_h[hi:])
