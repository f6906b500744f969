"""The no-alloc entry point (masw_dispersion_curve_noalloc) against
masw_dispersion_curve, through the C ABI: two calls in a row, the second with
a smaller input, each bitwise equal to the allocating entry point's outputs
on the same device-resident inputs; and a request beyond the scratch limit
refused before any work."""
import numpy as np
import pytest

import paper_2003_02256_amd as M
import workloads as WL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev(gpu):
    import torch
    return torch, torch.device("cuda:0")


def _dev(torch, dev, wl, lam):
    t = lambda x: torch.as_tensor(np.ascontiguousarray(x, np.float64), device=dev)
    m = wl.models[0]
    return [t(wl.c_test), t(lam), t(m.h), t(m.alpha), t(m.beta), t(m.rho)]


def _outs(torch, dev, W):
    return (torch.full((W,), -1.0, dtype=torch.float64, device=dev), torch.full((W,), -9, dtype=torch.int32, device=dev),
            torch.full((W,), -9, dtype=torch.int32, device=dev), torch.full((W,), -1.0, dtype=torch.float64, device=dev))


def _run(fn, ctx, args, prec, flags, outs, torch):
    fn(ctx.ctx, *args, prec, flags, None, *outs)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


@pytest.mark.parametrize("prec,flags", [(M.MASW_PREC_FP64, 0), (M.MASW_PREC_SPLIT, 0),
                                        (M.MASW_PREC_FP64, M.MASW_SEARCH_INERTIA)])
def test_noalloc_equals_the_allocating_call_twice(torch_dev, prec, flags):
    torch, dev = torch_dev
    big = WL.fine_scale_case()                     # 1000 wavelengths, 115,001 velocities, 20 layers
    small = WL.two_layer_case()                    # 30 wavelengths, 801 velocities, 2 layers
    with M.Context(0, 64 << 20) as ctx:
        for wl, lam in ((big, big.lambdas[0]), (small, small.lambdas[0])):
            args = _dev(torch, dev, wl, lam)
            W = len(lam)
            want = _run(M.masw_dispersion_curve, ctx, args, prec, flags, _outs(torch, dev, W), torch)
            got = _run(M.masw_dispersion_curve_noalloc, ctx, args, prec, flags, _outs(torch, dev, W), torch)
            for x, y, what in zip(want, got, ("C_t", "idx", "status", "c_ref")):
                np.testing.assert_array_equal(y, x, err_msg=f"{wl.name} {what}")
            assert np.all(got[1] >= 0) and np.all(got[2] == 0)
            print(f"noalloc {wl.name} prec={prec} flags={flags}: {W} wavelengths equal", flush=True)


def test_noalloc_refuses_a_request_beyond_the_scratch(torch_dev):
    torch, dev = torch_dev
    wl = WL.two_layer_case()
    n_c = (M.MASW_NOALLOC_SCRATCH_BYTES // 4) + 1024          # the FP32 grid alone exceeds the scratch
    c = WL.uniform_grid(50.0, 400.0 / n_c, n_c)
    lam = wl.lambdas[0][:3]
    t = lambda x: torch.as_tensor(np.ascontiguousarray(x, np.float64), device=dev)
    m = wl.models[0]
    outs = _outs(torch, dev, 3)
    with M.Context(0, 64 << 20) as ctx:
        with pytest.raises(M.MaswError) as e:
            M.masw_dispersion_curve_noalloc(ctx.ctx, t(c), t(lam), t(m.h), t(m.alpha), t(m.beta), t(m.rho),
                                            M.MASW_PREC_FP64, 0, None, *outs)
        assert e.value.code == M.MASW_ENOMEM and "scratch" in str(e.value)
        torch.cuda.synchronize()
        assert outs[1].cpu().tolist() == [-9, -9, -9]       # nothing ran
