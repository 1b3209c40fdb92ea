"""lrt_march_noalloc through the C ABI against lrt_march (the same kernels; the
partial sums in the library's static scratch instead of an allocated
workspace): bitwise the same wall intensities and band integrals, in both
precisions, on two calls in a row, the second on a smaller input (the short
last band, then a context with fewer rays); sizes beyond the scratch are
rejected."""
import numpy as np
import pytest

from paper_2604_11856_amd import lrt, synth
from parity_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch


def _both(ctx, band, prec, torch):
    sz = ctx.sizes()
    eta, kap, esc = ctx.coeffs_torch(band, prec)
    nb = ctx.band_len(band)
    out = []
    for fn in (ctx.march, ctx.march_noalloc):
        I = torch.full((sz["n_rays"], nb), float("nan"), dtype=torch.float64, device="cuda:0")
        Ii = torch.full((sz["n_rays"],), float("nan"), dtype=torch.float64, device="cuda:0")
        fn(band, prec, eta, kap, esc if prec == lrt.LRT_FP32_COMP else None, I, Ii)
        torch.cuda.synchronize()
        out.append((I.cpu().numpy(), Ii.cpu().numpy()))
    return out


def test_noalloc_march_matches_march(torch_dev):
    torch = torch_dev
    big = synth.stagnation_line(n_cells=60, n_atomic=600, n_rovib=1200, n_points=40000, band_points=16384,
                                n_mu=12, seed=31)
    small = synth.stagnation_line(n_cells=20, n_atomic=200, n_rovib=300, n_points=9000, band_points=4096,
                                  n_mu=3, seed=32)
    for prec in (lrt.LRT_FP64, lrt.LRT_FP32_COMP):
        ctx = lrt.Context(0).load(big)
        for band in (0, big.grid.n_bands - 1):           # full band, then the shorter last band
            (I0, i0), (I1, i1) = _both(ctx, band, prec, torch)
            assert np.all(np.isfinite(i1)) and np.array_equal(I0, I1) and np.array_equal(i0, i1), (prec, band)
            say("prec %d band %d: noalloc == march bitwise (%d rays x %d points)" % (prec, band, *I0.shape))
        ctx.close()
        ctx = lrt.Context(0).load(small)                 # fewer rays, fewer chunks
        (I0, i0), (I1, i1) = _both(ctx, 1, prec, torch)
        assert np.array_equal(I0, I1) and np.array_equal(i0, i1)
        ctx.close()


def test_noalloc_rejects_oversize(torch_dev):
    """Rays x march chunks above 2^23: a clear error, nothing launched."""
    torch = torch_dev
    wl = synth.stagnation_line(n_cells=1, n_atomic=10, n_rovib=0, n_points=(1 << 19) + 7, band_points=1 << 19,
                               n_mu=16400, seed=33)
    ctx = lrt.Context(0).load(wl)
    sz = ctx.sizes()
    eta = torch.zeros((1, 1 << 19), dtype=torch.float64, device="cuda:0")
    Ii = torch.zeros((sz["n_rays"],), dtype=torch.float64, device="cuda:0")
    with pytest.raises(lrt.LrtError) as e:
        ctx.march_noalloc(0, lrt.LRT_FP64, eta, eta, None, None, Ii)
    assert e.value.status == 1 and "partial sums" in str(e.value)
    ctx.close()
