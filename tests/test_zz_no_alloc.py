"""Allocation-free spectra (akra_alm_spectra_noalloc, static device scratch) against the plan's
akra_alm_spectra: equal bit for bit (same kernels, fixed summation order) on two calls in a row, the
second with a smaller band limit and fewer pairs, so that nothing of the first call's scratch
contents can leak into the second."""
import numpy as np
import pytest

import akra_workloads as wl

pytestmark = pytest.mark.gpu


def _case(torch, dev, lmax, n, seed):
    x = torch.from_numpy(np.stack([wl.random_alm(lmax, seed + k, lmin=0) for k in range(n)])).to(dev)
    y = torch.from_numpy(np.stack([wl.random_alm(lmax, seed + 100 + k, lmin=0) for k in range(n)])).to(dev)
    return x, y


def test_noalloc_spectra_match_plan_spectra_twice():
    import torch
    from paper_2606_06175_amd import Plan, akra
    dev = torch.device("cuda", 0)
    # first call at the largest band limit the scratch holds, 11 pairs (two launches of 8 and 3);
    # second call smaller: lmax 300, 3 pairs
    cases = [(1024, akra.NOALLOC_LMAX_MAX, 6, [(0, 0), (1, 2), (5, 5), (2, 4), (3, 3), (0, 5), (4, 1), (2, 2),
                                               (1, 1), (3, 0), (5, 4)]),
             (75, 300, 3, [(2, 1), (0, 0), (1, 2)])]
    for nside, lmax, n, pairs in cases:
        print("noalloc spectra lmax=%d pairs=%d" % (lmax, len(pairs)), flush=True)
        x, y = _case(torch, dev, lmax, n, 7 * lmax)
        got = akra.alm_spectra_noalloc(x, y, pairs, lmax)
        torch.cuda.synchronize()
        p = Plan(nside, lmax, precision="fp64", device=dev)
        ref = p.alm_spectra(x, y, pairs)
        torch.cuda.synchronize()
        p.close()
        assert got.shape == ref.shape == (len(pairs), lmax + 1)
        assert torch.equal(got, ref)
        assert bool(torch.isfinite(got).all()) and float(got[:, 2:].abs().min()) > 0
        # the auto spectrum of a set against itself with y = x
        auto = akra.alm_spectra_noalloc(x, x, [(k, k) for k in range(n)], lmax)
        assert bool((auto[:, 2:] > 0).all()) and bool((auto[:, :2] == 0).all())


def test_noalloc_spectra_rejects_band_limit_beyond_scratch():
    import torch
    from paper_2606_06175_amd import akra
    dev = torch.device("cuda", 0)
    lmax = akra.NOALLOC_LMAX_MAX + 1
    x = torch.zeros((1, akra.alm_size(lmax)), dtype=torch.complex128, device=dev)
    with pytest.raises(akra.AkraError) as e:
        akra.alm_spectra_noalloc(x, x, [(0, 0)], lmax)
    assert e.value.status == akra.AKRA_ERR_ARG
