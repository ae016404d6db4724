"""GPU parity of the weighted operator when rings carry no weight.

A ring whose weights W = M N^-1 are all zero adds nothing to H v or to the right-hand side, so the
weighted applies transform only the rings with weight and contract one side of a ring pair where
only that side carries weight.  These tests drive footprints that produce every class of 64-pair
group (weight on both rings of the pairs, on the north rings only, on the south rings only, on
none), check H against the oracle element by element (1e-10 FP64, 1e-5 FP32, globally, per m and
per right-hand side), check the same apply with ring skipping switched off (rounding order only),
the batched FP32 form with a different zero pattern per right-hand side, and a solve."""
import numpy as np
import pytest

import akra_workloads as wl
from oracle.core import Oracle
from oracle.geometry import healpix_rings

from test_gpu_parity import TOL, check_alm, rel

pytestmark = pytest.mark.gpu


def footprint(name, nside):
    vec = wl.pixel_vectors(nside)
    npix = 12 * nside * nside
    z = vec[2]
    if name == "south_cap":      # theta 120 deg: south rings only, and both near the equator
        return wl.cap_mask(nside, 2.1, 0.3, 0.1, vec)
    if name == "north_cap":      # theta 40 deg, radius 37 deg: north rings only
        return wl.cap_mask(nside, 0.7, 1.0, 0.1, vec)
    if name == "polar_north":    # the near-polar groups of FP32 plans, north side
        return wl.cap_mask(nside, 0.02, 0.0, 0.03, vec)
    if name == "polar_south":
        return wl.cap_mask(nside, np.pi - 0.02, 0.0, 0.03, vec)
    if name == "stripes":        # one narrow north stripe and one south stripe at other latitudes
        return ((z > 0.30) & (z < 0.36)) | ((z < -0.70) & (z > -0.78))
    if name == "full":
        return np.ones(npix, bool)
    if name == "empty":
        return np.zeros(npix, bool)
    raise KeyError(name)


FEET = ["south_cap", "north_cap", "polar_north", "polar_south", "stripes", "full", "empty"]


def weights(nside, foot, seed):
    g = np.random.default_rng(seed)
    n = g.poisson(3.0, 12 * nside * nside)
    mask = (footprint(foot, nside) & (n >= 1)).astype(np.uint8)
    return mask, n / wl.SIGMA_E ** 2


def live_rings(rings, mask, ninv):
    w = mask * ninv
    return np.array([np.any(w[rings.ofs[r]:rings.ofs[r] + rings.nphi[r]] != 0) for r in range(rings.nrings)])


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    return torch, torch.device("cuda", 0)


def _plan(nside, lmax, prec, nrhs=1):
    from paper_2606_06175_amd import Plan
    print("plan nside=%d lmax=%d %s nrhs=%d" % (nside, lmax, prec, nrhs), flush=True)
    return Plan(nside, lmax, nrhs=nrhs, precision=prec, device="cuda:0")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("foot", FEET)
@pytest.mark.parametrize("nside,lmax", [(13, 40), (64, 128), (100, 400)])
def test_apply_H_weighted_rings(torch_dev, nside, lmax, prec, foot):
    torch, dev = torch_dev
    o = Oracle(lmax, healpix_rings(nside))
    mask, ninv = weights(nside, foot, 3)
    lam = 0.02
    x = np.stack([wl.random_alm(lmax, 1, lmin=0), wl.random_alm(lmax, 2, lmin=0)])
    p = _plan(nside, lmax, prec)
    tn, tm = torch.from_numpy(ninv).to(dev), torch.from_numpy(mask).to(dev)
    tx = [torch.from_numpy(a).to(dev) for a in x]
    yE, yB = p.apply_H(tn, tm, tx[0], tx[1], lam)
    got = np.stack([yE.cpu().numpy(), yB.cpu().numpy()])
    ww = p.work_weighted()
    live = live_rings(o.rings, mask, ninv)
    print("%s: %d of %d rings carry weight, work %s" % (foot, live.sum(), o.rings.nrings, ww), flush=True)
    assert ww["live_rings"] == int(live.sum())
    full = p.work()
    assert ww["synth_two"] + ww["synth_one"] <= full["synth"]
    assert ww["adjoint_two"] + ww["adjoint_one"] <= full["adjoint"]
    if foot == "empty":
        # no ring carries weight: H x = lambda x exactly, and no Legendre work
        assert sum(v for k, v in ww.items() if k != "live_rings") == 0
        assert np.array_equal(got, lam * x)
        return
    ref = o.apply_H(x, o.weights(ninv, mask), lam)
    check_alm(got, ref, lmax, TOL[prec])
    # every ring and group transformed: the same H up to the adjoint's rounding order
    p.set_skip_unweighted(False)
    fE, fB = p.apply_H(tn, tm, tx[0], tx[1], lam)
    e = rel(got, np.stack([fE.cpu().numpy(), fB.cpu().numpy()]))
    print("skip against no skip: %.3e" % e, flush=True)
    assert e < (1e-13 if prec == "fp64" else 1e-6)


def test_one_sided_work_classes(torch_dev):
    # a south cap at Nside 256 (eight 64-pair groups) leaves groups weighted on one side, on both
    # sides and, near the north pole, on none: the weighted work is split accordingly and smaller than
    # the full work
    torch, dev = torch_dev
    nside, lmax = 256, 512
    mask, ninv = weights(nside, "south_cap", 4)
    p = _plan(nside, lmax, "fp64")
    x = [torch.from_numpy(wl.random_alm(lmax, s)).to(dev) for s in (5, 6)]
    p.apply_H(torch.from_numpy(ninv).to(dev), torch.from_numpy(mask).to(dev), x[0], x[1], 0.01)
    ww, full = p.work_weighted(), p.work()
    print(ww, full, flush=True)
    assert ww["synth_one"] > 0 and ww["synth_two"] > 0
    assert ww["synth_two"] + ww["synth_one"] < full["synth"]
    assert ww["adjoint_two"] + ww["adjoint_one"] < full["adjoint"]


def test_rhs_weighted_rings(torch_dev):
    torch, dev = torch_dev
    nside, lmax = 32, 96
    o = Oracle(lmax, healpix_rings(nside))
    mask, ninv = weights(nside, "stripes", 5)
    g1, g2 = wl.random_maps(o.rings.npix, 6)
    p = _plan(nside, lmax, "fp64")
    bE, bB = p.rhs(torch.from_numpy(g1).to(dev), torch.from_numpy(g2).to(dev), torch.from_numpy(ninv).to(dev),
                   torch.from_numpy(mask).to(dev))
    ref = o.rhs(g1, g2, o.weights(ninv, mask))
    check_alm(np.stack([bE.cpu().numpy(), bB.cpu().numpy()]), ref, lmax, 1e-10)


def test_batched_fp32_zero_patterns_per_rhs(torch_dev):
    # the batched form transforms the rings that carry weight in any right-hand side's W; a ring
    # without weight in one right-hand side contributes zero to it through its own W
    torch, dev = torch_dev
    nside, lmax, nrhs = 64, 128, 3
    o = Oracle(lmax, healpix_rings(nside))
    ms, ns = zip(*(weights(nside, f, 7 + k) for k, f in enumerate(["south_cap", "north_cap", "stripes"])))
    mask = np.ones(12 * nside * nside, np.uint8)
    ninvs = np.stack([m * n for m, n in zip(ms, ns)])
    A = np.stack([wl.random_alm(lmax, 60 + k) for k in range(nrhs)])
    B = np.stack([wl.random_alm(lmax, 80 + k) for k in range(nrhs)])
    p = _plan(nside, lmax, "fp32", nrhs=nrhs)
    yE, yB = p.apply_H(torch.from_numpy(ninvs).to(dev), torch.from_numpy(mask).to(dev),
                       torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev), 0.02)
    for k in range(nrhs):
        ref = o.apply_H(np.stack([A[k], B[k]]), o.weights(ninvs[k], mask), 0.02)
        print("rhs %d" % k, flush=True)
        check_alm(np.stack([yE[k].cpu().numpy(), yB[k].cpu().numpy()]), ref, lmax, TOL["fp32"])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_solve_skip_matches_full(torch_dev, prec):
    # the same solve with and without ring skipping: iterates agree to rounding, both meet the
    # tolerance in the oracle's true residual
    torch, dev = torch_dev
    nside, lmax = 32, 64
    o = Oracle(lmax, healpix_rings(nside))
    mask, ninv = weights(nside, "south_cap", 11)
    g1, g2 = wl.random_maps(o.rings.npix, 12)
    g1, g2 = 0.01 * g1 * mask, 0.01 * g2 * mask
    args = [torch.from_numpy(a).to(dev) for a in (g1, g2, ninv, mask)]
    out = []
    for skip in (True, False):
        p = _plan(nside, lmax, prec)
        p.set_skip_unweighted(skip)
        xE, xB, info = p.cg_solve(*args, tol=1e-9, maxiter=3000)
        print("skip %s: %s" % (skip, info), flush=True)
        x = np.stack([xE.cpu().numpy(), xB.cpu().numpy()])
        W = o.weights(ninv, mask)
        lam = o.lambda_eff(ninv, mask)
        b = o.rhs(g1, g2, W)
        r = b - o.apply_H(x, W, lam)
        assert np.sqrt(o.dot(r, r) / o.dot(b, b)) < 1e-9 * 1.01
        out.append((x, info["iters"]))
    assert abs(out[0][1] - out[1][1]) <= 2
    assert rel(out[0][0], out[1][0]) < 1e-8


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_class_chains_match_staged_apply(torch_dev, prec):
    # untimed weighted applies run one chain per class of ring groups on two streams, timed applies
    # run the stages in order; the kernels and their inputs are the same, so H x agrees bit for bit,
    # and both agree with the oracle
    torch, dev = torch_dev
    nside, lmax = 100, 400
    o = Oracle(lmax, healpix_rings(nside))
    mask, ninv = weights(nside, "south_cap", 13)
    x = np.stack([wl.random_alm(lmax, 14, lmin=0), wl.random_alm(lmax, 15, lmin=0)])
    p = _plan(nside, lmax, prec)
    tn, tm = torch.from_numpy(ninv).to(dev), torch.from_numpy(mask).to(dev)
    tx = [torch.from_numpy(a).to(dev) for a in x]
    out = []
    for timed in (False, True, False):
        p.set_timing(timed)
        yE, yB = p.apply_H(tn, tm, tx[0], tx[1], 0.02)
        out.append(np.stack([yE.cpu().numpy(), yB.cpu().numpy()]))
    p.set_timing(False)
    ww = p.work_weighted()
    assert ww["synth_two"] > 0 and ww["synth_one"] > 0, ww
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])
    check_alm(out[0], o.apply_H(x, o.weights(ninv, mask), 0.02), lmax, TOL[prec])
