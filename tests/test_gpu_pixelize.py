"""GPU parity of the catalogue pixelisation (Sec. III.B, eq. gamma_obs, eq. Neff_pixel, eq. noise_var,
eq. mask) against the oracle, through the C ABI, bit for bit: pixel indices of uniform directions and of
pixel centres at several Nside, and the per-pixel shear, N_eff, N^-1 and mask of synthetic catalogues
(dense, sparse with empty and masked pixels, zero weights, no galaxies), at small sizes and at the
benchmark grid (Nside 2048).  Also: argument errors and reproducibility.

Inputs: seeded synthetic catalogues (uniform positions in a southern box of f_sky 0.1, weights
U[0.2, 1.2], ellipticities R g + N(0, 0.26^2)) and uniform directions on the sphere."""
import math

import numpy as np
import pytest

import akra_workloads as wl
from oracle.geometry import healpix_rings
from oracle.pixelize import ang2pix_ring, pixelize

pytestmark = pytest.mark.gpu


def _plan(nside):
    from paper_2606_06175_amd import Plan
    print("plan nside=%d" % nside, flush=True)
    return Plan(nside, 2, device="cuda:0")


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda", 0))


@pytest.mark.parametrize("nside", [1, 7, 32, 1024])
def test_ang2pix_bit_exact(nside):
    z, phi = wl.sphere_points(400_000, nside)
    # include the poles, the cap/belt boundary and phi = 0
    z[:6] = [1.0, -1.0, 2.0 / 3.0, -2.0 / 3.0, 0.0, np.nextafter(2.0 / 3.0, 1.0)]
    phi[:3] = 0.0
    p = _plan(nside)
    got = p.ang2pix(_t(z), _t(phi)).cpu().numpy()
    assert np.array_equal(got, ang2pix_ring(nside, z, phi))
    # pixel centres
    r = healpix_rings(min(nside, 64))
    if r.npix == p.npix:
        zc = np.repeat(r.z, r.nphi)
        j = np.concatenate([np.arange(n) for n in r.nphi])
        phic = np.pi * np.repeat(r.p0num, r.nphi) / np.repeat(r.p0den, r.nphi) + 2 * np.pi * j / np.repeat(r.nphi, r.nphi)
        assert np.array_equal(p.ang2pix(_t(zc), _t(phic)).cpu().numpy(), np.arange(r.npix))


def test_ang2pix_rejects_out_of_range():
    from paper_2606_06175_amd import akra
    p = _plan(4)
    for z, phi in ((1.5, 0.1), (0.2, -0.1), (0.2, 2 * math.pi), (float("nan"), 1.0)):
        with pytest.raises(akra.AkraError, match="outside"):
            p.ang2pix(_t(np.array([0.1, z])), _t(np.array([0.2, phi])))
    # the flag is cleared: a good call afterwards succeeds
    assert p.ang2pix(_t(np.array([0.1])), _t(np.array([0.2]))).numel() == 1


def _compare(o, ref):
    for k in ("g1", "g2", "ninv", "neff", "mask"):
        assert np.array_equal(o[k].cpu().numpy(), ref[k]), k


@pytest.mark.parametrize("nside,n_gal", [(32, 200_000), (32, 3_000), (8, 50_000), (64, 1_000_000)])
def test_pixelize_bit_exact(nside, n_gal):
    c = wl.make_catalog(n_gal, nside)
    c["w"][::97] = 0.0  # some zero weights
    ref = pixelize(nside, c["z"], c["phi"], c["e1"], c["e2"], c["w"], c["R"], c["sigma_e"], c["n_th"])
    p = _plan(nside)
    o = p.pixelize(*(_t(c[k]) for k in ("z", "phi", "e1", "e2", "w")), c["R"], c["sigma_e"], c["n_th"])
    _compare(o, ref)
    masked = (ref["neff"] > 0) & (ref["mask"] == 0)
    print("occupied %d, masked with galaxies %d, unmasked %d" % ((ref["neff"] > 0).sum(), masked.sum(),
                                                                 ref["mask"].sum()), flush=True)
    # reproducible
    o2 = p.pixelize(*(_t(c[k]) for k in ("z", "phi", "e1", "e2", "w")), c["R"], c["sigma_e"], c["n_th"])
    _compare(o2, ref)


def test_pixelize_no_galaxies_and_errors():
    import torch
    from paper_2606_06175_amd import akra
    p = _plan(4)
    e = torch.zeros(0, dtype=torch.float64, device="cuda:0")
    o = p.pixelize(e, e, e, e, e, 0.7, 0.26, 0.0)
    assert float(o["neff"].abs().max()) == 0 and float(o["g1"].abs().max()) == 0
    assert bool((o["mask"] == 1).all())  # N_eff = 0 >= n_th = 0
    c = wl.make_catalog(1000, 5)
    args = {k: c[k].copy() for k in ("z", "phi", "e1", "e2", "w")}
    args["w"][10] = -1.0
    with pytest.raises(akra.AkraError, match="weight"):
        p.pixelize(*(_t(args[k]) for k in ("z", "phi", "e1", "e2", "w")), 0.7, 0.26, 1.0)
    args["w"][10] = 1.0
    args["e2"][3] = float("inf")
    with pytest.raises(akra.AkraError, match="ellipticity"):
        p.pixelize(*(_t(args[k]) for k in ("z", "phi", "e1", "e2", "w")), 0.7, 0.26, 1.0)
    args["e2"][3] = 0.0
    with pytest.raises(akra.AkraError, match="R must be"):
        p.pixelize(*(_t(args[k]) for k in ("z", "phi", "e1", "e2", "w")), 0.0, 0.26, 1.0)
    w = torch.empty(p.pixelize_work_bytes(1000) - 1, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(akra.AkraError, match="workspace too small"):
        p.pixelize(*(_t(args[k]) for k in ("z", "phi", "e1", "e2", "w")), 0.7, 0.26, 1.0, work=w)
    w = torch.empty(p.pixelize_work_bytes(1000) + 256, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(akra.AkraError, match="aligned"):
        p.pixelize(*(_t(args[k]) for k in ("z", "phi", "e1", "e2", "w")), 0.7, 0.26, 1.0, work=w[16:])
    o = p.pixelize(*(_t(args[k]) for k in ("z", "phi", "e1", "e2", "w")), 0.7, 0.26, 1.0)
    _compare(o, pixelize(4, *(args[k] for k in ("z", "phi", "e1", "e2", "w")), 0.7, 0.26, 1.0))


def test_pixelize_feeds_the_solve():
    # the outputs are the solver's inputs: a C1-sized catalogue pixelised and solved to 1e-8
    p = _plan(32)
    c = wl.make_catalog(300_000, 8)
    o = p.pixelize(*(_t(c[k]) for k in ("z", "phi", "e1", "e2", "w")), c["R"], c["sigma_e"], c["n_th"])
    from paper_2606_06175_amd import Plan
    s = Plan(32, 64, device="cuda:0")
    m = o["mask"].to(o["g1"].dtype)
    xE, xB, info = s.cg_solve(o["g1"] * m, o["g2"] * m, o["ninv"], o["mask"], tol=1e-8, maxiter=4000)
    assert info["status"] == 0 and info["rel_resid_true"] <= 1.05e-8
    assert bool(xE.isfinite().all())


def test_pixelize_full_grid():
    # the benchmark grid (Nside 2048) with 2e7 galaxies: every output bit for bit
    nside, n = 2048, 20_000_000
    c = wl.make_catalog(n, 12)
    print("oracle pixelisation of %d galaxies" % n, flush=True)
    ref = pixelize(nside, c["z"], c["phi"], c["e1"], c["e2"], c["w"], c["R"], c["sigma_e"], c["n_th"])
    p = _plan(nside)
    o = p.pixelize(*(_t(c[k]) for k in ("z", "phi", "e1", "e2", "w")), c["R"], c["sigma_e"], c["n_th"])
    _compare(o, ref)
