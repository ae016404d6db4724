"""Pins of the oracle's catalogue pixelisation (Sec. III.B, eq. gamma_obs, eq. Neff_pixel,
eq. noise_var, eq. mask).

Against:
  * the pixel-centre table of the oracle's geometry (itself pinned to the Nside = 1 base-pixel
    centres of Gorski et al. 2005): every centre maps to its own RING index, for Nside 1 to 16;
  * points jittered inside a pixel stay in it, in the caps and the belt;
  * the north-south mirror: (z, phi) in ring i, position j maps to (-z, phi) in ring 4 Nside - i,
    position j;
  * equal areas: uniform points fill every pixel equally, within 6 sigma;
  * hand-worked sums of a tiny catalogue (gamma_obs, N_eff, N^-1, mask), including empty pixels and
    zero weights.
"""
import math

import numpy as np
import pytest

import akra_workloads as wl
from oracle.geometry import healpix_rings
from oracle.pixelize import ang2pix_ring, pixelize


def _centres(nside):
    r = healpix_rings(nside)
    z = np.repeat(r.z, r.nphi)
    j = np.concatenate([np.arange(n) for n in r.nphi])
    nphi = np.repeat(r.nphi, r.nphi)
    phi0 = np.pi * np.repeat(r.p0num, r.nphi) / np.repeat(r.p0den, r.nphi)
    phi = phi0 + 2 * np.pi * j / nphi
    return r, z, phi, j


@pytest.mark.parametrize("nside", [1, 2, 3, 4, 8, 13, 16])
def test_centres_map_to_their_index(nside):
    r, z, phi, _ = _centres(nside)
    assert np.array_equal(ang2pix_ring(nside, z, phi), np.arange(r.npix))


@pytest.mark.parametrize("nside", [2, 5, 16])
def test_jittered_points_stay_in_their_pixel(nside):
    # a pixel reaches about half-way to the neighbouring rings along its meridian and pi / N_r along
    # its ring; points in a diamond of 20% of those half-sizes around the centre stay inside
    r, z, phi, _ = _centres(nside)
    g = np.random.default_rng(nside)
    nphi = np.repeat(r.nphi, r.nphi)
    ring = np.repeat(np.arange(r.nrings), r.nphi)
    zr = np.r_[1.0, r.z, -1.0]
    half = 0.5 * np.minimum(zr[ring] - zr[ring + 1], zr[ring + 1] - zr[ring + 2])
    for _ in range(4):
        u = g.uniform(-1, 1, z.size)
        v = (1 - np.abs(u)) * g.uniform(-1, 1, z.size)
        zz = z + 0.2 * half * u
        pp = np.mod(phi + 0.2 * (np.pi / nphi) * v, 2 * np.pi)
        assert np.array_equal(ang2pix_ring(nside, zz, pp), np.arange(r.npix))


@pytest.mark.parametrize("nside", [1, 4, 7])
def test_north_south_mirror(nside):
    r = healpix_rings(nside)
    z, phi = wl.sphere_points(20000, nside)
    p = ang2pix_ring(nside, z, phi)
    q = ang2pix_ring(nside, -z, phi)
    ring = np.searchsorted(r.ofs, p, side="right") - 1
    ring_q = np.searchsorted(r.ofs, q, side="right") - 1
    assert np.array_equal(ring_q, r.nrings - 1 - ring)
    assert np.array_equal(q - r.ofs[ring_q], p - r.ofs[ring])


@pytest.mark.parametrize("nside", [1, 4])
def test_equal_areas(nside):
    n = 1_200_000
    z, phi = wl.sphere_points(n, 30 + nside)
    c = np.bincount(ang2pix_ring(nside, z, phi), minlength=12 * nside * nside)
    mean = n / c.size
    assert np.all(np.abs(c - mean) < 6 * math.sqrt(mean))


def test_hand_worked_sums():
    nside = 1
    r, zc, phic, _ = _centres(nside)
    # galaxies at the centres of pixels 0 (three), 5 (one), 7 (two, one with zero weight), 11 (one,
    # zero weight); every other pixel is empty
    pix = np.array([0, 0, 0, 5, 7, 7, 11])
    w = np.array([1.0, 2.0, 1.0, 0.5, 3.0, 0.0, 0.0])
    e1 = np.array([0.1, -0.2, 0.4, 0.3, 0.05, 9.0, 1.0])
    e2 = np.array([0.0, 0.1, -0.1, -0.3, 0.2, 9.0, 1.0])
    o = pixelize(nside, zc[pix], phic[pix], e1, e2, w, R=0.5, sigma_e=0.25, n_th=1.5)
    assert np.array_equal(o["pix"], pix)
    # pixel 0: sum w = 4, sum w e1 = 0.1 - 0.4 + 0.4 = 0.1, sum w e2 = 0.2 - 0.1 = 0.1, sum w^2 = 6
    assert o["g1"][0] == pytest.approx(0.1 / (0.5 * 4)) and o["g2"][0] == pytest.approx(0.1 / (0.5 * 4))
    assert o["neff"][0] == pytest.approx(16 / 6) and o["ninv"][0] == pytest.approx(16 / 6 / 0.0625)
    # pixel 5: one galaxy, N_eff = 1 < 1.5 -> masked, but its shear and N^-1 are still defined
    assert o["g1"][5] == pytest.approx(0.3 / 0.5) and o["neff"][5] == 1.0 and o["mask"][5] == 0
    # pixel 7: the zero-weight galaxy adds nothing
    assert o["g1"][7] == pytest.approx(0.05 / 0.5) and o["g2"][7] == pytest.approx(0.2 / 0.5)
    assert o["neff"][7] == 1.0
    # pixel 11: only a zero weight -> no shear, N_eff = 0
    assert o["g1"][11] == 0 and o["neff"][11] == 0 and o["ninv"][11] == 0
    assert list(np.flatnonzero(o["mask"])) == [0]
    empty = np.setdiff1d(np.arange(12), [0, 5, 7, 11])
    assert np.all(o["g1"][empty] == 0) and np.all(o["neff"][empty] == 0) and np.all(o["mask"][empty] == 0)


def test_catalogue_recipe():
    c = wl.make_catalog(200_000, 3)
    assert c["z"].min() >= -0.95 and c["z"].max() < -0.35 and c["phi"].min() >= 0
    area = (0.6 * c["phi"].max()) / (4 * math.pi)
    assert abs(area - 0.1) < 1e-3
    o = pixelize(32, c["z"], c["phi"], c["e1"], c["e2"], c["w"], c["R"], c["sigma_e"], c["n_th"])
    inside = o["neff"] > 0
    # about 163 galaxies per occupied pixel; N_eff ~ 0.87 of the count for U[0.2, 1.2] weights
    assert 1000 < inside.sum() < 1500 and o["mask"].sum() > 0.9 * inside.sum()
