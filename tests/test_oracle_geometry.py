"""Pins of the oracle's ring tables against properties HEALPix fixes (Gorski et al. 2005) and
against the Gauss-Legendre rule."""
import math

import numpy as np
import pytest

from oracle.geometry import gl_rings, healpix_rings


def test_nside1_base_pixel_centres():
    # the 12 base pixels: rings at z = 2/3, 0, -2/3; polar rows start at phi = pi/4,
    # the equatorial row at phi = 0
    r = healpix_rings(1)
    np.testing.assert_allclose(r.z, [2 / 3, 0.0, -2 / 3], atol=1e-15)
    assert list(r.nphi) == [4, 4, 4]
    th, ph = r.pixel_angles()
    np.testing.assert_allclose(ph[:4], np.pi / 4 + np.arange(4) * np.pi / 2, atol=1e-15)
    np.testing.assert_allclose(ph[4:8], np.arange(4) * np.pi / 2, atol=1e-15)
    np.testing.assert_allclose(ph[8:], np.pi / 4 + np.arange(4) * np.pi / 2, atol=1e-15)
    assert r.npix == 12


@pytest.mark.parametrize("nside", [1, 2, 3, 8, 32, 100])
def test_counts_offsets_symmetry(nside):
    r = healpix_rings(nside)
    assert r.nrings == 4 * nside - 1
    assert int(r.nphi.sum()) == 12 * nside * nside == r.npix
    np.testing.assert_array_equal(r.ofs[1:], np.cumsum(r.nphi)[:-1])
    np.testing.assert_allclose(r.z, -r.z[::-1], atol=1e-15)
    np.testing.assert_array_equal(r.nphi, r.nphi[::-1])
    assert np.all(np.diff(r.z) < 0)
    np.testing.assert_allclose(r.st ** 2 + r.z ** 2, 1.0, atol=1e-15)


@pytest.mark.parametrize("nside", [2, 5, 16, 64])
def test_equal_area_ring_centres(nside):
    # equal-area property: the cap above a ring centre holds the pixels of all rings above it
    # plus half of the ring itself, each of area 4 pi / Npix
    r = healpix_rings(nside)
    om = 4 * math.pi / r.npix
    above = 0
    for k in range(2 * nside):
        cap = 2 * math.pi * (1 - r.z[k])
        assert abs(cap - om * (above + r.nphi[k] / 2)) < 1e-12
        above += int(r.nphi[k])


def test_gauss_legendre_rule():
    g = gl_rings(40)
    w = g.omega * g.nphi / (2 * np.pi)
    assert abs(w.sum() - 2.0) < 1e-14
    np.testing.assert_allclose(g.z, -g.z[::-1], atol=1e-15)
    # exact for polynomials up to degree 2 lmax + 1
    for deg in (0, 2, 40, 80):
        assert abs(np.sum(w * g.z ** deg) - (2.0 / (deg + 1))) < 1e-13
