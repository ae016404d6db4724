"""Pins of the oracle's noise-realisation and spectrum stage (Sec. IV power spectra).

Against:
  * per-degree Parseval on the Gauss-Legendre grid, where the quadrature is exact for band-limited
    products: the map-space integrals of the oracle's own synthesis give (2l+1) C_l.  For a field
    confined to one degree,
        int |gamma|^2 dOmega            = (2l+1) (C_l^EE + C_l^BB),
        int Re(gamma_X conj gamma_Y)    = (2l+1) C_l^{E_X E_Y},
        int Im(gamma_X conj gamma_Y)    = -(2l+1) C_l^{E_X B_Y}  (X pure E, Y pure B; from
    2a = -(a_E + i a_B): the product of coefficients is -i a_E conj(a_B)).
    A missing conjugate, a wrong m > 0 weight or a wrong (2l+1) fails these;
  * single-coefficient closed forms;
  * a hand-worked shuffle of a 12-pixel map;
  * the identity permutation reproducing the direct solve, and paired halves with equal data
    reproducing the auto spectrum.
"""
import numpy as np
import pytest

import akra_workloads as wl
from oracle.core import Oracle, alm_index, alm_lm
from oracle.geometry import gl_rings, healpix_rings
from oracle import spectra as sp


def _single_degree(lmax, l, seed):
    a = wl.random_alm(lmax, seed, 0)
    a[alm_lm(lmax)[0] != l] = 0
    return a


@pytest.fixture(scope="module")
def gl():
    lmax = 10
    o = Oracle(lmax, gl_rings(lmax))
    om = np.repeat(o.rings.omega, o.rings.nphi)
    return o, om


@pytest.mark.parametrize("l", [2, 3, 6, 10])
def test_parseval_auto_per_degree(gl, l):
    o, om = gl
    aE = _single_degree(o.lmax, l, 300 + l)
    aB = _single_degree(o.lmax, l, 400 + l)
    g1, g2 = o.synth(aE, aB)
    power = float(np.sum(om * (g1 * g1 + g2 * g2)))
    cee = sp.spectrum(aE, aE, o.lmax)
    cbb = sp.spectrum(aB, aB, o.lmax)
    assert abs(power - (2 * l + 1) * (cee[l] + cbb[l])) < 1e-12 * power
    # other degrees are empty
    assert np.all(np.delete(cee, l) == 0) and np.all(np.delete(cbb, l) == 0)


@pytest.mark.parametrize("l", [2, 5, 10])
def test_parseval_cross_per_degree(gl, l):
    o, om = gl
    z = np.zeros(o.nalm, np.complex128)
    x = _single_degree(o.lmax, l, 500 + l)
    y = _single_degree(o.lmax, l, 600 + l)
    gx1, gx2 = o.synth(x, z)
    gy1, gy2 = o.synth(y, z)
    re = float(np.sum(om * (gx1 * gy1 + gx2 * gy2)))
    c = sp.spectrum(x, y, o.lmax)[l]
    assert abs(re - (2 * l + 1) * c) < 1e-12 * np.sqrt(np.sum(om * (gx1**2 + gx2**2)) * np.sum(om * (gy1**2 + gy2**2)))
    # E of X against B of Y: the imaginary part of the map-space product
    gb1, gb2 = o.synth(z, y)
    im = float(np.sum(om * (gx2 * gb1 - gx1 * gb2)))
    ceb = sp.spectrum(x, y, o.lmax)[l]
    assert abs(im + (2 * l + 1) * ceb) < 1e-11 * abs(im)
    # symmetry and Cauchy-Schwarz
    assert sp.spectrum(y, x, o.lmax)[l] == pytest.approx(c, rel=1e-15)
    assert c * c <= sp.spectrum(x, x, o.lmax)[l] * sp.spectrum(y, y, o.lmax)[l]


def test_parseval_band_limited_total(gl):
    o, om = gl
    aE = wl.random_alm(o.lmax, 701)
    aB = wl.random_alm(o.lmax, 702)
    g1, g2 = o.synth(aE, aB)
    power = float(np.sum(om * (g1 * g1 + g2 * g2)))
    l = np.arange(o.lmax + 1)
    tot = float(np.sum((2 * l + 1) * (sp.spectrum(aE, aE, o.lmax) + sp.spectrum(aB, aB, o.lmax))))
    assert abs(power - tot) < 1e-12 * power


def test_single_coefficient_closed_forms():
    lmax = 9
    for l, m, z in ((4, 0, 1.5), (4, 3, 0.6 - 0.8j), (9, 9, 2j), (2, 1, -1.0)):
        a = np.zeros((lmax + 1) * (lmax + 2) // 2, np.complex128)
        a[alm_index(lmax, l, m)] = z
        c = sp.spectrum(a, a, lmax)
        want = (abs(z) ** 2 if m else z.real ** 2) * (2 if m else 1) / (2 * l + 1)
        assert c[l] == pytest.approx(want, rel=1e-15)
        assert np.count_nonzero(c) == 1
    # l < 2 is never part of the spectrum
    a = np.ones((lmax + 1) * (lmax + 2) // 2, np.complex128)
    c = sp.spectrum(a, a, lmax)
    assert c[0] == 0 and c[1] == 0 and c[2] > 0


def test_shuffle_hand_worked():
    mask = np.array([1, 0, 1, 1, 0, 0, 1, 1, 0, 1, 0, 1], np.uint8)
    assert list(sp.unmasked_index(mask)) == [0, 2, 3, 6, 7, 9, 11]
    g1 = 10.0 * np.arange(12) + 1
    g2 = -1.5 * np.arange(12)
    perm = np.array([3, 0, 6, 1, 5, 2, 4])
    o1, o2 = sp.shuffle_shear(g1, g2, mask, perm)
    assert list(o1) == [61, 0, 1, 111, 0, 0, 21, 91, 0, 31, 0, 71]
    assert list(o2) == [-9, 0, 0, -16.5, 0, 0, -3, -13.5, 0, -4.5, 0, -10.5]


def test_shuffle_preserves_values_and_identity():
    g = np.random.default_rng(9)
    mask = (g.random(3072) < 0.3).astype(np.uint8)
    g1, g2 = g.normal(size=3072), g.normal(size=3072)
    u = sp.unmasked_index(mask)
    o1, o2 = sp.shuffle_shear(g1, g2, mask, np.arange(u.size))
    assert np.array_equal(o1, g1 * mask) and np.array_equal(o2, g2 * mask)
    perm = wl.shuffle_perms(u.size, 1, 3)[0]
    o1, o2 = sp.shuffle_shear(g1, g2, mask, perm)
    assert np.array_equal(np.sort(o1[u]), np.sort(g1[u]))
    assert np.array_equal(np.sort(o2[u]), np.sort(g2[u]))
    assert np.all(o1[mask == 0] == 0) and np.all(o2[mask == 0] == 0)
    # the pair moves together: (g1, g2) of a source pixel stays a pair
    assert np.array_equal(o1[u] + 1j * o2[u], (g1 + 1j * g2)[u[perm]])


def test_shuffle_perms_are_permutations():
    p = wl.shuffle_perms(1000, 4, 5)
    assert p.dtype == np.int32 and p.shape == (4, 1000)
    for row in p:
        assert np.array_equal(np.sort(row), np.arange(1000))
    assert not np.array_equal(p[0], p[1])
    q = wl.shuffle_perms(1000, 4, 5, half=1)
    assert not np.array_equal(p[0], q[0])
    assert np.array_equal(p, wl.shuffle_perms(1000, 4, 5))


def test_moments():
    cls = np.array([[[1.0, 4.0]], [[2.0, 4.0]], [[3.0, 4.0]]])
    mean, std = sp.moments(cls)
    assert np.allclose(mean, [[2.0, 4.0]]) and np.allclose(std, [[1.0, 0.0]])
    mean, std = sp.moments(cls[:1])
    assert np.all(std == 0) and np.allclose(mean, cls[0])


@pytest.fixture(scope="module")
def tiny():
    nside, lmax = 4, 8
    o = Oracle(lmax, healpix_rings(nside))
    g = np.random.default_rng(81)
    foot = wl.cap_mask(nside, 1.1, 0.4, 0.4, wl.pixel_vectors(nside))
    n = g.poisson(5.0, o.rings.npix)
    mask = (foot & (n >= 1)).astype(np.uint8)
    ninv = n / wl.SIGMA_E ** 2
    g1, g2 = wl.random_maps(o.rings.npix, 82)
    return o, mask, ninv, g1 * mask, g2 * mask


@pytest.mark.parametrize("mode", [0, 1])
def test_identity_shuffle_reproduces_direct_solve(tiny, mode):
    o, mask, ninv, g1, g2 = tiny
    n_obs = int(mask.sum())
    perms = np.stack([np.arange(n_obs), np.arange(n_obs)])
    cls = sp.noise_spectra(o, g1, g2, ninv, mask, perms, mode=mode, tol=1e-12)
    x = sp.solve(o, g1, g2, ninv, mask, mode, tol=1e-12)
    want = sp.pair_spectra(o, x, x, mode)
    assert cls.shape == (2,) + want.shape
    assert np.allclose(cls[0], want, rtol=1e-9, atol=0) and np.array_equal(cls[0], cls[1])
    if mode == 0:
        # the cross EB spectrum of the joint solve is not identically zero on a masked sky
        assert np.abs(want[2]).max() > 0


def test_paired_halves_with_equal_data_give_auto(tiny):
    o, mask, ninv, g1, g2 = tiny
    n_obs = int(mask.sum())
    p = wl.shuffle_perms(n_obs, 2, 11)
    auto = sp.noise_spectra(o, g1, g2, ninv, mask, p, mode=1, tol=1e-12)
    pair = sp.noise_spectra(o, np.stack([g1, g1]), np.stack([g2, g2]), np.stack([ninv, ninv]), mask,
                            np.stack([p, p]), mode=1, tol=1e-12)
    assert np.allclose(pair, auto, rtol=1e-12, atol=0)
    # different shuffles give different realisations
    assert not np.allclose(auto[0], auto[1])
