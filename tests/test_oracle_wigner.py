"""Pins of the oracle's Wigner-d / spin-weighted harmonic columns.

Against: Wigner's explicit finite sum and the Jacobi-polynomial form (two independent closed
forms, mpmath), Legendre polynomials (scipy), orthonormality under exact Gauss-Legendre
quadrature, the reflection/transposition symmetries, and the textbook 2Y_20."""
import math

import mpmath as mp
import numpy as np
import pytest
import scipy.special as ss

from oracle.core import Oracle
from oracle.dense import wigner_d_jacobi, wigner_d_sum
from oracle.geometry import gl_rings, healpix_rings


def col(lmax, m, mp_, z, norm=False):
    return Oracle(lmax, gl_rings(2)).wigner(m, mp_, z, norm)


THETAS = [1e-3, 0.05, 0.7, 1.5707963267948966, 2.3, 3.1]


@pytest.mark.parametrize("theta", THETAS)
def test_against_wigner_sum(theta):
    z = math.cos(theta)
    worst = 0.0
    for mp_ in (-2, 0, 2):
        for m in range(-12, 13):
            c = col(12, m, mp_, z)
            for l in range(12 + 1):
                if l < max(abs(m), abs(mp_)):
                    assert c[l] == 0.0
                    continue
                ref = float(wigner_d_sum(l, m, mp_, z=z, dps=50))
                worst = max(worst, abs(c[l] - ref))
    assert worst < 1e-14


def test_two_closed_forms_agree():
    for (j, a, b) in [(3, 2, -2), (7, -5, 2), (9, 9, -2), (12, 0, 2), (5, -2, -2)]:
        for th in (0.3, 1.9):
            assert abs(wigner_d_sum(j, a, b, th) - wigner_d_jacobi(j, a, b, th)) < 1e-30


@pytest.mark.parametrize("ring,m,mp_", [(3, 7, 2), (10, 3000, -2), (1000, 1500, 2), (4095, 4000, -2),
                                        (2, 0, -2), (2047, 1, 2), (6000, 2048, -2), (8190, 5, 2)])
def test_large_l_against_jacobi(ring, m, mp_):
    # Nside 2048 ring positions, l up to 4096 (the headline size)
    z = float(healpix_rings(2048).z[ring])
    c = col(4096, m, mp_, z)
    for l in (max(abs(m), 2), 2049, 3333, 4096):
        if l < max(abs(m), 2):
            continue
        ref = float(wigner_d_jacobi(l, m, mp_, z=z, dps=80))
        if abs(ref) < 1e-250:
            assert abs(c[l]) < 1e-250
        else:
            assert abs(c[l] - ref) <= 2e-13 * abs(ref) + 1e-300


def test_legendre_special_case():
    x = np.array([-0.97, -0.3, 0.11, 0.5, 0.999])
    l = np.arange(2001)
    for xi in x:
        c = col(2000, 0, 0, xi)
        np.testing.assert_allclose(c, ss.eval_legendre(l, xi), atol=2e-13)
        # m = 2: d^l_{20} = sqrt((l-2)!/(l+2)!) P_l^2 with the Condon-Shortley phase
        c2 = col(40, 2, 0, xi)
        l2 = np.arange(2, 41)
        ref = np.sqrt(1.0 / ((l2 - 1.0) * l2 * (l2 + 1.0) * (l2 + 2.0))) * ss.lpmv(2, l2, xi)
        np.testing.assert_allclose(c2[2:], ref, atol=1e-13)


def test_symmetries():
    rng = np.random.default_rng(3)
    for _ in range(8):
        th = rng.uniform(0.05, 3.09)
        m = int(rng.integers(-30, 31))
        z = math.cos(th)
        zr = math.cos(math.pi - th)
        for mp_ in (-2, 2):
            a = col(60, m, mp_, z)
            # reflection: d^l_{m,mp}(pi - theta) = (-1)^(l+m) d^l_{m,-mp}(theta)
            b = col(60, m, -mp_, zr)
            sgn = np.array([(-1.0) ** (l + m) for l in range(61)])
            np.testing.assert_allclose(a, sgn * b, atol=1e-13)
            # transposition: d^l_{mp,m} = (-1)^(m-mp) d^l_{m,mp}
            t = col(60, mp_, m, z)
            np.testing.assert_allclose(t, (-1.0) ** (m - mp_) * a, atol=1e-13)


def test_orthonormal_under_gauss_legendre():
    # 2 pi int 2lambda_lm 2lambda_l'm sin(theta) dtheta = delta_ll'; the GL rule with lmax+1
    # nodes integrates these degree <= 2 lmax polynomials exactly.  The floor comes from rounding
    # the nodes to double.
    lmax = 512
    g = gl_rings(lmax)
    w = g.omega * g.nphi / (2 * np.pi)
    for m in (0, 2, 3, 200, 511):
        L = np.array([col(lmax, m, -2, zz, norm=True) for zz in g.z])
        M = 2 * np.pi * (L.T * w) @ L
        l0 = max(m, 2)
        assert np.abs(M[l0:, l0:] - np.eye(lmax + 1 - l0)).max() < 2e-10


def test_spin2_y20_textbook():
    # 2Y_20 = (1/4) sqrt(15/(2 pi)) sin^2(theta)
    for th in (0.2, 1.0, 2.5):
        c = col(2, 0, -2, math.cos(th), norm=True)
        assert abs(c[2] - 0.25 * math.sqrt(15 / (2 * math.pi)) * math.sin(th) ** 2) < 1e-15
