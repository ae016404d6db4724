"""Pins of the oracle's synthesis Y, adjoint Y^H, operator H and PCG.

Against: a brute-force dense evaluation of sum_{l,m} 2a_lm 2Y_lm from Wigner's explicit sum
(mpmath), textbook single-mode maps, the adjoint identity, exact quadrature on the
Gauss-Legendre grid (Y^H Y = I, H diagonal on a full uniform sky, closed-form shrinkage),
symmetry/positivity of H, a dense Cholesky solve, and the CG error bound."""
import math

import numpy as np
import pytest

import akra_workloads as wl
from oracle.core import Oracle, alm_index, kernel_l
from oracle.dense import alm_to_dof, dense_solve, dense_system, dense_Y, dof_to_alm, pixel_z_phi
from oracle.geometry import gl_rings, healpix_rings


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def test_kernel_closed_form():
    k = kernel_l(5)
    assert k[0] == 0 and k[1] == 0
    # D_2 = -sqrt(2/3), D_3 = -sqrt(5/6); K = sigma_D D with sigma_D = -1
    assert abs(k[2] - math.sqrt(2.0 / 3.0)) < 1e-16
    assert abs(k[3] - math.sqrt(5.0 / 6.0)) < 1e-16
    assert abs(kernel_l(5, sigma_d=+1.0)[4] + math.sqrt(18.0 / 20.0)) < 1e-16


@pytest.mark.parametrize("nside,lmax", [(2, 6), (4, 8), (3, 11)])
def test_synth_against_brute_force(nside, lmax):
    r = healpix_rings(nside)
    o = Oracle(lmax, r)
    aE = wl.random_alm(lmax, 11)
    aB = wl.random_alm(lmax, 12)
    g1, g2 = o.synth(aE, aB)
    z, phi = pixel_z_phi(r)
    u = alm_to_dof(np.stack([aE, aB]), lmax)
    gam = dense_Y(lmax, z, phi) @ u
    assert rel(g1 + 1j * g2, gam) < 1e-13


def test_single_mode_maps():
    lmax = 6
    r = healpix_rings(4)
    o = Oracle(lmax, r)
    th, ph = r.pixel_angles()
    a = np.zeros(o.nalm, complex)
    a[alm_index(lmax, 2, 0)] = 1.0
    g1, g2 = o.synth(a, 0 * a)
    # E_20 = 1:  gamma = 2a 2Y_20 = -(1/4) sqrt(15/(2pi)) sin^2(theta), real
    ref = -0.25 * math.sqrt(15 / (2 * math.pi)) * np.sin(th) ** 2
    assert np.abs(g1 - ref).max() < 1e-14 and np.abs(g2).max() < 1e-14
    # B modes enter as i times E modes (2a = -(aE + i aB))
    b = wl.random_alm(lmax, 5)
    e1, e2 = o.synth(b, 0 * b)
    f1, f2 = o.synth(0 * b, b)
    assert np.abs((f1 + 1j * f2) - 1j * (e1 + 1j * e2)).max() < 1e-13
    # Im(a_l0) is not a degree of freedom
    c = b.copy()
    c[: lmax + 1] += 1j * 7.0
    h1, h2 = o.synth(c, 0 * c)
    assert np.abs(h1 - e1).max() == 0 and np.abs(h2 - e2).max() == 0


@pytest.mark.parametrize("nside,lmax", [(4, 8), (8, 16), (4, 12), (5, 9)])
def test_adjoint_identity(nside, lmax):
    # <Y x, h>_pix = <x, Y^H h>_harm, Omega-weighted pixel product, full-m harmonic product;
    # includes lmax > 2 Nside (aliasing) and odd Nside
    r = healpix_rings(nside)
    o = Oracle(lmax, r)
    aE, aB = wl.random_alm(lmax, 1), wl.random_alm(lmax, 2)
    h1, h2 = wl.random_maps(r.npix, 3)
    g1, g2 = o.synth(aE, aB)
    lhs = float(np.sum(r.omega[0] * (g1 * h1 + g2 * h2)))
    cE, cB = o.adjoint(h1, h2)
    rhs = o.dot(aE, cE) + o.dot(aB, cB)
    assert abs(lhs - rhs) < 1e-13 * (abs(lhs) + 1)
    # outputs: l < 2 zero, Im at m = 0 zero
    assert np.all(cE[:2] == 0) and np.all(cE[: lmax + 1].imag == 0)


def test_adjoint_against_dense():
    lmax, nside = 6, 3
    r = healpix_rings(nside)
    o = Oracle(lmax, r)
    h1, h2 = wl.random_maps(r.npix, 7)
    z, phi = pixel_z_phi(r)
    Ar = dense_Y(lmax, z, phi)
    Ar = np.vstack([Ar.real, Ar.imag])
    ref = Ar.T @ (r.omega[0] * np.concatenate([h1, h2]))
    cE, cB = o.adjoint(h1, h2)
    assert rel(alm_to_dof(np.stack([cE, cB]), lmax), ref) < 1e-13


def test_adjoint_inverts_synth_on_gauss_legendre():
    # exact quadrature: Y^H Y = I on band-limited (l >= 2) spin-2 fields
    lmax = 24
    o = Oracle(lmax, gl_rings(lmax))
    aE, aB = wl.random_alm(lmax, 21), wl.random_alm(lmax, 22)
    cE, cB = o.adjoint(*o.synth(aE, aB))
    assert rel(np.stack([cE, cB]), np.stack([aE, aB])) < 1e-13


def test_H_full_sky_gauss_legendre_is_diagonal():
    # full uniform sky: H = w K_l^2 + lambda_eff, E and B decoupled (App. A; eq. precond exact)
    lmax = 20
    o = Oracle(lmax, gl_rings(lmax))
    w, lam = 3.7, 0.05
    W = np.full(o.rings.npix, w)
    x = np.stack([wl.random_alm(lmax, 31, lmin=0), wl.random_alm(lmax, 32, lmin=0)])
    y = o.apply_H(x, W, lam)
    Kl = o.kernel()[o.l_of]
    assert rel(y, (w * Kl ** 2 + lam) * x) < 1e-13
    # an E-only input leaves B untouched
    yE = o.apply_H(np.stack([x[0], 0 * x[0]]), W, lam)
    assert np.abs(yE[1]).max() < 1e-13


def _small_problem(nside=4, lmax=8, seed=5):
    r = healpix_rings(nside)
    o = Oracle(lmax, r)
    g = np.random.default_rng(seed)
    vec = wl.pixel_vectors(nside)
    foot = wl.cap_mask(nside, 1.0, 0.5, 0.35, vec)
    n = g.poisson(5.0, r.npix)
    mask = (foot & (n >= 1)).astype(np.uint8)
    ninv = n / wl.SIGMA_E ** 2
    return r, o, mask, ninv


def test_H_symmetric_positive_and_matches_dense():
    r, o, mask, ninv = _small_problem()
    W = o.weights(ninv, mask)
    lam = o.lambda_eff(ninv, mask)
    u = np.stack([wl.random_alm(o.lmax, 41, 0), wl.random_alm(o.lmax, 42, 0)])
    v = np.stack([wl.random_alm(o.lmax, 43, 0), wl.random_alm(o.lmax, 44, 0)])
    Hu, Hv = o.apply_H(u, W, lam), o.apply_H(v, W, lam)
    assert abs(o.dot(u, Hv) - o.dot(Hu, v)) < 1e-12 * abs(o.dot(u, Hv))
    assert o.dot(v, Hv) > 0
    z, phi = pixel_z_phi(r)
    H, Ar, wt = dense_system(o.lmax, z, phi, np.repeat(r.omega, r.nphi), W, lam, o.kernel())
    assert rel(alm_to_dof(Hv, o.lmax), H @ alm_to_dof(v, o.lmax)) < 1e-12
    # l < 2 rows are lambda_eff x only
    assert abs(Hv[0][0] - lam * v[0][0].real) < 1e-14


def test_cg_matches_dense_cholesky_and_obeys_bound():
    r, o, mask, ninv = _small_problem()
    W = o.weights(ninv, mask)
    lam = o.lambda_eff(ninv, mask)
    P = o.precond(ninv, mask, lam)
    g1, g2 = wl.random_maps(r.npix, 9)
    g1 *= mask
    g2 *= mask
    b = o.rhs(g1, g2, W)
    z, phi = pixel_z_phi(r)
    H, Ar, wt = dense_system(o.lmax, z, phi, np.repeat(r.omega, r.nphi), W, lam, o.kernel())
    u_ref, b_ref = dense_solve(H, Ar, wt, g1, g2)
    assert rel(alm_to_dof(b, o.lmax), b_ref) < 1e-13
    errs = []
    xs = []
    x, info = o.cg(b, W, lam, P, tol=1e-12, maxiter=2000, callback=lambda k, xx, rr: xs.append(xx))
    assert info["rel_resid_true"] < 1e-11
    assert rel(alm_to_dof(x, o.lmax), u_ref) < 1e-9
    # eq. cg_convergence in the energy norm: ||e_k||_H <= 2 ((sqrt k - 1)/(sqrt k + 1))^k ||e_0||_H
    ev = np.linalg.eigvalsh(H)
    kap = ev[-1] / ev[0]
    q = (math.sqrt(kap) - 1) / (math.sqrt(kap) + 1)
    e0 = u_ref @ H @ u_ref
    for k, xx in enumerate(xs[:60], start=1):
        e = alm_to_dof(xx, o.lmax) - u_ref
        assert math.sqrt(e @ H @ e) <= 2 * q ** k * math.sqrt(e0) * (1 + 1e-9) + 1e-12


def test_full_sky_shrinkage_closed_form():
    # noise-free full uniform sky on the GL grid: x_hat = w K^2 kappa / (w K^2 + lambda_eff)
    lmax = 16
    o = Oracle(lmax, gl_rings(lmax))
    kap = np.stack([wl.random_alm(lmax, 51, 0), wl.random_alm(lmax, 52, 0)])
    Kl = o.kernel()[o.l_of]
    g1, g2 = o.synth(Kl * kap[0], Kl * kap[1])
    w, lam = 2.0, 1e-3 * 2.0
    W = np.full(o.rings.npix, w)
    b = o.rhs(g1, g2, W)
    x, info = o.cg(b, W, lam, 1.0 / (w + lam), tol=1e-13, maxiter=100)
    ref = o._project(w * Kl ** 2 * kap / (w * Kl ** 2 + lam))
    assert rel(x, ref) < 1e-11


def test_zero_rhs_gives_zero_in_zero_iterations():
    r, o, mask, ninv = _small_problem()
    W = o.weights(ninv, mask)
    x, info = o.cg(np.zeros((2, o.nalm), complex), W, 1.0)
    assert info["iters"] == 0 and np.all(x == 0)
