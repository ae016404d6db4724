"""Pins of the oracle's block systems (App. A): the E-mode solve of the main text and the
conditional B-mode solve.

Against: dense Cholesky solves of the E and B blocks of the dense H (built from Wigner's explicit
sum, independent of the oracle's recurrence), block elimination (the conditional B solve given the
joint E solution returns the joint B solution, eq. lower_block), and exact E/B decoupling on a full
uniform sky with exact quadrature (App. A: H_EB = 0 when M = 1)."""
import numpy as np
import pytest
import scipy.linalg as sl

import akra_workloads as wl
from oracle.core import Oracle
from oracle.dense import alm_to_dof, dense_system, dof_layout, pixel_z_phi
from oracle.geometry import gl_rings, healpix_rings


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


@pytest.fixture(scope="module")
def small():
    nside, lmax = 4, 8
    r = healpix_rings(nside)
    o = Oracle(lmax, r)
    g = np.random.default_rng(71)
    foot = wl.cap_mask(nside, 1.1, 0.4, 0.4, wl.pixel_vectors(nside))
    n = g.poisson(5.0, r.npix)
    mask = (foot & (n >= 1)).astype(np.uint8)
    ninv = n / wl.SIGMA_E ** 2
    W = o.weights(ninv, mask)
    lam = o.lambda_eff(ninv, mask)
    g1, g2 = wl.random_maps(r.npix, 72)
    g1, g2 = g1 * mask, g2 * mask
    z, phi = pixel_z_phi(r)
    H, Ar, wt = dense_system(lmax, z, phi, np.repeat(r.omega, r.nphi), W, lam, o.kernel())
    bd = Ar.T @ (wt * np.concatenate([g1, g2]))
    fld = np.array([f for (f, _, _, _) in dof_layout(lmax)])
    return dict(o=o, W=W, lam=lam, g1=g1, g2=g2, H=H, bd=bd, e=fld == 0, bb=fld == 1,
                P=o.precond(ninv, mask, lam))


def _dof_block(o, v, block):
    x = np.zeros((2, o.nalm), np.complex128)
    x[block] = v
    u = alm_to_dof(x, o.lmax)
    return u


def test_block_apply_matches_dense_blocks(small):
    o, H, e, bb = small["o"], small["H"], small["e"], small["bb"]
    v = wl.random_alm(o.lmax, 73, 0)
    for out, inp in ((0, 0), (0, 1), (1, 0), (1, 1)):
        y = o.apply_block(v, small["W"], small["lam"], out, inp)
        ui = _dof_block(o, v, inp)
        ref = (H @ ui)[e if out == 0 else bb]
        assert rel(_dof_block(o, y, out)[e if out == 0 else bb], ref) < 1e-12, (out, inp)


def test_e_only_solve_matches_dense_cholesky(small):
    o, H, e = small["o"], small["H"], small["e"]
    b = o.rhs(small["g1"], small["g2"], small["W"])
    x, info = o.cg(b[0], small["W"], small["lam"], small["P"], tol=1e-12, maxiter=2000, block=0)
    assert info["rel_resid_true"] < 1e-11
    ref = sl.cho_solve(sl.cho_factor(H[np.ix_(e, e)]), small["bd"][e])
    assert rel(_dof_block(o, x, 0)[e], ref) < 1e-9
    # the masked sky couples E and B: the E-only estimate differs from the joint one
    xj, _ = o.cg(b, small["W"], small["lam"], small["P"], tol=1e-12, maxiter=2000)
    assert rel(x, xj[0]) > 1e-3


def test_conditional_b_matches_dense(small):
    o, H, e, bb = small["o"], small["H"], small["e"], small["bb"]
    b = o.rhs(small["g1"], small["g2"], small["W"])
    kE, _ = o.cg(b[0], small["W"], small["lam"], small["P"], tol=1e-12, maxiter=2000, block=0)
    bt = o.cond_b_rhs(small["g1"], small["g2"], small["W"], small["lam"], kE)
    ue = _dof_block(o, kE, 0)[e]
    bt_ref = small["bd"][bb] - H[np.ix_(bb, e)] @ ue
    assert rel(_dof_block(o, bt, 1)[bb], bt_ref) < 1e-11
    kB, info = o.cg(bt, small["W"], small["lam"], small["P"], tol=1e-12, maxiter=2000, block=1)
    ref = sl.cho_solve(sl.cho_factor(H[np.ix_(bb, bb)]), bt_ref)
    assert rel(_dof_block(o, kB, 1)[bb], ref) < 1e-9


def test_conditional_b_given_joint_e_returns_joint_b(small):
    # block elimination: with kE from the joint solve, the lower block row (eq. lower_block) is
    # solved by the joint kB
    o = small["o"]
    b = o.rhs(small["g1"], small["g2"], small["W"])
    xj, _ = o.cg(b, small["W"], small["lam"], small["P"], tol=1e-13, maxiter=3000)
    bt = o.cond_b_rhs(small["g1"], small["g2"], small["W"], small["lam"], xj[0])
    kB, _ = o.cg(bt, small["W"], small["lam"], small["P"], tol=1e-13, maxiter=3000, block=1)
    assert rel(kB, xj[1]) < 1e-10


def test_full_sky_blocks_decouple():
    # M = 1 with uniform weights and exact quadrature: H_BE = 0, so b~_B = b_B and the E-only and
    # conditional B solves equal the joint solve (App. A)
    lmax = 12
    o = Oracle(lmax, gl_rings(lmax))
    W = np.full(o.rings.npix, 2.5)
    lam = 2.5e-3
    g1, g2 = wl.random_maps(o.rings.npix, 74)
    b = o.rhs(g1, g2, W)
    kE = wl.random_alm(lmax, 75, 0)
    assert np.abs(o.apply_block(kE, W, lam, 1, 0)).max() < 1e-13 * np.abs(kE).max()
    assert rel(o.cond_b_rhs(g1, g2, W, lam, kE), b[1]) < 1e-13
    xj, _ = o.cg(b, W, lam, 1 / (2.5 + lam), tol=1e-13, maxiter=200)
    xe, _ = o.cg(b[0], W, lam, 1 / (2.5 + lam), tol=1e-13, maxiter=200, block=0)
    xb, _ = o.cg(b[1], W, lam, 1 / (2.5 + lam), tol=1e-13, maxiter=200, block=1)
    assert rel(xe, xj[0]) < 1e-11 and rel(xb, xj[1]) < 1e-11
