"""Pins of the flat-sky oracle (the four-step operator with a 2-D FFT in place of the SHT).

Against:
  * the operator built from explicit DFT sums (no FFT): layout, normalisation and sign of the FFTs;
  * plane waves, the textbook Kaiser-Squires patterns: an E mode varying along x1 gives
    gamma_1 = kappa, along x2 gamma_1 = -kappa, along the diagonal gamma_2 = kappa; a B mode along x1
    gives gamma_2 = kappa_B; a constant kappa gives no shear;
  * the adjoint identity <A z, g> = <z, A^H g>, and A^H A = I minus the mean;
  * a full uniform field: H is diagonal in k, and the solve has a closed form;
  * PCG against a dense Cholesky solve with a random mask and weights.
"""
import numpy as np
import pytest
import scipy.linalg as sl

from oracle.flat import FlatOracle, dense_A, ks_kernel


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _cz(shape, seed):
    g = np.random.default_rng(seed)
    return g.normal(size=shape) + 1j * g.normal(size=shape)


@pytest.mark.parametrize("nx,ny", [(4, 4), (8, 4), (6, 10), (16, 8)])
def test_fft_operator_equals_explicit_sums(nx, ny):
    o = FlatOracle(nx, ny)
    A = dense_A(nx, ny)
    z = _cz((ny, nx), nx * ny)
    assert rel(o.synth(z).ravel(), A @ z.ravel()) < 1e-13
    assert rel(o.adjoint(z).ravel(), np.conj(A.T) @ z.ravel()) < 1e-13


def test_plane_wave_closed_forms():
    n = 32
    o = FlatOracle(n, n)
    i1 = np.arange(n)[None, :]
    i2 = np.arange(n)[:, None]
    m = 3
    along1 = np.cos(2 * np.pi * m * i1 / n) * np.ones((n, 1))
    along2 = np.cos(2 * np.pi * m * i2 / n) * np.ones((1, n))
    diag = np.cos(2 * np.pi * m * (i1 + i2) / n)
    g = o.synth(along1)
    assert np.allclose(g.real, along1, atol=1e-13) and np.allclose(g.imag, 0, atol=1e-13)
    g = o.synth(along2)
    assert np.allclose(g.real, -along2, atol=1e-13) and np.allclose(g.imag, 0, atol=1e-13)
    g = o.synth(diag)
    assert np.allclose(g.real, 0, atol=1e-13) and np.allclose(g.imag, diag, atol=1e-13)
    g = o.synth(1j * along1)
    assert np.allclose(g.imag, along1, atol=1e-13) and np.allclose(g.real, 0, atol=1e-13)
    assert np.allclose(o.synth(np.full((n, n), 2.5 + 1j)), 0, atol=1e-13)
    # |D| = 1 away from k = 0, D(0) = 0
    D = ks_kernel(n, n)
    assert D[0, 0] == 0 and np.allclose(np.abs(D.ravel()[1:]), 1.0)


@pytest.mark.parametrize("nx,ny", [(8, 8), (16, 4)])
def test_adjoint_identity_and_unitarity(nx, ny):
    o = FlatOracle(nx, ny)
    z = _cz((ny, nx), 1)
    g = _cz((ny, nx), 2)
    assert abs(o.dot(o.synth(z), g) - o.dot(z, o.adjoint(g))) < 1e-12 * np.linalg.norm(z) * np.linalg.norm(g)
    # A^H A z = z - mean(z)
    assert rel(o.adjoint(o.synth(z)), z - z.mean()) < 1e-13


def test_full_uniform_field_closed_form():
    n = 16
    o = FlatOracle(n, n)
    w, lam = 3.0, 0.02
    W = np.full((n, n), w)
    g = _cz((n, n), 5)
    b = o.rhs(g.real, g.imag, W)
    x, info = o.cg(b, W, lam, P=1 / (w + lam), tol=1e-13, maxiter=50)
    xf = w * np.conj(o.D) * np.fft.fft2(g, norm="ortho") / (w + lam)
    xf[0, 0] = 0
    assert rel(x, np.fft.ifft2(xf, norm="ortho")) < 1e-12
    # diagonal H: one iteration (plus the k = 0 mode, which b does not excite)
    assert info["iters"] <= 2


def test_cg_matches_dense_cholesky():
    nx, ny = 8, 6
    o = FlatOracle(nx, ny)
    g = np.random.default_rng(7)
    mask = (g.random((ny, nx)) < 0.7).astype(np.uint8)
    ninv = g.uniform(1, 5, (ny, nx))
    W = o.weights(ninv, mask)
    lam = o.lambda_eff(ninv, mask)
    P = o.precond(ninv, mask, lam)
    gam = _cz((ny, nx), 8) * mask
    b = o.rhs(gam.real, gam.imag, W)
    x, info = o.cg(b, W, lam, P, tol=1e-12, maxiter=2000)
    A = dense_A(nx, ny)
    H = np.conj(A.T) @ (W.ravel()[:, None] * A) + lam * np.eye(nx * ny)
    # the complex system as a real one of twice the size (the product is Re <u, v>)
    Hr = np.block([[H.real, -H.imag], [H.imag, H.real]])
    br = np.r_[b.real.ravel(), b.imag.ravel()]
    xr = sl.cho_solve(sl.cho_factor(Hr), br)
    assert rel(np.r_[x.real.ravel(), x.imag.ravel()], xr) < 1e-9
    assert info["rel_resid_true"] < 1e-11
