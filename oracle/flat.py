"""Oracle of the flat-sky variant (test infrastructure only).

The paper notes that the method carries over to flat-sky fields by replacing each spherical harmonic
transform with a 2-D FFT, the four-step operator and the CG solver otherwise unchanged (Sec. II.B,
storage problem, footnote on the flat-sky case).  Written out (readings where the paper is silent):

  * field: an nx x ny grid of square pixels, periodic (the FFT's boundary), maps indexed [i2][i1]
    with i1 the fast (x) index;
  * unknown: the complex convergence z = kappa_E + i kappa_B on the grid (E and B at once, the flat
    analogue of the joint system of App. A);
  * A z = F^-1 (D . F z): F the unitary 2-D DFT (numpy's fft2 with norm="ortho"), D the flat-sky
    Kaiser-Squires kernel D(k) = (k1 + i k2)^2 / |k|^2 with D(0) = 0, k the signed FFT frequencies
    (n1 / nx, n2 / ny); gamma = gamma_1 + i gamma_2 = A z.  D depends only on the direction of k, so
    the pixel size drops out;
  * W = M N^-1 per pixel, lambda_eff = lambda <N^-1>_M, P = (<W> + lambda_eff)^-1 as on the sphere;
  * H z = A^H (W . A z) + lambda_eff z,  b = A^H (W . gamma_obs), with A^H z = F^-1 (conj(D) . F z),
    the adjoint for the product <u, v> = sum_p Re(conj(u_p) v_p);
  * PCG in that product from z0 = 0, stopping at ||r|| / ||b|| < tol.

Pins (tests/test_oracle_flat.py): the FFT-based A equals the operator built from explicit DFT sums;
plane-wave closed forms of the Kaiser-Squires kernel; the adjoint identity; H on a full uniform field
is diagonal and the solve has a closed form; PCG equals a dense Cholesky solve.
"""
import numpy as np


def ks_kernel(nx, ny):
    """D on the [n2][n1] FFT grid."""
    a = np.fft.fftfreq(nx)[None, :]
    b = np.fft.fftfreq(ny)[:, None]
    k2 = a * a + b * b
    D = np.zeros((ny, nx), np.complex128)
    nz = k2 > 0
    num = (a + 1j * b) ** 2
    D[nz] = (num * np.ones_like(k2))[nz] / k2[nz]
    return D


class FlatOracle:
    def __init__(self, nx, ny):
        self.nx, self.ny = int(nx), int(ny)
        self.D = ks_kernel(self.nx, self.ny)

    def synth(self, z):
        return np.fft.ifft2(self.D * np.fft.fft2(z, norm="ortho"), norm="ortho")

    def adjoint(self, g):
        return np.fft.ifft2(np.conj(self.D) * np.fft.fft2(g, norm="ortho"), norm="ortho")

    @staticmethod
    def weights(ninv, mask):
        return np.where(np.asarray(mask) != 0, np.asarray(ninv, dtype=np.float64), 0.0)

    @staticmethod
    def lambda_eff(ninv, mask, lam=1e-3):
        m = np.asarray(mask) != 0
        return lam * float(np.asarray(ninv)[m].mean()) if m.any() else 0.0

    @staticmethod
    def precond(ninv, mask, lam_eff):
        return 1.0 / (float(FlatOracle.weights(ninv, mask).mean()) + lam_eff)

    def apply_H(self, z, W, lam_eff):
        return self.adjoint(W * self.synth(z)) + lam_eff * z

    def rhs(self, g1, g2, W):
        return self.adjoint(W * (np.asarray(g1) + 1j * np.asarray(g2)))

    @staticmethod
    def dot(u, v):
        return float(np.sum(np.real(np.conj(u) * v)))

    def cg(self, b, W, lam_eff, P=1.0, tol=1e-3, maxiter=1000):
        x = np.zeros_like(b)
        r = b.copy()
        z = P * r
        p = z.copy()
        rz = self.dot(r, z)
        bn = np.sqrt(self.dot(b, b))
        hist = []
        it = 0
        if bn == 0:
            return x, dict(iters=0, rel_resid_true=0.0, hist=hist)
        while it < maxiter and np.sqrt(self.dot(r, r)) / bn >= tol:
            w = self.apply_H(p, W, lam_eff)
            alpha = rz / self.dot(p, w)
            x = x + alpha * p
            r = r - alpha * w
            z = P * r
            rz_new = self.dot(r, z)
            p = z + (rz_new / rz) * p
            rz = rz_new
            it += 1
            hist.append(np.sqrt(self.dot(r, r)) / bn)
        rt = b - self.apply_H(x, W, lam_eff)
        return x, dict(iters=it, rel_resid_true=float(np.sqrt(self.dot(rt, rt)) / bn), hist=hist)


def dense_A(nx, ny):
    """A as an explicit (nx ny) x (nx ny) complex matrix from the DFT sums (no FFT), flattened [i2][i1]."""
    def dft(n):
        j = np.arange(n)
        return np.exp(-2j * np.pi * np.outer(j, j) / n) / np.sqrt(n)
    F = np.kron(dft(ny), dft(nx))
    D = ks_kernel(nx, ny).ravel()
    return np.conj(F.T) @ (D[:, None] * F)
