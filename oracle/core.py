"""Oracle operator, right-hand side and PCG (test infrastructure only).

Definitions (paper Sec. II and App. A; where the paper is ambiguous the reading taken is stated inline):
  * alm storage: m >= 0, healpy order i(l, m) = m (2 lmax + 1 - m)/2 + l, complex128.
    Fields are real, so a_{l,-m} = (-1)^m conj(a_lm) (Sec. II.A); Im(a_l0) is not a
    degree of freedom.
  * full-m inner product  <a, b> = sum_l [Re(a_l0* b_l0) + 2 sum_{m>0} Re(a_lm* b_lm)]
    (the vector length (lmax+1)^2 per field used in eq. linear_model).
  * kernel  K_l = sigma_D D_l,  D_l = -sqrt((l-1)(l+2)/(l(l+1))) (eq. Dl_kernel), K_0 = K_1 = 0,
    sigma_D = -1 so that pure-E shear has 2a_lm = -a_E,lm = D_l kappa_lm (eq. Dl_kernel).
  * joint E/B unknowns x = (kappa_E, kappa_B) (App. A, eq. joint_forward);
    A = Y o K, with Y the spin-2 synthesis to pixel centres.
  * W_p = M_p N^-1_p (Sec. II.B storage problem; eq. noise_var, eq. mask), applied once.
  * H v = K Y^H (W (Y K v)) + lambda_eff v,  b = K Y^H (W gamma_obs)
    (eq. normal_eq and eq. ML_estimator_reg), Y^H the exact adjoint carrying the pixel area.
  * lambda_eff = lambda <N^-1>_M (mean over unmasked pixels), lambda = 1e-3.
  * P = (<M^2 N^-1> + lambda_eff)^-1 I, <.> the full-sphere pixel mean (eq. precond).
  * PCG (Sec. II.B inversion problem), x0 = 0, stop when ||r_k|| / ||b|| < tol.
  * block systems (App. A, eq. normal_block): H_kj is block (k, j) of H, k, j in {0: E, 1: B};
    the E-mode solve of the main text is (H_EE + lambda_eff) kappa_E = b_E, and the conditional
    B-mode solve is (H_BB + lambda_eff) kappa_B = b_B - H_BE kappa_E (eq. Bmode_reduced).
"""
import ctypes
import os
import subprocess

import numpy as np

from .geometry import Rings

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "akra_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None


def build(force=False):
    """Compile the C core with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)
        i32p = ctypes.POINTER(ctypes.c_int)
        L.orc_wigner_d.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, dp]
        L.orc_wigner_d.restype = None
        L.orc_synth.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, dp, ip, ip, ip, ip, dp, dp]
        L.orc_synth.restype = None
        L.orc_adjoint.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, dp, ip, ip, ip, ip, dp,
                                  ctypes.c_int, i32p, dp, dp]
        L.orc_adjoint.restype = None
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def alm_size(lmax):
    return (lmax + 1) * (lmax + 2) // 2


def alm_index(lmax, l, m):
    return m * (2 * lmax + 1 - m) // 2 + l


def alm_lm(lmax):
    """(l, m) of every stored coefficient."""
    ls, ms = [], []
    for m in range(lmax + 1):
        ls.append(np.arange(m, lmax + 1))
        ms.append(np.full(lmax + 1 - m, m))
    return np.concatenate(ls), np.concatenate(ms)


def kernel_l(lmax, sigma_d=-1.0):
    """K_l = sigma_D D_l with D_l = -sqrt((l-1)(l+2)/(l(l+1))) for l >= 2 (eq. Dl_kernel), 0 below."""
    k = np.zeros(lmax + 1)
    l = np.arange(2, lmax + 1, dtype=np.float64)
    k[2:] = sigma_d * (-np.sqrt((l - 1) * (l + 2) / (l * (l + 1))))
    return k


def full_dot(a, b, lmax):
    """Full-m inner product of real-field coefficient sets (m >= 0 storage); works on stacked arrays."""
    a = np.asarray(a)
    b = np.asarray(b)
    w = np.full(a.shape[-1], 2.0)
    w[: lmax + 1] = 1.0
    return float(np.sum(w * np.real(np.conj(a) * b)))


class Oracle:
    """Plain CPU evaluation of Y, Y^H, H and PCG on a ring grid (HEALPix or Gauss-Legendre)."""

    def __init__(self, lmax, rings: Rings):
        self.lmax = int(lmax)
        self.rings = rings
        self.nalm = alm_size(self.lmax)
        self.l_of, self.m_of = alm_lm(self.lmax)

    # -- Y ------------------------------------------------------------------------------------
    def synth(self, aE, aB, ring_idx=None):
        """gamma_1, gamma_2 at the pixel centres of the selected rings (others stay zero)."""
        L = lib()
        aE = np.ascontiguousarray(aE, dtype=np.complex128)
        aB = np.ascontiguousarray(aB, dtype=np.complex128)
        assert aE.shape == (self.nalm,) and aB.shape == (self.nalm,)
        rg = self.rings if ring_idx is None else self.rings.subset(ring_idx)
        g1 = np.zeros(self.rings.npix)
        g2 = np.zeros(self.rings.npix)
        if rg.nrings:
            L.orc_synth(self.lmax, _dp(aE.view(np.float64)), _dp(aB.view(np.float64)), rg.nrings,
                        _dp(np.ascontiguousarray(rg.z)),
                        _ip(np.ascontiguousarray(rg.nphi)), _ip(np.ascontiguousarray(rg.p0num)),
                        _ip(np.ascontiguousarray(rg.p0den)), _ip(np.ascontiguousarray(rg.ofs)), _dp(g1), _dp(g2))
        return g1, g2

    # -- Y^H ----------------------------------------------------------------------------------
    def wigner(self, m, mp, z, norm=True):
        """d^l_{m,mp} (times sqrt((2l+1)/4pi) if norm) for l = 0..lmax at cos(theta) = z."""
        out = np.zeros(self.lmax + 1)
        lib().orc_wigner_d(self.lmax, int(m), int(mp), float(z), int(bool(norm)), _dp(out))
        return out

    def adjoint(self, g1, g2, mlist=None, ring_idx=None):
        """Exact adjoint of synth (pixel product weighted by Omega, full-m harmonic product)."""
        L = lib()
        g1 = np.ascontiguousarray(g1, dtype=np.float64)
        g2 = np.ascontiguousarray(g2, dtype=np.float64)
        rg = self.rings if ring_idx is None else self.rings.subset(ring_idx)
        ms = np.arange(self.lmax + 1, dtype=np.int32) if mlist is None else np.asarray(mlist, dtype=np.int32)
        cE = np.zeros(self.nalm, np.complex128)
        cB = np.zeros(self.nalm, np.complex128)
        if rg.nrings and len(ms):
            L.orc_adjoint(self.lmax, _dp(g1), _dp(g2), rg.nrings,
                          _dp(np.ascontiguousarray(rg.z)),
                          _ip(np.ascontiguousarray(rg.nphi)), _ip(np.ascontiguousarray(rg.p0num)),
                          _ip(np.ascontiguousarray(rg.p0den)), _ip(np.ascontiguousarray(rg.ofs)),
                          _dp(np.ascontiguousarray(rg.omega)), len(ms),
                          ms.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                          _dp(cE.view(np.float64)), _dp(cB.view(np.float64)))
        return cE, cB

    # -- helpers ------------------------------------------------------------------------------
    def kernel(self, sigma_d=-1.0):
        return kernel_l(self.lmax, sigma_d)

    def dot(self, a, b):
        return full_dot(a, b, self.lmax)

    def _active_rings(self, W):
        """Rings carrying a nonzero weight; Y and Y^H elsewhere are multiplied by W = 0."""
        act = []
        for r in range(self.rings.nrings):
            o, n = int(self.rings.ofs[r]), int(self.rings.nphi[r])
            if np.any(W[o:o + n] != 0):
                act.append(r)
        return np.asarray(act, dtype=np.int64)

    @staticmethod
    def weights(ninv, mask):
        """W_p = M_p N^-1_p."""
        return np.where(np.asarray(mask) != 0, np.asarray(ninv, dtype=np.float64), 0.0)

    @staticmethod
    def lambda_eff(ninv, mask, lam=1e-3):
        m = np.asarray(mask) != 0
        return lam * float(np.sum(np.asarray(ninv)[m])) / float(np.sum(m))

    @staticmethod
    def precond(ninv, mask, lam_eff):
        W = Oracle.weights(ninv, mask)
        return 1.0 / (float(np.mean(W)) + lam_eff)

    def _project(self, v):
        """Zero Im(a_l0): not a degree of freedom of a real field."""
        v = np.array(v, dtype=np.complex128, copy=True)
        v[..., : self.lmax + 1] = v[..., : self.lmax + 1].real
        return v

    # -- operator -----------------------------------------------------------------------------
    def apply_H(self, x, W, lam_eff, kern=None):
        """H x for stacked x = [kappa_E, kappa_B] (shape (2, nalm))."""
        K = self.kernel() if kern is None else np.asarray(kern, np.float64)
        Kl = K[self.l_of]
        x = self._project(x)
        act = self._active_rings(W)
        g1, g2 = self.synth(Kl * x[0], Kl * x[1], ring_idx=act)
        h1, h2 = W * g1, W * g2
        cE, cB = self.adjoint(h1, h2, ring_idx=act)
        y = np.stack([Kl * cE, Kl * cB]) + lam_eff * x
        return self._project(y)

    def rhs(self, g1, g2, W, kern=None):
        """b = K Y^H (W gamma_obs)."""
        K = self.kernel() if kern is None else np.asarray(kern, np.float64)
        Kl = K[self.l_of]
        act = self._active_rings(W)
        cE, cB = self.adjoint(W * np.asarray(g1), W * np.asarray(g2), ring_idx=act)
        return self._project(np.stack([Kl * cE, Kl * cB]))

    def cg(self, b, W, lam_eff, P=1.0, tol=1e-3, maxiter=1000, x0=None, kern=None, callback=None, block=None):
        """Preconditioned CG with the scalar preconditioner P (eq. precond).

        block None: the joint system, b and x stacked (2, nalm).  block 0 or 1: the E or B block
        system (H_kk + lambda_eff) x = b of App. A, b and x single-block (nalm,) vectors.
        Returns x and a dict with iterations, the recursive residual history and the
        true relative residual ||b - H x|| / ||b||."""
        if block is None:
            def op(v):
                return self.apply_H(v, W, lam_eff, kern)
        else:
            def op(v):
                return self.apply_block(v, W, lam_eff, block, block, kern)
        b = self._project(b)
        bn = np.sqrt(self.dot(b, b))
        if bn == 0.0:
            return np.zeros_like(b), {"iters": 0, "hist": [0.0], "rel_resid_true": 0.0}
        x = np.zeros_like(b) if x0 is None else self._project(x0)
        r = b - op(x) if x0 is not None else b.copy()
        z = P * r
        p = z.copy()
        rz = self.dot(r, z)
        hist = [np.sqrt(self.dot(r, r)) / bn]
        it = 0
        while hist[-1] >= tol and it < maxiter:
            w = op(p)
            alpha = rz / self.dot(p, w)
            x = x + alpha * p
            r = r - alpha * w
            z = P * r
            rz_new = self.dot(r, z)
            p = z + (rz_new / rz) * p
            rz = rz_new
            it += 1
            hist.append(np.sqrt(self.dot(r, r)) / bn)
            if callback:
                callback(it, x, hist[-1])
        rt = b - op(x)
        return x, {"iters": it, "hist": hist, "rel_resid_true": float(np.sqrt(self.dot(rt, rt)) / bn)}

    # -- block systems (App. A) -----------------------------------------------------------------
    def apply_block(self, v, W, lam_eff, out, inp, kern=None):
        """Block (out, inp) of H applied to the single-block vector v, blocks 0 = E and 1 = B
        (eq. normal_block): H applied to v placed in block inp, block out of the result.  The
        regulariser lambda_eff enters the diagonal blocks only."""
        x = np.zeros((2, self.nalm), np.complex128)
        x[inp] = v
        return self.apply_H(x, W, lam_eff, kern)[out]

    def cond_b_rhs(self, g1, g2, W, lam_eff, kE, kern=None):
        """Effective right-hand side of the reduced B-mode system, b_B - H_BE kE (eq. lower_block,
        eq. Bmode_reduced)."""
        return self._project(self.rhs(g1, g2, W, kern)[1] - self.apply_block(kE, W, lam_eff, 1, 0, kern))
