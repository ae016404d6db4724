"""Brute-force definition at tiny sizes (test infrastructure only).

* Wigner d^j_{m'm}(beta) from Wigner's explicit finite sum, and independently from
  its Jacobi-polynomial form, both in mpmath at high precision.
* Spin-weighted harmonics sY_lm(theta, phi) = (-1)^s sqrt((2l+1)/(4pi)) d^l_{m,-s}(theta) e^{i m phi}
  (shear expansion, eq. shear_SH).
* Dense forward operator A = Y K on a real degree-of-freedom vector u whose Euclidean
  product equals the full-m product: per field and (l, m): u = a_l0 for m = 0 and
  u = (sqrt2 Re a_lm, sqrt2 Im a_lm) for m > 0.  Joint E/B unknowns (App. A).
* Dense H = A^T Omega W A + lambda_eff I and b = A^T Omega W gamma_obs (eq. normal_eq,
  eq. ML_estimator_reg), solved by Cholesky.
"""
import math

import mpmath as mp
import numpy as np

from .core import alm_size, alm_index


def _half(beta, z):
    """beta/2 at the working precision, from beta or (exactly) from z = cos(beta)."""
    return (mp.acos(mp.mpf(z)) if z is not None else mp.mpf(beta)) / 2


def wigner_d_sum(j, mprime, m, beta=None, dps=40, z=None):
    """d^j_{m' m}(beta) from Wigner's explicit sum (beta, or its exact cosine z)."""
    with mp.workdps(dps):
        b = _half(beta, z)
        c, s = mp.cos(b), mp.sin(b)
        pref = mp.sqrt(mp.factorial(j + mprime) * mp.factorial(j - mprime) * mp.factorial(j + m) * mp.factorial(j - m))
        tot = mp.mpf(0)
        for k in range(0, 2 * j + 1):
            a1, a2, a3, a4 = j + m - k, k, mprime - m + k, j - mprime - k
            if min(a1, a2, a3, a4) < 0:
                continue
            term = (-1) ** (mprime - m + k) * c ** (2 * j + m - mprime - 2 * k) * s ** (mprime - m + 2 * k)
            term /= mp.factorial(a1) * mp.factorial(a2) * mp.factorial(a3) * mp.factorial(a4)
            tot += term
        return pref * tot


def wigner_d_jacobi(j, mprime, m, beta=None, dps=60, z=None):
    """d^j_{m' m}(beta) from the Jacobi-polynomial form
    d = (-1)^lam sqrt(C(2j-k, k+a) / C(k+b, b)) sin^a(beta/2) cos^b(beta/2) P_k^{(a,b)}(cos beta)."""
    with mp.workdps(dps):
        k = min(j + m, j - m, j + mprime, j - mprime)
        if k == j + m:
            a, lam = mprime - m, mprime - m
        elif k == j - m:
            a, lam = m - mprime, 0
        elif k == j + mprime:
            a, lam = m - mprime, 0
        else:
            a, lam = mprime - m, mprime - m
        b = 2 * j - 2 * k - a
        hb = _half(beta, z)
        val = mp.sqrt(mp.binomial(2 * j - k, k + a) / mp.binomial(k + b, b))
        val *= mp.sin(hb) ** a * mp.cos(hb) ** b * mp.jacobi(k, a, b, mp.cos(2 * hb))
        return (-1) ** lam * val


def spin_lambda(s, l, m, z):
    """sY_lm(theta, 0) = (-1)^s sqrt((2l+1)/(4pi)) d^l_{m,-s}(theta) at cos(theta) = z, as float."""
    if l < max(abs(m), abs(s)):
        return 0.0
    with mp.workdps(40):
        return float((-1) ** s * mp.sqrt(mp.mpf(2 * l + 1) / (4 * mp.pi)) * wigner_d_sum(l, m, -s, z=z))


def dof_layout(lmax):
    """List of (field, l, m, part) for the real DOF vector; part 0 = Re (or the m=0 value), 1 = Im."""
    out = []
    for f in (0, 1):
        for m in range(lmax + 1):
            for l in range(m, lmax + 1):
                out.append((f, l, m, 0))
                if m > 0:
                    out.append((f, l, m, 1))
    return out


def alm_to_dof(x, lmax):
    """Stacked (2, nalm) complex -> real DOF vector (isometry for the full-m product)."""
    u = []
    for (f, l, m, part) in dof_layout(lmax):
        a = x[f][alm_index(lmax, l, m)]
        if m == 0:
            u.append(a.real)
        else:
            u.append(math.sqrt(2.0) * (a.real if part == 0 else a.imag))
    return np.asarray(u)


def dof_to_alm(u, lmax):
    x = np.zeros((2, alm_size(lmax)), np.complex128)
    for k, (f, l, m, part) in enumerate(dof_layout(lmax)):
        i = alm_index(lmax, l, m)
        if m == 0:
            x[f][i] += u[k]
        elif part == 0:
            x[f][i] += u[k] / math.sqrt(2.0)
        else:
            x[f][i] += 1j * u[k] / math.sqrt(2.0)
    return x


def dense_Y(lmax, z, phi):
    """Complex matrix mapping the DOF vector (no kernel) to gamma at points (cos theta = z, phi).

    gamma = sum_{l, all m} 2a_lm 2Y_lm with 2a = -(aE + i aB) and a_{l,-m} = (-1)^m conj(a_lm)."""
    z = np.asarray(z, np.float64)
    phi = np.asarray(phi, np.float64)
    uniq, inv = np.unique(z, return_inverse=True)
    lam = {}
    for ti, t in enumerate(uniq):
        for l in range(2, lmax + 1):
            for m in range(-l, l + 1):
                lam[(ti, l, m)] = spin_lambda(2, l, m, t)
    lay = dof_layout(lmax)
    Ymat = np.zeros((len(z), len(lay)), np.complex128)
    for k, (f, l, m, part) in enumerate(lay):
        if l < 2:
            continue
        lp = np.array([lam[(ti, l, m)] for ti in inv])
        lmn = np.array([lam[(ti, l, -m)] for ti in inv])
        ep = np.exp(1j * m * phi)
        em = np.exp(-1j * m * phi)
        if m == 0:
            a_p, a_m = 1.0, 0.0
        elif part == 0:
            a_p, a_m = 1 / math.sqrt(2.0), (-1) ** m / math.sqrt(2.0)
        else:
            a_p, a_m = 1j / math.sqrt(2.0), -((-1) ** m) * 1j / math.sqrt(2.0)
        fac = -1.0 if f == 0 else -1j          # 2a = -(aE + i aB)
        col = fac * (a_p * lp * ep + (a_m * lmn * em if m > 0 else 0.0))
        Ymat[:, k] = col
    return Ymat


def pixel_z_phi(rings):
    """cos(theta) and phi of every pixel of a ring table."""
    z = np.repeat(rings.z, rings.nphi)
    ring = np.repeat(np.arange(rings.nrings), rings.nphi)
    j = np.arange(rings.npix) - rings.ofs[ring]
    phi = np.pi * rings.p0num[ring] / rings.p0den[ring] + 2 * np.pi * j / rings.nphi[ring]
    return z, phi


def dense_system(lmax, z, phi, omega_pix, W, lam_eff, kern):
    """Dense H (real, DOF coordinates) and the real-row forward matrix Ar = [Re A; Im A]."""
    lay = dof_layout(lmax)
    Kd = np.array([kern[l] for (_, l, _, _) in lay])
    A = dense_Y(lmax, z, phi) * Kd[None, :]
    Ar = np.vstack([A.real, A.imag])
    wt = np.concatenate([omega_pix * W, omega_pix * W])
    H = Ar.T @ (wt[:, None] * Ar) + lam_eff * np.eye(len(lay))
    return H, Ar, wt


def dense_solve(H, Ar, wt, g1, g2):
    import scipy.linalg as sl
    b = Ar.T @ (wt * np.concatenate([g1, g2]))
    cf = sl.cho_factor(H)
    return sl.cho_solve(cf, b), b
