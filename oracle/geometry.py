"""Ring tables for the oracle (test infrastructure only).

HEALPix RING scheme (Gorski et al. 2005, the pixelisation the paper uses in
Sec. III.B): ring i = 1 .. 4 Nside - 1,
  north cap  i < Nside        : N_r = 4i,      z = 1 - i^2/(3 Nside^2),  phi0 = pi/(4i)
  belt       Nside <= i <= 3N : N_r = 4 Nside, z = 4/3 - 2i/(3 Nside),  phi0 = (pi/(4 Nside)) * ((i-Nside+1) mod 2)
  south cap  mirrors the north cap.
Pixel j of ring r sits at phi = phi0 + 2 pi j / N_r; RING index = ring offset + j.
All pixels have the area Omega = 4 pi / Npix.

Gauss-Legendre grid (test grid with exact quadrature): lmax+1 rings at the
Legendre nodes, 2 lmax + 2 pixels per ring, phi0 = 0, Omega_r = 2 pi w_r / N_r.

phi0 is stored as the exact fraction pi * p0num / p0den.
"""
from dataclasses import dataclass

import numpy as np


@dataclass
class Rings:
    z: np.ndarray       # cos(theta) per ring; a ring is defined by this double value
    st: np.ndarray      # sin(theta) derived from z
    nphi: np.ndarray    # pixels per ring (int64)
    p0num: np.ndarray   # phi0 = pi * p0num / p0den (int64)
    p0den: np.ndarray
    ofs: np.ndarray     # first pixel index of the ring (int64)
    omega: np.ndarray   # pixel area of the ring's pixels
    npix: int

    def subset(self, idx):
        idx = np.asarray(idx, dtype=np.int64)
        return Rings(self.z[idx], self.st[idx], self.nphi[idx], self.p0num[idx], self.p0den[idx],
                     self.ofs[idx], self.omega[idx], self.npix)

    @property
    def nrings(self):
        return len(self.z)

    def pixel_angles(self):
        """theta, phi of every pixel (RING order)."""
        th = np.empty(self.npix)
        ph = np.empty(self.npix)
        for r in range(self.nrings):
            n = int(self.nphi[r])
            o = int(self.ofs[r])
            th[o:o + n] = np.arctan2(self.st[r], self.z[r])
            ph[o:o + n] = np.pi * self.p0num[r] / self.p0den[r] + 2 * np.pi * np.arange(n) / n
        return th, ph


def _sin_from_z(z):
    """sin(theta) of rings defined by their double-precision z (1 - |z| is exact for |z| >= 1/2)."""
    az = np.abs(z)
    return np.sqrt((1.0 - az) * (1.0 + az))


def healpix_rings(nside):
    nside = int(nside)
    nr = 4 * nside - 1
    z = np.empty(nr)
    nphi = np.empty(nr, np.int64)
    p0num = np.empty(nr, np.int64)
    p0den = np.empty(nr, np.int64)
    for k in range(nr):
        i = k + 1
        if i < nside or i > 3 * nside:
            ii = i if i < nside else 4 * nside - i
            d = ii * ii / (3.0 * nside * nside)
            z[k] = (1.0 - d) if i < nside else -(1.0 - d)
            nphi[k] = 4 * ii
            p0num[k] = 1
            p0den[k] = 4 * ii
        else:
            z[k] = 4.0 / 3.0 - 2.0 * i / (3.0 * nside)
            nphi[k] = 4 * nside
            p0num[k] = (i - nside + 1) % 2
            p0den[k] = 4 * nside
    st = _sin_from_z(z)
    ofs = np.concatenate([[0], np.cumsum(nphi)[:-1]]).astype(np.int64)
    npix = 12 * nside * nside
    omega = np.full(nr, 4.0 * np.pi / npix)
    return Rings(z, st, nphi, p0num, p0den, ofs, omega, npix)


def gl_rings(lmax, nphi=None):
    lmax = int(lmax)
    x, w = np.polynomial.legendre.leggauss(lmax + 1)
    order = np.argsort(-x)          # north first
    x = x[order]
    w = w[order]
    n = int(nphi) if nphi else 2 * lmax + 2
    nr = lmax + 1
    nph = np.full(nr, n, np.int64)
    ofs = (np.arange(nr) * n).astype(np.int64)
    st = _sin_from_z(x)
    omega = 2.0 * np.pi * w / n
    return Rings(x.copy(), st, nph, np.zeros(nr, np.int64), np.ones(nr, np.int64), ofs, omega, nr * n)
