"""Oracle of the catalogue pixelisation (test infrastructure only).

Sec. III.B (pixelization): galaxies j with ellipticities (eps1_j, eps2_j) and weights w_j are binned
onto the HEALPix RING grid, and per pixel i
  gamma_obs^nu_i = sum_j w_j eps^nu_j / (R sum_j w_j)           (eq. gamma_obs, nu = 1, 2)
  N_eff,i        = (sum_j w_j)^2 / sum_j w_j^2                  (eq. Neff_pixel)
  sigma_n,i^2    = sigma_e^2 / N_eff,i,  N^-1_i = 1 / sigma_n,i^2 (eq. noise_var)
  M_i            = 1 if N_eff,i >= N_th else 0                   (eq. mask)
with R the mean shear response of the sample.

Readings: pixels with sum_j w_j^2 = 0 (no galaxies, or only zero weights) have N_eff = 0 and
N^-1 = 0; where sum_j w_j = 0 the shear is 0.  The sums run over the galaxies of a pixel in catalogue
order (np.bincount accumulates sequentially), products are rounded before they are added, and
R sum_j w_j is formed before the division; the GPU path takes the same operations in the same order,
so the mask decision and every output agree bit for bit.

The pixel of a direction (z = cos theta, phi in [0, 2 pi)) is the RING index of Gorski et al. 2005:
  equatorial belt |z| <= 2/3: with t = phi / (pi/2), the two families of pixel edges are the lines
    u = Nside (1/2 + t) - (3/4) Nside z and v = Nside (1/2 + t) + (3/4) Nside z; jp = floor(u),
    jm = floor(v); the ring, counted from z = 2/3, is ir = Nside + 1 + jp - jm, and the position in
    the ring (jp + jm - Nside + s + 1) / 2 mod 4 Nside with s = 1 - (ir mod 2);
  polar caps |z| > 2/3: with f = t - floor(t) and h = Nside sqrt(3 (1 - |z|)), jp = floor(f h),
    jm = floor((1 - f) h); the ring from the nearest pole is ir = jp + jm + 1 and the position
    floor(t ir) mod 4 ir; north rings start at 2 ir (ir - 1), south rings at Npix - 2 ir (ir + 1).

Pins (tests/test_oracle_pixelize.py): every pixel centre maps to its own index, points jittered inside
a pixel stay there, the north-south mirror relation, equal pixel areas on uniform points, and
hand-worked sums on a tiny catalogue.
"""
import numpy as np


def ang2pix_ring(nside, z, phi):
    """RING pixel index of the directions (z = cos theta, phi in [0, 2 pi))."""
    n = int(nside)
    z = np.asarray(z, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    za = np.abs(z)
    tt = phi / (np.pi / 2)
    pix = np.empty(z.shape, dtype=np.int64)
    eq = za <= 2.0 / 3.0
    # equatorial belt
    t1 = n * (0.5 + tt[eq])
    t2 = n * (z[eq] * 0.75)
    jp = np.floor(t1 - t2).astype(np.int64)
    jm = np.floor(t1 + t2).astype(np.int64)
    ir = n + 1 + jp - jm
    kshift = 1 - (ir & 1)
    ip = ((jp + jm - n + kshift + 1) // 2) % (4 * n)
    pix[eq] = 2 * n * (n - 1) + (ir - 1) * 4 * n + ip
    # polar caps
    pc = ~eq
    tp = tt[pc] - np.floor(tt[pc])
    tmp = n * np.sqrt(3.0 * (1.0 - za[pc]))
    jp = np.floor(tp * tmp).astype(np.int64)
    jm = np.floor((1.0 - tp) * tmp).astype(np.int64)
    ir = jp + jm + 1
    ip = np.floor(tt[pc] * ir).astype(np.int64) % (4 * ir)
    north = z[pc] > 0
    pix[pc] = np.where(north, 2 * ir * (ir - 1) + ip, 12 * n * n - 2 * ir * (ir + 1) + ip)
    return pix


def pixelize(nside, z, phi, e1, e2, w, R, sigma_e, n_th):
    """Per-pixel gamma_obs, N_eff, N^-1 and mask of a catalogue (definitions above)."""
    npix = 12 * int(nside) ** 2
    pix = ang2pix_ring(nside, z, phi)
    w = np.asarray(w, dtype=np.float64)
    sw = np.bincount(pix, weights=w, minlength=npix)
    s1 = np.bincount(pix, weights=w * np.asarray(e1, dtype=np.float64), minlength=npix)
    s2 = np.bincount(pix, weights=w * np.asarray(e2, dtype=np.float64), minlength=npix)
    sww = np.bincount(pix, weights=w * w, minlength=npix)
    den = R * sw
    ok = sw != 0
    g1 = np.zeros(npix)
    g2 = np.zeros(npix)
    g1[ok] = s1[ok] / den[ok]
    g2[ok] = s2[ok] / den[ok]
    has = sww != 0
    neff = np.zeros(npix)
    neff[has] = (sw[has] * sw[has]) / sww[has]
    se2 = sigma_e * sigma_e
    ninv = neff / se2
    mask = (neff >= n_th).astype(np.uint8)
    return dict(pix=pix, g1=g1, g2=g2, neff=neff, ninv=ninv, mask=mask, sw=sw, sww=sww)
