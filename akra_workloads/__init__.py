"""Seeded synthetic inputs shaped like the paper's DES Y3 workload (Sec. III).

These stand in for the DES Y3 shear catalog, which is not available: every
input is drawn from a seeded numpy generator with the shapes, sizes and value
distributions of the five benchmark configurations.  The module holds none of
the method's arithmetic (no harmonic transform, no kernel, no operator):
callers turn the convergence coefficients it returns into shear with their own
synthesis.  It serves both the oracle and the HIP path.

Per-pixel quantities follow the paper's pixelisation (Sec. III.B):
  counts n_p ~ Poisson(mu_p) stand in for N_eff (eq. Neff_pixel),
  N^-1_p = n_p / sigma_e^2 with sigma_e = 0.26 (eq. noise_var),
  M_p = footprint_p and n_p >= 1 (eq. mask with N_th in (0, 1]),
  per-component shape noise eps ~ N(0, sigma_e^2 / n_p).
Footprint: union of 3 spherical caps in a DES-like southern area, the common
radius bisected to f_sky, minus small circular holes of radius 2'-10'.
"""
import math

import numpy as np

SIGMA_E = 0.26

# name -> parameters (sizes and distributions of the benchmark configurations)
CONFIGS = {
    # plain FP64 CG, one cap with f_sky = 0.1, Poisson mean 5
    "C1": dict(nside=32, lmax=64, mask="cap", fsky=0.1, mu=5.0, amp=[1e-7], nrhs=1, holes=0),
    # mixed precision vs FP64: 3-cap footprint minus 200 holes, Poisson mean 3
    "C2": dict(nside=512, lmax=1024, mask="footprint", fsky=0.1, mu=3.0, amp=[1e-7], nrhs=1, holes=200),
    # headline single RHS: 2000 holes, mean 2 with a smooth x U[0.5,1.5] depth modulation
    "C3": dict(nside=2048, lmax=4096, mask="footprint", fsky=0.1, mu=2.0, amp=[1e-7], nrhs=1, holes=2000,
               depth=True),
    # batched: 4 tomographic bins x (1 signal + 3 noise realisations) = 16 RHS, shared footprint
    # (the noise right-hand sides rotate the galaxy ellipticities, see make_config)
    "C4": dict(nside=1024, lmax=2048, mask="footprint", fsky=0.1, mu=15.34, amp=[0.5e-7, 1e-7, 1.5e-7, 2e-7],
               nrhs=16, holes=2000, rotate=True),
    # differentiable solve
    "C5": dict(nside=256, lmax=512, mask="footprint", fsky=0.1, mu=5.0, amp=[1e-7], nrhs=1, holes=200),
}
_CFG_NUM = {"C1": 1, "C2": 2, "C3": 3, "C4": 4, "C5": 5}

# random-stream ids inside one configuration
S_KAPPA, S_FOOT, S_COUNTS, S_NOISE, S_DEPTH, S_ROT, S_SHUFFLE, S_SPLIT, S_CAT, S_FLAT = 1, 2, 3, 4, 5, 6, 7, 8, 9, 10


def rng(seed_base, stream):
    return np.random.default_rng(1000 * int(seed_base) + int(stream))


# ---------------------------------------------------------------------------------------------
# pixel centres (HEALPix RING order) -- used only to place caps and holes
# ---------------------------------------------------------------------------------------------
def ring_layout(nside):
    """Per ring: z, pixel count, phi0, first pixel."""
    nside = int(nside)
    zs, ns, p0, ofs = [], [], [], []
    o = 0
    for i in range(1, 4 * nside):
        if i < nside:
            z, n, ph = 1 - i * i / (3.0 * nside * nside), 4 * i, math.pi / (4 * i)
        elif i <= 3 * nside:
            z, n = 4.0 / 3.0 - 2.0 * i / (3.0 * nside), 4 * nside
            ph = math.pi / (4 * nside) * ((i - nside + 1) % 2)
        else:
            ii = 4 * nside - i
            z, n, ph = -(1 - ii * ii / (3.0 * nside * nside)), 4 * ii, math.pi / (4 * ii)
        zs.append(z); ns.append(n); p0.append(ph); ofs.append(o)
        o += n
    return np.array(zs), np.array(ns, np.int64), np.array(p0), np.array(ofs, np.int64)


def pixel_vectors(nside):
    """Unit vectors of all pixel centres, shape (3, Npix), RING order."""
    zs, ns, p0, ofs = ring_layout(nside)
    npix = int(ns.sum())
    z = np.repeat(zs, ns)
    ring = np.repeat(np.arange(len(ns)), ns)
    j = np.arange(npix) - ofs[ring]
    phi = p0[ring] + 2 * np.pi * j / ns[ring]
    s = np.sqrt(np.maximum(0.0, 1 - z * z))
    return np.stack([s * np.cos(phi), s * np.sin(phi), z])


def _unit(theta, phi):
    return np.array([math.sin(theta) * math.cos(phi), math.sin(theta) * math.sin(phi), math.cos(theta)])


def cap_mask(nside, centre_theta, centre_phi, fsky, vec=None):
    """Boolean mask of one spherical cap covering the fraction fsky (cos rho = 1 - 2 fsky)."""
    vec = pixel_vectors(nside) if vec is None else vec
    c = _unit(centre_theta, centre_phi)
    return (c @ vec) >= 1.0 - 2.0 * fsky


def footprint(nside, fsky, nholes, seed_base, vec=None):
    """Union of 3 caps (centres in theta in [95, 130] deg, phi in [0, 90] deg) with the common
    radius bisected so that the union covers fsky, minus nholes holes of radius U[2', 10']
    centred uniformly inside the union.  A pixel is inside when its centre is."""
    g = rng(seed_base, S_FOOT)
    vec = pixel_vectors(nside) if vec is None else vec
    th = np.radians(g.uniform(95.0, 130.0, 3))
    ph = np.radians(g.uniform(0.0, 90.0, 3))
    dots = np.stack([_unit(t, p) @ vec for t, p in zip(th, ph)])
    best = dots.max(axis=0)                      # union covers cos(angle) >= cos(rho)
    lo, hi = -1.0, 1.0                            # bisection on cos(rho)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if np.mean(best >= mid) > fsky:
            lo = mid
        else:
            hi = mid
    mask = best >= hi
    if nholes:
        inside = np.flatnonzero(mask)
        centres = inside[g.integers(0, len(inside), nholes)]
        radii = np.radians(g.uniform(2.0, 10.0, nholes) / 60.0)
        _punch_holes(nside, mask, vec, centres, radii)
    return mask


def _punch_holes(nside, mask, vec, centres, radii):
    zs, ns, p0, ofs = ring_layout(nside)
    th_r = np.arccos(np.clip(zs, -1, 1))
    for cpix, rad in zip(centres, radii):
        c = vec[:, cpix]
        tc = math.acos(max(-1.0, min(1.0, c[2])))
        rings = np.flatnonzero(np.abs(th_r - tc) <= rad + 2.0 / nside)
        if len(rings) == 0:
            continue
        lo, hi = int(ofs[rings[0]]), int(ofs[rings[-1]] + ns[rings[-1]])
        sub = c @ vec[:, lo:hi] >= math.cos(rad)
        mask[lo:hi] &= ~sub


def depth_modulation(nside, seed_base, vec=None, nwaves=16, kscale=20.0):
    """Smooth multiplicative depth u_p = 0.5 + Phi(g_p) in [0.5, 1.5]; g is a unit-variance smooth
    field made of random plane waves exp(i k.n) with |k| ~ kscale evaluated on the sphere."""
    g = rng(seed_base, S_DEPTH)
    vec = pixel_vectors(nside) if vec is None else vec
    k = g.normal(size=(nwaves, 3))
    k *= (kscale * g.uniform(0.5, 1.0, nwaves) / np.linalg.norm(k, axis=1))[:, None]
    phase = g.uniform(0, 2 * np.pi, nwaves)
    v32 = vec.astype(np.float32)
    field = np.zeros(vec.shape[1], np.float32)
    for i in range(nwaves):
        field += np.cos(k[i].astype(np.float32) @ v32 + np.float32(phase[i]))
    field = field.astype(np.float64)
    field = (field - field.mean()) / field.std()
    from scipy.special import ndtr
    return 0.5 + ndtr(field)


# ---------------------------------------------------------------------------------------------
# harmonic-space draws
# ---------------------------------------------------------------------------------------------
def alm_size(lmax):
    return (lmax + 1) * (lmax + 2) // 2


def _l_of(lmax):
    return np.concatenate([np.arange(m, lmax + 1) for m in range(lmax + 1)])


def cl_kappa(lmax, amp=1e-7):
    """C_l = amp (l + 10)^-1.2 for l >= 2, zero below."""
    l = np.arange(lmax + 1, dtype=np.float64)
    cl = amp * (l + 10.0) ** -1.2
    cl[:2] = 0.0
    return cl


def gaussian_alm(lmax, cl, g):
    """Real-field Gaussian coefficients (m >= 0 healpy order): a_l0 ~ N(0, C_l); Re, Im ~ N(0, C_l/2)."""
    l = _l_of(lmax)
    n = alm_size(lmax)
    sd = np.sqrt(np.asarray(cl)[l])
    re = g.normal(size=n)
    im = g.normal(size=n)
    a = sd * (re + 1j * im) / math.sqrt(2.0)
    a[: lmax + 1] = sd[: lmax + 1] * re[: lmax + 1]
    return a


def random_alm(lmax, seed, lmin=2):
    """Unit-variance random coefficients for operator tests (zero below lmin, Im(a_l0) = 0)."""
    g = np.random.default_rng(seed)
    n = alm_size(lmax)
    a = g.normal(size=n) + 1j * g.normal(size=n)
    a[: lmax + 1] = a[: lmax + 1].real
    a[_l_of(lmax) < lmin] = 0
    return a


def random_maps(npix, seed):
    g = np.random.default_rng(seed)
    return g.normal(size=npix), g.normal(size=npix)


# ---------------------------------------------------------------------------------------------
# configurations
# ---------------------------------------------------------------------------------------------
def make_config(name, nside=None, lmax=None):
    """Inputs of one benchmark configuration (optionally at other sizes, same distributions).

    Returns dict with: nside, lmax, nrhs, mask (uint8, Npix), ninv (float64, (nrhs_bins, Npix)),
    kappa (complex128, (nrhs, nalm)) -- E-mode convergence coefficients, B = 0 --,
    eps1/eps2 (float64, (nrhs, Npix)) -- shape noise, zero outside the mask --, bin (int per RHS),
    and rot1/rot2 (float64, (nrhs, Npix), or None when no right-hand side is rotated).
    The observed shear is gamma_obs = M (eps + R Y(K kappa)) with the complex per-pixel factor
    R = rot1 + i rot2 multiplying gamma = gamma_1 + i gamma_2 (R = 1 without rotation); callers
    apply Y and K themselves.

    Configurations with rotate=True (the batched workload) simulate galaxies: pixel p of bin b holds
    n_p galaxies with ellipticity e_j = e_int,j + gamma(p), e_int ~ N(0, sigma_e^2) per component.
    The first right-hand side of a bin is the per-pixel mean of e_j as observed; each further one is
    a shape-noise realisation, the mean of e_j exp(2 i psi_j) with psi_j ~ U[0, pi) drawn afresh, so
    that eps is the mean of the rotated e_int and R the mean of exp(2 i psi_j) (Sec. III.B
    pixelisation; Sec. IV noise realisations)."""
    p = dict(CONFIGS[name])
    c = _CFG_NUM[name]
    nside = int(nside or p["nside"])
    lmax = int(lmax or p["lmax"])
    vec = pixel_vectors(nside)
    npix = vec.shape[1]
    if p["mask"] == "cap":
        foot = cap_mask(nside, math.radians(60.0), math.radians(45.0), p["fsky"], vec)
    else:
        foot = footprint(nside, p["fsky"], p["holes"], c, vec)
    mu = np.full(npix, p["mu"])
    if p.get("depth"):
        mu = mu * depth_modulation(nside, c, vec)
    nb = len(p["amp"])
    nrhs = p["nrhs"]
    gc = rng(c, S_COUNTS)
    counts = np.stack([gc.poisson(mu) for _ in range(nb)])
    mask = (foot[None, :] & (counts >= 1)).all(axis=0) if nb > 1 else (foot & (counts[0] >= 1))
    ninv = counts / SIGMA_E ** 2
    gk = rng(c, S_KAPPA)
    kap = [gaussian_alm(lmax, cl_kappa(lmax, a), gk) for a in p["amp"]]
    per_bin = nrhs // nb
    kappa = np.stack([kap[k // per_bin] for k in range(nrhs)])
    bins = np.array([k // per_bin for k in range(nrhs)])
    if p.get("rotate"):
        e1, e2, r1, r2 = rotated_noise(counts, mask, per_bin, rng(c, S_ROT))
    else:
        gn = rng(c, S_NOISE)
        e1, e2 = [], []
        for k in range(nrhs):
            b = k // per_bin
            sd = np.where(counts[b] > 0, SIGMA_E / np.sqrt(np.maximum(counts[b], 1)), 0.0)
            e1.append(sd * gn.normal(size=npix) * mask)
            e2.append(sd * gn.normal(size=npix) * mask)
        e1, e2, r1, r2 = np.stack(e1), np.stack(e2), None, None
    return dict(name=name, nside=nside, lmax=lmax, nrhs=nrhs, mask=mask.astype(np.uint8), ninv=ninv,
                kappa=kappa, eps1=e1, eps2=e2, rot1=r1, rot2=r2, bin=bins)


def rotated_noise(counts, mask, per_bin, g):
    """Galaxy-level shape noise with random rotations (see make_config).

    counts (nbins, Npix): galaxies per pixel of each bin; only unmasked pixels are populated.  For
    each bin, right-hand side 0 is the per-pixel mean of e_int (the galaxies as observed) with
    R = 1; right-hand sides 1 .. per_bin-1 are the means of e_int exp(2 i psi) and R = the mean of
    exp(2 i psi), psi ~ U[0, pi) per galaxy and realisation.  Returns eps1, eps2, rot1, rot2, each
    (nbins * per_bin, Npix), zero outside the mask."""
    nb, npix = counts.shape
    idx = np.flatnonzero(mask)
    shape = (nb * per_bin, npix)
    e1, e2 = np.zeros(shape), np.zeros(shape)
    r1, r2 = np.zeros(shape), np.zeros(shape)
    for b in range(nb):
        n = counts[b][idx]
        gal = np.repeat(np.arange(len(idx)), n)
        inv_n = 1.0 / n

        def mean(v):
            return np.bincount(gal, weights=v, minlength=len(idx)) * inv_n

        i1 = g.normal(0.0, SIGMA_E, gal.size)
        i2 = g.normal(0.0, SIGMA_E, gal.size)
        k = b * per_bin
        e1[k, idx], e2[k, idx] = mean(i1), mean(i2)
        r1[k, idx] = 1.0
        for j in range(1, per_bin):
            psi = g.uniform(0.0, math.pi, gal.size)
            c2, s2 = np.cos(2.0 * psi), np.sin(2.0 * psi)
            del psi
            k = b * per_bin + j
            e1[k, idx] = mean(i1 * c2 - i2 * s2)
            e2[k, idx] = mean(i1 * s2 + i2 * c2)
            r1[k, idx], r2[k, idx] = mean(c2), mean(s2)
    return e1, e2, r1, r2


# ---------------------------------------------------------------------------------------------
# shape-noise realisations and split halves (Sec. IV power spectra)
# ---------------------------------------------------------------------------------------------
def shuffle_perms(n_obs, n_real, seed_base, half=0):
    """n_real independent uniform permutations of 0 .. n_obs-1 (int32, shape (n_real, n_obs)).

    The random draw of the pixel-shuffling procedure; `half` selects an independent stream for
    the second half of a split sample."""
    g = rng(seed_base, S_SHUFFLE + 100 * int(half))
    out = np.empty((int(n_real), int(n_obs)), np.int32)
    for k in range(int(n_real)):
        out[k] = g.permutation(int(n_obs))
    return out


def split_halves(cfg, seed_base):
    """Two disjoint random halves of the per-pixel galaxies of configuration `cfg` (first bin).

    Each galaxy goes to half A or B with probability 1/2: n_A ~ Binomial(n, 1/2), n_B = n - n_A.
    Returns ninv (2, Npix) = n_half / sigma_e^2 and independent shape noise eps1, eps2 (2, Npix)
    with per-component standard deviation sigma_e / sqrt(n_half), zero where n_half = 0 or the
    shared mask is 0."""
    counts = np.rint(cfg["ninv"][0] * SIGMA_E ** 2).astype(np.int64)
    g = rng(seed_base, S_SPLIT)
    na = g.binomial(counts, 0.5)
    halves = np.stack([na, counts - na])
    mask = cfg["mask"].astype(bool)
    sd = np.where(halves > 0, SIGMA_E / np.sqrt(np.maximum(halves, 1)), 0.0)
    e1 = sd * g.normal(size=halves.shape) * mask
    e2 = sd * g.normal(size=halves.shape) * mask
    return dict(ninv=halves / SIGMA_E ** 2, eps1=e1, eps2=e2)


# ---------------------------------------------------------------------------------------------
# shear catalogue (Sec. III.B pixelisation)
# ---------------------------------------------------------------------------------------------
CAT_R = 0.7      # mean shear response standing in for the sample's <R>
CAT_NTH = 5.0    # N_eff threshold of the mask


def make_catalog(n_gal, seed_base, fsky=0.1, amp=0.02):
    """Synthetic galaxy catalogue shaped like the DES Y3 sample (about 1e8 galaxies over f_sky ~ 0.1).

    Positions are uniform in area inside a southern box z in [-0.95, -0.35], phi in [0, dphi) with
    dphi set by f_sky.  Weights w ~ U[0.2, 1.2].  Ellipticities are eps = R g + n per component,
    g a smooth shear pattern of amplitude `amp` and n ~ N(0, sigma_e^2).  Returns float64 arrays z
    (= cos theta), phi, e1, e2, w and the scalars R, sigma_e, n_th."""
    g = rng(seed_base, S_CAT)
    n = int(n_gal)
    z0, z1 = -0.95, -0.35
    dphi = 4.0 * math.pi * fsky / (z1 - z0)
    z = g.uniform(z0, z1, n)
    phi = g.uniform(0.0, dphi, n)
    w = g.uniform(0.2, 1.2, n)
    s1 = amp * np.sin(3.0 * phi) * np.cos(7.0 * z)
    s2 = amp * np.cos(2.0 * phi) * np.sin(5.0 * z)
    e1 = CAT_R * s1 + SIGMA_E * g.normal(size=n)
    e2 = CAT_R * s2 + SIGMA_E * g.normal(size=n)
    return dict(z=z, phi=phi, e1=e1, e2=e2, w=w, R=CAT_R, sigma_e=SIGMA_E, n_th=CAT_NTH)


def sphere_points(n, seed_base):
    """Directions uniform on the sphere: z ~ U[-1, 1], phi ~ U[0, 2 pi)."""
    g = rng(seed_base, S_CAT + 100)
    return g.uniform(-1.0, 1.0, int(n)), g.uniform(0.0, 2.0 * math.pi, int(n))


# ---------------------------------------------------------------------------------------------
# flat-sky field (the four-step operator with a 2-D FFT)
# ---------------------------------------------------------------------------------------------
def make_flat(nx, ny, seed_base, mu=2.0, border=0.05, holes=2000, amp=1e-2):
    """A flat field of nx x ny square pixels (maps indexed [i2][i1]).

    Mask: the grid minus a border of `border` of each side (zero padding against the periodic
    boundary), minus `holes` circular holes of radius U[2, 10] pixels (scaled down on small grids),
    and pixels with no galaxy.  Counts n ~ Poisson(mu), N^-1 = n / sigma_e^2, shape noise
    eps ~ N(0, sigma_e^2 / n) per component.  kappa_E: a Gaussian random field of power
    amp (|k| + 0.01)^-1.2 in units of the grid frequency (B = 0).  Returns mask (uint8), ninv,
    kappa (complex, kappa_E + i 0), eps1, eps2."""
    g = rng(seed_base, S_FLAT)
    nx, ny = int(nx), int(ny)
    i1 = np.arange(nx)[None, :]
    i2 = np.arange(ny)[:, None]
    bx, by = int(border * nx), int(border * ny)
    foot = (i1 >= bx) & (i1 < nx - bx) & (i2 >= by) & (i2 < ny - by)
    scale = min(nx, ny) / 4096.0
    for _ in range(int(holes * min(1.0, scale * scale * 4))):
        cx, cy = g.uniform(0, nx), g.uniform(0, ny)
        r = max(1.0, g.uniform(2, 10) * max(scale, 0.25))
        x0, x1 = int(max(cx - r, 0)), int(min(cx + r + 1, nx))
        y0, y1 = int(max(cy - r, 0)), int(min(cy + r + 1, ny))
        yy, xx = np.mgrid[y0:y1, x0:x1]
        foot[y0:y1, x0:x1] &= (xx - cx) ** 2 + (yy - cy) ** 2 > r * r
    n = g.poisson(mu, (ny, nx))
    mask = foot & (n >= 1)
    ninv = n / SIGMA_E ** 2
    sd = np.where(n > 0, SIGMA_E / np.sqrt(np.maximum(n, 1)), 0.0)
    e1 = sd * g.normal(size=(ny, nx)) * mask
    e2 = sd * g.normal(size=(ny, nx)) * mask
    kx = np.fft.fftfreq(nx)[None, :]
    ky = np.fft.fftfreq(ny)[:, None]
    pk = amp * (np.sqrt(kx * kx + ky * ky) + 0.01) ** -1.2
    white = np.fft.fft2(g.normal(size=(ny, nx)), norm="ortho")
    kap = np.fft.ifft2(np.sqrt(pk) * white, norm="ortho").real
    return dict(nx=nx, ny=ny, mask=mask.astype(np.uint8), ninv=ninv, kappa=kap.astype(np.complex128), eps1=e1, eps2=e2)
