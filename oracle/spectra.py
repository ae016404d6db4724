"""Oracle of the noise-realisation and power-spectrum stage (test infrastructure only).

What the paper does (Sec. IV, power spectrum results; figure captions of the non-tomographic and
tomographic spectra):
  * shape-noise realisations are made by permuting the observed shear values at random among the
    unmasked pixels and passing each permuted map through the full reconstruction;
  * the noise bias N_l of an auto spectrum is estimated from those realisations (50 of them) and
    the error bars come from their scatter;
  * the cross spectrum correlates the reconstructions of two disjoint random halves of the sample;
    its error bars come from paired realisations, each half shuffled on its own.

Readings taken where the paper gives no formula:
  * spectrum of two reconstructed real fields X, Y (full-sky coefficients, m >= 0 storage):
        C_l^{XY} = (2l + 1)^-1 sum_{m=-l}^{l} Re(X_lm conj(Y_lm))
                 = (2l + 1)^-1 [Re(X_l0 conj(Y_l0)) + 2 sum_{m>0} Re(X_lm conj(Y_lm))]   (l >= 2),
    with C_0 = C_1 = 0 (spin-2 data carry no l < 2).  No f_sky, mask or multiplicative-bias
    correction is applied (the (1+m)^-2 shear-calibration factor is a scalar left to the caller);
  * the shuffle moves the shear only: W = M N^-1 stays with its pixel.  Unmasked pixel j (in
    ascending RING index) receives the shear of unmasked pixel perm[j]; masked pixels get 0;
  * N_l is the mean of the realisations' auto spectra and the error bar their sample standard
    deviation (n - 1 in the denominator; 0 for a single realisation);
  * spectra kept per realisation: EE for the E-mode solve, BB for the B-only solve, and (EE, BB, EB)
    for the joint solve.  For paired halves A, B they are (A_E B_E, A_B B_B, A_E B_B).

Pins (tests/test_oracle_spectra.py): per-degree Parseval on the Gauss-Legendre grid (exact
quadrature) for auto and cross spectra, single-coefficient closed forms, a hand-worked shuffle, and
the identity permutation reproducing the direct solve.
"""
import numpy as np

from .core import alm_index

SPEC_NAMES = {0: ("EE", "BB", "EB"), 1: ("EE",), 2: ("BB",)}


def unmasked_index(mask):
    """Ascending RING indices of the unmasked pixels."""
    return np.flatnonzero(np.asarray(mask) != 0)


def shuffle_shear(g1, g2, mask, perm):
    """Shear permuted among the unmasked pixels: out[u_j] = g[u_perm[j]], zero where masked."""
    u = unmasked_index(mask)
    perm = np.asarray(perm)
    assert perm.shape == u.shape
    o1 = np.zeros_like(np.asarray(g1, dtype=np.float64))
    o2 = np.zeros_like(o1)
    o1[u] = np.asarray(g1)[u[perm]]
    o2[u] = np.asarray(g2)[u[perm]]
    return o1, o2


def spectrum(x, y, lmax, ells=None):
    """C_l^{XY} of two coefficient sets (reading above); all l, or only those in `ells`."""
    x = np.asarray(x)
    y = np.asarray(y)
    out = np.zeros(lmax + 1)
    for l in (range(2, lmax + 1) if ells is None else ells):
        if l < 2:
            continue
        m = np.arange(l + 1)
        i = alm_index(lmax, l, m)
        t = np.real(x[i] * np.conj(y[i]))
        out[l] = (t[0] + 2.0 * np.sum(t[1:])) / (2 * l + 1)
    return out


def solve(o, g1, g2, ninv, mask, mode=0, tol=1e-10, maxiter=4000):
    """Reconstruction of one shear map: (kappa_E, kappa_B) of the joint, E-only or B-only solve."""
    W = o.weights(ninv, mask)
    lam = o.lambda_eff(ninv, mask)
    P = o.precond(ninv, mask, lam)
    b = o.rhs(g1, g2, W)
    z = np.zeros(o.nalm, np.complex128)
    if mode == 0:
        x, _ = o.cg(b, W, lam, P, tol=tol, maxiter=maxiter)
        return x[0], x[1]
    blk = mode - 1
    xk, _ = o.cg(b[blk], W, lam, P, tol=tol, maxiter=maxiter, block=blk)
    return (xk, z) if blk == 0 else (z, xk)


def pair_spectra(o, a, b, mode):
    """Spectra kept for one realisation from the solutions a = (E, B) and b = (E, B)."""
    L = o.lmax
    if mode == 1:
        return np.stack([spectrum(a[0], b[0], L)])
    if mode == 2:
        return np.stack([spectrum(a[1], b[1], L)])
    return np.stack([spectrum(a[0], b[0], L), spectrum(a[1], b[1], L), spectrum(a[0], b[1], L)])


def noise_spectra(o, g1, g2, ninv, mask, perms, mode=0, tol=1e-10, maxiter=4000):
    """Spectra of shuffled realisations.

    One set: g1, g2, ninv of shape (Npix,) and perms (n_real, n_obs); returns auto spectra
    (n_real, nspec, lmax + 1).  Two sets (split halves): g1, g2, ninv of shape (2, Npix) and perms
    (2, n_real, n_obs); realisation k shuffles half q with perms[q, k] and returns the cross spectra
    of the two reconstructions."""
    g1 = np.asarray(g1)
    paired = g1.ndim == 2
    perms = np.asarray(perms)
    nreal = perms.shape[1] if paired else perms.shape[0]
    out = []
    for k in range(nreal):
        if paired:
            sol = []
            for q in range(2):
                s1, s2 = shuffle_shear(g1[q], g2[q], mask, perms[q, k])
                sol.append(solve(o, s1, s2, ninv[q], mask, mode, tol, maxiter))
            out.append(pair_spectra(o, sol[0], sol[1], mode))
        else:
            s1, s2 = shuffle_shear(g1, g2, mask, perms[k])
            x = solve(o, s1, s2, ninv, mask, mode, tol, maxiter)
            out.append(pair_spectra(o, x, x, mode))
    return np.stack(out) if out else np.zeros((0, len(SPEC_NAMES[mode]), o.lmax + 1))


def moments(cls):
    """Mean and sample standard deviation over the realisation axis (axis 0)."""
    cls = np.asarray(cls, dtype=np.float64)
    n = cls.shape[0]
    mean = cls.mean(axis=0)
    std = cls.std(axis=0, ddof=1) if n > 1 else np.zeros_like(mean)
    return mean, std
