"""E-mode band power of a reconstructed convergence, as a differentiable torch loss.

The spectrum of a set of real-field coefficients (m >= 0 storage, healpy order) is the full-sky
estimator C_l = (|a_l0|^2 + 2 sum_{m>0} |a_lm|^2) / (2l + 1) for l >= 2; the band power of a bin is
the mean of C_l over the degrees of that bin, and the bins are logarithmic in l with edges
unique(round(geomspace(2, lmax + 1, nbins + 1))), bin b holding the degrees e_b <= l < e_{b+1}.
The loss is the sum of the band powers.  This is the objective the differentiable solve is timed
and checked with; it is a plain torch function of the solution, so gradients reach the solve's
inputs through AkraSolve's backward.
"""
import numpy as np
import torch


def log_bin_edges(lmax, nbins=8):
    """Degree edges of the logarithmic bins: unique(round(geomspace(2, lmax + 1, nbins + 1)))."""
    if lmax < 2:
        raise ValueError("band powers need lmax >= 2")
    return np.unique(np.round(np.geomspace(2.0, lmax + 1.0, int(nbins) + 1)).astype(np.int64))


class BandPower:
    """Band powers of coefficient sets with band limit lmax, on one device (tables built once)."""

    def __init__(self, lmax, nbins=8, device=None):
        self.lmax = int(lmax)
        self.edges = log_bin_edges(self.lmax, nbins)
        self.nbins = len(self.edges) - 1
        l = np.concatenate([np.arange(m, self.lmax + 1) for m in range(self.lmax + 1)])
        w = np.where(np.arange(len(l)) <= self.lmax, 1.0, 2.0)          # m = 0 once, m > 0 twice
        dev = torch.device(device) if device is not None else None
        self.l_of = torch.from_numpy(l).to(dev)
        self.w = torch.from_numpy(w / (2.0 * l + 1.0)).to(dev)
        # bin matrix: row b averages C_l over e_b <= l < e_{b+1}
        B = np.zeros((self.nbins, self.lmax + 1))
        for b in range(self.nbins):
            lo, hi = self.edges[b], self.edges[b + 1]
            B[b, lo:hi] = 1.0 / (hi - lo)
        self.B = torch.from_numpy(B).to(dev)

    def cl(self, a):
        """C_l of coefficients a (complex128, [..., n_alm]); zero for l < 2."""
        p = self.w * (a.real * a.real + a.imag * a.imag)
        out = torch.zeros(a.shape[:-1] + (self.lmax + 1,), dtype=p.dtype, device=p.device)
        out = out.index_add(-1, self.l_of, p)
        out[..., :2] = 0.0
        return out

    def powers(self, a):
        """Band powers P_b, [..., nbins]."""
        return self.cl(a) @ self.B.T

    def loss(self, a):
        """Sum of the band powers (summed over any leading dimensions)."""
        return self.powers(a).sum()
