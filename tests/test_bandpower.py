"""The band-power loss of the differentiable solve (E-mode C_l of the solution averaged over 8
logarithmic bins, summed) against hand-worked values: bin edges, powers and gradient."""
import numpy as np
import torch

from paper_2606_06175_amd.bandpower import BandPower, log_bin_edges


def idx(lmax, l, m):
    return m * (2 * lmax + 1 - m) // 2 + l


def test_bin_edges_hand_worked():
    # round(2 (lmax+1 / 2)^(k/8)), k = 0..8, duplicates dropped
    assert log_bin_edges(512).tolist() == [2, 4, 8, 16, 32, 64, 128, 256, 513]
    assert log_bin_edges(32).tolist() == [2, 3, 4, 6, 8, 12, 16, 23, 33]
    assert log_bin_edges(8).tolist() == [2, 3, 4, 5, 6, 7, 9]
    assert log_bin_edges(4).tolist() == [2, 3, 4, 5]


def test_band_powers_hand_worked():
    lmax = 4
    a = np.zeros((lmax + 1) * (lmax + 2) // 2, np.complex128)
    a[idx(lmax, 0, 0)] = 7.0          # l < 2: not part of any band
    a[idx(lmax, 1, 1)] = 5.0 + 5.0j
    a[idx(lmax, 2, 0)] = 1.0
    a[idx(lmax, 2, 1)] = 1.0 + 1.0j
    a[idx(lmax, 2, 2)] = 2.0j
    a[idx(lmax, 3, 0)] = 3.0
    a[idx(lmax, 4, 3)] = 0.5
    t = torch.tensor(a, requires_grad=True)
    bp = BandPower(lmax)
    # C_2 = (1 + 2 * 2 + 2 * 4) / 5, C_3 = 9 / 7, C_4 = 2 * 0.25 / 9; one degree per bin
    want = np.array([13 / 5, 9 / 7, 1 / 18])
    np.testing.assert_allclose(bp.cl(t.detach()).numpy(), [0, 0, 13 / 5, 9 / 7, 1 / 18], rtol=1e-15)
    np.testing.assert_allclose(bp.powers(t.detach()).numpy(), want, rtol=1e-15)
    L = bp.loss(t)
    assert abs(float(L.detach()) - 2483 / 630) < 1e-15
    L.backward()
    g = t.grad.numpy()
    # dL/dRe a_21 = 2 * 2 Re a_21 / 5, dL/dIm a_22 = 2 * 2 Im a_22 / 5, dL/dRe a_30 = 2 Re a_30 / 7
    # (torch's gradient of a real loss in a complex tensor is dL/dRe + i dL/dIm)
    assert abs(g[idx(lmax, 2, 1)] - (0.8 + 0.8j)) < 1e-15
    assert abs(g[idx(lmax, 2, 2)] - 1.6j) < 1e-15
    assert abs(g[idx(lmax, 3, 0)] - 6 / 7) < 1e-15
    assert g[idx(lmax, 0, 0)] == 0 and g[idx(lmax, 1, 1)] == 0


def test_bins_average_their_degrees():
    # C_l = l on every degree: the band power of [e_b, e_{b+1}) is the mean degree of the bin
    lmax = 32
    bp = BandPower(lmax)
    a = np.zeros((lmax + 1) * (lmax + 2) // 2, np.complex128)
    for l in range(2, lmax + 1):
        a[idx(lmax, l, 0)] = np.sqrt(l * (2 * l + 1))
    P = bp.powers(torch.tensor(a)).numpy()
    e = bp.edges
    np.testing.assert_allclose(P, [(e[b] + e[b + 1] - 1) / 2 for b in range(8)], rtol=1e-14)
