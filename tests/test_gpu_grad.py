"""Differentiable solve (AkraSolve, akra_cg_solve_vjp): gradients with respect to the shear maps and
the inverse-noise weights, against the dense-matrix reference differentiated by torch on the CPU
and against central finite differences of the GPU solve."""
import numpy as np
import pytest

import akra_workloads as wl
from oracle.core import Oracle, alm_size
from oracle.dense import dense_Y, dof_layout, dof_to_alm, pixel_z_phi
from oracle.geometry import healpix_rings

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.ravel(a)
    b = np.ravel(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _problem(nside, seed):
    g = np.random.default_rng(seed)
    npix = 12 * nside * nside
    vec = wl.pixel_vectors(nside)
    mask = wl.cap_mask(nside, 1.2, 0.7, 0.35, vec).astype(np.uint8)
    ninv = g.uniform(10.0, 60.0, npix)
    g1, g2 = wl.random_maps(npix, seed + 1)
    return mask, ninv, g1 * mask, g2 * mask


def _loss(torch, xE, xB, cE, cB):
    # a linear and a quadratic part, on the stored (Re, Im) of the solution
    return (cE.real * xE.real + cE.imag * xE.imag).sum() + 0.5 * (xB.real ** 2 + xB.imag ** 2).sum() \
        + 0.25 * (cB.real * xB.real).sum()


def _dense_grads(nside, lmax, mask, ninv, g1, g2, cE, cB, lam=1e-3, mode="joint"):
    """Gradient of the same loss with the dense H and b, differentiated by torch on the CPU.
    mode "E": the E block system of App. A (kappa_B = 0)."""
    import torch
    rings = healpix_rings(nside)
    o = Oracle(lmax, rings)
    z, phi = pixel_z_phi(rings)
    lay = dof_layout(lmax)
    K = o.kernel()
    A = dense_Y(lmax, z, phi) * np.array([K[l] for (_, l, _, _) in lay])[None, :]
    Ar = torch.from_numpy(np.vstack([A.real, A.imag]))
    nd = len(lay)
    Pm = np.stack([dof_to_alm(np.eye(nd)[k], lmax).reshape(-1) for k in range(nd)], axis=1)  # (2 nalm, nd)
    Pr, Pi = torch.from_numpy(Pm.real.copy()), torch.from_numpy(Pm.imag.copy())
    om = torch.from_numpy(np.repeat(rings.omega, rings.nphi))
    M = torch.from_numpy(mask.astype(np.float64))
    t_n = torch.tensor(ninv, dtype=torch.float64, requires_grad=True)
    t_1 = torch.tensor(g1, dtype=torch.float64, requires_grad=True)
    t_2 = torch.tensor(g2, dtype=torch.float64, requires_grad=True)
    W = M * t_n
    wt = torch.cat([om * W, om * W])
    lam_eff = lam * W.sum() / M.sum()
    H = Ar.T @ (wt[:, None] * Ar) + lam_eff * torch.eye(nd, dtype=torch.float64)
    b = Ar.T @ (wt * torch.cat([t_1, t_2]))
    if mode == "E":
        e = torch.tensor([f == 0 for (f, _, _, _) in lay])
        u = torch.zeros(nd, dtype=torch.float64)
        u = u.masked_scatter(e, torch.linalg.solve(H[e][:, e], b[e]))
    else:
        u = torch.linalg.solve(H, b)
    x = torch.complex(Pr @ u, Pi @ u)
    na = alm_size(lmax)
    L = _loss(torch, x[:na], x[na:], torch.from_numpy(cE), torch.from_numpy(cB))
    L.backward()
    return t_1.grad.numpy(), t_2.grad.numpy(), t_n.grad.numpy(), float(L.detach()), x.detach().numpy()


def _gpu(nside, lmax, prec, mask, ninv, g1, g2, cE, cB, tol, nrhs=1, mode="joint"):
    import torch
    from paper_2606_06175_amd import AkraSolve, Plan
    print("plan nside=%d lmax=%d %s nrhs=%d" % (nside, lmax, prec, nrhs), flush=True)
    dev = torch.device("cuda", 0)
    p = Plan(nside, lmax, nrhs=nrhs, precision=prec, device=dev)
    t = [torch.tensor(a, dtype=torch.float64, device=dev, requires_grad=True) for a in (g1, g2, ninv)]
    m = torch.from_numpy(mask).to(dev)
    xE, xB = AkraSolve.apply(t[0], t[1], t[2], m, p, dict(tol=tol, maxiter=5000, mode=mode))
    L = _loss(torch, xE, xB, torch.from_numpy(cE).to(dev), torch.from_numpy(cB).to(dev))
    L.backward()
    return [a.grad.cpu().numpy() for a in t], float(L.detach()), p


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", 1e-6)])
def test_gradient_matches_dense_reference(prec, tol):
    nside, lmax = 4, 8
    mask, ninv, g1, g2 = _problem(nside, 3)
    cE = wl.random_alm(lmax, 5)
    cB = wl.random_alm(lmax, 6)
    d1, d2, dn, Lref, _ = _dense_grads(nside, lmax, mask, ninv, g1, g2, cE, cB)
    (a1, a2, an), L, _ = _gpu(nside, lmax, prec, mask, ninv, g1, g2, cE, cB, tol=1e-13 if prec == "fp64" else 1e-12)
    print("L %.15e ref %.15e" % (L, Lref), flush=True)
    assert abs(L - Lref) < tol * abs(Lref)
    e = [rel(np.r_[a1, a2], np.r_[d1, d2]), rel(an, dn)]
    print("rel err d/dgamma %.3e d/dninv %.3e" % tuple(e), flush=True)
    assert e[0] < tol and e[1] < tol
    # masked pixels carry no gradient
    assert np.all(a1[mask == 0] == 0) and np.all(an[mask == 0] == 0)


def test_gradient_matches_finite_differences():
    import torch
    nside, lmax = 8, 16
    mask, ninv, g1, g2 = _problem(nside, 11)
    cE = wl.random_alm(lmax, 12)
    cB = wl.random_alm(lmax, 13)
    (a1, a2, an), L0, p = _gpu(nside, lmax, "fp64", mask, ninv, g1, g2, cE, cB, tol=1e-13)
    dev = torch.device("cuda", 0)
    m = torch.from_numpy(mask).to(dev)
    tcE, tcB = torch.from_numpy(cE).to(dev), torch.from_numpy(cB).to(dev)

    def L(a, b, n):
        xE, xB, _ = p.cg_solve(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev),
                               torch.from_numpy(n).to(dev), m, tol=1e-13, maxiter=5000)
        return float(_loss(torch, xE, xB, tcE, tcB))

    rng = np.random.default_rng(17)
    pix = rng.choice(np.flatnonzero(mask), 6, replace=False)
    for q in pix:
        # L is quadratic in gamma: the central difference is exact for any step up to rounding, and
        # a step of 0.1 keeps the solves' rounding small against the difference it divides
        h = 1e-1
        for which, grad in ((0, a1), (1, a2)):
            a, b = g1.copy(), g2.copy()
            (a if which == 0 else b)[q] += h
            Lp = L(a, b, ninv)
            (a if which == 0 else b)[q] -= 2 * h
            Lm = L(a, b, ninv)
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - grad[q]) < 1e-6 * max(abs(fd), 1e-3 * np.abs(grad).max()), (q, which, fd, grad[q])
        # L is not polynomial in ninv: Richardson extrapolation of two central differences cancels
        # the O(h^2) term, which lets the step be large against the solves' rounding
        def central(hn):
            n = ninv.copy()
            n[q] += hn
            Lp = L(g1, g2, n)
            n[q] -= 2 * hn
            return (Lp - L(g1, g2, n)) / (2 * hn)
        hn = 1e-3 * ninv[q]
        fd = (4 * central(hn) - central(2 * hn)) / 3
        assert abs(fd - an[q]) < 1e-5 * max(abs(fd), 1e-3 * np.abs(an).max()), (q, fd, an[q])


def test_batched_gradient_matches_single():
    import torch
    from paper_2606_06175_amd import AkraSolve, Plan
    nside, lmax = 8, 16
    mask, ninv, g1, g2 = _problem(nside, 21)
    cE = wl.random_alm(lmax, 22)
    cB = wl.random_alm(lmax, 23)
    single = [_gpu(nside, lmax, "fp64", mask, n, a, b, cE, cB, tol=1e-12)[0]
              for (n, a, b) in ((ninv, g1, g2), (0.5 * ninv + 7.0, -g2, g1))]
    dev = torch.device("cuda", 0)
    p = Plan(nside, lmax, nrhs=2, precision="fp64", device=dev)
    t = [torch.tensor(np.stack(v), dtype=torch.float64, device=dev, requires_grad=True)
         for v in ((g1, -g2), (g2, g1), (ninv, 0.5 * ninv + 7.0))]
    xE, xB = AkraSolve.apply(t[0], t[1], t[2], torch.from_numpy(mask).to(dev), p, dict(tol=1e-12, maxiter=5000))
    tcE, tcB = torch.from_numpy(cE).to(dev), torch.from_numpy(cB).to(dev)
    L = sum(_loss(torch, xE[k], xB[k], tcE, tcB) for k in range(2))
    L.backward()
    for k in range(2):
        for j in range(3):
            assert rel(t[j].grad[k].cpu().numpy(), single[k][j]) < 1e-9


def test_e_only_gradient_matches_dense_reference():
    # the differentiable E-mode solve (App. A E block): both solves of AkraSolve run on the block
    nside, lmax = 4, 8
    mask, ninv, g1, g2 = _problem(nside, 41)
    cE = wl.random_alm(lmax, 42)
    cB = wl.random_alm(lmax, 43)
    d1, d2, dn, Lref, xref = _dense_grads(nside, lmax, mask, ninv, g1, g2, cE, cB, mode="E")
    (a1, a2, an), L, _ = _gpu(nside, lmax, "fp64", mask, ninv, g1, g2, cE, cB, tol=1e-13, mode="E")
    print("L %.15e ref %.15e" % (L, Lref), flush=True)
    assert abs(L - Lref) < 1e-9 * abs(Lref)
    e = [rel(np.r_[a1, a2], np.r_[d1, d2]), rel(an, dn)]
    print("rel err d/dgamma %.3e d/dninv %.3e" % tuple(e), flush=True)
    assert e[0] < 1e-9 and e[1] < 1e-9
