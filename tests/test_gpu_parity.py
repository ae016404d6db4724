"""GPU parity: the HIP path through the C ABI against the oracle, element by element.

Tolerances: 1e-10 for FP64 plans, 1e-5 for FP32 plans, as a relative 2-norm over all outputs and
again locally, so that an error confined to a few pixels or coefficients is not diluted by the rest:
per ring for maps (a polar ring of four pixels carries its own bound) and per m for coefficients.
Sizes span several Legendre tiles with ragged tails (non-power-of-two Nside gives Bluestein belt
rings; lmax up to 4 Nside aliases the polar rings)."""
import numpy as np
import pytest

import akra_workloads as wl
from oracle.core import Oracle
from oracle.geometry import healpix_rings

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5}
CASES = [(1, 2), (2, 7), (4, 16), (8, 16), (13, 40), (24, 48), (32, 64), (100, 200), (64, 256)]


def rel(a, b):
    a = np.ravel(a)
    b = np.ravel(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def per_ring(g1, g2, r1, r2, rings):
    """Largest relative error over rings, each ring's (gamma_1, gamma_2) against its own norm."""
    worst, at = 0.0, -1
    for r in range(rings.nrings):
        a, n = int(rings.ofs[r]), int(rings.nphi[r])
        e = rel(np.r_[g1[a:a + n], g2[a:a + n]], np.r_[r1[a:a + n], r2[a:a + n]])
        if e > worst:
            worst, at = e, r
    return worst, at


def per_m(got, ref, lmax):
    """Largest relative error over m of stacked (E, B) coefficients, each m block against its own norm."""
    got = np.asarray(got).reshape(-1, got.shape[-1])
    ref = np.asarray(ref).reshape(-1, ref.shape[-1])
    worst, at = 0.0, -1
    for m in range(lmax + 1):
        lo = m * (2 * lmax + 1 - m) // 2 + m
        sl = slice(lo, lo + lmax + 1 - m)
        if not np.any(ref[:, sl]):
            assert not np.any(got[:, sl]), m
            continue
        e = rel(got[:, sl], ref[:, sl])
        if e > worst:
            worst, at = e, m
    return worst, at


def check_maps(g1, g2, r1, r2, rings, tol):
    assert rel(np.r_[g1, g2], np.r_[r1, r2]) < tol
    e, r = per_ring(g1, g2, r1, r2, rings)
    print("worst ring %d rel %.3e" % (r, e), flush=True)
    assert e < tol, (r, e)


def check_alm(got, ref, lmax, tol):
    assert rel(got, ref) < tol
    e, m = per_m(got, ref, lmax)
    print("worst m %d rel %.3e" % (m, e), flush=True)
    assert e < tol, (m, e)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    return torch, torch.device("cuda", 0)


def _plan(nside, lmax, prec, nrhs=1):
    from paper_2606_06175_amd import Plan
    print("plan nside=%d lmax=%d %s nrhs=%d" % (nside, lmax, prec, nrhs), flush=True)
    return Plan(nside, lmax, nrhs=nrhs, precision=prec, device="cuda:0")


def _mask_ninv(nside, seed):
    g = np.random.default_rng(seed)
    npix = 12 * nside * nside
    vec = wl.pixel_vectors(nside)
    foot = wl.cap_mask(nside, 1.9, 0.4, 0.3, vec)
    n = g.poisson(3.0, npix)
    mask = (foot & (n >= 1)).astype(np.uint8)
    return mask, n / wl.SIGMA_E ** 2


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nside,lmax", CASES)
def test_synth2(torch_dev, nside, lmax, prec):
    torch, dev = torch_dev
    o = Oracle(lmax, healpix_rings(nside))
    aE, aB = wl.random_alm(lmax, 100 + nside), wl.random_alm(lmax, 200 + nside)
    # Im(a_l0) and l < 2 entries must be ignored
    aE2 = aE.copy()
    aE2[: lmax + 1] += 5j
    aE2[0] = 3.0
    p = _plan(nside, lmax, prec)
    g1, g2 = p.synth2(torch.from_numpy(aE2).to(dev), torch.from_numpy(aB).to(dev))
    r1, r2 = o.synth(aE, aB)
    check_maps(g1.cpu().numpy(), g2.cpu().numpy(), r1, r2, o.rings, TOL[prec])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nside,lmax", CASES)
def test_adjoint2(torch_dev, nside, lmax, prec):
    torch, dev = torch_dev
    o = Oracle(lmax, healpix_rings(nside))
    h1, h2 = wl.random_maps(o.rings.npix, 300 + nside)
    p = _plan(nside, lmax, prec)
    cE, cB = p.adjoint2(torch.from_numpy(h1).to(dev), torch.from_numpy(h2).to(dev))
    rE, rB = o.adjoint(h1, h2)
    got = np.stack([cE.cpu().numpy(), cB.cpu().numpy()])
    check_alm(got, np.stack([rE, rB]), lmax, TOL[prec])
    assert np.all(got[:, : lmax + 1].imag == 0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nside,lmax", [(4, 16), (13, 40), (32, 64), (100, 200)])
def test_apply_H(torch_dev, nside, lmax, prec):
    torch, dev = torch_dev
    o = Oracle(lmax, healpix_rings(nside))
    mask, ninv = _mask_ninv(nside, 7)
    lam = o.lambda_eff(ninv, mask)
    x = np.stack([wl.random_alm(lmax, 1, lmin=0), wl.random_alm(lmax, 2, lmin=0)])
    p = _plan(nside, lmax, prec)
    yE, yB = p.apply_H(torch.from_numpy(ninv).to(dev), torch.from_numpy(mask).to(dev),
                       torch.from_numpy(x[0]).to(dev), torch.from_numpy(x[1]).to(dev), lam)
    ref = o.apply_H(x, o.weights(ninv, mask), lam)
    check_alm(np.stack([yE.cpu().numpy(), yB.cpu().numpy()]), ref, lmax, TOL[prec])


def test_rhs_and_custom_kernel(torch_dev):
    torch, dev = torch_dev
    nside, lmax = 16, 40
    o = Oracle(lmax, healpix_rings(nside))
    mask, ninv = _mask_ninv(nside, 8)
    g1, g2 = wl.random_maps(o.rings.npix, 9)
    kern = np.linspace(0.0, 1.5, lmax + 1)
    p = _plan(nside, lmax, "fp64")
    tn, tm = torch.from_numpy(ninv).to(dev), torch.from_numpy(mask).to(dev)
    bE, bB = p.rhs(torch.from_numpy(g1).to(dev), torch.from_numpy(g2).to(dev), tn, tm)
    ref = o.rhs(g1, g2, o.weights(ninv, mask))
    check_alm(np.stack([bE.cpu().numpy(), bB.cpu().numpy()]), ref, lmax, 1e-10)
    bE, bB = p.rhs(torch.from_numpy(g1).to(dev), torch.from_numpy(g2).to(dev), tn, tm, kernel=kern)
    ref = o.rhs(g1, g2, o.weights(ninv, mask), kern=kern)
    check_alm(np.stack([bE.cpu().numpy(), bB.cpu().numpy()]), ref, lmax, 1e-10)


def test_batched_plan_matches_single(torch_dev):
    torch, dev = torch_dev
    nside, lmax, nrhs = 16, 32, 3
    o = Oracle(lmax, healpix_rings(nside))
    A = np.stack([wl.random_alm(lmax, 40 + k) for k in range(nrhs)])
    B = np.stack([wl.random_alm(lmax, 50 + k) for k in range(nrhs)])
    p = _plan(nside, lmax, "fp64", nrhs=nrhs)
    g1, g2 = p.synth2(torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev))
    for k in range(nrhs):
        r1, r2 = o.synth(A[k], B[k])
        check_maps(g1[k].cpu().numpy(), g2[k].cpu().numpy(), r1, r2, o.rings, 1e-10)
    cE, cB = p.adjoint2(g1, g2)
    for k in range(nrhs):
        rE, rB = o.adjoint(g1[k].cpu().numpy(), g2[k].cpu().numpy())
        check_alm(np.stack([cE[k].cpu().numpy(), cB[k].cpu().numpy()]), np.stack([rE, rB]), lmax, 1e-10)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_adjoint_identity_on_gpu(torch_dev, prec):
    # <Y x, h>_pix = <x, Y^H h>_harm with the GPU's own Y and Y^H (property that holds at any size)
    torch, dev = torch_dev
    nside, lmax = 256, 512
    p = _plan(nside, lmax, prec)
    x = [torch.from_numpy(wl.random_alm(lmax, s)).to(dev) for s in (1, 2)]
    h = [torch.from_numpy(a).to(dev) for a in wl.random_maps(12 * nside * nside, 3)]
    g1, g2 = p.synth2(*x)
    cE, cB = p.adjoint2(*h)
    om = 4 * np.pi / (12 * nside * nside)
    lhs = om * float((g1 * h[0] + g2 * h[1]).sum())
    w = torch.full((p.nalm,), 2.0, dtype=torch.float64, device=dev)
    w[: lmax + 1] = 1.0
    rhs = float((w * (x[0].conj() * cE).real).sum() + (w * (x[1].conj() * cB).real).sum())
    assert abs(lhs - rhs) < (1e-12 if prec == "fp64" else 1e-5) * abs(lhs)


def test_zero_input_gives_zero(torch_dev):
    torch, dev = torch_dev
    p = _plan(8, 16, "fp64")
    z = torch.zeros(p.nalm, dtype=torch.complex128, device=dev)
    g1, g2 = p.synth2(z, z)
    assert float(g1.abs().max()) == 0 and float(g2.abs().max()) == 0


@pytest.mark.parametrize("nside,lmax,nrhs", [(8, 16, 3), (13, 40, 10), (32, 64, 9), (256, 512, 3)])
def test_batched_fp32_matrix_core_path(torch_dev, nside, lmax, nrhs):
    # FP32 plans with several right-hand sides synthesise all of them on the matrix cores and run the
    # adjoint on them in groups of eight; synthesis and H of every right-hand side against the oracle
    # (Nside 256: adjoint blocks of near-polar groups in the difference form and of plain groups)
    torch, dev = torch_dev
    o = Oracle(lmax, healpix_rings(nside))
    A = np.stack([wl.random_alm(lmax, 60 + k) for k in range(nrhs)])
    B = np.stack([wl.random_alm(lmax, 80 + k) for k in range(nrhs)])
    p = _plan(nside, lmax, "fp32", nrhs=nrhs)
    g1, g2 = p.synth2(torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev))
    for k in range(nrhs):
        r1, r2 = o.synth(A[k], B[k])
        print("rhs %d" % k, flush=True)
        check_maps(g1[k].cpu().numpy(), g2[k].cpu().numpy(), r1, r2, o.rings, TOL["fp32"])
    mask, ninv = _mask_ninv(nside, 5)
    ninvs = np.stack([ninv * (1.0 + 0.1 * k) for k in range(nrhs)])
    yE, yB = p.apply_H(torch.from_numpy(ninvs).to(dev), torch.from_numpy(mask).to(dev),
                       torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev), 0.02)
    for k in range(nrhs):
        ref = o.apply_H(np.stack([A[k], B[k]]), o.weights(ninvs[k], mask), 0.02)
        print("rhs %d" % k, flush=True)
        check_alm(np.stack([yE[k].cpu().numpy(), yB[k].cpu().numpy()]), ref, lmax, TOL["fp32"])


@pytest.fixture
def split_rings():
    # plans created meanwhile transform every ring whose length is not a power of two as two
    # sub-transforms of length N / 2 (the kernel the largest cap rings use at Nside above 1024)
    from paper_2606_06175_amd import akra
    akra.set_ring_whole_maxm(2)
    yield
    akra.set_ring_whole_maxm(8192)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nside,lmax", [(3, 12), (13, 40), (100, 200)])
def test_split_ring_kernel(torch_dev, split_rings, nside, lmax, prec):
    torch, dev = torch_dev
    o = Oracle(lmax, healpix_rings(nside))
    aE, aB = wl.random_alm(lmax, 400 + nside), wl.random_alm(lmax, 500 + nside)
    p = _plan(nside, lmax, prec)
    g1, g2 = p.synth2(torch.from_numpy(aE).to(dev), torch.from_numpy(aB).to(dev))
    r1, r2 = o.synth(aE, aB)
    check_maps(g1.cpu().numpy(), g2.cpu().numpy(), r1, r2, o.rings, TOL[prec])
    h1, h2 = wl.random_maps(o.rings.npix, 600 + nside)
    cE, cB = p.adjoint2(torch.from_numpy(h1).to(dev), torch.from_numpy(h2).to(dev))
    rE, rB = o.adjoint(h1, h2)
    check_alm(np.stack([cE.cpu().numpy(), cB.cpu().numpy()]), np.stack([rE, rB]), lmax, TOL[prec])
    mask, ninv = _mask_ninv(nside, 7)
    yE, yB = p.apply_H(torch.from_numpy(ninv).to(dev), torch.from_numpy(mask).to(dev),
                       torch.from_numpy(aE).to(dev), torch.from_numpy(aB).to(dev), 0.02)
    ref = o.apply_H(np.stack([aE, aB]), o.weights(ninv, mask), 0.02)
    check_alm(np.stack([yE.cpu().numpy(), yB.cpu().numpy()]), ref, lmax, TOL[prec])


def test_split_ring_kernel_gradient(torch_dev, split_rings):
    # the gradient epilogue of the split kernel against the same gradient with whole-ring kernels
    torch, dev = torch_dev
    from paper_2606_06175_amd import AkraSolve, Plan, akra
    nside, lmax = 13, 26
    mask, ninv = _mask_ninv(nside, 9)
    g1, g2 = (m * mask for m in wl.random_maps(12 * nside * nside, 10))
    cE = torch.from_numpy(wl.random_alm(lmax, 11)).to(dev)

    def grads():
        p = Plan(nside, lmax, precision="fp64", device=dev)
        t = [torch.tensor(a, dtype=torch.float64, device=dev, requires_grad=True) for a in (g1, g2, ninv)]
        xE, xB = AkraSolve.apply(t[0], t[1], t[2], torch.from_numpy(mask).to(dev), p, dict(tol=1e-13, maxiter=5000))
        L = (cE.real * xE.real + cE.imag * xE.imag).sum() + 0.5 * (xB.real ** 2 + xB.imag ** 2).sum()
        L.backward()
        return [a.grad.cpu().numpy() for a in t]

    split = grads()
    akra.set_ring_whole_maxm(8192)
    whole = grads()
    for a, b in zip(split, whole):
        assert rel(a, b) < 1e-9
