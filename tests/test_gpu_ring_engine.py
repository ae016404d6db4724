"""The register engine of the ring stage (rings whose transform length is 4096 or 8192: whole
power-of-two rings and whole-ring Bluestein convolutions) against the oracle, per ring and per m, and
against the LDS kernels it replaces on every mode: synthesis (F to maps), adjoint (maps to G), the
fused operator and the gradient epilogue.

HEALPix Nside 512 gives Bluestein rings of 4096 points (N = 1028 .. 2044); Nside 1024 adds the
4096-point belt and Bluestein rings of 8192 points (N = 2052 .. 4092).  The 8192-point belt of Nside
2048 is covered by the benchmark-size tests."""
import numpy as np
import pytest

import akra_workloads as wl
from oracle.core import Oracle
from oracle.geometry import healpix_rings

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5}


def rel(a, b):
    a = np.ravel(a)
    b = np.ravel(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _plan(nside, lmax, prec, engine=True, nrhs=1):
    from paper_2606_06175_amd import Plan, akra
    akra.set_ring_register_engine(engine)
    try:
        print("plan nside=%d lmax=%d %s engine=%d nrhs=%d" % (nside, lmax, prec, engine, nrhs), flush=True)
        return Plan(nside, lmax, nrhs=nrhs, precision=prec, device="cuda:0")
    finally:
        akra.set_ring_register_engine(True)


def _ring_classes(nside):
    """One ring index of each class the register engine takes, north and south, and two others."""
    rings = healpix_rings(nside)
    n = rings.nphi
    out = []

    def m_of(N):
        M = 1
        while M < 2 * N - 1:
            M <<= 1
        return M
    for want in ("p2_4096", "p2_8192", "blue_4096", "blue_8192"):
        for r in range(rings.nrings):
            N = int(n[r])
            p2 = (N & (N - 1)) == 0
            ok = {"p2_4096": p2 and N == 4096, "p2_8192": p2 and N == 8192,
                  "blue_4096": not p2 and m_of(N) == 4096, "blue_8192": not p2 and m_of(N) == 8192}[want]
            if ok:
                out += [r, rings.nrings - 1 - r]
                break
    return sorted(set(out + [0, rings.nrings // 2]))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nside,lmax", [(512, 1024), (1024, 2048), (1024, 4096)])
def test_engine_synth_and_adjoint_against_oracle(nside, lmax, prec):
    import torch
    dev = torch.device("cuda", 0)
    o = Oracle(lmax, healpix_rings(nside))
    rs = _ring_classes(nside)
    ms = [0, 2, lmax // 3, lmax]
    aE, aB = wl.random_alm(lmax, 31), wl.random_alm(lmax, 32)
    h1, h2 = wl.random_maps(o.rings.npix, 33)
    print("oracle: %d rings, %d m" % (len(rs), len(ms)), flush=True)
    r1, r2 = o.synth(aE, aB, ring_idx=rs)
    rE, rB = o.adjoint(h1, h2, mlist=ms)
    p = _plan(nside, lmax, prec)
    g1, g2 = p.synth2(torch.from_numpy(aE).to(dev), torch.from_numpy(aB).to(dev))
    g1, g2 = g1.cpu().numpy(), g2.cpu().numpy()
    cE, cB = p.adjoint2(torch.from_numpy(h1).to(dev), torch.from_numpy(h2).to(dev))
    cE, cB = cE.cpu().numpy(), cB.cpu().numpy()
    p.close()
    for r in rs:
        a, n = int(o.rings.ofs[r]), int(o.rings.nphi[r])
        e = rel(np.r_[g1[a:a + n], g2[a:a + n]], np.r_[r1[a:a + n], r2[a:a + n]])
        print("ring %d (N %d) rel %.3e" % (r, n, e), flush=True)
        assert e < TOL[prec], (r, e)
    for m in ms:
        sl = slice(m * (2 * lmax + 1 - m) // 2 + m, m * (2 * lmax + 1 - m) // 2 + lmax + 1)
        e = rel(np.r_[cE[sl], cB[sl]], np.r_[rE[sl], rB[sl]])
        print("m %d rel %.3e" % (m, e), flush=True)
        assert e < TOL[prec], (m, e)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nside,lmax,nrhs", [(512, 1024, 1), (1024, 2048, 1), (1024, 2048, 3)])
def test_engine_matches_lds_kernels(nside, lmax, nrhs, prec):
    # every ring-stage mode with the register engine against the LDS kernels: the two compute the
    # same transforms in different orders, so they agree to rounding
    import torch
    dev = torch.device("cuda", 0)
    tol = 1e-12 if prec == "fp64" else 2e-6
    npix = 12 * nside * nside
    A = torch.from_numpy(np.stack([wl.random_alm(lmax, 40 + k) for k in range(nrhs)])).to(dev)
    B = torch.from_numpy(np.stack([wl.random_alm(lmax, 50 + k) for k in range(nrhs)])).to(dev)
    hs = [wl.random_maps(npix, 60 + k) for k in range(nrhs)]
    h1 = torch.from_numpy(np.stack([h[0] for h in hs])).to(dev)
    h2 = torch.from_numpy(np.stack([h[1] for h in hs])).to(dev)
    g = np.random.default_rng(7)
    mask = torch.from_numpy((g.uniform(size=npix) < 0.7).astype(np.uint8)).to(dev)
    ninv = torch.from_numpy(np.stack([g.uniform(5.0, 60.0, npix) for _ in range(nrhs)])).to(dev)
    out = {}
    for engine in (True, False):
        p = _plan(nside, lmax, prec, engine, nrhs)
        if nrhs == 1:
            s = p.synth2(A[0].contiguous(), B[0].contiguous())
            a = p.adjoint2(h1[0].contiguous(), h2[0].contiguous())
            y = p.apply_H(ninv[0].contiguous(), mask, A[0].contiguous(), B[0].contiguous(), 0.01)
        else:
            s = p.synth2(A, B)
            a = p.adjoint2(h1, h2)
            y = p.apply_H(ninv, mask, A, B, 0.01)
        out[engine] = [t.cpu().numpy() for t in (*s, *a, *y)]
        p.close()
    for name, x, y in zip(("synth g1", "synth g2", "adjoint E", "adjoint B", "H E", "H B"), out[True], out[False]):
        e = rel(x, y)
        print("%s rel %.3e" % (name, e), flush=True)
        assert e < tol, (name, e)


def test_engine_gradient_matches_lds_kernels():
    # the gradient epilogue (ring mode 3) of the differentiable solve with and without the engine
    import torch
    from paper_2606_06175_amd import AkraSolve
    nside, lmax = 512, 1024
    dev = torch.device("cuda", 0)
    npix = 12 * nside * nside
    g = np.random.default_rng(8)
    mask = (g.uniform(size=npix) < 0.6).astype(np.uint8)
    ninv = g.uniform(5.0, 60.0, npix)
    a1, a2 = (m * mask for m in wl.random_maps(npix, 9))
    cE = torch.from_numpy(wl.random_alm(lmax, 10)).to(dev)
    res = {}
    for engine in (True, False):
        p = _plan(nside, lmax, "fp64", engine)
        t = [torch.tensor(v, dtype=torch.float64, device=dev, requires_grad=True) for v in (a1, a2, ninv)]
        xE, xB = AkraSolve.apply(t[0], t[1], t[2], torch.from_numpy(mask).to(dev), p, dict(tol=1e-12, maxiter=3000))
        L = (cE.real * xE.real + cE.imag * xE.imag).sum() + 0.5 * (xB.real ** 2 + xB.imag ** 2).sum()
        L.backward()
        res[engine] = [v.grad.cpu().numpy() for v in t]
        p.close()
    for x, y in zip(res[True], res[False]):
        assert rel(x, y) < 1e-9


@pytest.fixture
def split_rings():
    # plans created meanwhile transform every ring whose length is not a power of two as two
    # sub-transforms of length N / 2 (at Nside 1024 those of N > 2048 run in the register engine)
    from paper_2606_06175_amd import akra
    akra.set_ring_whole_maxm(2)
    yield
    akra.set_ring_whole_maxm(8192)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_engine_split_rings(split_rings, prec):
    import torch
    dev = torch.device("cuda", 0)
    nside, lmax = 1024, 2048
    npix = 12 * nside * nside
    o = Oracle(lmax, healpix_rings(nside))
    rs = [600, 801, 1022, 4094 - 801]  # N = 2404, 3208, 4092 and a south ring: halves of 4096 points
    aE, aB = wl.random_alm(lmax, 71), wl.random_alm(lmax, 72)
    r1, r2 = o.synth(aE, aB, ring_idx=rs)
    p = _plan(nside, lmax, prec)
    g1, g2 = p.synth2(torch.from_numpy(aE).to(dev), torch.from_numpy(aB).to(dev))
    g1, g2 = g1.cpu().numpy(), g2.cpu().numpy()
    for r in rs:
        a, n = int(o.rings.ofs[r]), int(o.rings.nphi[r])
        e = rel(np.r_[g1[a:a + n], g2[a:a + n]], np.r_[r1[a:a + n], r2[a:a + n]])
        print("ring %d (N %d) rel %.3e" % (r, n, e), flush=True)
        assert e < TOL[prec], (r, e)
    g = np.random.default_rng(11)
    mask = torch.from_numpy((g.uniform(size=npix) < 0.7).astype(np.uint8)).to(dev)
    ninv = torch.from_numpy(g.uniform(5.0, 60.0, npix)).to(dev)
    h1, h2 = (torch.from_numpy(m).to(dev) for m in wl.random_maps(npix, 73))
    x = [torch.from_numpy(a).to(dev) for a in (aE, aB)]
    out = {}
    for engine in (True, False):
        q = p if engine else _plan(nside, lmax, prec, engine=False)
        res = [*q.adjoint2(h1, h2), *q.apply_H(ninv, mask, x[0], x[1], 0.01)]
        out[engine] = [t.cpu().numpy() for t in res]
        q.close()
    tol = 1e-12 if prec == "fp64" else 2e-6
    for name, a, b in zip(("adjoint E", "adjoint B", "H E", "H B"), out[True], out[False]):
        e = rel(a, b)
        print("%s rel %.3e" % (name, e), flush=True)
        assert e < tol, (name, e)
