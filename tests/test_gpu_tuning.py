"""Every Legendre launch shape the autotuner may pick gives the oracle's result (GPU)."""
import numpy as np
import pytest

import akra_workloads as wl
from oracle.core import Oracle
from oracle.geometry import healpix_rings

pytestmark = pytest.mark.gpu

SYN = [(v, r) for v in (0, 1) for r in (1, 2, 4)]
ADJ = [(r, 1, c) for c in (8, 4) for r in range(1, 9)] + \
      [(1, 2, 8), (1, 4, 8), (2, 2, 8), (2, 4, 8), (4, 2, 8), (4, 4, 8), (8, 2, 8), (2, 4, 4), (4, 2, 4), (4, 4, 4)]


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_all_shapes_match_oracle(prec, tol):
    import torch
    from paper_2606_06175_amd import Plan
    nside, lmax = 100, 230           # 200 ring pairs: ragged for every shape
    dev = torch.device("cuda", 0)
    o = Oracle(lmax, healpix_rings(nside))
    aE, aB = wl.random_alm(lmax, 5), wl.random_alm(lmax, 6)
    h1, h2 = wl.random_maps(o.rings.npix, 7)
    r1, r2 = o.synth(aE, aB)
    rE, rB = o.adjoint(h1, h2)
    p = Plan(nside, lmax, precision=prec, device=dev, tuned=False)
    tE, tB = torch.from_numpy(aE).to(dev), torch.from_numpy(aB).to(dev)
    th1, th2 = torch.from_numpy(h1).to(dev), torch.from_numpy(h2).to(dev)
    for v, r in SYN:
        print("synth variant", v, "rings", r, flush=True)
        p.set_tuning(v, r, 1, 4, 8)
        g1, g2 = p.synth2(tE, tB)
        assert rel(np.r_[g1.cpu().numpy(), g2.cpu().numpy()], np.r_[r1, r2]) < tol, (v, r)
    for r, w, c in ADJ:
        print("adjoint rings", r, "waves", w, "chunk", c, flush=True)
        p.set_tuning(1, 2, r, w, c)
        cE, cB = p.adjoint2(th1, th2)
        assert rel(np.stack([cE.cpu().numpy(), cB.cpu().numpy()]), np.stack([rE, rB])) < tol, (r, w)
    p.close()


BATCHED = [(sw, aw) for sw in (1, 2, 4, 8) for aw in (2, 4, 8)]


def test_all_batched_shapes_match_oracle():
    # every (synthesis waves, adjoint waves) shape of the batched matrix-core kernels, on a plan with
    # polar groups in the difference form and a padded second group of right-hand sides
    import torch
    from paper_2606_06175_amd import Plan
    nside, lmax, nrhs = 300, 600, 9   # 600 ring pairs: ten 64-pair groups, ragged for every shape
    dev = torch.device("cuda", 0)
    o = Oracle(lmax, healpix_rings(nside))
    A = np.stack([wl.random_alm(lmax, 90 + k) for k in range(nrhs)])
    B = np.stack([wl.random_alm(lmax, 110 + k) for k in range(nrhs)])
    g = np.random.default_rng(12)
    mask = (g.uniform(size=o.rings.npix) < 0.8).astype(np.uint8)
    ninvs = np.stack([g.uniform(5.0, 60.0, o.rings.npix) for _ in range(nrhs)])
    check = (0, 8)   # first and last right-hand side (the second group is padded)
    ref_s = {k: o.synth(A[k], B[k]) for k in check}
    ref_h = {k: o.apply_H(np.stack([A[k], B[k]]), o.weights(ninvs[k], mask), 0.02) for k in check}
    p = Plan(nside, lmax, nrhs=nrhs, precision="fp32", device=dev, tuned=False)
    tA, tB = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
    tn, tm = torch.from_numpy(ninvs).to(dev), torch.from_numpy(mask).to(dev)
    for sw, aw in BATCHED:
        print("batched synthesis waves", sw, "adjoint waves", aw, flush=True)
        p.set_tuning_batched(sw, aw)
        assert p.get_tuning_batched() == (sw, aw)
        g1, g2 = p.synth2(tA, tB)
        yE, yB = p.apply_H(tn, tm, tA, tB, 0.02)
        for k in check:
            r1, r2 = ref_s[k]
            assert rel(np.r_[g1[k].cpu().numpy(), g2[k].cpu().numpy()], np.r_[r1, r2]) < 1e-5, (sw, aw, k)
            assert rel(np.stack([yE[k].cpu().numpy(), yB[k].cpu().numpy()]), ref_h[k]) < 1e-5, (sw, aw, k)
    with pytest.raises(Exception):
        p.set_tuning_batched(3, 4)
    with pytest.raises(Exception):
        p.set_tuning_batched(4, 1)
    p.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_single_wave_shapes_uneven_split(prec, tol):
    # Single-wave adjoint workgroups spread a list of n groups as ceil(n / R) workgroups of R and
    # R - 1 groups.  At Nside 400 (800 ring pairs: 13 groups, the last of 32 pairs) the full list and
    # an 11-group list of groups weighted on their south rings only leave workgroups of both sizes for
    # every R from 2 to 8: the unweighted adjoint and the weighted apply against the oracle.
    import torch
    from paper_2606_06175_amd import Plan
    nside, lmax = 400, 128
    dev = torch.device("cuda", 0)
    rings = healpix_rings(nside)
    o = Oracle(lmax, rings)
    npairs = 2 * nside
    # weight on the south rings of pairs 74..799 and the north rings of pairs 770..799: groups 1..11
    # are weighted on one side, group 12 on both, group 0 on neither
    w_ring = np.zeros(rings.nrings, bool)
    for p in range(74, npairs):
        w_ring[rings.nrings - 1 - p] = True
    w_ring[770:npairs] = True
    cls = []
    for g in range(13):
        ps = range(64 * g, min(npairs, 64 * g + 64))
        n = any(w_ring[p] for p in ps)
        s = any(w_ring[rings.nrings - 1 - p] for p in ps if rings.nrings - 1 - p != p)
        cls.append("both" if n and s else "south" if s else "north" if n else "none")
    assert cls.count("south") == 11 and cls.count("both") == 1
    mask = np.zeros(o.rings.npix, np.uint8)
    for r in np.flatnonzero(w_ring):
        mask[rings.ofs[r]:rings.ofs[r] + rings.nphi[r]] = 1
    ninv = np.random.default_rng(21).uniform(5.0, 60.0, o.rings.npix)
    h1, h2 = wl.random_maps(o.rings.npix, 22)
    rE, rB = o.adjoint(h1, h2)
    x = np.stack([wl.random_alm(lmax, 23, lmin=0), wl.random_alm(lmax, 24, lmin=0)])
    ref = o.apply_H(x, o.weights(ninv, mask), 0.02)
    p = Plan(nside, lmax, precision=prec, device=dev, tuned=False)
    th1, th2 = torch.from_numpy(h1).to(dev), torch.from_numpy(h2).to(dev)
    tn, tm = torch.from_numpy(ninv).to(dev), torch.from_numpy(mask).to(dev)
    tx = [torch.from_numpy(a).to(dev) for a in x]
    for r, w, c in [s for s in ADJ if s[1] == 1]:
        print("single-wave adjoint rings", r, "chunk", c, flush=True)
        p.set_tuning(1, 2, r, 1, c)
        cE, cB = p.adjoint2(th1, th2)
        assert rel(np.stack([cE.cpu().numpy(), cB.cpu().numpy()]), np.stack([rE, rB])) < tol, (r, c)
        p.set_tuning(1, 2, 4, 1, 8)
        p.set_tuning_one_sided(1, 2, r, 1, c)
        yE, yB = p.apply_H(tn, tm, tx[0], tx[1], 0.02)
        assert rel(np.stack([yE.cpu().numpy(), yB.cpu().numpy()]), ref) < tol, (r, c)
        assert p.work_weighted()["adjoint_one"] > 0
    p.close()
