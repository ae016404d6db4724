"""Every Legendre launch shape the autotuner may pick gives the oracle's result (GPU)."""
import numpy as np
import pytest

import akra_workloads as wl
from oracle.core import Oracle
from oracle.geometry import healpix_rings

pytestmark = pytest.mark.gpu

SYN = [(v, r) for v in (0, 1) for r in (1, 2, 4)]
ADJ = [(1, 1, 8), (1, 2, 8), (1, 4, 8), (2, 2, 8), (2, 4, 8), (4, 2, 8), (4, 4, 8), (8, 1, 8), (8, 2, 8),
       (2, 4, 4), (4, 2, 4), (4, 4, 4), (8, 1, 4), (2, 1, 8), (4, 1, 4), (4, 1, 8)]


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
