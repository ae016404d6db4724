"""GPU block solves of App. A against the oracle: the E-mode solve (kappa_B held at zero) and the
conditional B-mode solve (b~_B = b_B - H_BE kappa_E, then the B block system), their PCG iterates,
FP64 true residuals, the block-elimination identity, step-wise and batched forms.

Inputs are the C1 workload (HEALPix Nside 32, lmax 64, one cap with f_sky 0.1, Poisson mean 5)."""
import ctypes

import numpy as np
import pytest

import akra_workloads as wl
from oracle.core import Oracle
from oracle.geometry import healpix_rings

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.ravel(a)
    b = np.ravel(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def c1():
    import torch
    cfg = wl.make_config("C1")
    lmax, nside = cfg["lmax"], cfg["nside"]
    o = Oracle(lmax, healpix_rings(nside))
    K = o.kernel()[o.l_of]
    g1, g2 = o.synth(K * cfg["kappa"][0], np.zeros(o.nalm, np.complex128))
    m = cfg["mask"].astype(np.float64)
    g1 = m * (g1 + cfg["eps1"][0])
    g2 = m * (g2 + cfg["eps2"][0])
    ninv, mask = cfg["ninv"][0], cfg["mask"]
    W = o.weights(ninv, mask)
    lam = o.lambda_eff(ninv, mask)
    P = o.precond(ninv, mask, lam)
    b = o.rhs(g1, g2, W)
    kE_ref, _ = o.cg(b[0], W, lam, P, tol=1e-13, maxiter=4000, block=0)
    dev = torch.device("cuda", 0)
    t = dict(g1=torch.from_numpy(g1).to(dev), g2=torch.from_numpy(g2).to(dev),
             ninv=torch.from_numpy(ninv).to(dev), mask=torch.from_numpy(mask).to(dev))
    return dict(cfg=cfg, o=o, g1=g1, g2=g2, W=W, lam=lam, P=P, b=b, kE_ref=kE_ref, t=t, torch=torch, dev=dev)


def _plan(c, prec, nrhs=1):
    from paper_2606_06175_amd import Plan
    print("plan nside=%d lmax=%d %s nrhs=%d" % (c["cfg"]["nside"], c["cfg"]["lmax"], prec, nrhs), flush=True)
    return Plan(c["cfg"]["nside"], c["cfg"]["lmax"], nrhs=nrhs, precision=prec, device="cuda:0")


def _block_resid(c, x, bk, block):
    o = c["o"]
    r = bk - o.apply_block(x, c["W"], c["lam"], block, block)
    return float(np.sqrt(o.dot(r, r) / o.dot(bk, bk)))


def test_e_only_iterates_match_oracle(c1):
    t, o = c1["t"], c1["o"]
    p = _plan(c1, "fp64")
    xE, xB, info = p.cg_solve(t["g1"], t["g2"], t["ninv"], t["mask"], tol=1e-14, maxiter=12,
                              raise_not_converged=False, mode="E")
    assert info["status"] == 5 and info["iters"] == 12
    assert float(xB.abs().max()) == 0.0
    xr, ir = o.cg(c1["b"][0], c1["W"], c1["lam"], P=c1["P"], tol=1e-14, maxiter=12, block=0)
    assert ir["iters"] == 12
    assert rel(xE.cpu().numpy(), xr) < 1e-9


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-8)])
def test_e_only_solve_true_residual(c1, prec, tol):
    t = c1["t"]
    p = _plan(c1, prec)
    xE, xB, info = p.cg_solve(t["g1"], t["g2"], t["ninv"], t["mask"], tol=tol, maxiter=4000, mode="E")
    assert info["status"] == 0
    assert float(xB.abs().max()) == 0.0
    rt = _block_resid(c1, xE.cpu().numpy(), c1["b"][0], 0)
    print(prec, "iters", info["iters"], "true residual", rt, info["rel_resid_true"], flush=True)
    assert rt <= 1.05 * tol
    assert abs(rt - info["rel_resid_true"]) <= 1e-3 * tol + 1e-12
    assert rel(xE.cpu().numpy(), c1["kE_ref"]) < 1e4 * tol


def test_conditional_b_iterates_and_residual_match_oracle(c1):
    torch, dev, o, t = c1["torch"], c1["dev"], c1["o"], c1["t"]
    kE = c1["kE_ref"]
    bt = o.cond_b_rhs(c1["g1"], c1["g2"], c1["W"], c1["lam"], kE)
    p = _plan(c1, "fp64")
    tkE = torch.from_numpy(kE).to(dev)
    kB, info = p.cg_solve_cond_b(t["g1"], t["g2"], t["ninv"], t["mask"], tkE, tol=1e-14, maxiter=12,
                                 raise_not_converged=False)
    assert info["status"] == 5 and info["iters"] == 12
    xr, _ = o.cg(bt, c1["W"], c1["lam"], P=c1["P"], tol=1e-14, maxiter=12, block=1)
    assert rel(kB.cpu().numpy(), xr) < 1e-9
    kB, info = p.cg_solve_cond_b(t["g1"], t["g2"], t["ninv"], t["mask"], tkE, tol=1e-10, maxiter=4000)
    assert info["status"] == 0
    rt = _block_resid(c1, kB.cpu().numpy(), bt, 1)
    print("iters", info["iters"], "true residual", rt, info["rel_resid_true"], flush=True)
    assert rt <= 1.05e-10
    assert abs(rt - info["rel_resid_true"]) <= 1e-13


def test_conditional_b_given_joint_e_returns_joint_b(c1):
    # block elimination (eq. lower_block): the joint kappa_E in, the joint kappa_B out
    t = c1["t"]
    p = _plan(c1, "fp64")
    xE, xB, _ = p.cg_solve(t["g1"], t["g2"], t["ninv"], t["mask"], tol=1e-12, maxiter=4000)
    kB, info = p.cg_solve_cond_b(t["g1"], t["g2"], t["ninv"], t["mask"], xE, tol=1e-12, maxiter=4000)
    assert info["status"] == 0
    assert rel(kB.cpu().numpy(), xB.cpu().numpy()) < 1e-8


def test_step_wise_e_only_matches_oracle(c1):
    t, o = c1["t"], c1["o"]
    p = _plan(c1, "fp64")
    p.cg_start(t["g1"], t["g2"], t["ninv"], t["mask"], mode="E")
    p.cg_step(10)
    rr, it, xE, xB = p.cg_state(copy_x=True)
    assert it == 10 and float(xB.abs().max()) == 0.0
    xr, ir = o.cg(c1["b"][0], c1["W"], c1["lam"], P=c1["P"], tol=1e-14, maxiter=10, block=0)
    assert rel(xE.cpu().numpy(), xr) < 1e-9
    assert abs(rr - ir["hist"][-1]) < 1e-9 * ir["hist"][-1]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_block_solves(c1, prec):
    # three right-hand sides with their own weights: E-only, then the conditional B solve on the
    # E results; every right-hand side meets the tolerance in the oracle's FP64 residual
    torch, dev, o = c1["torch"], c1["dev"], c1["o"]
    nr = 3
    mask = c1["cfg"]["mask"]
    ninvs = np.stack([c1["cfg"]["ninv"][0] * (1.0 + 0.1 * k) for k in range(nr)])
    g1s = np.stack([c1["g1"] * (1.0 + 0.2 * k) for k in range(nr)])
    g2s = np.stack([c1["g2"] * (1.0 - 0.1 * k) + 0.01 * k * c1["g1"] for k in range(nr)])
    tol = 1e-9 if prec == "fp64" else 1e-8
    p = _plan(c1, prec, nrhs=nr)
    tg1, tg2, tn = (torch.from_numpy(a).to(dev) for a in (g1s, g2s, ninvs))
    xE, xB, info = p.cg_solve(tg1, tg2, tn, c1["t"]["mask"], tol=tol, maxiter=4000, mode="E")
    assert info["status"] == 0 and float(xB.abs().max()) == 0.0
    kB, info_b = p.cg_solve_cond_b(tg1, tg2, tn, c1["t"]["mask"], xE, tol=tol, maxiter=4000)
    assert info_b["status"] == 0
    for k in range(nr):
        W = o.weights(ninvs[k], mask)
        lam = o.lambda_eff(ninvs[k], mask)
        c = dict(o=o, W=W, lam=lam)
        b = o.rhs(g1s[k], g2s[k], W)
        assert _block_resid(c, xE[k].cpu().numpy(), b[0], 0) <= 1.05 * tol
        bt = o.cond_b_rhs(g1s[k], g2s[k], W, lam, xE[k].cpu().numpy())
        assert _block_resid(c, kB[k].cpu().numpy(), bt, 1) <= 1.05 * tol


def test_invalid_mode_is_an_argument_error(c1):
    from paper_2606_06175_amd import akra
    t = c1["t"]
    p = _plan(c1, "fp64")
    o, keep = p._opts(1e-6, 10, 1e-3, None, None, 0.1, 0)
    o.mode = 7
    xE, xB = p._alm_out(), p._alm_out()
    inf = akra.CgInfo()
    st = akra.lib().akra_cg_solve(p._h, t["g1"].data_ptr(), t["g2"].data_ptr(), t["ninv"].data_ptr(),
                                  t["mask"].data_ptr(), ctypes.byref(o), xE.data_ptr(), xB.data_ptr(),
                                  ctypes.byref(inf))
    assert st == akra.AKRA_ERR_ARG
    with pytest.raises(ValueError):
        p.cg_solve(t["g1"], t["g2"], t["ninv"], t["mask"], mode="EB")
    # the conditional B solve rejects kB aliasing kE
    st = akra.lib().akra_cg_solve_cond_b(p._h, t["g1"].data_ptr(), t["g2"].data_ptr(), t["ninv"].data_ptr(),
                                         t["mask"].data_ptr(), None, xE.data_ptr(), xE.data_ptr(), None)
    assert st == akra.AKRA_ERR_ARG and "alias" in akra.lib().akra_last_error().decode()
