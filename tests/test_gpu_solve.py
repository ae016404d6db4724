"""GPU solver against the oracle: PCG iterates, the FP64 true residual of converged solves (plain,
mixed precision, batched), and the error paths of the solve.

Inputs are the C1 workload (HEALPix Nside 32, lmax 64, one cap with f_sky 0.1, Poisson mean 5)
with gamma_obs = M (Y(K kappa) + eps) built by the oracle."""
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
    b = o.rhs(g1, g2, W)
    dev = torch.device("cuda", 0)
    t = dict(g1=torch.from_numpy(g1).to(dev), g2=torch.from_numpy(g2).to(dev),
             ninv=torch.from_numpy(ninv).to(dev), mask=torch.from_numpy(mask).to(dev))
    return dict(cfg=cfg, o=o, g1=g1, g2=g2, W=W, lam=lam, b=b, t=t, torch=torch, dev=dev)


def _plan(nside, lmax, prec, nrhs=1):
    from paper_2606_06175_amd import Plan
    print("plan nside=%d lmax=%d %s nrhs=%d" % (nside, lmax, prec, nrhs), flush=True)
    return Plan(nside, lmax, nrhs=nrhs, precision=prec, device="cuda:0")


def _true_resid(c, x):
    """||b - H x|| / ||b|| evaluated by the oracle."""
    o = c["o"]
    r = c["b"] - o.apply_H(x, c["W"], c["lam"])
    return float(np.sqrt(o.dot(r, r) / o.dot(c["b"], c["b"])))


def test_cg_iterates_match_oracle(c1):
    # same algorithm (PCG with scalar P, x0 = 0): after 15 iterations the iterates agree to rounding
    o, t = c1["o"], c1["t"]
    p = _plan(c1["cfg"]["nside"], c1["cfg"]["lmax"], "fp64")
    xE, xB, info = p.cg_solve(t["g1"], t["g2"], t["ninv"], t["mask"], tol=1e-14, maxiter=15,
                              raise_not_converged=False)
    assert info["status"] == 5 and info["iters"] == 15
    P = o.precond(c1["cfg"]["ninv"][0], c1["cfg"]["mask"], c1["lam"])
    xr, ir = o.cg(c1["b"], c1["W"], c1["lam"], P=P, tol=1e-14, maxiter=15)
    assert ir["iters"] == 15
    assert rel(np.stack([xE.cpu().numpy(), xB.cpu().numpy()]), xr) < 1e-9
    assert abs(info["lambda_eff"] - c1["lam"]) < 1e-14 * c1["lam"]
    assert abs(info["precond"] - P) < 1e-12 * P


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-8)])
def test_converged_solve_true_residual(c1, prec, tol):
    # the returned solution meets tol in the oracle's own FP64 residual
    t = c1["t"]
    p = _plan(c1["cfg"]["nside"], c1["cfg"]["lmax"], prec)
    xE, xB, info = p.cg_solve(t["g1"], t["g2"], t["ninv"], t["mask"], tol=tol, maxiter=3000)
    assert info["status"] == 0
    x = np.stack([xE.cpu().numpy(), xB.cpu().numpy()])
    rt = _true_resid(c1, x)
    assert rt <= 1.05 * tol, rt
    assert abs(rt - info["rel_resid_true"]) <= 1e-3 * tol + 1e-12
    if prec == "fp32":
        assert info["fp64_applies"] >= 1


def test_mixed_solution_matches_fp64(c1):
    t = c1["t"]
    nside, lmax = c1["cfg"]["nside"], c1["cfg"]["lmax"]
    sol = {}
    for prec in ("fp64", "fp32"):
        p = _plan(nside, lmax, prec)
        xE, xB, info = p.cg_solve(t["g1"], t["g2"], t["ninv"], t["mask"], tol=1e-10, maxiter=3000)
        sol[prec] = np.stack([xE.cpu().numpy(), xB.cpu().numpy()])
    assert rel(sol["fp32"], sol["fp64"]) < 1e-7


def test_batched_solve_matches_single(c1):
    # two right-hand sides with their own weights, solved in one plan, equal their single solves
    torch, dev = c1["torch"], c1["dev"]
    t = c1["t"]
    nside, lmax = c1["cfg"]["nside"], c1["cfg"]["lmax"]
    ninv2 = torch.stack([t["ninv"], 0.5 * t["ninv"] + 3.0])
    g1 = torch.stack([t["g1"], -t["g2"]])
    g2 = torch.stack([t["g2"], t["g1"]])
    pb = _plan(nside, lmax, "fp64", nrhs=2)
    xE, xB, info = pb.cg_solve(g1, g2, ninv2, t["mask"], tol=1e-10, maxiter=3000)
    ps = _plan(nside, lmax, "fp64")
    for k in range(2):
        yE, yB, _ = ps.cg_solve(g1[k].contiguous(), g2[k].contiguous(), ninv2[k].contiguous(), t["mask"],
                                tol=1e-10, maxiter=3000)
        a = np.stack([xE[k].cpu().numpy(), xB[k].cpu().numpy()])
        b = np.stack([yE.cpu().numpy(), yB.cpu().numpy()])
        assert rel(a, b) < 1e-12


def test_zero_data_gives_zero_in_zero_iterations(c1):
    torch = c1["torch"]
    t = c1["t"]
    p = _plan(c1["cfg"]["nside"], c1["cfg"]["lmax"], "fp64")
    z = torch.zeros_like(t["g1"])
    xE, xB, info = p.cg_solve(z, z, t["ninv"], t["mask"], tol=1e-8)
    assert info["iters"] == 0 and info["status"] == 0
    assert float(xE.abs().max()) == 0.0 and float(xB.abs().max()) == 0.0


def test_not_converged_returns_last_iterate(c1):
    t = c1["t"]
    p = _plan(c1["cfg"]["nside"], c1["cfg"]["lmax"], "fp64")
    xE, xB, info = p.cg_solve(t["g1"], t["g2"], t["ninv"], t["mask"], tol=1e-14, maxiter=3,
                              raise_not_converged=False)
    assert info["status"] == 5 and info["iters"] == 3
    assert bool(torch_isfinite(xE)) and bool(torch_isfinite(xB))
    from paper_2606_06175_amd import AkraError
    with pytest.raises(AkraError) as e:
        p.cg_solve(t["g1"], t["g2"], t["ninv"], t["mask"], tol=1e-14, maxiter=3)
    assert e.value.status == 5


def torch_isfinite(x):
    import torch
    return torch.isfinite(torch.view_as_real(x)).all()


@pytest.mark.parametrize("bad,status", [("nan", 4), ("inf", 4), ("neg", 1)])
def test_invalid_weights_are_reported(c1, bad, status):
    import math
    from paper_2606_06175_amd import AkraError
    t = c1["t"]
    ninv = t["ninv"].clone()
    ninv[17] = {"nan": math.nan, "inf": math.inf, "neg": -1.0}[bad]
    p = _plan(c1["cfg"]["nside"], c1["cfg"]["lmax"], "fp64")
    with pytest.raises(AkraError) as e:
        p.cg_solve(t["g1"], t["g2"], ninv, t["mask"], tol=1e-6)
    assert e.value.status == status
    z = c1["torch"].zeros(p.nalm, dtype=c1["torch"].complex128, device=c1["dev"])
    with pytest.raises(AkraError) as e:
        p.apply_H(ninv, t["mask"], z, z, 1.0)
    assert e.value.status == status


@pytest.mark.parametrize("shape", [(1, 1, 8), (2, 4, 4)])
def test_mixed_solve_with_polar_blocks(shape):
    # FP32 plan whose near-polar ring groups form their own adjoint blocks; the FP64 applies of the
    # refinement must use the same block layout.  The true residual is the oracle's.
    import torch
    nside, lmax = 256, 512
    dev = torch.device("cuda", 0)
    mask = wl.cap_mask(nside, 0.9, 0.7, 0.15).astype(np.uint8)
    ninv = np.random.default_rng(31).uniform(10.0, 60.0, 12 * nside * nside)
    g1, g2 = [m * mask for m in wl.random_maps(12 * nside * nside, 32)]
    p = _plan(nside, lmax, "fp32")
    p.set_tuning(1, 1, *shape)
    assert p.work()["adjoint"] > 0
    t = [torch.from_numpy(a).to(dev) for a in (g1, g2, ninv, mask)]
    xE, xB, info = p.cg_solve(*t, tol=1e-8, maxiter=3000)
    o = Oracle(lmax, healpix_rings(nside))
    W = o.weights(ninv, mask)
    lam = o.lambda_eff(ninv, mask)
    b = o.rhs(g1, g2, W)
    x = np.stack([xE.cpu().numpy(), xB.cpu().numpy()])
    r = b - o.apply_H(x, W, lam)
    rt = float(np.sqrt(o.dot(r, r) / o.dot(b, b)))
    print("shape", shape, "iters", info["iters"], "true residual", rt, info["rel_resid_true"], flush=True)
    assert rt <= 1.05e-8
    assert abs(rt - info["rel_resid_true"]) <= 1e-11


@pytest.mark.parametrize("nr", [3, 10])
def test_batched_fp32_solve(c1, nr):
    # lockstep PCG of several right-hand sides (own weights each) on the matrix-core synthesis; every
    # right-hand side meets the tolerance in the oracle's FP64 residual
    torch, dev = c1["torch"], c1["dev"]
    o = c1["o"]
    mask = c1["cfg"]["mask"]
    ninvs = np.stack([c1["cfg"]["ninv"][0] * (1.0 + 0.07 * k) for k in range(nr)])
    g1s = np.stack([c1["g1"] * (1.0 + 0.1 * k) for k in range(nr)])
    g2s = np.stack([c1["g2"] * (1.0 - 0.05 * k) for k in range(nr)])
    p = _plan(c1["cfg"]["nside"], c1["cfg"]["lmax"], "fp32", nrhs=nr)
    xE, xB, info = p.cg_solve(torch.from_numpy(g1s).to(dev), torch.from_numpy(g2s).to(dev),
                              torch.from_numpy(ninvs).to(dev), c1["t"]["mask"], tol=1e-8, maxiter=3000)
    assert info["status"] == 0
    worst = 0.0
    for k in range(nr):
        W = o.weights(ninvs[k], mask)
        lam = o.lambda_eff(ninvs[k], mask)
        b = o.rhs(g1s[k], g2s[k], W)
        x = np.stack([xE[k].cpu().numpy(), xB[k].cpu().numpy()])
        r = b - o.apply_H(x, W, lam)
        rt = float(np.sqrt(o.dot(r, r) / o.dot(b, b)))
        worst = max(worst, rt)
        assert rt <= 1.05e-8, (k, rt)
    assert abs(worst - info["rel_resid_true"]) <= 1e-11


def test_lambda_eff_and_precond_hand_worked():
    # the solver's lambda_eff and P against the hand-worked values of tests/golden/regulariser.json
    # (Sec. II.B, eq. ML_estimator_reg and eq. precond): HEALPix Nside 1 and a 4 x 4 flat field
    import json
    import os
    import torch
    from paper_2606_06175_amd import FlatPlan
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "regulariser.json")))
    dev = torch.device("cuda", 0)
    g = gold["sphere_nside1"]
    ninv = torch.tensor(g["ninv"], dtype=torch.float64, device=dev)
    mask = torch.tensor(g["mask"], dtype=torch.uint8, device=dev)
    g1, g2 = (torch.from_numpy(a).to(dev) for a in wl.random_maps(12, 5))
    p = _plan(1, 2, "fp64")
    for c in g["cases"]:
        _, _, info = p.cg_solve(g1, g2, ninv, mask, tol=1e-12, maxiter=200, lam=c["lambda"],
                                raise_not_converged=False)
        lam, P = c["lambda_eff"][0] / c["lambda_eff"][1], c["P"][0] / c["P"][1]
        print("sphere lambda %g: lambda_eff %.17g (%.17g) P %.17g (%.17g)"
              % (c["lambda"], info["lambda_eff"], lam, info["precond"], P), flush=True)
        assert abs(info["lambda_eff"] - lam) <= 1e-15 * lam
        assert abs(info["precond"] - P) <= 1e-15 * P
    p.close()
    g = gold["flat_4x4"]
    ninv = torch.tensor(g["ninv"], dtype=torch.float64, device=dev)
    mask = torch.tensor(g["mask"], dtype=torch.uint8, device=dev)
    rng = np.random.default_rng(6)
    g1, g2 = (torch.from_numpy(rng.normal(size=(4, 4))).to(dev) for _ in range(2))
    fp = FlatPlan(4, 4, device=dev)
    for c in g["cases"]:
        _, _, info = fp.cg_solve(g1, g2, ninv, mask, tol=1e-12, maxiter=200, lam=c["lambda"],
                                 raise_not_converged=False)
        lam, P = c["lambda_eff"][0] / c["lambda_eff"][1], c["P"][0] / c["P"][1]
        print("flat lambda %g: lambda_eff %.17g (%.17g) P %.17g (%.17g)"
              % (c["lambda"], info["lambda_eff"], lam, info["precond"], P), flush=True)
        assert abs(info["lambda_eff"] - lam) <= 1e-15 * lam
        assert abs(info["precond"] - P) <= 1e-15 * P
    fp.close()
