"""Stagnation stop of the PCG solves (opts.stall_iters): a solve stops with AKRA_STAGNATED at the first
iteration after which its relative residual has failed, stall_iters times in a row, to fall below the
smallest earlier value (the start counts as the first value).  The stop is checked against that rule
applied to the residual history the solve itself returns, on FP64 and mixed plans, the flat-sky
solver and a batched FP32 plan; with the test off (the default) the same solves converge as before.
Breakdown forced from the host (K_l = 0 and lambda = 0 make H = 0) in FP64, FP32 and batched plans.
Also the convergence test every k iterations (opts.check_every): the tested residuals equal those of
the solve testing every iteration, and the stop is the first tested iteration whose residual is
below the tolerance.

Inputs: the C1 workload (HEALPix Nside 32, lmax 64) with seeded random maps, and a 64 x 32 flat field
from the flat-field recipe."""
import numpy as np
import pytest

import akra_workloads as wl

pytestmark = pytest.mark.gpu


def expected_stop(hist, window, tol):
    """1-based iteration at which the rule stops, or None (converged first, or reached an iteration
    with no recorded residual: an FP32 plan's restart after a breakdown)."""
    best, since = 1.0, 0
    for i, r in enumerate(hist):
        if r < tol or r == 0.0:
            return None
        if r < best:
            best, since = r, 0
        else:
            since += 1
            if since >= window:
                return i + 1
    return None


def _c1():
    import torch
    cfg = wl.make_config("C1")
    m = cfg["mask"].astype(np.float64)
    g1, g2 = wl.random_maps(len(cfg["mask"]), 43)
    dev = torch.device("cuda", 0)
    return cfg, [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (m * g1, m * g2, cfg["ninv"][0],
                                                                             cfg["mask"])]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_stop_follows_the_rule(prec):
    from paper_2606_06175_amd import Plan, akra
    cfg, t = _c1()
    print("plan C1 %s" % prec, flush=True)
    p = Plan(cfg["nside"], cfg["lmax"], precision=prec, device="cuda:0")
    # the residual history of a run without the test
    _, _, ref = p.cg_solve(*t, tol=1e-13, maxiter=400, hist_len=400, raise_not_converged=False)
    hist = ref["hist"]
    stops = {w: expected_stop(hist, w, 1e-13) for w in (1, 2, 3, 5)}
    print("expected stops", stops, flush=True)
    assert stops[1] is not None  # the 2-norm residual of CG is not monotone
    for w, it in stops.items():
        xE, xB, info = p.cg_solve(*t, tol=1e-13, maxiter=400, hist_len=400, raise_not_converged=False, stall_iters=w)
        if it is None:
            assert info["status"] in (0, 5)
            continue
        assert info["status"] == akra.AKRA_STAGNATED and info["iters"] == it
        assert np.array_equal(info["hist"], hist[:it])
        assert info["rel_resid_true"] > 0 and bool(xE.isfinite().all())
    # raised by default
    w = min(k for k, v in stops.items() if v is not None)
    with pytest.raises(akra.AkraError, match="STAGNATED"):
        p.cg_solve(*t, tol=1e-13, maxiter=400, stall_iters=w)
    # off by default: a reachable tolerance converges as before
    _, _, info = p.cg_solve(*t, tol=1e-8, maxiter=2000)
    assert info["status"] == 0
    with pytest.raises(akra.AkraError, match="invalid solver options"):
        p.cg_solve(*t, tol=1e-8, stall_iters=-1)


def test_flat_stop_follows_the_rule():
    import torch
    from paper_2606_06175_amd import FlatPlan, akra
    nx, ny = 64, 32
    f = wl.make_flat(nx, ny, 7)
    g = np.random.default_rng(3)
    m = f["mask"].astype(np.float64)
    dev = torch.device("cuda", 0)
    t = [torch.from_numpy(np.ascontiguousarray(a)).to(dev)
         for a in (m * g.normal(size=(ny, nx)), m * g.normal(size=(ny, nx)), f["ninv"], f["mask"])]
    print("flat plan %d x %d" % (nx, ny), flush=True)
    p = FlatPlan(nx, ny, device="cuda:0")
    _, _, ref = p.cg_solve(*t, tol=1e-15, maxiter=300, hist_len=300, raise_not_converged=False)
    hist = ref["hist"]
    w = 1
    it = expected_stop(hist, w, 1e-15)
    print("expected stop", it, flush=True)
    assert it is not None
    _, _, info = p.cg_solve(*t, tol=1e-15, maxiter=300, hist_len=300, raise_not_converged=False, stall_iters=w)
    assert info["status"] == akra.AKRA_STAGNATED and info["iters"] == it
    assert np.array_equal(info["hist"], hist[:it])


def test_batched_plan_stops_each_rhs():
    import torch
    from paper_2606_06175_amd import Plan, akra
    cfg, t = _c1()
    n = 4
    print("batched FP32 plan C1 nrhs=%d" % n, flush=True)
    p = Plan(cfg["nside"], cfg["lmax"], nrhs=n, precision="fp32", device="cuda:0")
    g1 = torch.stack([t[0] * (1 + 0.1 * k) for k in range(n)])
    g2 = torch.stack([t[1] for k in range(n)])
    ninv = torch.stack([t[2] for k in range(n)])
    _, _, info = p.cg_solve(g1, g2, ninv, t[3], tol=1e-8, maxiter=2000)
    assert info["status"] == 0
    xE, xB, info = p.cg_solve(g1, g2, ninv, t[3], tol=1e-13, maxiter=2000, stall_iters=1, raise_not_converged=False)
    print("batched stagnation after %d lockstep iterations" % info["iters"], flush=True)
    assert info["status"] == akra.AKRA_STAGNATED and info["iters"] < 2000
    assert bool(xE.isfinite().all()) and bool(xB.isfinite().all())


def first_tested_below(hist, k, tol):
    """1-based first multiple of k whose residual in the history is below tol, or None."""
    for j in range(k, len(hist) + 1, k):
        if hist[j - 1] < tol:
            return j
    return None


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_check_every_runs_the_same_iterations(prec):
    # iterations between tests are the same kernels in the same order: the tested residuals equal
    # those of a run testing every iteration, bit for bit, and the stop is the first tested
    # iteration whose residual is below tol (the residual of CG is not monotone, so that can be
    # later than the first multiple of k after the first iteration below tol)
    from paper_2606_06175_amd import Plan
    cfg, t = _c1()
    print("plan C1 %s, check_every" % prec, flush=True)
    p = Plan(cfg["nside"], cfg["lmax"], precision=prec, device="cuda:0")
    # reference history, run past the tolerance used below
    x1, y1, ref = p.cg_solve(*t, tol=1e-10, maxiter=3000, hist_len=3000)
    hist = ref["hist"]
    for k in (2, 5, 8):
        xk, yk, ik = p.cg_solve(*t, tol=1e-8, maxiter=3000, hist_len=3000, check_every=k)
        print("check_every %d: %d iterations" % (k, ik["iters"]), flush=True)
        assert ik["status"] == 0 and ik["rel_resid_true"] <= 1e-8
        if prec == "fp64":
            assert ik["iters"] == first_tested_below(hist, k, 1e-8)
            tested = np.arange(k, ik["iters"] + 1, k) - 1
            assert np.array_equal(ik["hist"][tested], hist[tested])


def test_flat_check_every():
    import torch
    from paper_2606_06175_amd import FlatPlan
    nx, ny = 64, 32
    f = wl.make_flat(nx, ny, 7)
    g = np.random.default_rng(3)
    m = f["mask"].astype(np.float64)
    dev = torch.device("cuda", 0)
    t = [torch.from_numpy(np.ascontiguousarray(a)).to(dev)
         for a in (m * g.normal(size=(ny, nx)), m * g.normal(size=(ny, nx)), f["ninv"], f["mask"])]
    p = FlatPlan(nx, ny, device="cuda:0")
    # reference: a fixed 24 iterations (the residual settles at the rounding floor, far above 1e-300)
    _, _, ref = p.cg_solve(*t, tol=1e-300, maxiter=24, hist_len=24, raise_not_converged=False)
    _, _, i3 = p.cg_solve(*t, tol=1e-6, maxiter=500, hist_len=500, check_every=3)
    print("flat: reference %d iterations, check_every 3 stops after %d" % (ref["iters"], i3["iters"]), flush=True)
    assert i3["status"] == 0 and i3["iters"] == first_tested_below(ref["hist"], 3, 1e-6)
    tested = np.arange(3, i3["iters"] + 1, 3) - 1
    assert np.array_equal(i3["hist"][tested], ref["hist"][tested])
    assert i3["rel_resid_true"] <= 1e-6


@pytest.mark.parametrize("prec,nrhs", [("fp64", 1), ("fp32", 1), ("fp32", 2)])
def test_forced_breakdown(prec, nrhs):
    # p^T H p = 0 forced from the host: a given right-hand side b != 0 with the harmonic kernel K_l = 0
    # and lambda = 0 makes H = 0.  FP64 plans report AKRA_ERR_NUMERIC; FP32 plans restart with the
    # FP64 operator, break down again and stop with AKRA_NOT_CONVERGED and a finite last iterate
    # (x = 0: alpha is held at zero once the flag is up).  The same with convergence tested every 4
    # iterations, where the sticky flag keeps x from moving between tests.
    import torch
    from paper_2606_06175_amd import Plan, akra
    cfg, t = _c1()
    lmax = cfg["lmax"]
    print("plan C1 %s nrhs=%d, zero kernel" % (prec, nrhs), flush=True)
    p = Plan(cfg["nside"], lmax, nrhs=nrhs, precision=prec, device="cuda:0")
    bE = torch.stack([torch.from_numpy(wl.random_alm(lmax, 31 + k)).to(t[0].device) for k in range(nrhs)])
    bB = torch.stack([torch.from_numpy(wl.random_alm(lmax, 41 + k)).to(t[0].device) for k in range(nrhs)])
    ninv = torch.stack([t[2]] * nrhs) if nrhs > 1 else t[2]
    if nrhs == 1:
        bE, bB = bE[0], bB[0]
    zero = np.zeros(lmax + 1)
    for every in (1, 4):
        if prec == "fp64":
            with pytest.raises(akra.AkraError, match="NUMERIC"):
                p.cg_solve_b(bE, bB, ninv, t[3], tol=1e-8, maxiter=50, lam=0.0, kernel=zero, check_every=every)
            continue
        xE, xB, info = p.cg_solve_b(bE, bB, ninv, t[3], tol=1e-8, maxiter=50, lam=0.0, kernel=zero,
                                    raise_not_converged=False, check_every=every)
        assert info["status"] == akra.AKRA_NOT_CONVERGED
        assert float(xE.abs().max()) == 0.0 and float(xB.abs().max()) == 0.0
    # the plan is usable afterwards: a regular solve converges
    if nrhs == 1:
        _, _, info = p.cg_solve(*t, tol=1e-8, maxiter=3000)
        assert info["status"] == 0
