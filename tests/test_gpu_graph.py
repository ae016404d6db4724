"""Graph replay of the PCG iteration (Sec. II.B inversion problem) against direct kernel launches,
through the C ABI: the iterates, residuals and iteration counts of a plan that replays its recorded
iteration equal, bit for bit, those of a plan that launches the same kernels directly.  Every replay
is checked on its own, with unrelated torch work and host synchronisations between replays; the
recording is renewed when the launch shapes, lambda_eff or the unknowns change; the lockstep iteration
of a batched FP32 plan likewise, renewed whenever its set of active right-hand sides changes.

Inputs: the C1 workload (HEALPix Nside 32, lmax 64, one cap with f_sky 0.1, Poisson mean 5) and its
seeded random maps; the C5 workload (Nside 256, lmax 512) for one FP32 check."""
import numpy as np
import pytest

import akra_workloads as wl

pytestmark = pytest.mark.gpu


def _inputs(name):
    import torch
    cfg = wl.make_config(name)
    dev = torch.device("cuda", 0)
    m = cfg["mask"].astype(np.float64)
    g1, g2 = wl.random_maps(len(cfg["mask"]), 41)
    t = [torch.from_numpy(np.ascontiguousarray(a)).to(dev)
         for a in (m * g1, m * g2, cfg["ninv"][0], cfg["mask"])]
    return cfg, t


def _pair(cfg, prec):
    from paper_2606_06175_amd import Plan
    print("plans nside=%d lmax=%d %s" % (cfg["nside"], cfg["lmax"], prec), flush=True)
    a = Plan(cfg["nside"], cfg["lmax"], precision=prec, device="cuda:0")
    b = Plan(cfg["nside"], cfg["lmax"], precision=prec, device="cuda:0")
    b.set_graph(False)
    return a, b


def _other_work():
    # unrelated torch kernels on the same device between replays
    import torch
    x = torch.randn(512, 512, device="cuda:0")
    y = (x @ x.T).sum()
    torch.cuda.synchronize()
    return float(y)


def _same_state(a, b):
    ra, ia, xa, ya = a.cg_state(copy_x=True)
    rb, ib, xb, yb = b.cg_state(copy_x=True)
    assert ia == ib
    assert ra == rb
    assert bool((xa == xb).all()) and bool((ya == yb).all())
    return ra


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_step_replays_equal_direct_launches(prec):
    cfg, t = _inputs("C1")
    a, b = _pair(cfg, prec)
    for p in (a, b):
        p.cg_start(*t, lam=1e-3)
    prev = None
    for i in range(6):
        a.cg_step(1)
        b.cg_step(1)
        _other_work()
        r = _same_state(a, b)
        assert prev is None or r != prev  # each replay did an iteration
        prev = r
    # several replays queued back to back
    a.cg_step(7)
    b.cg_step(7)
    _same_state(a, b)
    # a new start with another lambda renews the recording
    for p in (a, b):
        p.cg_start(*t, lam=3e-2)
    for i in range(3):
        a.cg_step(2)
        b.cg_step(2)
        _same_state(a, b)
    # E-only unknowns
    for p in (a, b):
        p.cg_start(*t, lam=1e-3, mode="E")
    a.cg_step(5)
    b.cg_step(5)
    _same_state(a, b)


def test_new_launch_shape_renews_the_recording():
    cfg, t = _inputs("C1")
    a, b = _pair(cfg, "fp64")
    for p in (a, b):
        p.cg_start(*t, lam=1e-3)
    a.cg_step(3)
    b.cg_step(3)
    _same_state(a, b)
    shape = a.get_tuning()
    alt = (1, 2, 2, 2, 8) if tuple(shape) != (1, 2, 2, 2, 8) else (0, 1, 1, 2, 8)
    for p in (a, b):
        p.set_tuning(*alt)
    for i in range(3):
        a.cg_step(1)
        b.cg_step(1)
        _other_work()
        _same_state(a, b)
    # the plan launching directly after switching graphs off, and back on
    a.set_graph(False)
    a.cg_step(2)
    b.cg_step(2)
    _same_state(a, b)
    a.set_graph(True)
    a.cg_step(2)
    b.cg_step(2)
    _same_state(a, b)


@pytest.mark.parametrize("prec,mode", [("fp64", "joint"), ("fp32", "joint"), ("fp64", "B")])
def test_solve_equals_direct_launches(prec, mode):
    cfg, t = _inputs("C1")
    a, b = _pair(cfg, prec)
    for rep in range(2):
        xa, ya, ia = a.cg_solve(*t, tol=1e-8, maxiter=3000, mode=mode)
        xb, yb, ib = b.cg_solve(*t, tol=1e-8, maxiter=3000, mode=mode)
        _other_work()
        assert ia["iters"] == ib["iters"] and ia["status"] == ib["status"] == 0
        assert ia["rel_resid_true"] == ib["rel_resid_true"]
        assert bool((xa == xb).all()) and bool((ya == yb).all())
        print("solve %s %s: %d iterations, true residual %.3e" % (prec, mode, ia["iters"], ia["rel_resid_true"]),
              flush=True)


def test_stage_timing_launches_directly():
    cfg, t = _inputs("C1")
    a, b = _pair(cfg, "fp64")
    for p in (a, b):
        p.cg_start(*t, lam=1e-3)
    a.set_timing(True)
    a.cg_step(4)
    st = a.stage_times()
    assert st["cg_vec"][1] == 4  # one timed CG-update span per iteration
    a.set_timing(False)
    b.cg_step(4)
    _same_state(a, b)


def test_fp32_replays_at_nside_256():
    cfg, t = _inputs("C5")
    a, b = _pair(cfg, "fp32")
    for p in (a, b):
        p.cg_start(*t, lam=1e-3)
    for i in range(3):
        a.cg_step(2)
        b.cg_step(2)
        _other_work()
        _same_state(a, b)


@pytest.mark.parametrize("nrhs", [4, 9, 16])
def test_batched_solve_replays_equal_direct_launches(nrhs):
    # the lockstep iteration of an FP32 batch replayed from its recording; the right-hand sides have
    # their own noise patterns (a uniform rescaling of N^-1 would leave the relative system
    # unchanged), converge at different iterations, and every change of the active set renews the
    # recording
    import torch
    from paper_2606_06175_amd import Plan
    cfg, t = _inputs("C1")
    print("batched plans C1 nrhs=%d" % nrhs, flush=True)
    a = Plan(cfg["nside"], cfg["lmax"], nrhs=nrhs, precision="fp32", device="cuda:0")
    b = Plan(cfg["nside"], cfg["lmax"], nrhs=nrhs, precision="fp32", device="cuda:0")
    b.set_graph(False)
    gen = np.random.default_rng(5)
    npix = t[0].numel()
    mod = [torch.from_numpy(gen.uniform(0.05, 1.0, npix) ** (2 * k)).to(t[2].device) for k in range(nrhs)]
    g1 = torch.stack([t[0] * (1 + 0.3 * k) for k in range(nrhs)])
    g2 = torch.stack([t[1] * (1 - 0.02 * k) for k in range(nrhs)])
    ninv = torch.stack([t[2] * mod[k] for k in range(nrhs)])
    for rep in range(2):
        xa, ya, ia = a.cg_solve(g1, g2, ninv, t[3], tol=1e-8, maxiter=3000)
        xb, yb, ib = b.cg_solve(g1, g2, ninv, t[3], tol=1e-8, maxiter=3000)
        _other_work()
        print("batched nrhs=%d: %d lockstep iterations" % (nrhs, ia["iters"]), flush=True)
        assert ia["status"] == ib["status"] == 0 and ia["iters"] == ib["iters"]
        assert ia["rel_resid_true"] == ib["rel_resid_true"]
        assert bool((xa == xb).all()) and bool((ya == yb).all())
    # the right-hand sides converge at different iterations (the active set changes mid-solve)
    its = []
    for k in (0, nrhs - 1):
        s1 = Plan(cfg["nside"], cfg["lmax"], precision="fp64", device="cuda:0")
        _, _, inf = s1.cg_solve(g1[k], g2[k], ninv[k], t[3], tol=1e-8, maxiter=3000)
        its.append(inf["iters"])
    print("single-RHS iterations of the first and last right-hand side: %s" % its, flush=True)
    assert its[0] != its[1]
