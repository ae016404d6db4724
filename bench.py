#!/usr/bin/env python3
"""Benchmark of the matrix-free AKRA 3.0 operator on one MI355X.

Workload (default): HEALPix Nside 2048, lmax 4096, a 3-cap footprint with f_sky ~ 0.1 minus 2000
holes, Poisson counts of mean 2 modulated by a smooth x U[0.5, 1.5] depth, sigma_e = 0.26, kappa
from C_l = 1e-7 (l+10)^-1.2 -- synthetic stand-ins for the DES Y3 shapes.

One step = one preconditioned CG iteration (H v = K Y^H W Y K v + lambda_eff v and the vector
updates) on device-resident data.  value = steps per second = H v applies/s.  Also reported:
stage times from HIP events on the plan stream, the Legendre-stage roofline, time to a true
FP64 relative residual of 1e-8 for the FP64 solve and for the FP32 operator with FP64 reliable
updates, and the CPU oracle timed on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-solve] [--no-cpu-baseline]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H·v applies/s + CG time-to-1e-8 at Nside 2048 ℓmax 4096, mixed/batched vs FP64"
PEAK_FP64 = 78.6e12      # MI355X FP64 vector FMA, FLOP/s
PEAK_FP32 = 157.3e12     # MI355X FP32 vector (packed) FMA, FLOP/s
FLOP_PER_TRIPLE = 26     # per (l, m, ring pair) and direction: 2 recurrences (10) + 8 contraction FMAs (16)
FLOP_PER_TRIPLE_ONE = 18  # the same with one ring of the pair weighted: 2 recurrences + 4 contraction FMAs


def weighted_flops(ww):
    """Algorithmic flop of the weighted synthesis and adjoint launches (akra_plan_work_weighted)."""
    return {"leg_synth": FLOP_PER_TRIPLE * ww["synth_two"] + FLOP_PER_TRIPLE_ONE * ww["synth_one"],
            "leg_adj": FLOP_PER_TRIPLE * ww["adjoint_two"] + FLOP_PER_TRIPLE_ONE * ww["adjoint_one"]}


def live_ring_bytes(nside, lmax, w, fg_bytes):
    """Algorithmic HBM bytes of the weighted ring stage: F read and G written for every ring that
    carries weight (fg_bytes per (ring, m) each) and W read on those rings (8 B per pixel)."""
    import numpy as np
    import akra_workloads as wl
    zs, ns, p0, ofs = wl.ring_layout(nside)
    live = np.array([np.any(w[o:o + n] != 0) for o, n in zip(ofs, ns)])
    return int(2 * fg_bytes * live.sum() * (lmax + 1) + 8 * ns[live].sum()), int(live.sum())


# HBM bytes per apply of the dominant stage from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE at this
# workload, each scaled by the same counter's reading for a device copy of known size; valid only for
# the kernel sources and launch shapes they were taken with (the SHA-256 of the Legendre sources and
# the plan's two- and one-sided shapes are checked at run time).
TRAFFIC = {
    # profiles/k_leg_adj_nside2048_lmax4096_fp64.md: two-sided k_leg_adj<double, 4, 1, 8, 0, 0>
    # FETCH 6.1001e5 KiB x 2.0 + WRITE 8.3224e5 KiB, one-sided k_leg_adj<double, 7, 1, 8, 0, 2>
    # FETCH 6.0235e5 KiB x 2.0 + WRITE 9.8547e5 KiB (means of the two dispatches of each run)
    "leg_adj": {"bytes": 4.344e9, "workload": (2048, 4096), "shapes": ((0, 1, 5, 1, 8), (0, 2, 8, 1, 8)),
                "sources_sha256": "dad28f34f7f07a6d8186e7387dbe4b6f9f9c1495755f63a184261ce44d0388b1"},
}
LEG_SOURCES = ("akra_leg.h", "akra_leg_both.hip", "akra_leg_north.hip", "akra_leg_south.hip", "akra_kernels.hip")


def legendre_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for name in LEG_SOURCES:
        with open(os.path.join(ROOT, "paper_2606_06175_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic(stage, nside, lmax, shapes):
    rec = TRAFFIC.get(stage)
    if not rec or rec["workload"] != (nside, lmax) or tuple(map(tuple, shapes)) != rec["shapes"]:
        return None
    if legendre_sources_sha256() != rec["sources_sha256"]:
        return None
    return rec["bytes"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def triples(nside, lmax):
    """T = #(l, m, ring pair) with max(2, m) <= l <= lmax."""
    npairs = 2 * nside
    return npairs * sum(lmax - max(2, m) + 1 for m in range(lmax + 1))


def l_of(lmax):
    import numpy as np
    return np.concatenate([np.arange(m, lmax + 1) for m in range(lmax + 1)])


def make_inputs(name, nside, lmax, dev):
    """Synthetic inputs on the device; gamma_obs = M (Y(K kappa) + eps) with Y from the HIP path."""
    import numpy as np
    import torch

    import akra_workloads as wl
    from paper_2606_06175_amd import Plan

    t = time.time()
    cfg = wl.make_config(name, nside=nside, lmax=lmax)
    log("inputs generated in %.1f s (f_sky %.4f)" % (time.time() - t, cfg["mask"].mean()))
    l = l_of(lmax)
    K = np.zeros(lmax + 1)
    ll = np.arange(2, lmax + 1, dtype=np.float64)
    K[2:] = np.sqrt((ll - 1) * (ll + 2) / (ll * (ll + 1)))
    kap = torch.from_numpy(cfg["kappa"][0] * K[l]).to(dev)
    mask = torch.from_numpy(cfg["mask"]).to(dev)
    ninv = torch.from_numpy(cfg["ninv"][0]).to(dev)
    p = Plan(nside, lmax, precision="fp64", device=dev)
    g1, g2 = p.synth2(kap, torch.zeros_like(kap))
    p.close()
    m = mask.to(torch.float64)
    g1 = m * (g1 + torch.from_numpy(cfg["eps1"][0]).to(dev))
    g2 = m * (g2 + torch.from_numpy(cfg["eps2"][0]).to(dev))
    torch.cuda.synchronize()
    return cfg, g1, g2, ninv, mask


def fp32_roofline(plan32, g1, g2, ninv, mask, nside, lmax, steps=3):
    """The FP32 operator's Legendre kernels (the mixed solve's iterations) against the FP32 peaks:
    157.3 TFLOP/s is the packed-FP32 figure; the kernels issue plain FP32 VALU instructions, whose
    rate is that of FP64 (78.6 TFLOP/s).  Stage times are HIP events over `steps` PCG steps; the
    flop count is 26 per (l, m, ring-pair) triple the FP32 plan evaluates in ring groups weighted on
    both sides and 18 per triple of groups weighted on one side."""
    import torch
    plan32.cg_start(g1, g2, ninv, mask)
    plan32.cg_step(1)
    torch.cuda.synchronize()
    plan32.set_timing(True)
    plan32.stage_times()
    plan32.cg_step(steps)
    st = plan32.stage_times()
    plan32.set_timing(False)
    ww = plan32.work_weighted()
    fl = weighted_flops(ww)
    out = {"unit": "TFLOP/s", "peak_packed_fp32": PEAK_FP32 / 1e12, "peak_plain_fp32_issue": PEAK_FP64 / 1e12,
           "steps": steps}
    for stage, key in (("leg_synth", "synth"), ("leg_adj", "adjoint")):
        ms = st[stage][0] / max(st[stage][1], 1)
        achieved = fl[stage] / (ms * 1e-3)
        out[stage] = {"ms": ms, "evaluated_triples_two_sided": ww[key + "_two"],
                      "evaluated_triples_one_sided": ww[key + "_one"], "flop": fl[stage], "achieved": achieved / 1e12,
                      "frac_of_packed_peak": achieved / PEAK_FP32, "frac_of_plain_issue": achieved / PEAK_FP64}
    return out


def cpu_model():
    """Model name of the host CPU (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(cfg, nside, lmax, nsample):
    """The oracle (plain C, long double, direct ring sums) applying H on a stratified sample of rings;
    one full apply is extrapolated as sample time x nrings / nsample."""
    import numpy as np

    import akra_workloads as wl
    from oracle.core import Oracle
    from oracle.geometry import healpix_rings

    rings = healpix_rings(nside)
    o = Oracle(lmax, rings)
    idx = np.linspace(0, rings.nrings - 1, nsample + 2)[1:-1].round().astype(int)
    W = np.zeros(rings.npix)
    Wfull = o.weights(cfg["ninv"][0], cfg["mask"])
    for r in idx:
        a, n = int(rings.ofs[r]), int(rings.nphi[r])
        W[a:a + n] = np.where(Wfull[a:a + n] > 0, Wfull[a:a + n], 1.0)
    x = np.stack([wl.random_alm(lmax, 1, lmin=0), wl.random_alm(lmax, 2, lmin=0)])
    t = time.time()
    o.apply_H(x, W, 1e-3)
    dt = time.time() - t
    full = dt * rings.nrings / nsample
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count()))
    return {"value": 1.0 / full, "unit": "H·v applies/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": "oracle H v with the weight on %d of %d rings (stratified in z): %.1f s; one full apply "
                      "extrapolated as x%d = %.0f s" % (nsample, rings.nrings, dt, rings.nrings // nsample, full),
            "seconds_per_apply": full}


def batched_leg(name, tol, maxiter, solves=True, napply=20):
    """Batched form on the tomographic workload: all right-hand sides in one FP32 plan (matrix-core
    synthesis, lockstep PCG with FP64 reliable updates) against the FP64 solve of one right-hand side.
    solves=False times the batched applies only."""
    import numpy as np
    import torch

    import akra_workloads as wl
    from paper_2606_06175_amd import Plan

    dev = torch.device("cuda", 0)
    t = time.time()
    cfg = wl.make_config(name)
    nside, lmax, nr = cfg["nside"], cfg["lmax"], cfg["nrhs"]
    log("batched inputs %s (nside %d lmax %d, %d rhs) generated in %.1f s" % (name, nside, lmax, nr, time.time() - t))
    K = np.zeros(lmax + 1)
    ll = np.arange(2, lmax + 1, dtype=np.float64)
    K[2:] = np.sqrt((ll - 1) * (ll + 2) / (ll * (ll + 1)))
    kap = torch.from_numpy(cfg["kappa"] * K[l_of(lmax)][None, :]).to(dev)
    mask = torch.from_numpy(cfg["mask"]).to(dev)
    m = mask.to(torch.float64)
    p = Plan(nside, lmax, precision="fp64", device=dev)
    g1 = torch.empty((nr, 12 * nside * nside), dtype=torch.float64, device=dev)
    g2 = torch.empty_like(g1)
    for k in range(nr):
        a, b = p.synth2(kap[k].contiguous(), torch.zeros_like(kap[k]))
        if cfg["rot1"] is not None:
            # shape-noise realisations: the signal enters rotated, R gamma with R = rot1 + i rot2
            r1, r2 = (torch.from_numpy(cfg[n][k]).to(dev) for n in ("rot1", "rot2"))
            a, b = r1 * a - r2 * b, r1 * b + r2 * a
        g1[k] = m * (a + torch.from_numpy(cfg["eps1"][k]).to(dev))
        g2[k] = m * (b + torch.from_numpy(cfg["eps2"][k]).to(dev))
    ninv = torch.from_numpy(cfg["ninv"][cfg["bin"]]).to(dev)
    torch.cuda.synchronize()
    if solves:
        t = time.perf_counter()
        xE, xB, info64 = p.cg_solve(g1[0].contiguous(), g2[0].contiguous(), ninv[0].contiguous(), mask, tol=tol,
                                    maxiter=maxiter, raise_not_converged=False)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t
    p.close()
    pb = Plan(nside, lmax, nrhs=nr, precision="fp32", device=dev)
    # batched operator applies (all right-hand sides): 3 warm-ups, then the median of 20, each timed with
    # HIP events on the plan stream (torch's current stream); stage times averaged over the 20
    xs = [torch.from_numpy(np.stack([wl.random_alm(lmax, 70 + k) for k in range(nr)])).to(dev) for _ in (0, 1)]
    for _ in range(3):
        pb.apply_H(ninv, mask, xs[0], xs[1], 1e-3)
    torch.cuda.synchronize()
    pb.set_timing(True)
    pb.stage_times()
    ts = []
    for _ in range(napply):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        pb.apply_H(ninv, mask, xs[0], xs[1], 1e-3)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    st = pb.stage_times()
    pb.set_timing(False)
    t_apply = float(np.median(ts)) * 1e-3
    per_apply = {k: v[0] / napply for k, v in st.items() if v[1]}
    # matrix-core Legendre stages against the FP32 MFMA peak: (10 + 16 K) flop per evaluated
    # (l, m, ring-pair) triple and direction for K right-hand sides (two recurrence steps shared by the
    # right-hand sides, eight multiply-adds per right-hand side)
    tb_eval = pb.work_weighted()["batched"]  # ring groups with weight in some right-hand side
    flop = (10 + 16 * nr) * tb_eval
    mfma = {"unit": "TFLOP/s", "peak": PEAK_FP32 / 1e12, "evaluated_triples": tb_eval,
            "flop_per_launch_set": flop, "note": "per batched apply; the right-hand sides run in groups of 8"}
    for stage in ("leg_synth", "leg_adj"):
        if stage in per_apply:
            a = flop / (per_apply[stage] * 1e-3)
            mfma[stage] = {"ms": per_apply[stage], "achieved": a / 1e12, "frac": a / PEAK_FP32}
    apply_out = {"batched_apply_ms": t_apply * 1e3, "rhs_applies_per_s": nr / t_apply,
                 "batched_apply_timing": "median of %d applies after 3 warm-ups, HIP events" % napply,
                 "batched_apply_stages_ms": {k: round(v, 3) for k, v in per_apply.items()},
                 "mfma_roofline": mfma}
    if not solves:
        pb.close()
        out = {"workload": "%s: HEALPix Nside %d, lmax %d, %d right-hand sides (applies only)" % (name, nside, lmax, nr)}
        out.update(apply_out)
        log("batched: %s" % out)
        return out
    torch.cuda.synchronize()
    t = time.perf_counter()
    yE, yB, infob = pb.cg_solve(g1, g2, ninv, mask, tol=tol, maxiter=maxiter, raise_not_converged=False)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t
    err = full_norm(yE[0] - xE, yB[0] - xB, lmax) / full_norm(xE, xB, lmax)
    # shape-noise realisations (Sec. IV power spectra): the shear of the first bin shuffled nr ways
    # among the unmasked pixels, all reconstructed in one batch (E-mode solve), EE spectra and moments
    n_obs = int(cfg["mask"].sum())
    perm = torch.from_numpy(wl.shuffle_perms(n_obs, nr, 4)).to(dev)
    work = torch.empty(pb.noise_work_bytes(1), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    t = time.perf_counter()
    cl, _, _, infon = pb.noise_spectra(g1[0].contiguous(), g2[0].contiguous(), ninv[0].contiguous(), mask, perm,
                                       tol=tol, maxiter=maxiter, mode="E", raise_not_converged=False, work=work)
    torch.cuda.synchronize()
    tn = time.perf_counter() - t
    noise = {"workload": "%d shuffled realisations of bin 0 (%d unmasked pixels), E-mode solves in one FP32 batch, "
                        "EE spectra, mean and scatter" % (nr, n_obs),
             "seconds": tn, "realisations_per_s": nr / tn, "iters": infon["iters"],
             "fp64_applies": infon["fp64_applies"], "worst_rel_resid_true": infon["rel_resid_true"],
             "status": infon["status"], "finite": bool(torch.isfinite(cl).all())}
    del work, perm, cl
    pb.close()
    out = {"workload": "%s: HEALPix Nside %d, lmax %d, %d right-hand sides (4 bins with own N^-1, each a signal and "
                       "3 shape-noise realisations of randomly rotated galaxy ellipticities)" % (name, nside, lmax, nr),
           "fp64_single_rhs": {"seconds": t64, "iters": info64["iters"], "rel_resid_true": info64["rel_resid_true"]},
           "batched_fp32": {"seconds": tb, "iters": infob["iters"], "fp64_applies": infob["fp64_applies"],
                            "worst_rel_resid_true": infob["rel_resid_true"], "status": infob["status"],
                            "rel_err_rhs0_vs_fp64": err},
           "seconds_per_rhs_fp64": t64, "seconds_per_rhs_batched": tb / nr,
           "speedup_per_rhs_vs_fp64": t64 / (tb / nr),
           "noise_realisations": noise}
    out.update(apply_out)
    log("batched: %s" % out)
    return out


def grad_leg(name, tol, maxiter, reps=3):
    """Differentiable solve on the C5 workload (HEALPix Nside 256, lmax 512, FP64): forward solve
    through AkraSolve, loss = sum of the E-mode band powers of kappa_E over 8 log bins, backward
    (the adjoint CG solve and the pullback to gamma_1, gamma_2, N^-1).  Seconds are the median of
    `reps` runs after one warm-up, each phase between two device synchronisations."""
    import numpy as np
    import torch

    import akra_workloads as wl
    from paper_2606_06175_amd import AkraSolve, Plan
    from paper_2606_06175_amd.bandpower import BandPower

    dev = torch.device("cuda", 0)
    t = time.time()
    nside, lmax = wl.CONFIGS[name]["nside"], wl.CONFIGS[name]["lmax"]
    cfg, g1, g2, ninv, mask = make_inputs(name, nside, lmax, dev)
    log("grad inputs %s generated in %.1f s" % (name, time.time() - t))
    p = Plan(nside, lmax, precision="fp64", device=dev)
    bp = BandPower(lmax, device=dev)
    opts = dict(tol=tol, maxiter=maxiter)
    fw, bw = [], []
    for it in range(reps + 1):
        ts = [a.detach().clone().requires_grad_(True) for a in (g1, g2, ninv)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xE, xB = AkraSolve.apply(ts[0], ts[1], ts[2], mask, p, opts)
        L = bp.loss(xE)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if it:
            fw.append(t1 - t0)
            bw.append(t2 - t1)
    fi, bi = p.last_solve_info, p.last_vjp_info
    finite = all(bool(torch.isfinite(a.grad).all()) for a in ts)
    out = {"workload": "%s: HEALPix Nside %d, lmax %d, FP64, loss = sum of 8 log-bin E-mode band powers of kappa_E"
                       % (name, nside, lmax),
           "forward_s": float(np.median(fw)), "backward_s": float(np.median(bw)),
           "forward_backward_s": float(np.median(fw)) + float(np.median(bw)),
           "forward_iters": fi["iters"], "backward_iters": bi["iters"], "tol": tol,
           "forward_rel_resid_true": fi["rel_resid_true"], "backward_rel_resid_true": bi["rel_resid_true"],
           "loss": float(L.detach()), "gradients_finite": finite, "reps": reps}
    log("grad: %s" % out)
    p.close()
    return out


def pixelize_leg(n_gal, nside, reps=3):
    """Catalogue pixelisation (Sec. III.B): n_gal synthetic galaxies binned onto the HEALPix grid, with
    per-pixel weighted shear, N_eff, N^-1 and mask; inputs resident in HBM, workspace preallocated."""
    import torch

    import akra_workloads as wl
    from paper_2606_06175_amd import Plan

    dev = torch.device("cuda", 0)
    t = time.time()
    c = wl.make_catalog(n_gal, 3)
    log("catalogue of %d galaxies generated in %.1f s" % (n_gal, time.time() - t))
    ts = {k: torch.from_numpy(c[k]).to(dev) for k in ("z", "phi", "e1", "e2", "w")}
    del c["z"], c["phi"], c["e1"], c["e2"], c["w"]
    p = Plan(nside, 2, device=dev)
    work = torch.empty(p.pixelize_work_bytes(n_gal), dtype=torch.uint8, device=dev)
    args = [ts[k] for k in ("z", "phi", "e1", "e2", "w")] + [c["R"], c["sigma_e"], c["n_th"]]
    o = p.pixelize(*args, work=work)  # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        o = p.pixelize(*args, work=work)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    npix = p.npix
    alg = 40.0 * n_gal + 33.0 * npix  # five float64 per galaxy in; four float64 and a byte per pixel out
    out = {"workload": "%d galaxies (uniform in a southern box of f_sky 0.1) onto HEALPix Nside %d" % (n_gal, nside),
           "ms": dt * 1e3, "galaxies_per_s": n_gal / dt, "algorithmic_GBs": alg / dt / 1e9,
           "unmasked_pixels": int(o["mask"].sum()), "work_GB": work.numel() / 1e9}
    log("pixelize: %s" % out)
    del work, ts, o
    p.close()
    return out


# HBM bytes one flat-sky H apply must move per grid point: three row-transform passes that read and
# write the complex field (3 x 32 B), two transposes (2 x 32 B), the weight (8 B) and the + lambda x
# read of the last pass (16 B)
FLAT_BYTES_PER_POINT = 3 * 32 + 2 * 32 + 8 + 16


def flat_leg(n, steps, tol, maxiter):
    """Flat-sky variant: an n x n field (border and holes, Poisson mean 2), FP64 operator; applies/s
    from the step-wise PCG on device-resident data, the HBM roofline of one apply, and a solve."""
    import torch

    import akra_workloads as wl
    from paper_2606_06175_amd import FlatPlan

    dev = torch.device("cuda", 0)
    t = time.time()
    f = wl.make_flat(n, n, 3)
    log("flat field %d x %d generated in %.1f s (unmasked %.3f)" % (n, n, time.time() - t, f["mask"].mean()))
    p = FlatPlan(n, n, device=dev)
    kE = torch.from_numpy(f["kappa"].real.copy()).to(dev)
    g1, g2 = p.synth(kE, torch.zeros_like(kE))
    m = torch.from_numpy(f["mask"]).to(dev)
    mf = m.to(torch.float64)
    g1 = mf * (g1 + torch.from_numpy(f["eps1"]).to(dev))
    g2 = mf * (g2 + torch.from_numpy(f["eps2"]).to(dev))
    ninv = torch.from_numpy(f["ninv"]).to(dev)
    p.cg_start(g1, g2, ninv, m)
    p.cg_step(2)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    p.cg_step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, _, info = p.cg_solve(g1, g2, ninv, m, tol=tol, maxiter=maxiter, raise_not_converged=False)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t
    gbs = FLAT_BYTES_PER_POINT * n * n / (ms * 1e-3) / 1e9
    out = {"workload": "flat field %d x %d, FP64, joint E/B" % (n, n), "applies_per_s": 1e3 / ms,
           "ms_per_step": ms, "algorithmic_bytes_per_apply": FLAT_BYTES_PER_POINT * n * n,
           "hbm_GBs": gbs, "hbm_frac": gbs / 8000.0,
           "solve_to_%g" % tol: {"seconds": ts, "iters": info["iters"], "rel_resid_true": info["rel_resid_true"],
                                 "status": info["status"]}}
    log("flat: %s" % out)
    p.close()
    return out


def rates_leg(c3cfg, tol, maxiter):
    """Apply rates of akra_apply_H (FP64 and FP32, single right-hand side) at every configuration and
    time-to-tol below the headline size (the oracle beside them is part of cpu_baseline).  Each rate is the median
    of 20 applies after 3 warm-ups, HIP events on the plan stream; an apply includes its weight
    set-up (one reduction and one host synchronisation)."""
    import numpy as np
    import torch

    import akra_workloads as wl
    from paper_2606_06175_amd import Plan

    dev = torch.device("cuda", 0)
    out = {}
    for name in ("C1", "C5", "C2", "C3"):
        cfg = c3cfg if name == "C3" else wl.make_config(name)
        nside, lmax = cfg["nside"], cfg["lmax"]
        ninv = torch.from_numpy(cfg["ninv"][0]).to(dev)
        mask = torch.from_numpy(cfg["mask"]).to(dev)
        xa = [torch.from_numpy(wl.random_alm(lmax, 1 + k)).to(dev) for k in (0, 1)]
        row = {"workload": "%s: HEALPix Nside %d, lmax %d" % (name, nside, lmax)}
        if name != "C3":
            l = l_of(lmax)
            K = np.zeros(lmax + 1)
            ll = np.arange(2, lmax + 1, dtype=np.float64)
            K[2:] = np.sqrt((ll - 1) * (ll + 2) / (ll * (ll + 1)))
            kap = torch.from_numpy(cfg["kappa"][0] * K[l]).to(dev)
        for prec in ("fp64", "fp32"):
            p = Plan(nside, lmax, precision=prec, device=dev)
            for _ in range(3):
                p.apply_H(ninv, mask, xa[0], xa[1], 1e-3)
            ts = []
            for _ in range(20):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                p.apply_H(ninv, mask, xa[0], xa[1], 1e-3)
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            row[prec + "_applies_per_s"] = 1e3 / float(np.median(ts))
            if name != "C3":
                g1, g2 = p.synth2(kap, torch.zeros_like(kap))
                m = mask.to(torch.float64)
                g1 = m * (g1 + torch.from_numpy(cfg["eps1"][0]).to(dev))
                g2 = m * (g2 + torch.from_numpy(cfg["eps2"][0]).to(dev))
                torch.cuda.synchronize()
                t = time.perf_counter()
                _, _, info = p.cg_solve(g1, g2, ninv, mask, tol=tol, maxiter=maxiter, raise_not_converged=False)
                torch.cuda.synchronize()
                row[prec + "_solve"] = {"seconds": time.perf_counter() - t, "iters": info["iters"],
                                        "fp64_applies": info["fp64_applies"],
                                        "rel_resid_true": info["rel_resid_true"], "status": info["status"]}
                if prec == "fp64":
                    # the same solve testing convergence every 8 iterations (one synchronisation per test)
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    _, _, info = p.cg_solve(g1, g2, ninv, mask, tol=tol, maxiter=maxiter, raise_not_converged=False,
                                            check_every=8)
                    torch.cuda.synchronize()
                    row["fp64_solve_check_every_8"] = {"seconds": time.perf_counter() - t, "iters": info["iters"],
                                                       "rel_resid_true": info["rel_resid_true"],
                                                       "status": info["status"]}
            p.close()
        log("rates %s: %s" % (name, row))
        out[name] = row
    return out


def cpu_baseline_configs(rates, tol, maxiter):
    """The oracle beside the GPU rates of rates_leg: applies/s at C1, C5 and C2, its time-to-tol at C1
    (measured) and at C5 and C2 (extrapolated from the GPU FP64 iteration count)."""
    import numpy as np

    import akra_workloads as wl
    from oracle.core import Oracle
    from oracle.geometry import healpix_rings

    out = {}
    for name in ("C1", "C5", "C2"):
        cfg = wl.make_config(name)
        nside, lmax = cfg["nside"], cfg["lmax"]
        o = Oracle(lmax, healpix_rings(nside))
        W = o.weights(cfg["ninv"][0], cfg["mask"])
        x = np.stack([wl.random_alm(lmax, 1), wl.random_alm(lmax, 2)])
        t = time.time()
        o.apply_H(x, W, 1e-3)
        dt = time.time() - t
        orc = {"workload": "%s: HEALPix Nside %d, lmax %d" % (name, nside, lmax), "applies_per_s": 1.0 / dt,
               "seconds_per_apply": dt}
        iters = rates[name]["fp64_solve"]["iters"]
        if name == "C1":
            lam = o.lambda_eff(cfg["ninv"][0], cfg["mask"])
            g1, g2 = o.synth(o.kernel()[o.l_of] * cfg["kappa"][0], np.zeros(o.nalm, np.complex128))
            m = cfg["mask"].astype(np.float64)
            b = o.rhs(m * (g1 + cfg["eps1"][0]), m * (g2 + cfg["eps2"][0]), W)
            t = time.time()
            _, oi = o.cg(b, W, lam, o.precond(cfg["ninv"][0], cfg["mask"], lam), tol=tol, maxiter=maxiter)
            orc["time_to_tol"] = {"seconds": time.time() - t, "iters": oi["iters"], "measured": True}
        else:
            orc["time_to_tol"] = {"seconds": iters * dt, "iters": iters, "measured": False,
                                  "note": "extrapolated: GPU FP64 iteration count x oracle seconds per apply"}
        log("oracle %s: %s" % (name, orc))
        out[name] = orc
    return out


def full_norm(a, b, lmax):
    """Full-m norm of stacked (E, B) complex alm on the device."""
    import torch
    w = torch.full((a.shape[-1],), 2.0, dtype=torch.float64, device=a.device)
    w[: lmax + 1] = 1.0
    return float(torch.sqrt((w * (a.abs() ** 2)).sum() + (w * (b.abs() ** 2)).sum()))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="C3")
    ap.add_argument("--nside", type=int, default=None)
    ap.add_argument("--lmax", type=int, default=None)
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-workload", default="C4")
    ap.add_argument("--no-pixelize", action="store_true")
    ap.add_argument("--no-grad", action="store_true")
    ap.add_argument("--only", choices=("batched", "grad", "pixelize", "flat"), default=None,
                    help="run one leg alone and print its JSON (with --no-solve the batched leg times its applies "
                         "only); for profiling one group of kernels")
    ap.add_argument("--lds-rings", action="store_true",
                    help="run every ring on the LDS kernels (no register engine), for timing comparisons")
    ap.add_argument("--precision", choices=("fp64", "fp32"), default="fp64",
                    help="precision of the plan the timed PCG steps run on")
    ap.add_argument("--no-flat", action="store_true")
    ap.add_argument("--no-rates", action="store_true")
    ap.add_argument("--flat-n", type=int, default=4096)
    ap.add_argument("--pixelize-galaxies", type=int, default=100_000_000)
    ap.add_argument("--cpu-sample-rings", type=int, default=192)
    ap.add_argument("--solve-tol", type=float, default=1e-8)
    ap.add_argument("--maxiter", type=int, default=3000)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only time a plain device-to-device copy of MIB MiB (4 launches) and exit; the HBM "
                         "counters of that copy calibrate the counters of the operator's kernels")
    ap.add_argument("--mfma-probe", action="store_true",
                    help="print the sustained v_mfma_f32_32x32x2_f32 rate with 0, 4 or 8 pairs of FP32 FMAs "
                         "between the products (akra_mfma_rate) and exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        if int(os.environ.get("RANK", "0")) == 0:
            print("bench.py: the benchmark runs on exactly one GPU (the operator shards by m and by ring "
                  "across GPUs only in design); run with --gpus 1", flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import akra_workloads as wl
    from paper_2606_06175_amd import Plan

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.lds_rings:
        from paper_2606_06175_amd import akra
        akra.set_ring_register_engine(False)
    if args.mfma_probe:
        from paper_2606_06175_amd.akra import mfma_rate
        rows = [{"chains": k, "fma_pairs_between_products": v, "waves_per_simd": w,
                 "TFLOPs": mfma_rate(k, v, w)}
                for k, v, w in ((1, 0, 1), (2, 0, 1), (4, 0, 1), (4, 0, 2), (2, 4, 1), (2, 8, 1), (4, 4, 1), (4, 8, 2))]
        print(json.dumps({"mfma_probe": "v_mfma_f32_32x32x2_f32", "peak": 157.3, "rows": rows}), flush=True)
        return
    if args.copy_calibration:
        n = args.copy_calibration << 20
        src = torch.ones(n // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / 4
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "ms_per_copy": dt * 1e3,
                          "GB_per_s": 2 * n / dt / 1e9}), flush=True)
        return
    if args.only:
        if args.only == "batched":
            res = batched_leg(args.batched_workload, args.solve_tol, args.maxiter, solves=not args.no_solve,
                              napply=max(args.steps, 1))
        elif args.only == "grad":
            res = grad_leg("C5", args.solve_tol, args.maxiter)
        elif args.only == "pixelize":
            res = pixelize_leg(args.pixelize_galaxies, args.nside or 2048)
        else:
            res = flat_leg(args.flat_n, max(args.steps, 10), args.solve_tol, args.maxiter)
        print(json.dumps({"leg": args.only, **res}), flush=True)
        return
    p = wl.CONFIGS[args.workload]
    nside = args.nside or p["nside"]
    lmax = args.lmax or p["lmax"]
    log("workload %s nside %d lmax %d" % (args.workload, nside, lmax))
    cfg, g1, g2, ninv, mask = make_inputs(args.workload, nside, lmax, dev)

    t = time.time()
    plan = Plan(nside, lmax, precision=args.precision, device=dev)
    torch.cuda.synchronize()
    plan_s = time.time() - t
    log("%s plan built in %.1f s, %.2f GB on device" % (args.precision, plan_s, plan.device_bytes / 1e9))
    plan.cg_start(g1, g2, ninv, mask)
    plan.cg_step(args.warmup)
    torch.cuda.synchronize()
    plan.set_timing(True)
    plan.stage_times()  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.cg_step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = plan.stage_times()
    plan.set_timing(False)
    rel, iters = plan.cg_state()
    ms_step = (t1 - t0) * 1e3 / args.steps
    log("%d steps: %.2f ms/step; recursive rel. residual after %d iterations %.3e" % (args.steps, ms_step, iters, rel))
    stages = {k: {"ms_total": v[0], "launches": v[1], "ms_avg": v[0] / max(v[1], 1)} for k, v in st.items()}
    for k, v in stages.items():
        log("  stage %-9s %9.3f ms/launch (%d launches)" % (k, v["ms_avg"], v["launches"]))

    T = triples(nside, lmax)
    work = plan.work()
    assert work["all"] == T
    ww = plan.work_weighted()  # the weighted launches of the timed steps
    fl = weighted_flops(ww)
    dom = max(("leg_synth", "leg_adj"), key=lambda k: stages[k]["ms_avg"])
    achieved = fl[dom] / (stages[dom]["ms_avg"] * 1e-3)
    peak = PEAK_FP64 if args.precision == "fp64" else PEAK_FP32
    key = "synth" if dom == "leg_synth" else "adjoint"
    roofline = {"bound": "alu", "kernel": "k_leg_adj" if dom == "leg_adj" else "k_leg_synth",
                "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                "frac": achieved / peak,
                "traffic": (traffic(dom, nside, lmax, (plan.get_tuning(), plan.get_tuning_one_sided()))
                            if args.precision == "fp64" else None),
                "algorithmic": "26 flop x %d triples of ring groups weighted on both sides + 18 flop x %d of groups "
                               "weighted on one side = %.4g flop per launch (all (l, m, ring-pair) triples T = %d; "
                               "groups without a weighted ring and the terms below each group's entry degree, where "
                               "its recurrence values first reach 2^-100, are skipped)"
                               % (ww[key + "_two"], ww[key + "_one"], fl[dom], T)}
    # ring stage against HBM: F read and G written (32 B per (ring, m) each) and W read (8 B per pixel)
    # on the rings that carry weight (the others are skipped)
    fg_bytes = 32 if args.precision == "fp64" else 16  # (Q, U) complex entry of F or G per (ring, m)
    ring_bytes, n_live = live_ring_bytes(nside, lmax, cfg["mask"] * cfg["ninv"][0], fg_bytes)
    assert n_live == ww["live_rings"], (n_live, ww["live_rings"])
    roofline["evaluated_triples"] = ww  # per launch of each class (akra_plan_work_weighted)
    # the sustained plain FMA rate of this device under load (akra_fma_rate), beside the published peak
    from paper_2606_06175_amd.akra import fma_rate
    roofline["fma_ceiling_TFLOPs"] = fma_rate(args.precision)
    roofline["frac_of_fma_ceiling"] = roofline["achieved"] / roofline["fma_ceiling_TFLOPs"]
    roofline["ring_algorithmic_bytes"] = ring_bytes
    roofline["ring_rings_with_weight"] = n_live
    roofline["ring_hbm_GBs"] = ring_bytes / (stages["ring"]["ms_avg"] * 1e-3) / 1e9
    roofline["ring_hbm_frac"] = roofline["ring_hbm_GBs"] / 8000.0
    for k in ("leg_synth", "leg_adj"):
        t = stages[k]["ms_avg"] * 1e-3
        kk = "synth" if k == "leg_synth" else "adjoint"
        roofline["frac_" + k] = fl[k] / t / peak
        roofline["evaluated_fraction_" + k] = (ww[kk + "_two"] + ww[kk + "_one"]) / T
        roofline["full_T_rate_TFLOPs_" + k] = FLOP_PER_TRIPLE * T / t / 1e12
    out = {"metric": METRIC, "value": 1e3 / ms_step, "unit": "H·v applies/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32",
           "data": "synthetic",
           "config": {"workload": "%s: HEALPix Nside %d, lmax %d, single RHS, joint E/B, f_sky %.3f"
                                  % (args.workload, nside, lmax, float(cfg["mask"].mean())),
                      "nside": nside, "lmax": lmax, "nrhs": 1, "precision": args.precision},
           "roofline": roofline,
           "stages_ms": {k: round(v["ms_avg"], 4) for k, v in stages.items()},
           "plan_build_s": plan_s,
           "paper_context": {"applies_per_s": 0.044, "hardware": "one 72-CPU node",
                             "note": "derived from ~80 CG iterations in ~0.5 h at Nside 2048, lmax 4096 (DES Y3)"}}

    if args.precision != "fp64":
        args.no_solve = True  # the solve comparison runs its own FP64 and FP32 plans
    if not args.no_solve:
        solves = {}
        torch.cuda.synchronize()
        t = time.perf_counter()
        xE, xB, info = plan.cg_solve(g1, g2, ninv, mask, tol=args.solve_tol, maxiter=args.maxiter,
                                     raise_not_converged=False)
        torch.cuda.synchronize()
        solves["fp64"] = {"seconds": time.perf_counter() - t, "iters": info["iters"],
                          "rel_resid_true": info["rel_resid_true"], "status": info["status"]}
        log("fp64 solve: %s" % solves["fp64"])
        plan.close()
        plan32 = Plan(nside, lmax, precision="fp32", device=dev)
        torch.cuda.synchronize()
        t = time.perf_counter()
        yE, yB, info32 = plan32.cg_solve(g1, g2, ninv, mask, tol=args.solve_tol, maxiter=args.maxiter,
                                         raise_not_converged=False)
        torch.cuda.synchronize()
        err = full_norm(yE - xE, yB - xB, lmax) / full_norm(xE, xB, lmax)
        solves["mixed_fp32_fp64"] = {"seconds": time.perf_counter() - t, "iters": info32["iters"],
                                     "fp64_applies": info32["fp64_applies"],
                                     "rel_resid_true": info32["rel_resid_true"], "status": info32["status"],
                                     "rel_err_vs_fp64_solution": err}
        log("mixed solve: %s" % solves["mixed_fp32_fp64"])
        out["roofline_fp32"] = fp32_roofline(plan32, g1, g2, ninv, mask, nside, lmax)
        log("fp32 Legendre roofline: %s" % out["roofline_fp32"])
        plan32.close()
        out["time_to_1e-8"] = solves
        out["mixed_speedup_vs_fp64"] = solves["fp64"]["seconds"] / solves["mixed_fp32_fp64"]["seconds"]
    else:
        plan.close()

    if not args.no_solve and not args.no_batched:
        out["batched"] = batched_leg(args.batched_workload, args.solve_tol, args.maxiter)
    if not args.no_solve and not args.no_grad:
        out["differentiable"] = grad_leg("C5", args.solve_tol, args.maxiter)
    if not args.no_pixelize:
        out["pixelize"] = pixelize_leg(args.pixelize_galaxies, nside)
    if not args.no_flat:
        out["flat"] = flat_leg(args.flat_n, max(args.steps, 10), args.solve_tol, args.maxiter)
    rates = None
    if not args.no_solve and not args.no_rates and args.workload == "C3" and args.nside is None and args.lmax is None:
        rates = rates_leg(cfg, args.solve_tol, args.maxiter)
        out["apply_rates"] = rates

    if not args.no_cpu_baseline:
        t = time.time()
        out["cpu_baseline"] = cpu_baseline(cfg, nside, lmax, args.cpu_sample_rings)
        log("cpu baseline in %.1f s: %s" % (time.time() - t, out["cpu_baseline"]["sample"]))
        if rates is not None:
            out["cpu_baseline"]["per_config"] = cpu_baseline_configs(rates, args.solve_tol, args.maxiter)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
