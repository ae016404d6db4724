"""FP64 true residual of the benchmark-size solutions, computed by the oracle.

HEALPix Nside 2048, lmax 4096 (the headline workload: 3-cap footprint minus 2000 holes, Poisson mean
2 with the smooth depth modulation).  The GPU solves the regularised system to a relative residual
of 1e-8 twice, with the FP64 plan and with the FP32 plan and FP64 reliable updates; the oracle then
evaluates, for each solution x,

    ||b - H x|| / ||b||,   b - H x = K Y^H (W (gamma_obs - Y K x)) - lambda_eff x,   b = K Y^H (W gamma_obs)

with its own synthesis and adjoint (long-double recurrence, direct ring sums) on the rings that carry
weight, in the full-m norm (paper Sec. II.B, eq. normal_eq and eq. ML_estimator_reg).  Both inputs of
the oracle, gamma_obs and x, are the arrays the GPU used and returned.  One oracle apply at this size
takes minutes on the host cores, too long for the test suite, so this is a script; it prints its
progress per block of rings and writes its result as JSON.

    python tests/c3_oracle_residual.py [--out c3_oracle_residual.json] [--chunks 16]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def log(*a):
    print(*a, flush=True)


def gpu_solutions(tol, maxiter):
    """gamma_obs (built on the GPU from the seeded inputs), N^-1, mask and the FP64 and mixed solutions."""
    import torch

    import akra_workloads as wl
    from paper_2606_06175_amd import Plan

    dev = torch.device("cuda", 0)
    t = time.time()
    cfg = wl.make_config("C3")
    nside, lmax = cfg["nside"], cfg["lmax"]
    log("inputs generated in %.1f s (f_sky %.4f)" % (time.time() - t, cfg["mask"].mean()))
    l = np.concatenate([np.arange(m, lmax + 1) for m in range(lmax + 1)])
    K = np.zeros(lmax + 1)
    ll = np.arange(2, lmax + 1, dtype=np.float64)
    K[2:] = np.sqrt((ll - 1) * (ll + 2) / (ll * (ll + 1)))
    kap = torch.from_numpy(cfg["kappa"][0] * K[l]).to(dev)
    mask = torch.from_numpy(cfg["mask"]).to(dev)
    ninv = torch.from_numpy(cfg["ninv"][0]).to(dev)
    p = Plan(nside, lmax, precision="fp64", device=dev)
    g1, g2 = p.synth2(kap, torch.zeros_like(kap))
    m = mask.to(torch.float64)
    g1 = m * (g1 + torch.from_numpy(cfg["eps1"][0]).to(dev))
    g2 = m * (g2 + torch.from_numpy(cfg["eps2"][0]).to(dev))
    out = {"g1": g1.cpu().numpy(), "g2": g2.cpu().numpy(), "ninv": cfg["ninv"][0], "mask": cfg["mask"],
           "nside": nside, "lmax": lmax}
    sols = {}
    for prec in ("fp64", "fp32"):
        q = p if prec == "fp64" else Plan(nside, lmax, precision="fp32", device=dev)
        torch.cuda.synchronize()
        t = time.time()
        xE, xB, info = q.cg_solve(g1, g2, ninv, mask, tol=tol, maxiter=maxiter)
        torch.cuda.synchronize()
        dt = time.time() - t
        log("%s solve: %.2f s, %d iterations, GPU true residual %.4e" % (prec, dt, info["iters"],
                                                                        info["rel_resid_true"]))
        sols[prec] = {"x": np.stack([xE.cpu().numpy(), xB.cpu().numpy()]), "seconds": dt, "iters": info["iters"],
                      "gpu_rel_resid_true": info["rel_resid_true"], "fp64_applies": info["fp64_applies"]}
        q.close()
    out["solutions"] = sols
    return out


def oracle_residuals(d, nchunk):
    from oracle.core import Oracle
    from oracle.geometry import healpix_rings

    nside, lmax = d["nside"], d["lmax"]
    o = Oracle(lmax, healpix_rings(nside))
    W = o.weights(d["ninv"], d["mask"])
    lam = o.lambda_eff(d["ninv"], d["mask"])
    Kl = o.kernel()[o.l_of]
    act = o._active_rings(W)
    blocks = np.array_split(act, nchunk)
    log("oracle: %d of %d rings carry weight, %d blocks; lambda_eff %.6e" % (len(act), o.rings.nrings, nchunk, lam))

    def adjoint_active(h1, h2, what):
        cE = np.zeros(o.nalm, np.complex128)
        cB = np.zeros(o.nalm, np.complex128)
        t = time.time()
        for i, blk in enumerate(blocks):
            a, b = o.adjoint(h1, h2, ring_idx=blk)
            cE += a
            cB += b
            log("  %s adjoint: block %d/%d (%.0f s)" % (what, i + 1, nchunk, time.time() - t))
        return cE, cB

    def synth_active(aE, aB, what):
        s1 = np.zeros(o.rings.npix)
        s2 = np.zeros(o.rings.npix)
        t = time.time()
        for i, blk in enumerate(blocks):
            a, b = o.synth(aE, aB, ring_idx=blk)
            s1 += a
            s2 += b
            log("  %s synthesis: block %d/%d (%.0f s)" % (what, i + 1, nchunk, time.time() - t))
        return s1, s2

    cE, cB = adjoint_active(W * d["g1"], W * d["g2"], "b")
    b = o._project(np.stack([Kl * cE, Kl * cB]))
    bn = np.sqrt(o.dot(b, b))
    res = {"b_norm": bn, "lambda_eff": lam, "active_rings": int(len(act))}
    for prec, s in d["solutions"].items():
        x = o._project(s["x"])
        s1, s2 = synth_active(Kl * x[0], Kl * x[1], prec)
        cE, cB = adjoint_active(W * (d["g1"] - s1), W * (d["g2"] - s2), prec)
        r = o._project(np.stack([Kl * cE, Kl * cB]) - lam * x)
        rr = float(np.sqrt(o.dot(r, r)) / bn)
        log("%s: oracle true residual ||b - H x|| / ||b|| = %.4e (GPU reported %.4e)"
            % (prec, rr, s["gpu_rel_resid_true"]))
        res[prec] = {"oracle_rel_resid_true": rr, "gpu_rel_resid_true": s["gpu_rel_resid_true"],
                     "iters": s["iters"], "seconds": s["seconds"], "fp64_applies": s["fp64_applies"]}
    xa, xb = d["solutions"]["fp64"]["x"], d["solutions"]["fp32"]["x"]
    res["mixed_vs_fp64_rel_diff"] = float(np.sqrt(o.dot(xb - xa, xb - xa) / o.dot(xa, xa)))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="c3_oracle_residual.json")
    ap.add_argument("--chunks", type=int, default=16)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--maxiter", type=int, default=3000)
    args = ap.parse_args()
    t0 = time.time()
    d = gpu_solutions(args.tol, args.maxiter)
    res = oracle_residuals(d, args.chunks)
    res.update({"workload": "HEALPix Nside 2048, lmax 4096, 3-cap footprint minus 2000 holes, Poisson mean 2 x "
                            "U[0.5, 1.5] depth", "tol": args.tol, "threads": os.environ.get("OMP_NUM_THREADS"),
                "seconds_total": time.time() - t0})
    os.makedirs(os.path.dirname(args.out) or ".", exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)
    log(json.dumps(res))
    ok = all(res[p]["oracle_rel_resid_true"] <= 1.05 * args.tol for p in ("fp64", "fp32"))
    sys.exit(0 if ok else 1)


if __name__ == "__main__":
    main()
