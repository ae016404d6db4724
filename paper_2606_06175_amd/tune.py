"""Autotuner for the Legendre launch shapes.

For one (Nside, lmax, precision) it times every supported synthesis variant / ring-pairs-per-lane
choice and every adjoint (ring pairs per lane, waves per workgroup) shape with HIP events on the
plan stream (stage times of PCG iterations on synthetic data), and stores the fastest in
tuning.json next to this file.  It does so twice: on a full sky, where every ring group carries
weight on both of its rings, and on the sky south of z = 0.17 (colatitude 80 degrees), where the
groups near the equator carry weight on both sides and all others on their south rings only, as
in a southern survey footprint; the second sweep varies the shapes of the one-sided groups with the
two-sided ones fixed, and is kept as the entry's "one_sided" shapes.  Adjoint shapes are ranked by
the adjoint and epilogue time together (the epilogue adds the adjoint's ring-block slabs).  For FP32 plans with several right-hand sides (--nrhs K > 1) it tunes
the batched matrix-core kernels instead: waves per workgroup of the synthesis and of the adjoint,
timed over batched operator applies (synthesis, adjoint and the epilogues that add the adjoint's
slabs), cached per (Nside, lmax, K).  Plan() applies the cached shapes automatically.

    python -m paper_2606_06175_amd.tune --nside 2048 --lmax 4096 --precision fp64
    python -m paper_2606_06175_amd.tune --nside 1024 --lmax 2048 --precision fp32 --nrhs 16
"""
import argparse
import json
import os
import sys

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
SYN = [(v, r) for v in (0, 1) for r in (1, 2, 4)]
ADJ = [(r, 1, c) for c in (8, 4) for r in range(1, 9)] + \
      [(1, 2, 8), (1, 4, 8), (2, 2, 8), (2, 4, 8), (4, 2, 8), (4, 4, 8), (8, 2, 8), (2, 4, 4), (4, 2, 4), (4, 4, 4)]


BATCHED = [(sw, aw) for sw in (1, 2, 4, 8) for aw in (2, 4, 8)]


def key(nside, lmax, precision):
    return "%d:%d:%s" % (nside, lmax, precision)


def key_batched(nside, lmax, nrhs):
    return "%d:%d:fp32:nrhs%d" % (nside, lmax, nrhs)


def load_cache():
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            return json.load(f)
    return {}


def lookup(nside, lmax, precision):
    return load_cache().get(key(nside, lmax, precision))


def lookup_batched(nside, lmax, nrhs):
    return load_cache().get(key_batched(nside, lmax, nrhs))


def tune_batched(nside, lmax, nrhs, reps=3, log=print):
    """Time every batched shape over `reps` batched applies (after one warm-up) on random coefficients
    and weights; the figure of merit is synthesis + adjoint + epilogue time per apply."""
    import torch

    from .akra import Plan
    dev = torch.device("cuda", 0)
    plan = Plan(nside, lmax, nrhs=nrhs, precision="fp32", device=dev, tuned=False)
    npix = 12 * nside * nside
    g = torch.Generator(device="cpu").manual_seed(11)
    ninv = (5.0 + 50.0 * torch.rand(nrhs, npix, generator=g, dtype=torch.float64)).to(dev)
    mask = torch.ones(npix, dtype=torch.uint8, device=dev)
    x = [torch.randn(nrhs, plan.nalm, generator=g, dtype=torch.complex128).to(dev) for _ in (0, 1)]
    res = {}
    best, best_t = plan.get_tuning_batched(), float("inf")
    for sw, aw in BATCHED:
        plan.set_tuning_batched(sw, aw)
        plan.apply_H(ninv, mask, x[0], x[1], 1e-3)
        plan.set_timing(True)
        plan.stage_times()
        for _ in range(reps):
            plan.apply_H(ninv, mask, x[0], x[1], 1e-3)
        st = plan.stage_times()
        plan.set_timing(False)
        t = {k: st[k][0] / reps for k in ("leg_synth", "leg_adj", "epilogue")}
        tot = sum(t.values())
        res["%d,%d" % (sw, aw)] = t
        log("  batched synthesis waves %d adjoint waves %d: synth %.3f adj %.3f epi %.3f ms"
            % (sw, aw, t["leg_synth"], t["leg_adj"], t["epilogue"]))
        if tot < best_t:
            best, best_t = (sw, aw), tot
    plan.close()
    return {"syn_waves": best[0], "adj_waves": best[1], "ms": best_t, "reps": reps, "sweep": res}


def _time_stage(plan, stage, steps):
    plan.cg_step(1)
    plan.set_timing(True)
    plan.stage_times()
    plan.cg_step(steps)
    st = plan.stage_times()
    plan.set_timing(False)
    ms, n = st[stage]
    return ms / max(n, 1)


def _time_stages(plan, stages, steps):
    plan.cg_step(1)
    plan.set_timing(True)
    plan.stage_times()
    plan.cg_step(steps)
    st = plan.stage_times()
    plan.set_timing(False)
    return sum(st[s][0] / max(st[s][1], 1) for s in stages)


def pick_synth(syn_sweep, tol=0.02):
    """The synthesis shape of a sweep {"v,r": ms}: among the shapes within tol of the fastest, the
    one with the fewest ring pairs per lane (then the lower variant).  The tuning masks are not the
    user's footprint: fewer pairs per lane keep the entry-degree spread of a wave small on any
    footprint, so near-ties go to them."""
    best = min(syn_sweep.values())
    near = [tuple(map(int, k.split(","))) for k, t in syn_sweep.items() if t <= (1 + tol) * best]
    v, r = min(near, key=lambda vr: (vr[1], vr[0]))
    return (v, r), syn_sweep["%d,%d" % (v, r)]


def _sweep(plan, setter, base_syn, base_adj, steps, log, tag):
    from .akra import AkraError
    res = {"syn": {}, "adj": {}}
    for v, r in SYN:
        setter(v, r, *base_adj)
        t = _time_stage(plan, "leg_synth", steps)
        res["syn"]["%d,%d" % (v, r)] = t
        log("  %s synth variant %d rings/lane %d: %.3f ms" % (tag, v, r, t))
    best_syn, best_t = pick_synth(res["syn"])
    best_adj, best_ta = base_adj, float("inf")
    for r, w, c in ADJ:
        try:
            setter(best_syn[0], best_syn[1], r, w, c)
        except AkraError:
            continue
        t = _time_stages(plan, ("leg_adj", "epilogue"), steps)
        res["adj"]["%d,%d,%d" % (r, w, c)] = t
        log("  %s adjoint rings/lane %d waves %d chunk %d: %.3f ms with the epilogue" % (tag, r, w, c, t))
        if t < best_ta:
            best_adj, best_ta = (r, w, c), t
    setter(best_syn[0], best_syn[1], *best_adj)
    return {"syn_variant": best_syn[0], "syn_rings": best_syn[1], "adj_rings": best_adj[0],
            "adj_waves": best_adj[1], "adj_chunk": best_adj[2], "ms_syn": best_t, "ms_adj": best_ta, "sweep": res}


def tune(nside, lmax, precision="fp64", steps=2, log=print):
    import torch

    from .akra import Plan
    dev = torch.device("cuda", 0)
    plan = Plan(nside, lmax, precision=precision, device=dev, tuned=False)
    npix = 12 * nside * nside
    g = torch.Generator(device="cpu").manual_seed(7)
    g1 = torch.randn(npix, generator=g, dtype=torch.float64).to(dev)
    g2 = torch.randn(npix, generator=g, dtype=torch.float64).to(dev)
    ninv = torch.ones(npix, dtype=torch.float64, device=dev)
    # full sky: every group weighted on both sides
    mask = torch.ones(npix, dtype=torch.uint8, device=dev)
    plan.cg_start(g1, g2, ninv, mask)
    base = plan.get_tuning()
    entry = _sweep(plan, plan.set_tuning, (base[0], base[1]), (base[2], base[3], base[4]), steps, log, "two-sided")
    # the sky south of z = 0.17: in RING order the pixels from the first ring with z < 0.17 on
    # (rings i = 1 .. 4 Nside - 1; belt rings Nside <= i <= 3 Nside have z = 4/3 - 2 i / (3 Nside)
    # and 4 Nside pixels; the north cap holds 2 Nside (Nside - 1) pixels)
    i0 = next(i for i in range(nside, 3 * nside + 1) if 4.0 / 3.0 - 2.0 * i / (3.0 * nside) < 0.17)
    start = 2 * nside * (nside - 1) + 4 * nside * (i0 - nside)
    south = torch.zeros(npix, dtype=torch.uint8, device=dev)
    south[start:] = 1
    plan.cg_start(g1, g2, ninv, south)
    ww = plan.work_weighted()
    assert ww["synth_one"] > 0, ww
    one = _sweep(plan, plan.set_tuning_one_sided, (entry["syn_variant"], entry["syn_rings"]),
                 (entry["adj_rings"], entry["adj_waves"], entry["adj_chunk"]), steps, log, "one-sided")
    entry["one_sided"] = one
    plan.close()
    return entry


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nside", type=int, required=True)
    ap.add_argument("--lmax", type=int, required=True)
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--out", default=CACHE)
    a = ap.parse_args()
    logf = lambda *x: print(*x, flush=True)  # noqa: E731
    if a.nrhs > 1:
        if a.precision != "fp32":
            raise SystemExit("the batched kernels belong to FP32 plans")
        e = tune_batched(a.nside, a.lmax, a.nrhs, log=logf)
        k = key_batched(a.nside, a.lmax, a.nrhs)
    else:
        e = tune(a.nside, a.lmax, a.precision, a.steps, log=logf)
        k = key(a.nside, a.lmax, a.precision)
    cache = {}
    if os.path.exists(a.out):
        with open(a.out) as f:
            cache = json.load(f)
    cache[k] = e
    with open(a.out, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    print(json.dumps({k: ({kk: vv for kk, vv in v.items() if kk != "sweep"} if isinstance(v, dict) else v)
                      for k, v in e.items() if k != "sweep"}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
