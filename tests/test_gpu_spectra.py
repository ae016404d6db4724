"""GPU parity of the shape-noise realisation and spectrum stage (Sec. IV power spectra) against the
oracle, through the C ABI: the unmasked-pixel list and the shuffle bit for bit, spectra of coefficient
pairs to FP64 rounding, and the whole realisation pipeline (shuffle, solve, spectra, moments) to the
solve tolerance, for one shear set and for split halves, on FP64 plans and on batched FP32 plans with
a partial last group.

Inputs: the C1 workload (HEALPix Nside 32, lmax 64, one cap with f_sky 0.1, Poisson mean 5), seeded
random masks at sizes that leave a ragged compaction tile, and seeded random coefficients."""
import ctypes

import numpy as np
import pytest

import akra_workloads as wl
from oracle.core import Oracle
from oracle.geometry import healpix_rings
from oracle import spectra as sp

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.ravel(a)
    b = np.ravel(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _plan(nside, lmax, prec="fp64", nrhs=1):
    from paper_2606_06175_amd import Plan
    print("plan nside=%d lmax=%d %s nrhs=%d" % (nside, lmax, prec, nrhs), flush=True)
    return Plan(nside, lmax, nrhs=nrhs, precision=prec, device="cuda:0")


@pytest.mark.parametrize("nside,frac", [(13, 0.3), (40, 0.1), (40, 0.0), (40, 1.0), (32, 0.5)])
def test_unmasked_index_and_shuffle_bit_exact(nside, frac):
    import torch
    dev = torch.device("cuda", 0)
    npix = 12 * nside * nside
    g = np.random.default_rng(nside * 7 + int(100 * frac))
    mask = (g.random(npix) < frac).astype(np.uint8)
    g1, g2 = g.normal(size=npix), g.normal(size=npix)
    p = _plan(nside, 2 * nside)
    idx = p.unmasked_index(torch.from_numpy(mask).to(dev))
    u = sp.unmasked_index(mask)
    assert np.array_equal(idx.cpu().numpy(), u)
    n_obs = u.size
    perms = wl.shuffle_perms(n_obs, 3, nside)
    perms[0] = np.arange(n_obs)
    o1, o2 = p.shuffle_shear(torch.from_numpy(g1).to(dev), torch.from_numpy(g2).to(dev), idx,
                             torch.from_numpy(perms).to(dev))
    o1, o2 = o1.cpu().numpy(), o2.cpu().numpy()
    for k in range(3):
        r1, r2 = sp.shuffle_shear(g1, g2, mask, perms[k])
        assert np.array_equal(o1[k], r1) and np.array_equal(o2[k], r2), k


def test_shuffle_rejects_out_of_range_entries():
    import torch
    from paper_2606_06175_amd import akra
    dev = torch.device("cuda", 0)
    p = _plan(16, 32)
    mask = np.zeros(p.npix, np.uint8)
    mask[::3] = 1
    idx = p.unmasked_index(torch.from_numpy(mask).to(dev))
    n_obs = idx.numel()
    g1 = torch.ones(p.npix, dtype=torch.float64, device=dev)
    bad = torch.from_numpy(np.arange(n_obs, dtype=np.int32)[None, :].copy()).to(dev)
    bad[0, 5] = n_obs
    with pytest.raises(akra.AkraError, match="perm holds an entry"):
        p.shuffle_shear(g1, g1.clone(), idx, bad)
    bad[0, 5] = -1
    with pytest.raises(akra.AkraError, match="perm holds an entry"):
        p.shuffle_shear(g1, g1.clone(), idx, bad)
    # a good call afterwards is unaffected by the earlier flag
    good = torch.from_numpy(np.arange(n_obs, dtype=np.int32)[None, :].copy()).to(dev)
    o1, _ = p.shuffle_shear(g1, g1.clone(), idx, good)
    assert np.array_equal(o1[0].cpu().numpy(), mask.astype(np.float64))
    # outputs may not overlap the inputs
    L = akra.lib()
    st = L.akra_shuffle_shear(p._h, g1.data_ptr(), g1.data_ptr(), idx.data_ptr(), n_obs, good.data_ptr(), 1,
                              g1.data_ptr(), o1.data_ptr())
    assert st == akra.AKRA_ERR_ARG


@pytest.mark.parametrize("nside,lmax", [(96, 300), (32, 64), (4, 2)])
def test_alm_spectra_match_oracle(nside, lmax):
    import torch
    dev = torch.device("cuda", 0)
    n = 4
    x = np.stack([wl.random_alm(lmax, 900 + k, 0) for k in range(n)])
    x[1] *= np.exp(1j * 0.3)
    p = _plan(nside, lmax)
    tx = torch.from_numpy(x).to(dev)
    pairs = [(i, j) for i in range(n) for j in range(n) if i <= j][:11]  # more than one launch of 8
    cl = p.alm_spectra(tx, tx, pairs).cpu().numpy()
    for q, (i, j) in enumerate(pairs):
        ref = sp.spectrum(x[i], x[j], lmax)
        scale = np.sqrt(sp.spectrum(x[i], x[i], lmax) * sp.spectrum(x[j], x[j], lmax))
        assert np.all(np.abs(cl[q] - ref) <= 1e-13 * scale + 1e-300), (i, j)
        assert cl[q][0] == 0 and cl[q][1] == 0
    # repeat calls agree bit for bit
    assert np.array_equal(p.alm_spectra(tx, tx, pairs).cpu().numpy(), cl)


def test_alm_spectra_argument_errors():
    import torch
    from paper_2606_06175_amd import akra
    dev = torch.device("cuda", 0)
    p = _plan(8, 16)
    x = torch.zeros((2, p.nalm), dtype=torch.complex128, device=dev)
    with pytest.raises(akra.AkraError, match="out of range"):
        p.alm_spectra(x, x, [(0, 2)])
    assert p.alm_spectra(x, x, np.zeros((0, 2), np.int32)).shape == (0, 17)
    # misaligned coefficients through the C ABI
    cl = torch.empty((1, 17), dtype=torch.float64, device=dev)
    pr = np.zeros(2, np.int32)
    st = akra.lib().akra_alm_spectra(p._h, x.data_ptr() + 8, 1, x.data_ptr(), 1, pr.ctypes.data, 1, cl.data_ptr())
    assert st == akra.AKRA_ERR_ARG and "aligned" in akra.lib().akra_last_error().decode()


@pytest.fixture(scope="module")
def c1():
    """C1 shear (signal + noise), two split halves, and the oracle's realisation spectra."""
    cfg = wl.make_config("C1")
    lmax, nside = cfg["lmax"], cfg["nside"]
    o = Oracle(lmax, healpix_rings(nside))
    K = o.kernel()[o.l_of]
    s1, s2 = o.synth(K * cfg["kappa"][0], np.zeros(o.nalm, np.complex128))
    mask = cfg["mask"]
    m = mask.astype(np.float64)
    g1, g2 = m * (s1 + cfg["eps1"][0]), m * (s2 + cfg["eps2"][0])
    ninv = cfg["ninv"][0]
    hv = wl.split_halves(cfg, 1)
    h1 = np.stack([m * (s1 + hv["eps1"][q]) for q in range(2)])
    h2 = np.stack([m * (s2 + hv["eps2"][q]) for q in range(2)])
    n_obs = int(mask.sum())
    perm1 = wl.shuffle_perms(n_obs, 3, 1)
    perm2 = np.stack([wl.shuffle_perms(n_obs, 2, 1, half=q) for q in range(2)])
    print("oracle: 3 joint realisations, 2 paired E realisations", flush=True)
    ref_joint = sp.noise_spectra(o, g1, g2, ninv, mask, perm1, mode=0, tol=1e-12)
    ref_pair = sp.noise_spectra(o, h1, h2, hv["ninv"], mask, perm2, mode=1, tol=1e-12)
    return dict(cfg=cfg, o=o, g1=g1, g2=g2, ninv=ninv, mask=mask, h1=h1, h2=h2, hninv=hv["ninv"], perm1=perm1,
                perm2=perm2, ref_joint=ref_joint, ref_pair=ref_pair)


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda", 0))


def _check_moments(cl, mean, std, ref, tol):
    rm, rs = sp.moments(ref)
    assert rel(mean, rm) < 1e4 * tol
    # |std(a) - std(b)| <= sqrt(sum_k (a_k - b_k)^2 / (n - 1)) elementwise (triangle inequality on the
    # deviations from the mean), so the scatter differs from the oracle's by at most what the
    # spectra themselves differ
    n = cl.shape[0]
    bound = np.sqrt(np.sum((cl - ref) ** 2, axis=0) / max(n - 1, 1))
    assert np.all(np.abs(std - rs) <= bound * (1 + 1e-9) + 1e-15 * np.abs(rm).max())
    m2, s2 = sp.moments(cl)
    assert np.allclose(mean, m2, rtol=1e-12, atol=0) and np.allclose(std, s2, rtol=1e-10, atol=1e-300)


@pytest.mark.parametrize("prec,nrhs,tol", [("fp64", 1, 1e-11), ("fp32", 2, 1e-8), ("fp64", 2, 1e-11)])
def test_noise_spectra_joint_match_oracle(c1, prec, nrhs, tol):
    # 3 realisations in groups of nrhs: with nrhs = 2 the last group is padded with zero shear
    p = _plan(c1["cfg"]["nside"], c1["cfg"]["lmax"], prec, nrhs)
    cl, mean, std, info = p.noise_spectra(_t(c1["g1"]), _t(c1["g2"]), _t(c1["ninv"]), _t(c1["mask"]),
                                          _t(c1["perm1"]), tol=tol, maxiter=4000, mode="joint")
    print(prec, nrhs, "iters", info["iters"], "true residual", info["rel_resid_true"], flush=True)
    assert info["status"] == 0 and info["rel_resid_true"] <= 1.05 * tol
    cl, mean, std = cl.cpu().numpy(), mean.cpu().numpy(), std.cpu().numpy()
    ref = c1["ref_joint"]
    assert cl.shape == ref.shape == (3, 3, c1["cfg"]["lmax"] + 1)
    for k in range(3):
        for s in range(3):
            assert rel(cl[k, s], ref[k, s]) < 1e4 * tol, (k, s)
    _check_moments(cl, mean, std, ref, tol)


@pytest.mark.parametrize("prec,nrhs,tol", [("fp64", 1, 1e-11), ("fp32", 4, 1e-8)])
def test_noise_spectra_split_halves_match_oracle(c1, prec, nrhs, tol):
    p = _plan(c1["cfg"]["nside"], c1["cfg"]["lmax"], prec, nrhs)
    cl, mean, std, info = p.noise_spectra(_t(c1["h1"]), _t(c1["h2"]), _t(c1["hninv"]), _t(c1["mask"]),
                                          _t(c1["perm2"]), tol=tol, maxiter=4000, mode="E")
    assert info["status"] == 0 and info["rel_resid_true"] <= 1.05 * tol
    cl = cl.cpu().numpy()
    ref = c1["ref_pair"]
    assert cl.shape == ref.shape == (2, 1, c1["cfg"]["lmax"] + 1)
    for k in range(2):
        assert rel(cl[k, 0], ref[k, 0]) < 1e4 * tol, k
    _check_moments(cl, mean.cpu().numpy(), std.cpu().numpy(), ref, tol)


def test_noise_spectra_identity_equals_direct_solve(c1):
    # identity permutations: the pipeline's EE spectrum is that of the plain E-mode solve
    p = _plan(c1["cfg"]["nside"], c1["cfg"]["lmax"])
    n_obs = int(c1["mask"].sum())
    perm = np.stack([np.arange(n_obs, dtype=np.int32)] * 2)
    cl, mean, std, _ = p.noise_spectra(_t(c1["g1"]), _t(c1["g2"]), _t(c1["ninv"]), _t(c1["mask"]), _t(perm),
                                       tol=1e-11, maxiter=4000, mode="E")
    xE, _, _ = p.cg_solve(_t(c1["g1"]), _t(c1["g2"]), _t(c1["ninv"]), _t(c1["mask"]), tol=1e-11, maxiter=4000,
                          mode="E")
    direct = p.alm_spectra(xE, xE, [(0, 0)]).cpu().numpy()[0]
    cl = cl.cpu().numpy()
    assert np.array_equal(cl[0, 0], cl[1, 0]) and np.array_equal(cl[0, 0], direct)
    assert np.all(std.cpu().numpy() == 0)


def test_noise_spectra_argument_errors(c1):
    import torch
    from paper_2606_06175_amd import akra
    p = _plan(c1["cfg"]["nside"], c1["cfg"]["lmax"], "fp32", 3)
    t = dict(g1=_t(c1["g1"]), g2=_t(c1["g2"]), ninv=_t(c1["ninv"]), mask=_t(c1["mask"]))
    n_obs = int(c1["mask"].sum())
    # split halves need an even batch
    with pytest.raises(akra.AkraError, match="even nrhs"):
        p.noise_spectra(_t(c1["h1"]), _t(c1["h2"]), _t(c1["hninv"]), t["mask"], _t(c1["perm2"]))
    # n_obs must match the mask
    short = _t(np.zeros((1, n_obs - 1), np.int32))
    with pytest.raises(akra.AkraError, match="differs from the unmasked"):
        p.noise_spectra(t["g1"], t["g2"], t["ninv"], t["mask"], short)
    # a perm entry out of range
    bad = np.stack([np.arange(n_obs, dtype=np.int32)])
    bad[0, 3] = n_obs + 7
    with pytest.raises(akra.AkraError, match="perm holds an entry"):
        p.noise_spectra(t["g1"], t["g2"], t["ninv"], t["mask"], _t(bad))
    # too small a workspace
    w = torch.empty(p.noise_work_bytes(1) - 1, dtype=torch.uint8, device=t["g1"].device)
    with pytest.raises(akra.AkraError, match="workspace too small"):
        p.noise_spectra(t["g1"], t["g2"], t["ninv"], t["mask"], _t(bad), work=w)
    # a workspace that is not 256-byte aligned
    w = torch.empty(p.noise_work_bytes(1) + 256, dtype=torch.uint8, device=t["g1"].device)
    with pytest.raises(akra.AkraError, match="aligned"):
        p.noise_spectra(t["g1"], t["g2"], t["ninv"], t["mask"], _t(np.stack([np.arange(n_obs, dtype=np.int32)])),
                        work=w[8:])
    # no realisations: nothing solved, zero moments
    cl, mean, std, info = p.noise_spectra(t["g1"], t["g2"], t["ninv"], t["mask"], _t(np.zeros((0, n_obs), np.int32)))
    assert cl.shape[0] == 0 and info["iters"] == 0
    assert float(mean.abs().max()) == 0 and float(std.abs().max()) == 0
    # invalid nset through the C ABI
    o, keep = p._opts(1e-3, 10, 1e-3, None, None, 0.1, 0)
    st = akra.lib().akra_noise_spectra(p._h, 3, t["g1"].data_ptr(), t["g2"].data_ptr(), t["ninv"].data_ptr(),
                                       t["mask"].data_ptr(), None, 0, 0, ctypes.byref(o), None, 0, None, None, None,
                                       None)
    assert st == akra.AKRA_ERR_ARG
