"""GPU parity of the flat-sky variant (the four-step operator with a 2-D FFT) against the flat oracle,
through the C ABI: A, A^H, H and b on grids from 4 x 4 to rows of 8192, the Kaiser-Squires plane
waves, PCG iterates and solves (true residual checked with the oracle's own H), the full-field
closed form, a 4096 x 4096 apply, and argument errors.

Inputs: the flat-field recipe (border and circular holes, Poisson counts of mean 2, N^-1 = n /
sigma_e^2, a Gaussian kappa field with shape noise) and seeded random maps."""
import numpy as np
import pytest

import akra_workloads as wl
from oracle.flat import FlatOracle

pytestmark = pytest.mark.gpu

TOL = 1e-12  # FP64 FFTs of length <= 8192: rounding grows like log2 n


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _plan(nx, ny):
    from paper_2606_06175_amd import FlatPlan
    print("flat plan %d x %d" % (nx, ny), flush=True)
    return FlatPlan(nx, ny, device="cuda:0")


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda", 0))


def _c(p, a, b):
    return a.cpu().numpy() + 1j * b.cpu().numpy()


def _rand(ny, nx, seed):
    g = np.random.default_rng(seed)
    return g.normal(size=(ny, nx)), g.normal(size=(ny, nx))


@pytest.mark.parametrize("nx,ny", [(4, 4), (8, 16), (64, 32), (256, 256), (8192, 4), (4, 8192), (2048, 512)])
def test_synth_and_adjoint_match_oracle(nx, ny):
    o = FlatOracle(nx, ny)
    p = _plan(nx, ny)
    a, b = _rand(ny, nx, nx + 3 * ny)
    g = _c(p, *p.synth(_t(a), _t(b)))
    assert rel(g, o.synth(a + 1j * b)) < TOL
    y = _c(p, *p.adjoint(_t(a), _t(b)))
    assert rel(y, o.adjoint(a + 1j * b)) < TOL


def test_plane_waves():
    n = 256
    p = _plan(n, n)
    i1 = np.arange(n)[None, :]
    i2 = np.arange(n)[:, None]
    m = 5
    along1 = np.cos(2 * np.pi * m * i1 / n) * np.ones((n, 1))
    along2 = np.cos(2 * np.pi * m * i2 / n) * np.ones((1, n))
    diag = np.cos(2 * np.pi * m * (i1 + i2) / n)
    z = np.zeros((n, n))
    g1, g2 = (t.cpu().numpy() for t in p.synth(_t(along1), _t(z)))
    assert np.abs(g1 - along1).max() < 1e-13 and np.abs(g2).max() < 1e-13
    g1, g2 = (t.cpu().numpy() for t in p.synth(_t(along2), _t(z)))
    assert np.abs(g1 + along2).max() < 1e-13 and np.abs(g2).max() < 1e-13
    g1, g2 = (t.cpu().numpy() for t in p.synth(_t(diag), _t(z)))
    assert np.abs(g1).max() < 1e-13 and np.abs(g2 - diag).max() < 1e-13
    g1, g2 = (t.cpu().numpy() for t in p.synth(_t(z), _t(along1)))
    assert np.abs(g2 - along1).max() < 1e-13 and np.abs(g1).max() < 1e-13


@pytest.fixture(scope="module")
def field():
    nx, ny = 128, 64
    f = wl.make_flat(nx, ny, 2)
    o = FlatOracle(nx, ny)
    s = o.synth(f["kappa"])
    m = f["mask"].astype(np.float64)
    g1 = m * (s.real + f["eps1"])
    g2 = m * (s.imag + f["eps2"])
    W = o.weights(f["ninv"], f["mask"])
    lam = o.lambda_eff(f["ninv"], f["mask"])
    P = o.precond(f["ninv"], f["mask"], lam)
    b = o.rhs(g1, g2, W)
    return dict(f=f, o=o, g1=g1, g2=g2, W=W, lam=lam, P=P, b=b, nx=nx, ny=ny)


def test_apply_H_and_rhs_match_oracle(field):
    F, o = field, field["o"]
    p = _plan(F["nx"], F["ny"])
    a, b = _rand(F["ny"], F["nx"], 11)
    y = _c(p, *p.apply_H(_t(F["f"]["ninv"]), _t(F["f"]["mask"]), _t(a), _t(b), F["lam"]))
    assert rel(y, o.apply_H(a + 1j * b, F["W"], F["lam"])) < TOL
    bb = _c(p, *p.rhs(_t(F["g1"]), _t(F["g2"]), _t(F["f"]["ninv"]), _t(F["f"]["mask"])))
    assert rel(bb, F["b"]) < TOL


def test_cg_iterates_and_solve_match_oracle(field):
    F, o = field, field["o"]
    p = _plan(F["nx"], F["ny"])
    args = (_t(F["g1"]), _t(F["g2"]), _t(F["f"]["ninv"]), _t(F["f"]["mask"]))
    kE, kB, info = p.cg_solve(*args, tol=1e-14, maxiter=10, raise_not_converged=False, hist_len=10)
    assert info["status"] == 5 and info["iters"] == 10
    xr, ir = o.cg(F["b"], F["W"], F["lam"], F["P"], tol=1e-14, maxiter=10)
    assert rel(_c(p, kE, kB), xr) < 1e-9
    assert np.allclose(info["hist"], ir["hist"], rtol=1e-8)
    kE, kB, info = p.cg_solve(*args, tol=1e-10, maxiter=2000)
    x = _c(p, kE, kB)
    r = F["b"] - o.apply_H(x, F["W"], F["lam"])
    rt = np.sqrt(o.dot(r, r) / o.dot(F["b"], F["b"]))
    print("iters", info["iters"], "true residual", rt, info["rel_resid_true"], flush=True)
    assert info["status"] == 0 and rt <= 1.05e-10 and abs(rt - info["rel_resid_true"]) < 1e-12
    assert abs(info["lambda_eff"] - F["lam"]) < 1e-12 * F["lam"] and abs(info["precond"] - F["P"]) < 1e-12 * F["P"]
    # a start vector: the solution itself converges at once
    kE2, kB2, info2 = p.cg_solve(*args, tol=1e-9, maxiter=2000, x0=(kE, kB))
    assert info2["iters"] == 0 and rel(_c(p, kE2, kB2), x) < 1e-13


def test_full_field_closed_form():
    n = 512
    p = _plan(n, n)
    o = FlatOracle(n, n)
    w, lam = 3.0, 1e-3
    a, b = _rand(n, n, 13)
    ninv = np.full((n, n), w)
    mask = np.ones((n, n), np.uint8)
    kE, kB, info = p.cg_solve(_t(a), _t(b), _t(ninv), _t(mask), tol=1e-12, maxiter=20, lam=lam)
    le = lam * w
    xf = w * np.conj(o.D) * np.fft.fft2(a + 1j * b, norm="ortho") / (w + le)
    xf[0, 0] = 0
    assert rel(_c(p, kE, kB), np.fft.ifft2(xf, norm="ortho")) < 1e-11
    assert info["iters"] <= 2


def test_full_size_apply_matches_oracle():
    n = 4096
    f = wl.make_flat(n, n, 5)
    o = FlatOracle(n, n)
    W = o.weights(f["ninv"], f["mask"])
    lam = o.lambda_eff(f["ninv"], f["mask"])
    a, b = _rand(n, n, 17)
    p = _plan(n, n)
    y = _c(p, *p.apply_H(_t(f["ninv"]), _t(f["mask"]), _t(a), _t(b), lam))
    print("oracle apply at 4096 x 4096", flush=True)
    assert rel(y, o.apply_H(a + 1j * b, W, lam)) < TOL
    # symmetry <u, H v> = <H u, v>
    hu = _c(p, *p.apply_H(_t(f["ninv"]), _t(f["mask"]), _t(b), _t(a), lam))
    u, v = b + 1j * a, a + 1j * b
    assert abs(o.dot(u, y) - o.dot(hu, v)) < 1e-12 * abs(o.dot(u, y))


def test_flat_errors_and_zero_rhs():
    import torch
    from paper_2606_06175_amd import FlatPlan, akra
    for nx, ny in ((3, 8), (16384, 4), (2, 2), (8, 12)):
        with pytest.raises(akra.AkraError, match="powers of two"):
            FlatPlan(nx, ny, device="cuda:0")
    p = _plan(16, 8)
    z = torch.zeros((8, 16), dtype=torch.float64, device="cuda:0")
    m = torch.ones((8, 16), dtype=torch.uint8, device="cuda:0")
    kE, kB, info = p.cg_solve(z, z, z + 1.0, m, tol=1e-8)
    assert info["iters"] == 0 and float(kE.abs().max()) == 0 and float(kB.abs().max()) == 0
    with pytest.raises(akra.AkraError, match="negative"):
        p.cg_solve(z + 1.0, z, z - 1.0, m)
    with pytest.raises(akra.AkraError, match="NaN"):
        p.cg_solve(z + 1.0, z, z + float("nan"), m)
    with pytest.raises(akra.AkraError, match="after akra_flat_cg_start"):
        p.cg_step(1)
    p.cg_start(z + 1.0, z, z + 1.0, m)
    p.cg_step(3)
    torch.cuda.synchronize()
