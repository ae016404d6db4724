"""Host-side logic of the C ABI that runs without a GPU: argument validation of akra_plan_create and
akra_flat_plan_create (rejected before any HIP call), the error message channel, NULL-plan handling
of every entry point that takes a plan, and the default solver options."""
import ctypes
import os

import pytest

from paper_2606_06175_amd import akra


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(akra.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return akra.lib()


@pytest.mark.parametrize("nside,lmax,nrhs,prec,msg", [
    (0, 2, 1, 0, "nside"),
    (4097, 8192, 1, 0, "nside"),
    (4, 1, 1, 0, "lmax"),
    (4, 17, 1, 0, "lmax"),
    (4, 8, 0, 0, "nrhs"),
    (4, 8, 65, 0, "nrhs"),
    (4, 8, 1, 2, "precision"),
])
def test_plan_create_rejects_bad_arguments(L, nside, lmax, nrhs, prec, msg):
    h = ctypes.c_void_p()
    st = L.akra_plan_create(nside, lmax, nrhs, prec, None, ctypes.byref(h))
    assert st == akra.AKRA_ERR_ARG
    assert not h.value
    assert msg in L.akra_last_error().decode()


def test_null_plan_is_an_argument_error(L):
    assert L.akra_synth2(None, None, None, None, None) == akra.AKRA_ERR_ARG
    assert L.akra_cg_step(None, 1) == akra.AKRA_ERR_ARG
    out = (ctypes.c_int64 * 3)()
    assert L.akra_plan_work(None, out) == akra.AKRA_ERR_ARG
    L.akra_plan_destroy(None)  # a no-op


def test_default_options(L):
    o = akra.CgOpts()
    L.akra_cg_opts_default(ctypes.byref(o))
    assert o.lambda_ == 1e-3 and o.tol == 1e-3 and o.maxiter == 1000
    assert o.use_x0 == 0 and not o.kernel_l and o.reliable_delta == 0.1
    assert not o.resid_hist and o.resid_hist_len == 0
    assert o.mode == 0 and o.stall_iters == 0 and o.check_every == 0
    # the C struct is no larger than the binding's: the defaults leave the bytes past it alone
    n = ctypes.sizeof(akra.CgOpts)
    buf = (ctypes.c_ubyte * (n + 32))(*([0xAB] * (n + 32)))
    L.akra_cg_opts_default(ctypes.cast(buf, ctypes.POINTER(akra.CgOpts)))
    assert list(buf[n:]) == [0xAB] * 32
    assert akra.CgOpts.from_buffer(buf).stall_iters == 0


def test_null_plan_of_the_stage_calls(L):
    # every entry point that takes a plan rejects NULL before touching the device
    n = ctypes.c_int64()
    assert L.akra_unmasked_index(None, None, None, ctypes.byref(n)) == akra.AKRA_ERR_ARG
    assert L.akra_shuffle_shear(None, None, None, None, 0, None, 1, None, None) == akra.AKRA_ERR_ARG
    assert L.akra_alm_spectra(None, None, 1, None, 1, None, 1, None) == akra.AKRA_ERR_ARG
    assert L.akra_noise_work_size(None, 1, ctypes.byref(n)) == akra.AKRA_ERR_ARG
    assert L.akra_noise_spectra(None, 1, None, None, None, None, None, 0, 0, None, None, 0, None, None, None,
                                None) == akra.AKRA_ERR_ARG
    assert L.akra_ang2pix(None, None, None, 1, None) == akra.AKRA_ERR_ARG
    assert L.akra_pixelize_work_size(None, 1, ctypes.byref(n)) == akra.AKRA_ERR_ARG
    assert L.akra_pixelize(None, None, None, None, None, None, 0, 0.7, 0.26, 1.0, None, 0, None, None, None, None,
                           None) == akra.AKRA_ERR_ARG
    assert "plan is NULL" in L.akra_last_error().decode()


@pytest.mark.parametrize("nx,ny", [(3, 8), (8, 3), (2, 8), (16384, 8), (8, 16384), (12, 16), (0, 4)])
def test_flat_plan_rejects_bad_sizes(L, nx, ny):
    h = ctypes.c_void_p()
    assert L.akra_flat_plan_create(nx, ny, None, ctypes.byref(h)) == akra.AKRA_ERR_ARG
    assert not h.value
    assert "powers of two" in L.akra_last_error().decode()


def test_null_flat_plan(L):
    assert L.akra_flat_synth(None, None, None, None, None) == akra.AKRA_ERR_ARG
    assert L.akra_flat_adjoint(None, None, None, None, None) == akra.AKRA_ERR_ARG
    assert L.akra_flat_apply_H(None, None, None, 0.0, None, None, None, None) == akra.AKRA_ERR_ARG
    assert L.akra_flat_rhs(None, None, None, None, None, None, None) == akra.AKRA_ERR_ARG
    assert L.akra_flat_cg_solve(None, None, None, None, None, None, None, None, None) == akra.AKRA_ERR_ARG
    assert L.akra_flat_cg_start(None, None, None, None, None, 1e-3) == akra.AKRA_ERR_ARG
    assert L.akra_flat_cg_step(None, 1) == akra.AKRA_ERR_ARG
    assert L.akra_flat_plan_device_bytes(None) == 0
    L.akra_flat_plan_destroy(None)  # a no-op
    assert L.akra_flat_plan_create(8, 8, None, None) == akra.AKRA_ERR_ARG


def test_noalloc_spectra_rejects_bad_arguments_before_any_hip_call(L):
    # the allocation-free spectrum call checks its arguments on the host first
    assert L.akra_alm_spectra_noalloc(4097, None, 0, None, 0, None, 1, None, None) == akra.AKRA_ERR_ARG
    assert "4096" in L.akra_last_error().decode()
    assert L.akra_alm_spectra_noalloc(-1, None, 0, None, 0, None, 1, None, None) == akra.AKRA_ERR_ARG
    assert L.akra_alm_spectra_noalloc(8, None, 0, None, 0, None, -1, None, None) == akra.AKRA_ERR_ARG
    assert L.akra_alm_spectra_noalloc(8, None, 0, None, 0, None, 0, None, None) == akra.AKRA_OK
    assert L.akra_alm_spectra_noalloc(8, None, 1, None, 1, None, 1, None, None) == akra.AKRA_ERR_ARG
    assert "null" in L.akra_last_error().decode()
    x = ctypes.c_void_p(16)
    pairs = (ctypes.c_int32 * 2)(0, 1)
    assert L.akra_alm_spectra_noalloc(8, x, 1, x, 1, pairs, 1, x, None) == akra.AKRA_ERR_ARG
    assert "out of range" in L.akra_last_error().decode()


def test_fma_rate_rejects_bad_arguments_before_any_hip_call(L):
    v = ctypes.c_double()
    assert L.akra_fma_rate(2, ctypes.byref(v)) == akra.AKRA_ERR_ARG
    assert "precision" in L.akra_last_error().decode()
    assert L.akra_fma_rate(0, None) == akra.AKRA_ERR_ARG


def test_mfma_rate_rejects_bad_arguments_before_any_hip_call(L):
    v = ctypes.c_double()
    for chains, valu, waves in ((3, 0, 1), (4, 2, 1), (4, 0, 3), (0, 0, 1)):
        assert L.akra_mfma_rate(chains, valu, waves, ctypes.byref(v)) == akra.AKRA_ERR_ARG
    assert "chains" in L.akra_last_error().decode()
    assert L.akra_mfma_rate(4, 0, 2, None) == akra.AKRA_ERR_ARG
