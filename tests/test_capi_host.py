"""Host-side logic of the C ABI that runs without a GPU: argument validation of akra_plan_create
(rejected before any HIP call), the error message channel, NULL-plan handling and the default
solver options."""
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
