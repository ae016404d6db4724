"""ctypes binding of libakra (include/akra.h) on torch device tensors.

Argument marshalling only: every step of the operator and the solver runs in libakra's HIP
kernels.  There is no fallback: without the built library every call raises.

Tensors: alm are complex128 with n_alm = (lmax+1)(lmax+2)/2 entries (m >= 0, healpy order)
and an optional leading [nrhs] dimension; maps are float64 [.., Npix] in HEALPix RING order;
the mask is uint8 [Npix].  Calls run on the plan's HIP stream, which defaults to torch's
current stream, so they are ordered with surrounding torch work.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# AKRA_LIBRARY names another build of the same library (the sanitizer-instrumented one in tests)
LIB_PATH = os.environ.get("AKRA_LIBRARY") or os.path.join(_HERE, "libakra.so")
_lib = None

AKRA_OK, AKRA_ERR_ARG, AKRA_ERR_ALLOC, AKRA_ERR_HIP, AKRA_ERR_NUMERIC, AKRA_NOT_CONVERGED, AKRA_STAGNATED = range(7)
STAGES = ("prologue", "leg_synth", "ring", "leg_adj", "epilogue", "cg_vec")
STATUS_NAMES = {0: "AKRA_OK", 1: "AKRA_ERR_ARG", 2: "AKRA_ERR_ALLOC", 3: "AKRA_ERR_HIP", 4: "AKRA_ERR_NUMERIC",
                5: "AKRA_NOT_CONVERGED", 6: "AKRA_STAGNATED"}
PRECISIONS = {"fp64": 0, "fp32": 1}


class AkraError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class CgOpts(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("tol", ctypes.c_double), ("maxiter", ctypes.c_int),
                ("use_x0", ctypes.c_int), ("kernel_l", ctypes.POINTER(ctypes.c_double)),
                ("reliable_delta", ctypes.c_double), ("resid_hist", ctypes.POINTER(ctypes.c_double)),
                ("resid_hist_len", ctypes.c_int), ("mode", ctypes.c_int), ("stall_iters", ctypes.c_int),
                ("check_every", ctypes.c_int)]


# unknowns of a solve (akra_mode): joint (kappa_E, kappa_B), the E block only, the B block only
MODES = {"joint": 0, "E": 1, "B": 2}


class CgInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("fp64_applies", ctypes.c_int), ("rel_resid", ctypes.c_double),
                ("rel_resid_true", ctypes.c_double), ("lambda_eff", ctypes.c_double), ("precond", ctypes.c_double),
                ("ms_total", ctypes.c_double), ("status", ctypes.c_int)]


def lib():
    """Load libakra.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libakra.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, dp, i64 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int64
    L.akra_plan_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, ctypes.POINTER(vp)]
    L.akra_plan_destroy.argtypes = [vp]
    L.akra_plan_destroy.restype = None
    L.akra_last_error.restype = ctypes.c_char_p
    L.akra_plan_device_bytes.argtypes = [vp]
    L.akra_plan_device_bytes.restype = i64
    L.akra_cg_opts_default.argtypes = [ctypes.POINTER(CgOpts)]
    L.akra_cg_opts_default.restype = None
    L.akra_synth2.argtypes = [vp, vp, vp, vp, vp]
    L.akra_adjoint2.argtypes = [vp, vp, vp, vp, vp]
    L.akra_apply_H.argtypes = [vp, vp, vp, dp, ctypes.c_double, vp, vp, vp, vp]
    L.akra_rhs.argtypes = [vp, vp, vp, vp, vp, dp, vp, vp]
    L.akra_cg_solve.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(CgOpts), vp, vp, ctypes.POINTER(CgInfo)]
    L.akra_cg_solve_b.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(CgOpts), vp, vp, ctypes.POINTER(CgInfo)]
    L.akra_cg_start.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(CgOpts)]
    L.akra_cg_step.argtypes = [vp, ctypes.c_int]
    L.akra_cg_state.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_int), vp, vp]
    L.akra_plan_set_timing.argtypes = [vp, ctypes.c_int]
    L.akra_plan_set_graph.argtypes = [vp, ctypes.c_int]
    L.akra_plan_set_tuning.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.akra_plan_get_tuning.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    L.akra_plan_set_tuning_one_sided.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                 ctypes.c_int]
    L.akra_plan_get_tuning_one_sided.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    L.akra_fma_rate.argtypes = [ctypes.c_int, dp]
    L.akra_mfma_rate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
    L.akra_plan_set_tuning_batched.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    L.akra_plan_get_tuning_batched.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    L.akra_plan_work.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    L.akra_plan_work_batched.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    L.akra_plan_work_weighted.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    L.akra_plan_set_skip_unweighted.argtypes = [vp, ctypes.c_int]
    L.akra_cg_solve_vjp.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(CgOpts), vp, vp, vp, vp, vp, vp, vp,
                                    ctypes.POINTER(CgInfo)]
    L.akra_cg_solve_cond_b.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(CgOpts), vp, vp, ctypes.POINTER(CgInfo)]
    L.akra_set_ring_whole_maxm.argtypes = [ctypes.c_int]
    L.akra_set_ring_register_engine.argtypes = [ctypes.c_int]
    L.akra_plan_stage_times.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_int)]
    L.akra_unmasked_index.argtypes = [vp, vp, vp, ctypes.POINTER(i64)]
    L.akra_shuffle_shear.argtypes = [vp, vp, vp, vp, i64, vp, ctypes.c_int, vp, vp]
    L.akra_alm_spectra.argtypes = [vp, vp, ctypes.c_int, vp, ctypes.c_int, vp, ctypes.c_int, vp]
    L.akra_noise_work_size.argtypes = [vp, ctypes.c_int, ctypes.POINTER(i64)]
    L.akra_alm_spectra_noalloc.argtypes = [ctypes.c_int, vp, ctypes.c_int, vp, ctypes.c_int, vp, ctypes.c_int, vp,
                                           vp]
    L.akra_ang2pix.argtypes = [vp, vp, vp, i64, vp]
    L.akra_flat_plan_create.argtypes = [ctypes.c_int, ctypes.c_int, vp, ctypes.POINTER(vp)]
    L.akra_flat_plan_destroy.argtypes = [vp]
    L.akra_flat_plan_destroy.restype = None
    L.akra_flat_plan_device_bytes.argtypes = [vp]
    L.akra_flat_plan_device_bytes.restype = i64
    L.akra_flat_synth.argtypes = [vp, vp, vp, vp, vp]
    L.akra_flat_adjoint.argtypes = [vp, vp, vp, vp, vp]
    L.akra_flat_apply_H.argtypes = [vp, vp, vp, ctypes.c_double, vp, vp, vp, vp]
    L.akra_flat_rhs.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.akra_flat_cg_solve.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(CgOpts), vp, vp, ctypes.POINTER(CgInfo)]
    L.akra_flat_cg_start.argtypes = [vp, vp, vp, vp, vp, ctypes.c_double]
    L.akra_flat_cg_step.argtypes = [vp, ctypes.c_int]
    L.akra_pixelize_work_size.argtypes = [vp, i64, ctypes.POINTER(i64)]
    L.akra_pixelize.argtypes = [vp, vp, vp, vp, vp, vp, i64, ctypes.c_double, ctypes.c_double, ctypes.c_double, vp,
                                i64, vp, vp, vp, vp, vp]
    L.akra_noise_spectra.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp, vp, i64, ctypes.c_int,
                                     ctypes.POINTER(CgOpts), vp, i64, vp, vp, vp, ctypes.POINTER(CgInfo)]
    for f in ("akra_plan_create", "akra_synth2", "akra_adjoint2", "akra_apply_H", "akra_rhs", "akra_cg_solve",
              "akra_cg_solve_b", "akra_cg_start", "akra_cg_step", "akra_cg_state", "akra_plan_set_timing",
              "akra_plan_stage_times", "akra_plan_set_tuning", "akra_plan_get_tuning", "akra_plan_work",
              "akra_plan_set_tuning_batched", "akra_plan_get_tuning_batched",
              "akra_plan_work_batched", "akra_plan_work_weighted", "akra_plan_set_skip_unweighted",
              "akra_plan_set_tuning_one_sided", "akra_plan_get_tuning_one_sided", "akra_fma_rate", "akra_mfma_rate",
              "akra_cg_solve_vjp", "akra_cg_solve_cond_b", "akra_set_ring_whole_maxm", "akra_set_ring_register_engine", "akra_unmasked_index",
              "akra_shuffle_shear", "akra_alm_spectra", "akra_alm_spectra_noalloc", "akra_noise_work_size", "akra_noise_spectra", "akra_ang2pix",
              "akra_pixelize_work_size", "akra_pixelize", "akra_flat_plan_create", "akra_flat_synth",
              "akra_flat_adjoint", "akra_flat_apply_H", "akra_flat_rhs", "akra_flat_cg_solve", "akra_flat_cg_start",
              "akra_flat_cg_step", "akra_plan_set_graph"):
        getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def _check(st):
    if st != AKRA_OK:
        raise AkraError(st, lib().akra_last_error().decode())


def set_ring_whole_maxm(maxm):
    """Ring-stage kernel choice of plans created afterwards (see akra_set_ring_whole_maxm)."""
    _check(lib().akra_set_ring_whole_maxm(int(maxm)))


def fma_rate(precision="fp64"):
    """Sustained plain FMA rate of the current device in TFLOP/s (akra_fma_rate)."""
    v = ctypes.c_double()
    _check(lib().akra_fma_rate(PRECISIONS[precision], ctypes.byref(v)))
    return v.value


def mfma_rate(chains=4, valu=0, waves=2):
    """Sustained v_mfma_f32_32x32x2_f32 rate in TFLOP/s with valu pairs of FP32 FMAs between the
    products (akra_mfma_rate)."""
    v = ctypes.c_double()
    _check(lib().akra_mfma_rate(int(chains), int(valu), int(waves), ctypes.byref(v)))
    return v.value


def set_ring_register_engine(on):
    """Register engine of the ring stage for plans created afterwards (see akra_set_ring_register_engine)."""
    _check(lib().akra_set_ring_register_engine(1 if on else 0))


def alm_size(lmax):
    return (lmax + 1) * (lmax + 2) // 2


def _kernel_arg(kernel):
    if kernel is None:
        return None, None
    import numpy as np
    k = np.ascontiguousarray(kernel, dtype=np.float64)
    return k, k.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


NOALLOC_LMAX_MAX = 4096  # AKRA_NOALLOC_LMAX_MAX


def alm_spectra_noalloc(x, y, pairs, lmax, out=None, stream=None):
    """C_l of coefficient pairs without a plan and without device allocation by the library
    (akra_alm_spectra_noalloc): x [nx, n_alm], y [ny, n_alm] complex128 on one device, pairs a list of
    (i, j); returns (or fills) float64 [npairs, lmax + 1].  Calls overlapping on one GPU race (they
    share the library's static scratch)."""
    import numpy as np
    lmax = int(lmax)
    nalm = alm_size(lmax)
    if x.dtype != torch.complex128 or y.dtype != torch.complex128 or x.device != y.device:
        raise TypeError("x and y must be complex128 on one device")
    if x.shape[-1] != nalm or y.shape[-1] != nalm:
        raise ValueError("coefficient arrays must have n_alm = %d entries per row" % nalm)
    x, y = x.contiguous(), y.contiguous()
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    if out is None:
        out = torch.empty((len(pr), lmax + 1), dtype=torch.float64, device=x.device)
    elif out.dtype != torch.float64 or out.device != x.device or out.numel() != len(pr) * (lmax + 1) \
            or not out.is_contiguous():
        raise ValueError("out must be contiguous float64 [npairs, lmax + 1] on the coefficients' device")
    with torch.cuda.device(x.device):
        s = stream if stream is not None else torch.cuda.current_stream(x.device)
        _check(lib().akra_alm_spectra_noalloc(lmax, x.data_ptr(), x.numel() // nalm, y.data_ptr(),
                                               y.numel() // nalm, pr.ctypes.data, len(pr), out.data_ptr(),
                                               ctypes.c_void_p(s.cuda_stream)))
    return out


class Plan:
    """A libakra plan: HEALPix nside, band limit lmax, nrhs right-hand sides, FP64 or FP32 transforms."""

    def __init__(self, nside, lmax, nrhs=1, precision="fp64", device=None, stream=None, tuned=True):
        """tuned: apply the launch shapes cached by the autotuner (tune.py) for this size, if any."""
        L = lib()
        self.nside, self.lmax, self.nrhs = int(nside), int(lmax), int(nrhs)
        self.precision = precision
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.npix = 12 * self.nside * self.nside
        self.nalm = alm_size(self.lmax)
        with torch.cuda.device(self.device):
            s = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.stream = s
            h = ctypes.c_void_p()
            _check(L.akra_plan_create(self.nside, self.lmax, self.nrhs, PRECISIONS[precision],
                                      ctypes.c_void_p(s.cuda_stream), ctypes.byref(h)))
        self._h = h
        if tuned:
            from .tune import lookup, lookup_batched
            e = lookup(self.nside, self.lmax, precision)
            if e:
                self.set_tuning(e["syn_variant"], e["syn_rings"], e["adj_rings"], e["adj_waves"],
                                e.get("adj_chunk", 8))
                o = e.get("one_sided", e)
                self.set_tuning_one_sided(o["syn_variant"], o["syn_rings"], o["adj_rings"], o["adj_waves"],
                                          o.get("adj_chunk", 8))
            if precision == "fp32" and self.nrhs > 1:
                b = lookup_batched(self.nside, self.lmax, self.nrhs)
                if b:
                    self.set_tuning_batched(b["syn_waves"], b["adj_waves"])

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().akra_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def device_bytes(self):
        return lib().akra_plan_device_bytes(self._h)

    # -- helpers ------------------------------------------------------------------------------
    def _alm(self, a, name):
        if a.dtype != torch.complex128 or a.device != self.device:
            raise TypeError("%s must be complex128 on %s" % (name, self.device))
        if a.shape[-1] != self.nalm or a.numel() != self.nrhs * self.nalm:
            raise ValueError("%s must hold nrhs x n_alm = %d x %d entries" % (name, self.nrhs, self.nalm))
        return a.contiguous()

    def _map(self, g, name, dtype=torch.float64, per_rhs=True):
        if g.dtype != dtype or g.device != self.device:
            raise TypeError("%s must be %s on %s" % (name, dtype, self.device))
        n = (self.nrhs if per_rhs else 1) * self.npix
        if g.numel() != n:
            raise ValueError("%s must hold %d entries" % (name, n))
        return g.contiguous()

    def _alm_out(self):
        shape = (self.nalm,) if self.nrhs == 1 else (self.nrhs, self.nalm)
        return torch.empty(shape, dtype=torch.complex128, device=self.device)

    def _map_out(self):
        shape = (self.npix,) if self.nrhs == 1 else (self.nrhs, self.npix)
        return torch.empty(shape, dtype=torch.float64, device=self.device)

    # -- operator -----------------------------------------------------------------------------
    def synth2(self, almE, almB):
        almE, almB = self._alm(almE, "almE"), self._alm(almB, "almB")
        g1, g2 = self._map_out(), self._map_out()
        with torch.cuda.device(self.device):
            _check(lib().akra_synth2(self._h, almE.data_ptr(), almB.data_ptr(), g1.data_ptr(), g2.data_ptr()))
        return g1, g2

    def adjoint2(self, g1, g2):
        g1, g2 = self._map(g1, "g1"), self._map(g2, "g2")
        aE, aB = self._alm_out(), self._alm_out()
        with torch.cuda.device(self.device):
            _check(lib().akra_adjoint2(self._h, g1.data_ptr(), g2.data_ptr(), aE.data_ptr(), aB.data_ptr()))
        return aE, aB

    def apply_H(self, ninv, mask, xE, xB, lambda_eff, kernel=None):
        ninv = self._map(ninv, "ninv")
        mask = self._map(mask, "mask", torch.uint8, per_rhs=False)
        xE, xB = self._alm(xE, "xE"), self._alm(xB, "xB")
        yE, yB = self._alm_out(), self._alm_out()
        keep, kp = _kernel_arg(kernel)
        with torch.cuda.device(self.device):
            _check(lib().akra_apply_H(self._h, ninv.data_ptr(), mask.data_ptr(), kp, float(lambda_eff),
                                      xE.data_ptr(), xB.data_ptr(), yE.data_ptr(), yB.data_ptr()))
        return yE, yB

    def rhs(self, g1, g2, ninv, mask, kernel=None):
        g1, g2 = self._map(g1, "g1"), self._map(g2, "g2")
        ninv = self._map(ninv, "ninv")
        mask = self._map(mask, "mask", torch.uint8, per_rhs=False)
        bE, bB = self._alm_out(), self._alm_out()
        keep, kp = _kernel_arg(kernel)
        with torch.cuda.device(self.device):
            _check(lib().akra_rhs(self._h, g1.data_ptr(), g2.data_ptr(), ninv.data_ptr(), mask.data_ptr(), kp,
                                  bE.data_ptr(), bB.data_ptr()))
        return bE, bB

    def _opts(self, tol, maxiter, lam, x0, kernel, reliable_delta, hist_len, mode="joint", stall_iters=0,
              check_every=1):
        o = CgOpts()
        lib().akra_cg_opts_default(ctypes.byref(o))
        o.lambda_, o.tol, o.maxiter = float(lam), float(tol), int(maxiter)
        o.stall_iters = int(stall_iters)
        o.check_every = int(check_every)
        if mode not in MODES:
            raise ValueError("mode must be one of %s" % sorted(MODES))
        o.mode = MODES[mode]
        o.use_x0 = 1 if x0 is not None else 0
        o.reliable_delta = float(reliable_delta)
        keep = []
        if kernel is not None:
            k, kp = _kernel_arg(kernel)
            keep.append(k)
            o.kernel_l = kp
        if hist_len:
            import numpy as np
            h = np.zeros(hist_len)
            keep.append(h)
            o.resid_hist = h.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            o.resid_hist_len = hist_len
        return o, keep

    @staticmethod
    def _info(inf, keep, hist_len):
        d = {k: getattr(inf, k) for k, _ in CgInfo._fields_}
        if hist_len:
            d["hist"] = keep[-1][: inf.iters].copy()
        return d

    def cg_solve(self, g1, g2, ninv, mask, tol=1e-3, maxiter=1000, lam=1e-3, x0=None, kernel=None,
                 reliable_delta=0.1, hist_len=0, raise_not_converged=True, mode="joint", stall_iters=0, check_every=1):
        """Regularised ML estimate (kappa_E, kappa_B).  mode "joint" solves the full E/B system, "E"
        the E block alone (kappa_B returned as zero), "B" the B block alone.  stall_iters > 0 stops
        with AKRA_STAGNATED once the residual has reached no new minimum for that many tests;
        check_every > 1 tests convergence every that many iterations (akra_cg_opts).  A solve
        stopped by maxiter or stagnation raises unless raise_not_converged is False."""
        g1, g2 = self._map(g1, "g1"), self._map(g2, "g2")
        ninv = self._map(ninv, "ninv")
        mask = self._map(mask, "mask", torch.uint8, per_rhs=False)
        xE, xB = self._alm_out(), self._alm_out()
        if x0 is not None:
            xE.copy_(x0[0].reshape(xE.shape))
            xB.copy_(x0[1].reshape(xB.shape))
        o, keep = self._opts(tol, maxiter, lam, x0, kernel, reliable_delta, hist_len, mode, stall_iters, check_every)
        inf = CgInfo()
        with torch.cuda.device(self.device):
            st = lib().akra_cg_solve(self._h, g1.data_ptr(), g2.data_ptr(), ninv.data_ptr(), mask.data_ptr(),
                                     ctypes.byref(o), xE.data_ptr(), xB.data_ptr(), ctypes.byref(inf))
        if st != AKRA_OK and (st not in (AKRA_NOT_CONVERGED, AKRA_STAGNATED) or raise_not_converged):
            _check(st)
        return xE, xB, self._info(inf, keep, hist_len)

    def cg_solve_vjp(self, g1, g2, ninv, mask, xE, xB, vE, vB, tol=1e-3, maxiter=1000, lam=1e-3, kernel=None,
                     reliable_delta=0.1, raise_not_converged=True, mode="joint", stall_iters=0, check_every=1):
        """dL/dg1, dL/dg2, dL/dninv for x = cg_solve(g1, g2, ninv, mask, ...) and the upstream
        gradient (vE, vB) on the stored (Re, Im) of x (one more CG solve, see akra_cg_solve_vjp)."""
        g1, g2 = self._map(g1, "g1"), self._map(g2, "g2")
        ninv = self._map(ninv, "ninv")
        mask = self._map(mask, "mask", torch.uint8, per_rhs=False)
        xE, xB = self._alm(xE, "xE"), self._alm(xB, "xB")
        vE, vB = self._alm(vE, "vE"), self._alm(vB, "vB")
        dg1, dg2, dn = self._map_out(), self._map_out(), self._map_out()
        o, keep = self._opts(tol, maxiter, lam, None, kernel, reliable_delta, 0, mode, stall_iters, check_every)
        inf = CgInfo()
        with torch.cuda.device(self.device):
            st = lib().akra_cg_solve_vjp(self._h, g1.data_ptr(), g2.data_ptr(), ninv.data_ptr(), mask.data_ptr(),
                                         ctypes.byref(o), xE.data_ptr(), xB.data_ptr(), vE.data_ptr(), vB.data_ptr(),
                                         dg1.data_ptr(), dg2.data_ptr(), dn.data_ptr(), ctypes.byref(inf))
        if st != AKRA_OK and (st not in (AKRA_NOT_CONVERGED, AKRA_STAGNATED) or raise_not_converged):
            _check(st)
        return dg1, dg2, dn, self._info(inf, keep, 0)

    def cg_solve_b(self, bE, bB, ninv, mask, tol=1e-3, maxiter=1000, lam=1e-3, x0=None, kernel=None,
                   reliable_delta=0.1, hist_len=0, raise_not_converged=True, mode="joint", stall_iters=0, check_every=1):
        bE, bB = self._alm(bE, "bE"), self._alm(bB, "bB")
        ninv = self._map(ninv, "ninv")
        mask = self._map(mask, "mask", torch.uint8, per_rhs=False)
        xE, xB = self._alm_out(), self._alm_out()
        if x0 is not None:
            xE.copy_(x0[0].reshape(xE.shape))
            xB.copy_(x0[1].reshape(xB.shape))
        o, keep = self._opts(tol, maxiter, lam, x0, kernel, reliable_delta, hist_len, mode, stall_iters, check_every)
        inf = CgInfo()
        with torch.cuda.device(self.device):
            st = lib().akra_cg_solve_b(self._h, ninv.data_ptr(), mask.data_ptr(), bE.data_ptr(), bB.data_ptr(),
                                       ctypes.byref(o), xE.data_ptr(), xB.data_ptr(), ctypes.byref(inf))
        if st != AKRA_OK and (st not in (AKRA_NOT_CONVERGED, AKRA_STAGNATED) or raise_not_converged):
            _check(st)
        return xE, xB, self._info(inf, keep, hist_len)

    def cg_solve_cond_b(self, g1, g2, ninv, mask, kE, tol=1e-3, maxiter=1000, lam=1e-3, kernel=None,
                        reliable_delta=0.1, hist_len=0, raise_not_converged=True, stall_iters=0, check_every=1):
        """Conditional B-mode solve: kappa_B of (H_BB + lambda_eff) kappa_B = b_B - H_BE kE for a given
        E-mode solution kE (see akra_cg_solve_cond_b)."""
        g1, g2 = self._map(g1, "g1"), self._map(g2, "g2")
        ninv = self._map(ninv, "ninv")
        mask = self._map(mask, "mask", torch.uint8, per_rhs=False)
        kE = self._alm(kE, "kE")
        kB = self._alm_out()
        o, keep = self._opts(tol, maxiter, lam, None, kernel, reliable_delta, hist_len, "joint", stall_iters, check_every)
        inf = CgInfo()
        with torch.cuda.device(self.device):
            st = lib().akra_cg_solve_cond_b(self._h, g1.data_ptr(), g2.data_ptr(), ninv.data_ptr(), mask.data_ptr(),
                                            ctypes.byref(o), kE.data_ptr(), kB.data_ptr(), ctypes.byref(inf))
        if st != AKRA_OK and (st not in (AKRA_NOT_CONVERGED, AKRA_STAGNATED) or raise_not_converged):
            _check(st)
        return kB, self._info(inf, keep, hist_len)

    # -- shape-noise realisations and spectra (Sec. IV power spectra) --------------------------
    def _dev(self, t, name, dtype, numel=None):
        if t.dtype != dtype or t.device != self.device:
            raise TypeError("%s must be %s on %s" % (name, dtype, self.device))
        if numel is not None and t.numel() != numel:
            raise ValueError("%s must hold %d entries" % (name, numel))
        return t.contiguous()

    def unmasked_index(self, mask):
        """Ascending RING indices of the unmasked pixels (int32, length n_obs)."""
        mask = self._dev(mask, "mask", torch.uint8, self.npix)
        idx = torch.empty(self.npix, dtype=torch.int32, device=self.device)
        n = ctypes.c_int64()
        with torch.cuda.device(self.device):
            _check(lib().akra_unmasked_index(self._h, mask.data_ptr(), idx.data_ptr(), ctypes.byref(n)))
        return idx[: n.value]

    def shuffle_shear(self, g1, g2, idx, perm):
        """Shear permuted among the unmasked pixels `idx` by each row of `perm` (int32 [n_real, n_obs]):
        out[k][idx[j]] = g[idx[perm[k][j]]], zero elsewhere; returns g1_out, g2_out [n_real, Npix]."""
        g1 = self._dev(g1, "g1", torch.float64, self.npix)
        g2 = self._dev(g2, "g2", torch.float64, self.npix)
        idx = self._dev(idx, "idx", torch.int32)
        perm = self._dev(perm, "perm", torch.int32)
        n_obs = idx.numel()
        if perm.dim() != 2 or perm.shape[1] != n_obs:
            raise ValueError("perm must have shape [n_real, %d]" % n_obs)
        n_real = perm.shape[0]
        o1 = torch.empty((n_real, self.npix), dtype=torch.float64, device=self.device)
        o2 = torch.empty_like(o1)
        with torch.cuda.device(self.device):
            _check(lib().akra_shuffle_shear(self._h, g1.data_ptr(), g2.data_ptr(), idx.data_ptr(), n_obs,
                                            perm.data_ptr(), n_real, o1.data_ptr(), o2.data_ptr()))
        return o1, o2

    def alm_spectra(self, x, y, pairs):
        """C_l^{x[i] y[j]} for every (i, j) in `pairs`; x, y complex128 [n, n_alm] (or [n_alm]).
        Returns float64 [npairs, lmax+1]."""
        import numpy as np
        x = self._dev(x, "x", torch.complex128).reshape(-1, self.nalm)
        y = self._dev(y, "y", torch.complex128).reshape(-1, self.nalm)
        pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        cl = torch.empty((pr.shape[0], self.lmax + 1), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().akra_alm_spectra(self._h, x.data_ptr(), x.shape[0], y.data_ptr(), y.shape[0],
                                          pr.ctypes.data, pr.shape[0], cl.data_ptr()))
        return cl

    def noise_work_bytes(self, nset=1):
        n = ctypes.c_int64()
        _check(lib().akra_noise_work_size(self._h, int(nset), ctypes.byref(n)))
        return n.value

    def noise_spectra(self, g1, g2, ninv, mask, perm, tol=1e-3, maxiter=1000, lam=1e-3, kernel=None,
                      reliable_delta=0.1, mode="E", raise_not_converged=True, work=None, stall_iters=0, check_every=1):
        """Shape-noise realisations through the full solve and their spectra (akra_noise_spectra).

        One shear set: g1, g2, ninv [Npix], perm int32 [n_real, n_obs] -> auto spectra.  Split halves:
        g1, g2, ninv [2, Npix], perm [2, n_real, n_obs] -> cross spectra of the halves.  mode "E"
        (default, the E-mode reconstruction) keeps EE, "B" keeps BB, "joint" keeps (EE, BB, EB).
        Returns cl [n_real, nspec, lmax+1], its mean and sample standard deviation [nspec, lmax+1],
        and the solve info."""
        nset = 1 if g1.dim() == 1 else g1.shape[0]
        g1 = self._dev(g1, "g1", torch.float64, nset * self.npix)
        g2 = self._dev(g2, "g2", torch.float64, nset * self.npix)
        ninv = self._dev(ninv, "ninv", torch.float64, nset * self.npix)
        mask = self._dev(mask, "mask", torch.uint8, self.npix)
        perm = self._dev(perm, "perm", torch.int32)
        if perm.dim() != (2 if nset == 1 else 3) or (nset == 2 and perm.shape[0] != 2):
            raise ValueError("perm must have shape [n_real, n_obs] (one set) or [2, n_real, n_obs] (halves)")
        n_real, n_obs = perm.shape[-2], perm.shape[-1]
        nspec = 3 if mode == "joint" else 1
        if work is None:
            work = torch.empty(self.noise_work_bytes(nset), dtype=torch.uint8, device=self.device)
        cl = torch.empty((n_real, nspec, self.lmax + 1), dtype=torch.float64, device=self.device)
        mean = torch.empty((nspec, self.lmax + 1), dtype=torch.float64, device=self.device)
        std = torch.empty_like(mean)
        o, keep = self._opts(tol, maxiter, lam, None, kernel, reliable_delta, 0, mode, stall_iters, check_every)
        inf = CgInfo()
        with torch.cuda.device(self.device):
            st = lib().akra_noise_spectra(self._h, nset, g1.data_ptr(), g2.data_ptr(), ninv.data_ptr(),
                                          mask.data_ptr(), perm.data_ptr(), n_obs, n_real, ctypes.byref(o),
                                          work.data_ptr(), work.numel(), cl.data_ptr(), mean.data_ptr(),
                                          std.data_ptr(), ctypes.byref(inf))
        if st != AKRA_OK and (st not in (AKRA_NOT_CONVERGED, AKRA_STAGNATED) or raise_not_converged):
            _check(st)
        return cl, mean, std, self._info(inf, keep, 0)

    # -- catalogue pixelisation (Sec. III.B) -----------------------------------------------------
    def ang2pix(self, z, phi):
        """RING pixel (int32) of the directions z = cos(theta), phi in [0, 2 pi) (float64 tensors)."""
        z = self._dev(z, "z", torch.float64)
        phi = self._dev(phi, "phi", torch.float64, z.numel())
        pix = torch.empty(z.numel(), dtype=torch.int32, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().akra_ang2pix(self._h, z.data_ptr(), phi.data_ptr(), z.numel(), pix.data_ptr()))
        return pix

    def pixelize_work_bytes(self, n_gal):
        n = ctypes.c_int64()
        _check(lib().akra_pixelize_work_size(self._h, int(n_gal), ctypes.byref(n)))
        return n.value

    def pixelize(self, z, phi, e1, e2, w, R, sigma_e, n_th, work=None):
        """Per-pixel gamma_obs (g1, g2), N^-1, N_eff and mask of a galaxy catalogue (akra_pixelize);
        all inputs float64 tensors of one length on the plan's device."""
        n = z.numel()
        z = self._dev(z, "z", torch.float64)
        phi, e1, e2, w = (self._dev(t, k, torch.float64, n) for t, k in ((phi, "phi"), (e1, "e1"), (e2, "e2"), (w, "w")))
        if work is None:
            work = torch.empty(self.pixelize_work_bytes(n), dtype=torch.uint8, device=self.device)
        out = {k: torch.empty(self.npix, dtype=torch.float64, device=self.device) for k in ("g1", "g2", "ninv", "neff")}
        out["mask"] = torch.empty(self.npix, dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().akra_pixelize(self._h, z.data_ptr(), phi.data_ptr(), e1.data_ptr(), e2.data_ptr(), w.data_ptr(),
                                       n, float(R), float(sigma_e), float(n_th), work.data_ptr(), work.numel(),
                                       out["g1"].data_ptr(), out["g2"].data_ptr(), out["ninv"].data_ptr(),
                                       out["neff"].data_ptr(), out["mask"].data_ptr()))
        return out

    # -- step-wise PCG ------------------------------------------------------------------------
    def cg_start(self, g1, g2, ninv, mask, lam=1e-3, kernel=None, mode="joint"):
        """Form b, lambda_eff and P and set x0 = 0 (first right-hand side of the plan)."""
        g1, g2 = self._map(g1, "g1"), self._map(g2, "g2")
        ninv = self._map(ninv, "ninv")
        mask = self._map(mask, "mask", torch.uint8, per_rhs=False)
        o, keep = self._opts(1e-3, 0, lam, None, kernel, 0.1, 0, mode)
        with torch.cuda.device(self.device):
            _check(lib().akra_cg_start(self._h, g1.data_ptr(), g2.data_ptr(), ninv.data_ptr(), mask.data_ptr(),
                                       ctypes.byref(o)))

    def cg_step(self, n=1):
        """n PCG iterations, stream-ordered, no host synchronisation."""
        with torch.cuda.device(self.device):
            _check(lib().akra_cg_step(self._h, int(n)))

    def cg_state(self, copy_x=False):
        rel = ctypes.c_double()
        it = ctypes.c_int()
        xE = xB = None
        if copy_x:
            xE, xB = torch.empty(self.nalm, dtype=torch.complex128, device=self.device), \
                torch.empty(self.nalm, dtype=torch.complex128, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().akra_cg_state(self._h, ctypes.byref(rel), ctypes.byref(it),
                                       xE.data_ptr() if copy_x else None, xB.data_ptr() if copy_x else None))
        return (rel.value, it.value, xE, xB) if copy_x else (rel.value, it.value)

    # -- stage timing -------------------------------------------------------------------------
    def set_timing(self, on=True):
        _check(lib().akra_plan_set_timing(self._h, 1 if on else 0))

    def set_graph(self, on=True):
        """Replay the PCG iteration as a recorded HIP graph (default) or launch its kernels directly."""
        _check(lib().akra_plan_set_graph(self._h, 1 if on else 0))

    def stage_times(self):
        """{stage: (total_ms, launches)} since the last call; synchronises the plan stream."""
        ms = (ctypes.c_double * len(STAGES))()
        calls = (ctypes.c_int * len(STAGES))()
        _check(lib().akra_plan_stage_times(self._h, ms, calls))
        return {s: (ms[i], calls[i]) for i, s in enumerate(STAGES)}

    # -- launch shapes ------------------------------------------------------------------------
    def set_tuning(self, syn_variant, syn_rings, adj_rings, adj_waves, adj_chunk=8):
        _check(lib().akra_plan_set_tuning(self._h, int(syn_variant), int(syn_rings), int(adj_rings),
                                          int(adj_waves), int(adj_chunk)))

    def get_tuning(self):
        v = (ctypes.c_int * 5)()
        _check(lib().akra_plan_get_tuning(self._h, v))
        return tuple(v)

    def set_tuning_one_sided(self, syn_variant, syn_rings, adj_rings, adj_waves, adj_chunk=8):
        """Launch shapes of the ring groups weighted on one side only (akra_plan_set_tuning_one_sided)."""
        _check(lib().akra_plan_set_tuning_one_sided(self._h, int(syn_variant), int(syn_rings), int(adj_rings),
                                                    int(adj_waves), int(adj_chunk)))

    def get_tuning_one_sided(self):
        v = (ctypes.c_int * 5)()
        _check(lib().akra_plan_get_tuning_one_sided(self._h, v))
        return tuple(v)

    def set_tuning_batched(self, syn_waves, adj_waves):
        """Waves per workgroup of the batched matrix-core synthesis and adjoint (FP32, nrhs > 1)."""
        _check(lib().akra_plan_set_tuning_batched(self._h, int(syn_waves), int(adj_waves)))

    def get_tuning_batched(self):
        v = (ctypes.c_int * 2)()
        _check(lib().akra_plan_get_tuning_batched(self._h, v))
        return tuple(v)

    def work(self):
        """(l, m, ring-pair) triples per Legendre launch: all, evaluated by the synthesis, by the adjoint."""
        v = (ctypes.c_int64 * 3)()
        _check(lib().akra_plan_work(self._h, v))
        b = ctypes.c_int64()
        _check(lib().akra_plan_work_batched(self._h, ctypes.byref(b)))
        return {"all": v[0], "synth": v[1], "adjoint": v[2], "batched": b.value}

    def work_weighted(self):
        """Rings that carry weight in the last weight set-up, and the (l, m, ring-pair) triples the
        weighted Legendre launches evaluate: synthesis and adjoint, in groups weighted on both sides
        (26 flop each) and on one side (18 flop each), and per right-hand side of the batched kernels."""
        v = (ctypes.c_int64 * 6)()
        _check(lib().akra_plan_work_weighted(self._h, v))
        return {"live_rings": v[0], "synth_two": v[1], "synth_one": v[2], "adjoint_two": v[3],
                "adjoint_one": v[4], "batched": v[5]}

    def set_skip_unweighted(self, on):
        """Skip rings without weight in weighted applies (the default), or run every ring (on False)."""
        _check(lib().akra_plan_set_skip_unweighted(self._h, 1 if on else 0))


class FlatPlan:
    """A flat-sky plan (akra_flat_*): an nx x ny periodic field, maps float64 [ny, nx] on the device."""

    def __init__(self, nx, ny, device=None, stream=None):
        L = lib()
        self.nx, self.ny = int(nx), int(ny)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.device(self.device):
            s = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.stream = s
            h = ctypes.c_void_p()
            _check(L.akra_flat_plan_create(self.nx, self.ny, ctypes.c_void_p(s.cuda_stream), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().akra_flat_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def device_bytes(self):
        return lib().akra_flat_plan_device_bytes(self._h)

    def _m(self, t, name, dtype=torch.float64):
        if t.dtype != dtype or t.device != self.device:
            raise TypeError("%s must be %s on %s" % (name, dtype, self.device))
        if t.numel() != self.nx * self.ny:
            raise ValueError("%s must hold ny x nx = %d x %d entries" % (name, self.ny, self.nx))
        return t.contiguous()

    def _out(self):
        return torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)

    def synth(self, kE, kB):
        kE, kB = self._m(kE, "kE"), self._m(kB, "kB")
        g1, g2 = self._out(), self._out()
        with torch.cuda.device(self.device):
            _check(lib().akra_flat_synth(self._h, kE.data_ptr(), kB.data_ptr(), g1.data_ptr(), g2.data_ptr()))
        return g1, g2

    def adjoint(self, g1, g2):
        g1, g2 = self._m(g1, "g1"), self._m(g2, "g2")
        yE, yB = self._out(), self._out()
        with torch.cuda.device(self.device):
            _check(lib().akra_flat_adjoint(self._h, g1.data_ptr(), g2.data_ptr(), yE.data_ptr(), yB.data_ptr()))
        return yE, yB

    def apply_H(self, ninv, mask, kE, kB, lambda_eff):
        ninv, mask = self._m(ninv, "ninv"), self._m(mask, "mask", torch.uint8)
        kE, kB = self._m(kE, "kE"), self._m(kB, "kB")
        yE, yB = self._out(), self._out()
        with torch.cuda.device(self.device):
            _check(lib().akra_flat_apply_H(self._h, ninv.data_ptr(), mask.data_ptr(), float(lambda_eff), kE.data_ptr(),
                                           kB.data_ptr(), yE.data_ptr(), yB.data_ptr()))
        return yE, yB

    def rhs(self, g1, g2, ninv, mask):
        g1, g2 = self._m(g1, "g1"), self._m(g2, "g2")
        ninv, mask = self._m(ninv, "ninv"), self._m(mask, "mask", torch.uint8)
        bE, bB = self._out(), self._out()
        with torch.cuda.device(self.device):
            _check(lib().akra_flat_rhs(self._h, g1.data_ptr(), g2.data_ptr(), ninv.data_ptr(), mask.data_ptr(),
                                       bE.data_ptr(), bB.data_ptr()))
        return bE, bB

    def cg_solve(self, g1, g2, ninv, mask, tol=1e-3, maxiter=1000, lam=1e-3, x0=None, hist_len=0,
                 raise_not_converged=True, stall_iters=0, check_every=1):
        """Regularised flat-sky estimate (kappa_E, kappa_B) by PCG (see akra_flat_cg_solve);
        stall_iters and check_every as for Plan.cg_solve."""
        g1, g2 = self._m(g1, "g1"), self._m(g2, "g2")
        ninv, mask = self._m(ninv, "ninv"), self._m(mask, "mask", torch.uint8)
        kE, kB = self._out(), self._out()
        if x0 is not None:
            kE.copy_(x0[0].reshape(kE.shape))
            kB.copy_(x0[1].reshape(kB.shape))
        o = CgOpts()
        lib().akra_cg_opts_default(ctypes.byref(o))
        o.lambda_, o.tol, o.maxiter = float(lam), float(tol), int(maxiter)
        o.use_x0 = 1 if x0 is not None else 0
        o.stall_iters = int(stall_iters)
        o.check_every = int(check_every)
        keep = []
        if hist_len:
            import numpy as np
            h = np.zeros(hist_len)
            keep.append(h)
            o.resid_hist = h.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            o.resid_hist_len = hist_len
        inf = CgInfo()
        with torch.cuda.device(self.device):
            st = lib().akra_flat_cg_solve(self._h, g1.data_ptr(), g2.data_ptr(), ninv.data_ptr(), mask.data_ptr(),
                                          ctypes.byref(o), kE.data_ptr(), kB.data_ptr(), ctypes.byref(inf))
        if st != AKRA_OK and (st not in (AKRA_NOT_CONVERGED, AKRA_STAGNATED) or raise_not_converged):
            _check(st)
        d = {k: getattr(inf, k) for k, _ in CgInfo._fields_}
        if hist_len:
            d["hist"] = keep[0][: inf.iters].copy()
        return kE, kB, d

    def cg_start(self, g1, g2, ninv, mask, lam=1e-3):
        g1, g2 = self._m(g1, "g1"), self._m(g2, "g2")
        ninv, mask = self._m(ninv, "ninv"), self._m(mask, "mask", torch.uint8)
        with torch.cuda.device(self.device):
            _check(lib().akra_flat_cg_start(self._h, g1.data_ptr(), g2.data_ptr(), ninv.data_ptr(), mask.data_ptr(),
                                            float(lam)))

    def cg_step(self, nsteps=1):
        with torch.cuda.device(self.device):
            _check(lib().akra_flat_cg_step(self._h, int(nsteps)))


class AkraSolve(torch.autograd.Function):
    """Differentiable regularised solve x = H^-1 b(g1, g2, ninv) on a plan.

        xE, xB = AkraSolve.apply(g1, g2, ninv, mask, plan, dict(tol=1e-8))

    Gradients flow to g1, g2 and ninv (not to the mask).  The backward pass is one more CG solve
    with the same operator, run by akra_cg_solve_vjp; solver options (the mode of the unknowns
    included) apply to both solves.  The solve information of the last forward and backward solve
    is left in plan.last_solve_info and plan.last_vjp_info."""

    @staticmethod
    def forward(ctx, g1, g2, ninv, mask, plan, opts=None):
        opts = dict(opts or {})
        xE, xB, info = plan.cg_solve(g1, g2, ninv, mask, **opts)
        plan.last_solve_info = info
        ctx.plan, ctx.opts = plan, opts
        ctx.save_for_backward(g1, g2, ninv, mask, xE, xB)
        ctx.mark_non_differentiable(mask)
        return xE, xB

    @staticmethod
    def backward(ctx, vE, vB):
        g1, g2, ninv, mask, xE, xB = ctx.saved_tensors
        if vE is None:
            vE = torch.zeros_like(xE)
        if vB is None:
            vB = torch.zeros_like(xB)
        opts = {k: v for k, v in ctx.opts.items() if k not in ("x0", "hist_len")}
        dg1, dg2, dn, info = ctx.plan.cg_solve_vjp(g1, g2, ninv, mask, xE, xB, vE.contiguous(), vB.contiguous(),
                                                   **opts)
        ctx.plan.last_vjp_info = info
        return dg1, dg2, dn, None, None, None
