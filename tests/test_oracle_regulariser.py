"""The oracle's regulariser lambda_eff = lambda <N^-1>_M and scalar preconditioner
P = (<M^2 N^-1> + lambda_eff)^-1 (paper Sec. II.B, eq. ML_estimator_reg and eq. precond) against the
hand-worked values of tests/golden/regulariser.json, for the sphere and for the flat field.

The fixtures are chosen so that the plausible slips (averaging over every pixel instead of the
unmasked ones, averaging W in lambda_eff, or averaging only the unmasked pixels in P) give other
numbers; the test checks that they do, so a fixture that cannot tell them apart fails too."""
import json
import os

import numpy as np

from oracle.core import Oracle
from oracle.flat import FlatOracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "regulariser.json")))


def _frac(v):
    return v[0] / v[1]


def test_sphere_lambda_eff_and_precond_hand_worked():
    g = GOLD["sphere_nside1"]
    ninv = np.asarray(g["ninv"], np.float64)
    mask = np.asarray(g["mask"], np.uint8)
    assert ninv.shape == (12,)
    for c in g["cases"]:
        lam = Oracle.lambda_eff(ninv, mask, lam=c["lambda"])
        assert abs(lam - _frac(c["lambda_eff"])) <= 4e-16 * _frac(c["lambda_eff"]), (c, lam)
        P = Oracle.precond(ninv, mask, lam)
        assert abs(P - _frac(c["P"])) <= 4e-16 * _frac(c["P"]), (c, P)
    # the default lambda of the method is 1e-3 (Sec. II.B)
    assert Oracle.lambda_eff(ninv, mask) == Oracle.lambda_eff(ninv, mask, lam=1e-3)


def test_sphere_fixture_separates_the_slips():
    g = GOLD["sphere_nside1"]
    ninv = np.asarray(g["ninv"], np.float64)
    mask = np.asarray(g["mask"], np.uint8)
    s = g["slips"]
    want = _frac(g["cases"][0]["lambda_eff"])
    W = np.where(mask != 0, ninv, 0.0)
    assert abs(1e-3 * ninv.mean() - _frac(s["lambda_eff_mean_over_all_pixels"])) < 1e-16
    assert abs(1e-3 * W.mean() - _frac(s["lambda_eff_mean_of_W_over_all_pixels"])) < 1e-16
    assert abs(1.0 / (ninv[mask != 0].mean() + want) - _frac(s["P_mean_over_unmasked_pixels"])) < 1e-16
    for v in s.values():
        if isinstance(v, list):
            assert abs(_frac(v) - want) > 1e-4 and abs(_frac(v) - _frac(g["cases"][0]["P"])) > 1e-4


def test_flat_lambda_eff_and_precond_hand_worked():
    for key, shape in (("flat_2x3", (2, 3)), ("flat_4x4", (4, 4))):
        g = GOLD[key]
        ninv = np.asarray(g["ninv"], np.float64)
        mask = np.asarray(g["mask"], np.uint8)
        assert ninv.shape == shape
        _flat_cases(g, ninv, mask)


def _flat_cases(g, ninv, mask):
    for c in g["cases"]:
        lam = FlatOracle.lambda_eff(ninv, mask, lam=c["lambda"])
        assert abs(lam - _frac(c["lambda_eff"])) <= 4e-16 * _frac(c["lambda_eff"]), (c, lam)
        P = FlatOracle.precond(ninv, mask, lam)
        assert abs(P - _frac(c["P"])) <= 4e-16 * _frac(c["P"]), (c, P)


def test_masked_weights_do_not_enter():
    # changing N^-1 on masked pixels (even to a huge value) leaves both quantities unchanged
    g = GOLD["sphere_nside1"]
    ninv = np.asarray(g["ninv"], np.float64)
    mask = np.asarray(g["mask"], np.uint8)
    lam = Oracle.lambda_eff(ninv, mask)
    P = Oracle.precond(ninv, mask, lam)
    ninv2 = np.where(mask != 0, ninv, 1e9)
    assert Oracle.lambda_eff(ninv2, mask) == lam
    assert Oracle.precond(ninv2, mask, lam) == P
