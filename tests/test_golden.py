"""Oracle against the closed-form values stored in tests/golden/closed_forms.json."""
import json
import math
import os

import numpy as np

from oracle.core import Oracle, kernel_l
from oracle.geometry import gl_rings, healpix_rings

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def test_kernel_values():
    k = kernel_l(4096, sigma_d=+1.0)          # sigma_D = +1 gives D_l itself
    for l, v in GOLD["D_l_squared"].items():
        if l.startswith("_"):
            continue
        num, den = v
        assert abs(k[int(l)] + math.sqrt(num / den)) < 2e-16


def test_healpix_nside1():
    r = healpix_rings(1)
    g = GOLD["healpix_nside1"]
    np.testing.assert_allclose(r.z, g["z"], atol=1e-16)
    np.testing.assert_allclose(r.p0num / r.p0den, g["phi0_over_pi"], atol=1e-16)


def test_y20_coefficient():
    g = GOLD["spin2_Y20_coeff_squared"]
    c = math.sqrt(g["num"] / (g["den_over_pi"] * math.pi))
    lam = Oracle(2, gl_rings(2)).wigner(0, -2, math.cos(0.9), norm=True)
    assert abs(lam[2] - c * math.sin(0.9) ** 2) < 1e-16
