"""CPU oracle for the AKRA 3.0 matrix-free operator -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP path
(``paper_2606_06175_amd``) and neither imports the other.

Contents
  geometry  HEALPix RING and Gauss-Legendre ring tables (plain numpy).
  core      ctypes binding of the plain C core (long-double Wigner-d recurrence,
            direct ring sums), the operator H = K Y^H W Y K + lambda_eff I,
            the right-hand side b and preconditioned CG, all in float64 numpy.
  dense     brute-force definition at tiny sizes: spin-2 harmonics from Wigner's
            explicit sum (mpmath), dense A and H, Cholesky solve.
"""
from .geometry import healpix_rings, gl_rings, Rings  # noqa: F401
from .core import Oracle, alm_size, alm_index, kernel_l, full_dot  # noqa: F401
