"""MI355X-native matrix-free mass-mapping operator of AKRA 3.0 (HIP kernels behind a C ABI).

    from paper_2606_06175_amd import Plan
    plan = Plan(nside, lmax, precision="fp64")
    xE, xB, info = plan.cg_solve(g1, g2, ninv, mask, tol=1e-8)
    xE, xB = AkraSolve.apply(g1, g2, ninv, mask, plan, dict(tol=1e-8))   # differentiable
"""
from .akra import AkraError, AkraSolve, FlatPlan, Plan, alm_size, lib  # noqa: F401
