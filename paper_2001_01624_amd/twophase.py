"""Time stepping of the two-phase model with the CPR preconditioner (the
solution procedure of the paper's section "Description of the solution
procedure": linearise, decouple, multiscale pressure predictor, ILU(0)
corrector, GMRES), driving the C ABI only.

Dynamic bases follow the update approach of the subsection "Iterative
multiscale multibasis solver": before the first Newton iteration of a time
step from the last pressure update of the previous step, and again before
the second iteration from the first update of this step (Dp(Inf)); with
``every_iteration`` before each iteration (Dp(1)).
"""
from __future__ import annotations

from . import capi


def time_step(tp, p, s, dt, *, newton_tol=1e-6, max_newton=20, lin_rtol=1e-6, lin_max=500, basis_sweeps=3,
              dynamic=True, every_iteration=False, last_dp=None, q=None):
    """One backward-Euler step from (p, s) (device tensors, updated in
    place).  Convergence: ``||R||_2 <= newton_tol * ||R_0||_2`` with ``R_0``
    the residual at the step's start.  Returns a dict with the Newton
    iterations, the GMRES iterations of each, the residual norms and the
    last pressure update (for the next step's dynamic basis)."""
    import torch

    ms = tp.ms
    s_old = s.clone()
    stats = {"linear": [], "res": [], "dyn_blocks": []}
    dp_last = last_dp
    r0 = None
    for it in range(max_newton):
        if dynamic and dp_last is not None and (it < 2 or every_iteration):
            stats["dyn_blocks"].append(ms.add_dynamic_basis([dp_last]))
        nr = tp.assemble(dt, p, s, s_old, q=q, basis_sweeps=basis_sweeps)
        stats["res"].append(nr)
        if r0 is None:
            r0 = nr if nr > 0 else 1.0
        if nr <= newton_tol * r0:
            break
        dx, its, rel, rc = tp.solve(rtol=lin_rtol, max_iters=lin_max)
        stats["linear"].append(its)
        if rc != capi.OK:
            stats["failed"] = True
            break
        tp.update(dx, p, s)
        dp_last = dx[0::2].contiguous()
    stats["newton"] = len(stats["linear"])
    stats["last_dp"] = dp_last
    return stats
