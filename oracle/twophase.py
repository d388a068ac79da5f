"""CPU FP64 oracle of the two-phase model and the two-stage CPR preconditioner.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no
code with the GPU library and never imports it.

Model (section "Model equations", the two-phase case with an aqueous and a
liquid phase, one component each; section "Discrete equations": backward
Euler, two-point fluxes, single-point upstream mobilities): unknowns per
active cell ``x = (p_i, s_i)`` with ``s`` the water saturation; no gravity
and no capillary pressure (the setting of Example 1 with unit density
ratio); Corey relative permeabilities ``k_rw = s^n_w``, ``k_ro = (1-s)^n_o``;
mobilities ``lambda = k_r / mu``.  Residuals (volumes per time step):

    R_w,i = pv_i/dt (s_i - s_i^n) + sum_f T_f lambda_w(up) (p_i - p_l)
            + sum_c WI_c lambda_w(s_i) (p_i - p_c) - q_i
    R_o,i = -pv_i/dt (s_i - s_i^n) + sum_f T_f lambda_o(up) (p_i - p_l)
            + sum_c WI_c lambda_o(s_i) (p_i - p_c)

with ``up`` the cell the face flux leaves (``p_a >= p_b`` -> ``a`` for the
face ``a < b``), ``c`` the well connections (bottom-hole pressure ``p_c``)
and ``q`` the injected water rate.

CPR (section "Preconditioning: the constrained pressure residual (CPR)
method"): IMPES weights cancel the accumulation derivatives with respect to
the saturation; here ``w_w pv/dt - w_o pv/dt = 0`` with ``w_w + w_o = 1``, so
``w = (1/2, 1/2)`` in every cell and the pressure block ``J_pp* = (J_wp +
J_op)/2`` is the two-point operator with face coefficients
``T_f lambda_t(up)/2`` and well terms ``WI_c lambda_t(s_i)/2``.  One
application of the two-stage preconditioner to ``v``: the pressure
predictor ``dp = M_ms^{-1} ((v_w + v_o)/2)`` (one multistage cycle of the
multiscale multibasis solver on ``J_pp*``), then ``y = (dp, 0) +
ILU0(J)^{-1} (v - J (dp, 0))`` with ILU(0) of the full system in red-black
cell order (the corrector step of section "Description of the solution
procedure").
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .msrsb import _coords, _faces, ilu0_apply, ilu0_factor


def mobilities(s, fluid):
    """``(lambda_w, lambda_o, dlambda_w/ds, dlambda_o/ds)``."""
    mw, mo, nw, no = fluid["mu_w"], fluid["mu_o"], fluid["n_w"], fluid["n_o"]
    s = np.asarray(s, dtype=np.float64)
    lw = s ** nw / mw
    lo = (1.0 - s) ** no / mo
    dlw = nw * s ** (nw - 1.0) / mw if nw != 1.0 else np.full_like(s, 1.0 / mw)
    dlo = -no * (1.0 - s) ** (no - 1.0) / mo if no != 1.0 else np.full_like(s, -1.0 / mo)
    return lw, lo, dlw, dlo


def residual_jacobian(prob, pv, fluid, dt, p, s, s_old, q=None):
    """Residual ``R`` (``2 n``, interleaved ``(R_w,i, R_o,i)`` over the active
    cells) and Jacobian ``J = dR/dx`` with ``x`` interleaved ``(p_i, s_i)``,
    from the formulas above.  ``p, s, s_old, pv, q`` in box numbering."""
    cells = np.nonzero(prob.active)[0]
    n = cells.size
    loc = np.full(prob.n_cells, -1, dtype=np.int64)
    loc[cells] = np.arange(n)
    q = np.asarray(prob.source if q is None else q, dtype=np.float64)
    lw, lo, dlw, dlo = mobilities(s, fluid)
    R = np.zeros(2 * n)
    rows, cols, vals = [], [], []

    def add(r, c, v):
        rows.append(r)
        cols.append(c)
        vals.append(v)

    acc = pv[cells] / dt
    ds = s[cells] - s_old[cells]
    R[0::2] += acc * ds - q[cells]
    R[1::2] += -acc * ds
    li = np.arange(n)
    add(2 * li, 2 * li + 1, acc)
    add(2 * li + 1, 2 * li + 1, -acc)
    # structural zeros: every 2x2 block that the stencil touches is stored in full
    add(2 * li, 2 * li, 0.0 * acc)
    add(2 * li + 1, 2 * li, 0.0 * acc)
    a, b, T = _faces(prob)
    up = np.where(p[a] >= p[b], a, b)
    dp = p[a] - p[b]
    la, lb = loc[a], loc[b]
    for ph, (lam, dlam) in enumerate(((lw, dlw), (lo, dlo))):
        F = T * lam[up] * dp  # flux a -> b
        np.add.at(R, 2 * la + ph, F)
        np.add.at(R, 2 * lb + ph, -F)
        c = T * lam[up]
        # d/dp
        add(2 * la + ph, 2 * la, c)
        add(2 * la + ph, 2 * lb, -c)
        add(2 * lb + ph, 2 * lb, c)
        add(2 * lb + ph, 2 * la, -c)
        # d/ds of the upstream cell
        g = T * dlam[up] * dp
        ua = up == a
        add(2 * la + ph, 2 * la + 1, np.where(ua, g, 0.0))
        add(2 * la + ph, 2 * lb + 1, np.where(ua, 0.0, g))
        add(2 * lb + ph, 2 * la + 1, np.where(ua, -g, 0.0))
        add(2 * lb + ph, 2 * lb + 1, np.where(ua, 0.0, -g))
    wc = np.asarray(prob.bc_cell, dtype=np.int64)
    wi = np.asarray(prob.bc_trans, dtype=np.float64)
    pc = np.asarray(prob.bc_value, dtype=np.float64)
    lc = loc[wc]
    for ph, (lam, dlam) in enumerate(((lw, dlw), (lo, dlo))):
        np.add.at(R, 2 * lc + ph, wi * lam[wc] * (p[wc] - pc))
        add(2 * lc + ph, 2 * lc, wi * lam[wc])
        add(2 * lc + ph, 2 * lc + 1, wi * dlam[wc] * (p[wc] - pc))
    J = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(2 * n, 2 * n)).tocsr()
    J.sum_duplicates()
    J.sort_indices()
    return R, J


def pressure_coefficients(prob, fluid, p, s):
    """IMPES pressure operator: face coefficients ``T lambda_t(up) / 2`` in the
    structured layout ``(tx, ty, tz)`` and well terms ``WI lambda_t(s_i) / 2``."""
    nx, ny, nz = prob.dims
    lw, lo, _, _ = mobilities(s, fluid)
    lt = lw + lo
    out = []
    for T, step in ((prob.tx, 1), (prob.ty, nx), (prob.tz, nx * ny)):
        c = np.zeros(prob.n_cells)
        a = np.nonzero(T)[0]
        up = np.where(p[a] >= p[a + step], a, a + step)
        c[a] = 0.5 * T[a] * lt[up]
        out.append(c)
    wc = np.asarray(prob.bc_cell, dtype=np.int64)
    bc = 0.5 * np.asarray(prob.bc_trans) * lt[wc]
    return out[0], out[1], out[2], bc


def red_black_cell_order(prob):
    """Unknowns of red cells (even ``i+j+k``) first, then black, each cell's
    ``(p, s)`` pair kept together, cells ascending within a colour."""
    cells = np.nonzero(prob.active)[0]
    ix, iy, iz = _coords(prob.dims)
    col = (ix + iy + iz)[cells] % 2
    order_cells = np.concatenate([np.nonzero(col == 0)[0], np.nonzero(col == 1)[0]])
    return np.stack([2 * order_cells, 2 * order_cells + 1], axis=1).reshape(-1)


def cpr_apply(J, v, pressure_precond, ilu):
    """One application of the two-stage CPR preconditioner (IMPES weights
    1/2, 1/2): pressure predictor by ``pressure_precond`` (a function of the
    pressure residual), then ILU(0) of the full system on what is left."""
    vp = 0.5 * (v[0::2] + v[1::2])
    dp = pressure_precond(vp)
    y = np.zeros_like(v)
    y[0::2] = dp
    r2 = v - J @ y
    return y + ilu0_apply(ilu, r2)


def gmres(Aop, b, M, rtol, max_iters, restart=30):
    """Restarted GMRES with right preconditioner ``M`` (Saad & Schultz;
    modified Gram-Schmidt, least squares solved directly), from zero.
    Returns ``(x, iterations, relres)`` with ``relres`` the true residual."""
    x = np.zeros_like(b)
    nb = np.linalg.norm(b)
    nb = nb if nb > 0 else 1.0
    its = 0
    while True:
        r = b - Aop(x)
        beta = np.linalg.norm(r)
        if beta / nb <= rtol or its >= max_iters:
            return x, its, beta / nb
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        y = None
        for j in range(restart):
            z = M(V[j])
            Z.append(z)
            w = Aop(z)
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            its += 1
            e1 = np.zeros(j + 2)
            e1[0] = beta
            y = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)[0]
            est = np.linalg.norm(e1 - H[:j + 2, :j + 1] @ y)
            if H[j + 1, j] == 0.0 or est / nb <= rtol or its >= max_iters:
                break
            V.append(w / H[j + 1, j])
        x = x + np.column_stack(Z[:y.size]) @ y


class TwoPhase:
    """Newton steps of the two-phase model with GMRES + CPR, around an oracle
    multiscale solver (``oracle.msrsb.Oracle``) for the pressure predictor."""

    def __init__(self, prob, pv, fluid, dt, ms_oracle):
        self.prob, self.pv, self.fluid, self.dt = prob, np.asarray(pv, dtype=np.float64), fluid, dt
        self.ms = ms_oracle
        self.cells = np.nonzero(prob.active)[0]
        self.order = red_black_cell_order(prob)

    def linear_system(self, p, s, s_old, q=None):
        R, J = residual_jacobian(self.prob, self.pv, self.fluid, self.dt, p, s, s_old, q)
        return R, J

    def update_pressure_operator(self, p, s, sweeps=3):
        """The pressure block of the current Jacobian in the multiscale solver:
        new face and well coefficients, then ``sweeps`` extra smoothing sweeps
        of every basis from its current state (local basis updates)."""
        tx, ty, tz, bc = pressure_coefficients(self.prob, self.fluid, p, s)
        self.ms.update_basis(max_sweeps=sweeps, tol=0.0, warm=True, new_trans=(tx, ty, tz), new_bc_trans=bc)

    def cpr(self, J):
        ilu = ilu0_factor(J, self.order, positive=False)
        return lambda v: cpr_apply(J, v, self.ms.precondition, ilu)

    def newton_step(self, p, s, s_old, rtol=1e-8, max_iters=500, restart=30, q=None):
        """One Newton update ``dx = -J^{-1} R`` by GMRES with CPR.  Returns
        ``(p_new, s_new, iterations, relres, R)`` (saturations clamped to
        [0, 1])."""
        R, J = self.linear_system(p, s, s_old, q)
        M = self.cpr(J)
        dx, its, rel = gmres(lambda v: J @ v, -R, M, rtol, max_iters, restart)
        pn, sn = p.copy(), s.copy()
        pn[self.cells] += dx[0::2]
        sn[self.cells] = np.clip(s[self.cells] + dx[1::2], 0.0, 1.0)
        return pn, sn, its, rel, R
