"""Pins of the two-phase oracle (sections "Model equations", "Discrete
equations" and "Preconditioning: the constrained pressure residual (CPR)
method"): the Jacobian against central finite differences of the residual,
the sum of the residuals against the well and source terms (fluxes and
accumulation cancel), the IMPES pressure block against a two-point assembly
of the total-mobility coefficients, the defining property of ILU(0) on the
full system, and Newton with GMRES + CPR converging with mass balance."""
import numpy as np
import pytest

import oracle as O
from oracle import twophase as TP
from workloads import make_config1, make_config2

FLUID = dict(mu_w=1.0, mu_o=5.0, n_w=2.0, n_o=2.0)


def state(prob, seed):
    rng = np.random.default_rng(seed)
    p = rng.uniform(0.0, 1.0, prob.n_cells)
    s = rng.uniform(0.15, 0.85, prob.n_cells)
    return p * prob.active, s * prob.active


def pore_volume(prob):
    return np.full(prob.n_cells, 0.2 * np.prod(prob.h)) * prob.active


@pytest.mark.parametrize("mk", [lambda: make_config1(dims=(5, 6, 3), seed=1), lambda: make_config2(dims=(6, 5, 4), seed=2)])
def test_jacobian_matches_finite_differences(mk):
    prob = mk()
    pv = pore_volume(prob)
    p, s = state(prob, 3)
    s_old = np.clip(s - 0.05, 0, 1) * prob.active
    R, J = TP.residual_jacobian(prob, pv, FLUID, 10.0, p, s, s_old)
    cells = np.nonzero(prob.active)[0]
    Jd = J.toarray()
    h = 1e-6
    for k in range(0, cells.size, 3):
        c = cells[k]
        for var in (0, 1):
            xp, xm = (p.copy(), s.copy()), (p.copy(), s.copy())
            xp[var][c] += h
            xm[var][c] -= h
            Rp, _ = TP.residual_jacobian(prob, pv, FLUID, 10.0, xp[0], xp[1], s_old)
            Rm, _ = TP.residual_jacobian(prob, pv, FLUID, 10.0, xm[0], xm[1], s_old)
            fd = (Rp - Rm) / (2 * h)
            col = Jd[:, 2 * k + var]
            assert np.abs(fd - col).max() <= 1e-5 * max(np.abs(col).max(), 1.0), (c, var)


def test_residual_sum_is_wells_and_sources():
    prob = make_config1(dims=(6, 7, 3), seed=3)
    pv = pore_volume(prob)
    p, s = state(prob, 4)
    R, _ = TP.residual_jacobian(prob, pv, FLUID, 5.0, p, s, s * 0.9)
    lw, lo, _, _ = TP.mobilities(s, FLUID)
    wells = sum(t * (lw[c] + lo[c]) * (p[c] - v) for c, t, v in zip(prob.bc_cell, prob.bc_trans, prob.bc_value))
    assert abs(R.sum() - (wells - prob.source.sum())) <= 1e-12 * max(abs(wells), 1.0)


def test_impes_pressure_block_is_two_point_operator():
    prob = make_config2(dims=(7, 6, 4), seed=5)
    pv = pore_volume(prob)
    p, s = state(prob, 6)
    R, J = TP.residual_jacobian(prob, pv, FLUID, 3.0, p, s, s)
    Jpp = 0.5 * (J[0::2][:, 0::2] + J[1::2][:, 0::2])
    tx, ty, tz, bc = TP.pressure_coefficients(prob, FLUID, p, s)
    q = prob.with_source()
    q.tx, q.ty, q.tz, q.bc_trans = tx, ty, tz, bc
    A, _, _, _ = O.assemble(q)
    assert abs(Jpp - A).max() <= 1e-13 * abs(A).max()
    # the IMPES weights cancel the accumulation terms: the pressure rows of the
    # saturation columns hold only flux and well derivatives
    Jps = 0.5 * (J[0::2][:, 1::2] + J[1::2][:, 1::2])
    dt_small = 1e-6
    _, J2 = TP.residual_jacobian(prob, pv, FLUID, dt_small, p, s, s)
    Jps2 = 0.5 * (J2[0::2][:, 1::2] + J2[1::2][:, 1::2])
    assert abs(Jps - Jps2).max() <= 1e-9 * max(abs(Jps).max(), 1e-30)  # no pv/dt term survives


def test_full_system_ilu0_defining_property():
    prob = make_config1(dims=(5, 4, 3), seed=7)
    pv = pore_volume(prob)
    p, s = state(prob, 8)
    _, J = TP.residual_jacobian(prob, pv, FLUID, 2.0, p, s, s)
    order = TP.red_black_cell_order(prob)
    L, U, _ = O.ilu0_factor(J, order, positive=False)
    B = J[order][:, order].toarray()
    LU = (L @ U).toarray()
    Bs = J[order][:, order].tocoo()
    on = np.zeros_like(B, dtype=bool)
    on[Bs.row, Bs.col] = True
    assert np.abs((LU - B)[on]).max() <= 1e-12 * np.abs(B).max()


def test_newton_with_cpr_converges_and_balances_mass():
    prob = make_config1(dims=(10, 12, 4), seed=9)
    pv = pore_volume(prob)
    parts = [{"kind": "cartesian", "coarse_dims": (2, 3, 2)}]
    ms = O.Oracle(prob, parts, smoother="ilu0_rb")
    ms.update_basis(max_sweeps=20, tol=0.0)
    sim = TP.TwoPhase(prob, pv, FLUID, 50.0, ms)
    p = np.zeros(prob.n_cells)
    s_old = np.full(prob.n_cells, 0.2) * prob.active
    s = s_old.copy()
    norms = []
    for it in range(8):
        sim.update_pressure_operator(p, s)
        p, s, its, rel, R = sim.newton_step(p, s, s_old, rtol=1e-10)
        assert rel <= 1e-10 and its < 200
        norms.append(np.abs(R).max())
    Rf, _ = TP.residual_jacobian(prob, pv, FLUID, 50.0, p, s, s_old)
    assert np.abs(Rf).max() <= 1e-9 * norms[0]
    # water volume: pv (s - s_old)/dt = injected - produced
    lw, lo, _, _ = TP.mobilities(s, FLUID)
    prod_w = sum(t * lw[c] * (p[c] - v) for c, t, v in zip(prob.bc_cell, prob.bc_trans, prob.bc_value))
    dv = (pv * (s - s_old)).sum() / 50.0
    assert abs(dv - (prob.source.sum() - prod_w)) <= 1e-8 * prob.source.sum()
    assert np.all((s >= 0) & (s <= 1))
