"""GPU parity of the two-phase model and the two-stage CPR preconditioner
(msrsb_tp_*) against the two-phase oracle: residual and Jacobian products
within 1e-12 relative, one CPR application within 1e-9 (the multistage
cycle's parity bound), GMRES + CPR Newton updates within 1e-6 of the
oracle's (both linear solves to 1e-10), and Newton time steps converging
with water-volume balance."""
import numpy as np
import pytest

import oracle as O
from oracle import twophase as TP
from workloads import make_config1, make_config2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FLUID = dict(mu_w=1.0, mu_o=5.0, n_w=2.0, n_o=2.0)


@pytest.fixture(scope="module")
def capi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2001_01624_amd import capi as c
    return c


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def say(*a):
    print(*a, flush=True)


def relerr(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def pore_volume(prob):
    return np.full(prob.n_cells, 0.2 * np.prod(prob.h)) * prob.active


def inter(R, cells, N):
    """Oracle interleaved vector over active cells -> box-numbered [2N]."""
    out = np.zeros(2 * N)
    out[2 * cells] = R[0::2]
    out[2 * cells + 1] = R[1::2]
    return out


CASES = {
    "layered": (lambda: make_config1(dims=(14, 16, 6), seed=3), (2, 2, 2)),
    "faulted": (lambda: make_config2(dims=(12, 14, 6), seed=4), (2, 2, 2)),
}


def setup(capi, name, sweeps=3, dt=20.0, seed=0, smoother="ilu0_rb"):
    mk, cd = CASES[name]
    prob = mk()
    parts = [{"kind": "cartesian", "coarse_dims": cd}]
    pv = pore_volume(prob)
    g = capi.Solver(prob, parts, capi.default_options(smoother=smoother, outer="gmres"))
    g.update_basis(max_sweeps=20, tol=0.0)
    o = O.Oracle(prob, parts, smoother=smoother)
    o.update_basis(max_sweeps=20, tol=0.0)
    tp = capi.TwoPhase(g, pv, FLUID, restart=30)
    rng = np.random.default_rng(seed)
    p = rng.uniform(0.0, 1.0, prob.n_cells) * prob.active
    s = rng.uniform(0.15, 0.85, prob.n_cells) * prob.active
    s_old = np.clip(s - 0.05, 0.0, 1.0) * prob.active
    return prob, pv, g, o, tp, p, s, s_old


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("smoother", ["ilu0_rb", "ilu0_line"])
def test_residual_jacobian_and_cpr(capi, name, smoother):
    prob, pv, g, o, tp, p, s, s_old = setup(capi, name, smoother=smoother)
    say(f"two-phase {name} dims={prob.dims} pressure smoother {smoother}")
    N = prob.n_cells
    res = torch.empty(2 * N, dtype=torch.float64, device="cuda")
    nr = tp.assemble(20.0, dev(p), dev(s), dev(s_old), basis_sweeps=3, res=res)
    R, J = TP.residual_jacobian(prob, pv, FLUID, 20.0, p, s, s_old)
    Rb = inter(R, o.cells, N)
    assert relerr(host(res), Rb) <= 1e-12 and abs(nr - np.linalg.norm(R)) <= 1e-12 * np.linalg.norm(R)
    x = np.random.default_rng(1).standard_normal(2 * N)
    x[np.repeat(~prob.active, 2)] = 0.0
    xl = np.empty(2 * o.cells.size)
    xl[0::2], xl[1::2] = x[2 * o.cells], x[2 * o.cells + 1]
    Jx = host(tp.apply(tp.OP_MATVEC, dev(x)))
    assert relerr(Jx, inter(J @ xl, o.cells, N)) <= 1e-12
    # CPR: the oracle's pressure solver with the same IMPES operator and local basis updates
    tx, ty, tz, bc = TP.pressure_coefficients(prob, FLUID, p, s)
    o.update_basis(max_sweeps=3, tol=0.0, warm=True, new_trans=(tx, ty, tz), new_bc_trans=bc)
    ilu = O.ilu0_factor(J, TP.red_black_cell_order(prob), positive=False)
    yo = TP.cpr_apply(J, xl, o.precondition, ilu)
    y = host(tp.apply(tp.OP_CPR, dev(x)))
    assert relerr(y, inter(yo, o.cells, N)) <= 1e-9
    # the pressure context now holds the IMPES operator
    e = g.export_stage(0)
    assert relerr(e["Ac"], o.stages[0].Ac) <= 1e-12
    tp.close()
    g.close()


@pytest.mark.parametrize("name", list(CASES))
def test_newton_update_matches_oracle(capi, name):
    prob, pv, g, o, tp, p, s, s_old = setup(capi, name, seed=2)
    say(f"two-phase newton update {name}")
    N = prob.n_cells
    tp.assemble(20.0, dev(p), dev(s), dev(s_old), basis_sweeps=2)
    dx, its, rel, rc = tp.solve(rtol=1e-10, max_iters=3000)
    say(f"  GMRES + CPR: {its} iterations, relres {rel:.2e}")
    assert rc == capi.OK and rel <= 1e-10
    R, J = TP.residual_jacobian(prob, pv, FLUID, 20.0, p, s, s_old)
    xl = np.empty(2 * o.cells.size)
    d = host(dx)
    xl[0::2], xl[1::2] = d[2 * o.cells], d[2 * o.cells + 1]
    assert np.linalg.norm(J @ xl + R) <= 1.0001e-10 * np.linalg.norm(R)  # true residual on the oracle's system
    Jd = J.toarray()
    xo = np.linalg.solve(Jd, -R)
    # forward error within what the residual allows: |x - x*| <= |J^-1|_2 |J x + R|
    smin = np.linalg.svd(Jd, compute_uv=False)[-1]
    assert np.linalg.norm(xl - xo) <= 1.01 * np.linalg.norm(J @ xl + R) / smin + 1e-14 * np.linalg.norm(xo)
    say(f"  GMRES + CPR iterations {its}")
    tp.close()
    g.close()


def test_time_steps_converge_and_balance_water(capi):
    from paper_2001_01624_amd import twophase

    prob = make_config1(dims=(16, 20, 6), seed=5)
    parts = [{"kind": "cartesian", "coarse_dims": (2, 2, 2)}]
    pv = pore_volume(prob)
    g = capi.Solver(prob, parts, capi.default_options(smoother="ilu0_rb", outer="gmres"))
    g.update_basis(max_sweeps=30, tol=1e-3)
    tp = capi.TwoPhase(g, pv, FLUID, restart=30)
    p = torch.zeros(prob.n_cells, dtype=torch.float64, device="cuda")
    s = dev(np.full(prob.n_cells, 0.2) * prob.active)
    dt = 200.0
    last = None
    for step in range(3):
        s0 = host(s).copy()
        st = twophase.time_step(tp, p, s, dt, newton_tol=1e-9, lin_rtol=1e-8, last_dp=last)
        last = st["last_dp"]
        say(f"  step {step}: newton {st['newton']}, linear {st['linear']}, dyn {st['dyn_blocks']}")
        assert not st.get("failed") and st["res"][-1] <= 1e-9 * st["res"][0]
        ph, sh = host(p), host(s)
        R, _ = TP.residual_jacobian(prob, pv, FLUID, dt, ph, sh, s0)
        assert np.linalg.norm(R) <= 1e-8 * st["res"][0]
        lw, lo, _, _ = TP.mobilities(sh, FLUID)
        prod_w = sum(t * lw[c] * (ph[c] - v) for c, t, v in zip(prob.bc_cell, prob.bc_trans, prob.bc_value))
        dv = (pv * (sh - s0)).sum() / dt
        assert abs(dv - (prob.source.sum() - prod_w)) <= 1e-6 * prob.source.sum()
        assert np.all((sh >= 0) & (sh <= 1))
    tp.close()
    g.close()


def test_twophase_errors(capi):
    prob = make_config1(dims=(8, 8, 4), seed=1)
    g = capi.Solver(prob, [{"kind": "cartesian", "coarse_dims": (2, 2, 1)}])
    pv = pore_volume(prob)
    say("two-phase error paths")
    with pytest.raises(capi.MsrsbError):
        capi.TwoPhase(g, pv, dict(mu_w=0.0, mu_o=1.0, n_w=2.0, n_o=2.0))
    tp = capi.TwoPhase(g, pv, FLUID)
    x = torch.zeros(2 * prob.n_cells, dtype=torch.float64, device="cuda")
    with pytest.raises(capi.MsrsbError) as ei:
        tp.apply(tp.OP_CPR, x)
    assert ei.value.code == capi.E_STATE
    z = torch.zeros(prob.n_cells, dtype=torch.float64, device="cuda")
    with pytest.raises(capi.MsrsbError) as ei:  # bases missing
        tp.assemble(1.0, z, z, z)
    assert ei.value.code == capi.E_STATE
    tp.close()
    g.close()
