"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on
the same seeded inputs, step by step and end to end.

Tolerances (FP64 path): integer structure bit-exact; single kernels 1e-12
relative; basis entries 1e-12 absolute; coarse operators 1e-12 relative to
their largest entry; iterates after a fixed number of cycles 1e-9 relative
(cycles amplify summation-order differences); converged solutions within
1e-8 relative of the direct solve at rtol 1e-10.
"""
import numpy as np
import pytest

import oracle as O
from workloads import (make_config0, make_config1, make_config2, make_homogeneous, make_lognormal_box,
                       pressure_increment_pair, rng_for)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


CASES = {
    "cfg0": (lambda: make_config0(0), (6, 6, 1)),
    "ragged3d": (lambda: make_lognormal_box((13, 11, 7), rng_for(7, 1), sigma=1.5, corr=(2, 2, 1)), (3, 2, 2)),
    "layered": (lambda: make_config1(dims=(20, 36, 14), seed=1), (4, 3, 2)),
    "faulted_inactive": (lambda: make_config2(dims=(18, 30, 12), seed=2), (3, 3, 2)),
    "line1d": (lambda: make_lognormal_box((33, 1, 1), rng_for(7, 2), sigma=1.0), (5, 1, 1)),
    # row lengths around the kernels' layout limits: 62 (widest fused ILU
    # row), 64 (one full wavefront), 70 and 130 (two and three 64-cell runs
    # per row: several x tiles in the sweep, chunked rows in the transfer
    # kernels, the general residual and two-pass ILU)
    "edge62": (lambda: make_lognormal_box((62, 7, 6), rng_for(7, 3), sigma=1.5, corr=(4, 2, 1)), (4, 2, 2)),
    "edge64": (lambda: make_lognormal_box((64, 5, 4), rng_for(7, 4), sigma=1.5, corr=(4, 2, 1)), (5, 2, 1)),
    "wide": (lambda: make_lognormal_box((70, 9, 5), rng_for(7, 5), sigma=1.5, corr=(3, 2, 1)), (5, 2, 2)),
    "wider": (lambda: make_config2(dims=(130, 6, 4), seed=4), (9, 2, 2)),
    # degenerate shapes: rows of one cell along y or z only (one active lane
    # per wavefront, every x face a boundary face), and the longest row the
    # library accepts (256 cells: four full 64-cell runs)
    "zline": (lambda: make_lognormal_box((1, 1, 40), rng_for(7, 6), sigma=1.5, corr=(1, 1, 3)), (1, 1, 5)),
    "yline": (lambda: make_lognormal_box((1, 37, 1), rng_for(7, 7), sigma=1.5, corr=(1, 3, 1)), (1, 4, 1)),
    "maxrow": (lambda: make_lognormal_box((256, 3, 2), rng_for(7, 8), sigma=1.5, corr=(8, 1, 1)), (16, 1, 1)),
    # tall columns around the z-line ILU layout limit: 512 cells (64 chunks of
    # 8 held in registers) and 600 (the kernel that walks chunks from memory)
    "tall512": (lambda: make_lognormal_box((5, 3, 512), rng_for(7, 12), sigma=1.5, corr=(1, 1, 8)), (2, 1, 16)),
    "tall600": (lambda: make_lognormal_box((4, 3, 600), rng_for(7, 13), sigma=1.5, corr=(1, 1, 8)), (2, 1, 16)),
}


def build(capi, name, smoother="jacobi", outer="richardson", precision="fp64"):
    mk, cd = CASES[name]
    prob = mk()
    parts = [{"kind": "cartesian", "coarse_dims": cd}]
    opt = capi.default_options(smoother=smoother, outer=outer, precision=precision)
    say(f"case {name} dims={prob.dims} coarse={cd} smoother={smoother} outer={outer} precision={precision}")
    g = capi.Solver(prob, parts, opt)
    o = O.Oracle(prob, parts, smoother=smoother)
    return prob, g, o


def relerr(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("name", list(CASES))
def test_residual_and_matvec(capi, name):
    prob, g, o = build(capi, name)
    x = np.random.default_rng(1).standard_normal(prob.n_cells) * prob.active
    r = host(g.apply(capi.OP_RESIDUAL, dev(x)))
    y = host(g.apply(capi.OP_MATVEC, dev(x)))
    ro = np.zeros(prob.n_cells)
    ro[o.cells] = o.residual(x)
    yo = np.zeros(prob.n_cells)
    yo[o.cells] = o.A @ x[o.cells]
    assert relerr(r, ro) <= 1e-13 and relerr(y, yo) <= 1e-13
    assert np.all(r[~prob.active] == 0) and np.all(y[~prob.active] == 0)


@pytest.mark.parametrize("name", ["cfg0", "ragged3d", "faulted_inactive", "edge62", "edge64", "wide", "wider",
                                  "zline", "yline", "maxrow", "tall512", "tall600"])
@pytest.mark.parametrize("smoother", ["jacobi", "ilu0_rb", "ilu0_line"])
def test_smoother(capi, name, smoother):
    prob, g, o = build(capi, name, smoother=smoother)
    r = np.random.default_rng(2).standard_normal(prob.n_cells) * prob.active
    e = host(g.apply(capi.OP_SMOOTH, dev(r)))
    eo = np.zeros(prob.n_cells)
    eo[o.cells] = o.smooth(r[o.cells])
    assert relerr(e, eo) <= 1e-12


def oracle_support_slots(o, stage=0):
    """(cell, block) pairs of the oracle's support matrix, in box numbering."""
    S = o.stages[stage].S.tocoo()
    return set(zip(o.cells[S.row].tolist(), S.col.tolist()))


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("sweeps", [0, 1, 5, 37])
def test_basis_fixed_sweeps(capi, name, sweeps):
    prob, g, o = build(capi, name)
    sw, _ = g.update_basis(max_sweeps=sweeps, tol=0.0)
    o.update_basis(max_sweeps=sweeps, tol=0.0)
    assert sw == sweeps == o.stages[0].sweeps
    e = g.export_stage(0)
    # integer structure: partition and supports bit-exact
    assert np.array_equal(e["block"], np.where(prob.active, o.stages[0].block, -1))
    sb = e["slot_block"]
    pairs = {(i, int(b)) for s in range(sb.shape[0]) for i, b in zip(np.nonzero(sb[s] >= 0)[0].tolist(),
                                                                     sb[s][sb[s] >= 0].tolist())}
    assert pairs == oracle_support_slots(o)
    P = g.dense_basis(0)
    Po = o.export_basis(0)
    assert np.abs(P - Po).max() <= 1e-12
    # Galerkin coarse operator
    Ac = e["Ac"]
    assert relerr(Ac, o.stages[0].Ac) <= 1e-12


@pytest.mark.parametrize("name", ["cfg0", "layered"])
def test_basis_stop_rule(capi, name):
    prob, g, o = build(capi, name)
    sw, ch = g.update_basis(max_sweeps=100, tol=1e-3)
    o.update_basis(max_sweeps=100, tol=1e-3)
    assert abs(sw - o.stages[0].sweeps) <= 1
    if sw == o.stages[0].sweeps:
        assert ch == pytest.approx(o.stages[0].change, rel=1e-9)


@pytest.mark.parametrize("name", ["cfg0", "layered"])
def test_stop_rule_equals_fixed_count(capi, name):
    # the device decides sweeps in pairs: when the first of a pair meets the
    # tolerance the second has already run and must leave no trace, so the
    # basis, the count and the last change equal those of exactly that many
    # sweeps; the tolerances give stopping counts of both parities
    prob, g, o = build(capi, name)
    counts = []
    for tol in (3e-2, 1e-2, 5e-3, 3e-3, 2e-3, 1e-3):
        n, ch = g.update_basis(max_sweeps=100, tol=tol)
        P = g.dense_basis(0)
        n2, ch2 = g.update_basis(max_sweeps=n, tol=0.0)
        say(f"{name}: tol {tol:g}: {n} sweeps, change {ch:.3e}")
        assert n2 == n and ch2 == ch
        assert np.array_equal(g.dense_basis(0), P)
        counts.append(n)
    assert {n % 2 for n in counts} == {0, 1}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("smoother", ["jacobi", "ilu0_rb", "ilu0_line"])
def test_preconditioner(capi, name, smoother):
    prob, g, o = build(capi, name, smoother=smoother)
    g.update_basis(max_sweeps=20, tol=0.0)
    o.update_basis(max_sweeps=20, tol=0.0)
    r = np.random.default_rng(3).standard_normal(prob.n_cells) * prob.active
    z = host(g.apply(capi.OP_PRECOND, dev(r)))
    zo = np.zeros(prob.n_cells)
    zo[o.cells] = o.precondition(r[o.cells])
    assert relerr(z, zo) <= 1e-10


@pytest.mark.parametrize("name", ["cfg0", "layered", "faulted_inactive"])
@pytest.mark.parametrize("smoother", ["jacobi", "ilu0_rb", "ilu0_line"])
def test_richardson_fixed_cycles(capi, name, smoother):
    prob, g, o = build(capi, name, smoother=smoother)
    g.update_basis(max_sweeps=30, tol=0.0)
    o.update_basis(max_sweeps=30, tol=0.0)
    p = dev(np.zeros(prob.n_cells))
    it, rel, rc = g.solve(p, rtol=0.0, max_iters=7)
    xo, cyc, relo, st = o.solve(rtol=0.0, max_cycles=7)
    assert rc == capi.E_NOCONV and it == cyc == 7
    assert relerr(host(p), xo) <= 1e-9
    assert rel == pytest.approx(relo, rel=1e-8)


@pytest.mark.parametrize("smoother", ["jacobi", "ilu0_rb", "ilu0_line"])
def test_richardson_converges_cfg0(capi, smoother):
    prob, g, o = build(capi, "cfg0", smoother=smoother)
    g.update_basis(max_sweeps=100, tol=1e-3)
    o.update_basis(max_sweeps=100, tol=1e-3)
    p = dev(np.zeros(prob.n_cells))
    it, rel, rc = g.solve(p, rtol=1e-10, max_iters=3000)
    assert rc == capi.OK and rel <= 1e-10
    xo, cyc, relo, st = o.solve(rtol=1e-10, max_cycles=3000)
    assert abs(it - cyc) <= 1
    xd = o.direct_solve()
    x = host(p)
    assert relerr(x, xd) <= 1e-8
    # the relative residual recomputed by the oracle in FP64
    assert np.linalg.norm(o.residual(x)) / np.linalg.norm(o.b) <= 1.0001e-10


@pytest.mark.parametrize("name,smoother", [(n, "ilu0_rb") for n in ("cfg0", "layered", "faulted_inactive", "wide",
                                                                     "zline", "maxrow")]
                         + [(n, "ilu0_line") for n in ("layered", "faulted_inactive", "zline", "wide")])
def test_gmres_converges(capi, name, smoother):
    prob, g, o = build(capi, name, smoother=smoother, outer="gmres")
    g.update_basis(max_sweeps=60, tol=1e-3)
    o.update_basis(max_sweeps=60, tol=1e-3)
    p = dev(np.zeros(prob.n_cells))
    it, rel, rc = g.solve(p, rtol=1e-10, max_iters=1000)
    assert rc == capi.OK and rel <= 1e-10
    x = host(p)
    assert np.linalg.norm(o.residual(x)) / np.linalg.norm(o.b) <= 1.0001e-10
    xo, ito, relo, st = o.solve_gmres(rtol=1e-10, restart=30, max_iters=1000)
    assert abs(it - ito) <= max(2, ito // 10)
    assert relerr(x, o.direct_solve()) <= 1e-7


@pytest.mark.parametrize("restart", [1, 2, 5])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gmres_short_restarts(capi, restart, precision):
    # every restart ends with the update x += Z T^-1 y over the kept
    # preconditioned candidates; with restart 1 or 2 the triangle T is 1x1 or
    # 2x2 and the last column is finalised after every step or two
    prob = make_config0(0)
    parts = [{"kind": "cartesian", "coarse_dims": (6, 6, 1)}]
    opt = capi.default_options(smoother="ilu0_rb", outer="gmres", restart=restart, precision=precision)
    g = capi.Solver(prob, parts, opt)
    o = O.Oracle(prob, parts, smoother="ilu0_rb")
    g.update_basis(max_sweeps=60, tol=1e-3)
    p = dev(np.zeros(prob.n_cells))
    it, rel, rc = g.solve(p, rtol=1e-8, max_iters=3000)
    true = np.linalg.norm(o.residual(host(p))) / np.linalg.norm(o.b)
    say(f"GMRES({restart}) {precision}: {it} iterations, reported {rel:.2e}, true {true:.2e}")
    assert rc == capi.OK and true <= 1.0001e-8


def test_gmres_first_steps_match_oracle(capi):
    prob, g, o = build(capi, "layered", smoother="ilu0_rb", outer="gmres")
    g.update_basis(max_sweeps=30, tol=0.0)
    o.update_basis(max_sweeps=30, tol=0.0)
    for k in (1, 3, 8):
        p = dev(np.zeros(prob.n_cells))
        it, rel, rc = g.solve(p, rtol=0.0, max_iters=k)
        xo, ito, relo, st = o.solve_gmres(rtol=0.0, restart=30, max_iters=k)
        assert it == ito == k
        assert rel == pytest.approx(relo, rel=1e-7)
        assert relerr(host(p), xo) <= 1e-8


@pytest.mark.parametrize("name", ["cfg0", "layered", "faulted_inactive"])
def test_dynamic_partition_and_coarse(capi, name):
    prob, g, o = build(capi, name)
    g.update_basis(max_sweeps=10, tol=0.0)
    o.update_basis(max_sweeps=10, tol=0.0)
    dps = pressure_increment_pair(prob, rng_for(8, 1))
    counts = g.add_dynamic_basis([dev(d) for d in dps])
    oc = o.add_dynamic_basis(dps)
    assert counts == oc
    assert g.num_stages() == 1 + sum(1 for c in counts if c > 0)
    for k in range(len(o.dyn)):
        e = g.export_stage(1 + k)
        assert e["kind"] == 3 and e["M"] == o.dyn[k].M
        assert np.array_equal(e["block"], o.dyn[k].block)
        assert relerr(e["Ac"], o.dyn[k].Ac) <= 1e-12
    # cycles with the dynamic stages
    p = dev(np.zeros(prob.n_cells))
    it, rel, rc = g.solve(p, rtol=0.0, max_iters=5)
    xo, cyc, relo, st = o.solve(rtol=0.0, max_cycles=5)
    assert relerr(host(p), xo) <= 1e-9


def test_dynamic_edge_cases(capi):
    prob, g, o = build(capi, "cfg0")
    g.update_basis(max_sweeps=5, tol=0.0)
    z = dev(np.zeros(prob.n_cells))
    assert g.add_dynamic_basis([z]) == [0]
    assert g.num_stages() == 1
    dp = pressure_increment_pair(prob, rng_for(8, 2))[0]
    c1 = g.add_dynamic_basis([dev(dp)])
    c2 = g.add_dynamic_basis([dev(-dp * 2.0 ** 7)])
    assert c1 == c2 and c1[0] > 0
    g.clear_dynamic_basis()
    assert g.num_stages() == 1


def test_fluxes_and_mass_balance(capi):
    prob, g, o = build(capi, "layered", smoother="ilu0_rb", outer="gmres")
    g.update_basis(max_sweeps=50, tol=1e-3)
    p = dev(np.zeros(prob.n_cells))
    it, rel, rc = g.solve(p, rtol=1e-10, max_iters=1000)
    face, bcf = g.fluxes(p)
    x = host(p)
    fo, bo = o.fluxes(x)
    assert relerr(host(face), fo) <= 1e-13 and relerr(host(bcf), bo) <= 1e-13
    assert abs(prob.source.sum() - host(bcf).sum()) <= 1e-8 * abs(prob.source.sum())


def test_source_change_and_warm_start(capi):
    prob, g, o = build(capi, "layered", smoother="ilu0_rb", outer="gmres")
    g.update_basis(max_sweeps=40, tol=1e-3)
    o.update_basis(max_sweeps=40, tol=1e-3)
    q2 = prob.source * 0.0
    inj = prob.wells["injector"]
    q2[inj[: len(inj) // 2]] = 2.0 / max(1, len(inj) // 2)
    p = dev(np.zeros(prob.n_cells))
    it, rel, rc = g.solve(p, source=dev(q2), rtol=1e-9, max_iters=1000)
    assert rc == capi.OK
    xd = o.direct_solve(source=q2)
    assert relerr(host(p), xd) <= 1e-6
    # warm start: extra sweeps from the current basis equal sweeps from scratch
    g.update_basis(max_sweeps=5, tol=0.0, warm=True)
    o.update_basis(max_sweeps=5, tol=0.0, warm=True)
    assert np.abs(g.dense_basis(0) - o.export_basis(0)).max() <= 1e-12


def test_error_paths(capi):
    prob = make_config0(0)
    parts = [{"kind": "cartesian", "coarse_dims": (6, 6, 1)}]
    g = capi.Solver(prob, parts)
    p = dev(np.zeros(prob.n_cells))
    with pytest.raises(capi.MsrsbError) as e:
        g.solve(p)
    assert e.value.code == capi.E_STATE
    with pytest.raises(capi.MsrsbError) as e:
        g.update_basis(stage=3)
    assert e.value.code == capi.E_INVAL
    bad = make_config0(0)
    bad.bc_trans = np.zeros_like(bad.bc_trans)
    with pytest.raises(capi.MsrsbError) as e:
        capi.Solver(bad, parts)
    assert e.value.code == capi.E_SINGULAR
    with pytest.raises(capi.MsrsbError) as e:
        capi.Solver(prob, [{"kind": "cartesian", "coarse_dims": (61, 1, 1)}])
    assert e.value.code == capi.E_INVAL
    # size limits: rows of at most 256 cells, at most 1024 coarse layers
    for dims, cd in (((257, 2, 1), (4, 1, 1)), ((1, 1, 1100), (1, 1, 1025))):
        with pytest.raises(capi.MsrsbError) as e:
            capi.Solver(make_lognormal_box(dims, rng_for(7, 9)), [{"kind": "cartesian", "coarse_dims": cd}])
        assert e.value.code == capi.E_INVAL
    g.update_basis(max_sweeps=3, tol=0.0)
    it, rel, rc = g.solve(p, rtol=1e-14, max_iters=1)
    assert rc == capi.E_NOCONV and it == 1 and 0 < rel < 1


@pytest.mark.parametrize("outer", ["richardson", "gmres"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_single_cell(capi, outer, precision):
    # one cell between the two Dirichlet faces (p = 1 and p = 0) with equal
    # half-face transmissibilities: the pressure is 1/2, and in FP64 the first
    # step (exact ILU(0), one block with P = 1) reaches it to rounding.  In
    # mixed precision a Krylov vector passes through the FP32 smoother, so
    # GMRES may need a second step
    prob = make_lognormal_box((1, 1, 1), rng_for(7, 10), sigma=1.0)
    opt = capi.default_options(smoother="ilu0_rb", outer=outer, precision=precision)
    g = capi.Solver(prob, [{"kind": "cartesian", "coarse_dims": (1, 1, 1)}], opt)
    g.update_basis(max_sweeps=5, tol=0.0)
    p = dev(np.zeros(1))
    it, rel, rc = g.solve(p, rtol=1e-12, max_iters=10)
    say(f"single cell {outer} {precision}: {it} iterations, relres {rel:.2e}, p = {host(p)[0]!r}")
    assert rc == capi.OK and rel <= 1e-12
    if precision == "fp64":
        assert it == 1 and abs(host(p)[0] - 0.5) <= 1e-15
    else:
        assert abs(host(p)[0] - 0.5) <= 1e-12


def test_special_bases(capi):
    # one block: P == 1; one block per cell: P == I, and the cycle is exact
    prob = make_lognormal_box((6, 5, 3), rng_for(7, 3), sigma=1.0)
    g1 = capi.Solver(prob, [{"kind": "cartesian", "coarse_dims": (1, 1, 1)}])
    g1.update_basis(max_sweeps=9, tol=0.0)
    assert np.all(g1.dense_basis(0) == 1.0)
    gN = capi.Solver(prob, [{"kind": "cartesian", "coarse_dims": (6, 5, 3)}])
    gN.update_basis(max_sweeps=4, tol=0.0)
    assert np.array_equal(gN.dense_basis(0), np.eye(90))
    p = dev(np.zeros(90))
    it, rel, rc = gN.solve(p, rtol=1e-12, max_iters=3)
    assert it == 1 and rel <= 1e-12


def test_deterministic_repeat(capi):
    prob, g, o = build(capi, "layered", smoother="ilu0_rb", outer="gmres")
    g.update_basis(max_sweeps=40, tol=1e-3)
    a = dev(np.zeros(prob.n_cells))
    b = dev(np.zeros(prob.n_cells))
    g.solve(a, rtol=1e-8, max_iters=500)
    g.update_basis(max_sweeps=40, tol=1e-3)
    g.solve(b, rtol=1e-8, max_iters=500)
    assert torch.equal(a, b)


# ------------------------------------------------------------- fault cut ----

FAULT_PARTS = [{"kind": "cartesian", "coarse_dims": (3, 3, 2)}, {"kind": "fault_cut", "parent": 0}]


def build_fault(capi, smoother="jacobi", outer="richardson", precision="fp64", dims=(18, 30, 12), seed=2):
    prob = make_config2(dims=dims, seed=seed)
    say(f"fault-cut case dims={dims} seed={seed} faults={int(prob.fault.sum())} smoother={smoother}")
    opt = capi.default_options(smoother=smoother, outer=outer, precision=precision)
    g = capi.Solver(prob, FAULT_PARTS, opt)
    o = O.Oracle(prob, FAULT_PARTS, smoother=smoother)
    return prob, g, o


def test_fault_cut_structure(capi):
    prob, g, o = build_fault(capi)
    M, kind, ns = g.stage_info(1)
    st = o.stages[1]
    assert kind == 2 and M == st.M and M > o.stages[0].M
    e = g.export_stage(1, values=False, coarse=False)
    assert np.array_equal(e["block"], np.where(prob.active, st.block, -1))
    sb = e["slot_block"]
    pairs = {(i, int(b)) for s in range(ns) for i, b in zip(np.nonzero(sb[s] >= 0)[0].tolist(),
                                                           sb[s][sb[s] >= 0].tolist())}
    assert pairs == oracle_support_slots(o, 1)
    # slot lists ascending, padded with -1
    for s in range(1, ns):
        both = (sb[s] >= 0)
        assert np.all(sb[s - 1][both] < sb[s][both]) and np.all(sb[s - 1][~both | (sb[s - 1] >= 0)] >= -1)


@pytest.mark.parametrize("sweeps", [0, 1, 6, 25])
def test_fault_cut_basis_and_coarse(capi, sweeps):
    prob, g, o = build_fault(capi)
    g.update_basis(max_sweeps=sweeps, tol=0.0)
    o.update_basis(max_sweeps=sweeps, tol=0.0)
    for k in (0, 1):
        assert np.abs(g.dense_basis(k) - o.export_basis(k)).max() <= 1e-12
        assert relerr(g.export_stage(k)["Ac"], o.stages[k].Ac) <= 1e-12


@pytest.mark.parametrize("smoother", ["jacobi", "ilu0_rb", "ilu0_line"])
def test_fault_cut_cycles(capi, smoother):
    prob, g, o = build_fault(capi, smoother=smoother)
    g.update_basis(max_sweeps=20, tol=0.0)
    o.update_basis(max_sweeps=20, tol=0.0)
    p = dev(np.zeros(prob.n_cells))
    it, rel, rc = g.solve(p, rtol=0.0, max_iters=6)
    xo, cyc, relo, st = o.solve(rtol=0.0, max_cycles=6)
    assert it == cyc == 6 and relerr(host(p), xo) <= 1e-9


def test_fault_cut_gmres_converges(capi):
    prob, g, o = build_fault(capi, smoother="ilu0_rb", outer="gmres", dims=(24, 40, 14), seed=3)
    g.update_basis(max_sweeps=60, tol=1e-3)
    p = dev(np.zeros(prob.n_cells))
    it, rel, rc = g.solve(p, rtol=1e-10, max_iters=1000)
    assert rc == capi.OK
    x = host(p)
    assert np.linalg.norm(o.residual(x)) / np.linalg.norm(o.b) <= 1.0001e-10
    assert relerr(x, o.direct_solve()) <= 1e-7


# ------------------------------------------------------- mixed precision ----
# Stated per-result bounds against the FP64 oracle: basis entries within
# 2^-8 |P| + 2e-5 (BF16 rounding of the stored basis, at most 2^-8 relative, plus the
# drift of FP32 sweeps); coarse operators within 1e-2 relative to their
# largest entry; solves reach the same FP64 relative residual.

@pytest.mark.parametrize("name", ["cfg0", "layered", "faulted_inactive", "wide", "wider"])
def test_mixed_basis_within_bound(capi, name):
    prob, g, o = build(capi, name, precision="mixed")
    g.update_basis(max_sweeps=20, tol=0.0)
    o.update_basis(max_sweeps=20, tol=0.0)
    P = g.dense_basis(0)
    Po = o.export_basis(0)
    err = np.abs(P - Po)
    say(f"mixed basis max error {err.max():.2e}")
    assert np.all(err <= 2.0 ** -8 * np.abs(Po) + 2e-5)
    # stored values are exact BF16 numbers
    v = P[P != 0].astype(np.float32).view(np.uint32)
    assert np.all(v & 0xFFFF == 0)
    Ac = g.export_stage(0)["Ac"]
    assert np.abs(Ac - Ac.T).max() == 0.0
    assert relerr(Ac, o.stages[0].Ac) <= 1e-2


@pytest.mark.parametrize("name", ["cfg0", "layered", "faulted_inactive", "wide"])
def test_mixed_solve_meets_fp64_tolerance(capi, name):
    prob, g, o = build(capi, name, smoother="ilu0_rb", outer="gmres", precision="mixed")
    g.update_basis(max_sweeps=60, tol=1e-3)
    p = dev(np.zeros(prob.n_cells))
    it, rel, rc = g.solve(p, rtol=1e-6, max_iters=2000)
    assert rc == capi.OK
    x = host(p)
    true = np.linalg.norm(o.residual(x)) / np.linalg.norm(o.b)
    xd = o.direct_solve()
    say(f"mixed {name}: {it} its, relres {true:.2e}, solution error {relerr(x, xd):.2e}")
    assert true <= 1.0001e-6
    f64 = capi.Solver(prob, [{"kind": "cartesian", "coarse_dims": CASES[name][1]}],
                      capi.default_options(smoother="ilu0_rb", outer="gmres"))
    f64.update_basis(max_sweeps=60, tol=1e-3)
    q = dev(np.zeros(prob.n_cells))
    it64, _, _ = f64.solve(q, rtol=1e-6, max_iters=2000)
    # equal accuracy: both within 1e-6 of the FP64 residual; mixed needs at most a few more iterations
    assert it <= it64 + max(3, it64 // 5)


def test_mixed_fault_cut(capi):
    prob, g, o = build_fault(capi, smoother="ilu0_rb", outer="gmres", precision="mixed")
    g.update_basis(max_sweeps=15, tol=0.0)
    o.update_basis(max_sweeps=15, tol=0.0)
    for k in (0, 1):
        err = np.abs(g.dense_basis(k) - o.export_basis(k))
        assert np.all(err <= 2.0 ** -8 * np.abs(o.export_basis(k)) + 2e-5)
    p = dev(np.zeros(prob.n_cells))
    it, rel, rc = g.solve(p, rtol=1e-6, max_iters=2000)
    assert rc == capi.OK
    assert np.linalg.norm(o.residual(host(p))) / np.linalg.norm(o.b) <= 1.0001e-6
