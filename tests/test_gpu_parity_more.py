"""GPU parity for paths the first parity suite reaches only indirectly: the
coarse solve element by element (several 64-wide Gauss-Jordan panels), the
mixed-precision smoother, preconditioner and Galerkin operator against the
FP64 oracle with stated bounds, a dual z-interval taller than one wavefront,
GMRES restarts above the DCGS2 limit, the dynamic-block cap on the device,
and argument checks of the binding.

Bounds:
* coarse solve: |p_c - p_c*|_inf <= M kappa(A_c) eps |p_c*|_inf against the
  oracle's Cholesky solve of the same A_c (an explicit inverse applied by a
  GEMV is forward stable to about kappa eps per entry; M is a margin for
  the summation lengths);
* FP32 smoother: |e - e*| <= 2^-17 (M^-1 |r|) entry by entry, M^-1 the
  oracle's smoother (for these M-matrices M^-1 >= 0 entry-wise, so M^-1|r|
  bounds every partial sum, and each entry takes at most about 40
  correctly rounded FP32 operations: 40 * 2^-24 < 2^-17);
* mixed preconditioner: 1e-4 relative (max norm) against the oracle's FP64
  cycle on the same stored BF16 basis (FP32 smoother and transfer arithmetic,
  about 1e-6 per application, through two coarse corrections, with margin);
* mixed Galerkin operator: exactly the FP64 product of the stored BF16 basis,
  1e-12 relative.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from workloads import make_config0, make_config1, make_config2, make_lognormal_box, pressure_increment_pair, rng_for

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def capi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2001_01624_amd import capi as c
    return c


def say(*a):
    print(*a, flush=True)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def check_coarse(g, k, Ac, seed):
    """GPU coarse solve of stage k against a Cholesky solve of A_c."""
    M = Ac.shape[0]
    d = np.random.default_rng(seed).standard_normal(M)
    pc = g.coarse_apply(k, d)
    L = O.coarse_factor(Ac)
    ref = O.coarse_solve(L, d)
    lam = np.linalg.eigvalsh(Ac)
    kappa = lam[-1] / lam[0]
    err = np.abs(pc - ref).max() / np.abs(ref).max()
    say(f"stage {k}: M = {M}, kappa = {kappa:.2e}, coarse-solve error {err:.2e}, bound {M * kappa * EPS:.2e}")
    assert err <= M * kappa * EPS


# ----------------------------------------------------------- coarse solve ----

@pytest.mark.parametrize("dims,cd", [((24, 20, 8), (8, 5, 4)), ((36, 36, 4), (12, 12, 2)), ((40, 30, 6), (10, 10, 3))])
def test_coarse_solve_several_panels(capi, dims, cd):
    # M = 160, 288, 300: three to five 64-wide panels, ragged last panel
    prob = make_lognormal_box(dims, rng_for(12, dims[0]), sigma=1.5, corr=(2, 2, 1))
    parts = [{"kind": "cartesian", "coarse_dims": cd}]
    say(f"coarse solve case {dims} / {cd}")
    g = capi.Solver(prob, parts)
    o = O.Oracle(prob, parts)
    g.update_basis(max_sweeps=12, tol=0.0)
    o.update_basis(max_sweeps=12, tol=0.0)
    Ac = g.export_stage(0)["Ac"]
    assert relerr(Ac, o.stages[0].Ac) <= 1e-12
    check_coarse(g, 0, o.stages[0].Ac, 1)


def test_coarse_solve_dynamic_and_fault_stages(capi):
    prob = make_config2(dims=(18, 30, 12), seed=2)
    parts = [{"kind": "cartesian", "coarse_dims": (3, 3, 2)}, {"kind": "fault_cut", "parent": 0}]
    g = capi.Solver(prob, parts)
    o = O.Oracle(prob, parts)
    g.update_basis(max_sweeps=10, tol=0.0)
    o.update_basis(max_sweeps=10, tol=0.0)
    dps = pressure_increment_pair(prob, rng_for(8, 1))
    assert g.add_dynamic_basis([dev(d) for d in dps]) == o.add_dynamic_basis(dps)
    for k, st in enumerate(o.all_stages()):
        check_coarse(g, k, st.Ac, 10 + k)


# -------------------------------------------------------- mixed precision ----

@pytest.mark.parametrize("name,mk,cd", [
    ("layered", lambda: make_config1(dims=(20, 36, 14), seed=1), (4, 3, 2)),
    ("faulted_inactive", lambda: make_config2(dims=(18, 30, 12), seed=2), (3, 3, 2)),
    ("wider", lambda: make_config2(dims=(130, 6, 4), seed=4), (9, 2, 2)),
    ("tall512", lambda: make_lognormal_box((5, 3, 512), rng_for(7, 12), sigma=1.5, corr=(1, 1, 8)), (2, 1, 16)),
    ("tall600", lambda: make_lognormal_box((4, 3, 600), rng_for(7, 13), sigma=1.5, corr=(1, 1, 8)), (2, 1, 16)),
])
@pytest.mark.parametrize("smoother", ["jacobi", "ilu0_rb", "ilu0_line"])
def test_mixed_smoother_bound(capi, name, mk, cd, smoother):
    prob = mk()
    parts = [{"kind": "cartesian", "coarse_dims": cd}]
    g = capi.Solver(prob, parts, capi.default_options(smoother=smoother, precision="mixed"))
    o = O.Oracle(prob, parts, smoother=smoother)
    r = np.random.default_rng(4).standard_normal(prob.n_cells) * prob.active
    e = host(g.apply(capi.OP_SMOOTH, dev(r)))[o.cells]
    eo = o.smooth(r[o.cells])
    mag = o.smooth(np.abs(r[o.cells]))
    assert np.all(mag >= 0)
    ratio = np.abs(e - eo).max() / mag.max()
    say(f"mixed {smoother} smoother on {name}: max |e - e*| / max M^-1|r| = {ratio:.2e}")
    # the z-line order runs recurrences along whole columns: at most about 16 nz + 64
    # correctly rounded FP32 operations per entry
    bound = 2.0 ** -24 * (16 * prob.dims[2] + 64) if smoother == "ilu0_line" else 2.0 ** -17
    assert np.all(np.abs(e - eo) <= bound * mag)


def oracle_on_exported_basis(g, prob, parts, smoother):
    """The oracle's cycle on the basis the GPU stores (BF16 values, upcast)."""
    o = O.Oracle(prob, parts, smoother=smoother)
    o.update_basis(max_sweeps=0, tol=0.0)
    for k, st in enumerate(o.stages):
        P = sp.csr_matrix(g.dense_basis(k)[o.cells])
        st.P = P
        st.Ac = O.galerkin(P, o.A)
        st.L = O.coarse_factor(st.Ac)
    return o


@pytest.mark.parametrize("name,mk,parts", [
    ("layered", lambda: make_config1(dims=(20, 36, 14), seed=1), [{"kind": "cartesian", "coarse_dims": (4, 3, 2)}]),
    ("two_stages", lambda: make_config1(dims=(24, 30, 12), seed=2),
     [{"kind": "cartesian", "coarse_dims": (4, 5, 2)}, {"kind": "cartesian", "coarse_dims": (3, 3, 3)}]),
    ("fault_cut", lambda: make_config2(dims=(18, 30, 12), seed=2),
     [{"kind": "cartesian", "coarse_dims": (3, 3, 2)}, {"kind": "fault_cut", "parent": 0}]),
])
@pytest.mark.parametrize("smoother", ["jacobi", "ilu0_rb"])
def test_mixed_galerkin_and_preconditioner(capi, name, mk, parts, smoother):
    prob = mk()
    g = capi.Solver(prob, parts, capi.default_options(smoother=smoother, precision="mixed"))
    g.update_basis(max_sweeps=20, tol=0.0)
    o = oracle_on_exported_basis(g, prob, parts, smoother)
    for k, st in enumerate(o.stages):
        Ac = g.export_stage(k)["Ac"]
        err = relerr(Ac, st.Ac)
        say(f"{name} stage {k}: A_c against the FP64 product of the stored BF16 basis: {err:.2e}")
        assert err <= 1e-12
    r = np.random.default_rng(5).standard_normal(prob.n_cells) * prob.active
    z = host(g.apply(capi.OP_PRECOND, dev(r)))
    zo = np.zeros(prob.n_cells)
    zo[o.cells] = o.precondition(r[o.cells])
    err = relerr(z, zo)
    say(f"{name} {smoother}: mixed preconditioner against the FP64 cycle on the BF16 basis: {err:.2e}")
    assert err <= 1e-4
    # and one Richardson cycle from zero agrees the same way
    p = dev(np.zeros(prob.n_cells))
    g.solve(p, rtol=0.0, max_iters=1)
    xo, _, _, _ = o.solve(rtol=0.0, max_cycles=1)
    assert relerr(host(p), xo) <= 1e-4


# ------------------------------------------------- tall dual z-intervals ----

def test_tall_dual_interval(capi):
    # one coarse layer over 80 fine layers: the restriction's z-interval is
    # wider than one wavefront (its general gather path)
    prob = make_lognormal_box((16, 8, 80), rng_for(12, 7), sigma=1.5, corr=(2, 2, 4))
    parts = [{"kind": "cartesian", "coarse_dims": (2, 2, 1)}]
    for smoother in ("jacobi", "ilu0_rb"):
        g = capi.Solver(prob, parts, capi.default_options(smoother=smoother))
        o = O.Oracle(prob, parts, smoother=smoother)
        for sweeps in (0, 7):
            g.update_basis(max_sweeps=sweeps, tol=0.0)
            o.update_basis(max_sweeps=sweeps, tol=0.0)
            assert np.abs(g.dense_basis(0) - o.export_basis(0)).max() <= 1e-12
            assert relerr(g.export_stage(0)["Ac"], o.stages[0].Ac) <= 1e-12
        r = np.random.default_rng(6).standard_normal(prob.n_cells)
        z = host(g.apply(capi.OP_PRECOND, dev(r)))
        assert relerr(z, o.precondition(r)) <= 1e-10
        p = dev(np.zeros(prob.n_cells))
        it, rel, rc = g.solve(p, rtol=0.0, max_iters=4)
        xo, cyc, relo, st = o.solve(rtol=0.0, max_cycles=4)
        assert it == cyc == 4 and relerr(host(p), xo) <= 1e-9


# ------------------------------------------------- GMRES, long restarts ----

def test_gmres_restart_above_dcgs2_limit(capi):
    # restart 40 runs classical Gram-Schmidt with the DGKS second-pass test
    prob = make_config1(dims=(20, 36, 14), seed=1)
    parts = [{"kind": "cartesian", "coarse_dims": (4, 3, 2)}]
    g = capi.Solver(prob, parts, capi.default_options(smoother="ilu0_rb", outer="gmres", restart=40))
    o = O.Oracle(prob, parts, smoother="ilu0_rb")
    g.update_basis(max_sweeps=30, tol=0.0)
    o.update_basis(max_sweeps=30, tol=0.0)
    for k in (1, 3, 8, 35):
        p = dev(np.zeros(prob.n_cells))
        it, rel, rc = g.solve(p, rtol=0.0, max_iters=k)
        xo, ito, relo, st = o.solve_gmres(rtol=0.0, restart=40, max_iters=k)
        say(f"GMRES(40) {k} steps: relres gpu {rel:.3e} oracle {relo:.3e}")
        assert it == ito == k
        assert rel == pytest.approx(relo, rel=1e-6)
        assert relerr(host(p), xo) <= 1e-7
    p = dev(np.zeros(prob.n_cells))
    it, rel, rc = g.solve(p, rtol=1e-10, max_iters=2000)
    assert rc == capi.OK
    assert np.linalg.norm(o.residual(host(p))) / np.linalg.norm(o.b) <= 1.0001e-10


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gmres_restart_above_dcgs2_limit_converges(capi, precision):
    prob = make_config2(dims=(18, 30, 12), seed=2)
    parts = [{"kind": "cartesian", "coarse_dims": (3, 3, 2)}, {"kind": "fault_cut", "parent": 0}]
    g = capi.Solver(prob, parts, capi.default_options(smoother="ilu0_rb", outer="gmres", restart=48,
                                                       precision=precision))
    o = O.Oracle(prob, parts)
    g.update_basis(max_sweeps=40, tol=1e-3)
    p = dev(np.zeros(prob.n_cells))
    it, rel, rc = g.solve(p, rtol=1e-8, max_iters=2000)
    true = np.linalg.norm(o.residual(host(p))) / np.linalg.norm(o.b)
    say(f"GMRES(48) {precision}: {it} iterations, true relres {true:.2e}")
    assert rc == capi.OK and true <= 1.0001e-8


# --------------------------------------------------- dynamic-block cap ----

def test_dynamic_cap_halves_bins_on_device(capi):
    prob = make_config0(4)
    parts = [{"kind": "cartesian", "coarse_dims": (6, 6, 1)}]
    dp = np.random.default_rng(3).standard_normal(prob.n_cells)
    o = O.Oracle(prob, parts)
    _, M4, _ = O.dynamic_partition(prob, dp, o.stages[0].block, n_bins=4, max_blocks=10 ** 9)
    for cap in (M4, M4 - 1, 100):
        g = capi.Solver(prob, parts, capi.default_options(max_dyn_blocks=cap))
        g.update_basis(max_sweeps=5, tol=0.0)
        oc = O.Oracle(prob, parts, max_dyn_blocks=cap)
        oc.update_basis(max_sweeps=5, tol=0.0)
        counts = g.add_dynamic_basis([dev(dp)])
        assert counts == oc.add_dynamic_basis([dp])
        e = g.export_stage(1)
        say(f"cap {cap}: {counts[0]} blocks")
        assert counts[0] <= cap and np.array_equal(e["block"], oc.dyn[0].block)
        assert relerr(e["Ac"], oc.dyn[0].Ac) <= 1e-12
    # with one bin the 36 general blocks are 36 pieces: a cap of 35 is an error
    # on both sides, and the context keeps no dynamic stage
    g = capi.Solver(prob, parts, capi.default_options(n_bins=1, max_dyn_blocks=35))
    g.update_basis(max_sweeps=5, tol=0.0)
    with pytest.raises(capi.MsrsbError) as e:
        g.add_dynamic_basis([dev(dp)])
    assert e.value.code == capi.E_INVAL
    with pytest.raises(O.OracleError):
        O.dynamic_partition(prob, dp, o.stages[0].block, n_bins=1, max_blocks=35)
    assert g.num_stages() == 1
    p = dev(np.zeros(prob.n_cells))
    it, rel, rc = g.solve(p, rtol=1e-4, max_iters=3000)
    assert rc == capi.OK


# ------------------------------------------------------ argument checks ----

def test_wrong_vectors_rejected(capi):
    prob = make_config0(0)
    g = capi.Solver(prob, [{"kind": "cartesian", "coarse_dims": (6, 6, 1)}])
    g.update_basis(max_sweeps=5, tol=0.0)
    short = dev(np.zeros(prob.n_cells - 1))
    for call in (lambda: g.solve(short), lambda: g.apply(capi.OP_RESIDUAL, short),
                 lambda: g.add_dynamic_basis([short]), lambda: g.fluxes(short),
                 lambda: g.solve(dev(np.zeros(prob.n_cells)), source=short)):
        with pytest.raises(capi.MsrsbError) as e:
            call()
        assert e.value.code == capi.E_INVAL
    with pytest.raises(capi.MsrsbError):
        g.coarse_apply(0, np.zeros(35))
    with pytest.raises(capi.MsrsbError) as e:
        g.coarse_apply(3, np.zeros(36))
    assert e.value.code == capi.E_INVAL
