"""GPU parity of the finite-volume mode (msrsb_solve_fv: restriction that sums
each block, section "Multiscale methods", and conservative fine fluxes)
against the oracle: multiscale pressure within 1e-10 relative (the coarse
system is solved by an explicit inverse on the GPU and by LU in the oracle:
kappa(A_fv) eps), fluxes within 1e-8 of the largest flux (local conjugate
gradients to 1e-13), every cell's imbalance within 1e-9 of the largest
source term.  Mixed precision: against the oracle on the stored BF16 basis."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from workloads import make_config1, make_config2

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


def relerr(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _wells(prob):
    prod = prob.wells["producers"]
    return [prob.wells["injector"]] + [prod[k * (prod.size // 4):(k + 1) * (prod.size // 4)] for k in range(4)]


FCASES = {
    "layered": (lambda: make_config1(dims=(20, 24, 10), seed=2), lambda c, p: [
        {"kind": "cartesian", "coarse_dims": (3, 3, 2)}]),
    "faulted": (lambda: make_config2(dims=(16, 18, 8), seed=3), lambda c, p: [
        {"kind": "cartesian", "coarse_dims": (2, 3, 2)}, {"kind": "fault_cut", "parent": 0}]),
    "indicator": (lambda: make_config1(dims=(16, 20, 8), seed=5), lambda c, p: [
        {"kind": "cartesian", "coarse_dims": (2, 2, 2)},
        {"kind": "graph", "block_of_cell": c.partition_indicator(p, np.log(p.perm), 3, (2, 3, 2), 16),
         "overlap": 2}]),
    # blocks that are single columns (most of them without a boundary term:
    # singular Neumann chains) for the z-line preconditioned local solves
    "columns": (lambda: make_config1(dims=(6, 5, 12), seed=8), lambda c, p: [
        {"kind": "cartesian", "coarse_dims": (6, 5, 2)}]),
    # one block of 3,840 cells: above the z-line local solver's 2,304-cell
    # limit, solved by the Jacobi-preconditioned kernel
    "large_block": (lambda: make_config1(dims=(24, 20, 8), seed=7), lambda c, p: [
        {"kind": "cartesian", "coarse_dims": (1, 1, 1)}]),
}


def check_stage(capi, prob, g, o, k, precision):
    st = o.stages[k]
    bl = st.block[o.cells]
    if precision == "fp64":
        P = st.P
    else:
        P = sp.csr_matrix(g.dense_basis(k)[o.cells])  # the stored BF16 basis
    pms_o, _ = O.fv_multiscale_pressure(P, o.A, o.b, bl, st.M)
    bcd = np.zeros(prob.n_cells)
    np.add.at(bcd, prob.bc_cell, prob.bc_trans)
    pf_o = O.conservative_pressure(o.A, o.b, bl, st.M, pms_o, bcd[o.cells])
    face_o, bcf_o = O.reconstructed_fluxes(prob, o.cells, bl, pms_o, pf_o)
    p, pf, face, bcf, its, imb = g.solve_fv(stage=k, local_rtol=1e-13, max_local_iters=20000)
    p, face, bcf = host(p), host(face), host(bcf)
    say(f"  stage {k}: M={st.M} local CG steps {its}, max imbalance {imb:.2e}")
    assert relerr(p[o.cells], pms_o) <= 1e-10
    fscale = max(np.abs(face_o).max(), np.abs(bcf_o).max())
    assert np.abs(face - face_o).max() <= 1e-8 * fscale
    assert np.abs(bcf - bcf_o).max() <= 1e-8 * fscale
    qscale = np.abs(o.b).max()
    mine = np.abs(O.cell_imbalance(prob, face, bcf)).max()
    assert imb <= 1e-9 * qscale and mine <= 1e-9 * qscale and abs(mine - imb) <= 1e-12 * qscale + 1e-3 * imb


@pytest.mark.parametrize("name", list(FCASES))
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fv_matches_oracle(capi, name, precision):
    mk, parts_of = FCASES[name]
    prob = mk()
    parts = parts_of(capi, prob)
    say(f"fv case {name} dims={prob.dims} {precision}")
    g = capi.Solver(prob, parts, capi.default_options(precision=precision))
    o = O.Oracle(prob, parts)
    g.update_basis(max_sweeps=15, tol=0.0)
    o.update_basis(max_sweeps=15, tol=0.0)
    for k in range(len(parts)):
        check_stage(capi, prob, g, o, k, precision)
    g.close()


def test_fv_follows_basis_and_source_changes(capi):
    prob = make_config1(dims=(16, 18, 8), seed=6)
    parts = [{"kind": "cartesian", "coarse_dims": (2, 3, 2)}]
    say("fv after a basis update and a source change")
    g = capi.Solver(prob, parts)
    o = O.Oracle(prob, parts)
    g.update_basis(max_sweeps=3, tol=0.0)
    o.update_basis(max_sweeps=3, tol=0.0)
    check_stage(capi, prob, g, o, 0, "fp64")
    g.update_basis(max_sweeps=40, tol=0.0)  # the FV operator is rebuilt for the new basis
    o.update_basis(max_sweeps=40, tol=0.0)
    check_stage(capi, prob, g, o, 0, "fp64")
    q = prob.source.copy()
    q[prob.n_cells // 2] += 0.3
    q[prob.n_cells // 3] -= 0.3
    p, pf, face, bcf, its, imb = g.solve_fv(stage=0, source=dev(q), local_rtol=1e-13, max_local_iters=20000)
    b = O.msrsb.rhs_for(prob, o.cells, q)
    st = o.stages[0]
    pms_o, _ = O.fv_multiscale_pressure(st.P, o.A, b, st.block[o.cells], st.M)
    assert relerr(host(p)[o.cells], pms_o) <= 1e-10
    mine = O.cell_imbalance(prob, host(face), host(bcf), source=q)
    assert np.abs(mine).max() <= 1e-9 * np.abs(b).max()
    g.close()


def test_fv_errors(capi):
    prob = make_config1(dims=(10, 12, 4), seed=1)
    g = capi.Solver(prob, [{"kind": "cartesian", "coarse_dims": (2, 2, 1)}])
    say("fv error paths")
    with pytest.raises(capi.MsrsbError) as ei:
        g.solve_fv(stage=0)
    assert ei.value.code == capi.E_STATE
    g.update_basis(max_sweeps=2, tol=0.0)
    with pytest.raises(capi.MsrsbError) as ei:
        g.solve_fv(stage=1)
    assert ei.value.code == capi.E_INVAL
    g.close()
    # blocks above the local-solve limit
    big = make_config1(dims=(40, 40, 8), seed=1)
    g = capi.Solver(big, [{"kind": "cartesian", "coarse_dims": (1, 1, 1)}])
    g.update_basis(max_sweeps=1, tol=0.0)
    with pytest.raises(capi.MsrsbError) as ei:
        g.solve_fv(stage=0)
    assert ei.value.code == capi.E_INVAL
    g.close()
