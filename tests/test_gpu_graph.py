"""GPU parity of GRAPH stages (partitions given as a block id per cell:
graph partitions, well partitions and indicator agglomerations; types
"General" and "Static" of the subsection "Iterative multiscale multibasis
solver") against the CPU oracle: structure bit-exact, basis entries within
1e-12, coarse operators within 1e-12 of their largest entry, fixed cycle
counts within 1e-9, solves to the tolerance on the oracle's residual; in
mixed precision the basis within the BF16 bound and the coarse operator the
FP64 Galerkin product of the stored basis (1e-12)."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from workloads import make_config1, make_config2, make_lognormal_box, rng_for

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


def _random_ids(prob):
    rng = np.random.default_rng(5)
    # blocks of 3x3x2 boxes with randomly merged neighbours: irregular, some ids unused
    nx, ny, nz = prob.dims
    i = np.arange(prob.n_cells)
    box = (i % nx) // 3 + 100 * (((i // nx) % ny) // 3) + 10000 * ((i // (nx * ny)) // 2)
    remap = {b: int(rng.integers(0, 40)) * 7 for b in np.unique(box)}
    return np.array([remap[b] for b in box])


def _wells(prob):
    w = [prob.wells["injector"]]
    prod = prob.wells["producers"]
    nz = prob.dims[2]
    w += [prod[k * (prod.size // 4):(k + 1) * (prod.size // 4)] for k in range(4)]
    return w


GCASES = {
    "random_ids": (lambda: make_config2(dims=(15, 18, 8), seed=6), lambda c, p: _random_ids(p), 2),
    "wells": (lambda: make_config1(dims=(16, 24, 8), seed=2), lambda c, p: c.partition_wells(p, _wells(p), 2), 3),
    "indicator": (lambda: make_lognormal_box((20, 16, 6), rng_for(9, 3), sigma=2.0, corr=(3.0, 3.0, 1.0)),
                  lambda c, p: c.partition_indicator(p, np.log(p.perm), 4, (2, 2, 1), 8), 2),
    "constant": (lambda: make_config2(dims=(12, 10, 6), seed=7), lambda c, p: _random_ids(p), 0),
}


def build(capi, name, smoother="jacobi", outer="richardson", precision="fp64"):
    mk, ids_of, overlap = GCASES[name]
    prob = mk()
    ids = ids_of(capi, prob)
    parts = [{"kind": "cartesian", "coarse_dims": (2, 3, 2)},
             {"kind": "graph", "block_of_cell": ids, "overlap": overlap}]
    say(f"graph case {name} dims={prob.dims} overlap={overlap} smoother={smoother} outer={outer} {precision}")
    g = capi.Solver(prob, parts, capi.default_options(smoother=smoother, outer=outer, precision=precision))
    o = O.Oracle(prob, parts, smoother=smoother)
    return prob, g, o


@pytest.mark.parametrize("name", list(GCASES))
def test_graph_structure(capi, name):
    prob, g, o = build(capi, name)
    M, kind, ns = g.stage_info(1)
    st = o.stages[1]
    assert kind == capi.PART_GRAPH and M == st.M
    e = g.export_stage(1, values=False, coarse=False)
    assert np.array_equal(e["block"], np.where(prob.active, st.block, -1))
    sb = e["slot_block"]
    got = {(i, int(b)) for s in range(ns) for i, b in zip(np.nonzero(sb[s] >= 0)[0].tolist(),
                                                         sb[s][sb[s] >= 0].tolist())}
    S = st.S.tocoo()
    want = {(int(o.cells[r]), int(c)) for r, c in zip(S.row, S.col)}
    assert got == want
    g.close()


@pytest.mark.parametrize("name", list(GCASES))
@pytest.mark.parametrize("sweeps", [0, 1, 7, 30])
def test_graph_basis_and_coarse(capi, name, sweeps):
    prob, g, o = build(capi, name)
    g.update_basis(max_sweeps=sweeps, tol=0.0)
    o.update_basis(max_sweeps=sweeps, tol=0.0)
    for k in (0, 1):
        assert np.abs(g.dense_basis(k) - o.export_basis(k)).max() <= 1e-12
        assert relerr(g.export_stage(k)["Ac"], o.stages[k].Ac) <= 1e-12
    g.close()


@pytest.mark.parametrize("name", ["random_ids", "wells", "indicator"])
@pytest.mark.parametrize("smoother", ["jacobi", "ilu0_rb"])
def test_graph_cycles(capi, name, smoother):
    prob, g, o = build(capi, name, smoother=smoother)
    g.update_basis(max_sweeps=20, tol=0.0)
    o.update_basis(max_sweeps=20, tol=0.0)
    p = dev(np.zeros(prob.n_cells))
    it, rel, rc = g.solve(p, rtol=0.0, max_iters=6)
    xo, cyc, relo, st = o.solve(rtol=0.0, max_cycles=6)
    assert it == cyc == 6 and relerr(host(p), xo) <= 1e-9
    g.close()


@pytest.mark.parametrize("name", ["random_ids", "wells", "indicator"])
def test_graph_gmres_converges(capi, name):
    prob, g, o = build(capi, name, smoother="ilu0_rb", outer="gmres")
    g.update_basis(max_sweeps=60, tol=1e-3)
    p = dev(np.zeros(prob.n_cells))
    it, rel, rc = g.solve(p, rtol=1e-10, max_iters=1000)
    assert rc == capi.OK
    x = host(p)
    assert np.linalg.norm(o.residual(x)) / np.linalg.norm(o.b) <= 1.0001e-10
    assert relerr(x, o.direct_solve()) <= 1e-7
    g.close()


@pytest.mark.parametrize("name", ["random_ids", "wells", "indicator"])
def test_graph_mixed(capi, name):
    prob, g, o = build(capi, name, smoother="ilu0_rb", outer="gmres", precision="mixed")
    g.update_basis(max_sweeps=15, tol=0.0)
    o.update_basis(max_sweeps=15, tol=0.0)
    for k in (0, 1):
        P = g.dense_basis(k)
        Po = o.export_basis(k)
        assert np.all(np.abs(P - Po) <= 2.0 ** -8 * np.abs(Po) + 2e-5)
        # the coarse operator is the FP64 Galerkin product of the stored BF16 basis
        Pb = sp.csr_matrix(P[o.cells])
        assert relerr(g.export_stage(k)["Ac"], O.galerkin(Pb, o.A)) <= 1e-12
    p = dev(np.zeros(prob.n_cells))
    it, rel, rc = g.solve(p, rtol=1e-6, max_iters=2000)
    assert rc == capi.OK
    assert np.linalg.norm(o.residual(host(p))) / np.linalg.norm(o.b) <= 1.0001e-6
    g.close()


def test_graph_errors(capi):
    prob = make_config1(dims=(10, 12, 4), seed=1)
    ids = np.zeros(prob.n_cells, np.int32)
    ids[3] = -2
    say("graph error paths")
    with pytest.raises(capi.MsrsbError) as ei:
        capi.Solver(prob, [{"kind": "cartesian", "coarse_dims": (2, 2, 1)},
                           {"kind": "graph", "block_of_cell": ids, "overlap": 1}])
    assert ei.value.code == capi.E_INVAL
    # one block per cell and a wide overlap: more than 32 supports hold a cell
    with pytest.raises(capi.MsrsbError) as ei:
        capi.Solver(prob, [{"kind": "cartesian", "coarse_dims": (2, 2, 1)},
                           {"kind": "graph", "block_of_cell": np.arange(prob.n_cells), "overlap": 3}])
    assert ei.value.code == capi.E_INVAL
    # GRAPH cannot be the first (general) stage
    with pytest.raises(capi.MsrsbError):
        capi.Solver(prob, [{"kind": "graph", "block_of_cell": np.zeros(prob.n_cells), "overlap": 1}])


def test_graph_long_coarse_rows(capi):
    # one block per cell on 8,640 cells: coarse rows of 8,640 entries, longer
    # than the Galerkin kernel keeps in LDS, so the rows are summed in memory
    prob = make_lognormal_box((24, 24, 15), rng_for(9, 4), sigma=1.0)
    ids = np.arange(prob.n_cells)
    parts = [{"kind": "cartesian", "coarse_dims": (2, 2, 1)}, {"kind": "graph", "block_of_cell": ids, "overlap": 1}]
    say(f"graph long rows dims={prob.dims} M={prob.n_cells}")
    g = capi.Solver(prob, parts, capi.default_options())
    o = O.Oracle(prob, parts, smoother="jacobi")
    g.update_basis(max_sweeps=2, tol=0.0)
    o.update_basis(max_sweeps=2, tol=0.0)
    M, kind, ns = g.stage_info(1)
    assert M == prob.n_cells and 8 * M > 65536
    A = g.export_stage(1)["Ac"]
    assert relerr(A, o.stages[1].Ac) <= 1e-12
    g.close()
