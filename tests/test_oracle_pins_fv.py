"""Pins of the oracle's finite-volume restriction and conservative flux
reconstruction (section "Multiscale methods": a restriction that sums the
cells of each block when fine-scale fluxes are needed) against what the
definitions and the mathematics fix: mass balance of every cell and of every
block, the coarse two-point operator for constant bases, exactness when every
cell is its own block."""
import numpy as np
import pytest

import oracle as O
from workloads import make_config1, make_config2, make_lognormal_box, rng_for


def coarse_tpfa(prob, block, M):
    """Coarse two-point operator of a partition by a loop over the faces."""
    nx, ny = prob.dims[0], prob.dims[1]
    Ac = np.zeros((M, M))
    for T, step in ((prob.tx, 1), (prob.ty, nx), (prob.tz, nx * ny)):
        for i in np.nonzero(T)[0]:
            j, k = block[i], block[i + step]
            if j != k:
                Ac[j, k] -= T[i]
                Ac[k, j] -= T[i]
                Ac[j, j] += T[i]
                Ac[k, k] += T[i]
    for c, t in zip(prob.bc_cell, prob.bc_trans):
        Ac[block[c], block[c]] += t
    return Ac


CASES = [
    (lambda: make_config1(dims=(12, 14, 6), seed=1), [{"kind": "cartesian", "coarse_dims": (3, 2, 2)}]),
    (lambda: make_config2(dims=(12, 12, 6), seed=2),
     [{"kind": "cartesian", "coarse_dims": (2, 2, 2)}, {"kind": "fault_cut", "parent": 0}]),
    (lambda: make_lognormal_box((16, 10, 3), rng_for(9, 4), sigma=2.0, corr=(2, 2, 1)),
     [{"kind": "cartesian", "coarse_dims": (4, 2, 1)}]),
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("sweeps", [0, 3, 25])
def test_fv_every_cell_and_block_balances(case, sweeps):
    mk, parts = CASES[case]
    prob = mk()
    o = O.Oracle(prob, parts)
    o.update_basis(max_sweeps=sweeps, tol=0.0)
    qscale = np.abs(o.b).max()
    for k in range(len(parts)):
        pms, pf, face, bcf, Afv = o.solve_fv(stage=k)
        # every cell: outflow - q = 0 (the conservative fluxes)
        imb = O.cell_imbalance(prob, face, bcf)
        assert np.abs(imb).max() <= 1e-10 * qscale
        # every block: the fluxes of p_ms through its boundary balance its sources
        st = o.stages[k]
        r = o.b - o.A @ pms[o.cells]
        for j in range(st.M):
            assert abs(r[st.block[o.cells] == j].sum()) <= 1e-10 * qscale
        # fluxes between blocks come from p_ms, fluxes inside blocks from p'
        nx, ny = prob.dims[0], prob.dims[1]
        for d, (T, step) in enumerate(((prob.tx, 1), (prob.ty, nx), (prob.tz, nx * ny))):
            a = np.nonzero(T)[0]
            cross = st.block[a] != st.block[a + step]
            assert np.allclose(face[d, a[cross]], T[a[cross]] * (pms[a[cross]] - pms[a[cross] + step]), rtol=0,
                               atol=1e-14 * qscale)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_fv_constant_basis_is_coarse_tpfa(case):
    mk, parts = CASES[case]
    prob = mk()
    o = O.Oracle(prob, parts)
    o.update_basis(max_sweeps=0, tol=0.0)
    for k in range(len(parts)):
        *_, Afv = o.solve_fv(stage=k)
        st = o.stages[k]
        ref = coarse_tpfa(prob, st.block, st.M)
        assert np.abs(Afv - ref).max() <= 1e-13 * np.abs(ref).max()
        assert np.abs(Afv - st.Ac).max() <= 1e-13 * np.abs(ref).max()  # R_fv = P^T for a constant basis


def test_fv_every_cell_its_own_block_is_exact():
    prob = make_config2(dims=(7, 6, 4), seed=3)
    ids = np.arange(prob.n_cells)
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (2, 2, 1)},
                        {"kind": "graph", "block_of_cell": ids, "overlap": 0}])
    o.update_basis(max_sweeps=4, tol=0.0)
    pms, pf, face, bcf, _ = o.solve_fv(stage=1)
    xd = o.direct_solve()
    assert np.abs(pms - xd).max() <= 1e-12 * np.abs(xd).max()
    assert np.abs(pf - xd).max() <= 1e-12 * np.abs(xd).max()
    fd, bd = O.fluxes(prob, xd)
    assert np.abs(face - fd).max() <= 1e-11 * np.abs(fd).max()
    assert np.abs(bcf - bd).max() <= 1e-11 * np.abs(bd).max()


def test_fv_unanchored_blocks_keep_the_block_sum():
    # blocks without a boundary term: p' is fixed up to a constant, chosen with the sum of p_ms
    mk, parts = CASES[0]
    prob = mk()
    o = O.Oracle(prob, parts)
    o.update_basis(max_sweeps=10, tol=0.0)
    pms, pf, *_ = o.solve_fv(stage=0)
    st = o.stages[0]
    bc = np.zeros(prob.n_cells)
    np.add.at(bc, prob.bc_cell, prob.bc_trans)
    for j in range(st.M):
        I = np.nonzero(st.block == j)[0]
        if not np.any(bc[I] > 0):
            assert abs(pf[I].sum() - pms[I].sum()) <= 1e-10 * np.abs(pms[I]).sum()
