"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these compare the oracle with itself: each checks a closed form, a
hand-worked example (``tests/golden``), a definition-level invariant, a
special case that reduces to a textbook/library routine, or brute force on a
tiny input written independently of the oracle's code.
"""
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as O
from oracle.msrsb import support_1d, rhs_for
from workloads import Problem, make_config0, make_config1, make_config2, make_homogeneous, make_lognormal_box, rng_for
from workloads.grids import face_transmissibility, half_transmissibility

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
EPS = np.finfo(np.float64).eps


def chain(T, bc_left=1.0):
    """1-D chain of len(T)+1 cells with given face transmissibilities and one
    Dirichlet face on cell 0 (keeps A nonsingular; A_b ignores it)."""
    n = len(T) + 1
    tx = np.zeros(n)
    tx[:-1] = T
    z = np.zeros(n)
    return Problem((n, 1, 1), (1.0, 1.0, 1.0), np.ones(n, bool), tx, z.copy(), z.copy(),
                   np.array([0], np.int32), np.array([bc_left]), np.array([1.0]), np.zeros(n), np.ones(n),
                   np.zeros((3, n), np.uint8), "chain")


# ----------------------------------------------------------------- TPFA ----

def test_two_cell_transmissibility_by_hand():
    # K = (1, 3), dx = 2, unit face: half transmissibilities K*1/(2/2) = K,
    # harmonic combination 1/(1/1 + 1/3) = 3/4; Dirichlet face keeps t = K.
    perm = np.array([1.0, 3.0])
    tx, ty, tz = face_transmissibility(perm, (2, 1, 1), (2.0, 1.0, 1.0), np.ones(2, bool))
    assert tx[0] == pytest.approx(0.75, rel=1e-15) and tx[1] == 0.0
    assert not ty.any() and not tz.any()
    assert half_transmissibility(perm, (2, 1, 1), (2.0, 1.0, 1.0), 0)[1] == 3.0


@pytest.mark.parametrize("dims", [(8, 5, 1), (6, 4, 3), (16, 1, 1)])
def test_tpfa_homogeneous_linear_pressure_closed_form(dims):
    # Homogeneous K with p=1 on x=0 and p=0 on x=Lx: the two-point scheme
    # reproduces p(x) = 1 - x/Lx exactly at the cell centres.
    prob = make_homogeneous(dims, h=(2.0, 1.0, 0.5), K=3.0)
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (2, 1, 1)}])
    x = o.direct_solve()
    nx = dims[0]
    xc = (np.arange(prob.n_cells) % nx + 0.5) / nx
    np.testing.assert_allclose(x, 1.0 - xc, rtol=0, atol=1e-13)


def test_tpfa_structure():
    prob = make_config0(3)
    A, b, Ab, cells = O.assemble(prob)
    assert abs(A - A.T).max() == 0.0
    rowsum = A @ np.ones(A.shape[0])
    bc_rows = np.zeros(A.shape[0], bool)
    bc_rows[prob.bc_cell] = True
    assert np.all(rowsum[~bc_rows] == 0.0) or np.abs(rowsum[~bc_rows]).max() < 1e-13
    assert np.all(rowsum[bc_rows] > 0)
    assert np.abs(Ab @ np.ones(A.shape[0])).max() < 1e-13
    # M-matrix sign pattern
    off = A - sp.diags(A.diagonal())
    assert off.max() <= 0.0
    # sparse LU, dense solve and CG agree
    x1 = spla.spsolve(A.tocsc(), b)
    x2 = np.linalg.solve(A.toarray(), b)
    x3, info = spla.cg(A, b, rtol=1e-14, maxiter=10000)
    assert info == 0
    np.testing.assert_allclose(x1, x2, rtol=0, atol=1e-12)
    np.testing.assert_allclose(x3, x2, rtol=0, atol=1e-10)


def test_singular_component_rejected():
    prob = make_homogeneous((4, 1, 1))
    prob.bc_trans = np.zeros_like(prob.bc_trans)
    with pytest.raises(O.OracleError) as e:
        O.assemble(prob)
    assert e.value.code == O.msrsb.E_SINGULAR


def test_invalid_transmissibility_rejected():
    prob = make_homogeneous((4, 1, 1))
    prob.tx = prob.tx.copy()
    prob.tx[1] = -1.0
    with pytest.raises(O.OracleError):
        O.assemble(prob)
    prob.tx[1] = np.nan
    with pytest.raises(O.OracleError):
        O.assemble(prob)


# ---------------------------------------------------- partitions/supports ----

def test_support_1d_hand_examples():
    # n=15, m=3: blocks of 5, doubled centres 5, 15, 25.
    assert support_1d(15, 3) == [list(range(0, 7)), list(range(3, 12)), list(range(8, 15))]
    # n=8, m=2: doubled centres 4, 12.
    assert support_1d(8, 2) == [list(range(0, 6)), list(range(2, 8))]
    # n=10, m=3: edges 0,4,7,10 (ceil), doubled centres 4, 11, 17.
    assert support_1d(10, 3) == [list(range(0, 5)), list(range(2, 8)), list(range(6, 10))]
    # one block per cell: supports collapse to the cell itself
    assert support_1d(5, 5) == [[i] for i in range(5)]
    # one block: everything
    assert support_1d(7, 1) == [list(range(7))]


@pytest.mark.parametrize("dims,cd", [((13, 9, 1), (3, 2, 1)), ((10, 7, 6), (3, 2, 2)), ((11, 11, 5), (4, 3, 2))])
def test_support_invariants(dims, cd):
    active = np.ones(int(np.prod(dims)), bool)
    block, M, present = O.cartesian_partition(dims, cd, active)
    S = O.cartesian_support(dims, cd, active, present)
    # requirement 2: Omega_j inside S_j
    assert np.all(S[np.arange(block.size), block].A1 == 1)
    # at most 2^dim overlapping supports per cell, at least one
    cnt = np.asarray(S.sum(axis=1)).ravel()
    dimc = sum(1 for m in cd if m > 1)
    assert cnt.min() >= 1 and cnt.max() <= 2 ** dimc
    # partition blocks have floor(i m / n) sizes
    sizes = np.bincount(block, minlength=M)
    assert sizes.sum() == block.size


def test_partition_drops_empty_blocks():
    dims = (6, 2, 1)
    active = np.ones(12, bool)
    active[[0, 1, 6, 7]] = False  # kills Cartesian block (0,0) of a 3x1 coarse grid
    block, M, present = O.cartesian_partition(dims, (3, 1, 1), active)
    assert M == 2 and list(present) == [1, 2]
    assert list(block[[2, 3, 4, 5]]) == [0, 0, 1, 1] and block[0] == -1


# ------------------------------------------------------------------ MsRSB ----

def _load_golden():
    rows, change = {}, {}
    with open(os.path.join(GOLDEN, "msrsb_1d_two_sweeps.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            t = line.split()
            if t[0] == "change":
                change[int(t[1])] = Fraction(int(t[2]), int(t[3]))
            else:
                s, i = int(t[0]), int(t[1])
                rows[(s, i)] = (Fraction(int(t[2]), int(t[3])), Fraction(int(t[4]), int(t[5])))
    return rows, change


@pytest.mark.parametrize("sweeps", [1, 2])
def test_msrsb_hand_worked_example(sweeps):
    rows, change = _load_golden()
    prob = chain([1.0, 2.0, 3.0])
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (2, 1, 1)}])
    o.update_basis(max_sweeps=sweeps, tol=0.0)
    P = o.export_basis(0)
    for i in range(4):
        exp = rows[(sweeps, i)]
        assert P[i, 0] == pytest.approx(float(exp[0]), abs=4 * EPS)
        assert P[i, 1] == pytest.approx(float(exp[1]), abs=4 * EPS)
    assert o.stages[0].change == pytest.approx(float(change[sweeps]), abs=4 * EPS)


def test_msrsb_zero_sweeps_is_indicator():
    prob = make_config0(1)
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (6, 6, 1)}])
    o.update_basis(max_sweeps=0, tol=0.0)
    P = o.export_basis(0)
    block = o.stages[0].block
    assert np.array_equal(P, np.eye(36)[block])


def test_msrsb_single_block_is_one():
    prob = make_lognormal_box((7, 5, 3), rng_for(9, 0), sigma=1.0)
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (1, 1, 1)}])
    for s in (1, 5, 20):
        o.update_basis(max_sweeps=s, tol=0.0)
        assert np.all(o.export_basis(0) == 1.0)


def test_msrsb_one_block_per_cell_is_identity():
    prob = make_lognormal_box((5, 4, 2), rng_for(9, 1), sigma=1.0)
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (5, 4, 2)}])
    o.update_basis(max_sweeps=7, tol=0.0)
    assert np.array_equal(o.export_basis(0), np.eye(40))


@pytest.mark.parametrize("sweeps", [1, 5, 50])
def test_msrsb_partition_of_unity_and_support(sweeps):
    prob = make_lognormal_box((12, 10, 4), rng_for(9, 2), sigma=2.0)
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (3, 2, 2)}])
    o.update_basis(max_sweeps=sweeps, tol=0.0)
    P = o.export_basis(0)
    S = o.stages[0].S.toarray()
    assert np.abs(P.sum(axis=1) - 1.0).max() <= 8 * EPS
    assert np.all(P[S == 0] == 0.0)
    assert P.min() >= -1e-12


def test_msrsb_converges_to_linear_hats_in_1d():
    # Homogeneous 1-D chain, blocks of odd width: the fixed point of restricted
    # smoothing is the piecewise-linear hat through the block-centre cells.
    prob = make_homogeneous((15, 1, 1))
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (3, 1, 1)}])
    o.update_basis(max_sweeps=5000, tol=1e-15)
    P = o.export_basis(0)
    i = np.arange(15)
    hat1 = np.clip(1.0 - np.abs(i - 7) / 5.0, 0.0, 1.0)
    hat0 = np.where(i <= 2, 1.0, np.clip(1.0 - (i - 2) / 5.0, 0.0, 1.0))
    hat2 = hat0[::-1]
    np.testing.assert_allclose(P[:, 1], hat1, atol=1e-12)
    np.testing.assert_allclose(P[:, 0], hat0, atol=1e-12)
    np.testing.assert_allclose(P[:, 2], hat2, atol=1e-12)


def test_msrsb_mirror_symmetry():
    prob = make_homogeneous((12, 10, 1))
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (3, 2, 1)}])
    o.update_basis(max_sweeps=30, tol=0.0)
    P = o.export_basis(0).reshape(10, 12, 6)  # (y, x, block)
    # block (Jx, Jy) mirrored in x maps to (2-Jx, Jy)
    mirror_blocks = [2, 1, 0, 5, 4, 3]
    np.testing.assert_allclose(P[:, ::-1, :][:, :, mirror_blocks], P, atol=1e-14)


def test_msrsb_brute_force_dense_loops():
    # Independent per-entry loops over cells, blocks and neighbours on a tiny
    # heterogeneous grid, compared at fixed sweep counts.
    prob = make_lognormal_box((6, 5, 2), rng_for(9, 3), sigma=1.5)
    cd = (2, 2, 1)
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": cd}])
    nx, ny, nz = prob.dims
    N = prob.n_cells
    nbrs = [[] for _ in range(N)]
    for i in range(N):
        if prob.tx[i] > 0:
            nbrs[i].append((i + 1, prob.tx[i])); nbrs[i + 1].append((i, prob.tx[i]))
        if prob.ty[i] > 0:
            nbrs[i].append((i + nx, prob.ty[i])); nbrs[i + nx].append((i, prob.ty[i]))
        if prob.tz[i] > 0:
            nbrs[i].append((i + nx * ny, prob.tz[i])); nbrs[i + nx * ny].append((i, prob.tz[i]))
    S = o.stages[0].S.toarray()
    M = S.shape[1]
    P = np.zeros((N, M))
    P[np.arange(N), o.stages[0].block] = 1.0
    for sweep in range(1, 6):
        Q = np.zeros_like(P)
        for i in range(N):
            d = sum(t for _, t in nbrs[i])
            for j in range(M):
                if not S[i, j]:
                    continue
                flow = sum(t * (P[i, j] - P[k, j]) for k, t in nbrs[i])
                Q[i, j] = P[i, j] - (2.0 / 3.0) * flow / d
        P = Q / Q.sum(axis=1, keepdims=True)
        o.update_basis(max_sweeps=sweep, tol=0.0)
        np.testing.assert_allclose(o.export_basis(0), P, atol=1e-14)


# --------------------------------------------------- Galerkin / coarse solve ----

def test_galerkin_identity_basis_is_fine_operator():
    prob = make_lognormal_box((4, 3, 2), rng_for(9, 4), sigma=1.0)
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (4, 3, 2)}])
    o.update_basis(max_sweeps=3, tol=0.0)
    np.testing.assert_array_equal(o.stages[0].Ac, o.A.toarray())


def test_galerkin_constant_basis_is_coarse_tpfa():
    # P = indicator: A_c[j,k] = -sum of face T between blocks j,k; diagonal =
    # sum of T over faces leaving j plus its boundary T.
    prob = make_config0(2)
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (6, 6, 1)}])
    o.update_basis(max_sweeps=0, tol=0.0)
    blk = o.stages[0].block
    nx = prob.dims[0]
    ref = np.zeros((36, 36))
    for i in range(prob.n_cells):
        for T, step in ((prob.tx[i], 1), (prob.ty[i], nx)):
            if T > 0:
                j, k = blk[i], blk[i + step]
                if j != k:
                    ref[j, k] -= T; ref[k, j] -= T; ref[j, j] += T; ref[k, k] += T
    for c, t in zip(prob.bc_cell, prob.bc_trans):
        ref[blk[c], blk[c]] += t
    np.testing.assert_allclose(o.stages[0].Ac, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


def test_galerkin_symmetry_and_row_sums():
    prob = make_config1(dims=(12, 16, 8), seed=1)
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (3, 2, 2)}])
    o.update_basis(max_sweeps=20, tol=0.0)
    st = o.stages[0]
    Ac = st.Ac
    scale = np.abs(Ac).max()
    assert np.abs(Ac - Ac.T).max() <= 1e-13 * scale
    np.testing.assert_allclose(Ac @ np.ones(st.M), st.P.T @ (o.A @ np.ones(o.A.shape[0])),
                               atol=1e-12 * scale)
    L = st.L
    np.testing.assert_allclose(L @ L.T, Ac, atol=1e-13 * scale)
    d = np.random.default_rng(0).standard_normal(st.M)
    pc = O.coarse_solve(L, d)
    # backward-stable solve: residual within a small multiple of eps ||A_c|| ||p_c||
    assert np.linalg.norm(Ac @ pc - d) <= 10 * st.M * EPS * np.linalg.norm(Ac, 2) * np.linalg.norm(pc)


# --------------------------------------------------------------- smoothers ----

def test_ilu0_on_chain_is_exact_lu():
    # Tridiagonal matrices have no fill: ILU(0) is the exact LU (Thomas).
    prob = chain([1.0, 2.0, 0.5, 4.0, 3.0, 1.5])
    A, b, _, cells = O.assemble(prob)
    fac = O.ilu0_factor(A, np.arange(A.shape[0]))
    r = np.random.default_rng(1).standard_normal(A.shape[0])
    e = O.ilu0_apply(fac, r)
    np.testing.assert_allclose(A @ e, r, atol=1e-13)


@pytest.mark.parametrize("order", ["natural", "red_black"])
def test_ilu0_matches_matrix_on_its_pattern(order):
    # Defining property of ILU(0): (L U)_ij = a_ij for every (i,j) in pattern(A).
    prob = make_lognormal_box((6, 5, 3), rng_for(9, 5), sigma=1.0)
    A, b, _, cells = O.assemble(prob)
    perm = O.natural_order(cells, prob.dims) if order == "natural" else O.red_black_order(cells, prob.dims)
    L, U, p = O.ilu0_factor(A, perm)
    B = A[p][:, p].tocoo()
    LU = (L @ U).toarray()
    np.testing.assert_allclose(LU[B.row, B.col], B.data, rtol=1e-13, atol=1e-13)
    assert np.all(np.diag(U.toarray()) > 0)


@pytest.mark.parametrize("case", ["box", "inactive"])
def test_ilu0_rb_fill_is_lu_minus_a(case):
    # Red-black ILU(0) differs from A exactly by the dropped black-black fill:
    # the textbook factor (itself pinned by its defining property above) must
    # satisfy L U - A = F entry by entry, so (A + F) e = r for e = ilu0_apply(r).
    if case == "box":
        prob = make_lognormal_box((7, 5, 4), rng_for(9, 6), sigma=1.5)
    else:
        prob = make_config2(dims=(8, 9, 5), seed=3)
    A, b, _, cells = O.assemble(prob)
    perm = O.red_black_order(cells, prob.dims)
    L, U, p = O.ilu0_factor(A, perm)
    inv = np.empty_like(p)
    inv[p] = np.arange(p.size)
    LU = (L @ U).tocsr()[inv][:, inv]
    F = O.ilu0_rb_fill(A, cells, prob.dims)
    assert abs(LU - A - F).max() <= 1e-13 * abs(A).max()
    assert F.nnz > 0
    r = np.random.default_rng(2).standard_normal(A.shape[0])
    e = O.ilu0_apply((L, U, p), r)
    np.testing.assert_allclose((A + F) @ e, r, atol=1e-12 * np.abs(r).max())


def test_red_black_order_colours():
    prob = make_homogeneous((4, 3, 2))
    cells = np.arange(prob.n_cells)
    order = O.red_black_order(cells, prob.dims)
    ix, iy, iz = cells % 4, (cells // 4) % 3, cells // 12
    col = (ix + iy + iz) % 2
    assert np.all(col[order[:12]] == 0) and np.all(col[order[12:]] == 1)
    assert np.all(np.diff(order[:12]) > 0) and np.all(np.diff(order[12:]) > 0)


# ------------------------------------------------------------------- cycle ----

def _energy(o, x, xs):
    e = (x - xs)[o.cells]
    return float(np.sqrt(e @ (o.A @ e)))


def test_cycle_galerkin_orthogonality_and_energy_decrease():
    prob = make_config1(dims=(12, 16, 8), seed=2)
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (3, 2, 2)}], smoother="jacobi")
    o.update_basis(max_sweeps=30, tol=0.0)
    st = o.stages[0]
    xs = o.direct_solve()
    x = np.zeros(o.cells.size)
    b = o.b
    xb = lambda v: np.concatenate([v])  # noqa: E731
    prev = None
    for _ in range(4):
        xh = x + o.smooth(b - o.A @ x)
        r = b - o.A @ xh
        xn = xh + st.P @ O.coarse_solve(st.L, st.P.T @ r)
        rn = b - o.A @ xn
        assert np.abs(st.P.T @ rn).max() <= 1e-11 * np.abs(st.P.T @ r).max()
        full = lambda v: np.bincount(o.cells, v, minlength=prob.n_cells)  # noqa: E731
        e0, e1, e2 = _energy(o, full(x), xs), _energy(o, full(xh), xs), _energy(o, full(xn), xs)
        assert e1 <= e0 * (1 + 1e-13) and e2 <= e1 * (1 + 1e-13)
        if prev is not None:
            assert e2 <= prev
        prev = e2
        x = xn


def test_cycle_with_identity_basis_converges_in_one_cycle():
    prob = make_lognormal_box((6, 5, 1), rng_for(9, 6), sigma=1.0)
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (6, 5, 1)}])
    o.update_basis(max_sweeps=1, tol=0.0)
    x, cycles, rel, status = o.solve(rtol=1e-12, max_cycles=5)
    assert cycles == 1 and rel <= 1e-13 and status == 0


@pytest.mark.parametrize("smoother", ["jacobi", "ilu0_nat", "ilu0_rb"])
def test_cycle_converges_to_direct_solution(smoother):
    prob = make_config0(0)
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (6, 6, 1)}], smoother=smoother)
    o.update_basis(max_sweeps=100, tol=1e-3)
    x, cycles, rel, status = o.solve(rtol=1e-10, max_cycles=2000)
    assert status == 0 and rel <= 1e-10
    xs = o.direct_solve()
    assert np.abs(x - xs).max() <= 1e-10 * 1e3 * np.abs(xs).max()


def test_noconv_returns_best_iterate():
    prob = make_config0(0)
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (6, 6, 1)}])
    o.update_basis(max_sweeps=10, tol=0.0)
    x, cycles, rel, status = o.solve(rtol=1e-12, max_cycles=1)
    assert status == O.msrsb.E_NOCONV and cycles == 1 and 0 < rel < 1


def test_solve_before_basis_is_state_error():
    o = O.Oracle(make_config0(0), [{"kind": "cartesian", "coarse_dims": (6, 6, 1)}])
    with pytest.raises(O.OracleError) as e:
        o.solve()
    assert e.value.code == O.msrsb.E_STATE


def test_mass_conservation_of_fluxes():
    prob = make_config1(dims=(12, 16, 8), seed=3)
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (3, 2, 2)}], smoother="ilu0_nat")
    o.update_basis(max_sweeps=50, tol=1e-3)
    x, cycles, rel, status = o.solve_gmres(rtol=1e-10, restart=30)
    assert status == 0
    flux, bcf = o.fluxes(x)
    nx, ny = prob.dims[0], prob.dims[1]
    net = flux[0] + flux[1] + flux[2]
    net[1:] -= flux[0][:-1]
    net[nx:] -= flux[1][:-nx]
    net[nx * ny:] -= flux[2][:-nx * ny]
    np.add.at(net, prob.bc_cell, bcf)
    r = np.zeros(prob.n_cells)
    r[o.cells] = o.residual(x)
    np.testing.assert_allclose(net - prob.source, -r, atol=1e-12 * np.abs(prob.source).max())
    nb = np.linalg.norm(o.b)
    assert abs(r.sum()) <= 1e-10 * nb * np.sqrt(o.cells.size)
    # global balance: injected = produced
    assert abs(prob.source.sum() + bcf.sum() * -1.0) <= 1e-8


def test_gmres_minimises_residual_over_krylov_space():
    # Definition of right-preconditioned GMRES: after k steps x_k minimises
    # ||b - A x|| over x0 + M^{-1} K_k(A M^{-1}, r0).  Brute force: build the
    # Krylov matrix explicitly (orthonormalised by a library QR) and solve the
    # least-squares problem with a library routine.
    prob = make_config1(dims=(12, 16, 8), seed=4)
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (3, 2, 2)}], smoother="ilu0_rb")
    o.update_basis(max_sweeps=30, tol=1e-3)
    x, its, rel, status, hist = o.solve_gmres(rtol=1e-14, restart=40, max_iters=8, history=True)
    b = o.b
    nb = np.linalg.norm(b)
    K = [b / nb]
    for k in range(1, 9):
        v = o.A @ o.precondition(K[-1])
        Q, _ = np.linalg.qr(np.column_stack(K + [v]))
        K = [Q[:, c] for c in range(Q.shape[1])]
        AMK = np.column_stack([o.A @ o.precondition(q) for q in K[:k]])
        y = np.linalg.lstsq(AMK, b, rcond=None)[0]
        best = np.linalg.norm(b - AMK @ y) / nb
        assert hist[k] == pytest.approx(best, rel=1e-7, abs=1e-15)
    # the returned iterate realises the last estimate
    assert rel == pytest.approx(np.linalg.norm(o.residual(x)) / nb, rel=1e-6)


def test_gmres_converges_to_direct_solution():
    prob = make_config1(dims=(12, 16, 8), seed=4)
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (3, 2, 2)}], smoother="ilu0_rb")
    o.update_basis(max_sweeps=30, tol=1e-3)
    x, its, rel, status = o.solve_gmres(rtol=1e-10, restart=20)
    assert status == 0 and rel <= 1e-10
    xd = o.direct_solve()
    assert np.abs(x - xd).max() <= 1e-6 * np.abs(xd).max()


# ------------------------------------------------------------ dynamic basis ----

def test_dynamic_partition_hand_example():
    # 1-D chain of 8 cells, one general block; |dp| = 8,8,1,1,0.25,0.25,8,0:
    # thresholds amax/4 = 2, amax/16 = 0.5, amax/64 = 0.125.
    # bins: 8 -> 0, 1 -> 1, 0.25 -> 2, 0 -> 3.  Pieces along the chain:
    # {0,1} bin0, {2,3} bin1, {4,5} bin2, {6} bin0, {7} bin3.
    prob = chain([1.0] * 7)
    general = np.zeros(8, np.int64)
    dp = np.array([8, -8, 1, 1, 0.25, -0.25, 8, 0.0])
    block, M, nb = O.dynamic_partition(prob, dp, general, n_bins=4)
    assert M == 5 and nb == 4
    assert list(block) == [0, 0, 1, 1, 2, 2, 3, 4]


def test_dynamic_partition_invariances_and_bruteforce():
    prob = make_config1(dims=(12, 16, 8), seed=5)
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (3, 2, 2)}])
    from workloads import pressure_increment_pair
    dp = pressure_increment_pair(prob, rng_for(9, 7))[0]
    g = o.stages[0].block
    block, M, nb = O.dynamic_partition(prob, dp, g)
    for scale in (-1.0, 2.0 ** 5, -(2.0 ** -7)):
        b2, M2, _ = O.dynamic_partition(prob, dp * scale, g)
        assert M2 == M and np.array_equal(b2, block)
    assert O.dynamic_partition(prob, np.zeros_like(dp), g) is None
    # each dynamic block lies inside one general block
    for j in range(M):
        assert np.unique(g[block == j]).size == 1
    # brute force: bins by repeated comparison, flood fill in cell order
    a = np.abs(dp)
    amax = a.max()
    bins = np.array([sum(1 for k in (1, 2, 3) if v <= amax / 4 ** k) for v in a])
    nx, ny = prob.dims[0], prob.dims[1]
    lab = -np.ones(prob.n_cells, np.int64)
    comps = []
    for s in range(prob.n_cells):
        if lab[s] >= 0:
            continue
        stack = [s]
        lab[s] = len(comps)
        members = [s]
        while stack:
            c = stack.pop()
            for T, nb_ in ((prob.tx, c + 1), (prob.ty, c + nx), (prob.tz, c + nx * ny)):
                if T[c] > 0 and lab[nb_] < 0 and g[nb_] == g[c] and bins[nb_] == bins[c]:
                    lab[nb_] = lab[s]; stack.append(nb_); members.append(nb_)
            for T, nb_ in ((prob.tx, c - 1), (prob.ty, c - nx), (prob.tz, c - nx * ny)):
                if nb_ >= 0 and T[nb_] > 0 and lab[nb_] < 0 and g[nb_] == g[c] and bins[nb_] == bins[c]:
                    lab[nb_] = lab[s]; stack.append(nb_); members.append(nb_)
        comps.append((g[s], min(members)))
    order = sorted(range(len(comps)), key=lambda c: comps[c])
    rank = np.empty(len(comps), np.int64)
    rank[order] = np.arange(len(comps))
    assert M == len(comps)
    np.testing.assert_array_equal(block, rank[lab])


def test_dynamic_basis_cap_halves_bins():
    prob = make_config0(4)
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (6, 6, 1)}])
    dp = np.random.default_rng(3).standard_normal(prob.n_cells)
    b4, M4, nb4 = O.dynamic_partition(prob, dp, o.stages[0].block, n_bins=4, max_blocks=10 ** 9)
    b2, M2, nb2 = O.dynamic_partition(prob, dp, o.stages[0].block, n_bins=4, max_blocks=M4 - 1)
    assert nb4 == 4 and nb2 <= 2 and M2 < M4


def test_fault_cut_partition_splits_blocks():
    # 4x1x1, one general block, a fault on the face between cells 1 and 2:
    # two pieces; supports stay on their side of the fault.
    prob = make_homogeneous((4, 1, 1))
    prob.fault = prob.fault.copy()
    prob.fault[0, 1] = 1
    prob.tx = prob.tx.copy()
    prob.tx[1] *= 0.01
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (1, 1, 1)}, {"kind": "fault_cut", "parent": 0}])
    st = o.stages[1]
    assert st.M == 2 and list(st.block) == [0, 0, 1, 1]
    assert st.S.toarray().tolist() == [[1, 0], [1, 0], [0, 1], [0, 1]]
    o.update_basis(max_sweeps=10, tol=0.0)
    np.testing.assert_array_equal(o.export_basis(1), [[1, 0], [1, 0], [0, 1], [0, 1]])


# --- ILU(0) in z-line red-black order (the ordering of the GPU's line smoother)

def test_zline_order_structure():
    from workloads import make_lognormal_box, rng_for

    prob = make_lognormal_box((5, 4, 6), rng_for(7, 9), sigma=1.0)
    cells = np.nonzero(prob.active)[0]
    order = O.zline_red_black_order(cells, prob.dims)
    nx, ny = prob.dims[0], prob.dims[1]
    c = cells[order]
    ix, iy, iz = c % nx, (c // nx) % ny, c // (nx * ny)
    colour = (ix + iy) % 2
    assert np.all(np.diff(colour) >= 0)  # even columns first
    col = iy * nx + ix
    for a in range(len(c) - 1):  # a column's cells are consecutive, k ascending
        if col[a] == col[a + 1]:
            assert iz[a + 1] == iz[a] + 1


def test_zline_ilu0_is_exact_on_a_column():
    # one column (nx = ny = 1): ILU(0) keeps the whole tridiagonal pattern, so it is the exact LU
    from workloads import make_lognormal_box, rng_for

    prob = make_lognormal_box((1, 1, 17), rng_for(7, 10), sigma=2.0)
    A, b, _, cells = O.assemble(prob)
    fac = O.ilu0_factor(A, O.zline_red_black_order(cells, prob.dims))
    r = np.random.default_rng(1).standard_normal(cells.size)
    assert np.abs(O.ilu0_apply(fac, r) - np.linalg.solve(A.toarray(), r)).max() <= 1e-12 * np.abs(r).max() * 1e3


def test_zline_ilu0_equals_point_red_black_in_2d():
    # one layer: every column is a single cell and the colours are those of the red-black order
    from workloads import make_lognormal_box, rng_for

    prob = make_lognormal_box((9, 7, 1), rng_for(7, 11), sigma=1.5)
    A, b, _, cells = O.assemble(prob)
    r = np.random.default_rng(2).standard_normal(cells.size)
    f1 = O.ilu0_factor(A, O.zline_red_black_order(cells, prob.dims))
    f2 = O.ilu0_factor(A, O.red_black_order(cells, prob.dims))
    assert np.abs(O.ilu0_apply(f1, r) - O.ilu0_apply(f2, r)).max() <= 1e-13 * np.abs(O.ilu0_apply(f2, r)).max()
