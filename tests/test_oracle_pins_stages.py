"""More pins of the CPU oracle: the smoother's diagonal, the right-hand side
of a new source, fault-cut partitions with several parent blocks, the order
of the stages in a multistage cycle, warm-started basis sweeps and the
rectilinear supports on a ragged 3-D grid.

As in ``test_oracle_pins.py``, nothing here compares the oracle with itself:
each test checks a hand-worked value, a definition written out independently
(dense error-propagation operators, explicit per-entry loops) or a property
that a plausible slip in the oracle would break.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from oracle.msrsb import rhs_for
from workloads import Problem, make_config2, make_lognormal_box, rng_for

EPS = np.finfo(np.float64).eps


def chain_problem(T, bc, source=None):
    """1-D chain of len(T)+1 cells; ``bc`` is a list of (cell, T_bc, p_bc)."""
    n = len(T) + 1
    tx = np.zeros(n)
    tx[:-1] = T
    z = np.zeros(n)
    bc_cell = np.array([c for c, _, _ in bc], np.int32)
    bc_t = np.array([t for _, t, _ in bc], np.float64)
    bc_v = np.array([v for _, _, v in bc], np.float64)
    q = np.zeros(n) if source is None else np.asarray(source, np.float64)
    return Problem((n, 1, 1), (1.0, 1.0, 1.0), np.ones(n, bool), tx, z.copy(), z.copy(), bc_cell, bc_t, bc_v, q,
                   np.ones(n), np.zeros((3, n), np.uint8), "chain")


# ------------------------------------------------------------- smoother ----

def test_jacobi_uses_the_diagonal_of_A_with_its_boundary_terms():
    # Chain with faces T = (1, 2) and a Dirichlet connection T_bc = 1 on cell 0:
    #   A = [[2, -1, 0], [-1, 3, -2], [0, -2, 2]],  diag(A) = (2, 3, 2),
    #   while the basis operator A_b = A - diag(A 1) has diagonal (1, 3, 2).
    # Damped Jacobi with omega_s = 2/3 on r = (1, 1, 1):
    #   (2/3)(1/2, 1/3, 1/2) = (1/3, 2/9, 1/3).
    prob = chain_problem([1.0, 2.0], [(0, 1.0, 0.0)])
    A, b, Ab, cells = O.assemble(prob)
    np.testing.assert_array_equal(A.toarray(), [[2, -1, 0], [-1, 3, -2], [0, -2, 2]])
    np.testing.assert_array_equal(Ab.diagonal(), [1, 3, 2])
    r = np.ones(3)
    np.testing.assert_allclose(O.jacobi_correction(A, r), [1 / 3, 2 / 9, 1 / 3], rtol=2 * EPS)
    # another damping factor: omega_s = 1 is the plain D^-1 r
    np.testing.assert_allclose(O.jacobi_correction(A, r, omega_s=1.0), [1 / 2, 1 / 3, 1 / 2], rtol=2 * EPS)
    # the solver's smoother step uses the same correction with the configured damping
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (1, 1, 1)}], smoother="jacobi", omega_s=0.5)
    np.testing.assert_allclose(o.smooth(np.array([2.0, 3.0, 4.0])), [0.5, 0.5, 1.0], rtol=2 * EPS)


# ---------------------------------------------------------- right-hand side ----

def test_rhs_for_new_source_by_hand():
    # b_i = q_i + sum over connections on i of T_bc p_bc.  Cell 0 carries two
    # connections (2 at p = 3 and 1 at p = 1), cell 2 one (0.5 at p = -1):
    #   b = q + (2*3 + 1*1, 0, 0.5*(-1)) = q + (7, 0, -0.5).
    prob = chain_problem([1.0, 1.0], [(0, 2.0, 3.0), (2, 0.5, -1.0), (0, 1.0, 1.0)], source=[0.0, 0.0, 0.0])
    q = np.array([0.25, -4.0, 1.5])
    cells = np.arange(3)
    np.testing.assert_array_equal(rhs_for(prob, cells, q), [7.25, -4.0, 1.0])
    # the oracle's solve with that source reaches A x = b(q)
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (3, 1, 1)}])
    o.update_basis(max_sweeps=1, tol=0.0)
    x, cycles, rel, status = o.solve(source=q, rtol=1e-14, max_cycles=5)
    np.testing.assert_allclose(o.A @ x, [7.25, -4.0, 1.0], atol=1e-13)


def test_rhs_for_skips_inactive_cells():
    # 4 cells, cell 2 inactive (no faces touch it): b holds the active cells only,
    # in ascending box order, with the connections of cells 0 and 3.
    tx = np.array([1.0, 0.0, 0.0, 0.0])
    z = np.zeros(4)
    act = np.array([True, True, False, True])
    prob = Problem((4, 1, 1), (1.0, 1.0, 1.0), act, tx, z.copy(), z.copy(), np.array([0, 3], np.int32),
                   np.array([1.0, 2.0]), np.array([5.0, -2.0]), np.zeros(4), np.ones(4),
                   np.zeros((3, 4), np.uint8), "gap")
    cells = np.nonzero(act)[0]
    q = np.array([1.0, 2.0, 100.0, 3.0])
    np.testing.assert_array_equal(rhs_for(prob, cells, q), [6.0, 2.0, -1.0])


# ------------------------------------------------------------ fault cuts ----

def test_fault_cut_two_parents_by_hand():
    # 6 x 2 cells, parent Cartesian 2 x 1 blocks (x < 3 and x >= 3).  A fault
    # lies on the y faces between rows 0 and 1 at x = 0..3.  Parent block 0 is
    # cut into its two rows; parent block 1 stays connected through x = 4, 5.
    # Pieces in (parent block, smallest cell) order:
    #   0: cells 0, 1, 2 (parent 0), 1: cells 6, 7, 8 (parent 0),
    #   2: cells 3, 4, 5, 9, 10, 11 (parent 1)
    # (by smallest cell alone piece 2 would come second).  Parent supports
    # along x (n = 6, m = 2, doubled centres 3 and 9): S_0 = x <= 3,
    # S_1 = x >= 2.  A piece's support is what it reaches inside its
    # parent's support without crossing the fault: piece 0 cannot reach row 1
    # inside x <= 3 (the way round through x = 4 lies outside S_0).
    nx, ny = 6, 2
    N = nx * ny
    tx = np.zeros(N)
    ty = np.zeros(N)
    for j in range(ny):
        tx[j * nx:j * nx + nx - 1] = 1.0
    ty[:nx] = 1.0
    fault = np.zeros((3, N), np.uint8)
    fault[1, 0:4] = 1
    ty[0:4] *= 0.05
    prob = Problem((nx, ny, 1), (1.0, 1.0, 1.0), np.ones(N, bool), tx, ty, np.zeros(N), np.array([0, 5], np.int32),
                   np.array([1.0, 1.0]), np.array([1.0, 0.0]), np.zeros(N), np.ones(N), fault, "cut")
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (2, 1, 1)}, {"kind": "fault_cut", "parent": 0}])
    st = o.stages[1]
    assert st.M == 3
    assert st.block.tolist() == [0, 0, 0, 2, 2, 2, 1, 1, 1, 2, 2, 2]
    S = st.S.toarray().astype(int)
    supp = [sorted(np.nonzero(S[:, j])[0].tolist()) for j in range(3)]
    assert supp[0] == [0, 1, 2, 3]
    assert supp[1] == [6, 7, 8, 9]
    assert supp[2] == [2, 3, 4, 5, 8, 9, 10, 11]


def test_fault_cut_brute_force_on_a_faulted_grid():
    # Independent twin on a faulted model with inactive cells: pieces by a
    # stack flood fill, numbered by (parent block, smallest cell); supports by
    # a queue search that stays inside the parent's support box and active
    # cells and never crosses a fault face.
    prob = make_config2(dims=(12, 14, 6), seed=5)
    cd = (3, 2, 2)
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": cd}, {"kind": "fault_cut", "parent": 0}])
    nx, ny, nz = prob.dims
    N = prob.n_cells
    T = (prob.tx, prob.ty, prob.tz)
    step = (1, nx, nx * ny)
    coord = lambda i: (i % nx, (i // nx) % ny, i // (nx * ny))  # noqa: E731

    def open_nbrs(i):
        for a in range(3):
            if T[a][i] > 0 and not prob.fault[a, i]:
                yield i + step[a]
            if i - step[a] >= 0 and coord(i)[a] > 0 and T[a][i - step[a]] > 0 and not prob.fault[a, i - step[a]]:
                yield i - step[a]

    parent = o.stages[0].block
    piece = -np.ones(N, np.int64)
    keys = []
    for s in range(N):
        if not prob.active[s] or piece[s] >= 0:
            continue
        piece[s] = len(keys)
        stack, members = [s], [s]
        while stack:
            c = stack.pop()
            for l in open_nbrs(c):
                if piece[l] < 0 and parent[l] == parent[c]:
                    piece[l] = piece[s]
                    stack.append(l)
                    members.append(l)
        keys.append((int(parent[s]), min(members)))
    order = sorted(range(len(keys)), key=lambda k: keys[k])
    rank = np.empty(len(keys), np.int64)
    rank[order] = np.arange(len(keys))
    st = o.stages[1]
    assert st.M == len(keys) and st.M > o.stages[0].M
    np.testing.assert_array_equal(st.block[prob.active], rank[piece[prob.active]])
    # parent support boxes from the 1-D rule of requirement 2
    def box1(n, m, J):
        e = [-((-K * n) // m) for K in range(m + 1)]
        c2 = [e[K] + e[K + 1] for K in range(m)]
        return [i for i in range(n) if (J == 0 or c2[J - 1] < 2 * i + 1) and (J == m - 1 or 2 * i + 1 < c2[J + 1])]

    present = np.unique([int(v) for v in ((np.arange(N) % nx) * cd[0] // nx
                                          + cd[0] * (((np.arange(N) // nx) % ny) * cd[1] // ny
                                                     + cd[1] * ((np.arange(N) // (nx * ny)) * cd[2] // nz)))[prob.active]])
    loc = -np.ones(N, np.int64)
    loc[prob.active] = np.arange(prob.n_active)
    S = st.S.toarray()
    for j in range(st.M):
        pb = keys[order[j]][0]
        cid = int(present[pb])
        J = (cid % cd[0], (cid // cd[0]) % cd[1], cid // (cd[0] * cd[1]))
        bx = [set(box1(n, m, Jd)) for n, m, Jd in zip((nx, ny, nz), cd, J)]
        inbox = lambda i: prob.active[i] and all(coord(i)[a] in bx[a] for a in range(3))  # noqa: E731
        seen = set(np.nonzero(st.block == j)[0].tolist())
        queue = list(seen)
        while queue:
            c = queue.pop(0)
            for l in open_nbrs(c):
                if l not in seen and inbox(l):
                    seen.add(l)
                    queue.append(l)
        expect = np.zeros(prob.n_active)
        expect[loc[sorted(seen)]] = 1
        np.testing.assert_array_equal(S[:, j], expect)


# -------------------------------------------------------- stage ordering ----

def _dense_stage_error_operator(A, P, Dinv_or_Minv):
    """Error propagation of one stage, written from its definition: the
    smoother step e <- (I - M^-1 A) e, then the Galerkin coarse correction
    e <- (I - P (P^T A P)^-1 P^T A) e."""
    n = A.shape[0]
    I = np.eye(n)
    S = I - Dinv_or_Minv @ A
    C = I - P @ np.linalg.solve(P.T @ A @ P, P.T @ A)
    return C @ S


def test_two_stage_cycle_order_general_then_static():
    # A two-stage cycle (a rectilinear stage, then a fault-cut stage) equals
    # E_2 E_1 applied to the error, with E_l the dense error operator of stage
    # l; the reversed order E_1 E_2 gives a different iterate.  After the
    # cycle the residual is orthogonal to the last stage's basis only.
    prob = make_config2(dims=(9, 10, 4), seed=7)
    parts = [{"kind": "cartesian", "coarse_dims": (3, 2, 2)}, {"kind": "fault_cut", "parent": 0}]
    o = O.Oracle(prob, parts, smoother="jacobi")
    o.update_basis(max_sweeps=6, tol=0.0)
    A = o.A.toarray()
    Minv = np.diag((2.0 / 3.0) / np.diag(A))
    P1 = o.stages[0].P.toarray()
    P2 = o.stages[1].P.toarray()
    assert o.stages[1].M > o.stages[0].M
    E1 = _dense_stage_error_operator(A, P1, Minv)
    E2 = _dense_stage_error_operator(A, P2, Minv)
    xs = np.linalg.solve(A, o.b)
    x0 = np.zeros_like(xs)
    x_expect = xs - E2 @ E1 @ (xs - x0)
    x_wrong = xs - E1 @ E2 @ (xs - x0)
    assert np.abs(x_expect - x_wrong).max() > 1e-6 * np.abs(xs).max()
    xb, cycles, rel, status = o.solve(rtol=0.0, max_cycles=1)
    x = xb[o.cells]
    np.testing.assert_allclose(x, x_expect, rtol=0, atol=1e-11 * np.abs(xs).max())
    r = o.b - o.A @ x
    assert np.abs(P2.T @ r).max() <= 1e-11 * np.abs(o.b).max()
    assert np.abs(P1.T @ r).max() > 1e-6 * np.abs(o.b).max()
    # the preconditioner is the same cycle from zero: M^-1 b = (I - E2 E1) A^-1 b
    z = o.precondition(o.b)
    np.testing.assert_allclose(z, x_expect, rtol=0, atol=1e-11 * np.abs(xs).max())


def test_dynamic_stages_run_newest_first():
    # Two dynamic (constant-basis) stages after the general one: the cycle is
    # E_old E_new E_gen, so after one cycle the residual is orthogonal to the
    # older increment's stage, the last one applied.
    from workloads import pressure_increment_pair

    prob = make_lognormal_box((10, 8, 3), rng_for(11, 0), sigma=1.5)
    parts = [{"kind": "cartesian", "coarse_dims": (2, 2, 1)}]
    o = O.Oracle(prob, parts, smoother="jacobi")
    o.update_basis(max_sweeps=5, tol=0.0)
    dps = pressure_increment_pair(prob, rng_for(11, 1))
    counts = o.add_dynamic_basis(dps)
    assert all(c > 0 for c in counts) and len(o.dyn) == 2
    A = o.A.toarray()
    Minv = np.diag((2.0 / 3.0) / np.diag(A))
    Ps = [o.stages[0].P.toarray(), o.dyn[0].P.toarray(), o.dyn[1].P.toarray()]
    # each dynamic basis is the indicator of the partition of its own increment
    for st, dp in zip(o.dyn, dps):
        blk, M, _ = O.dynamic_partition(prob, dp, o.stages[0].block)
        np.testing.assert_array_equal(st.P.toarray(), np.eye(M)[blk[o.cells]])
    E = [_dense_stage_error_operator(A, P, Minv) for P in Ps]
    xs = np.linalg.solve(A, o.b)
    x_expect = xs - E[2] @ E[1] @ E[0] @ xs
    xb, _, _, _ = o.solve(rtol=0.0, max_cycles=1)
    np.testing.assert_allclose(xb[o.cells], x_expect, rtol=0, atol=1e-11 * np.abs(xs).max())
    r = o.b - o.A @ xb[o.cells]
    assert np.abs(Ps[2].T @ r).max() <= 1e-11 * np.abs(o.b).max()


def test_ilu_stage_is_exact_on_a_chain_before_the_coarse_step():
    # With ILU(0) on a 1-D chain the smoother is the exact inverse, so one
    # stage leaves zero error whatever the basis: pins that the smoother of
    # each stage acts on the current residual b - A x.
    prob = chain_problem([1.0, 3.0, 0.5, 2.0, 1.0], [(0, 1.0, 1.0), (5, 2.0, 0.0)], source=np.zeros(6))
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (2, 1, 1)}, {"kind": "cartesian",
                                                                          "coarse_dims": (3, 1, 1)}],
                 smoother="ilu0_nat")
    o.update_basis(max_sweeps=3, tol=0.0)
    xb, cycles, rel, status = o.solve(rtol=0.0, max_cycles=1)
    np.testing.assert_allclose(xb, o.direct_solve(), rtol=0, atol=1e-14)


# ------------------------------------------------------------ warm start ----

@pytest.mark.parametrize("k,j", [(1, 1), (3, 4), (7, 2)])
def test_warm_start_continues_the_sweeps(k, j):
    # k sweeps, then j more from the current basis, equal k + j sweeps from
    # the indicator (the sweep depends on P alone).
    prob = make_lognormal_box((9, 8, 3), rng_for(11, 2), sigma=1.5)
    parts = [{"kind": "cartesian", "coarse_dims": (3, 2, 1)}]
    a = O.Oracle(prob, parts)
    a.update_basis(max_sweeps=k, tol=0.0)
    a.update_basis(max_sweeps=j, tol=0.0, warm=True)
    b = O.Oracle(prob, parts)
    b.update_basis(max_sweeps=k + j, tol=0.0)
    np.testing.assert_allclose(a.export_basis(0), b.export_basis(0), rtol=0, atol=4 * EPS)
    assert a.stages[0].change == pytest.approx(b.stages[0].change, rel=1e-12)
    # a cold start ignores the current basis
    a.update_basis(max_sweeps=j, tol=0.0, warm=False)
    c = O.Oracle(prob, parts)
    c.update_basis(max_sweeps=j, tol=0.0)
    np.testing.assert_array_equal(a.export_basis(0), c.export_basis(0))


# ------------------------------------------------------ 3-D supports ----

@pytest.mark.parametrize("dims,cd", [((11, 7, 9), (4, 3, 2)), ((10, 13, 5), (3, 5, 5)), ((7, 6, 8), (7, 1, 3))])
def test_cartesian_support_3d_brute_force(dims, cd):
    # Every (cell, block) pair evaluated against the support inequality of
    # requirement 2 (per axis 2c_{J-1} < 2i+1 < 2c_{J+1}, 2c_J = e_J + e_{J+1},
    # e_J = ceil(J n / m), open at the domain ends), on a ragged grid with
    # inactive cells and a dropped block.
    nx, ny, nz = dims
    N = nx * ny * nz
    rng = np.random.default_rng(17)
    active = rng.uniform(size=N) > 0.15
    # empty one whole Cartesian block so that compaction matters
    i = np.arange(N)
    ix, iy, iz = i % nx, (i // nx) % ny, i // (nx * ny)
    active[(ix * cd[0] // nx == 0) & (iy * cd[1] // ny == 0) & (iz * cd[2] // nz == 0)] = False
    block, M, present = O.cartesian_partition(dims, cd, active)
    S = O.cartesian_support(dims, cd, active, present).toarray()
    assert M == cd[0] * cd[1] * cd[2] - 1

    def e(J, n, m):
        return -((-J * n) // m)

    cells = np.nonzero(active)[0]
    expect = np.zeros((cells.size, M))
    for r, c in enumerate(cells):
        cc = (c % nx, (c // nx) % ny, c // (nx * ny))
        for j, cid in enumerate(present):
            Jc = (cid % cd[0], (cid // cd[0]) % cd[1], cid // (cd[0] * cd[1]))
            ok = True
            for a, (n, m) in enumerate(zip(dims, cd)):
                J = Jc[a]
                lo_ok = J == 0 or (e(J - 1, n, m) + e(J, n, m)) < 2 * cc[a] + 1
                hi_ok = J == m - 1 or 2 * cc[a] + 1 < (e(J + 1, n, m) + e(J + 2, n, m))
                ok = ok and lo_ok and hi_ok
            expect[r, j] = 1.0 if ok else 0.0
    np.testing.assert_array_equal(S, expect)
    # and every active cell's own block is in its support
    assert np.all(S[np.arange(cells.size), block[cells]] == 1)


def test_dynamic_cap_beyond_one_bin_is_an_error():
    # With one bin every general block is one key; a general block cut in two
    # by an inactive column gives two pieces, so 36 general blocks plus the cut
    # exceed a cap of 36 even with a single bin.
    from workloads import make_config0

    prob = make_config0(4)
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (6, 6, 1)}], n_bins=1, max_dyn_blocks=36)
    dp = np.random.default_rng(3).standard_normal(prob.n_cells)
    blk, M, nb = O.dynamic_partition(prob, dp, o.stages[0].block, n_bins=1, max_blocks=36)
    assert M == 36 and nb == 1
    with pytest.raises(O.OracleError) as e:
        O.dynamic_partition(prob, dp, o.stages[0].block, n_bins=1, max_blocks=35)
    assert e.value.code == O.msrsb.E_INVAL
    with pytest.raises(O.OracleError):
        o2 = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (6, 6, 1)}], n_bins=4, max_dyn_blocks=20)
        o2.add_dynamic_basis([dp])


# --- transmissibility updates with local basis updates ("changing reservoir/fluid
# properties ... iterating a few times extra", subsection "Iterative multiscale
# multibasis solver")

def _scaled_trans(prob, factor=10.0):
    """Face transmissibilities multiplied by `factor` on the faces of a
    y-slab of cells (a changed mobility region)."""
    nx, ny, nz = prob.dims
    y = (np.arange(prob.n_cells) // nx) % ny
    band = (y >= ny // 3) & (y < ny // 2)
    return tuple(np.where(band, T * factor, T) for T in (prob.tx, prob.ty, prob.tz))


def test_trans_update_equals_fresh_setup():
    from workloads import make_config2

    prob = make_config2(dims=(10, 12, 5), seed=2)
    parts = [{"kind": "cartesian", "coarse_dims": (2, 3, 2)}, {"kind": "fault_cut", "parent": 0}]
    o = O.Oracle(prob, parts, smoother="ilu0_rb")
    o.update_basis(max_sweeps=4, tol=0.0)
    T = _scaled_trans(prob)
    o.update_basis(max_sweeps=6, tol=0.0, new_trans=T)
    fresh_prob = prob.with_source()
    fresh_prob.tx, fresh_prob.ty, fresh_prob.tz = T
    f = O.Oracle(fresh_prob, parts, smoother="ilu0_rb")
    f.update_basis(max_sweeps=6, tol=0.0)
    assert (o.A != f.A).nnz == 0 and np.array_equal(o.b, f.b)
    for a, b in zip(o.stages, f.stages):
        assert (a.P != b.P).nnz == 0 and np.array_equal(a.Ac, b.Ac)
    x1, c1, r1, _ = o.solve(rtol=1e-9)
    x2, c2, r2, _ = f.solve(rtol=1e-9)
    assert c1 == c2 and np.array_equal(x1, x2)


def test_trans_update_keeps_other_bases_and_rebuilds_their_coarse_operators():
    from workloads import make_config1

    prob = make_config1(dims=(8, 10, 4), seed=3)
    parts = [{"kind": "cartesian", "coarse_dims": (2, 2, 2)}, {"kind": "cartesian", "coarse_dims": (4, 2, 1)}]
    o = O.Oracle(prob, parts)
    o.update_basis(max_sweeps=5, tol=0.0)
    P0 = o.stages[0].P.copy()
    dp = np.zeros(prob.n_cells)
    dp[:prob.n_cells // 3] = 1.0
    o.add_dynamic_basis([dp])
    T = _scaled_trans(prob, 7.0)
    # only stage 1 is smoothed again (warm, two extra sweeps)
    P1 = o.stages[1].P.copy()
    o.update_basis(max_sweeps=2, tol=0.0, stage=1, warm=True, new_trans=T)
    assert (o.stages[0].P != P0).nnz == 0
    # stage 0: the dense triple product with the new operator
    dense = P0.toarray().T @ o.A.toarray() @ P0.toarray()
    assert np.abs(o.stages[0].Ac - dense).max() <= 1e-13 * np.abs(dense).max()
    # stage 1: two sweeps of the new basis operator from the old basis
    Pw, _, _ = O.msrsb_basis(o.Ab, o.stages[1].block[o.cells], o.stages[1].S, max_sweeps=2, tol=0.0, P0=P1)
    assert abs(o.stages[1].P - Pw).max() == 0.0
    # dynamic stage: constant basis, so A_c is the coarse two-point operator of the new T
    st = o.dyn[0]
    blk = st.block
    nx, ny = prob.dims[0], prob.dims[1]
    Ac = np.zeros((st.M, st.M))
    for Tarr, step in ((T[0], 1), (T[1], nx), (T[2], nx * ny)):
        for i in np.nonzero(Tarr)[0]:
            j, k = blk[i], blk[i + step]
            if j != k:
                Ac[j, k] -= Tarr[i]
                Ac[k, j] -= Tarr[i]
                Ac[j, j] += Tarr[i]
                Ac[k, k] += Tarr[i]
    for c, t in zip(prob.bc_cell, prob.bc_trans):
        Ac[blk[c], blk[c]] += t
    assert np.abs(st.Ac - Ac).max() <= 1e-13 * np.abs(Ac).max()
