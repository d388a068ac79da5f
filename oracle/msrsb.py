"""CPU FP64 oracle of the iterative multiscale-multibasis pressure solver.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the GPU library (no kernels, headers, helpers or tables) and never imports
it; the two meet only through the seeded inputs of ``workloads``.

Each function is a plain statement of the definition or algorithm it cites,
on numpy / scipy.sparse in float64, with library primitives (sparse products,
Cholesky, triangular solves, connected components) as single steps and no
blocking or fusion.  Paper references are to Klemetsdal, Moyner & Lie,
"Accelerating Multiscale Simulation of Complex Geomodels by Use of
Dynamically Adapted Basis Functions" (arXiv 2001.01624).

Where the paper is silent the oracle takes these readings (the GPU library
takes the same ones):

* Operator (section "Discrete equations", eq. pressure_system): ``A`` is the
  SPD two-point-flux matrix, ``A_ii = sum_f T_f + sum_bc T_bc``,
  ``A_ab = -T_f``; ``b = q + sum_bc T_bc p_bc`` (``q > 0`` injects).
* Basis (the MsRSB basis the section "Multiscale methods" builds on):
  ``P^0`` is the block indicator; one sweep is
  ``P <- rownorm(mask_S(P - omega D_b^{-1} A_b P))`` with
  ``A_b = A - diag(A 1)`` and ``D_b = diag(A_b)``; every row is renormalised;
  stop after the first sweep whose max-entry change is ``<= tol``.
* Supports (requirement 2 of the feasible operator pairs): per dimension,
  cell ``i`` lies in the support of block ``J`` iff
  ``2 c_{J-1} < 2 i + 1 < 2 c_{J+1}`` with ``2 c_J = e_J + e_{J+1}`` and
  ``e_J = ceil(J n / m)``; the support is the tensor product of the 1-D sets
  intersected with the active cells.
* Dynamic partitions (subsection "Iterative multiscale multibasis solver",
  type "Dynamic"): ``a = |dp|``; bin = number of thresholds
  ``ldexp(max a, -2k)``, k = 1..n_bins-1, that ``a`` does not exceed; cells
  with equal (general block, bin) key that are face-connected form one block;
  blocks are numbered by (general block, smallest cell index); constant basis.
* Fault-cut static partitions: connected pieces of each general block over
  faces that are not on a fault; the support of a piece is the part of its
  parent block's support reachable from it without crossing a fault face.
* Cycle (eq. multiscale-multibasis): stages in the order general, static,
  dynamic (newest first); each stage applies its smoother once to
  ``b - A x`` and then the Galerkin (``R = P^T``) coarse correction; the
  relative residual ``||b - A x||_2 / ||b||_2`` is tested after every full
  cycle.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.sparse.csgraph import connected_components, shortest_path

E_INVAL = -1
E_SINGULAR = -4
E_NOCONV = -5
E_STATE = -6


class OracleError(Exception):
    def __init__(self, code: int, msg: str):
        super().__init__(msg)
        self.code = code


# ---------------------------------------------------------------------------
# Fine-scale operator: two-point flux assembly (section "Discrete equations";
# eq. pressure_system: A p = q).
# ---------------------------------------------------------------------------

def _coords(dims):
    nx, ny, nz = dims
    idx = np.arange(nx * ny * nz)
    return idx % nx, (idx // nx) % ny, idx // (nx * ny)


def _faces(prob):
    """Interior faces ``(a, b, T)`` in box numbering, validated."""
    nx, ny, nz = prob.dims
    ix, iy, iz = _coords(prob.dims)
    out = []
    for T, step, coord, n in ((prob.tx, 1, ix, nx), (prob.ty, nx, iy, ny), (prob.tz, nx * ny, iz, nz)):
        T = np.asarray(T, dtype=np.float64)
        if not np.all(np.isfinite(T)) or np.any(T < 0):
            raise OracleError(E_INVAL, "transmissibilities must be finite and >= 0")
        a = np.nonzero(T)[0]
        if np.any(coord[a] >= n - 1):
            raise OracleError(E_INVAL, "face leaves the grid")
        b = a + step
        if not (np.all(prob.active[a]) and np.all(prob.active[b])):
            raise OracleError(E_INVAL, "face touches an inactive cell")
        out.append((a, b, T[a]))
    a = np.concatenate([o[0] for o in out])
    b = np.concatenate([o[1] for o in out])
    t = np.concatenate([o[2] for o in out])
    return a, b, t


def assemble(prob):
    """Return ``(A, b, A_b, cells)`` over the active cells.

    ``cells`` are the box indices of the active cells (ascending); row ``r`` of
    ``A`` is cell ``cells[r]``.  ``A_b = A - diag(A 1)`` is the zero-row-sum
    operator that the basis smoothing uses."""
    N = prob.n_cells
    cells = np.nonzero(prob.active)[0]
    n = cells.size
    loc = np.full(N, -1, dtype=np.int64)
    loc[cells] = np.arange(n)
    a, b, t = _faces(prob)
    la, lb = loc[a], loc[b]
    bc_cell = np.asarray(prob.bc_cell, dtype=np.int64)
    bc_t = np.asarray(prob.bc_trans, dtype=np.float64)
    bc_v = np.asarray(prob.bc_value, dtype=np.float64)
    if bc_cell.size and (np.any(bc_cell < 0) or np.any(bc_cell >= N) or not np.all(prob.active[bc_cell])):
        raise OracleError(E_INVAL, "boundary connection on a missing or inactive cell")
    if not (np.all(np.isfinite(bc_t)) and np.all(bc_t >= 0) and np.all(np.isfinite(bc_v))):
        raise OracleError(E_INVAL, "boundary transmissibility/value not finite or negative")
    q = np.asarray(prob.source, dtype=np.float64)
    if not np.all(np.isfinite(q)):
        raise OracleError(E_INVAL, "source not finite")
    lc = loc[bc_cell]
    rows = np.concatenate([la, lb, la, lb, lc])
    cols = np.concatenate([la, lb, lb, la, lc])
    vals = np.concatenate([t, t, -t, -t, bc_t])
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    rhs = q[cells].copy()
    np.add.at(rhs, lc, bc_t * bc_v)
    Ab = (A - sp.diags(A @ np.ones(n))).tocsr()
    Ab.sort_indices()
    # every connected component needs a Dirichlet/well connection, else A is singular
    G = sp.coo_matrix((np.ones(la.size), (la, lb)), shape=(n, n))
    ncomp, lab = connected_components(G, directed=False)
    anchored = np.zeros(ncomp, dtype=bool)
    anchored[lab[lc[bc_t > 0]]] = True
    if not np.all(anchored):
        raise OracleError(E_SINGULAR, "a connected component has no boundary or well connection")
    return A, rhs, Ab, cells


def rhs_for(prob, cells, source):
    """``b = q + sum_bc T_bc p_bc`` for a new source vector (box numbering)."""
    N = prob.n_cells
    loc = np.full(N, -1, dtype=np.int64)
    loc[cells] = np.arange(cells.size)
    rhs = np.asarray(source, dtype=np.float64)[cells].copy()
    np.add.at(rhs, loc[np.asarray(prob.bc_cell, dtype=np.int64)],
              np.asarray(prob.bc_trans) * np.asarray(prob.bc_value))
    return rhs


# ---------------------------------------------------------------------------
# Coarse partitions and supports (section "Multiscale methods", feasibility
# requirements 1-2; general rectilinear partitions).
# ---------------------------------------------------------------------------

def cartesian_partition(dims, coarse_dims, active):
    """Rectilinear partition: along each axis cell ``i`` of ``n`` goes to block
    ``floor(i m / n)``.  Blocks without active cells are dropped and the rest
    numbered by ascending Cartesian block index.  Returns ``(block, M,
    present)`` with ``block`` in box numbering (-1 on inactive cells) and
    ``present`` the Cartesian index of each kept block."""
    ix, iy, iz = _coords(dims)
    (nx, ny, nz), (mx, my, mz) = dims, coarse_dims
    if not (1 <= mx <= nx and 1 <= my <= ny and 1 <= mz <= nz):
        raise OracleError(E_INVAL, "coarse dimensions must lie in [1, fine dimension]")
    bx, by, bz = ix * mx // nx, iy * my // ny, iz * mz // nz
    cart = bx + mx * (by + my * bz)
    present = np.unique(cart[active])
    block = np.full(cart.size, -1, dtype=np.int64)
    block[active] = np.searchsorted(present, cart[active])
    return block, present.size, present


def support_1d(n, m):
    """Member lists of the 1-D supports: ``i`` is in ``S_J`` iff
    ``(J == 0 or 2c_{J-1} < 2i+1) and (J == m-1 or 2i+1 < 2c_{J+1})``."""
    e = [-((-J * n) // m) for J in range(m + 1)]  # ceil(J n / m)
    c2 = [e[J] + e[J + 1] for J in range(m)]
    sets = []
    for J in range(m):
        sets.append([i for i in range(n)
                     if (J == 0 or c2[J - 1] < 2 * i + 1) and (J == m - 1 or 2 * i + 1 < c2[J + 1])])
    return sets


def cartesian_support(dims, coarse_dims, active, present):
    """Boolean ``n_active x M`` support matrix of a rectilinear partition."""
    nx, ny, nz = dims
    mx, my, mz = coarse_dims
    sx, sy, sz = support_1d(nx, mx), support_1d(ny, my), support_1d(nz, mz)
    cells = np.nonzero(active)[0]
    loc = np.full(nx * ny * nz, -1, dtype=np.int64)
    loc[cells] = np.arange(cells.size)
    rows, cols = [], []
    for j, cid in enumerate(present):
        Jx, Jy, Jz = cid % mx, (cid // mx) % my, cid // (mx * my)
        X, Y, Z = np.meshgrid(sx[Jx], sy[Jy], sz[Jz], indexing="ij")
        box = (X + nx * (Y + ny * Z)).reshape(-1)
        box = box[active[box]]
        rows.append(loc[box])
        cols.append(np.full(box.size, j))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    S = sp.coo_matrix((np.ones(r.size), (r, c)), shape=(cells.size, present.size)).tocsr()
    S.sort_indices()
    return S


def _face_graph(prob, keep=None):
    """Undirected cell graph over faces with ``T > 0`` (optionally filtered)."""
    a, b, t = _faces(prob)
    if keep is not None:
        m = keep(a, b)
        a, b = a[m], b[m]
    N = prob.n_cells
    return sp.coo_matrix((np.ones(a.size), (a, b)), shape=(N, N)).tocsr(), a, b


def _fault_face_mask(prob, a, b):
    """True for faces ``(a, b)`` that lie on a fault."""
    nx, ny = prob.dims[0], prob.dims[1]
    step = b - a
    d = np.where(step == 1, 0, np.where(step == nx, 1, 2))
    return prob.fault[d, a] != 0


def fault_cut_partition(prob, parent_block, parent_S, cells):
    """Static partition tracing faults: the connected pieces of every parent
    block over faces that are not on a fault, numbered by (parent block,
    smallest cell index).  Support of a piece: the cells of its parent's
    support reachable from the piece without crossing a fault face.  Returns
    ``(block, M, S)``."""
    N = prob.n_cells
    loc = np.full(N, -1, dtype=np.int64)
    loc[cells] = np.arange(cells.size)
    G, a, b = _face_graph(prob, keep=lambda a, b: ~_fault_face_mask(prob, a, b))
    same = parent_block[a] == parent_block[b]
    Gin = sp.coo_matrix((np.ones(int(same.sum())), (a[same], b[same])), shape=(N, N)).tocsr()
    _, lab = connected_components(Gin, directed=False)
    act = cells
    pieces = {}
    for c in act:
        key = lab[c]
        if key not in pieces:
            pieces[key] = (int(parent_block[c]), int(c))
    order = sorted(pieces.items(), key=lambda kv: kv[1])
    newid = {key: j for j, (key, _) in enumerate(order)}
    block = np.full(N, -1, dtype=np.int64)
    block[act] = [newid[lab[c]] for c in act]
    M = len(order)
    # supports: BFS inside the parent's support without crossing fault faces
    Gcsr = G.tocsr()
    Gsym = ((Gcsr + Gcsr.T) > 0).tocsr()
    parentS = parent_S.tocsc()
    rows, cols = [], []
    for j, (key, (pb, _)) in enumerate(order):
        inS = np.zeros(N, dtype=bool)
        inS[cells[parentS[:, pb].indices]] = True
        seen = np.zeros(N, dtype=bool)
        frontier = np.nonzero(block == j)[0]
        seen[frontier] = True
        while frontier.size:
            nb = np.unique(Gsym[frontier].indices)
            nb = nb[inS[nb] & ~seen[nb]]
            seen[nb] = True
            frontier = nb
        members = np.nonzero(seen)[0]
        rows.append(loc[members])
        cols.append(np.full(members.size, j))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    S = sp.coo_matrix((np.ones(r.size), (r, c)), shape=(cells.size, M)).tocsr()
    S.sort_indices()
    return block, M, S


def _active_adjacency(prob, cells):
    """Symmetric 0/1 adjacency of the active cells (local numbering) over the
    faces with ``T > 0``."""
    N = prob.n_cells
    loc = np.full(N, -1, dtype=np.int64)
    loc[cells] = np.arange(cells.size)
    a, b, _ = _faces(prob)
    G = sp.coo_matrix((np.ones(a.size), (loc[a], loc[b])), shape=(cells.size, cells.size)).tocsr()
    return ((G + G.T) > 0).astype(np.float64).tocsr()


def graph_partition(prob, block_of_cell, overlap, cells):
    """Partition given as a block id per cell (types "General" from a graph
    partitioner, "Static" from indicators or wells): the ids of the active
    cells, renumbered by ascending id with unused ids dropped.  The support of
    a block is every active cell within ``overlap`` face steps of it, i.e.
    ``R_0`` = block indicator and ``R_{t+1} = R_t or G R_t`` with ``G`` the
    face adjacency.  Returns ``(block, M, S)``."""
    if overlap < 0:
        raise OracleError(E_INVAL, "overlap must be >= 0")
    ids = np.asarray(block_of_cell, dtype=np.int64)[cells]
    if np.any(ids < 0):
        raise OracleError(E_INVAL, "an active cell has a negative block id")
    present = np.unique(ids)
    local = np.searchsorted(present, ids)
    M = present.size
    block = np.full(prob.n_cells, -1, dtype=np.int64)
    block[cells] = local
    G = _active_adjacency(prob, cells)
    R = indicator(local, M)
    for _ in range(overlap):
        R = ((R + G @ R) > 0).astype(np.float64).tocsr()
    R.sort_indices()
    return block, M, R


def well_partition(prob, well_cells, radius):
    """Well partition (type "Static": one block per well plus one block for
    the rest, so that the blocks cover the grid): cell ``i`` joins well
    ``w`` when its face-step distance to the well's cells (faces with
    ``T > 0``) is at most ``radius`` and smaller than to any other well (ties
    to the lower well index); every other active cell joins block
    ``n_wells``.  ``well_cells`` is a list of box-index arrays.  Returns the
    block per cell in box numbering (-1 inactive)."""
    cells = np.nonzero(prob.active)[0]
    N = prob.n_cells
    loc = np.full(N, -1, dtype=np.int64)
    loc[cells] = np.arange(cells.size)
    G = _active_adjacency(prob, cells)
    n_w = len(well_cells)
    if n_w < 1 or radius < 0:
        raise OracleError(E_INVAL, "need at least one well and radius >= 0")
    # unweighted shortest paths from a virtual node joined to all cells of one well
    dist = np.full((n_w, cells.size), np.inf)
    n = cells.size
    for w, wc in enumerate(well_cells):
        wc = np.asarray(wc, dtype=np.int64)
        if wc.size == 0 or np.any(wc < 0) or np.any(wc >= N) or not np.all(prob.active[wc]):
            raise OracleError(E_INVAL, "well cells must be active cells of the grid")
        src = np.zeros(n + 1)
        Gs = sp.bmat([[G, sp.csr_matrix((np.ones(wc.size), (loc[wc], np.zeros(wc.size))), shape=(n, 1))],
                      [sp.csr_matrix((np.ones(wc.size), (np.zeros(wc.size), loc[wc])), shape=(1, n)), None]]).tocsr()
        d = shortest_path(Gs, unweighted=True, indices=n, directed=False)
        dist[w] = d[:n] - 1.0
    best = np.argmin(dist, axis=0)  # first minimum: the lower well index wins ties
    dmin = dist[best, np.arange(n)]
    out = np.full(N, -1, dtype=np.int64)
    out[cells] = np.where(dmin <= radius, best, n_w)
    return out


def indicator_partition(prob, ind, n_bins, coarse_dims, min_cells):
    """Indicator agglomeration (type "Static": blocks that follow a cell
    indicator such as log-permeability or a velocity magnitude):

    1. equal-count bins: the active cells ranked by (indicator, cell index),
       ``bin = floor(rank * n_bins / n_active)``;
    2. pieces: face-connected cells (``T > 0``) with the same (rectilinear
       parent block of ``coarse_dims``, bin);
    3. merging: while a piece has fewer than ``min_cells`` cells and a
       face-neighbour piece in the same parent block, the smallest such piece
       (by size, then smallest cell index) joins the neighbour piece it shares
       the most faces with (ties: the neighbour with the smaller smallest
       cell index);
    4. blocks numbered by their smallest cell index.
    Returns the block per cell in box numbering (-1 inactive)."""
    cells = np.nonzero(prob.active)[0]
    N, n = prob.n_cells, cells.size
    ind = np.asarray(ind, dtype=np.float64)
    if n_bins < 1 or min_cells < 0 or not np.all(np.isfinite(ind[cells])):
        raise OracleError(E_INVAL, "n_bins >= 1, min_cells >= 0 and a finite indicator on active cells")
    order = np.lexsort((cells, ind[cells]))  # by value, then cell index
    rank = np.empty(n, dtype=np.int64)
    rank[order] = np.arange(n)
    bins = np.full(N, -1, dtype=np.int64)
    bins[cells] = rank * n_bins // n
    parent, _, _ = cartesian_partition(prob.dims, coarse_dims, np.ones(N, dtype=bool))
    a, b, _ = _faces(prob)
    same = (bins[a] == bins[b]) & (parent[a] == parent[b])
    Gk = sp.coo_matrix((np.ones(int(same.sum())), (a[same], b[same])), shape=(N, N))
    _, lab = connected_components(Gk, directed=False)
    piece = {}
    for c in cells:  # ascending: the first cell seen is the smallest
        piece.setdefault(int(lab[c]), []).append(int(c))
    members = {min(v): set(v) for v in piece.values()}  # pieces keyed by their smallest cell
    owner = np.full(N, -1, dtype=np.int64)
    for key, v in members.items():
        owner[list(v)] = key
    while True:
        cand = None
        for key, v in members.items():
            if len(v) >= min_cells:
                continue
            # shared faces with each neighbour piece of the same parent block
            count = {}
            for c in v:
                for d, (T, step) in enumerate(((prob.tx, 1), (prob.ty, prob.dims[0]),
                                               (prob.tz, prob.dims[0] * prob.dims[1]))):
                    for nb, t in ((c + step, T[c]), (c - step, T[c - step] if c - step >= 0 else 0.0)):
                        if t > 0 and owner[nb] != key and parent[nb] == parent[c]:
                            count[int(owner[nb])] = count.get(int(owner[nb]), 0) + 1
            if not count:
                continue
            if cand is None or (len(v), key) < (len(members[cand[0]]), cand[0]):
                target = min(count, key=lambda k: (-count[k], k))
                cand = (key, target)
        if cand is None:
            break
        small, target = cand
        merged = members.pop(small) | members.pop(target)
        newkey = min(small, target)
        members[newkey] = merged
        owner[list(merged)] = newkey
    keys = sorted(members)
    out = np.full(N, -1, dtype=np.int64)
    for j, key in enumerate(keys):
        out[list(members[key])] = j
    return out


def indicator(block_local, M):
    """``P_ij = 1`` if cell ``i`` is in block ``j`` (constant basis)."""
    n = block_local.size
    return sp.csr_matrix((np.ones(n), (np.arange(n), block_local)), shape=(n, M))


# ---------------------------------------------------------------------------
# Restricted-smoothing basis (MsRSB, cited in section "Multiscale methods";
# local updates by a few extra iterations, subsection "Iterative multiscale
# multibasis solver").
# ---------------------------------------------------------------------------

def msrsb_basis(Ab, block_local, S, omega=2.0 / 3.0, tol=1e-3, max_sweeps=100, P0=None):
    """Damped-Jacobi smoothing of the prolongation restricted to the supports.

    Returns ``(P, sweeps, last_change)``; ``last_change`` is NaN when no sweep
    ran.  Raises ``OracleError(E_SINGULAR)`` if a row sum is not positive."""
    n, M = S.shape
    P = indicator(block_local, M) if P0 is None else sp.csr_matrix(P0)
    dg = Ab.diagonal()
    dinv = np.zeros(n)
    dinv[dg > 0] = 1.0 / dg[dg > 0]
    Dinv = sp.diags(dinv)
    change = float("nan")
    sweeps = 0
    for s in range(max_sweeps):
        Z = Ab @ P
        Pn = (P - omega * (Dinv @ Z)).multiply(S).tocsr()
        rs = np.asarray(Pn.sum(axis=1)).ravel()
        if np.any(~(rs > 0)):
            raise OracleError(E_SINGULAR, "basis row sum not positive")
        Pn = (sp.diags(1.0 / rs) @ Pn).tocsr()
        change = float(abs(Pn - P).max())
        P = Pn
        sweeps = s + 1
        if change <= tol:
            break
    P.sort_indices()
    return P, sweeps, change


# ---------------------------------------------------------------------------
# Coarse operator and coarse solve (eq. pressure_system_reduced with R = P^T).
# ---------------------------------------------------------------------------

def galerkin(P, A):
    """``A_c = P^T A P`` as a dense array."""
    return np.asarray((P.T @ (A @ P)).todense())


def coarse_factor(Ac):
    """Cholesky factor ``L`` of the SPD coarse matrix."""
    try:
        return np.linalg.cholesky(Ac)
    except np.linalg.LinAlgError as exc:
        raise OracleError(E_SINGULAR, f"coarse matrix not SPD: {exc}")


def coarse_solve(L, d):
    """``A_c^{-1} d`` by forward and backward substitution."""
    y = sla.solve_triangular(L, d, lower=True)
    return sla.solve_triangular(L.T, y, lower=False)


# ---------------------------------------------------------------------------
# Fine-scale smoothers S(A, r) (eq. iterative_multiscale; ILU(0) as in
# section "Computational efficiency").
# ---------------------------------------------------------------------------

def jacobi_correction(A, r, omega_s=2.0 / 3.0):
    """Damped Jacobi: ``omega_s D^{-1} r``."""
    return omega_s * r / A.diagonal()


def natural_order(cells, dims):
    return np.arange(cells.size)


def red_black_order(cells, dims):
    """Cells with even ``i+j+k`` first, then odd; ascending within each colour."""
    ix, iy, iz = _coords(dims)
    col = (ix + iy + iz)[cells] % 2
    loc = np.arange(cells.size)
    return np.concatenate([loc[col == 0], loc[col == 1]])


def zline_red_black_order(cells, dims):
    """Whole columns (i, j) coloured by the parity of ``i + j``, even columns
    first; within a colour column by column, each column's cells in
    ascending ``k``."""
    ix, iy, iz = _coords(dims)
    nx = dims[0]
    c = cells
    return np.lexsort((iz[c], iy[c] * nx + ix[c], (ix[c] + iy[c]) % 2))


def ilu0_factor(A, order, positive=True):
    """Textbook ILU(0) (row-wise IKJ elimination restricted to the pattern of
    the matrix) of ``A`` permuted to ``order``.  Returns ``(L, U, order)``
    with ``L`` unit lower triangular and ``U`` upper triangular, both CSR in
    the permuted numbering.  Pivots must be positive (the M-matrices of the
    pressure equation) or, with ``positive=False`` (a general matrix such as
    the two-phase Jacobian), non-zero."""
    B = A[order][:, order].tocsr()
    B.sort_indices()
    n = B.shape[0]
    rows = []
    for i in range(n):
        s, e = B.indptr[i], B.indptr[i + 1]
        rows.append(dict(zip(B.indices[s:e].tolist(), B.data[s:e].tolist())))
    for i in range(n):
        row = rows[i]
        for k in sorted(c for c in row if c < i):
            row[k] = row[k] / rows[k][k]
            lik = row[k]
            for j, ukj in rows[k].items():
                if j > k and j in row:
                    row[j] -= lik * ukj
        piv = row.get(i, 0.0)
        if not (piv > 0.0 if positive else (piv != 0.0 and np.isfinite(piv))):
            raise OracleError(E_SINGULAR, "ILU(0) pivot not positive" if positive else "ILU(0) pivot zero")
    lr, lc, lv, ur, uc, uv = [], [], [], [], [], []
    for i, row in enumerate(rows):
        for j, v in row.items():
            if j < i:
                lr.append(i); lc.append(j); lv.append(v)
            else:
                ur.append(i); uc.append(j); uv.append(v)
    L = sp.csr_matrix((lv + [1.0] * n, (lr + list(range(n)), lc + list(range(n)))), shape=(n, n))
    U = sp.csr_matrix((uv, (ur, uc)), shape=(n, n))
    L.sort_indices()
    U.sort_indices()
    return L, U, np.asarray(order)


def ilu0_rb_fill(A, cells, dims):
    """The fill that red-black ILU(0) drops: for the order of
    ``red_black_order`` (even i+j+k first), ``L U - A`` is zero except on the
    black (odd) rows and columns, where it is the off-diagonal part of
    ``A_br D_rr^-1 A_rb``.  No two cells of one colour share a face, so the
    red rows are eliminated without fill and each black pivot keeps only the
    diagonal of its Schur complement.  Returned in the original (active)
    numbering; ``A + F`` is the matrix whose inverse the smoother applies."""
    ix, iy, iz = _coords(dims)
    black = ((ix + iy + iz)[cells] % 2) == 1
    bi, ri = np.nonzero(black)[0], np.nonzero(~black)[0]
    Acsr = A.tocsr()
    d_r = Acsr.diagonal()[ri]
    S = (Acsr[bi][:, ri] @ sp.diags(1.0 / d_r) @ Acsr[ri][:, bi]).tocsr()
    S.setdiag(0.0)
    S.eliminate_zeros()
    S = S.tocoo()
    n = A.shape[0]
    return sp.csr_matrix((S.data, (bi[S.row], bi[S.col])), shape=(n, n))


def ilu0_apply(fac, r):
    """``(L U)^{-1} r`` in the original numbering."""
    L, U, order = fac
    y = spla.spsolve_triangular(L, r[order], lower=True, unit_diagonal=True)
    z = spla.spsolve_triangular(U, y, lower=False)
    e = np.empty_like(z)
    e[order] = z
    return e


# ---------------------------------------------------------------------------
# Dynamic partitions (subsection "Iterative multiscale multibasis solver",
# type "Dynamic"): bins of the pressure-update magnitude, agglomerated into
# connected blocks inside each general block; constant basis functions.
# ---------------------------------------------------------------------------

def dynamic_partition(prob, dp, general_block, n_bins=4, max_blocks=4096):
    """Return ``(block, M, n_bins_used)`` (box numbering, -1 inactive) or
    ``None`` when ``max |dp|`` is zero or not finite."""
    act = prob.active
    cells = np.nonzero(act)[0]
    a = np.abs(np.asarray(dp, dtype=np.float64))
    amax = float(a[cells].max()) if cells.size else 0.0
    if not math.isfinite(amax) or amax == 0.0:
        return None
    fa, fb, _ = _faces(prob)
    nb = int(n_bins)
    while True:
        thresholds = [math.ldexp(amax, -2 * k) for k in range(1, nb)]
        bins = np.zeros(prob.n_cells, dtype=np.int64)
        for t in thresholds:
            bins += (a <= t)
        key = general_block * nb + bins
        same = key[fa] == key[fb]
        N = prob.n_cells
        G = sp.coo_matrix((np.ones(int(same.sum())), (fa[same], fb[same])), shape=(N, N))
        _, lab = connected_components(G, directed=False)
        first = {}
        for c in cells:  # ascending box index: first visit is the smallest member
            if lab[c] not in first:
                first[lab[c]] = (int(general_block[c]), int(c))
        order = sorted(first.items(), key=lambda kv: kv[1])
        if len(order) <= max_blocks:
            break
        if nb == 1:
            raise OracleError(E_INVAL, "dynamic partition exceeds max_blocks even with one bin")
        nb //= 2
    newid = {key: j for j, (key, _) in enumerate(order)}
    block = np.full(prob.n_cells, -1, dtype=np.int64)
    block[cells] = [newid[lab[c]] for c in cells]
    return block, len(order), nb


# ---------------------------------------------------------------------------
# Finite-volume restriction and conservative flux reconstruction (section
# "Multiscale methods": for fine-scale fluxes, a restriction operator that sums
# the entries of the cells of each block).
# ---------------------------------------------------------------------------

def fv_restriction(block_local, M):
    """``R_fv[j, i] = 1`` for cell ``i`` in block ``j`` (sparse ``M x n``)."""
    return indicator(block_local, M).T.tocsr()


def fv_multiscale_pressure(P, A, b, block_local, M):
    """``A_fv = R_fv A P`` and ``p_ms = P A_fv^{-1} R_fv b`` (dense LU for the
    coarse system).  Returns ``(p_ms, A_fv)`` over the active cells."""
    R = fv_restriction(block_local, M)
    Afv = np.asarray((R @ (A @ P)).todense())
    pc = np.linalg.solve(Afv, R @ b)
    return P @ pc, Afv


def conservative_pressure(A, b, block_local, M, pms, bc_diag):
    """Fine pressure ``p'`` inside every block from the block's own equations
    with the fluxes of ``pms`` imposed on the faces leaving it: for ``I`` the
    cells of a block, ``A_N = A[I, I] + diag(sum_{l not in I} A_il)`` and
    ``rhs_i = b_i + sum_{l not in I} A_il (pms_i - pms_l)``.  Each connected
    piece of a block is solved on its own; a piece without a boundary or well
    term (``bc_diag = 0`` on all its cells) has a singular ``A_N``, and its
    ``p'`` is the solution with the same sum as ``pms`` on the piece (that sum
    as an extra equation with a multiplier)."""
    A = A.tocsr()
    n = A.shape[0]
    pf = np.zeros(n)
    for j in range(M):
        I = np.nonzero(block_local == j)[0]
        out = np.setdiff1d(np.arange(n), I)
        AII = A[I][:, I]
        AIo = A[I][:, out]
        off = np.asarray(AIo.sum(axis=1)).ravel()
        AN = (AII + sp.diags(off)).tocsr()
        rhs = b[I] + off * pms[I] - AIo @ pms[out]
        ncomp, lab = connected_components(AN, directed=False)
        for c in range(ncomp):
            C = np.nonzero(lab == c)[0]
            ACC = AN[C][:, C].tocsc()
            if np.any(bc_diag[I[C]] > 0):
                pf[I[C]] = spla.spsolve(ACC, rhs[C]) if C.size > 1 else rhs[C] / ACC.toarray()[0, 0]
            else:
                one = sp.csc_matrix(np.ones((C.size, 1)))
                K = sp.bmat([[ACC, one], [one.T, None]]).tocsc()
                sol = spla.spsolve(K, np.append(rhs[C], pms[I[C]].sum()))
                pf[I[C]] = sol[:C.size]
    return pf


def reconstructed_fluxes(prob, cells, block_local, pms, pf):
    """Face fluxes in the structured layout ``[3, N]``: ``T (p'_a - p'_b)`` on
    faces inside a block, ``T (pms_a - pms_b)`` on faces between blocks; well
    and boundary fluxes ``T_bc (p'_i - p_bc)``."""
    nx, ny, nz = prob.dims
    N = prob.n_cells
    blk = np.full(N, -1, dtype=np.int64)
    blk[cells] = block_local
    P = np.zeros(N)
    F = np.zeros(N)
    P[cells] = pms
    F[cells] = pf
    out = np.zeros((3, N))
    for d, (T, step) in enumerate(((prob.tx, 1), (prob.ty, nx), (prob.tz, nx * ny))):
        a = np.nonzero(T)[0]
        inside = blk[a] == blk[a + step]
        out[d, a] = np.where(inside, T[a] * (F[a] - F[a + step]), T[a] * (P[a] - P[a + step]))
    bc = np.asarray(prob.bc_trans) * (F[np.asarray(prob.bc_cell)] - np.asarray(prob.bc_value))
    return out, bc


def cell_imbalance(prob, face, bcf, source=None):
    """Per-cell ``outflow - q_i`` of face and connection fluxes (box numbering)."""
    nx, ny, nz = prob.dims
    N = prob.n_cells
    q = np.asarray(prob.source if source is None else source, dtype=np.float64)
    out = np.zeros(N)
    for d, step in enumerate((1, nx, nx * ny)):
        out += face[d]
        out[step:] -= face[d][:N - step]
    np.add.at(out, np.asarray(prob.bc_cell), bcf)
    return np.where(prob.active, out - q, 0.0)


# ---------------------------------------------------------------------------
# Post-processing: fluxes and mass balance.
# ---------------------------------------------------------------------------

def fluxes(prob, x):
    """Face fluxes ``T_f (x_a - x_b)`` in the structured layout ``[3, N]``
    and well/boundary fluxes ``T_bc (x_i - p_bc)``."""
    nx, ny, nz = prob.dims
    N = prob.n_cells
    out = np.zeros((3, N))
    for d, (T, step) in enumerate(((prob.tx, 1), (prob.ty, nx), (prob.tz, nx * ny))):
        a = np.nonzero(T)[0]
        out[d, a] = T[a] * (x[a] - x[a + step])
    bc = np.asarray(prob.bc_trans) * (x[np.asarray(prob.bc_cell)] - np.asarray(prob.bc_value))
    return out, bc


# ---------------------------------------------------------------------------
# The whole solver with the same four calls as the GPU library.
# ---------------------------------------------------------------------------

class _Stage:
    def __init__(self, kind, block, M, S, P=None):
        self.kind, self.block, self.M, self.S, self.P = kind, block, M, S, P
        self.Ac = None
        self.L = None
        self.sweeps = 0
        self.change = float("nan")


class Oracle:
    """``setup`` / ``update_basis`` / ``add_dynamic_basis`` / ``solve``.

    ``partitions`` is a list of dicts: ``{"kind": "cartesian", "coarse_dims":
    (mx, my, mz)}`` (the first entry must be one: the general partition) or
    ``{"kind": "fault_cut", "parent": 0}``."""

    def __init__(self, prob, partitions, omega=2.0 / 3.0, smoother="jacobi", omega_s=2.0 / 3.0,
                 n_bins=4, max_dyn_blocks=4096):
        self.prob = prob
        self.A, self.b, self.Ab, self.cells = assemble(prob)
        self.omega, self.omega_s = omega, omega_s
        self.n_bins, self.max_dyn_blocks = n_bins, max_dyn_blocks
        self.smoother = smoother
        if not partitions or partitions[0].get("kind") != "cartesian":
            raise OracleError(E_INVAL, "the first partition must be a Cartesian (general) one")
        self.stages = []
        for part in partitions:
            if part["kind"] == "cartesian":
                block, M, present = cartesian_partition(prob.dims, part["coarse_dims"], prob.active)
                S = cartesian_support(prob.dims, part["coarse_dims"], prob.active, present)
            elif part["kind"] == "fault_cut":
                par = self.stages[part["parent"]]
                block, M, S = fault_cut_partition(prob, par.block, par.S, self.cells)
            elif part["kind"] == "graph":
                block, M, S = graph_partition(prob, part["block_of_cell"], part.get("overlap", 0), self.cells)
            else:
                raise OracleError(E_INVAL, f"unknown partition kind {part['kind']}")
            self.stages.append(_Stage(part["kind"], block, M, S))
        self.dyn = []
        self._factor_smoother()
        self.ready = False

    # -- basis ---------------------------------------------------------------
    def _factor_smoother(self):
        if self.smoother == "jacobi":
            self.fac = None
        elif self.smoother == "ilu0_nat":
            self.fac = ilu0_factor(self.A, natural_order(self.cells, self.prob.dims))
        elif self.smoother == "ilu0_rb":
            self.fac = ilu0_factor(self.A, red_black_order(self.cells, self.prob.dims))
        elif self.smoother == "ilu0_line":
            self.fac = ilu0_factor(self.A, zline_red_black_order(self.cells, self.prob.dims))
        else:
            raise OracleError(E_INVAL, f"unknown smoother {self.smoother}")

    def update_basis(self, max_sweeps=100, tol=1e-3, stage=-1, warm=False, new_trans=None, new_bc_trans=None):
        """Restricted smoothing of one stage (or all general/static stages),
        then Galerkin operators and coarse factors.  ``new_trans = (tx, ty,
        tz)`` first replaces the face transmissibilities ("changing
        reservoir/fluid properties"; ``new_bc_trans`` likewise replaces the
        boundary/well connection coefficients): the operator and smoother are rebuilt,
        the named stages are smoothed with the new operator (from their
        current basis when ``warm``), and every other stage keeps its basis
        and gets its coarse operator rebuilt for the new operator."""
        import copy

        todo = range(len(self.stages)) if stage < 0 else [stage]
        changed = new_trans is not None or new_bc_trans is not None
        if changed:
            prob = copy.copy(self.prob)
            if new_trans is not None:
                prob.tx, prob.ty, prob.tz = (np.asarray(t, dtype=np.float64).copy() for t in new_trans)
            if new_bc_trans is not None:
                prob.bc_trans = np.asarray(new_bc_trans, dtype=np.float64).copy()
            A, b, Ab, cells = assemble(prob)
            if not np.array_equal(cells, self.cells):
                raise OracleError(E_INVAL, "the active cells cannot change")
            self.prob, self.A, self.b, self.Ab = prob, A, b, Ab
            self._factor_smoother()
        for s in todo:
            st = self.stages[s]
            P0 = st.P if (warm and st.P is not None) else None
            st.P, st.sweeps, st.change = msrsb_basis(self.Ab, st.block[self.cells], st.S, self.omega, tol,
                                                     max_sweeps, P0)
            st.Ac = galerkin(st.P, self.A)
            st.L = coarse_factor(st.Ac)
        if changed:
            for k, st in enumerate(self.stages):
                if k not in todo and st.P is not None:
                    st.Ac = galerkin(st.P, self.A)
                    st.L = coarse_factor(st.Ac)
            for st in self.dyn:
                st.Ac = galerkin(st.P, self.A)
                st.L = coarse_factor(st.Ac)
        self.ready = all(st.P is not None for st in self.stages)
        return [self.stages[s].sweeps for s in todo]

    def add_dynamic_basis(self, increments):
        """One constant-basis stage per increment (newest first, at most 2);
        replaces the previous dynamic stages.  Returns blocks per increment."""
        if len(increments) > 2:
            raise OracleError(E_INVAL, "at most two increments")
        self.dyn = []
        counts = []
        for dp in increments:
            res = dynamic_partition(self.prob, dp, self.stages[0].block, self.n_bins, self.max_dyn_blocks)
            if res is None:
                counts.append(0)
                continue
            block, M, _ = res
            P = indicator(block[self.cells], M)
            st = _Stage("dynamic", block, M, None, P)
            st.Ac = galerkin(P, self.A)
            st.L = coarse_factor(st.Ac)
            self.dyn.append(st)
            counts.append(M)
        return counts

    def clear_dynamic_basis(self):
        self.dyn = []

    def all_stages(self):
        return list(self.stages) + list(self.dyn)

    # -- smoother / cycle ----------------------------------------------------
    def smooth(self, r):
        if self.fac is None:
            return jacobi_correction(self.A, r, self.omega_s)
        return ilu0_apply(self.fac, r)

    def stage_step(self, st, x, b):
        """One stage of eq. multiscale-multibasis: smoother, then coarse correction."""
        x = x + self.smooth(b - self.A @ x)
        r = b - self.A @ x
        pc = coarse_solve(st.L, st.P.T @ r)
        return x + st.P @ pc

    def solve(self, source=None, x0=None, rtol=1e-6, max_cycles=500, history=False):
        """Returns ``(x_box, cycles, relres, status[, hist])``."""
        if not self.ready:
            raise OracleError(E_STATE, "update_basis has not run")
        b = self.b if source is None else rhs_for(self.prob, self.cells, source)
        x = np.zeros(self.cells.size) if x0 is None else np.asarray(x0, dtype=np.float64)[self.cells].copy()
        nb = float(np.linalg.norm(b))
        denom = nb if nb > 0 else 1.0
        rel = float(np.linalg.norm(b - self.A @ x)) / denom
        hist = [rel]
        cycles = 0
        status = 0
        stages = self.all_stages()
        while rel > rtol:
            if cycles >= max_cycles:
                status = E_NOCONV
                break
            for st in stages:
                x = self.stage_step(st, x, b)
            cycles += 1
            rel = float(np.linalg.norm(b - self.A @ x)) / denom
            hist.append(rel)
        xb = np.zeros(self.prob.n_cells)
        xb[self.cells] = x
        if history:
            return xb, cycles, rel, status, hist
        return xb, cycles, rel, status

    def precondition(self, r):
        """One multistage cycle from a zero guess applied to ``r`` (the
        multiscale preconditioner ``M^{-1} r``)."""
        x = np.zeros_like(r)
        for st in self.all_stages():
            x = self.stage_step(st, x, r)
        return x

    def solve_gmres(self, source=None, x0=None, rtol=1e-6, max_iters=500, restart=30, history=False):
        """Restarted GMRES(m) with the multistage cycle as right preconditioner
        (section "Description of the solution procedure"), following the
        Arnoldi/least-squares form of Saad & Schultz (modified Gram-Schmidt,
        least-squares problem solved directly).  Convergence is tested on the
        least-squares residual after every inner step and confirmed on the
        true residual at each restart.  Returns ``(x_box, iterations, relres,
        status[, hist])``."""
        if not self.ready:
            raise OracleError(E_STATE, "update_basis has not run")
        b = self.b if source is None else rhs_for(self.prob, self.cells, source)
        x = np.zeros(self.cells.size) if x0 is None else np.asarray(x0, dtype=np.float64)[self.cells].copy()
        nb = float(np.linalg.norm(b))
        denom = nb if nb > 0 else 1.0
        its = 0
        status = 0
        hist = []
        while True:
            r = b - self.A @ x
            beta = float(np.linalg.norm(r))
            hist.append(beta / denom)
            if beta / denom <= rtol:
                break
            if its >= max_iters:
                status = E_NOCONV
                break
            V = [r / beta]
            H = np.zeros((restart + 1, restart))
            y = None
            for j in range(restart):
                w = self.A @ self.precondition(V[j])
                for i in range(j + 1):
                    H[i, j] = float(w @ V[i])
                    w = w - H[i, j] * V[i]
                H[j + 1, j] = float(np.linalg.norm(w))
                its += 1
                e1 = np.zeros(j + 2)
                e1[0] = beta
                y = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)[0]
                est = float(np.linalg.norm(e1 - H[:j + 2, :j + 1] @ y))
                hist.append(est / denom)
                if H[j + 1, j] == 0.0 or est / denom <= rtol or its >= max_iters:
                    break
                V.append(w / H[j + 1, j])
            k = y.size
            x = x + self.precondition(np.column_stack(V[:k]) @ y)
        xb = np.zeros(self.prob.n_cells)
        xb[self.cells] = x
        rel = hist[-1]
        if history:
            return xb, its, rel, status, hist
        return xb, its, rel, status

    def solve_fv(self, stage=0, source=None):
        """Finite-volume multiscale pressure of a general/static stage and the
        conservative reconstruction.  Returns ``(pms_box, pfine_box, face[3,
        N], bc_flux, A_fv)``."""
        if not self.ready:
            raise OracleError(E_STATE, "update_basis has not run")
        st = self.stages[stage]
        b = self.b if source is None else rhs_for(self.prob, self.cells, source)
        bl = st.block[self.cells]
        pms, Afv = fv_multiscale_pressure(st.P, self.A, b, bl, st.M)
        bcd = np.zeros(self.prob.n_cells)
        np.add.at(bcd, np.asarray(self.prob.bc_cell), np.asarray(self.prob.bc_trans))
        pf = conservative_pressure(self.A, b, bl, st.M, pms, bcd[self.cells])
        face, bcf = reconstructed_fluxes(self.prob, self.cells, bl, pms, pf)
        box = lambda v: np.bincount(self.cells, weights=v, minlength=self.prob.n_cells)
        return box(pms), box(pf), face, bcf, Afv

    def direct_solve(self, source=None):
        """The exact fine-scale solution ``A^{-1} b`` (sparse LU)."""
        b = self.b if source is None else rhs_for(self.prob, self.cells, source)
        x = spla.spsolve(self.A.tocsc(), b)
        xb = np.zeros(self.prob.n_cells)
        xb[self.cells] = x
        return xb

    def residual(self, x_box, source=None):
        b = self.b if source is None else rhs_for(self.prob, self.cells, source)
        return b - self.A @ np.asarray(x_box)[self.cells]

    def export_basis(self, stage):
        """Dense ``N_box x M`` basis of a general/static stage (tests only)."""
        st = self.all_stages()[stage]
        P = np.zeros((self.prob.n_cells, st.M))
        P[self.cells] = st.P.toarray()
        return P

    def fluxes(self, x_box):
        return fluxes(self.prob, np.asarray(x_box))
