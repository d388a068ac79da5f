"""Pins of the oracle's graph, well and indicator partitions (partition types
"General" and "Static" of the subsection "Iterative multiscale multibasis
solver") against independent statements: hand-worked examples and
brute-force loops over every (cell, block) pair on small grids."""
from collections import deque

import numpy as np
import pytest

import oracle as O
from workloads import make_config1, make_config2, make_lognormal_box, rng_for


def neighbours(prob):
    """Face adjacency (T > 0) by explicit loops over the three face arrays."""
    nx, ny, nz = prob.dims
    adj = {i: [] for i in range(prob.n_cells)}
    for T, step in ((prob.tx, 1), (prob.ty, nx), (prob.tz, nx * ny)):
        for i in range(prob.n_cells):
            if T[i] > 0:
                adj[i].append(i + step)
                adj[i + step].append(i)
    return adj


def bfs_dist(adj, sources, n):
    d = [None] * n
    q = deque()
    for s in sources:
        d[s] = 0
        q.append(s)
    while q:
        u = q.popleft()
        for v in adj[u]:
            if d[v] is None:
                d[v] = d[u] + 1
                q.append(v)
    return d


def small_problem(seed):
    prob = make_config2(dims=(7, 6, 4), seed=seed, p_inactive=0.1)
    return prob


def test_graph_support_hand_example_chain():
    # six cells in a line, blocks [5,5,9,9,9,2] -> ascending ids 2,5,9 -> 0,1,2
    from workloads.grids import make_homogeneous

    prob = make_homogeneous((6, 1, 1))
    blk = np.array([5, 5, 9, 9, 9, 2])
    cells = np.arange(6)
    block, M, S = O.graph_partition(prob, blk, 1, cells)
    assert M == 3 and list(block) == [1, 1, 2, 2, 2, 0]
    sets = [set(np.nonzero(S[:, j].toarray().ravel())[0]) for j in range(M)]
    assert sets == [{4, 5}, {0, 1, 2}, {1, 2, 3, 4, 5}]
    _, _, S0 = O.graph_partition(prob, blk, 0, cells)
    assert (S0.toarray() == O.indicator(block, M).toarray()).all()


@pytest.mark.parametrize("seed,overlap", [(0, 0), (1, 1), (2, 2), (3, 3)])
def test_graph_support_brute_force(seed, overlap):
    prob = small_problem(seed)
    rng = np.random.default_rng(seed)
    cells = np.nonzero(prob.active)[0]
    ids = rng.integers(0, 12, prob.n_cells) * 3 + 1  # sparse ids
    block, M, S = O.graph_partition(prob, ids, overlap, cells)
    present = sorted(set(ids[cells].tolist()))
    assert M == len(present)
    for c in cells:
        assert block[c] == present.index(ids[c])
    adj = neighbours(prob)
    Sd = S.toarray() > 0
    loc = {c: r for r, c in enumerate(cells)}
    for j, pid in enumerate(present):
        members = [c for c in cells if ids[c] == pid]
        d = bfs_dist(adj, members, prob.n_cells)
        for c in cells:
            assert Sd[loc[c], j] == (d[c] is not None and d[c] <= overlap), (c, j)


def test_graph_basis_overlap_zero_is_indicator():
    prob = small_problem(4)
    cells = np.nonzero(prob.active)[0]
    ids = np.arange(prob.n_cells) % 5
    o = O.Oracle(prob, [{"kind": "cartesian", "coarse_dims": (2, 2, 1)},
                        {"kind": "graph", "block_of_cell": ids, "overlap": 0}])
    o.update_basis(max_sweeps=7, tol=0.0)
    P = o.stages[1].P.toarray()
    assert np.array_equal(P, O.indicator(o.stages[1].block[cells], o.stages[1].M).toarray())


def test_well_partition_hand_example():
    from workloads.grids import make_homogeneous

    prob = make_homogeneous((7, 1, 1))
    # wells at cells 1 and 5; radius 2: cell 3 is two steps from both -> the lower well index
    out = O.well_partition(prob, [np.array([1]), np.array([5])], 2)
    assert list(out) == [0, 0, 0, 0, 1, 1, 1]
    out1 = O.well_partition(prob, [np.array([1]), np.array([5])], 1)
    assert list(out1) == [0, 0, 0, 2, 1, 1, 1]
    out0 = O.well_partition(prob, [np.array([1]), np.array([5])], 0)
    assert list(out0) == [2, 0, 2, 2, 2, 1, 2]


@pytest.mark.parametrize("seed,radius", [(0, 0), (1, 1), (2, 3)])
def test_well_partition_brute_force(seed, radius):
    prob = small_problem(seed)
    rng = np.random.default_rng(10 + seed)
    cells = np.nonzero(prob.active)[0]
    wells = [rng.choice(cells, size=int(rng.integers(1, 4)), replace=False) for _ in range(3)]
    out = O.well_partition(prob, wells, radius)
    adj = neighbours(prob)
    dists = [bfs_dist(adj, list(w), prob.n_cells) for w in wells]
    for c in range(prob.n_cells):
        if not prob.active[c]:
            assert out[c] == -1
            continue
        best, bd = len(wells), None
        for w in range(len(wells)):  # first minimum wins
            d = dists[w][c]
            if d is not None and d <= radius and (bd is None or d < bd):
                best, bd = w, d
        assert out[c] == best, c


def test_indicator_partition_hand_example():
    from workloads.grids import make_homogeneous

    prob = make_homogeneous((8, 1, 1))
    ind = np.array([0.1, 0.2, 5.0, 6.0, 0.3, 7.0, 0.4, 8.0])
    # two bins of four: low {0,1,4,6}, high {2,3,5,7}; pieces {0,1},{2,3},{4},{5},{6},{7}
    out = O.indicator_partition(prob, ind, 2, (1, 1, 1), 0)
    assert list(out) == [0, 0, 1, 1, 2, 3, 4, 5]
    # min_cells 2: {4} (smallest of the size-1 pieces by smallest cell) has neighbours {2,3} (1 face) and
    # {5} (1 face): tie -> smaller smallest cell {2,3}; then {5} joins {2,3,4} (its only... shares 1 face
    # with each of {2,3,4} and {6}: tie -> {2,3,4}); then {6} joins ... {7} joins {6}? -> by the rule
    out2 = O.indicator_partition(prob, ind, 2, (1, 1, 1), 2)
    # after {4}->{2,3,4} and {5}->{2,3,4,5}: {6} (size 1) neighbours {2..5} only (1 face) and {7} (1 face):
    # tie -> {2..5}; then {7} (size 1) joins {2..6}
    assert list(out2) == [0, 0, 1, 1, 1, 1, 1, 1]
    # parent blocks bound the pieces: two parents of four cells, no merges across them
    out3 = O.indicator_partition(prob, ind, 2, (2, 1, 1), 3)
    assert len(set(out3[:4]) & set(out3[4:])) == 0


def test_indicator_partition_properties():
    prob = make_lognormal_box((12, 10, 4), rng_for(9, 0), sigma=2.0, corr=(2.0, 2.0, 1.0))
    ind = np.log(prob.perm)
    cd = (3, 2, 2)
    out = O.indicator_partition(prob, ind, 4, cd, 6)
    cells = np.nonzero(prob.active)[0]
    parent, _, _ = O.cartesian_partition(prob.dims, cd, np.ones(prob.n_cells, bool))
    adj = neighbours(prob)
    M = out.max() + 1
    firsts = []
    for j in range(M):
        mem = np.nonzero(out == j)[0]
        assert mem.size > 0
        firsts.append(mem.min())
        assert len(set(parent[mem])) == 1  # inside one parent block
        d = bfs_dist({c: [v for v in adj[c] if out[v] == j] for c in adj}, [mem[0]], prob.n_cells)
        assert all(d[c] is not None for c in mem)  # connected
    assert firsts == sorted(firsts)  # numbered by smallest cell
    # every block below min_cells has no same-parent neighbour block
    for j in range(M):
        mem = np.nonzero(out == j)[0]
        if mem.size < 6:
            for c in mem:
                assert all(out[v] == j or parent[v] != parent[c] for v in adj[c])
    # equal-count bins: without merging, bins split the ranked cells into four equal groups
    raw = O.indicator_partition(prob, ind, 4, (1, 1, 1), 0)
    order = np.lexsort((cells, ind[cells]))
    q = cells.size // 4
    for k in range(4):
        grp = cells[order[k * q:(k + 1) * q]]
        other = np.setdiff1d(cells, grp)
        assert not (set(raw[grp]) & set(raw[other]))  # no block mixes bins
