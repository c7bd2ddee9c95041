"""Host logic of the multigrid preconditioner: the node aggregation rule
(lgdm_amg_aggregate runs on the host, no device call)."""
import numpy as np
import pytest

from paper_2301_06503_amd import binding


def _csr(n, edges):
    """CSR with sorted neighbour lists that include the node itself."""
    nb = [{a} for a in range(n)]
    for a, b in edges:
        nb[a].add(b)
        nb[b].add(a)
    ptr = np.zeros(n + 1, dtype=np.int32)
    adj = []
    for a in range(n):
        adj.extend(sorted(nb[a]))
        ptr[a + 1] = len(adj)
    return ptr, np.array(adj, dtype=np.int32)


def _grid(nx, ny, nz):
    """Node graph of an nx x ny x nz-element hex8 mesh (nodes share an element)."""
    idx = lambda i, j, k: i + (nx + 1) * (j + (ny + 1) * k)
    edges = []
    for k in range(nz + 1):
        for j in range(ny + 1):
            for i in range(nx + 1):
                for dk in (-1, 0, 1):
                    for dj in (-1, 0, 1):
                        for di in (-1, 0, 1):
                            ii, jj, kk = i + di, j + dj, k + dk
                            if 0 <= ii <= nx and 0 <= jj <= ny and 0 <= kk <= nz:
                                edges.append((idx(i, j, k), idx(ii, jj, kk)))
    return _csr((nx + 1) * (ny + 1) * (nz + 1), edges)


def test_path_graph_by_hand():
    # 0-1-2-3-4: node 0 takes {0, 1}; node 2 sees aggregated node 1; node 3
    # takes {2, 3, 4}
    ptr, adj = _csr(5, [(0, 1), (1, 2), (2, 3), (3, 4)])
    agg, na = binding.amg_aggregate(ptr, adj)
    assert na == 2
    assert agg.tolist() == [0, 0, 1, 1, 1]


def test_3x3_nine_point_by_hand():
    # 3 x 3 nodes, every pair in a common square connected: node 0 takes
    # {0, 1, 3, 4}; no other node has all neighbours free; the rest join
    # aggregate 0 through their first aggregated neighbour
    ptr, adj = _grid(2, 2, 0)
    agg, na = binding.amg_aggregate(ptr, adj)
    assert na == 1
    assert agg.tolist() == [0] * 9


def test_hex_grid_partition():
    """9 x 9 x 9 nodes: every node in exactly one aggregate, aggregates
    connected, numbered in order of creation; the first-pass aggregates are
    the 27-node neighbourhoods of their roots (2 x 2 x 2 at the corner)."""
    ptr, adj = _grid(8, 8, 8)
    n = len(ptr) - 1
    agg, na = binding.amg_aggregate(ptr, adj)
    assert agg.min() == 0 and agg.max() == na - 1
    # creation order: the first node of aggregate j has a lower id than the
    # first node of aggregate j + 1
    first = np.array([np.flatnonzero(agg == j)[0] for j in range(na)])
    assert np.all(np.diff(first) > 0)
    # connectivity of every aggregate within the graph
    for j in range(na):
        mem = set(np.flatnonzero(agg == j).tolist())
        seen, stack = set(), [next(iter(mem))]
        while stack:
            a = stack.pop()
            if a in seen:
                continue
            seen.add(a)
            stack.extend(b for b in adj[ptr[a]:ptr[a + 1]] if b in mem and b not in seen)
        assert seen == mem
    # node 0 (corner) is the first root: its aggregate is its 2 x 2 x 2 block
    assert sorted(np.flatnonzero(agg == 0).tolist()) == sorted(
        i + 9 * (j + 9 * k) for i in (0, 1) for j in (0, 1) for k in (0, 1))
    # node (3, 0, 0) is the next root: its neighbourhood x in 2..4
    assert agg[3] == 1
    assert sorted(np.flatnonzero(agg == 1).tolist()) == sorted(
        i + 9 * (j + 9 * k) for i in (2, 3, 4) for j in (0, 1) for k in (0, 1))
    # coarsening factor between 8 and 27 on this graph
    assert 8 <= n / na <= 27


def test_invalid_graph_rejected():
    ptr = np.array([0, 2], dtype=np.int32)
    adj = np.array([0, 5], dtype=np.int32)  # neighbour id out of range
    with pytest.raises(binding.LgdmError):
        binding.amg_aggregate(ptr, adj)


def test_empty_graph():
    agg, na = binding.amg_aggregate(np.zeros(1, dtype=np.int32), np.zeros(0, dtype=np.int32))
    assert na == 0 and agg.size == 0
