"""Host logic of the process-zone solve: the breadth-first level sets that
make the zone's block tridiagonal (lgdm_zone_levels runs on the host, no
device call).  Checked against properties any correct breadth-first search
has, on graphs whose level counts are known by hand."""
import numpy as np
import pytest

from paper_2301_06503_amd import binding
from tests.test_amg_host import _csr, _grid


def _check_bfs_levels(ptr, adj, level, n_levels):
    """Every edge joins equal or consecutive levels; within a connected
    component the levels form one contiguous run that starts at a single
    node, and every other node has a neighbour one level closer to it."""
    n = len(ptr) - 1
    assert level.min() == 0 and level.max() == n_levels - 1
    nb = [adj[ptr[a]:ptr[a + 1]] for a in range(n)]
    for a in range(n):
        for b in nb[a]:
            assert abs(int(level[a]) - int(level[b])) <= 1, (a, b)
    # components (by a plain traversal), their level runs
    comp = -np.ones(n, dtype=int)
    runs = []
    for s in range(n):
        if comp[s] >= 0:
            continue
        stack, members = [s], []
        comp[s] = len(runs)
        while stack:
            v = stack.pop()
            members.append(v)
            for w in nb[v]:
                if comp[w] < 0:
                    comp[w] = len(runs)
                    stack.append(w)
        lv = level[members]
        assert set(lv.tolist()) == set(range(lv.min(), lv.max() + 1))
        assert np.count_nonzero(lv == lv.min()) == 1          # one start node
        for v in members:
            if level[v] > lv.min():
                assert any(level[w] == level[v] - 1 for w in nb[v]), v
        runs.append((int(lv.min()), int(lv.max()), min(members)))
    # components follow each other in the order of their lowest node
    runs.sort(key=lambda r: r[2])
    for (a0, a1, _), (b0, b1, _) in zip(runs, runs[1:]):
        assert b0 == a1 + 1
    return runs


def test_path_graph_starts_at_an_end():
    # a path in scrambled numbering: from any node, the pseudo-peripheral
    # search ends at an end of the path, so the levels run along it
    rng = np.random.default_rng(3)
    n = 37
    perm = rng.permutation(n)
    ptr, adj = _csr(n, [(perm[i], perm[i + 1]) for i in range(n - 1)])
    level, nl = binding.zone_levels(ptr, adj)
    assert nl == n
    assert {int(level[perm[0]]), int(level[perm[-1]])} == {0, n - 1}
    _check_bfs_levels(ptr, adj, level, nl)


@pytest.mark.parametrize("nx,ny,nz", [(6, 3, 2), (2, 9, 4), (3, 3, 3)])
def test_hex8_node_graph(nx, ny, nz):
    # node graph of a hex8 block: a breadth-first level is a shell of
    # Chebyshev distance from a corner, so there are max(nx, ny, nz) + 1
    ptr, adj = _grid(nx, ny, nz)
    level, nl = binding.zone_levels(ptr, adj)
    assert nl == max(nx, ny, nz) + 1
    _check_bfs_levels(ptr, adj, level, nl)


def test_components_follow_each_other():
    # two hex8 blocks and an isolated node, interleaved in numbering
    pa, aa = _grid(2, 1, 1)
    na = len(pa) - 1
    edges = []
    for a in range(na):
        for b in aa[pa[a]:pa[a + 1]]:
            edges.append((2 * a, 2 * b))              # block A on even ids
    for a in range(na):
        for b in aa[pa[a]:pa[a + 1]]:
            if a < na - 1 and b < na - 1:
                edges.append((2 * a + 1, 2 * b + 1))  # block B on odd ids, minus its last node
    n = 2 * na
    ptr, adj = _csr(n, edges)
    level, nl = binding.zone_levels(ptr, adj)
    runs = _check_bfs_levels(ptr, adj, level, nl)
    assert len(runs) == 3                             # A, B and the lone node 2 na - 1
    assert runs[-1][0] == runs[-1][1] == nl - 1


def test_self_loops_and_errors():
    ptr, adj = _csr(4, [(0, 1), (1, 2), (2, 3)])       # lists include the node itself
    level, nl = binding.zone_levels(ptr, adj)
    assert nl == 4 and sorted(level.tolist()) == [0, 1, 2, 3]
    level, nl = binding.zone_levels(np.zeros(1, dtype=np.int32), np.zeros(0, dtype=np.int32))
    assert nl == 0 and len(level) == 0
    with pytest.raises(binding.LgdmError):
        binding.zone_levels(np.array([0, 1], dtype=np.int32), np.array([5], dtype=np.int32))
    with pytest.raises(binding.LgdmError):
        binding.zone_levels(np.array([1, 1], dtype=np.int32), np.array([0], dtype=np.int32))


@pytest.mark.parametrize("n_groups", [1, 2, 3, 4, 5, 8, 9])
def test_twisted_block_solve_formulas(n_groups):
    """The algebra the process-zone solve runs on the GPU, written out on a
    random block-tridiagonal system: twisted block LU from both ends toward
    the middle group (inverses G_k of the Schur complements, P_k = G_k
    Z_k,k-1, N_k = G_k Z_k,k+1), sweeps from both ends, the middle group,
    and the sweeps back out, equals a dense solve."""
    rng = np.random.default_rng(n_groups)
    L = n_groups
    ms = rng.integers(3, 7, size=L)
    off = np.concatenate([[0], np.cumsum(ms)])
    n = int(off[-1])
    Z = np.zeros((n, n))
    for k in range(L):
        sk = slice(off[k], off[k + 1])
        Z[sk, sk] = rng.standard_normal((ms[k], ms[k])) + 4.0 * np.eye(ms[k])
        if k > 0:
            Z[sk, off[k - 1]:off[k]] = rng.standard_normal((ms[k], ms[k - 1]))
            Z[off[k - 1]:off[k], sk] = rng.standard_normal((ms[k - 1], ms[k]))
    blk = lambda i, j: Z[off[i]:off[i + 1], off[j]:off[j + 1]]
    c = L // 2
    G, P, N = [None] * L, [None] * L, [None] * L

    def finish(k, S):
        G[k] = np.linalg.inv(S)
        if k > 0:
            P[k] = G[k] @ blk(k, k - 1)
        if k < L - 1:
            N[k] = G[k] @ blk(k, k + 1)

    for k in range(c):
        finish(k, blk(k, k) - (blk(k, k - 1) @ N[k - 1] if k > 0 else 0.0))
    for k in range(L - 1, c, -1):
        finish(k, blk(k, k) - (blk(k, k + 1) @ P[k + 1] if k < L - 1 else 0.0))
    S = blk(c, c).copy()
    if c > 0:
        S -= blk(c, c - 1) @ N[c - 1]
    if c < L - 1:
        S -= blk(c, c + 1) @ P[c + 1]
    finish(c, S)
    b = rng.standard_normal(n)
    x = np.zeros(n)
    seg = lambda k: slice(off[k], off[k + 1])
    for s in range(max(c, L - 1 - c)):
        if s < c:
            x[seg(s)] = G[s] @ b[seg(s)] - (P[s] @ x[seg(s - 1)] if s > 0 else 0.0)
        k = L - 1 - s
        if k > c:
            x[seg(k)] = G[k] @ b[seg(k)] - (N[k] @ x[seg(k + 1)] if k < L - 1 else 0.0)
    x[seg(c)] = (G[c] @ b[seg(c)] - (P[c] @ x[seg(c - 1)] if c > 0 else 0.0)
                 - (N[c] @ x[seg(c + 1)] if c < L - 1 else 0.0))
    for s in range(max(c, L - 1 - c)):
        if c - 1 - s >= 0:
            k = c - 1 - s
            x[seg(k)] -= N[k] @ x[seg(k + 1)]
        if c + 1 + s <= L - 1:
            k = c + 1 + s
            x[seg(k)] -= P[k] @ x[seg(k - 1)]
    ref = np.linalg.solve(Z, b)
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)
