"""Host arithmetic of bench.py's measurement (no device): the algorithmic
bytes of the SpMV against a closed form of the structured hex8 node graph,
the combined assembly + SpMV roofline, the load-path phase split, and the
rule that counter traffic is reported only for the source it was taken on."""
import json
import os
import types

import pytest

import bench


def _hex8_pairs(nx, ny, nz):
    """Node pairs of the 27-neighbour graph of an nx x ny x nz hex8 grid,
    self pairs included: per axis, a node has 3 neighbours along it (2 at
    either end), and the counts multiply."""
    def axis(n):
        return 3 * (n + 1) - 2
    return axis(nx) * axis(ny) * axis(nz)


def _prob(nx, ny, nz):
    nn = (nx + 1) * (ny + 1) * (nz + 1)
    ne = nx * ny * nz
    return types.SimpleNamespace(ndof=4 * nn, n_nodes=nn, n_elems=ne, ngp=8, dim=3, nen=8)


def test_hex8_pair_count_by_brute_force():
    nx, ny, nz = 3, 2, 4
    idx = [(i, j, k) for i in range(nx + 1) for j in range(ny + 1) for k in range(nz + 1)]
    brute = sum(1 for a in idx for b in idx if all(abs(p - q) <= 1 for p, q in zip(a, b)))
    assert brute == _hex8_pairs(nx, ny, nz)


def test_spmv_algorithmic_bytes_of_the_bench_beam():
    # 256 x 64 x 32 hex8, FP32 values: the figure the bench line reports
    nx, ny, nz = 256, 64, 32
    prob = _prob(nx, ny, nz)
    npairs = _hex8_pairs(nx, ny, nz)
    nnz = 16 * npairs
    asm, spmv = bench.algorithmic_bytes(prob, nnz, npairs, 4)
    assert spmv == 1018649616
    # values, one int32 per node pair, the row offset of each node and the
    # node-graph offsets, x read and y written in FP64
    assert spmv == nnz * 4 + npairs * 4 + prob.n_nodes * 4 + (prob.n_nodes + 1) * 4 + prob.ndof * 16
    assert asm > nnz * 4


def test_assembly_spmv_roofline():
    res = {"assemblies": 10, "assembly_bytes": 1.0e9, "spmv_launches": 1000,
           "kernel_ms": {"gauss_point": 0.5, "node_assembly": 3.5},
           "probe": {"gbs": 5000.0, "algorithmic_bytes": 1.0e9, "avg_ms": 0.2}}
    r = bench.assembly_spmv_roofline(res)
    # (10 + 1000) GB in (40 + 200) ms
    assert r["bytes"] == pytest.approx(1010e9)
    assert r["kernel_ms"] == pytest.approx(240.0)
    assert r["achieved"] == pytest.approx(1010e9 / 0.240 / 1e9, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.HBM_PEAK_GBS, rel=1e-3)
    res["spmv_launches"] = 0
    assert bench.assembly_spmv_roofline(res) is None


def test_window_phases():
    # increment, ms, newton, krylov, reaction: the peak at increment 3
    rows = [[1, 100.0, 4, 400, -10.0], [2, 120.0, 5, 500, -20.0], [3, 300.0, 6, 900, -30.0],
            [4, 500.0, 8, 1600, -25.0], [5, 700.0, 10, 3000, -20.0]]
    ph = bench.window_phases(rows)
    assert ph["pre_peak"]["increments"] == [1, 2]
    assert ph["near_peak"]["increments"] == [3, 3]
    assert ph["post_peak"]["increments"] == [4, 5]
    assert ph["post_peak"]["ms_per_increment_median"] == pytest.approx(600.0)
    assert ph["post_peak"]["krylov_per_newton_median"] == pytest.approx((200.0 + 300.0) / 2)
    assert bench.window_phases([]) is None


def test_committed_traffic_follows_the_source():
    path = os.path.join(bench.ROOT, "profiles", "pmc_traffic.json")
    rec = json.load(open(path))
    key = "c3_mixed_spmv"
    assert key in rec
    import hashlib
    src = os.path.join(bench.ROOT, rec[key]["source"])
    current = hashlib.sha256(open(src, "rb").read()).hexdigest() == rec[key]["source_sha256"]
    # the counters are reported for the source they were taken on, else null
    expect = rec[key]["hbm_bytes_per_launch"] if current else None
    assert bench.committed_traffic(key, None) == expect
    assert bench.committed_traffic("no_such_kernel", None) is None
