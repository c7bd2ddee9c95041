"""Host logic of the serving loop's report (no device): per-increment and
per-request latency statistics, finished-request throughput, failures and
retries, computed from request records by ServingLoop.summary."""
import numpy as np
import pytest

from paper_2301_06503_amd import serving


def _loop(records, wall_s):
    loop = object.__new__(serving.ServingLoop)   # the report only, no batch on a device
    loop.records = {r.rid: r for r in records}
    loop.wall_s = wall_s
    loop.gp_assembled = 1000
    loop.t_assembly_ms = 2.0
    loop.ticks = 7
    return loop


def _rec(rid, arrival, admitted, finished, state, increments, lat, gp=100, retries=0, cutbacks=0):
    r = serving.RequestRecord(rid, arrival)
    r.admitted_s, r.finished_s, r.state, r.increments = admitted, finished, state, increments
    r.increment_latency_ms = list(lat)
    r.gauss_points = gp
    r.retries = retries
    r.cutbacks = cutbacks
    return r


def test_summary_whole_requests():
    recs = [_rec(0, 0.0, 0.5, 4.5, "finished", 3, [1000.0, 1500.0, 1500.0], retries=1),
            _rec(1, 1.0, 1.0, 3.0, "finished", 2, [900.0, 1100.0]),
            _rec(2, 2.0, 2.5, 6.0, "failed(NOT_CONVERGED)", 1, [800.0], retries=1, cutbacks=3),
            _rec(3, 3.0, None, None, "queued", 0, [])]
    s = _loop(recs, 10.0).summary()
    assert s["requests_arrived"] == 4
    assert s["requests_finished"] == 2 and s["requests_failed"] == 1
    assert s["failed_requests"] == [(2, "failed(NOT_CONVERGED)", 1)]
    assert s["increment_retries"] == 2
    assert s["load_step_cutbacks"] == 3
    # completion latency: arrival to the last commit, finished requests only
    assert s["request_latency_p50_s"] == pytest.approx(np.percentile([4.5, 2.0], 50))
    assert s["request_latency_max_s"] == pytest.approx(4.5)
    assert s["request_service_p50_s"] == pytest.approx(np.percentile([4.0, 2.0], 50))
    assert s["requests_per_s"] == pytest.approx(0.2)
    # Gauss-point increments of the finished requests per second
    assert s["finished_gauss_point_increments_per_s"] == pytest.approx((100 * 3 + 100 * 2) / 10.0)
    # per-increment latency over every committed increment, failed requests included
    lat = [1000.0, 1500.0, 1500.0, 900.0, 1100.0, 800.0]
    assert s["increments_committed"] == 6
    assert s["latency_p50_ms"] == pytest.approx(np.percentile(lat, 50))
    assert s["latency_p99_ms"] == pytest.approx(np.percentile(lat, 99))
    assert s["admission_wait_max_s"] == pytest.approx(0.5)


def test_summary_without_finished_requests():
    s = _loop([_rec(0, 0.0, 0.1, None, "running", 1, [500.0])], 3.0).summary()
    assert s["requests_finished"] == 0
    assert s["request_latency_p50_s"] is None and s["request_latency_max_s"] is None
    assert s["requests_per_s"] == 0.0
