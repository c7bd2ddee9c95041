"""Serving loop: continuous batching of LGDM simulation requests.

Requests arrive over time (each an lgdm_workloads.Request: arrival time and
problem).  Arrived requests wait in a FIFO queue and are admitted into the
device batch as soon as a slot and enough of the HBM budget are free; every
tick advances all admitted requests by one Newton iteration (one fused launch
of each element kernel for all of them, per-request solves overlapping on the
device); requests whose load path is complete (or that failed) are retired,
which frees their slot and memory for the queue.

Reported per run: per-increment latency (wall time from the tick that starts
an increment's first Newton iteration to the tick that commits it), p50 and
p99 over all committed increments; per finished request, the latency from
arrival to its last commit and the service time from admission, p50 and p99;
finished requests per second; aggregate assembled Gauss points per second,
admission waits and per-request outcomes.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Dict, List, Optional

import numpy as np

from . import binding


@dataclasses.dataclass
class RequestRecord:
    rid: int
    arrival_s: float
    admitted_s: Optional[float] = None
    finished_s: Optional[float] = None
    slot: Optional[int] = None
    increments: int = 0
    n_increments: int = 0
    state: str = "queued"
    newton: int = 0
    krylov: int = 0
    gauss_points: int = 0
    assemblies: int = 0
    max_damage: float = 0.0
    retries: int = 0
    cutbacks: int = 0
    increment_latency_ms: List[float] = dataclasses.field(default_factory=list)


class ServingLoop:
    def __init__(self, requests, precision=binding.MIXED, max_slots=64, hbm_budget_bytes=0,
                 opts: Optional[binding.SolverOpts] = None, keep_results=False):
        self.requests = sorted(requests, key=lambda r: r.arrival_s)
        self.batch = binding.Batch(device=0, precision=precision, max_slots=max_slots,
                                   hbm_budget_bytes=hbm_budget_bytes)
        # the stream's brittle plates take the Newton line search: it
        # converges load steps that full steps do not
        self.opts = opts or binding.solver_opts(max_newton=40, tol_newton=1e-8, tol_krylov=1e-3,
                                                max_krylov=20000, check_every=32,
                                                line_search=binding.LINE_SEARCH_ON)
        self.records: Dict[int, RequestRecord] = {}
        self.keep_results = keep_results
        self.results: Dict[int, dict] = {}
        self.ticks = 0
        self.gp_assembled = 0
        self.t_assembly_ms = 0.0

    def run(self, time_limit_s: Optional[float] = None, realtime: bool = True, log=None):
        """Serve the stream.  realtime: arrivals follow the wall clock (an idle
        device sleeps until the next arrival); otherwise arrival times are
        ignored and requests queue in arrival order from the start."""
        pending = collections.deque(self.requests)
        queue = collections.deque()
        running: Dict[int, int] = {}          # slot -> rid
        inc_start: Dict[int, float] = {}      # slot -> start of its current increment
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        next_report = 30.0
        while pending or queue or running:
            t = now()
            if time_limit_s is not None and t > time_limit_s:
                break
            while pending and (not realtime or pending[0].arrival_s <= t):
                r = pending.popleft()
                self.records[r.rid] = RequestRecord(r.rid, r.arrival_s,
                                                    n_increments=r.problem.n_increments)
                queue.append(r)
            # FIFO admission while a slot and budget are free
            while queue:
                slot = self.batch.admit(queue[0].problem)
                if slot is None:
                    break
                r = queue.popleft()
                rec = self.records[r.rid]
                rec.admitted_s, rec.slot, rec.state = now(), slot, "running"
                running[slot] = r.rid
                inc_start[slot] = None
            if not running:
                if pending and realtime:
                    time.sleep(max(0.0, min(pending[0].arrival_s - now(), 0.05)))
                continue
            t_tick0 = now()
            for slot in running:
                if inc_start[slot] is None:
                    inc_start[slot] = t_tick0
            rep = self.batch.tick(self.opts)
            t_tick1 = now()
            self.ticks += 1
            if log and t_tick1 >= next_report:
                # a progress line every 30 s of serving (long runs)
                done = sum(1 for r in self.records.values() if r.state != "running" and r.state != "queued")
                log("serving t=%.0fs: %d ticks, %d running, %d retired, %d queued, %d increments committed"
                    % (t_tick1, self.ticks, len(running), done, len(queue) + len(pending),
                       sum(r.increments for r in self.records.values())))
                next_report = t_tick1 + 30.0
            self.gp_assembled += rep["gauss_points"]
            self.t_assembly_ms += rep["t_assembly_ms"]
            for slot, rid in list(running.items()):
                info = self.batch.info(slot)
                rec = self.records[rid]
                if info["increment"] > rec.increments:
                    # one increment committed in this tick
                    rec.increment_latency_ms.append((t_tick1 - inc_start[slot]) * 1e3)
                    rec.increments = info["increment"]
                    inc_start[slot] = None
                rec.newton, rec.krylov = info["newton_total"], info["krylov_total"]
                rec.assemblies = info["assemblies_total"]
                rec.gauss_points = info["n_gauss"]
                rec.max_damage = info["max_damage"]
                rec.retries = info["retries"]
                rec.cutbacks = info["cutbacks"]
                if info["state"] in (binding.SLOT_FINISHED, binding.SLOT_FAILED):
                    rec.state = "finished" if info["state"] == binding.SLOT_FINISHED else \
                        "failed(%s)" % binding.STATUS_NAMES.get(info["last_status"])
                    rec.finished_s = now()
                    if self.keep_results:
                        self.results[rid] = {
                            "x": self.batch.query(slot, binding.FIELD_X, info["ndof"]),
                            "D": self.batch.query(slot, binding.FIELD_DAMAGE, info["n_gauss"]),
                        }
                    self.batch.retire(slot)
                    del running[slot]
                    del inc_start[slot]
                    if log:
                        log("request %d %s after %d increments (%d Newton, %d Krylov)"
                            % (rid, rec.state, rec.increments, rec.newton, rec.krylov))
        self.wall_s = now()
        return self.summary()

    def summary(self):
        lat = [v for r in self.records.values() for v in r.increment_latency_ms]
        done = [r for r in self.records.values() if r.state == "finished"]
        failed = [r for r in self.records.values() if r.state.startswith("failed")]
        waits = [r.admitted_s - r.arrival_s for r in self.records.values() if r.admitted_s is not None]
        # whole requests: arrival to the commit of the last increment, and
        # admission to that commit (service time)
        compl = [r.finished_s - r.arrival_s for r in done]
        serv = [r.finished_s - r.admitted_s for r in done]
        pct = lambda v, q: float(np.percentile(v, q)) if v else None
        return {
            "requests_arrived": len(self.records),
            "requests_finished": len(done),
            "requests_failed": len(failed),
            "failed_requests": sorted((r.rid, r.state, r.increments) for r in failed),
            "increment_retries": sum(r.retries for r in self.records.values()),
            "load_step_cutbacks": sum(r.cutbacks for r in self.records.values()),
            "request_latency_p50_s": pct(compl, 50),
            "request_latency_p99_s": pct(compl, 99),
            "request_latency_max_s": float(max(compl)) if compl else None,
            "request_service_p50_s": pct(serv, 50),
            "request_service_p99_s": pct(serv, 99),
            "requests_per_s": len(done) / self.wall_s if self.wall_s > 0 else None,
            "finished_gauss_point_increments_per_s": (
                sum(r.gauss_points * r.increments for r in done) / self.wall_s if self.wall_s > 0 else None),
            "increments_committed": len(lat),
            "latency_p50_ms": float(np.percentile(lat, 50)) if lat else None,
            "latency_p99_ms": float(np.percentile(lat, 99)) if lat else None,
            "gauss_points_per_s": self.gp_assembled / self.wall_s if self.wall_s > 0 else None,
            "assembled_gp_per_s_device": (self.gp_assembled / (self.t_assembly_ms * 1e-3)
                                          if self.t_assembly_ms > 0 else None),
            "ticks": self.ticks,
            "wall_s": self.wall_s,
            "admission_wait_p50_s": float(np.percentile(waits, 50)) if waits else None,
            "admission_wait_max_s": float(max(waits)) if waits else None,
        }

    def close(self):
        self.batch.close()
