#!/usr/bin/env python
"""Benchmark of the LGDM hot path on one MI355X.

A step is one load increment of Algorithm 2 along the load path of the
workload: Newton iterations (compute and assemble K and F with the
Gauss-point and node-row assembly kernels, the per-field residual test, the
linear solve with block-Jacobi-preconditioned IDR(s) or BiCGSTAB, the update
of the primary fields) until ||R||/||F|| < 1e-8 per field, then the commit of
the history variable (Eq. A.2).  Inputs are resident in HBM before timing
starts.

Metric: Gauss points assembled per second of wall time over the timed
increments (whole job, solves included) and the Newton-step ms, in the
FP32-mixed precision the workload names, with the plain FP64 path run
beside it on the same GPU.  Kernel rates (assembly Gauss points per second
of assembly-kernel time, SpMV and assembly GB/s against the HBM roofline)
are measured with HIP events on the library's stream.

Prints one JSON line.
"""
import argparse
import dataclasses
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "assembled Gauss pts/s + Newton-step ms, FP32-mixed vs FP64, ||R||/||F||<1e-8"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "c3": "3D notched beam, three-point bending, 256x64x32 hex8 (524,288 elements, 4,194,304 "
          "Gauss points, 2,205,060 dofs), notch E x 0.01, 150 increments to 0.5 mm",
    "c2": "3D notched beam, three-point bending, 128x32x16 hex8 (65,536 elements, 524,288 Gauss "
          "points, 289,476 dofs), notch E x 0.01, 150 increments to 0.5 mm",
    "c1": "2D plane-stress single-edge-notched plate 200x100 Q4 (80,000 Gauss points, 60,903 "
          "dofs), 200 increments to 0.1 mm",
    "c0": "1D bar, 100 line2 elements, 100 increments to 0.02 mm",
    "c3p": "3D notched beam, three-point bending, 64x16x8 hex8 (8,192 elements, 65,536 Gauss points, "
           "39,780 dofs), notch E x 0.01, 150 increments to 0.5 mm",
    "c0q": "1D bar, 100 quadratic-u / linear-ebar elements (line3, 3 Gauss points), 100 increments to 0.02 mm",
    "c1q": "2D plane-stress single-edge-notched plate 200x100 biquadratic-u / bilinear-ebar elements (quad9, "
           "180,000 Gauss points, 80,601 nodes, 241,803 dofs of which 161,202 u and 20,301 ebar), "
           "200 increments to 0.1 mm",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class PathRunner:
    """Drives the load path through the C ABI, one converged increment per
    step: Newton iterations (assembly, residual test, linear solve, update)
    until ||R||/||F|| < tol per field, then the history commit."""

    def __init__(self, ctx, prob, opts, binding):
        self.ctx, self.prob, self.opts, self.b = ctx, prob, opts, binding
        self.inc = 0                  # committed increments
        self.verbose = True

    def step(self, acc):
        lam = (self.inc + 1) / self.prob.n_increments
        t_inc = time.perf_counter()
        self.ctx.begin_increment(lam)
        rep = self.b.IncrementReport()
        it = 0
        while True:
            before = (rep.t_assembly_ms, rep.t_solve_ms, rep.t_update_ms, rep.n_assemblies,
                      rep.krylov_iters, rep.krylov_spmv)
            t_it = time.perf_counter()
            conv, r = self.ctx.newton_iteration(self.opts, rep)
            if not conv:
                acc["step_ms"].append((time.perf_counter() - t_it) * 1e3)
            if self.verbose:
                log(newton_line(self.inc + 1, it, r, before))
            acc["t_asm"] += r.t_assembly_ms - before[0]
            acc["t_sol"] += r.t_solve_ms - before[1]
            acc["t_upd"] += r.t_update_ms - before[2]
            acc["n_asm"] += r.n_assemblies - before[3]
            acc["krylov"] += r.krylov_iters - before[4]
            acc["spmv"] += r.krylov_spmv - before[5]
            if conv:
                self.ctx.commit_increment()
                self.inc += 1
                acc["increments"] += 1
                acc["per_increment"].append([self.inc, round((time.perf_counter() - t_inc) * 1e3, 1), it,
                                             r.krylov_iters, r.reaction])
                acc["last_rel_u"] = r.res_u / max(r.ref_u, 1e-300)
                acc["last_rel_e"] = r.res_e / max(r.ref_e, 1e-300)
                acc["zone_ms"] += r.t_zone_ms
                acc["zone_factorizations"] += r.zone_factorizations
                acc["zone_restarts"] += r.zone_restarts
                acc["backtracks"] += r.backtracks
                return
            it += 1
            acc["newton"] += 1
            if it > self.opts.max_newton:
                raise RuntimeError("Newton did not converge in increment %d" % (self.inc + 1))


def newton_line(inc, it, r, before):
    """One log line per Newton iteration: residuals of the assembly, then the
    linear solve that followed it (steps, reached relative residual, status)."""
    return ("  inc %d it %d |R_u|/|F_u|=%.3e |R_e|/|F_e|=%.3e krylov=%d spmv=%d rel=(%.1e, %.1e) "
            "status=%d inexact=%d restarts=%d backtracks=%d zone<=%d asm=%.3fms solve=%.1fms "
            "(so far: zone setup %.1fms, %d factorizations, %d restarts)" % (
                inc, it, r.res_u / max(r.ref_u, 1e-300), r.res_e / max(r.ref_e, 1e-300),
                r.krylov_iters - before[4], r.krylov_spmv - before[5], r.krylov_rel_u, r.krylov_rel_e,
                r.krylov_status, r.inexact_solves, r.restarts, r.backtracks, r.zone_dofs,
                r.t_assembly_ms - before[0], r.t_solve_ms - before[1], r.t_zone_ms, r.zone_factorizations,
                r.zone_restarts))


def zone_opts(args, binding):
    """Process-zone and line-search options of the Newton solves."""
    return dict(process_zone={"default": binding.ZONE_DEFAULT, "off": binding.ZONE_OFF,
                              "every": binding.ZONE_EVERY_TANGENT}[args.zone],
                zone_damage=args.zone_damage,
                line_search=binding.LINE_SEARCH_ON if args.line_search else binding.LINE_SEARCH_OFF)


def new_acc():
    return dict(t_asm=0.0, t_sol=0.0, t_upd=0.0, n_asm=0, krylov=0, spmv=0, newton=0, increments=0,
                last_rel_u=None, last_rel_e=None, step_ms=[], per_increment=[], zone_ms=0.0,
                zone_factorizations=0, zone_restarts=0, backtracks=0)


def window_phases(per_inc):
    """Split the timed increments by load-path phase, judged from the
    reactions the run has seen so far (the peak is the largest |reaction|
    up to the last timed increment): before the peak, within 2% of it, and
    after it.  Per phase: increments, ms per increment, Newton iterations per
    increment and Krylov steps per Newton iteration (medians)."""
    if not per_inc:
        return None
    rmax = max(abs(v[4]) for v in per_inc)
    ipk = max(range(len(per_inc)), key=lambda j: abs(per_inc[j][4]))
    groups = {"pre_peak": [], "near_peak": [], "post_peak": []}
    for j, v in enumerate(per_inc):
        if abs(abs(v[4]) - rmax) <= 0.02 * rmax:
            groups["near_peak"].append(v)
        elif j > ipk:
            groups["post_peak"].append(v)
        else:
            groups["pre_peak"].append(v)
    out = {}
    for k, vs in groups.items():
        if vs:
            out[k] = {"increments": [vs[0][0], vs[-1][0]], "count": len(vs),
                      "ms_per_increment_median": statistics.median(v[1] for v in vs),
                      "newton_per_increment_median": statistics.median(v[2] for v in vs),
                      "krylov_per_newton_median": statistics.median(v[3] / max(v[2], 1) for v in vs)}
    return out


def algorithmic_bytes(prob, nnz, npairs, s_val):
    """Per launch: assembly (reads x, coords, conn, kappa_n, E-scale; writes
    CSR values and R) and SpMV (values, node-graph columns, the row offset of
    each node and the node-graph offsets, FP64 x and y)."""
    ndof, nn, ne, ng = prob.ndof, prob.n_nodes, prob.n_elems, prob.n_elems * prob.ngp
    asm = (ndof * 8 + nn * prob.dim * 8 + ne * prob.nen * 4 + ng * 8 + ne * 8
           + nnz * s_val + ndof * 8)
    spmv = nnz * s_val + npairs * 4 + nn * 4 + (nn + 1) * 4 + ndof * 8 * 2
    return asm, spmv


def assembly_spmv_roofline(res):
    """Assembly and SpMV together over the timed steps: the algorithmic bytes
    of every assembly and every SpMV launch over their kernel time (assembly:
    back-to-back launch time; SpMV: the live probe), against the HBM peak."""
    pr, kt = res["probe"], res["kernel_ms"]
    if not pr.get("gbs") or res["spmv_launches"] <= 0:
        return None
    nb_tot = res["assemblies"] * res["assembly_bytes"] + res["spmv_launches"] * pr["algorithmic_bytes"]
    ms_tot = (res["assemblies"] * (kt["gauss_point"] + kt["node_assembly"]) +
              res["spmv_launches"] * pr["avg_ms"])
    gbs = nb_tot / (ms_tot * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": "assembly + IDR SpMV", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes": nb_tot, "kernel_ms": round(ms_tot, 1)}


def committed_traffic(kernel_key, launches_bytes):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE counters (scaled by the same counters
    of a plain copy of known size), or None when the kernel's source changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(kernel_key)
    if not rec:
        return None
    src = os.path.join(ROOT, rec["source"])
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if sha != rec["source_sha256"]:
        return None
    return rec["hbm_bytes_per_launch"]


def run_precision(prob, precision, args, binding):
    import torch
    ctx = binding.Context(device=0, precision=precision)
    t0 = time.time()
    ctx.setup_problem(prob)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    log("setup %.2fs precision=%s ndof=%d nGP=%d" % (setup_s, precision, ctx.ndof, ctx.ngauss))
    opts = binding.solver_opts(max_newton=args.max_newton, tol_newton=1e-8, tol_krylov=args.tol_krylov,
                               max_krylov=args.max_krylov, check_every=32,
                               krylov_method=binding.KRYLOV_BICGSTAB if args.krylov == "bicgstab"
                               else binding.KRYLOV_IDRS, idr_s=args.idr_s,
                               forcing=binding.FORCING_FIXED if args.fixed_forcing else binding.FORCING_ADAPTIVE,
                               precond={"default": binding.PRECOND_DEFAULT, "bj": binding.PRECOND_BLOCK_JACOBI,
                                        "amg": binding.PRECOND_AMG}[args.precond],
                               **zone_opts(args, binding))
    runner = PathRunner(ctx, prob, opts, binding)
    warm = new_acc()
    for i in range(args.warmup):
        runner.step(warm)
        log("warmup step %d done (increment %d, spmv %d)" % (i + 1, runner.inc, warm["spmv"]))
    acc = new_acc()
    # live timing of the dominant solver kernel over the timed steps: the
    # IDR SpMV (the only pass over the matrix per Krylov step, with either
    # preconditioner)
    ctx.probe_start(binding.PROBE_IDR_SPMV)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        runner.step(acc)
        log("step %d done (increment %d, Newton so far %d, spmv so far %d)"
            % (i + 1, runner.inc, acc["newton"], acc["spmv"]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    probe_ms, probe_n = ctx.probe_stop()
    amg_levels = ctx.amg_levels()
    view, _ = ctx.assemble(-1.0, want_R=False)
    kt = ctx.kernel_times(args.kernel_reps)
    nnz = view.nnz
    npairs = nnz // (prob.ndpn ** 2)
    s_val = 4 if precision == binding.MIXED else 8
    asm_b, spmv_b = algorithmic_bytes(prob, nnz, npairs, s_val)
    probe_b = spmv_b
    probe_name = "spmv_kernel<%s, %d, 16, 3, 8> (IDR SpMV)" % (
        "float" if precision == binding.MIXED else "double", prob.ndpn)
    ng = ctx.ngauss
    res = {
        "gp_per_s": ng * acc["n_asm"] / wall,
        "ms_per_increment": wall * 1e3 / args.steps,
        "newton_step_ms": wall * 1e3 / max(acc["newton"], 1),
        "newton_step_ms_median": statistics.median(acc["step_ms"]) if acc["step_ms"] else None,
        "newton_step_ms_min": min(acc["step_ms"]) if acc["step_ms"] else None,
        "newton_step_ms_each": [round(v, 2) for v in acc["step_ms"]],
        "newton_iterations": acc["newton"], "assemblies": acc["n_asm"],
        "increments_in_timed_region": acc["increments"], "increments_committed": runner.inc,
        "assembly_gp_per_s_device": ng * acc["n_asm"] / (acc["t_asm"] / 1e3) if acc["t_asm"] > 0 else None,
        "phase_ms_per_increment": {"assembly": acc["t_asm"] / args.steps, "solve": acc["t_sol"] / args.steps,
                                   "update": acc["t_upd"] / args.steps,
                                   "zone_setup_within_solve": acc["zone_ms"] / args.steps},
        "process_zone": {"factorizations": acc["zone_factorizations"],
                         "increment_restarts": acc["zone_restarts"],
                         "line_search_halvings": acc["backtracks"]},
        "krylov_iters": acc["krylov"], "spmv_launches": acc["spmv"],
        "spmv_per_newton_step": acc["spmv"] / max(acc["newton"], 1),
        "final_rel_residual": [acc["last_rel_u"], acc["last_rel_e"]],
        "per_increment": {"columns": ["increment", "ms", "newton", "krylov", "reaction"],
                          "rows": acc["per_increment"]},
        "window_phases": window_phases(acc["per_increment"]),
        "kernel_ms": {"gauss_point": kt[0], "node_assembly": kt[1], "spmv": kt[2], "block_jacobi": kt[3]},
        "assembly_bytes": asm_b, "spmv_bytes": spmv_b,
        "assembly_gbs": asm_b / ((kt[0] + kt[1]) * 1e-3) / 1e9,
        "spmv_gbs": spmv_b / (kt[2] * 1e-3) / 1e9,
        "probe": {"kernel": probe_name, "key": "spmv", "avg_ms": probe_ms,
                  "launches_timed": probe_n, "algorithmic_bytes": probe_b,
                  "gbs": probe_b / (probe_ms * 1e-3) / 1e9 if probe_ms > 0 else None,
                  "note": "HIP events around each launch on the context's stream during the timed steps"},
        "multigrid_levels": amg_levels,
        "footprint_gb": ctx.footprint() / 1e9,
        "setup_ms": setup_s * 1e3,   # mesh upload, CSR pattern build (once per mesh), material, Dirichlet set
        "solver": {"krylov": args.krylov, "idr_s": args.idr_s if args.krylov == "idr" else None,
                   "forcing": "fixed" if args.fixed_forcing else "adaptive", "tol_krylov": args.tol_krylov,
                   "precond": args.precond, "process_zone": args.zone, "zone_damage": args.zone_damage,
                   "line_search": args.line_search},
    }
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    return res


def load_path_run(prob, precision, args, binding, n_inc):
    """Whole load path: increments 1..n_inc, each solved to the Newton test
    through the stepwise C ABI (one log line per Newton iteration) and timed
    on the host.  Each
    increment's reaction force and maximum damage classify it as elastic (no
    damage yet), near the peak (reaction within 2% of the path maximum) or
    post-peak (after the maximum), the three phases the step time is
    reported for."""
    import statistics
    import torch
    ctx = binding.Context(device=0, precision=precision)
    ctx.setup_problem(prob)
    torch.cuda.synchronize()
    opts = binding.solver_opts(max_newton=args.max_newton, tol_newton=1e-8, tol_krylov=args.tol_krylov,
                               max_krylov=args.max_krylov, check_every=32, krylov_method=binding.KRYLOV_IDRS,
                               idr_s=args.idr_s, forcing=binding.FORCING_ADAPTIVE,
                               precond={"default": binding.PRECOND_DEFAULT, "bj": binding.PRECOND_BLOCK_JACOBI,
                                        "amg": binding.PRECOND_AMG}[args.precond],
                               max_increment_krylov=args.max_increment_krylov,
                               max_increment_seconds=args.max_increment_seconds, **zone_opts(args, binding))
    incs = []
    stop = None
    keys = ("newton_iters", "n_assemblies", "krylov_iters", "t_assembly_ms", "t_solve_ms")
    label = "mixed" if precision == binding.MIXED else "fp64"

    def solve_step(lam, inc):
        """One load step through the stepwise C ABI (the same sequence as
        lgdm_solve_increment, with the same work bounds in the options),
        printing one line per Newton iteration."""
        rep = binding.IncrementReport()
        ctx.begin_increment(lam)
        it = 0
        status = 0
        while True:
            before = (rep.t_assembly_ms, rep.t_solve_ms, rep.t_update_ms, rep.n_assemblies,
                      rep.krylov_iters, rep.krylov_spmv)
            try:
                conv, r = ctx.newton_iteration(opts, rep)
            except binding.LgdmError as e:
                status = e.status
                log("  %s inc %d it %d: %s" % (label, inc, it, e))
                break
            log(label + newton_line(inc, it, r, before))
            if conv:
                break
            it += 1
            if it > opts.max_newton:
                status = binding.LGDM_ERR_NOT_CONVERGED
                log("  %s inc %d: no convergence within %d Newton iterations" % (label, inc, opts.max_newton))
                break
        d = rep.as_dict()
        if status == 0:
            ctx.commit_increment()
            d["max_damage"] = float(ctx.query(binding.FIELD_DAMAGE).max())
            d["converged"] = 1
        else:
            ctx.abort_increment()
        d["status"] = status
        return d

    def advance(lam0, lam1, depth, inc):
        """Solve the load step lam0 -> lam1; a step that fails (the state is
        restored) is split into two halves, at most `cutback` times.
        Returns (status, summed report, sub-steps)."""
        d = solve_step(lam1, inc)
        if d["status"] == 0 or depth >= args.cutback:
            return d["status"], d, 1
        mid = 0.5 * (lam0 + lam1)
        log("  %s inc %d: load step split (depth %d)" % (label, inc, depth + 1))
        st1, d1, n1 = advance(lam0, mid, depth + 1, inc)
        if st1 != 0:
            return st1, d1, n1
        st2, d2, n2 = advance(mid, lam1, depth + 1, inc)
        for k in keys:
            d2[k] = d2[k] + d1[k]
        return st2, d2, n1 + n2

    for i in range(n_inc):
        t0 = time.perf_counter()
        status, d, nsub = advance(i / prob.n_increments, (i + 1) / prob.n_increments, 0, i + 1)
        dt = time.perf_counter() - t0
        if status != 0:
            stop = {"increment": i + 1, "status": status, "cutbacks": args.cutback,
                    "error": ctx.lib.lgdm_last_error(ctx.h).decode()}
            log("load path stops at increment %d: %s" % (i + 1, stop["error"]))
            break
        if (i + 1) in args.dump_state:
            # the committed state, for re-solving a later increment elsewhere
            import numpy as np
            os.makedirs(os.path.join(ROOT, "gpurun_out"), exist_ok=True)
            path = os.path.join(ROOT, "gpurun_out", "state_%s_%s_%04d.npz" % (args.config, label, i + 1))
            np.savez_compressed(path, x=ctx.query(binding.FIELD_X), kappa=ctx.query(binding.FIELD_KAPPA),
                                increment=i + 1, n_increments=prob.n_increments)
            log("saved the committed state of increment %d to %s" % (i + 1, path))
        incs.append({"inc": i + 1, "ms": dt * 1e3, "newton": d["newton_iters"], "assemblies": d["n_assemblies"],
                     "krylov": d["krylov_iters"], "t_asm": d["t_assembly_ms"], "t_sol": d["t_solve_ms"],
                     "reaction": d["reaction"], "max_damage": d["max_damage"], "substeps": nsub})
        log("load path %s: increment %d, %.1f ms, %d Newton, %d Krylov, reaction %.4e, max D %.4f, "
            "%d sub-steps" % (label, i + 1, dt * 1e3, d["newton_iters"], d["krylov_iters"], d["reaction"],
                              d["max_damage"], nsub))
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    ng = prob.n_elems * prob.ngp
    rmax = max(abs(r["reaction"]) for r in incs) if incs else 0.0
    ipk = max(range(len(incs)), key=lambda j: abs(incs[j]["reaction"])) if incs else 0
    phases = {"elastic": [], "near_peak": [], "post_peak": [], "pre_peak_damaged": []}
    for j, r in enumerate(incs):
        if r["max_damage"] <= 0.0:
            phases["elastic"].append(r)
        elif abs(abs(r["reaction"]) - rmax) <= 0.02 * rmax:
            phases["near_peak"].append(r)
        elif j > ipk:
            phases["post_peak"].append(r)
        else:
            phases["pre_peak_damaged"].append(r)

    def summ(rs):
        if not rs:
            return None
        steps = [r["ms"] / max(r["newton"], 1) for r in rs]
        asm = [r["t_asm"] / max(r["assemblies"], 1) for r in rs]
        return {"increments": [rs[0]["inc"], rs[-1]["inc"]], "count": len(rs),
                "newton_step_ms_median": statistics.median(steps), "newton_step_ms_min": min(steps),
                "ms_per_increment_median": statistics.median(r["ms"] for r in rs),
                "newton_per_increment_median": statistics.median(r["newton"] for r in rs),
                "krylov_per_newton_median": statistics.median(r["krylov"] / max(r["newton"], 1) for r in rs),
                "assembly_gp_per_s_device_median": ng / (statistics.median(asm) * 1e-3),
                "gp_per_s": ng * sum(r["assemblies"] for r in rs) / (sum(r["ms"] for r in rs) * 1e-3)}
    return {"increments_run": len(incs), "stopped": stop, "peak_increment": incs[ipk]["inc"] if incs else None,
            "peak_reaction": incs[ipk]["reaction"] if incs else None,
            "whole_path": summ(incs), "phases": {k: summ(v) for k, v in phases.items()},
            "per_increment": [[r["inc"], round(r["ms"], 2), r["newton"], r["krylov"], r["reaction"],
                               round(r["max_damage"], 6), r["substeps"]] for r in incs]}


def cpu_baseline(name, prob, budget_s=20.0):
    """The oracle on the host with BLAS on every host core (its dense
    element contractions run there; the sparse LU is single threaded):
    whole Newton iterations (element evaluation, triplet assembly, Dirichlet
    rows, sparse LU solve, update) of the first load increment, scaled to
    Gauss points per second of wall time like the GPU value.  The 3D beams
    are sampled at 64x16x8 (a sparse LU of the full mesh does not fit a
    bounded run); the element evaluation + assembly rate on a slab of the
    full mesh is reported beside it."""
    import numpy as np
    import scipy.sparse.linalg as spla
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle.lgdm import Oracle, eval_elements, assemble
    from oracle.mixed_order import MixedOracle, eval_elements_mixed
    import lgdm_workloads as W
    sample_name = "c3p" if name in ("c2", "c3") else name
    sample = W.config(sample_name)
    mixed_order = prob.elem_type in W.MIXED_ORDER
    host_cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    with threadpool_limits(limits=host_cores, user_api="blas"):
        blas_threads = max([p.get("num_threads", 1) for p in threadpool_info() if p.get("user_api") == "blas"]
                           or [1])
        o = MixedOracle(sample) if mixed_order else Oracle(sample)
        o.x[o.bc_dofs] = (1.0 / sample.n_increments) * o.bc_vals
        its = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s * 0.75:
            st = o.eval_state()
            o.x = o.x + spla.splu(st["K"].tocsc()).solve(st["R"])
            its += 1
        dt = time.perf_counter() - t0
        whole = its * sample.n_elems * sample.ngp / dt
        # element evaluation + triplet assembly on a slab of the full mesh
        x, kn = W.injected_state(prob, seed=0, noise=0.02, kappa_spread=1.5)
        mat = prob.material.as_dict()
        n_el = min(prob.n_elems, 2048)
        done_el = 0
        t1 = time.perf_counter()
        if mixed_order:
            mo = MixedOracle(prob)
            xo = mo.from_interleaved(x)
            u_nodal = xo[:prob.n_nodes * prob.dim].reshape(-1, prob.dim)
            ebar_v = xo[prob.n_nodes * prob.dim:]
        while True:
            sl = np.arange(done_el, done_el + n_el) % prob.n_elems
            if mixed_order:
                # element evaluation + triplet assembly (sum of duplicates) of the slab
                import scipy.sparse as sps
                ev = eval_elements_mixed(prob.dim, prob.coords, prob.conn[sl], prob.e_scale[sl], mat, u_nodal,
                                         ebar_v, mo.vidx, kn.reshape(prob.n_elems, -1)[sl])
                ed = mo.edofs[sl]
                nl = ed.shape[1]
                sps.coo_matrix((ev["Ke"].ravel(), (np.repeat(ed, nl, axis=1).ravel(), np.tile(ed, (1, nl)).ravel())),
                               shape=(mo.ndof, mo.ndof)).tocsr()
            else:
                ev = eval_elements(prob.dim, prob.coords, prob.conn, prob.e_scale, mat, x, kn, elems=sl)
                assemble(prob.dim, prob.conn[sl], prob.n_nodes, ev["fint"], ev["Ke"])
            done_el += n_el
            if time.perf_counter() - t1 > budget_s * 0.25 or done_el >= prob.n_elems:
                break
        dt_asm = time.perf_counter() - t1
    return {"value": whole, "unit": "GP/s", "cores": blas_threads, "kind": "oracle",
            "sample": "%d Newton iterations (assembly + sparse LU + update) of the oracle on %s (%d Gauss "
                      "points, %d dofs) in %.1f s; BLAS on %d threads (the SuperLU factorisation is single "
                      "threaded); %d cores in the affinity mask" % (
                          its, sample_name, sample.n_elems * sample.ngp, sample.ndof, dt, blas_threads,
                          host_cores),
            "assembly_only_gp_per_s": done_el * prob.ngp / dt_asm,
            "assembly_only_sample": "element evaluation + triplet assembly of %d of %d elements of %s (%.1f s)"
                                    % (done_el, prob.n_elems, name, dt_asm)}


def copy_calibration(nbytes=1 << 30):
    """A plain elementwise copy of known size (reads and writes nbytes), so
    that hardware byte counters of the same run can be scaled to bytes."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.mul(a, 1.0, out=b)                       # warm-up (module load)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(5):
        torch.mul(a, 1.0, out=b)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / 5
    del a, b
    return {"kernel": "torch.mul(a, 1.0, out=b) float32", "bytes_read": nbytes, "bytes_written": nbytes,
            "ms": ms, "gbs": 2 * nbytes / (ms * 1e-3) / 1e9}


def serving_leg(seconds, n_requests, increments):
    """The continuous-batching workload: seeded 2D notched-plate requests
    (40x20 .. 400x200 Q4, 50-200 increments) with Poisson arrivals at 20/s,
    mixed precision, 64 slots, served until every request is retired or the
    wall time runs out.  increments > 0 keeps only the first increments of
    each request's load path (the same load steps), so that whole requests
    finish within the bench; 0 runs every load path to its end."""
    import lgdm_workloads as W
    from paper_2301_06503_amd import binding, serving
    reqs = W.serving_stream(n_requests=n_requests, rate_per_s=20.0, seed=0,
                            first_increments=increments if increments > 0 else None)
    loop = serving.ServingLoop(reqs, precision=binding.MIXED, max_slots=64)
    summ = loop.run(time_limit_s=seconds, realtime=True, log=log)
    loop.close()
    summ["workload"] = ("%d requests, Poisson arrivals 20/s, 2D notched plates 40x20..400x200 Q4 with 50-200 "
                        "increments, %s, mixed precision, 64 slots; served for at most %.0f s" % (
                            n_requests, "the first %d increments of each load path" % increments
                            if increments > 0 else "whole load paths", seconds))
    return summ


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tol-krylov", type=float, default=3e-4,
                    help="relative tolerance of the Newton corrections far from convergence (the last "
                         "ones solve only as far as the Newton test needs); 3e-4 converges the 128x32x16 "
                         "beam's whole load path, where 1e-3 stops in the softening branch")
    ap.add_argument("--krylov", default="idr", choices=["idr", "bicgstab"])
    ap.add_argument("--idr-s", type=int, default=8)
    ap.add_argument("--precond", default="default", choices=["default", "bj", "amg"],
                    help="block-Jacobi or aggregation multigrid (IDR only); the default is multigrid on 3D meshes")
    ap.add_argument("--zone", default="default", choices=["default", "off", "every"],
                    help="exact process-zone solve in the multigrid preconditioner: default (factors kept while "
                         "the zone's nodes stay the same within an increment), off, or every (rebuilt for every "
                         "tangent)")
    ap.add_argument("--zone-damage", type=float, default=0.99,
                    help="trial damage from which a loading element joins the process zone")
    ap.add_argument("--line-search", action="store_true",
                    help="Newton line search: halve a correction that blows the residual up (default: full steps)")
    ap.add_argument("--fixed-forcing", action="store_true",
                    help="solve every Newton correction to --tol-krylov (default: adaptive forcing)")
    ap.add_argument("--max-krylov", type=int, default=20000)
    ap.add_argument("--max-newton", type=int, default=40)
    ap.add_argument("--kernel-reps", type=int, default=5)
    ap.add_argument("--serving-seconds", type=float, default=45.0,
                    help="wall-time bound of the serving leg (0: no serving leg)")
    ap.add_argument("--serving-requests", type=int, default=128)
    ap.add_argument("--serving-increments", type=int, default=12,
                    help="increments served per request (the first ones of its load path; 0: all)")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving leg and print its report as the JSON line")
    ap.add_argument("--coupling", type=int, default=0, choices=[0, 1],
                    help="1: the stress of Eq. 2 with its h term and the consistent tangent (material coupling "
                         "variant); 0: the executed-code form (default)")
    ap.add_argument("--max-increment-krylov", type=int, default=0,
                    help="load-path mode: Krylov iterations one load step may spend before it fails (0: no bound)")
    ap.add_argument("--max-increment-seconds", type=float, default=300.0,
                    help="load-path mode: wall time one load step may spend before it fails (0: no bound)")
    ap.add_argument("--cutback", type=int, default=0,
                    help="load-path mode: split a load step that fails into halves, at most this many times")
    ap.add_argument("--dump-state", type=str, default="",
                    help="load-path mode: comma-separated increments whose committed state (x, kappa_n) is "
                         "saved to gpurun_out/state_<config>_<precision>_<increment>.npz")
    ap.add_argument("--load-path", type=int, default=0,
                    help="instead of the bench line: run this many increments of the load path (-1: all) in "
                         "mixed precision and FP64 and report the step time per phase (elastic, near the "
                         "peak, post-peak)")
    args = ap.parse_args()
    args.dump_state = {int(v) for v in args.dump_state.split(",") if v.strip()}
    if args.gpus != 1:
        print("bench.py runs on one GPU: the LGDM hot path here is built and measured on a single "
              "MI355X; multi-GPU runs are not implemented (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    import lgdm_workloads as W
    from paper_2301_06503_amd import binding
    if args.serving_only:
        print(json.dumps({"metric": "serving", "serving": serving_leg(args.serving_seconds, args.serving_requests,
                                                                      args.serving_increments)}))
        return
    prob = W.config(args.config)
    if args.coupling:
        prob.material = dataclasses.replace(prob.material, coupling=args.coupling)
    prec = binding.MIXED if args.precision == "mixed" else binding.FP64
    if args.load_path:
        n_inc = prob.n_increments if args.load_path < 0 else min(args.load_path, prob.n_increments)
        lp = {"workload": WORKLOADS[args.config], "name": args.config, "increments_requested": n_inc,
              "columns": ["increment", "ms", "newton", "krylov", "reaction", "max_damage", "substeps"],
              "cutback": args.cutback}
        runs = [("mixed", binding.MIXED), ("fp64", binding.FP64)] if prec == binding.MIXED else [("fp64", binding.FP64)]
        for label, pr in runs:
            if label == "fp64" and prec == binding.MIXED and args.no_fp64_compare:
                continue
            lp[label] = load_path_run(prob, pr, args, binding, n_inc)
        print(json.dumps({"metric": METRIC, "load_path": lp}))
        return
    main_res = run_precision(prob, prec, args, binding)
    fp64_res = None
    if prec == binding.MIXED and not args.no_fp64_compare:
        fp64_res = run_precision(prob, binding.FP64, args, binding)
    # dominant kernel of a step: the probed solver kernel (one launch per
    # Krylov step) vs the assembly kernels (one launch each per Newton step)
    kt = main_res["kernel_ms"]
    pr = main_res["probe"]
    solver_share = main_res["krylov_iters"] * pr["avg_ms"]
    asm_share = main_res["assemblies"] * (kt["gauss_point"] + kt["node_assembly"])
    if solver_share >= asm_share and pr["gbs"]:
        achieved, kern, key_kern, nbytes = pr["gbs"], pr["kernel"], pr["key"], pr["algorithmic_bytes"]
    else:
        achieved, kern, key_kern, nbytes = (main_res["assembly_gbs"], "gauss_point+node_assembly", "assembly",
                                            main_res["assembly_bytes"])
    key = "%s_%s_%s" % (args.config, args.precision, key_kern)
    roofline = {"bound": "hbm", "kernel": kern, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": committed_traffic(key, None), "algorithmic_bytes": nbytes,
                "launch_ms": pr["avg_ms"] if key_kern != "assembly" else None}
    roof_asm = {"bound": "hbm", "kernel": "gauss_point+node_assembly",
                "achieved": round(main_res["assembly_gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(main_res["assembly_gbs"] / HBM_PEAK_GBS, 4)}
    roof_asm_spmv = assembly_spmv_roofline(main_res)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.config, prob)
    copy_cal = copy_calibration()
    serving_res = None
    if args.serving_seconds > 0:
        serving_res = serving_leg(args.serving_seconds, args.serving_requests, args.serving_increments)
    out = {
        "metric": METRIC,
        "value": main_res["gp_per_s"],
        "unit": "GP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_increment"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec == binding.MIXED else "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.config], "name": args.config,
                   "precision": args.precision, "ndof": prob.ndof, "gauss_points": prob.n_elems * prob.ngp,
                   "coupling": "eq2" if args.coupling else "executed",
                   "tol_newton": 1e-8, "step": "one load increment: Newton iterations to "
                   "||R||/||F|| < 1e-8 per field, then the history commit",
                   "newton_step_ms": main_res["newton_step_ms"],
                   "fp64_newton_step_ms": fp64_res["newton_step_ms"] if fp64_res else None},
        "roofline": roofline,
        "roofline_assembly": roof_asm,
        "roofline_assembly_spmv": roof_asm_spmv,
        "cpu_baseline": cpu,
        "copy_calibration": copy_cal,
        "serving": serving_res,
        "detail": main_res,
        "fp64": fp64_res,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
