"""Python binding of the LGDM C ABI (include/lgdm.h): argument marshalling only.

Every step of the hot path runs in the HIP library liblgdm.so built in this
directory; if it is missing this module raises ImportError instead of falling
back to anything else.  PyTorch supplies device memory (through the
allocator hook) and the stream.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblgdm.so")

LGDM_OK, LGDM_ERR_INVALID_ARG, LGDM_ERR_OOM, LGDM_ERR_DEVICE = 0, 1, 2, 3
LGDM_ERR_NOT_CONVERGED, LGDM_ERR_NAN, LGDM_ERR_BREAKDOWN, LGDM_ERR_STATE = 4, 5, 6, 7
FP64, MIXED = 0, 1
FIELD_X, FIELD_KAPPA, FIELD_DAMAGE, FIELD_KAPPA_TRIAL, FIELD_DAMAGE_TRIAL = 0, 1, 2, 3, 4
FIELD_RESIDUAL, FIELD_REACTION, FIELD_EEQ = 5, 6, 7
ZONE_DEFAULT, ZONE_OFF, ZONE_EVERY_TANGENT = 0, 1, 2
LINE_SEARCH_OFF, LINE_SEARCH_ON = 0, 1

LGDM_ERR_BUSY = 8
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "OOM", 3: "DEVICE", 4: "NOT_CONVERGED", 5: "NAN",
                6: "BREAKDOWN", 7: "STATE", 8: "BUSY"}
SLOT_FREE, SLOT_RUNNING, SLOT_FINISHED, SLOT_FAILED = 0, 1, 2, 3
KRYLOV_DEFAULT, KRYLOV_BICGSTAB, KRYLOV_IDRS = 0, 1, 2
FORCING_ADAPTIVE, FORCING_FIXED = 0, 1
PRECOND_DEFAULT, PRECOND_BLOCK_JACOBI, PRECOND_AMG = 0, 1, 2
PROBE_IDR_SPMV, PROBE_MG_FINEST = 0, 1

# every entry point the header declares
EXPORTS = [
    "lgdm_create", "lgdm_destroy", "lgdm_last_error", "lgdm_set_allocator", "lgdm_upload_mesh",
    "lgdm_set_material", "lgdm_set_dirichlet", "lgdm_assemble_tangent_residual",
    "lgdm_solve_linear", "lgdm_solve_linear_noalloc", "lgdm_solve_increment", "lgdm_begin_increment",
    "lgdm_newton_iteration", "lgdm_commit_increment", "lgdm_abort_increment", "lgdm_get_csr",
    "lgdm_get_connectivity", "lgdm_get_sizes", "lgdm_query_state", "lgdm_set_state",
    "lgdm_debug_element_blocks", "lgdm_kernel_times", "lgdm_footprint", "lgdm_amg_aggregate",
    "lgdm_amg_levels", "lgdm_probe_start", "lgdm_probe_stop", "lgdm_zone_levels",
    "lgdm_batch_create", "lgdm_batch_destroy", "lgdm_batch_last_error", "lgdm_request_footprint",
    "lgdm_batch_admit", "lgdm_batch_tick", "lgdm_batch_slot_info", "lgdm_batch_query",
    "lgdm_batch_retire", "lgdm_batch_usage", "lgdm_batch_set_allocator",
]


class Material(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("E", "nu", "kappa0", "alpha", "beta", "c", "R", "eta", "k", "h", "tol_hist",
                 "tol_dmg")] + [("plane", ctypes.c_int32), ("coupling", ctypes.c_int32),
                                ("thickness", ctypes.c_double)]


class SolverOpts(ctypes.Structure):
    _fields_ = [("max_newton", ctypes.c_int32), ("max_krylov", ctypes.c_int32),
                ("tol_newton", ctypes.c_double), ("tol_krylov", ctypes.c_double),
                ("check_every", ctypes.c_int32), ("max_restarts", ctypes.c_int32),
                ("krylov_method", ctypes.c_int32), ("idr_s", ctypes.c_int32),
                ("forcing", ctypes.c_int32), ("precond", ctypes.c_int32), ("process_zone", ctypes.c_int32),
                ("max_increment_krylov", ctypes.c_int64), ("max_increment_seconds", ctypes.c_double),
                ("line_search", ctypes.c_int32), ("zone_damage", ctypes.c_double)]


class IncrementReport(ctypes.Structure):
    _fields_ = [("converged", ctypes.c_int32), ("newton_iters", ctypes.c_int32),
                ("krylov_iters", ctypes.c_int64)] + [
        (n, ctypes.c_double) for n in ("res_u", "res_e", "ref_u", "ref_e", "du_norm", "de_norm",
                                       "reaction", "max_damage", "t_assembly_ms", "t_solve_ms",
                                       "t_update_ms")] + [
        ("n_assemblies", ctypes.c_int32), ("restarts", ctypes.c_int32),
        ("krylov_status", ctypes.c_int32), ("inexact_solves", ctypes.c_int32),
        ("krylov_rel_u", ctypes.c_double), ("krylov_rel_e", ctypes.c_double),
        ("krylov_spmv", ctypes.c_int64), ("precond_fallbacks", ctypes.c_int32), ("backtracks", ctypes.c_int32),
        ("zone_dofs", ctypes.c_int64), ("t_zone_ms", ctypes.c_double),
        ("zone_factorizations", ctypes.c_int32), ("zone_restarts", ctypes.c_int32),
        ("zone_errors", ctypes.c_int32)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class CsrView(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("vals", ctypes.c_void_p), ("vals32", ctypes.c_void_p)]


class Request(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("elem_type", ctypes.c_int32), ("n_nodes", ctypes.c_int64),
                ("coords", ctypes.c_void_p), ("n_elems", ctypes.c_int64), ("conn", ctypes.c_void_p),
                ("e_scale", ctypes.c_void_p), ("material", Material), ("n_bc", ctypes.c_int64),
                ("bc_dofs", ctypes.c_void_p), ("bc_values", ctypes.c_void_p),
                ("n_increments", ctypes.c_int64)]


class SlotInfo(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("newton_in_increment", ctypes.c_int32)] + [
        (n, ctypes.c_int64) for n in ("increment", "n_increments", "newton_total", "krylov_total",
                                      "assemblies_total", "n_gauss", "ndof", "footprint_bytes")] + [
        ("max_damage", ctypes.c_double), ("last_status", ctypes.c_int32), ("retries", ctypes.c_int32),
        ("cutbacks", ctypes.c_int64)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class TickReport(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("running", "solves", "committed", "finished")] + [
        ("gauss_points", ctypes.c_int64), ("krylov_iters", ctypes.c_int64),
        ("t_assembly_ms", ctypes.c_double), ("t_tick_ms", ctypes.c_double)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


_lib = None
_hip = None
_ALLOC_T = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_T = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


def load_library(path: str = LIB_PATH):
    """Load liblgdm.so from the package directory (raises ImportError if absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("liblgdm.so is not built (%s); run `python -m paper_2301_06503_amd.build`"
                          % path)
    lib = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "lgdm_create": [ctypes.POINTER(P), I32, P, I32],
        "lgdm_destroy": [P],
        "lgdm_set_allocator": [P, _ALLOC_T, _FREE_T, P],
        "lgdm_upload_mesh": [P, I32, I32, I64, P, I64, P, P],
        "lgdm_set_material": [P, ctypes.POINTER(Material)],
        "lgdm_set_dirichlet": [P, I64, P, P],
        "lgdm_assemble_tangent_residual": [P, D, ctypes.POINTER(CsrView), P],
        "lgdm_solve_linear": [P, P, P, ctypes.POINTER(SolverOpts), ctypes.POINTER(IncrementReport)],
        "lgdm_solve_linear_noalloc": [P, P, P, ctypes.POINTER(SolverOpts), ctypes.POINTER(IncrementReport)],
        "lgdm_solve_increment": [P, D, ctypes.POINTER(SolverOpts), ctypes.POINTER(IncrementReport)],
        "lgdm_begin_increment": [P, D],
        "lgdm_newton_iteration": [P, ctypes.POINTER(SolverOpts), ctypes.POINTER(I32),
                                  ctypes.POINTER(IncrementReport)],
        "lgdm_commit_increment": [P],
        "lgdm_abort_increment": [P],
        "lgdm_get_csr": [P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(P),
                         ctypes.POINTER(P)],
        "lgdm_get_connectivity": [P, ctypes.POINTER(P), ctypes.POINTER(I64), ctypes.POINTER(I32)],
        "lgdm_get_sizes": [P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(I64)],
        "lgdm_query_state": [P, I32, P, I64],
        "lgdm_set_state": [P, P, P, I64],
        "lgdm_debug_element_blocks": [P, I64, I64, P, P],
        "lgdm_footprint": [P, ctypes.POINTER(I64)],
        "lgdm_kernel_times": [P, I32, P],
        "lgdm_amg_aggregate": [I64, P, P, P, ctypes.POINTER(I64)],
        "lgdm_zone_levels": [I64, P, P, P, ctypes.POINTER(I64)],
        "lgdm_amg_levels": [P, I32, P, ctypes.POINTER(I32)],
        "lgdm_probe_start": [P, I32],
        "lgdm_probe_stop": [P, ctypes.POINTER(D), ctypes.POINTER(I64)],
        "lgdm_batch_create": [ctypes.POINTER(P), I32, P, I32, I32, I64],
        "lgdm_batch_destroy": [P],
        "lgdm_request_footprint": [I32, I64, I64, I32, ctypes.POINTER(I64)],
        "lgdm_batch_admit": [P, ctypes.POINTER(Request), ctypes.POINTER(I32)],
        "lgdm_batch_tick": [P, ctypes.POINTER(SolverOpts), ctypes.POINTER(TickReport)],
        "lgdm_batch_slot_info": [P, I32, ctypes.POINTER(SlotInfo)],
        "lgdm_batch_query": [P, I32, I32, P, I64],
        "lgdm_batch_retire": [P, I32],
        "lgdm_batch_usage": [P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(I32)],
        "lgdm_batch_set_allocator": [P, _ALLOC_T, _FREE_T, P],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = I32
    lib.lgdm_last_error.argtypes = [P]
    lib.lgdm_last_error.restype = ctypes.c_char_p
    lib.lgdm_batch_last_error.argtypes = [P]
    lib.lgdm_batch_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _hiprt():
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    return _hip


class LgdmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


def material_struct(m) -> Material:
    d = m.as_dict() if hasattr(m, "as_dict") else dict(m)
    s = Material()
    for k in ("E", "nu", "kappa0", "alpha", "beta", "c", "R", "eta", "k", "h", "tol_hist", "tol_dmg",
              "thickness"):
        setattr(s, k, float(d[k]))
    s.plane = int(d.get("plane", 0))
    s.coupling = int(d.get("coupling", 0))
    return s


def solver_opts(**kw) -> SolverOpts:
    o = SolverOpts()
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Context:
    """One LGDM problem on one device (C-ABI context)."""

    def __init__(self, device: int = 0, precision: int = FP64, stream=None, torch_allocator=True):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        st = self.lib.lgdm_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream),
                                  precision)
        if st != LGDM_OK:
            raise LgdmError(st, "lgdm_create failed")
        self.h = h
        self.precision = precision
        self._cb = None
        if torch_allocator:
            dev = device
            strm = stream

            def _alloc(n, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(n), dev, strm)
                except Exception:
                    return None

            def _free(p, user):
                torch.cuda.caching_allocator_delete(p)

            self._cb = (_ALLOC_T(_alloc), _FREE_T(_free))
            self._check(self.lib.lgdm_set_allocator(self.h, self._cb[0], self._cb[1], None))
        self.dim = 0

    # -- plumbing ---------------------------------------------------------
    def _check(self, st, ok=(LGDM_OK,)):
        if st not in ok:
            raise LgdmError(st, self.lib.lgdm_last_error(self.h).decode())
        return st

    def close(self):
        if getattr(self, "h", None):
            self.torch.cuda.synchronize(self.device)
            self.lib.lgdm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _ptr(a):
        if a is None:
            return None
        if hasattr(a, "data_ptr"):
            assert a.is_contiguous()
            return ctypes.c_void_p(a.data_ptr())
        assert isinstance(a, np.ndarray) and a.flags["C_CONTIGUOUS"]
        return a.ctypes.data_as(ctypes.c_void_p)

    # -- problem definition -----------------------------------------------
    def upload_mesh(self, dim, elem_type, coords, conn, e_scale=None):
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        conn = np.ascontiguousarray(conn, dtype=np.int32)
        es = None if e_scale is None else np.ascontiguousarray(e_scale, dtype=np.float64)
        self._check(self.lib.lgdm_upload_mesh(self.h, dim, elem_type, coords.shape[0],
                                              self._ptr(coords), conn.shape[0], self._ptr(conn),
                                              self._ptr(es)))
        self.dim = dim
        nd, ng, inc = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.lgdm_get_sizes(self.h, ctypes.byref(nd), ctypes.byref(ng), ctypes.byref(inc)))
        self.ndof, self.ngauss = nd.value, ng.value

    def set_material(self, m):
        s = material_struct(m)
        self._check(self.lib.lgdm_set_material(self.h, ctypes.byref(s)))

    def set_dirichlet(self, dofs, values):
        dofs = np.ascontiguousarray(dofs, dtype=np.int64)
        values = np.ascontiguousarray(values, dtype=np.float64)
        self._check(self.lib.lgdm_set_dirichlet(self.h, dofs.size, self._ptr(dofs), self._ptr(values)))

    def setup_problem(self, prob):
        """Upload an lgdm_workloads.Problem (mesh, material, Dirichlet set)."""
        self.upload_mesh(prob.dim, prob.elem_type, prob.coords, prob.conn, prob.e_scale)
        self.set_material(prob.material)
        self.set_dirichlet(prob.bc_dofs(), prob.bc_values)
        self.n_increments = prob.n_increments

    # -- hot path -----------------------------------------------------------
    def assemble(self, lam: float = -1.0, want_R=True):
        """Compute and assemble K and R at the current state; returns (CsrView, R)."""
        view = CsrView()
        R = self.torch.empty(self.ndof, dtype=self.torch.float64, device="cuda:%d" % self.device) \
            if want_R else None
        st = self.lib.lgdm_assemble_tangent_residual(self.h, float(lam), ctypes.byref(view), self._ptr(R))
        self._check(st)
        return view, R

    def solve_linear(self, b, opts: Optional[SolverOpts] = None):
        x = self.torch.empty_like(b)
        rep = IncrementReport()
        o = opts or SolverOpts()
        self._check(self.lib.lgdm_solve_linear(self.h, self._ptr(b), self._ptr(x), ctypes.byref(o),
                                               ctypes.byref(rep)))
        return x, rep.as_dict()

    def solve_linear_noalloc(self, b, delta, opts: Optional[SolverOpts] = None):
        """lgdm_solve_linear_noalloc: b, delta are device tensors of ndof doubles;
        delta receives the solution.  Returns the report."""
        rep = IncrementReport()
        o = opts or SolverOpts()
        self._check(self.lib.lgdm_solve_linear_noalloc(self.h, self._ptr(b), self._ptr(delta),
                                                       ctypes.byref(o), ctypes.byref(rep)))
        return rep.as_dict()

    def solve_increment(self, lam: float, opts: Optional[SolverOpts] = None, raise_on_fail=True):
        rep = IncrementReport()
        o = opts or SolverOpts()
        st = self.lib.lgdm_solve_increment(self.h, float(lam), ctypes.byref(o), ctypes.byref(rep))
        d = rep.as_dict()
        d["status"] = st
        if raise_on_fail:
            self._check(st)
        return d

    def begin_increment(self, lam: float):
        self._check(self.lib.lgdm_begin_increment(self.h, float(lam)))

    def newton_iteration(self, opts: Optional[SolverOpts] = None, rep: Optional[IncrementReport] = None):
        conv = ctypes.c_int32(0)
        o = opts or SolverOpts()
        r = rep if rep is not None else IncrementReport()
        self._check(self.lib.lgdm_newton_iteration(self.h, ctypes.byref(o), ctypes.byref(conv),
                                                   ctypes.byref(r)))
        return bool(conv.value), r

    def commit_increment(self):
        self._check(self.lib.lgdm_commit_increment(self.h))

    def abort_increment(self):
        self._check(self.lib.lgdm_abort_increment(self.h))

    # -- state --------------------------------------------------------------
    def query(self, field: int, device=False):
        n = {FIELD_X: self.ndof, FIELD_RESIDUAL: self.ndof, FIELD_REACTION: 1}.get(field, self.ngauss)
        if device and field != FIELD_REACTION:
            out = self.torch.empty(n, dtype=self.torch.float64, device="cuda:%d" % self.device)
        else:
            out = np.empty(n, dtype=np.float64)
        self._check(self.lib.lgdm_query_state(self.h, field, self._ptr(out), n))
        return out

    def set_state(self, x=None, kappa_n=None, increment=0):
        x = None if x is None else np.ascontiguousarray(x, dtype=np.float64)
        k = None if kappa_n is None else np.ascontiguousarray(kappa_n, dtype=np.float64)
        self._check(self.lib.lgdm_set_state(self.h, self._ptr(x), self._ptr(k), int(increment)))

    def sizes(self):
        nd, ng, inc = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.lgdm_get_sizes(self.h, ctypes.byref(nd), ctypes.byref(ng), ctypes.byref(inc)))
        return nd.value, ng.value, inc.value

    def csr_pattern(self):
        """Copy the CSR pattern (row_ptr, col_idx) to host numpy arrays."""
        nr, nz = ctypes.c_int64(), ctypes.c_int64()
        rp, ci = ctypes.c_void_p(), ctypes.c_void_p()
        self._check(self.lib.lgdm_get_csr(self.h, ctypes.byref(nr), ctypes.byref(nz), ctypes.byref(rp),
                                          ctypes.byref(ci)))
        self.torch.cuda.synchronize(self.device)
        row_ptr = np.empty(nr.value + 1, dtype=np.int32)
        col_idx = np.empty(nz.value, dtype=np.int32)
        hip = _hiprt()
        assert hip.hipMemcpy(row_ptr.ctypes.data, rp, row_ptr.nbytes, 2) == 0
        assert hip.hipMemcpy(col_idx.ctypes.data, ci, col_idx.nbytes, 2) == 0
        return row_ptr, col_idx

    def csr_values(self, view: CsrView):
        """Copy the values of an assembled CsrView to a host numpy array (FP64 or FP32)."""
        self.torch.cuda.synchronize(self.device)
        hip = _hiprt()
        if view.vals:
            out = np.empty(view.nnz, dtype=np.float64)
            assert hip.hipMemcpy(out.ctypes.data, view.vals, out.nbytes, 2) == 0
        else:
            out = np.empty(view.nnz, dtype=np.float32)
            assert hip.hipMemcpy(out.ctypes.data, view.vals32, out.nbytes, 2) == 0
        return out

    def connectivity(self):
        p, ne, nen = ctypes.c_void_p(), ctypes.c_int64(), ctypes.c_int32()
        self._check(self.lib.lgdm_get_connectivity(self.h, ctypes.byref(p), ctypes.byref(ne), ctypes.byref(nen)))
        out = np.empty((ne.value, nen.value), dtype=np.int32)
        self.torch.cuda.synchronize(self.device)
        assert _hiprt().hipMemcpy(out.ctypes.data, p, out.nbytes, 2) == 0
        return out

    def element_blocks(self, e0: int, e1: int):
        c, n, nen = ctypes.c_void_p(), ctypes.c_int64(), ctypes.c_int32()
        self._check(self.lib.lgdm_get_connectivity(self.h, ctypes.byref(c), ctypes.byref(n), ctypes.byref(nen)))
        nl = nen.value * (self.dim + 1)
        Ke = np.empty((e1 - e0, nl, nl))
        fe = np.empty((e1 - e0, nl))
        self._check(self.lib.lgdm_debug_element_blocks(self.h, e0, e1, self._ptr(Ke), self._ptr(fe)))
        return Ke, fe

    def kernel_times(self, reps=10):
        """Average device ms of [gauss-point kernel, node assembly kernel, SpMV,
        block-Jacobi setup] at the last assembled state."""
        out = np.zeros(4)
        self._check(self.lib.lgdm_kernel_times(self.h, int(reps), self._ptr(out)))
        return out

    def footprint(self):
        b = ctypes.c_int64()
        self._check(self.lib.lgdm_footprint(self.h, ctypes.byref(b)))
        return b.value

    def probe_start(self, kind):
        """Start live timing of one kernel kind inside the solves."""
        self._check(self.lib.lgdm_probe_start(self.h, int(kind)))

    def probe_stop(self):
        """(average ms, launches timed) since probe_start."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        self._check(self.lib.lgdm_probe_stop(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def amg_levels(self):
        """Node counts of the multigrid levels (finest first); empty before
        the first multigrid solve."""
        nodes = np.zeros(16, dtype=np.int64)
        n = ctypes.c_int32()
        self._check(self.lib.lgdm_amg_levels(self.h, 16, nodes.ctypes.data, ctypes.byref(n)))
        return [int(v) for v in nodes[:n.value]]


class Batch:
    """Continuous batching of requests on one device (lgdm_batch_* of the C ABI)."""

    def __init__(self, device: int = 0, precision: int = MIXED, max_slots: int = 64,
                 hbm_budget_bytes: int = 0, stream=None, torch_allocator=True):
        import torch
        self.torch = torch
        self.lib = load_library()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        st = self.lib.lgdm_batch_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream),
                                        precision, max_slots, int(hbm_budget_bytes))
        if st != LGDM_OK:
            raise LgdmError(st, "lgdm_batch_create failed")
        self.h = h
        self.precision = precision
        self._keep = {}
        self._cb = None
        if torch_allocator:
            dev = device
            strm = stream

            def _alloc(n, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(n), dev, strm)
                except Exception:
                    return None

            def _free(p, user):
                torch.cuda.caching_allocator_delete(p)

            self._cb = (_ALLOC_T(_alloc), _FREE_T(_free))
            self._check(self.lib.lgdm_batch_set_allocator(self.h, self._cb[0], self._cb[1], None))

    def _check(self, st, ok=(LGDM_OK,)):
        if st not in ok:
            raise LgdmError(st, self.lib.lgdm_batch_last_error(self.h).decode())
        return st

    def close(self):
        if getattr(self, "h", None):
            self.lib.lgdm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def footprint(self, prob) -> int:
        b = ctypes.c_int64()
        self._check(self.lib.lgdm_request_footprint(prob.dim, prob.n_nodes, prob.n_elems,
                                                    self.precision, ctypes.byref(b)))
        return b.value

    def admit(self, prob):
        """Admit an lgdm_workloads.Problem; returns its slot, or None if the
        batch has no free slot or HBM budget right now."""
        coords = np.ascontiguousarray(prob.coords, dtype=np.float64)
        conn = np.ascontiguousarray(prob.conn, dtype=np.int32)
        es = np.ascontiguousarray(prob.e_scale, dtype=np.float64)
        dofs = np.ascontiguousarray(prob.bc_dofs(), dtype=np.int64)
        vals = np.ascontiguousarray(prob.bc_values, dtype=np.float64)
        r = Request(dim=prob.dim, elem_type=prob.elem_type, n_nodes=prob.n_nodes,
                    coords=coords.ctypes.data, n_elems=prob.n_elems, conn=conn.ctypes.data,
                    e_scale=es.ctypes.data, material=material_struct(prob.material),
                    n_bc=dofs.size, bc_dofs=dofs.ctypes.data, bc_values=vals.ctypes.data,
                    n_increments=prob.n_increments)
        slot = ctypes.c_int32(-1)
        st = self.lib.lgdm_batch_admit(self.h, ctypes.byref(r), ctypes.byref(slot))
        if st == LGDM_ERR_BUSY:
            return None
        self._check(st)
        return slot.value

    def tick(self, opts: Optional[SolverOpts] = None):
        rep = TickReport()
        o = opts or SolverOpts()
        self._check(self.lib.lgdm_batch_tick(self.h, ctypes.byref(o), ctypes.byref(rep)))
        return rep.as_dict()

    def info(self, slot: int):
        i = SlotInfo()
        self._check(self.lib.lgdm_batch_slot_info(self.h, slot, ctypes.byref(i)))
        return i.as_dict()

    def query(self, slot: int, field: int, n: int):
        out = np.empty(n, dtype=np.float64)
        self._check(self.lib.lgdm_batch_query(self.h, slot, field, out.ctypes.data_as(ctypes.c_void_p), n))
        return out

    def retire(self, slot: int):
        self._check(self.lib.lgdm_batch_retire(self.h, slot))

    def usage(self):
        u, b, o = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        self._check(self.lib.lgdm_batch_usage(self.h, ctypes.byref(u), ctypes.byref(b), ctypes.byref(o)))
        return u.value, b.value, o.value


def zone_levels(ptr, adj):
    """The breadth-first level sets that order the process zone, on a host
    CSR graph (no device): returns (level [n] int32, number of levels)."""
    lib = load_library()
    ptr = np.ascontiguousarray(ptr, dtype=np.int32)
    adj = np.ascontiguousarray(adj, dtype=np.int32)
    n = len(ptr) - 1
    level = np.empty(max(n, 0), dtype=np.int32)
    nl = ctypes.c_int64()
    st = lib.lgdm_zone_levels(n, ptr.ctypes.data, adj.ctypes.data, level.ctypes.data, ctypes.byref(nl))
    if st != LGDM_OK:
        raise LgdmError(st, "lgdm_zone_levels")
    return level, nl.value


def amg_aggregate(ptr, adj):
    """The multigrid node aggregation rule on a host CSR graph (no device):
    returns (agg [n] int32, number of aggregates)."""
    lib = load_library()
    ptr = np.ascontiguousarray(ptr, dtype=np.int32)
    adj = np.ascontiguousarray(adj, dtype=np.int32)
    n = len(ptr) - 1
    agg = np.empty(max(n, 0), dtype=np.int32)
    na = ctypes.c_int64()
    st = lib.lgdm_amg_aggregate(n, ptr.ctypes.data, adj.ctypes.data, agg.ctypes.data, ctypes.byref(na))
    if st != LGDM_OK:
        raise LgdmError(st, "lgdm_amg_aggregate")
    return agg, na.value
