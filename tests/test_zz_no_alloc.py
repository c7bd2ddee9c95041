"""lgdm_solve_linear_noalloc against lgdm_solve_linear, through the C ABI.

The allocation-free solve runs the same kernels as lgdm_solve_linear with its
reduction partials and device scalars in a static device array, so its
corrections and reports must be bitwise those of lgdm_solve_linear on the
same assembled system.  Two calls in a row share the array (the second on a
smaller mesh, after the first left its contents there); neither may call the
context's allocator, where lgdm_solve_linear allocates its solution buffer.
"""
import ctypes

import numpy as np
import pytest

import lgdm_workloads as W
from paper_2301_06503_amd import binding as B
from tests.gpu_util import tiny_problems

pytestmark = pytest.mark.gpu

TINY = tiny_problems()
REP_KEYS = ("krylov_iters", "krylov_spmv", "restarts", "krylov_status", "krylov_rel_u", "krylov_rel_e",
            "precond_fallbacks", "inexact_solves")


class CountingContext(B.Context):
    """A context whose device allocations go through torch's caching
    allocator and are counted."""

    def __init__(self, precision):
        super().__init__(device=0, precision=precision, torch_allocator=False)
        import torch
        self.n_alloc = 0
        self.n_free = 0

        def _alloc(n, user):
            self.n_alloc += 1
            try:
                return torch.cuda.caching_allocator_alloc(int(n), 0, self.stream)
            except Exception:
                return None

        def _free(p, user):
            self.n_free += 1
            torch.cuda.caching_allocator_delete(p)

        self._cb = (B._ALLOC_T(_alloc), B._FREE_T(_free))
        self._check(self.lib.lgdm_set_allocator(self.h, self._cb[0], self._cb[1], None))


def _prepared(prob, precision, seed):
    ctx = CountingContext(precision)
    ctx.setup_problem(prob)
    # a mildly perturbed state (below the damage threshold on the larger
    # meshes, whose randomly damaged tangents are too ill-conditioned for a
    # tight solve), partly damaged on the small ones
    mild = prob.n_nodes > 1000
    spread, escale = (0.5, 0.05) if mild else (1.5, 1.0)
    x, kn = W.injected_state(prob, seed=seed, noise=0.02, kappa_spread=spread, ebar_scale=escale)
    ctx.set_state(x, kn)
    _, R = ctx.assemble()
    return ctx, R


def _compare(ctx, R, opts):
    import torch
    ref, rep_ref = ctx.solve_linear(R, opts)             # allocates its solution buffer
    a0 = ctx.n_alloc
    delta = torch.full_like(R, float("nan"))
    rep = ctx.solve_linear_noalloc(R, delta, opts)
    torch.cuda.synchronize()
    assert ctx.n_alloc == a0, "the allocation-free solve called the allocator"
    np.testing.assert_array_equal(delta.cpu().numpy(), ref.cpu().numpy())
    for k in REP_KEYS:
        assert rep[k] == rep_ref[k], (k, rep[k], rep_ref[k])
    return rep


@pytest.mark.parametrize("precision", [B.FP64, B.MIXED])
@pytest.mark.parametrize("big,small,precond", [("beam3d_24x8x6", "beam3d_10x4x3", 1),
                                               ("beam3d_24x8x6", "beam3d_10x4x3", 2),
                                               ("sen2d_13x7_ps", "bar1d_37", 0)])
def test_noalloc_solve_matches_solve_linear(big, small, precond, precision):
    print("case:", big, "then", small, "precond", precond, "precision", precision, flush=True)
    opts = B.solver_opts(tol_krylov=1e-10, max_krylov=50000, precond=precond)
    ctx1, R1 = _prepared(TINY[big], precision, seed=2)
    rep1 = _compare(ctx1, R1, opts)
    # second call in a row, smaller mesh: the static array holds the first
    # call's partials and scalars
    ctx2, R2 = _prepared(TINY[small], precision, seed=4)
    assert ctx2.ndof < ctx1.ndof
    rep2 = _compare(ctx2, R2, opts)
    # and the first context again, after the smaller one
    _compare(ctx1, R1, opts)
    print("iters", rep1["krylov_iters"], rep2["krylov_iters"])
    ctx1.close()
    ctx2.close()


def test_noalloc_solve_argument_errors():
    import torch
    prob = TINY["beam3d_10x4x3"]
    ctx, R = _prepared(prob, B.FP64, seed=2)
    delta = torch.empty_like(R)
    # multigrid (the 3D default) before the hierarchy exists: refused, no work done
    with pytest.raises(B.LgdmError) as ei:
        ctx.solve_linear_noalloc(R, delta, B.solver_opts(tol_krylov=1e-10))
    assert ei.value.status == B.LGDM_ERR_STATE
    # host memory is refused
    host = np.zeros(ctx.ndof)
    st = ctx.lib.lgdm_solve_linear_noalloc(ctx.h, ctypes.c_void_p(R.data_ptr()),
                                           host.ctypes.data_as(ctypes.c_void_p), None, None)
    assert st == B.LGDM_ERR_INVALID_ARG
    # a misaligned solution buffer is refused
    buf = torch.empty(ctx.ndof + 1, dtype=torch.float64, device="cuda:0")
    st = ctx.lib.lgdm_solve_linear_noalloc(ctx.h, ctypes.c_void_p(R.data_ptr()),
                                           ctypes.c_void_p(buf.data_ptr() + 8), None, None)
    assert st == B.LGDM_ERR_INVALID_ARG
    # once a multigrid solve has built the hierarchy, the default works
    ctx.solve_linear(R, B.solver_opts(tol_krylov=1e-10))
    a0 = ctx.n_alloc
    ctx.solve_linear_noalloc(R, delta, B.solver_opts(tol_krylov=1e-10))
    assert ctx.n_alloc == a0
    ctx.close()
