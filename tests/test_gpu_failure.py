"""Failure, work-bound and checkpoint paths of the increment driver, through
the C ABI on the GPU.

  NOT_CONVERGED (max_newton, or the increment work bounds) leaves the
  committed state bitwise unchanged (x, kappa_n, D) and the context usable;
  a non-finite state gives LGDM_ERR_NAN from the assembly and from
  lgdm_solve_increment; a state saved with lgdm_query_state and restored
  into a fresh context with lgdm_set_state continues the load path bitwise
  as the uninterrupted run does.
"""
import numpy as np
import pytest

from paper_2301_06503_amd import binding as B
from tests.gpu_util import context, tiny_problems

pytestmark = pytest.mark.gpu

TINY = tiny_problems()
OPTS = dict(tol_newton=1e-10, tol_krylov=1e-12, max_krylov=50000)


def _state(ctx):
    return ctx.query(B.FIELD_X), ctx.query(B.FIELD_KAPPA), ctx.query(B.FIELD_DAMAGE)


def _run(ctx, prob, n0, n1, opts):
    for n in range(n0, n1):
        ctx.solve_increment((n + 1) / prob.n_increments, opts)


@pytest.mark.parametrize("name", ["sen2d_13x7_ps", "beam3d_10x4x3"])
def test_not_converged_keeps_committed_state(name):
    print("case:", name, flush=True)
    prob = TINY[name]
    ctx = context(prob)
    opts = B.solver_opts(**OPTS)
    _run(ctx, prob, 0, 6, opts)
    before = _state(ctx)
    assert before[2].max() > 0.0            # damaged
    lam = 7 / prob.n_increments
    for kw, msg in ((dict(max_newton=1), "max_newton"),
                    (dict(max_increment_krylov=3), "work bound"),
                    (dict(max_increment_seconds=1e-9), "work bound")):
        d = ctx.solve_increment(lam, B.solver_opts(**dict(OPTS, **kw)), raise_on_fail=False)
        assert d["status"] == B.LGDM_ERR_NOT_CONVERGED, (kw, d["status"])
        err = ctx.lib.lgdm_last_error(ctx.h).decode()
        assert msg in err, err
        after = _state(ctx)
        for a, b in zip(before, after):
            np.testing.assert_array_equal(a, b)
        assert ctx.sizes()[2] == 6
    # the context stays usable: the same increment converges without the bounds
    d = ctx.solve_increment(lam, opts)
    assert d["converged"] == 1 and ctx.sizes()[2] == 7
    ctx.close()


def test_work_bound_caps_krylov_iterations():
    prob = TINY["beam3d_10x4x3"]
    print("case: beam3d_10x4x3 work bound", flush=True)
    ctx = context(prob)
    opts = B.solver_opts(**OPTS)
    _run(ctx, prob, 0, 6, opts)
    d = ctx.solve_increment(7 / prob.n_increments, B.solver_opts(**dict(OPTS, max_increment_krylov=40)),
                            raise_on_fail=False)
    assert d["status"] == B.LGDM_ERR_NOT_CONVERGED
    # each solve is limited to the iterations left; IDR(8) runs whole cycles of 9 steps
    assert d["krylov_iters"] <= 40 + 8, d["krylov_iters"]
    ctx.close()


def test_nan_state_is_reported():
    prob = TINY["sen2d_13x7_ps"]
    print("case: sen2d_13x7_ps NaN", flush=True)
    ctx = context(prob)
    x = np.zeros(prob.ndof)
    x[prob.ndpn * 20 + 1] = np.nan
    ctx.set_state(x, np.zeros(prob.n_elems * prob.ngp))
    view = B.CsrView()
    st = ctx.lib.lgdm_assemble_tangent_residual(ctx.h, -1.0, view, None)
    assert st == B.LGDM_ERR_NAN, st
    d = ctx.solve_increment(1 / prob.n_increments, B.solver_opts(**OPTS), raise_on_fail=False)
    assert d["status"] == B.LGDM_ERR_NAN, d["status"]
    assert ctx.sizes()[2] == 0
    # a finite state assembles again
    ctx.set_state(np.zeros(prob.ndof), np.zeros(prob.n_elems * prob.ngp))
    d = ctx.solve_increment(1 / prob.n_increments, B.solver_opts(**OPTS))
    assert d["converged"] == 1
    ctx.close()


@pytest.mark.parametrize("precision", [B.FP64, B.MIXED])
@pytest.mark.parametrize("name", ["sen2d_13x7_ps", "beam3d_10x4x3"])
def test_checkpoint_resume_bitwise(name, precision):
    print("case:", name, "precision", precision, flush=True)
    prob = TINY[name]
    opts = B.solver_opts(**dict(OPTS, tol_newton=1e-8, tol_krylov=1e-3))
    ref = context(prob, precision)
    _run(ref, prob, 0, 9, opts)
    want = _state(ref)
    ref.close()
    a = context(prob, precision)
    _run(a, prob, 0, 4, opts)
    x, kap = a.query(B.FIELD_X), a.query(B.FIELD_KAPPA)
    a.close()
    b = context(prob, precision)
    b.set_state(x, kap, 4)
    _run(b, prob, 4, 9, opts)
    got = _state(b)
    assert b.sizes()[2] == 9
    b.close()
    assert want[2].max() > 0.0
    for w, g in zip(want, got):
        np.testing.assert_array_equal(w, g)
