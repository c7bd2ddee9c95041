"""Continuous batching: each request's results are the same alone and in a
mix (bitwise: every reduction belongs to one request and runs in a fixed
order), admission respects the HBM budget, and a served request matches the
FP64 oracle."""
import numpy as np
import pytest

import lgdm_workloads as W
from oracle.lgdm import Oracle

pytestmark = pytest.mark.gpu


def _reqs():
    # the first `inc` increments of 200-increment paths to 0.1 mm (past damage onset)
    mk = lambda nx, inc, **kw: W.sen2d(nx=nx, ny=nx // 2, notch_len=nx // 4, n_increments=inc,
                                       u_top=0.1 * inc / 200, material=W.base_material(**kw))
    return [mk(40, 6), mk(60, 5, E=3e4, kappa0=1.5e-4, beta=200.0, c=8.0),
            mk(50, 7, E=2.5e4, c=2.0, R=0.01), mk(40, 4, kappa0=6e-5)]


def _run(batch, probs, arrive_at, opts, max_ticks=2000):
    from paper_2301_06503_amd import binding
    slots, out, tick = {}, {}, 0
    waiting = list(range(len(probs)))
    while (waiting or slots) and tick < max_ticks:
        for i in list(waiting):
            if arrive_at[i] <= tick:
                s = batch.admit(probs[i])
                if s is not None:
                    slots[s] = i
                    waiting.remove(i)
        batch.tick(opts)
        tick += 1
        for s, i in list(slots.items()):
            inf = batch.info(s)
            if inf["state"] in (binding.SLOT_FINISHED, binding.SLOT_FAILED):
                assert inf["state"] == binding.SLOT_FINISHED, (i, inf)
                out[i] = (batch.query(s, binding.FIELD_X, inf["ndof"]),
                          batch.query(s, binding.FIELD_DAMAGE, inf["n_gauss"]), inf)
                batch.retire(s)
                del slots[s]
    assert not waiting and not slots
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_alone_vs_mix_bitwise(precision):
    from paper_2301_06503_amd import binding
    probs = _reqs()
    opts = binding.solver_opts(max_newton=40, tol_newton=1e-9, tol_krylov=1e-10, check_every=8)
    alone = {}
    for i, p in enumerate(probs):
        b = binding.Batch(precision=precision, max_slots=4)
        alone[i] = _run(b, [p], [0], opts)[0]
        b.close()
    b = binding.Batch(precision=precision, max_slots=4)
    mix = _run(b, probs, [0, 1, 3, 6], opts)
    b.close()
    for i in range(len(probs)):
        xa, da, ia = alone[i]
        xm, dm, im = mix[i]
        print("request %d: %d increments, %d Newton, max D %.3f; alone vs mix identical: %s"
              % (i, ia["increment"], ia["newton_total"], da.max(), np.array_equal(xa, xm)))
        np.testing.assert_array_equal(xa, xm)
        np.testing.assert_array_equal(da, dm)
        assert ia["newton_total"] == im["newton_total"] and ia["krylov_total"] == im["krylov_total"]


def test_admission_respects_budget():
    from paper_2301_06503_amd import binding
    probs = _reqs()
    b0 = binding.Batch(precision=1, max_slots=8)
    fp = [b0.footprint(p) for p in probs]
    b0.close()
    budget = fp[0] + fp[1] + fp[1] // 2          # room for two of the first three
    b = binding.Batch(precision=1, max_slots=8, hbm_budget_bytes=budget)
    s0 = b.admit(probs[0])
    s1 = b.admit(probs[1])
    assert s0 is not None and s1 is not None
    assert b.admit(probs[2]) is None              # over budget: refused, nothing changed
    used, bud, occ = b.usage()
    assert occ == 2 and used <= bud
    opts = binding.solver_opts(max_newton=40, tol_newton=1e-8, tol_krylov=1e-8)
    for _ in range(500):
        b.tick(opts)
        if b.info(s0)["state"] != binding.SLOT_RUNNING:
            break
    assert b.info(s0)["state"] == binding.SLOT_FINISHED
    b.retire(s0)
    assert b.admit(probs[2]) is not None          # admitted once memory is free
    b.close()
    b = binding.Batch(precision=1, max_slots=1)
    assert b.admit(probs[3]) is not None
    assert b.admit(probs[0]) is None              # no free slot
    b.close()


def test_served_request_matches_oracle():
    from paper_2301_06503_amd import binding
    p = _reqs()[0]
    b = binding.Batch(precision=0, max_slots=2)
    out = _run(b, [p], [0], binding.solver_opts(max_newton=40, tol_newton=1e-10, tol_krylov=1e-13))
    b.close()
    o = Oracle(p)
    for _ in range(p.n_increments):
        assert o.solve_increment(tol=1e-10)["converged"]
    x, D, info = out[0]
    err = np.abs(D - o.D_n).max()
    print("served request vs oracle: max damage error %.3e (max D %.3f)" % (err, o.D_n.max()))
    assert err <= 1e-8
    np.testing.assert_allclose(x, o.x, rtol=0, atol=1e-9 * np.abs(o.x).max())


def test_serving_loop_stream():
    """A short seeded stream through the scheduler: every request finishes,
    latency statistics are produced."""
    from paper_2301_06503_amd import binding, serving
    reqs = W.serving_stream(n_requests=6, rate_per_s=50.0, seed=1, nx_min=40, nx_max=80,
                            first_increments=5)
    loop = serving.ServingLoop(reqs, precision=1, max_slots=4)
    summ = loop.run(time_limit_s=240, realtime=True, log=print)
    loop.close()
    print(summ)
    assert summ["requests_finished"] == 6
    assert summ["latency_p50_ms"] is not None and summ["latency_p99_ms"] >= summ["latency_p50_ms"]


@pytest.mark.parametrize("precision", [0, 1])
def test_fused_assembly_matches_single(precision):
    """The fused multi-request launch computes exactly what the single-request
    launch computes (same residual, bitwise) for every request of the mix."""
    from paper_2301_06503_amd import binding
    probs = _reqs()[:3]
    b = binding.Batch(precision=precision, max_slots=4)
    slots = [b.admit(p) for p in probs]
    b.tick(binding.solver_opts(max_newton=5, tol_newton=1e-9, tol_krylov=1e-10))
    for p, s in zip(probs, slots):
        Rb = b.query(s, binding.FIELD_RESIDUAL, p.ndof)
        Db = b.query(s, binding.FIELD_DAMAGE_TRIAL, p.n_elems * p.ngp)
        ctx = binding.Context(precision=precision)
        ctx.setup_problem(p)
        ctx.begin_increment(1.0 / p.n_increments)
        _, R = ctx.assemble()
        Rs = R.cpu().numpy()
        print("slot %d: max |R_fused - R_single| = %.3e (max |R| %.3e)"
              % (s, np.abs(Rb - Rs).max(), np.abs(Rs).max()))
        np.testing.assert_array_equal(Rb, Rs)
        np.testing.assert_array_equal(Db, ctx.query(binding.FIELD_DAMAGE_TRIAL))
        ctx.close()
    b.close()


def test_alone_vs_mix_bitwise_large_requests():
    """Requests large enough that the batched solve's per-request workgroup
    counts hit their caps (grid-stride within the request) give the same
    results alone and beside smaller requests."""
    from paper_2301_06503_amd import binding
    mk = lambda nx, inc, **kw: W.sen2d(nx=nx, ny=nx // 2, notch_len=nx // 4, n_increments=inc,
                                       u_top=0.1 * inc / 200, material=W.base_material(**kw))
    probs = [mk(210, 3), mk(40, 4, kappa0=6e-5), mk(150, 3, E=3e4)]
    opts = binding.solver_opts(max_newton=40, tol_newton=1e-8, tol_krylov=1e-3, check_every=32)
    alone = {}
    for i, p in enumerate(probs):
        b = binding.Batch(precision=1, max_slots=4)
        alone[i] = _run(b, [p], [0], opts)[0]
        b.close()
    b = binding.Batch(precision=1, max_slots=4)
    mix = _run(b, probs, [0, 0, 2], opts)
    b.close()
    for i in range(len(probs)):
        xa, da, ia = alone[i]
        xm, dm, im = mix[i]
        print("request %d (%d dofs): %d Newton, identical %s" % (i, probs[i].ndof, ia["newton_total"],
                                                                 np.array_equal(xa, xm)))
        np.testing.assert_array_equal(xa, xm)
        np.testing.assert_array_equal(da, dm)
