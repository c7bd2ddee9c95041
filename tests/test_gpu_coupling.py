"""GPU parity of the coupling variant (material coupling = 1: the stress of
Eq. 2 with its h term, Eq. 11b as printed, K^uu completed by the
linearisation of Eq. 2) against the oracle, through the C ABI: assembled
CSR values and residuals on injected states, element blocks, and damage over
whole load paths.  The coupling modulus is raised from the workloads' h =
1e-9 E so that the variant's terms are visible next to (1 - D) C."""
import dataclasses

import numpy as np
import pytest

import lgdm_workloads as W
from oracle.lgdm import Oracle, eval_elements
from tests.gpu_util import context, blockwise_error, fieldwise_error, tiny_problems

pytestmark = pytest.mark.gpu

TINY = tiny_problems()


def _coupled(name, h_over_e):
    prob = TINY[name] if name in TINY else W.config(name)
    prob.material = dataclasses.replace(prob.material, coupling=1, h=h_over_e * prob.material.E)
    return prob


def _print_case(name):
    print("case", name, flush=True)


@pytest.mark.parametrize("name", ["bar1d_37", "sen2d_13x7_ps", "sen2d_13x7_pe", "beam3d_6x4x3_distorted", "c3p"])
@pytest.mark.parametrize("seed", [0, 1])
def test_coupled_injected_state_assembly_parity(name, seed):
    _print_case("%s seed=%d" % (name, seed))
    prob = _coupled(name, 0.3)
    x, kn = W.injected_state(prob, seed=seed)
    ctx = context(prob)
    ctx.set_state(x, kn)
    view, R = ctx.assemble()
    vals = ctx.csr_values(view)
    rp, ci = ctx.csr_pattern()
    st = Oracle(prob).eval_state(x, kn)
    K = st["K"]
    np.testing.assert_array_equal(K.indptr, rp.astype(np.int64))
    err = blockwise_error(vals, K.data, rp, ci, prob.ndpn)
    print("blockwise error", err)
    assert max(err.values()) <= 1e-12, err
    ferr = fieldwise_error(R.cpu().numpy(), st["R"], prob.ndpn)
    assert max(ferr.values()) <= 1e-12, ferr
    assert ctx.query(6)[0] == pytest.approx(st["reaction"], rel=1e-10, abs=1e-12)
    ctx.close()


@pytest.mark.parametrize("name", ["bar1d_37", "sen2d_9x6_distorted", "beam3d_6x4x3_distorted"])
def test_coupled_element_blocks_parity(name):
    _print_case(name)
    prob = _coupled(name, 0.3)
    x, kn = W.injected_state(prob, seed=7)
    ctx = context(prob)
    ctx.set_state(x, kn)
    ctx.assemble()
    Ke, fe = ctx.element_blocks(0, prob.n_elems)
    ev = eval_elements(prob.dim, prob.coords, prob.conn, prob.e_scale, prob.material.as_dict(), x, kn)
    nd = prob.ndpn
    nl = prob.nen * nd
    iu = np.array([i for i in range(nl) if i % nd != prob.dim])
    ie = np.arange(prob.dim, nl, nd)
    for rows, cols in [(iu, iu), (iu, ie), (ie, iu), (ie, ie)]:
        a = Ke[:, rows[:, None], cols[None, :]]
        b = ev["Ke"][:, rows[:, None], cols[None, :]]
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
    for rows in (iu, ie):
        assert np.abs(fe[:, rows] - ev["fint"][:, rows]).max() <= 1e-12 * np.abs(ev["fint"][:, rows]).max()
    ctx.close()


def test_coupled_differs_from_executed_form():
    """The variant's terms are present on the GPU: with the same state, the
    coupled assembly differs from the executed-code form, and switching the
    material back gives the executed form's oracle values again."""
    prob = _coupled("beam3d_6x4x3_distorted", 0.3)
    x, kn = W.injected_state(prob, seed=3)
    ctx = context(prob)
    ctx.set_state(x, kn)
    view, _ = ctx.assemble()
    v1 = ctx.csr_values(view).copy()
    ctx.set_material(dataclasses.replace(prob.material, coupling=0))
    ctx.set_state(x, kn)
    view, _ = ctx.assemble()
    v0 = ctx.csr_values(view).copy()
    assert np.abs(v1 - v0).max() > 1e-3 * np.abs(v0).max()
    p0 = dataclasses.replace(prob, material=dataclasses.replace(prob.material, coupling=0))
    K0 = Oracle(p0).eval_state(x, kn)["K"]
    assert np.abs(v0 - K0.data).max() <= 1e-12 * np.abs(K0.data).max()
    ctx.close()


@pytest.mark.parametrize("name,precision", [("bar1d_37", 0), ("sen2d_13x7_ps", 0), ("beam3d_10x4x3", 0),
                                            ("sen2d_13x7_ps", 1), ("beam3d_10x4x3", 1)])
def test_coupled_load_path_damage_parity(name, precision):
    """Damage after every increment of the whole path against the oracle:
    1e-8 in FP64 contexts, 1e-7 in mixed ones (FP32 tangent, FP64 residual,
    so the converged states differ only by the Newton tolerance)."""
    from paper_2301_06503_amd import binding
    _print_case("%s precision %d" % (name, precision))
    prob = _coupled(name, 0.01)
    ctx = context(prob, precision)
    o = Oracle(prob)
    opts = binding.solver_opts(tol_newton=1e-10, tol_krylov=1e-13, max_krylov=50000)
    worst = 0.0
    for n in range(1, prob.n_increments + 1):
        lam = n / prob.n_increments
        rg = ctx.solve_increment(lam, opts, raise_on_fail=False)
        ro = o.solve_increment(lam=lam, tol=1e-10)
        assert ro["converged"], n
        assert rg["status"] == 0, (n, ctx.lib.lgdm_last_error(ctx.h).decode())
        worst = max(worst, float(np.abs(ctx.query(2) - ro["D"]).max()))
        assert rg["reaction"] == pytest.approx(ro["reaction"], rel=1e-7, abs=1e-10)
    print("max damage error over the path", worst, "max D", float(ro["D"].max()))
    assert worst <= (1e-8 if precision == 0 else 1e-7)
    ctx.close()


def test_batch_rejects_coupling_variant():
    from paper_2301_06503_amd import binding
    prob = _coupled("sen2d_13x7_ps", 0.01)
    b = binding.Batch(device=0, precision=binding.MIXED, max_slots=2)
    with pytest.raises(binding.LgdmError):
        b.admit(prob)
    b.close()


def test_coupling_value_checked():
    from paper_2301_06503_amd import binding
    prob = TINY["bar1d_37"]
    ctx = context(prob)
    bad = dataclasses.replace(prob.material, coupling=2)
    with pytest.raises(binding.LgdmError):
        ctx.set_material(bad)
    ctx.close()
