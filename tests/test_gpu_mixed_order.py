"""GPU parity of the mixed-order elements (quadratic u, linear ebar; Sec. 2.1,
Secs. 3.1-3.2) against the mixed-order oracle, through the C ABI.

  pattern and connectivity: bit-exact (the node-interleaved node-graph
    pattern, every element-coupled node pair);
  injected states: assembled tangent values per block type and the residual
    to 1e-12 of their scale, Gauss-point kappa / D / eeq, element blocks
    (the oracle's [u | ebar] blocks mapped to the node-interleaved layout;
    ebar rows and columns of non-vertex nodes exactly zero, their assembled
    rows identity);
  whole load paths: damage at every Gauss point after every increment to
    1e-8 (FP64) and 1e-7 (mixed precision), reactions to 1e-6.
"""
import numpy as np
import pytest

import lgdm_workloads as W
from oracle.lgdm import csr_pattern_bruteforce
from oracle.mixed_order import MixedOracle, eval_elements_mixed
from paper_2301_06503_amd import binding as B
from tests.gpu_util import blockwise_error, context

pytestmark = pytest.mark.gpu


def _distorted_q9(nx=5, ny=3, seed=3, amp=0.2):
    prob = W.sen2d_quadratic(nx=nx, ny=ny, lx=2.0 * nx, ly=2.0 * ny, notch_len=1, u_top=0.004,
                             n_increments=10)
    rng = np.random.default_rng(seed)
    coords = prob.coords.copy()
    nxn = 2 * nx + 1
    I = np.arange(prob.n_nodes) % nxn
    J = np.arange(prob.n_nodes) // nxn
    vert = (I % 2 == 0) & (J % 2 == 0) & (I > 0) & (I < 2 * nx) & (J > 0) & (J < 2 * ny)
    coords[vert] += amp * 2.0 * rng.uniform(-1, 1, (int(vert.sum()), 2))
    for c in prob.conn:
        for m, (p, q) in zip(range(4, 8), [(0, 1), (1, 2), (2, 3), (3, 0)]):
            coords[c[m]] = 0.5 * (coords[c[p]] + coords[c[q]])
        coords[c[8]] = coords[c[:4]].mean(axis=0)
    prob.coords = coords
    prob.name = "sen2dq_%dx%d_distorted" % (nx, ny)
    return prob


def problems():
    out = {
        "bar1dq_37": W.bar1d_quadratic(nx=37, lx=37.0, u_end=0.01, weak_elem=18, n_increments=30,
                                       material=W.base_material(beta=25.0)),
        "sen2dq_13x7_ps": W.sen2d_quadratic(nx=13, ny=7, lx=26.0, ly=14.0, notch_len=4, u_top=0.006,
                                            n_increments=30),
        "sen2dq_13x7_pe": W.sen2d_quadratic(nx=13, ny=7, lx=26.0, ly=14.0, notch_len=4, u_top=0.006,
                                            n_increments=20, material=W.base_material(plane=1)),
        "sen2dq_40x20": W.sen2d_quadratic(nx=40, ny=20, lx=80.0, ly=40.0, notch_len=10, u_top=0.01,
                                          n_increments=30),
    }
    d = _distorted_q9()
    out[d.name] = d
    return out


PROBS = problems()


def _case(msg):
    print("case:", msg, flush=True)


@pytest.mark.parametrize("name", sorted(PROBS))
def test_mixed_order_pattern_bitexact(name):
    _case(name)
    prob = PROBS[name]
    ctx = context(prob)
    rp, ci = ctx.csr_pattern()
    rp0, ci0 = csr_pattern_bruteforce(prob.conn, prob.n_nodes, prob.ndpn)
    np.testing.assert_array_equal(rp, rp0)
    np.testing.assert_array_equal(ci, ci0)
    np.testing.assert_array_equal(ctx.connectivity(), prob.conn)
    assert ctx.ngauss == prob.n_elems * prob.ngp
    ctx.close()


def _oracle_in_interleaved(o, prob, K, R):
    """The oracle's tangent and residual in the node-interleaved layout, with
    the identity rows of the ebar dofs of non-vertex nodes."""
    import scipy.sparse as sp
    idx = o.interleaved_index()
    Kc = K.tocoo()
    n = prob.ndof
    inactive = np.setdiff1d(np.arange(prob.n_nodes), prob.ebar_nodes()) * prob.ndpn + prob.dim
    rows = np.concatenate([idx[Kc.row], inactive])
    cols = np.concatenate([idx[Kc.col], inactive])
    vals = np.concatenate([Kc.data, np.ones(len(inactive))])
    Kil = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    Ril = np.zeros(n)
    Ril[idx] = R
    return Kil, Ril, inactive


@pytest.mark.parametrize("name", ["bar1dq_37", "sen2dq_13x7_ps", "sen2dq_13x7_pe", "sen2dq_5x3_distorted",
                                  "sen2dq_40x20"])
@pytest.mark.parametrize("seed", [1, 2])
def test_mixed_order_injected_state_parity(name, seed):
    _case("%s seed %d" % (name, seed))
    prob = PROBS[name]
    x, kn = W.injected_state(prob, seed=seed, noise=0.25, kappa_spread=3.0)
    ctx = context(prob)
    ctx.set_state(x, kn)
    view, R = ctx.assemble()
    o = MixedOracle(prob)
    st = o.eval_state(o.from_interleaved(x), kn)
    Kil, Ril, inactive = _oracle_in_interleaved(o, prob, st["K"], st["R"])
    rp, ci = ctx.csr_pattern()
    vals = ctx.csr_values(view)
    rows = np.repeat(np.arange(prob.ndof), np.diff(rp))
    ref = np.asarray(Kil[rows, ci]).ravel()
    # every oracle entry lies in the GPU pattern
    assert abs(Kil.sum() - ref.sum()) <= 1e-9 * np.abs(Kil).sum()
    err = blockwise_error(vals, ref, rp, ci, prob.ndpn)
    print("blockwise", err)
    assert max(err.values()) <= 1e-12, err
    # constrained ebar rows of non-vertex nodes: identity; their columns: zero
    for d in inactive[:20]:
        row = vals[rp[d]:rp[d + 1]]
        assert np.all(row[ci[rp[d]:rp[d + 1]] != d] == 0.0) and row[ci[rp[d]:rp[d + 1]] == d][0] == 1.0
    assert np.all(vals[np.isin(ci, inactive) & ~np.isin(rows, inactive)] == 0.0)
    r = R.cpu().numpy()
    nd = prob.ndpn
    for fld in (np.arange(prob.ndof) % nd != nd - 1, np.arange(prob.ndof) % nd == nd - 1):
        sc = np.abs(Ril[fld]).max()
        assert np.abs(r[fld] - Ril[fld]).max() <= 1e-12 * sc
    assert np.all(r[inactive] == 0.0)
    # Gauss-point state of this assembly
    for fld, key in ((B.FIELD_KAPPA_TRIAL, "kappa"), (B.FIELD_DAMAGE_TRIAL, "D"), (B.FIELD_EEQ, "eeq")):
        g = ctx.query(fld)
        refv = st[key].ravel()
        assert np.abs(g - refv).max() <= 1e-12 * max(np.abs(refv).max(), 1e-300), key
    assert st["D"].max() > 0.0
    ctx.close()


@pytest.mark.parametrize("name", ["bar1dq_37", "sen2dq_5x3_distorted"])
def test_mixed_order_element_blocks_parity(name):
    _case(name)
    prob = PROBS[name]
    x, kn = W.injected_state(prob, seed=3, noise=0.25, kappa_spread=3.0)
    ctx = context(prob)
    ctx.set_state(x, kn)
    ctx.assemble()
    ne = prob.n_elems
    Ke, fe = ctx.element_blocks(0, ne)
    o = MixedOracle(prob)
    dim, nd, nen = prob.dim, prob.ndpn, prob.nen
    xo = o.from_interleaved(x)
    st = eval_elements_mixed(dim, o.coords, o.conn, o.e_scale, o.mat, xo[:o.n_nodes * dim].reshape(-1, dim),
                             xo[o.n_nodes * dim:], o.vidx, kn)
    loc = np.concatenate([(np.arange(nen)[:, None] * nd + np.arange(dim)).ravel(),
                          np.arange(2 ** dim) * nd + dim])          # oracle local -> interleaved local
    nu_ = nen * dim
    for rs, cs in ((slice(0, nu_), slice(0, nu_)), (slice(0, nu_), slice(nu_, None)),
                   (slice(nu_, None), slice(0, nu_)), (slice(nu_, None), slice(nu_, None))):
        a = Ke[:, loc[rs][:, None], loc[cs][None, :]]
        b = st["Ke"][:, rs, cs]
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
    # ebar rows / columns of the non-vertex local nodes are exactly zero
    other = np.setdiff1d(np.arange(nen * nd), loc)
    assert np.all(Ke[:, other, :] == 0.0) and np.all(Ke[:, :, other] == 0.0)
    for sl in (slice(0, nu_), slice(nu_, None)):
        assert np.abs(fe[:, loc[sl]] - st["fint"][:, sl]).max() <= 1e-12 * np.abs(st["fint"][:, sl]).max()
    ctx.close()


def _paths(prob, precision, n_inc):
    o = MixedOracle(prob)
    ctx = context(prob, precision=precision)
    opts = B.solver_opts(tol_newton=1e-10, tol_krylov=1e-13, max_krylov=50000, max_newton=40)
    out = []
    for n in range(n_inc):
        lam = (n + 1) / prob.n_increments
        r = o.solve_increment(lam=lam, tol=1e-10, max_iter=40)
        assert r["converged"], "oracle increment %d" % (n + 1)
        rep = ctx.solve_increment(lam, opts)
        Dg = ctx.query(B.FIELD_DAMAGE)
        out.append((np.abs(Dg - o.D_n).max(), rep["reaction"], r["reaction"], o.D_n.max()))
    xg = ctx.query(B.FIELD_X)
    ctx.close()
    return out, xg, o


@pytest.mark.parametrize("name,precision", [("bar1dq_37", B.FP64), ("sen2dq_13x7_ps", B.FP64),
                                            ("sen2dq_13x7_pe", B.FP64), ("bar1dq_37", B.MIXED),
                                            ("sen2dq_13x7_ps", B.MIXED)])
def test_mixed_order_load_path_damage_parity(name, precision):
    _case("%s precision %d" % (name, precision))
    prob = PROBS[name]
    out, xg, o = _paths(prob, precision, prob.n_increments)
    bound = 1e-8 if precision == B.FP64 else 1e-7
    worst = max(e for e, _, _, _ in out)
    print("max damage error over the path %.3e, final max D %.4f" % (worst, out[-1][3]))
    assert worst <= bound
    assert out[-1][3] > 0.5                      # the path damages
    for _, rg, ro, _ in out:
        assert abs(rg - ro) <= 1e-6 * max(abs(ro), 1e-12)
    # ebar dofs of non-vertex nodes stay exactly zero
    inactive = np.setdiff1d(np.arange(prob.n_nodes), prob.ebar_nodes()) * prob.ndpn + prob.dim
    assert np.all(xg[inactive] == 0.0)
    assert np.abs(o.from_interleaved(xg) - o.x).max() <= 1e-6 * np.abs(o.x).max()


def test_mixed_order_argument_errors():
    prob = PROBS["bar1dq_37"]
    ctx = B.Context(device=0, precision=B.FP64)
    # an element type that does not match the dimension is refused before
    # any array is read
    q9 = PROBS["sen2dq_5x3_distorted"]
    with pytest.raises(B.LgdmError):
        ctx.upload_mesh(2, W.LINE3, q9.coords, q9.conn)
    ctx.upload_mesh(1, W.LINE3, prob.coords, prob.conn, prob.e_scale)
    m = prob.material.as_dict()
    m["coupling"] = 1
    with pytest.raises(B.LgdmError):
        ctx.set_material(m)
    # Dirichlet conditions on ebar dofs are refused, as for equal-order meshes
    ctx.set_material(prob.material)
    with pytest.raises(B.LgdmError):
        ctx.set_dirichlet(np.array([1]), np.array([0.0]))
    ctx.close()
