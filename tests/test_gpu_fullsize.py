"""Parity at the full sizes the benchmark runs (the 128x32x16 and 256x64x32
beams), in the launch configuration the benchmark times, on sampled outputs
the oracle computes one by one: for sampled nodes (around the notch, on the
supports and at random) the GPU's CSR rows and residual entries are compared
with the oracle's element evaluation of just the elements around each node,
summed as the paper's assembly sums them (Fig. 2), with the Dirichlet
treatment of reading R8; for sampled element ranges the GPU's element blocks
are compared with the oracle's.  Injected (seeded) states."""
import numpy as np
import pytest

import lgdm_workloads as W
from oracle.lgdm import eval_elements
from tests.gpu_util import context

pytestmark = pytest.mark.gpu


def _sample_nodes(prob, rng, n_rand=24):
    weak = np.flatnonzero(prob.e_scale < 1.0)
    near_notch = np.unique(prob.conn[weak[:: max(1, len(weak) // 8)]].ravel())[:24]
    bc = np.unique(prob.bc_nodes)[:: max(1, len(np.unique(prob.bc_nodes)) // 8)][:8]
    rand = rng.choice(prob.n_nodes, n_rand, replace=False)
    return np.unique(np.concatenate([near_notch, bc, rand, [0, prob.n_nodes - 1]]))


def _node_elements(prob):
    flat = prob.conn.ravel().astype(np.int64)
    order = np.argsort(flat, kind="stable")
    starts = np.searchsorted(flat[order], np.arange(prob.n_nodes + 1))
    return order, starts


def _oracle_rows(prob, x, kn, a, order, starts, isbc):
    """Row block of node a (dict: neighbour dof -> values over the node's
    (dim+1) rows) and its residual entries, from the elements around a."""
    nd = prob.ndpn
    nen = prob.conn.shape[1]
    els = order[starts[a]:starts[a + 1]] // nen
    ev = eval_elements(prob.dim, prob.coords, prob.conn, prob.e_scale, prob.material.as_dict(), x, kn, elems=els)
    rows = {}
    R = np.zeros(nd)
    Rabs = np.zeros(nd)   # sum of |element contributions|: the scale of the sum's rounding
    for k, e in enumerate(els):
        la = int(np.flatnonzero(prob.conn[e] == a)[0])
        R -= ev["fint"][k, la * nd:(la + 1) * nd]
        Rabs += np.abs(ev["fint"][k, la * nd:(la + 1) * nd])
        for lb in range(nen):
            b = int(prob.conn[e, lb])
            for j in range(nd):
                col = b * nd + j
                rows.setdefault(col, np.zeros(nd))
                rows[col] += ev["Ke"][k, la * nd:(la + 1) * nd, lb * nd + j]
    # R8: identity rows and zero columns at Dirichlet dofs, zero residual there
    for i in range(nd):
        if isbc[a * nd + i]:
            R[i] = 0.0
            for col in rows:
                rows[col][i] = 1.0 if col == a * nd + i else 0.0
    for col in rows:
        if isbc[col]:
            for i in range(nd):
                if col != a * nd + i:
                    rows[col][i] = 0.0
    return rows, R, Rabs


@pytest.mark.parametrize("name,precision", [("c2", 0), ("c3", 1)])
def test_fullsize_sampled_rows_and_residual(name, precision):
    print("case", name, "precision", precision, flush=True)
    prob = W.config(name)
    x, kn = W.injected_state(prob, seed=5)
    ctx = context(prob, precision)
    ctx.set_state(x, kn)
    view, Rg = ctx.assemble()
    rp, ci = ctx.csr_pattern()
    vals = ctx.csr_values(view)
    Rg = Rg.cpu().numpy()
    nd = prob.ndpn
    isbc = np.zeros(prob.ndof, dtype=bool)
    isbc[prob.bc_dofs()] = True
    order, starts = _node_elements(prob)
    rng = np.random.default_rng(11)
    nodes = _sample_nodes(prob, rng)
    # FP64 contexts: the oracle's sums to 1e-12 of the row's largest entry per
    # block type; mixed contexts store each FP64 sum rounded once to FP32
    worst = {"uu": 0.0, "ue": 0.0, "eu": 0.0, "ee": 0.0, "R": 0.0}
    for a in nodes:
        rows, Ro, Rabs = _oracle_rows(prob, x, kn, int(a), order, starts, isbc)
        for i in range(nd):
            r = int(a) * nd + i
            cols = ci[rp[r]:rp[r + 1]]
            g = vals[rp[r]:rp[r + 1]].astype(np.float64)
            assert sorted(cols.tolist()) == sorted(rows.keys()), (a, i)
            o = np.array([rows[int(c)][i] for c in cols])
            for kind, m in (("u", cols % nd != nd - 1), ("e", cols % nd == nd - 1)):
                key = ("e" if i == nd - 1 else "u") + kind
                scale = np.abs(o[m]).max()
                if scale == 0:
                    continue
                err = np.abs(g[m] - o[m]).max() / scale
                worst[key] = max(worst[key], err)
        dR = np.abs(Rg[int(a) * nd:(int(a) + 1) * nd] - Ro)
        worst["R"] = max(worst["R"], float(np.max(dR / np.maximum(Rabs, 1e-300))))
    print("sampled nodes", len(nodes), "max relative error", worst)
    tol = 1e-12 if precision == 0 else 1.2e-7
    for k in ("uu", "ue", "eu", "ee"):
        assert worst[k] <= tol, worst
    assert worst["R"] <= 1e-12, worst      # the residual is FP64 in both precisions
    ctx.close()


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_fullsize_sampled_element_blocks(name):
    print("case", name, flush=True)
    prob = W.config(name)
    x, kn = W.injected_state(prob, seed=6)
    ctx = context(prob, 1 if name == "c3" else 0)
    ctx.set_state(x, kn)
    ctx.assemble()
    weak = np.flatnonzero(prob.e_scale < 1.0)
    for e0 in (0, int(weak[0]), prob.n_elems // 2 + 17, prob.n_elems - 64):
        e1 = min(e0 + 64, prob.n_elems)
        Ke, fe = ctx.element_blocks(e0, e1)
        ev = eval_elements(prob.dim, prob.coords, prob.conn, prob.e_scale, prob.material.as_dict(), x, kn,
                           elems=np.arange(e0, e1))
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
