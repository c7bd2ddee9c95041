"""Pins of the mixed-order oracle (quadratic u / linear ebar, Sec. 2.1,
Secs. 3.1-3.2) against what the mathematics fixes independently of it:
the Gauss-Legendre rule, Lagrange interpolation identities, exact solutions
the quadratic element reproduces (pure bending in 2D, a quadratic bar field
under uniform body load in 1D), the elastic bar's closed form, rigid-body
null spaces, finite differences of the residual, the structure of the
blocks without a history update, and an index-notation element loop."""
import math

import numpy as np
import pytest

import lgdm_workloads as W
from oracle.mixed_order import (MixedOracle, element_loop_eval_mixed, eval_elements_mixed,
                                gauss_points_3, reference_nodes_q, shape_functions_q)


def _oracle_of(prob, **kw):
    return MixedOracle(prob, **kw)


# -- quadrature (F1) ---------------------------------------------------------

def test_gauss3_rule_matches_legendre_and_degree():
    p, w = gauss_points_3(1)
    t, wt = np.polynomial.legendre.leggauss(3)
    np.testing.assert_allclose(p[:, 0], t, atol=1e-15)
    np.testing.assert_allclose(w, wt, atol=1e-15)
    for deg in range(6):                        # exact up to degree 5
        exact = 0.0 if deg % 2 else 2.0 / (deg + 1)
        assert abs(np.sum(w * p[:, 0] ** deg) - exact) < 1e-15
    assert abs(np.sum(w * p[:, 0] ** 6) - 2.0 / 7.0) > 1e-3     # and not beyond
    p2, w2 = gauss_points_3(2)
    assert p2.shape == (9, 2) and abs(w2.sum() - 4.0) < 1e-14
    # g = i_xi + 3 i_eta
    np.testing.assert_allclose(p2[5], [p[2, 0], p[1, 0]])
    # 2D: x^4 y^2 exactly
    assert abs(np.sum(w2 * p2[:, 0] ** 4 * p2[:, 1] ** 2) - (2 / 5) * (2 / 3)) < 1e-15


# -- shape functions (F3, F4) ------------------------------------------------

@pytest.mark.parametrize("dim", [1, 2])
def test_quadratic_shape_function_identities(dim):
    nodes = reference_nodes_q(dim)
    nen = len(nodes)
    for a in range(nen):                        # Kronecker delta at the nodes
        N, _ = shape_functions_q(dim, nodes[a])
        np.testing.assert_allclose(N, np.eye(nen)[a], atol=1e-15)
    rng = np.random.default_rng(0)
    mons = [(0, 0), (1, 0), (2, 0)] if dim == 1 else \
        [(i, j) for i in range(3) for j in range(3)]             # complete biquadratic space
    for _ in range(5):
        xi = rng.uniform(-1, 1, dim)
        N, dN = shape_functions_q(dim, xi)
        assert abs(N.sum() - 1.0) < 1e-14 and np.abs(dN.sum(axis=0)).max() < 1e-14
        for (i, j) in mons:
            f = lambda z: z[0] ** i * (z[1] ** j if dim == 2 else 1.0)
            vals = np.array([f(nd) for nd in nodes])
            assert abs(N @ vals - f(xi)) < 1e-14
        hstep = 1e-6                            # derivatives against central differences
        for d in range(dim):
            e = np.zeros(dim); e[d] = hstep
            fd = (shape_functions_q(dim, xi + e)[0] - shape_functions_q(dim, xi - e)[0]) / (2 * hstep)
            np.testing.assert_allclose(dN[:, d], fd, atol=1e-9)


# -- exact solutions the quadratic element reproduces ----------------------

def test_pure_bending_is_reproduced_exactly_plane_stress():
    """u_x = k x (y - y0), u_y = -k (x^2 + nu (y - y0)^2) / 2 is the
    plane-stress pure-bending field (sigma_xx = E k (y - y0), all other
    stresses zero, div sigma = 0).  It is biquadratic, so the 9-node element
    reproduces it exactly on rectangles: zero internal force at every node
    off the boundary, and the right edge's nodal forces carry the moment
    E k t ly^3 / 12 and no net axial force."""
    nx, ny, lx, ly = 5, 3, 10.0, 4.5
    mat = W.base_material(nu=0.25, thickness=2.0)
    prob = W.sen2d_quadratic(nx=nx, ny=ny, lx=lx, ly=ly, notch_len=0, n_increments=1, material=mat)
    o = _oracle_of(prob)
    kb, y0 = 1.3e-6, ly / 2
    X, Y = o.coords[:, 0], o.coords[:, 1]
    x = np.zeros(o.ndof)
    x[0:o.n_nodes * 2:2] = kb * X * (Y - y0)
    x[1:o.n_nodes * 2:2] = -0.5 * kb * (X ** 2 + mat.nu * (Y - y0) ** 2)
    # ebar = 0 and kappa_n = 0: no Gauss point damages
    st = o.eval_state(x, np.zeros(prob.n_elems * 9), want_K=False)
    f = st["fint"][:o.n_nodes * 2].reshape(-1, 2)
    scale = np.abs(f).max()
    tol = 1e-9 * scale
    interior = (X > 1e-9) & (X < lx - 1e-9) & (Y > 1e-9) & (Y < ly - 1e-9)
    assert np.abs(f[interior]).max() <= tol
    right = np.abs(X - lx) < 1e-9
    moment = np.sum(f[right, 0] * (Y[right] - y0))
    expect = mat.E * kb * mat.thickness * ly ** 3 / 12.0
    assert abs(moment - expect) <= 1e-12 * expect, (moment, expect)
    assert abs(np.sum(f[right, 0])) <= tol
    # the top and bottom edges carry no normal traction: their y forces vanish too
    top_bottom = ((np.abs(Y) < 1e-9) | (np.abs(Y - ly) < 1e-9)) & (X > 1e-9) & (X < lx - 1e-9)
    assert np.abs(f[top_bottom, 1]).max() <= tol


def test_bar_quadratic_field_and_linear_ebar():
    """1D, u = a x + b x^2 (quadratic, reproduced exactly), ebar at the
    vertices set to eps = a + 2 b x (linear, reproduced exactly by the linear
    ebar element), below the damage threshold (D = 0, g = 1):
      f_u at a node off the ends = -2 E b int N_a dx, i.e. -2 E b (2L/3) at a
      midpoint and -2 E b (L_left + L_right)/6 at a vertex;
      f_ebar at an interior vertex = 0 (ebar - eeq vanishes pointwise and the
      constant flux g h c 2 b has zero divergence)."""
    mat = W.base_material()
    prob = W.bar1d_quadratic(nx=7, lx=7.0, weak_elem=-1, material=mat)
    rng = np.random.default_rng(1)
    xs = np.concatenate([[0.0], np.cumsum(rng.uniform(0.5, 1.5, 7))])   # uneven element lengths
    coords = np.zeros((15, 1))
    coords[0::2, 0] = xs
    coords[1::2, 0] = 0.5 * (xs[:-1] + xs[1:])
    o = _oracle_of(prob, coords=coords)
    a, b = 2e-6, 3e-7
    X = coords[:, 0]
    x = np.zeros(o.ndof)
    x[:15] = a * X + b * X ** 2
    x[15:] = a + 2 * b * xs
    st = o.eval_state(x, np.zeros(7 * 3), want_K=False)
    f = st["fint"]
    L = np.diff(xs)
    E = mat.E * mat.thickness
    for e in range(7):                          # midpoints
        assert abs(f[2 * e + 1] - (-2 * E * b * 2 * L[e] / 3)) <= 1e-12 * abs(2 * E * b * L[e])
    for v in range(1, 7):                       # interior vertices
        assert abs(f[2 * v] - (-2 * E * b * (L[v - 1] + L[v]) / 6)) <= 1e-12 * abs(2 * E * b * L[v])
        assert abs(f[15 + v]) <= 1e-12 * mat.h * mat.c * 2 * b
    # the end vertices carry the flux -/+ g h c d ebar/dx
    assert abs(f[15] - (-mat.h * mat.c * 2 * b)) <= 1e-12 * mat.h * mat.c * 2 * b
    assert abs(f[15 + 7] - (mat.h * mat.c * 2 * b)) <= 1e-12 * mat.h * mat.c * 2 * b


def test_bar_elastic_closed_form_quadratic():
    """Closed form of the elastic bar (weak centre element E x 0.9): the
    exact solution is piecewise linear, so the quadratic elements give the
    reaction n * u_end/N / (99/E + 1/(0.9 E)) and midpoint displacements
    equal to the mean of their vertices, while max ebar < kappa0."""
    prob = W.config("c0q")
    o = _oracle_of(prob)
    E = prob.material.E
    for n in range(1, 6):
        r = o.solve_increment(tol=1e-12)
        assert r["converged"] and r["max_D"] == 0.0
        expect = n * (0.02 / 100) / (99 / E + 1 / (0.9 * E))
        assert abs(r["reaction"] - expect) <= 1e-11 * expect, (r["reaction"], expect)
    u = o.x[:o.n_nodes]
    np.testing.assert_allclose(u[1::2], 0.5 * (u[0:-1:2] + u[2::2]), rtol=0, atol=1e-16)


# -- null spaces, consistent tangent, structure ------------------------------

def _distorted_q9(seed=3, amp=0.2):
    prob = W.sen2d_quadratic(nx=4, ny=3, lx=8.0, ly=6.0, notch_len=1, n_increments=10)
    rng = np.random.default_rng(seed)
    coords = prob.coords.copy()
    nxn = 2 * 4 + 1
    I = np.arange(prob.n_nodes) % nxn
    J = np.arange(prob.n_nodes) // nxn
    vert = (I % 2 == 0) & (J % 2 == 0) & (I > 0) & (I < 8) & (J > 0) & (J < 6)
    coords[vert] += amp * 2.0 * rng.uniform(-1, 1, (int(vert.sum()), 2))
    # mid-side nodes at edge midpoints, centres at the mean of the corners
    for c in prob.conn:
        for m, (p, q) in zip(range(4, 8), [(0, 1), (1, 2), (2, 3), (3, 0)]):
            coords[c[m]] = 0.5 * (coords[c[p]] + coords[c[q]])
        coords[c[8]] = coords[c[:4]].mean(axis=0)
    prob.coords = coords
    return prob


def _random_state(o, prob, seed, kappa_scale=3.0):
    rng = np.random.default_rng(seed)
    dim = prob.dim
    x = np.zeros(o.ndof)
    x[:o.n_nodes * dim] = 4e-4 * rng.uniform(-1, 1, o.n_nodes * dim) * np.max(np.ptp(o.coords, axis=0))
    x[o.n_nodes * dim:] = prob.material.kappa0 * rng.uniform(0.0, 3.0, o.nvert)
    kn = prob.material.kappa0 * kappa_scale * rng.uniform(0, 1, prob.n_elems * o.ngp)
    return x, kn


@pytest.mark.parametrize("plane", [0, 1])
def test_rigid_body_null_space_q9(plane):
    prob = _distorted_q9()
    prob.material = W.base_material(plane=plane)
    o = _oracle_of(prob)
    x, kn = _random_state(o, prob, seed=4)
    ev = eval_elements_mixed(2, o.coords, o.conn, o.e_scale, o.mat,
                             x[:o.n_nodes * 2].reshape(-1, 2), x[o.n_nodes * 2:], o.vidx, kn)
    assert ev["D"].max() > 0.0                  # damaged points present
    Ke = ev["Ke"]
    for e in range(len(o.conn)):
        xe = o.coords[o.conn[e]]
        modes = [np.tile([1.0, 0.0], 9), np.tile([0.0, 1.0], 9),
                 np.stack([-xe[:, 1], xe[:, 0]], axis=1).ravel()]
        sc = np.abs(Ke[e, :18, :18]).max()
        se = np.abs(Ke[e, 18:, :18]).max()
        for m in modes:
            assert np.abs(Ke[e, :18, :18] @ m).max() <= 1e-12 * sc * np.abs(m).max() * 9
            assert np.abs(Ke[e, 18:, :18] @ m).max() <= 1e-12 * se * np.abs(m).max() * 9


def _fd_check(o, prob, x, kn):
    st = o.eval_state(x, kn)
    K = st["K"].toarray()
    free = np.setdiff1d(np.arange(o.ndof), o.bc_dofs)
    fd = np.zeros((o.ndof, len(free)))
    for j, d in enumerate(free):
        hstep = 1e-7 * max(abs(x[d]), prob.material.kappa0 if d >= o.n_nodes * prob.dim else 1e-4)
        xp = x.copy(); xp[d] += hstep
        xm = x.copy(); xm[d] -= hstep
        Rp = o.eval_state(xp, kn, want_K=False)["R"]
        Rm = o.eval_state(xm, kn, want_K=False)["R"]
        fd[:, j] = -(Rp - Rm) / (2 * hstep)
    um = o.u_mask
    for rows in (um, ~um):
        for cols in (um[free], ~um[free]):
            A = K[np.ix_(rows, free[cols])]
            B = fd[np.ix_(rows, cols)]
            sc = np.abs(B).max()
            if sc > 0:
                assert np.abs(A - B).max() <= 1e-6 * sc, np.abs(A - B).max() / sc


def _away_from_bands(o, prob, x, kn):
    """True if every Gauss point is >= 1e-6 relative away from the history
    and damage bands and from the cone point of A.3."""
    dim = prob.dim
    ev = eval_elements_mixed(dim, o.coords, o.conn, o.e_scale, o.mat, x[:o.n_nodes * dim].reshape(-1, dim),
                             x[o.n_nodes * dim:], o.vidx, kn, want_K=False)
    k0 = prob.material.kappa0
    eb = ev["ebar"].ravel()
    return (np.abs(eb - kn).min() > 1e-6 * k0 and np.abs(ev["kappa"].ravel() - k0).min() > 1e-6 * k0)


@pytest.mark.parametrize("case", ["bar", "ps", "pe"])
def test_consistent_tangent_fd_mixed(case):
    if case == "bar":
        prob = W.bar1d_quadratic(nx=6, lx=6.0, u_end=0.003, material=W.base_material(beta=25.0))
    else:
        prob = _distorted_q9(seed=5)
        prob.material = W.base_material(plane=0 if case == "ps" else 1)
    o = _oracle_of(prob)
    for seed in range(20):
        x, kn = _random_state(o, prob, seed=10 + seed, kappa_scale=2.0)
        if _away_from_bands(o, prob, x, kn):
            break
    else:
        pytest.fail("no state away from the bands")
    _fd_check(o, prob, x, kn)


def test_no_history_update_structure_mixed():
    """With kappa_n above every ebar (chi = 0): K^ue = 0, and K^uu, K^ee are
    symmetric (P9)."""
    prob = _distorted_q9(seed=6)
    o = _oracle_of(prob)
    x, _ = _random_state(o, prob, seed=7)
    kn = np.full(prob.n_elems * 9, 10 * prob.material.kappa0)
    ev = eval_elements_mixed(2, o.coords, o.conn, o.e_scale, o.mat, x[:o.n_nodes * 2].reshape(-1, 2),
                             x[o.n_nodes * 2:], o.vidx, kn)
    Ke = ev["Ke"]
    assert ev["D"].min() > 0
    assert np.abs(Ke[:, :18, 18:]).max() == 0.0
    for blk in (Ke[:, :18, :18], Ke[:, 18:, 18:]):
        sc = np.abs(blk).max()
        assert np.abs(blk - np.transpose(blk, (0, 2, 1))).max() <= 1e-13 * sc
    assert np.abs(Ke[:, 18:, :18]).max() > 0


@pytest.mark.parametrize("case", ["bar", "ps", "pe"])
def test_index_loop_matches_vectorised_mixed(case):
    if case == "bar":
        prob = W.bar1d_quadratic(nx=5, lx=5.0, u_end=0.003)
    else:
        prob = _distorted_q9(seed=8)
        prob.material = W.base_material(plane=0 if case == "ps" else 1)
    o = _oracle_of(prob)
    x, kn = _random_state(o, prob, seed=9)
    dim = prob.dim
    u = x[:o.n_nodes * dim].reshape(-1, dim)
    eb = x[o.n_nodes * dim:]
    ev = eval_elements_mixed(dim, o.coords, o.conn, o.e_scale, o.mat, u, eb, o.vidx, kn)
    Kl, fl = element_loop_eval_mixed(dim, o.coords, o.conn, o.e_scale, o.mat, u, eb, o.vidx, kn)
    nu_ = o.conn.shape[1] * dim
    for sl in ((slice(0, nu_), slice(0, nu_)), (slice(0, nu_), slice(nu_, None)),
               (slice(nu_, None), slice(0, nu_)), (slice(nu_, None), slice(nu_, None))):
        a, b = ev["Ke"][:, sl[0], sl[1]], Kl[:, sl[0], sl[1]]
        sc = np.abs(b).max()
        assert np.abs(a - b).max() <= 1e-12 * max(sc, 1e-300)
    for sl in (slice(0, nu_), slice(nu_, None)):
        sc = np.abs(fl[:, sl]).max()
        assert np.abs(ev["fint"][:, sl] - fl[:, sl]).max() <= 1e-12 * sc


def test_h_invariance_mixed_bar():
    """Under R1 the ebar equation is h [ ... ] = 0: the damaged load path does
    not depend on h (P8), here with quadratic / linear elements."""
    def run(h):
        m = W.base_material(beta=25.0)
        m.h = h
        prob = W.bar1d_quadratic(nx=21, lx=21.0, u_end=0.02, weak_elem=10, n_increments=20, material=m)
        o = _oracle_of(prob)
        for _ in range(14):
            r = o.solve_increment(tol=1e-11)
            assert r["converged"]
        return o
    a, b = run(2e4 * 1e-9), run(2e4)
    assert a.D_n.max() > 0.1
    np.testing.assert_allclose(a.D_n, b.D_n, rtol=0, atol=1e-9)
    np.testing.assert_allclose(a.x[:a.n_nodes], b.x[:b.n_nodes], rtol=0,
                               atol=1e-9 * np.abs(a.x[:a.n_nodes]).max())


def test_layout_maps_round_trip():
    prob = W.sen2d_quadratic(nx=3, ny=2, lx=6.0, ly=4.0, notch_len=1, n_increments=5)
    o = _oracle_of(prob)
    x = np.arange(o.ndof, dtype=float) + 1.0
    xi = o.to_interleaved(x)
    assert xi.shape == (prob.ndof,)
    np.testing.assert_array_equal(o.from_interleaved(xi), x)
    np.testing.assert_array_equal(xi[o.interleaved_index()], x)
    # ebar entries of non-vertex nodes are zero in the interleaved layout
    nonv = np.setdiff1d(np.arange(prob.n_nodes), prob.ebar_nodes())
    assert np.all(xi[nonv * 3 + 2] == 0.0)
