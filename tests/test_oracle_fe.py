"""Pins of the oracle's finite-element layer (Eqs. 9-11f, Fig. 2 assembly)
against facts that do not come from the oracle: shape-function identities,
patch tests, rigid-body null spaces, finite differences of the residual,
symmetry, the closed-form elastic bar, brute-force sparsity patterns and the
h-invariance of the solution.  CPU only."""
import math

import numpy as np
import pytest

import lgdm_workloads as W
from oracle.lgdm import (reference_nodes, gauss_points, shape_functions, eval_elements,
                         element_loop_eval, csr_pattern_bruteforce, csr_pattern_unique,
                         assemble, Oracle, equivalent_strain_voigt)


def tiny(dim, plane=0, seed=0, distort=0.0):
    mat = W.base_material(plane=plane)
    if dim == 1:
        p = W.bar1d(nx=6, lx=6.0, u_end=1.2e-3, weak_elem=2, n_increments=10, material=mat)
    elif dim == 2:
        p = W.sen2d(nx=4, ny=2, lx=4.0, ly=2.0, notch_len=1, u_top=4e-4, n_increments=10,
                    material=mat)
    else:
        p = W.beam3d(nx=4, ny=2, nz=2, lx=4.0, ly=2.0, lz=2.0, u_load=-6e-4, n_increments=10,
                     material=mat)
    if distort:
        p.coords = W.perturbed_coords(p, seed, distort)
    return p


# ----------------------------------------------------------------- shape functions

@pytest.mark.parametrize("dim", [1, 2, 3])
def test_shape_functions_identities(dim):
    nodes = reference_nodes(dim)
    for a, xa in enumerate(nodes):
        N, _ = shape_functions(dim, xa)
        np.testing.assert_allclose(N, np.eye(len(nodes))[a], atol=1e-15)
    pts, w = gauss_points(dim)
    assert w.sum() == pytest.approx(2.0 ** dim)          # reference volume
    for xi in pts:
        N, dN = shape_functions(dim, xi)
        assert N.sum() == pytest.approx(1.0)
        np.testing.assert_allclose(dN.sum(axis=0), 0.0, atol=1e-15)
        # linear completeness: sum_a x_a dN_a/dxi = identity on the reference element
        np.testing.assert_allclose(nodes.T @ dN, np.eye(dim), atol=1e-15)
    # 2-point rule integrates xi^2 exactly (int_{-1}^{1} xi^2 = 2/3)
    assert sum(p[0] ** 2 for p in pts) * 2 ** (1 - dim) == pytest.approx(2.0 / 3.0)


def test_workload_meshes_are_valid():
    for p in [W.config("c0"), W.sen2d(20, 10, 20.0, 10.0), W.beam3d(8, 4, 2)]:
        ev = eval_elements(p.dim, p.coords, p.conn, p.e_scale, p.material.as_dict(),
                           np.zeros(p.ndof), np.zeros(p.n_elems * p.ngp), want_K=False)
        assert np.all(np.isfinite(ev["fint"]))
        # element volumes from the Gauss rule sum to the body volume
        pts, w = gauss_points(p.dim)
        vol = 0.0
        for g in range(p.ngp):
            _, dN = shape_functions(p.dim, pts[g])
            J = np.einsum("ead,aj->edj", p.coords[p.conn], dN)
            d = np.linalg.det(J)
            assert np.all(d > 0)
            vol += (w[g] * d).sum()
        ext = np.prod(p.coords.max(0) - p.coords.min(0))
        assert vol == pytest.approx(ext, rel=1e-12)


# ----------------------------------------------------------------- patch tests (P5)

@pytest.mark.parametrize("dim,distort", [(2, 0.0), (2, 0.25), (3, 0.0), (3, 0.2)])
def test_patch_test_linear_field(dim, distort):
    p = tiny(dim, seed=5, distort=distort)
    rng = np.random.default_rng(1)
    A = rng.normal(0, 1e-5, (dim, dim))
    b = rng.normal(0, 1e-3, dim)
    x = np.zeros(p.ndof)
    u = p.coords @ A.T + b
    for i in range(dim):
        x[i::dim + 1] = u[:, i]
    eps_t = 0.5 * (A + A.T)
    if dim == 2:
        ev_ = np.array([eps_t[0, 0], eps_t[1, 1], 2 * eps_t[0, 1]])
    else:
        ev_ = np.array([eps_t[0, 0], eps_t[1, 1], eps_t[2, 2], 2 * eps_t[0, 1],
                        2 * eps_t[1, 2], 2 * eps_t[0, 2]])
    eeq, _ = equivalent_strain_voigt(dim, 0, p.material.k, p.material.nu, ev_)
    x[dim::dim + 1] = eeq                   # constant ebar equal to the constant eeq
    p.e_scale[:] = 1.0
    mat = p.material.as_dict()
    ev = eval_elements(dim, p.coords, p.conn, p.e_scale, mat, x, np.full(p.n_elems * p.ngp, 1.0))
    np.testing.assert_allclose(ev["eeq"], eeq, rtol=1e-10)
    f, _ = assemble(dim, p.conn, p.n_nodes, ev["fint"])
    lo = p.coords.min(0); hi = p.coords.max(0)
    interior = np.all((p.coords > lo + 1e-9) & (p.coords < hi - 1e-9), axis=1)
    fu = f.reshape(-1, dim + 1)
    scale = np.abs(fu[:, :dim]).max()
    assert scale > 0
    np.testing.assert_allclose(fu[interior, :dim], 0.0, atol=1e-11 * scale)
    np.testing.assert_allclose(fu[:, dim], 0.0, atol=1e-18)   # h(ebar - eeq) = 0, grad ebar = 0


# ----------------------------------------------------------------- null space (P6)

def rigid_modes(coords, dim):
    n = coords.shape[0]
    modes = []
    for i in range(dim):
        m = np.zeros((n, dim)); m[:, i] = 1.0; modes.append(m)
    if dim >= 2:
        pairs = [(0, 1)] if dim == 2 else [(0, 1), (1, 2), (0, 2)]
        for i, j in pairs:
            m = np.zeros((n, dim)); m[:, i] = -coords[:, j]; m[:, j] = coords[:, i]; modes.append(m)
    return modes


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_rigid_body_null_space(dim):
    p = tiny(dim, seed=2, distort=0.15 if dim > 1 else 0.0)
    x, kn = W.injected_state(p, seed=4)
    ev = eval_elements(dim, p.coords, p.conn, p.e_scale, p.material.as_dict(), x, kn)
    _, K = assemble(dim, p.conn, p.n_nodes, ev["fint"], ev["Ke"])
    K = K.toarray()
    nd = dim + 1
    iu = np.array([i for i in range(p.ndof) if i % nd != dim])
    ie = np.arange(dim, p.ndof, nd)
    for m in rigid_modes(p.coords, dim):
        v = m.ravel()
        kuu = K[np.ix_(iu, iu)]
        assert np.abs(kuu @ v).max() <= 1e-12 * np.abs(kuu).max() * np.abs(v).max()
        keu = K[np.ix_(ie, iu)]
        if dim == 1 or m[:, 0].std() == 0.0:
            # translations: the strain, hence eeq, does not change
            assert np.abs(keu @ v).max() <= 1e-12 * np.abs(keu).max() * np.abs(v).max()
    # gradient operator annihilates constants: set D' chi = 0 via kappa_n huge
    ev = eval_elements(dim, p.coords, p.conn, p.e_scale, dict(p.material.as_dict(), h=1.0), x,
                       np.full(p.n_elems * p.ngp, 1.0))
    _, K = assemble(dim, p.conn, p.n_nodes, ev["fint"], ev["Ke"])
    kee = K.toarray()[np.ix_(ie, ie)]
    # K_ee 1 = int h N (sum N) = int h N, which equals the lumped 'mass' h*vol per node
    ones = np.ones(len(ie))
    mass = np.zeros(p.n_nodes)
    pts, w = gauss_points(dim)
    th = p.material.thickness if dim < 3 else 1.0
    for e, nodes in enumerate(p.conn):
        for g in range(p.ngp):
            N, dN = shape_functions(dim, pts[g])
            J = p.coords[nodes].T @ dN
            mass[nodes] += w[g] * np.linalg.det(J) * N * th
    np.testing.assert_allclose(kee @ ones, mass, rtol=1e-12)


# ----------------------------------------------------------------- consistent tangent (P7)

def _fd_check(p, x, kn, rel=1e-6):
    mat = p.material.as_dict()
    ev = eval_elements(p.dim, p.coords, p.conn, p.e_scale, mat, x, kn)
    # keep every Gauss point away from both bands and the s = 0 kink
    assert np.all(np.abs(ev["ebar"] - kn.reshape(-1, p.ngp)) > 1e-7)
    assert np.all(np.abs(ev["kappa"] - p.material.kappa0) > 1e-7)
    Ke = ev["Ke"]
    nd = p.dim + 1
    nl = p.nen * nd
    dofs = (p.conn[:, :, None].astype(np.int64) * nd + np.arange(nd)).reshape(p.n_elems, nl)
    Kfd = np.zeros_like(Ke)
    for j in range(nl):
        is_e = (j % nd) == p.dim
        step = 1e-10 if is_e else 1e-8
        xp = x.copy(); xm = x.copy()
        # perturb the local dof j of every element at once is not possible
        # (shared nodes), so loop over elements by colour-free brute force
        for e in range(p.n_elems):
            d = dofs[e, j]
            xp[d] += step; xm[d] -= step
            fp = eval_elements(p.dim, p.coords, p.conn, p.e_scale, mat, xp, kn, elems=[e], want_K=False)["fint"][0]
            fm = eval_elements(p.dim, p.coords, p.conn, p.e_scale, mat, xm, kn, elems=[e], want_K=False)["fint"][0]
            Kfd[e, :, j] = (fp - fm) / (2 * step)
            xp[d] -= step; xm[d] += step
    iu = np.array([i for i in range(nl) if i % nd != p.dim])
    ie = np.arange(p.dim, nl, nd)
    for rows, cols, name in [(iu, iu, "uu"), (iu, ie, "ue"), (ie, iu, "eu"), (ie, ie, "ee")]:
        A = Ke[:, rows[:, None], cols[None, :]]
        B = Kfd[:, rows[:, None], cols[None, :]]
        scale = np.abs(A).max()
        assert scale > 0, name
        err = np.abs(A - B).max() / scale
        assert err < rel, (name, err)


@pytest.mark.parametrize("dim,plane", [(1, 0), (2, 0), (2, 1), (3, 0)])
def test_consistent_tangent_fd(dim, plane):
    p = tiny(dim, plane=plane, seed=3, distort=0.1 if dim > 1 else 0.0)
    for seed in (11, 12):
        x, kn = W.injected_state(p, seed=seed)
        _fd_check(p, x, kn)


# ----------------------------------------------------------------- symmetry (P9)

@pytest.mark.parametrize("dim", [2, 3])
def test_symmetry_without_history_update(dim):
    p = tiny(dim, seed=1, distort=0.1)
    x, _ = W.injected_state(p, seed=6)
    kn = np.full(p.n_elems * p.ngp, 1.0)          # chi = 0 everywhere
    ev = eval_elements(dim, p.coords, p.conn, p.e_scale, p.material.as_dict(), x, kn)
    Ke = ev["Ke"]
    nd = dim + 1
    nl = p.nen * nd
    iu = np.array([i for i in range(nl) if i % nd != dim])
    ie = np.arange(dim, nl, nd)
    kuu = Ke[:, iu[:, None], iu[None, :]]
    kee = Ke[:, ie[:, None], ie[None, :]]
    np.testing.assert_allclose(kuu, kuu.transpose(0, 2, 1), rtol=0, atol=1e-12 * np.abs(kuu).max())
    np.testing.assert_allclose(kee, kee.transpose(0, 2, 1), rtol=0, atol=1e-12 * np.abs(kee).max())
    np.testing.assert_array_equal(Ke[:, iu[:, None], ie[None, :]], 0.0)


# ----------------------------------------------------------------- two formulations agree

@pytest.mark.parametrize("dim,plane", [(1, 0), (2, 0), (2, 1), (3, 0)])
def test_index_form_loop_matches_vectorised(dim, plane):
    p = tiny(dim, plane=plane, seed=9, distort=0.15 if dim > 1 else 0.0)
    x, kn = W.injected_state(p, seed=21)
    mat = p.material.as_dict()
    ev = eval_elements(dim, p.coords, p.conn, p.e_scale, mat, x, kn)
    Kl, fl = element_loop_eval(dim, p.coords, p.conn.astype(np.int64), p.e_scale, mat, x, kn)
    nd = dim + 1
    nl = p.nen * nd
    iu = np.array([i for i in range(nl) if i % nd != dim])
    ie = np.arange(dim, nl, nd)
    for rows, cols in [(iu, iu), (iu, ie), (ie, iu), (ie, ie)]:
        A = ev["Ke"][:, rows[:, None], cols[None, :]]
        B = Kl[:, rows[:, None], cols[None, :]]
        assert np.abs(A - B).max() <= 1e-12 * max(np.abs(A).max(), 1e-300)
    for rows in (iu, ie):
        A = ev["fint"][:, rows]
        B = fl[:, rows]
        assert np.abs(A - B).max() <= 1e-12 * np.abs(A).max()


# ----------------------------------------------------------------- CSR pattern (P10)

@pytest.mark.parametrize("shape", [(5,), (4, 3), (3, 2, 2)])
def test_csr_pattern_bruteforce_and_count(shape):
    dim = len(shape)
    if dim == 1:
        p = W.bar1d(nx=shape[0], lx=float(shape[0]))
    elif dim == 2:
        p = W.sen2d(*shape, lx=float(shape[0]), ly=float(shape[1]), notch_len=1)
    else:
        p = W.beam3d(4, 2, 2) if shape == (4, 2, 2) else W.beam3d(*((shape[0] + 1) // 2 * 2,) + shape[1:])
    rp, ci = csr_pattern_bruteforce(p.conn, p.n_nodes, p.ndpn)
    rp2, ci2 = csr_pattern_unique(p.conn, p.n_nodes, p.ndpn)
    np.testing.assert_array_equal(rp, rp2)
    np.testing.assert_array_equal(ci, ci2)
    nnz = math.prod(3 * s + 1 for s in p.shape) * p.ndpn ** 2
    assert rp[-1] == nnz
    # the assembled matrix has exactly this pattern (structural zeros kept)
    x, kn = W.injected_state(p, 0)
    ev = eval_elements(p.dim, p.coords, p.conn, p.e_scale, p.material.as_dict(), x, kn)
    _, K = assemble(p.dim, p.conn, p.n_nodes, ev["fint"], ev["Ke"])
    np.testing.assert_array_equal(K.indptr, rp)
    np.testing.assert_array_equal(K.indices, ci)


def test_config_nnz_closed_form():
    for name, nnz in [("c0", 1204), ("c1", 1628109)]:
        p = W.config(name)
        rp, _ = csr_pattern_unique(p.conn, p.n_nodes, p.ndpn)
        assert rp[-1] == nnz


# ----------------------------------------------------------------- 1D closed forms (P4)

def test_bar_elastic_closed_form():
    p = W.config("c0")
    o = Oracle(p)
    E = p.material.E
    for n in range(1, 6):
        rep = o.solve_increment(tol=1e-12)
        assert rep["converged"] and rep["max_D"] == 0.0
        u_end = n / p.n_increments * 0.02
        # springs in series: 99 unit elements of E and one of 0.9 E (area 1)
        F = u_end / (99.0 / E + 1.0 / (0.9 * E))
        assert rep["reaction"] == pytest.approx(F, rel=1e-12)
        # nodal exactness of the piecewise-linear field
        u = o.x[0::2]
        xs = p.coords[:, 0]
        exact = np.where(xs <= 50, F / E * xs,
                         np.where(xs <= 51, F / E * 50 + F / (0.9 * E) * (xs - 50),
                                  F / E * 50 + F / (0.9 * E) + F / E * (xs - 51)))
        np.testing.assert_allclose(u, exact, rtol=1e-11, atol=1e-16)


def test_bar_homogeneous_ebar_equals_strain():
    p = W.bar1d(nx=20, lx=20.0, weak_elem=-1, u_end=0.001, n_increments=2)
    o = Oracle(p)
    rep = o.solve_increment(tol=1e-13)
    eps = 0.0005 / 20.0
    np.testing.assert_allclose(o.x[1::2], eps, rtol=1e-10)
    np.testing.assert_allclose(o.x[0::2], eps * p.coords[:, 0], rtol=1e-10, atol=1e-18)


# ----------------------------------------------------------------- h invariance (P8)

def test_h_invariance_1d_with_damage():
    # the ebar equation is h * [...] = 0 (reading R1), so fields do not depend on h
    p = W.bar1d(nx=40, lx=40.0, weak_elem=20, u_end=0.012, n_increments=30,
                material=W.base_material(beta=25.0))
    a = Oracle(p)
    b = Oracle(p, h_override=p.material.E * 1e-3)
    for _ in range(30):
        ra = a.solve_increment(tol=1e-12)
        rb = b.solve_increment(tol=1e-12)
        assert ra["converged"] and rb["converged"]
    assert a.D_n.max() > 0.3
    np.testing.assert_allclose(a.x, b.x, rtol=1e-7, atol=1e-12 * np.abs(a.x).max())
    np.testing.assert_allclose(a.D_n, b.D_n, atol=1e-7)


# ----------------------------------------------------------------- Newton (Eq. 11)

def test_newton_quadratic_convergence_near_onset():
    p = W.bar1d(nx=40, lx=40.0, weak_elem=20, u_end=0.012, n_increments=30,
                material=W.base_material(beta=25.0))
    o = Oracle(p)
    seen = False
    for _ in range(30):
        r = o.solve_increment(tol=1e-13)
        assert r["converged"]
        rel = [h["res_u"] / h["ref_u"] for h in r["history"]]
        if len(rel) >= 4 and rel[1] < 1e-2:
            # quadratic: each error is at most ~C * previous^2
            for a, b in zip(rel[1:-1], rel[2:]):
                # terminal phase (no more history flips): quadratic contraction
                if a < 1e-5 and b > 1e-15:
                    assert b < 1e3 * a * a + 1e-13
                    seen = True
    assert seen


def test_convergence_test_rejects_non_finite_norms():
    """Reading R9: an overflowed state (infinite internal force and
    residual) is not a converged one, although inf <= tol * inf holds."""
    inf, nan = float("inf"), float("nan")
    ok = dict(res_u=1e-12, res_e=1e-14, ref_u=1.0, ref_e=1e-3)
    assert Oracle.converged(ok, 1e-8)
    for key, val in (("res_u", inf), ("ref_u", inf), ("res_e", nan), ("ref_e", inf)):
        bad = dict(ok, **{key: val})
        assert not Oracle.converged(bad, 1e-8), key
    assert not Oracle.converged(dict(res_u=inf, res_e=inf, ref_u=inf, ref_e=inf), 1e-8)
