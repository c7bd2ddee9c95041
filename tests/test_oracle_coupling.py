"""Pins of the oracle's coupling variant (the stress of Eq. 2 with its h
term, Eq. 11b as printed, K^uu completed by the linearisation of Eq. 2)
against facts that do not come from the oracle's own formulas: finite
differences of the equivalent-strain gradient (its second derivative), the
gradient of the free energy of Eq. 1 (the stress, by the Coleman-Noll
relation that gives Eq. 2), finite differences of the residual (the whole
tangent), and the closed-form elastic bar.  CPU only."""
import dataclasses

import numpy as np
import pytest

import lgdm_workloads as W
from oracle.lgdm import (Oracle, eval_elements, equivalent_strain_voigt,
                         equivalent_strain_hessian_voigt, elasticity_matrix, gauss_points,
                         shape_functions, strain_displacement, damage, history)
from test_oracle_fe import tiny, _fd_check


def coupled(p, h_over_E=0.3):
    """The problem with the Eq. 2 coupling and a coupling modulus large
    enough that its terms are visible next to (1 - D) C."""
    p.material = dataclasses.replace(p.material, coupling=1, h=h_over_E * p.material.E)
    return p


@pytest.mark.parametrize("dim,plane", [(2, 0), (2, 1), (3, 0)])
def test_hessian_is_fd_of_gradient(dim, plane):
    rng = np.random.default_rng(7)
    nstr = 3 if dim == 2 else 6
    k, nu, kappa0 = 10.0, 0.2, 1e-4
    for _ in range(20):
        ev = rng.normal(0.0, 3e-4, nstr)
        H = equivalent_strain_hessian_voigt(dim, plane, k, nu, ev, kappa0)
        Hfd = np.zeros((nstr, nstr))
        for j in range(nstr):
            st = 1e-9
            e1 = ev.copy(); e1[j] += st
            e0 = ev.copy(); e0[j] -= st
            Hfd[:, j] = (equivalent_strain_voigt(dim, plane, k, nu, e1)[1]
                         - equivalent_strain_voigt(dim, plane, k, nu, e0)[1]) / (2 * st)
        assert np.abs(H - Hfd).max() <= 1e-6 * np.abs(H).max()
        np.testing.assert_allclose(H, H.T, rtol=0, atol=1e-12 * np.abs(H).max())


def test_hessian_zero_in_1d_and_at_the_cone_point():
    assert not np.any(equivalent_strain_hessian_voigt(1, 0, 10.0, 0.2, np.array([3e-4]), 1e-4))
    for dim, nstr in ((2, 3), (3, 6)):
        assert not np.any(equivalent_strain_hessian_voigt(dim, 0, 10.0, 0.2, np.zeros(nstr), 1e-4))


def _element_energy(p, x, kn, e):
    """Stored energy of element e by Eq. 1 at the damage of its Gauss points:
    sum_g w detJ [1/2 (1-D) s_e eps.C.eps + 1/2 h (eeq - ebar)^2 + 1/2 g h c |grad ebar|^2]
    (the last term does not depend on u)."""
    m = p.material
    nd = p.dim + 1
    cn = p.conn[e].astype(np.int64)
    xe = p.coords[cn]
    ue = np.stack([x[cn * nd + i] for i in range(p.dim)], axis=1).reshape(-1)
    ee = x[cn * nd + p.dim]
    C = elasticity_matrix(p.dim, m.plane, m.E, m.nu)
    pts, w = gauss_points(p.dim)
    th = m.thickness if p.dim < 3 else 1.0
    tot = 0.0
    for g in range(p.ngp):
        N, dNdxi = shape_functions(p.dim, pts[g])
        J = xe.T @ dNdxi
        dNdx = dNdxi @ np.linalg.inv(J)
        B = strain_displacement(dNdx[None])[0]
        eps = B @ ue
        eeq, _ = equivalent_strain_voigt(p.dim, m.plane, m.k, m.nu, eps[None])
        eb = N @ ee
        kap, _ = history(np.array([eb]), np.array([kn[e * p.ngp + g]]), m.tol_hist)
        D, _ = damage(kap, m.kappa0, m.alpha, m.beta, m.tol_dmg)
        tot += w[g] * np.linalg.det(J) * th * (0.5 * (1 - D[0]) * p.e_scale[e] * eps @ C @ eps
                                              + 0.5 * m.h * (eeq[0] - eb) ** 2)
    return tot


@pytest.mark.parametrize("dim,plane", [(1, 0), (2, 0), (2, 1), (3, 0)])
def test_coupled_stress_is_gradient_of_free_energy(dim, plane):
    """F^u of the variant is d/du of the element energy of Eq. 1 (Eq. 2 by
    Coleman-Noll; D held at its Gauss-point values, which depend on ebar only)."""
    p = coupled(tiny(dim, plane=plane, seed=4, distort=0.1 if dim > 1 else 0.0))
    x, kn = W.injected_state(p, seed=21)
    mat = p.material.as_dict()
    nd = p.dim + 1
    for e in (0, p.n_elems - 1):
        f = eval_elements(p.dim, p.coords, p.conn, p.e_scale, mat, x, kn, elems=[e], want_K=False)["fint"][0]
        cn = p.conn[e].astype(np.int64)
        for a in range(p.nen):
            for i in range(p.dim):
                d = cn[a] * nd + i
                st = 1e-8
                xp = x.copy(); xp[d] += st
                xm = x.copy(); xm[d] -= st
                fd = (_element_energy(p, xp, kn, e) - _element_energy(p, xm, kn, e)) / (2 * st)
                assert fd == pytest.approx(f[a * nd + i], rel=1e-6, abs=1e-9 * np.abs(f).max())


@pytest.mark.parametrize("dim,plane", [(1, 0), (2, 0), (2, 1), (3, 0)])
def test_coupled_tangent_fd(dim, plane):
    p = coupled(tiny(dim, plane=plane, seed=3, distort=0.1 if dim > 1 else 0.0))
    for seed in (11, 12):
        x, kn = W.injected_state(p, seed=seed)
        _fd_check(p, x, kn)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_coupling_terms_present_and_vanish_with_h(dim):
    p = tiny(dim, seed=3, distort=0.1 if dim > 1 else 0.0)
    x, kn = W.injected_state(p, seed=11)
    base = p.material.as_dict()
    ex = eval_elements(p.dim, p.coords, p.conn, p.e_scale, dict(base, h=0.3 * base["E"]), x, kn)
    cp = eval_elements(p.dim, p.coords, p.conn, p.e_scale, dict(base, h=0.3 * base["E"], coupling=1), x, kn)
    assert np.abs(cp["Ke"] - ex["Ke"]).max() > 1e-3 * np.abs(ex["Ke"]).max()
    z0 = eval_elements(p.dim, p.coords, p.conn, p.e_scale, dict(base, h=0.0), x, kn)
    z1 = eval_elements(p.dim, p.coords, p.conn, p.e_scale, dict(base, h=0.0, coupling=1), x, kn)
    np.testing.assert_array_equal(z0["fint"], z1["fint"])
    np.testing.assert_array_equal(z0["Ke"], z1["Ke"])


def test_coupled_bar_elastic_closed_form():
    """A homogeneous bar below the damage threshold: ebar = eps, so the h
    term of Eq. 2 vanishes and u is linear, u(x) = u_end x / L."""
    mat = dataclasses.replace(W.base_material(), coupling=1, h=0.3 * 2.0e4)
    p = W.bar1d(nx=8, lx=8.0, u_end=4e-4, weak_elem=-1, n_increments=1, material=mat)
    o = Oracle(p)
    rep = o.solve_increment(1.0, tol=1e-12)
    assert rep["converged"]
    u = o.x[0::2]
    np.testing.assert_allclose(u, 4e-4 * p.coords[:, 0] / 8.0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(o.x[1::2], 4e-4 / 8.0, rtol=1e-10)
