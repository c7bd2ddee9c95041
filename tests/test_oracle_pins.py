"""Pins of the oracle's constitutive functions (Appendix A) to facts other
than the oracle itself: special cases that reduce to a known law, limits,
invariances, and finite differences.  CPU only."""
import math

import numpy as np
import pytest

from oracle.lgdm import (damage, history, interaction, equivalent_strain_tensor,
                         equivalent_strain_voigt, elasticity_matrix, mvm_coefficients)

K0 = 1e-4


# --------------------------------------------------------------------- Eq. A.1

def test_damage_zero_up_to_threshold():
    k = np.array([0.0, 0.5e-4, 1e-4, 1e-4 + 0.5e-10])
    D, dD = damage(k, K0, 0.99, 300.0, tol_dmg=1e-10)
    assert np.all(D == 0.0) and np.all(dD == 0.0)


@pytest.mark.parametrize("beta", [25.0, 300.0])
def test_damage_alpha0_is_stress_plateau(beta):
    # alpha = 0: 1D stress (1 - D) E kappa stays at E kappa0 once damage starts
    k = np.linspace(1.01e-4, 5e-3, 50)
    D, _ = damage(k, K0, 0.0, beta, tol_dmg=0.0)
    np.testing.assert_allclose((1.0 - D) * k, K0, rtol=1e-13)


@pytest.mark.parametrize("beta", [25.0, 300.0])
def test_damage_alpha1_is_exponential_softening(beta):
    # alpha = 1: stress decays as exp(-beta (kappa - kappa0)) from its peak E kappa0
    k = np.linspace(1.01e-4, 5e-3, 50)
    D, _ = damage(k, K0, 1.0, beta, tol_dmg=0.0)
    np.testing.assert_allclose((1.0 - D) * k / K0, np.exp(-beta * (k - K0)), rtol=1e-12)


def test_damage_affine_in_alpha_and_limits():
    k = np.linspace(1.01e-4, 2e-2, 40)
    D0, _ = damage(k, K0, 0.0, 300.0, 0.0)
    D1, _ = damage(k, K0, 1.0, 300.0, 0.0)
    for a in (0.3, 0.99):
        Da, _ = damage(k, K0, a, 300.0, 0.0)
        np.testing.assert_allclose(Da, (1 - a) * D0 + a * D1, rtol=1e-13, atol=1e-15)
    # continuous at the threshold, increasing, and D -> 1 for kappa -> inf
    Dth, _ = damage(np.array([K0 * (1 + 1e-12)]), K0, 0.99, 300.0, 0.0)
    assert abs(Dth[0]) < 1e-9
    Da, _ = damage(k, K0, 0.99, 300.0, 0.0)
    assert np.all(np.diff(Da) > 0)
    Dinf, _ = damage(np.array([1e6]), K0, 0.99, 300.0, 0.0)
    assert 1.0 - Dinf[0] < 1e-9


def test_damage_derivative_fd():
    k = np.linspace(1.05e-4, 3e-3, 30)
    for a, b in [(0.99, 300.0), (0.5, 25.0)]:
        _, dD = damage(k, K0, a, b, 0.0)
        s = 1e-9
        Dp, _ = damage(k + s, K0, a, b, 0.0)
        Dm, _ = damage(k - s, K0, a, b, 0.0)
        np.testing.assert_allclose(dD, (Dp - Dm) / (2 * s), rtol=1e-6)


# --------------------------------------------------------------------- Eq. A.2

def test_history_is_running_max():
    rng = np.random.default_rng(3)
    seq = np.cumsum(rng.normal(0, 1e-5, (40, 7)), axis=0) + 2e-4
    kn = np.zeros(7)
    for t in range(40):
        kn, chi = history(seq[t], kn, tol_hist=0.0)
        np.testing.assert_array_equal(kn, np.max(np.vstack([np.zeros((1, 7)), seq[:t + 1]]), axis=0))
    # band: an increase of less than tol_hist keeps the old value
    k, chi = history(np.array([1.0 + 5e-11, 1.0 + 2e-10]), np.array([1.0, 1.0]), tol_hist=1e-10)
    np.testing.assert_array_equal(k, [1.0, 1.0 + 2e-10])
    np.testing.assert_array_equal(chi, [0.0, 1.0])


# --------------------------------------------------------------------- Eq. A.4

def test_interaction_end_values_and_limits():
    for R, n in [(0.05, 5.0), (0.005, 5.0), (0.3, 2.0)]:
        g, _ = interaction(np.array([0.0, 1.0]), R, n)
        np.testing.assert_allclose(g, [1.0, R], rtol=1e-14)
        D = np.linspace(0, 1, 21)
        g, dg = interaction(D, R, n)
        assert np.all(np.diff(g) < 0)
    # R = 1: no interaction decay at all
    g, dg = interaction(np.linspace(0, 1, 11), 1.0, 5.0)
    np.testing.assert_allclose(g, 1.0, rtol=1e-14)
    np.testing.assert_allclose(dg, 0.0, atol=1e-14)
    # eta -> 0: linear decay from 1 to R
    D = np.linspace(0, 1, 11)
    g, _ = interaction(D, 0.05, 1e-7)
    np.testing.assert_allclose(g, 1 - 0.95 * D, atol=1e-6)


def test_interaction_derivative_fd():
    D = np.linspace(0.01, 0.99, 25)
    g, dg = interaction(D, 0.05, 5.0)
    s = 1e-7
    gp, _ = interaction(D + s, 0.05, 5.0)
    gm, _ = interaction(D - s, 0.05, 5.0)
    np.testing.assert_allclose(dg, (gp - gm) / (2 * s), rtol=1e-7)


# --------------------------------------------------------------------- Eq. A.3

def _uniaxial_stress_tensor(e, nu):
    return np.diag([e, -nu * e, -nu * e])


@pytest.mark.parametrize("k,nu", [(10.0, 0.2), (1.0, 0.3), (3.0, 0.0), (20.0, 0.45)])
def test_eqstrain_uniaxial_tension_compression(k, nu):
    # k is the compressive/tensile strength ratio: uniaxial tension gives
    # eeq = eps, uniaxial compression eeq = |eps| / k
    for e in (1e-4, 3.7e-3):
        eq, _ = equivalent_strain_tensor(_uniaxial_stress_tensor(e, nu), k, nu)
        assert eq == pytest.approx(e, rel=1e-12)
        eq, _ = equivalent_strain_tensor(_uniaxial_stress_tensor(-e, nu), k, nu)
        assert eq == pytest.approx(e / k, rel=1e-11)
    # the same state through the plane-stress Voigt path (eps_zz from nu)
    e = 2e-4
    eq, _ = equivalent_strain_voigt(2, 0, k, nu, np.array([e, -nu * e, 0.0]))
    assert eq == pytest.approx(e, rel=1e-12)
    eq, _ = equivalent_strain_voigt(2, 0, k, nu, np.array([-nu * e, e, 0.0]))
    assert eq == pytest.approx(e, rel=1e-12)


def test_eqstrain_invariance_homogeneity_nonneg():
    rng = np.random.default_rng(7)
    for _ in range(20):
        A = rng.normal(0, 1e-3, (3, 3))
        eps = 0.5 * (A + A.T)
        Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        e1, _ = equivalent_strain_tensor(eps, 10.0, 0.2)
        e2, _ = equivalent_strain_tensor(Q @ eps @ Q.T, 10.0, 0.2)
        e3, _ = equivalent_strain_tensor(2.5 * eps, 10.0, 0.2)
        assert e2 == pytest.approx(e1, rel=1e-11)
        assert e3 == pytest.approx(2.5 * e1, rel=1e-12)
        assert e1 >= 0.0


def test_eqstrain_pure_shear_k1():
    # k = 1: eeq = sqrt(3 J2)/(1+nu); pure engineering shear gamma has
    # J2 = gamma^2 / 4, so eeq = sqrt(3) |gamma| / (2 (1 + nu))
    nu = 0.25
    for gam in (1e-4, -3e-3):
        eq, _ = equivalent_strain_voigt(3, 0, 1.0, nu, np.array([0, 0, 0, gam, 0, 0.0]))
        assert eq == pytest.approx(math.sqrt(3.0) * abs(gam) / (2 * (1 + nu)), rel=1e-12)


@pytest.mark.parametrize("dim,plane", [(2, 0), (2, 1), (3, 0)])
def test_eqstrain_gradient_fd(dim, plane):
    rng = np.random.default_rng(11 + dim + plane)
    nstr = 3 if dim == 2 else 6
    for _ in range(10):
        ev = rng.normal(0, 1e-3, nstr)
        eq, n = equivalent_strain_voigt(dim, plane, 10.0, 0.2, ev)
        fd = np.zeros(nstr)
        for i in range(nstr):
            s = 1e-9
            ep = ev.copy(); ep[i] += s
            em = ev.copy(); em[i] -= s
            fd[i] = (equivalent_strain_voigt(dim, plane, 10.0, 0.2, ep)[0]
                     - equivalent_strain_voigt(dim, plane, 10.0, 0.2, em)[0]) / (2 * s)
        np.testing.assert_allclose(n, fd, rtol=1e-6, atol=1e-9)


def test_eqstrain_zero_strain_subgradient():
    c1, _, _ = mvm_coefficients(10.0, 0.2)
    eq, n = equivalent_strain_voigt(3, 0, 10.0, 0.2, np.zeros(6))
    assert eq == 0.0
    np.testing.assert_allclose(n, [c1, c1, c1, 0, 0, 0])
    # plane stress: dI1/deps_xx = 1 - nu/(1-nu)
    eq, n = equivalent_strain_voigt(2, 0, 10.0, 0.2, np.zeros(3))
    np.testing.assert_allclose(n, [c1 * (1 - 0.25), c1 * (1 - 0.25), 0.0])


def test_eqstrain_1d_is_strain():
    eq, n = equivalent_strain_voigt(1, 0, 10.0, 0.2, np.array([[3e-4], [1e-5]]))
    np.testing.assert_array_equal(eq, [3e-4, 1e-5])
    np.testing.assert_array_equal(n, [[1.0], [1.0]])


# --------------------------------------------------------------------- elasticity

@pytest.mark.parametrize("dim,plane", [(2, 0), (3, 0)])
def test_elasticity_uniaxial_stress(dim, plane):
    E, nu = 2e4, 0.2
    C = elasticity_matrix(dim, plane, E, nu)
    e = 1e-3
    if dim == 2:
        s = C @ np.array([e, -nu * e, 0.0])
        np.testing.assert_allclose(s, [E * e, 0, 0], atol=1e-12)
        s = C @ np.array([0, 0, 1e-3])
        assert s[2] == pytest.approx(E / (2 * (1 + nu)) * 1e-3)
    else:
        s = C @ np.array([e, -nu * e, -nu * e, 0, 0, 0])
        np.testing.assert_allclose(s, [E * e, 0, 0, 0, 0, 0], atol=1e-12)
        s = C @ np.array([0, 0, 0, 0, 1e-3, 0])
        assert s[4] == pytest.approx(E / (2 * (1 + nu)) * 1e-3)


def test_elasticity_plane_strain_has_no_out_of_plane_strain_energy_shortcut():
    # plane strain equals the 3D law restricted to in-plane strains
    E, nu = 3e4, 0.3
    C2 = elasticity_matrix(2, 1, E, nu)
    C3 = elasticity_matrix(3, 0, E, nu)
    np.testing.assert_allclose(C2[:2, :2], C3[:2, :2])
    assert C2[2, 2] == pytest.approx(C3[3, 3])
