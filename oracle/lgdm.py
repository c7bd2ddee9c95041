"""LGDM oracle: the discrete Newton iteration of Eq. 11 in plain FP64 NumPy/SciPy.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the product
path may import this module.

What it computes
----------------
One Newton iteration of the coupled displacement / micro-equivalent-strain
problem (Sec. 2.1): evaluate every Gauss point (Eqs. A.1-A.4), form the
element tangent blocks (Eqs. 11a-d) and internal forces (Eqs. 11e-f),
assemble them into a global sparse tangent and residual (Fig. 2 assembly by
summing duplicate triplets), solve (Eq. 11; a sparse direct LU stands in for
the direct solve the paper uses), update the primary fields (Algorithm 2,
step "Update Primary Var") and, at convergence, commit the history variable
(Eq. A.2).  It is vectorised over (element, Gauss point) like Algorithm 2;
`element_loop_eval` is an element-by-element variant with the structure of
Algorithm 1 used to cross-check it on tiny meshes.

Readings (where the paper is silent, ambiguous or garbled)
----------------------------------------------------------
R1  u-equation stress.  The executed code of Fig. 2 forms the u residual as
    -k_uu * u and passes no h to Build_kue, so sigma = (1 - D) C : eps and
    K^{u ebar} = -int B_u^T (C eps dD/dkappa dkappa/debar) N (Eq. 11b without
    its h term).  Eqs. 11a, 11c, 11d are kept as printed.
R2  Sign of the gradient term of Eq. 11f: the residual is
    F^ebar = int N h (eeq - ebar) - int B^T g h c grad(ebar), the sign for
    which Eq. 11d (positive B^T g h c B) is its derivative.
R3  Eq. 11d's dg/dkappa is chained through kappa(ebar):
    dg/debar = g'(D) D'(kappa) chi N, chi = 1 where the history was updated.
R4  Eq. A.3's J2 coefficient is read as 12k/(1+nu)^2 with J2 = dev(eps):dev(eps)/2
    (the coefficient for which uniaxial tension gives eeq = eps and uniaxial
    compression eeq = |eps|/k, as the definition of k requires).
R5  2D plane stress uses the full 3D strain tensor with
    eps_zz = -nu/(1-nu)(eps_xx + eps_yy); plane strain uses eps_zz = 0; 1D uses
    eeq = eps (the uniaxial-stress value of A.3 in tension).
R6  Where the square-root argument of A.3 is zero, deeq/deps is taken as its
    minimum-norm subgradient c1 dI1/deps.
R7  History and damage use the condition vectors of Fig. 8b with bands
    tol_hist and tol_dmg (1e-10): chi = (ebar - kappa_n) > tol_hist,
    D = D' = 0 where (kappa - kappa0) < tol_dmg.  kappa_n starts at 0.
R8  Dirichlet dofs: u_c = lambda * u_ref at the start of each increment;
    assembled rows and columns of constrained dofs become identity, their
    residual entries zero.  No Dirichlet condition on ebar (zeta = 0, Eq. 8).
R9  Convergence: ||R_u|| <= tol max(||f_int,u||, tiny) and
    ||R_ebar|| <= tol max(||int N h eeq||, tiny), per field.
R10 Equal-order elements (line2 / quad4 / hex8) for u and ebar; full 2-point
    Gauss-Legendre per direction, Gauss point g = i_xi + 2 i_eta + 4 i_zeta.
R11 The element stiffness scale multiplies C only (not h, not c).
R12 D, kappa, g and their derivatives are evaluated at the current iterate
    from the committed kappa_n; kappa_n is committed only at convergence.
R13 Coupling variant (material coupling = 1): the stress of Eq. 2,
    sigma = (1 - D) C : eps + h (eeq - ebar) d eeq/d eps, the derivative of
    the free energy of Eq. 1, in place of R1.  K^{u ebar} is Eq. 11b as
    printed (with its -h d eeq/d eps N term), and K^uu is Eq. 11a completed
    by the consistent linearisation of Eq. 2:
    + int B^T h [n n^T + (eeq - ebar) d^2 eeq/d eps^2] B, n = d eeq/d eps.
    The second derivative of A.3 is dropped where sqrt(s) <= 1e-6 kappa0
    (s the square-root argument; the cone point of A.3, cf. R6).  Eqs. 11c,
    11d, 11f are unchanged.
"""
from __future__ import annotations

import math
from typing import Dict, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

__all__ = [
    "reference_nodes", "gauss_points", "shape_functions", "damage", "history",
    "interaction", "mvm_coefficients", "equivalent_strain_tensor",
    "equivalent_strain_voigt", "elasticity_matrix", "strain_displacement",
    "eval_elements", "element_loop_eval", "csr_pattern_bruteforce",
    "csr_pattern_unique", "assemble", "apply_dirichlet", "Oracle",
]

# ---------------------------------------------------------------------------
# reference element and quadrature (shape functions N, B of Eqs. 9-11)
# ---------------------------------------------------------------------------


def reference_nodes(dim: int) -> np.ndarray:
    """Reference coordinates of the element nodes in the local node order
    line2 (x0, x1); quad4 counter-clockwise; hex8 bottom face then top face."""
    if dim == 1:
        return np.array([[-1.0], [1.0]])
    if dim == 2:
        return np.array([[-1.0, -1.0], [1.0, -1.0], [1.0, 1.0], [-1.0, 1.0]])
    if dim == 3:
        q = np.array([[-1.0, -1.0], [1.0, -1.0], [1.0, 1.0], [-1.0, 1.0]])
        return np.vstack([np.hstack([q, -np.ones((4, 1))]), np.hstack([q, np.ones((4, 1))])])
    raise ValueError(dim)


def gauss_points(dim: int):
    """2-point Gauss-Legendre per direction (reading R10): points and weights."""
    a = 1.0 / math.sqrt(3.0)
    pts = []
    for g in range(2 ** dim):
        pts.append([(-a, a)[(g >> d) & 1] for d in range(dim)])
    return np.array(pts), np.ones(2 ** dim)


def shape_functions(dim: int, xi: np.ndarray):
    """Multilinear Lagrange shape functions at one reference point.

    N_a = prod_k (1 + xi_a,k xi_k) / 2; returns N [nen], dN/dxi [nen, dim]."""
    nodes = reference_nodes(dim)
    fac = (1.0 + nodes * xi[None, :]) / 2.0          # [nen, dim]
    N = np.prod(fac, axis=1)
    dN = np.zeros_like(nodes)
    for j in range(dim):
        others = np.prod(np.delete(fac, j, axis=1), axis=1) if dim > 1 else np.ones(len(nodes))
        dN[:, j] = nodes[:, j] / 2.0 * others
    return N, dN


# ---------------------------------------------------------------------------
# constitutive functions (Appendix A)
# ---------------------------------------------------------------------------


def damage(kappa, kappa0, alpha, beta, tol_dmg=1e-10):
    """Damage law, Eq. A.1, with the band of the vectorised update (Fig. 8b,
    reading R7): D = 0 where kappa - kappa0 < tol_dmg, otherwise
    D = 1 - (kappa0/kappa)(1 - alpha + alpha exp(-beta (kappa - kappa0))).
    Returns D and dD/dkappa."""
    kappa = np.asarray(kappa, dtype=np.float64)
    below = (kappa - kappa0) < tol_dmg
    ks = np.where(below, 1.0, kappa)
    ex = np.exp(-beta * (ks - kappa0))
    bracket = 1.0 - alpha + alpha * ex
    D = 1.0 - (kappa0 / ks) * bracket
    dD = (kappa0 / ks ** 2) * bracket + (kappa0 / ks) * alpha * beta * ex
    return np.where(below, 0.0, D), np.where(below, 0.0, dD)


def history(ebar, kappa_n, tol_hist=1e-10):
    """History variable, Eq. A.2 as updated in Fig. 8b (reading R7):
    kappa = ebar where ebar - kappa_n > tol_hist (chi = 1), else kappa_n (chi = 0)."""
    ebar = np.asarray(ebar, dtype=np.float64)
    chi = (ebar - kappa_n) > tol_hist
    return np.where(chi, ebar, kappa_n), chi.astype(np.float64)


def interaction(D, R, eta):
    """Interaction function g(D), Eq. A.4, and dg/dD."""
    D = np.asarray(D, dtype=np.float64)
    den = 1.0 - math.exp(-eta)
    e = np.exp(-eta * D)
    g = ((1.0 - R) * e + R - math.exp(-eta)) / den
    dg = -eta * (1.0 - R) * e / den
    return g, dg


def mvm_coefficients(k, nu):
    """Coefficients of the modified von Mises equivalent strain, Eq. A.3
    (reading R4): eeq = c1 I1 + sqrt(c2^2 I1^2 + c3 J2) / (2k)."""
    c1 = (k - 1.0) / (2.0 * k * (1.0 - 2.0 * nu))
    c2 = (k - 1.0) / (1.0 - 2.0 * nu)
    c3 = 12.0 * k / (1.0 + nu) ** 2
    return c1, c2, c3


def equivalent_strain_tensor(eps, k, nu):
    """Eq. A.3 on a full symmetric strain tensor eps [..., 3, 3].

    I1 = tr eps, J2 = dev(eps):dev(eps)/2.  Returns eeq [...] and the tensor
    gradient G [..., 3, 3] with d eeq = G : d eps (reading R6 where the
    square-root argument vanishes)."""
    c1, c2, c3 = mvm_coefficients(k, nu)
    eps = np.asarray(eps, dtype=np.float64)
    eye = np.eye(3)
    I1 = np.trace(eps, axis1=-2, axis2=-1)
    dev = eps - I1[..., None, None] / 3.0 * eye
    J2 = 0.5 * np.sum(dev * dev, axis=(-2, -1))
    s = c2 * c2 * I1 * I1 + c3 * J2
    pos = s > 0.0
    sq = np.sqrt(np.where(pos, s, 0.0))
    eeq = c1 * I1 + sq / (2.0 * k)
    inv = np.where(pos, 1.0 / np.where(pos, sq, 1.0), 0.0)
    G = c1 * eye + (inv / (4.0 * k))[..., None, None] * (
        2.0 * c2 * c2 * I1[..., None, None] * eye + c3 * dev)
    return eeq, G


def _voigt_to_tensor(dim, plane, nu, ev):
    """Voigt strain (engineering shears) to the 3x3 tensor used by A.3 (R5).
    2D order [xx, yy, xy]; 3D order [xx, yy, zz, xy, yz, xz]."""
    shp = ev.shape[:-1]
    t = np.zeros(shp + (3, 3))
    if dim == 2:
        t[..., 0, 0] = ev[..., 0]
        t[..., 1, 1] = ev[..., 1]
        t[..., 0, 1] = t[..., 1, 0] = 0.5 * ev[..., 2]
        if plane == 0:
            t[..., 2, 2] = -nu / (1.0 - nu) * (ev[..., 0] + ev[..., 1])
    else:
        t[..., 0, 0] = ev[..., 0]
        t[..., 1, 1] = ev[..., 1]
        t[..., 2, 2] = ev[..., 2]
        t[..., 0, 1] = t[..., 1, 0] = 0.5 * ev[..., 3]
        t[..., 1, 2] = t[..., 2, 1] = 0.5 * ev[..., 4]
        t[..., 0, 2] = t[..., 2, 0] = 0.5 * ev[..., 5]
    return t


def equivalent_strain_voigt(dim, plane, k, nu, ev):
    """eeq and n = d eeq / d eps_voigt for a Voigt strain [..., nstr] (R5)."""
    ev = np.asarray(ev, dtype=np.float64)
    if dim == 1:
        return ev[..., 0].copy(), np.ones_like(ev)
    t = _voigt_to_tensor(dim, plane, nu, ev)
    eeq, G = equivalent_strain_tensor(t, k, nu)
    if dim == 2:
        n = np.zeros(ev.shape)
        a = -nu / (1.0 - nu) if plane == 0 else 0.0
        n[..., 0] = G[..., 0, 0] + a * G[..., 2, 2]
        n[..., 1] = G[..., 1, 1] + a * G[..., 2, 2]
        n[..., 2] = G[..., 0, 1]
    else:
        n = np.stack([G[..., 0, 0], G[..., 1, 1], G[..., 2, 2],
                      G[..., 0, 1], G[..., 1, 2], G[..., 0, 2]], axis=-1)
    return eeq, n


def equivalent_strain_hessian_voigt(dim, plane, k, nu, ev, kappa0):
    """d^2 eeq / d eps_voigt^2 [..., nstr, nstr] for the coupling variant (R13).

    On the 3D tensor (R5), with s = c2^2 I1^2 + c3 J2 and q = ds/deps =
    2 c2^2 I1 1 + c3 dev(eps):
        d^2 eeq = (1 / (4 k sqrt(s))) (2 c2^2 1 (x) 1 + c3 P_dev)
                  - (1 / (8 k s^(3/2))) q (x) q,
    P_dev the deviatoric projector.  The Voigt form contracts it with the
    tensor of each unit Voigt strain (the linear map of R5, which carries the
    plane-stress eps_zz).  Zero where sqrt(s) <= 1e-6 kappa0, and in 1D
    (eeq = eps is linear)."""
    ev = np.asarray(ev, dtype=np.float64)
    nstr = ev.shape[-1]
    if dim == 1:
        return np.zeros(ev.shape + (nstr,))
    c1, c2, c3 = mvm_coefficients(k, nu)
    eye = np.eye(3)
    t = _voigt_to_tensor(dim, plane, nu, ev)
    I1 = np.trace(t, axis1=-2, axis2=-1)
    dev = t - I1[..., None, None] / 3.0 * eye
    s = c2 * c2 * I1 * I1 + c3 * 0.5 * np.sum(dev * dev, axis=(-2, -1))
    sq = np.sqrt(np.maximum(s, 0.0))
    on = sq > 1e-6 * kappa0
    sqs = np.where(on, sq, 1.0)
    al = np.where(on, 1.0 / (4.0 * k * sqs), 0.0)
    be = np.where(on, 1.0 / (8.0 * k * sqs ** 3), 0.0)
    q = 2.0 * c2 * c2 * I1[..., None, None] * eye + c3 * dev
    T = _voigt_to_tensor(dim, plane, nu, np.eye(nstr))          # [nstr, 3, 3] tensor of each unit strain
    trT = np.trace(T, axis1=-2, axis2=-1)                       # [nstr]
    devT = T - trT[:, None, None] / 3.0 * eye
    dd = np.einsum("aij,bij->ab", devT, devT)                   # dev T_a : dev T_b
    qT = np.einsum("...ij,aij->...a", q, T)                     # q : T_a
    H = (al[..., None, None] * (2.0 * c2 * c2 * np.outer(trT, trT) + c3 * dd)
         - be[..., None, None] * qT[..., :, None] * qT[..., None, :])
    return H


def elasticity_matrix(dim, plane, E, nu):
    """Elasticity matrix C in Voigt form (engineering shears)."""
    if dim == 1:
        return np.array([[E]])
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    if dim == 2:
        if plane == 0:
            f = E / (1.0 - nu * nu)
            return f * np.array([[1.0, nu, 0.0], [nu, 1.0, 0.0], [0.0, 0.0, (1.0 - nu) / 2.0]])
        return np.array([[lam + 2 * mu, lam, 0.0], [lam, lam + 2 * mu, 0.0], [0.0, 0.0, mu]])
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[0, 0] = C[1, 1] = C[2, 2] = lam + 2 * mu
    C[3, 3] = C[4, 4] = C[5, 5] = mu
    return C


def strain_displacement(dNdx):
    """B_u for Voigt strain from shape-function gradients dNdx [..., nen, dim].
    Columns are node-major: a * dim + i."""
    dim = dNdx.shape[-1]
    nen = dNdx.shape[-2]
    shp = dNdx.shape[:-2]
    nstr = {1: 1, 2: 3, 3: 6}[dim]
    B = np.zeros(shp + (nstr, nen * dim))
    for a in range(nen):
        dx = dNdx[..., a, 0]
        if dim == 1:
            B[..., 0, a] = dx
            continue
        dy = dNdx[..., a, 1]
        if dim == 2:
            B[..., 0, 2 * a] = dx
            B[..., 1, 2 * a + 1] = dy
            B[..., 2, 2 * a] = dy
            B[..., 2, 2 * a + 1] = dx
            continue
        dz = dNdx[..., a, 2]
        c = 3 * a
        B[..., 0, c] = dx
        B[..., 1, c + 1] = dy
        B[..., 2, c + 2] = dz
        B[..., 3, c] = dy
        B[..., 3, c + 1] = dx
        B[..., 4, c + 1] = dz
        B[..., 4, c + 2] = dy
        B[..., 5, c] = dz
        B[..., 5, c + 2] = dx
    return B


# ---------------------------------------------------------------------------
# element evaluation, vectorised over (element, Gauss point) -- Algorithm 2
# ---------------------------------------------------------------------------


def _mat(m, key):
    return m[key] if isinstance(m, dict) else getattr(m, key)


def eval_elements(dim, coords, conn, e_scale, mat, x, kappa_n, elems=None, want_K=True):
    """Gauss-point state, element internal forces and element tangents.

    Follows Eqs. 11a-11f under readings R1-R3, R5-R7, R10-R12 with the
    constitutive functions of Appendix A.  `elems` selects a subset of
    elements (default: all).  Local element dofs are node-interleaved:
    u_i of node a -> a*(dim+1)+i, ebar of node a -> a*(dim+1)+dim.

    Returns a dict with
      fint  [ne, nen*(dim+1)]  element internal force (f_u, f_ebar)
      fref  [ne, nen]          int N h eeq (scale of the ebar equation, R9)
      Ke    [ne, nen*(dim+1), nen*(dim+1)]  element tangent d fint / d x
      kappa, D, eeq, ebar [ne, ngp]
    """
    E = _mat(mat, "E"); nu = _mat(mat, "nu"); k = _mat(mat, "k"); h = _mat(mat, "h")
    c = _mat(mat, "c"); R = _mat(mat, "R"); eta = _mat(mat, "eta")
    kappa0 = _mat(mat, "kappa0"); alpha = _mat(mat, "alpha"); beta = _mat(mat, "beta")
    tol_h = _mat(mat, "tol_hist"); tol_d = _mat(mat, "tol_dmg")
    plane = int(_mat(mat, "plane")); thick = _mat(mat, "thickness")
    coupling = int(mat.get("coupling", 0) if isinstance(mat, dict) else getattr(mat, "coupling", 0))
    if elems is None:
        elems = np.arange(conn.shape[0])
    elems = np.asarray(elems, dtype=np.int64)
    cn = conn[elems].astype(np.int64)
    ne, nen = cn.shape
    nd = dim + 1
    ngp = 2 ** dim
    xe = coords[cn]                                    # [ne, nen, dim]
    dofs = cn[:, :, None] * nd + np.arange(nd)         # [ne, nen, nd]
    xl = x[dofs]
    ue = xl[:, :, :dim].reshape(ne, nen * dim)         # node-major u
    ee = xl[:, :, dim]                                 # [ne, nen]
    Cm = elasticity_matrix(dim, plane, E, nu)
    es = e_scale[elems]
    kn = np.asarray(kappa_n).reshape(-1, ngp)[elems]

    fu = np.zeros((ne, nen * dim)); fe = np.zeros((ne, nen)); fr = np.zeros((ne, nen))
    Kuu = np.zeros((ne, nen * dim, nen * dim)); Kue = np.zeros((ne, nen * dim, nen))
    Keu = np.zeros((ne, nen, nen * dim)); Kee = np.zeros((ne, nen, nen))
    out_k = np.zeros((ne, ngp)); out_D = np.zeros((ne, ngp))
    out_eeq = np.zeros((ne, ngp)); out_eb = np.zeros((ne, ngp))
    pts, wts = gauss_points(dim)
    for g in range(ngp):
        N, dNdxi = shape_functions(dim, pts[g])
        J = np.einsum("ead,aj->edj", xe, dNdxi)        # J_dj = dx_d/dxi_j
        detJ = np.linalg.det(J)
        invJ = np.linalg.inv(J)                        # (J^-1)_jd = dxi_j/dx_d
        dNdx = np.einsum("aj,ejd->ead", dNdxi, invJ)   # [ne, nen, dim]
        B = strain_displacement(dNdx)                  # [ne, nstr, nen*dim]
        eps = np.einsum("esc,ec->es", B, ue)
        eeq, n = equivalent_strain_voigt(dim, plane, k, nu, eps)
        ebar = ee @ N
        gradb = np.einsum("ead,ea->ed", dNdx, ee)
        kap, chi = history(ebar, kn[:, g], tol_h)
        D, dD = damage(kap, kappa0, alpha, beta, tol_d)
        gv, dg = interaction(D, R, eta)
        wJ = wts[g] * detJ * (thick if dim < 3 else 1.0)
        Cs = es[:, None, None] * Cm                    # [ne, nstr, nstr]
        Ceps = np.einsum("est,et->es", Cs, eps)
        sigma = (1.0 - D)[:, None] * Ceps              # R1
        if coupling:                                   # R13: Eq. 2
            sigma = sigma + (h * (eeq - ebar))[:, None] * n
        fu += np.einsum("esc,es->ec", B, sigma) * wJ[:, None]
        fe += (np.outer(h * (ebar - eeq) * wJ, N)
               + np.einsum("ead,ed->ea", dNdx, (gv * h * c * wJ)[:, None] * gradb))  # R2
        fr += np.outer(h * eeq * wJ, N)
        out_k[:, g] = kap; out_D[:, g] = D; out_eeq[:, g] = eeq; out_eb[:, g] = ebar
        if not want_K:
            continue
        # Eq. 11a
        Kuu += np.einsum("esc,est,etd->ecd", B, ((1.0 - D) * wJ)[:, None, None] * Cs, B, optimize=True)
        # Eq. 11b (R1): -B^T (C eps dD/dkappa dkappa/debar) N
        v = Ceps * (dD * chi * wJ)[:, None]
        Kue -= np.einsum("esc,es,a->eca", B, v, N, optimize=True)
        if coupling:
            # R13: Eq. 11b's -B^T h n N, and Eq. 11a completed by the linearisation of Eq. 2
            Kue -= np.einsum("esc,es,a->eca", B, (h * wJ)[:, None] * n, N, optimize=True)
            Hv = equivalent_strain_hessian_voigt(dim, plane, k, nu, eps, kappa0)
            Dc = (h * wJ)[:, None, None] * (n[:, :, None] * n[:, None, :]
                                            + (eeq - ebar)[:, None, None] * Hv)
            Kuu += np.einsum("esc,est,etd->ecd", B, Dc, B, optimize=True)
        # Eq. 11c: -N h n^T B
        Keu -= np.einsum("a,es,esc->eac", N, (h * wJ)[:, None] * n, B, optimize=True)
        # Eq. 11d (R3): h N N^T + h c g' D' chi (B_e grad ebar) N^T + g h c B_e^T B_e
        Kee += (h * wJ)[:, None, None] * np.outer(N, N)[None]
        Kee += np.einsum("e,ea,b->eab", h * c * dg * dD * chi * wJ,
                         np.einsum("ead,ed->ea", dNdx, gradb), N, optimize=True)
        Kee += np.einsum("e,ead,ebd->eab", gv * h * c * wJ, dNdx, dNdx, optimize=True)

    res = {"kappa": out_k, "D": out_D, "eeq": out_eeq, "ebar": out_eb, "fref": fr}
    nl = nen * nd
    iu = (np.arange(nen)[:, None] * nd + np.arange(dim)[None, :]).ravel()   # node-major u
    ie = np.arange(nen) * nd + dim
    fint = np.zeros((ne, nl))
    fint[:, iu] = fu
    fint[:, ie] = fe
    res["fint"] = fint
    if want_K:
        Ke = np.zeros((ne, nl, nl))
        Ke[:, iu[:, None], iu[None, :]] = Kuu
        Ke[:, iu[:, None], ie[None, :]] = Kue
        Ke[:, ie[:, None], iu[None, :]] = Keu
        Ke[:, ie[:, None], ie[None, :]] = Kee
        res["Ke"] = Ke
    return res


def element_loop_eval(dim, coords, conn, e_scale, mat, x, kappa_n):
    """Element-by-element, Gauss-point-by-Gauss-point evaluation with the
    structure of Algorithm 1, written in index notation instead of B
    matrices:  K^uu_{ai,bj} = sum_g w (1-D) s [lam dN_a/dx_i dN_b/dx_j +
    mu dN_a/dx_j dN_b/dx_i + mu delta_ij grad N_a . grad N_b] (3D and plane
    strain; plane stress uses the plane-stress lam*).  Only for tiny meshes;
    used to cross-check eval_elements."""
    E = _mat(mat, "E"); nu = _mat(mat, "nu"); k = _mat(mat, "k"); h = _mat(mat, "h")
    c = _mat(mat, "c"); R = _mat(mat, "R"); eta = _mat(mat, "eta")
    kappa0 = _mat(mat, "kappa0"); alpha = _mat(mat, "alpha"); beta = _mat(mat, "beta")
    tol_h = _mat(mat, "tol_hist"); tol_d = _mat(mat, "tol_dmg")
    if int(mat.get("coupling", 0) if isinstance(mat, dict) else getattr(mat, "coupling", 0)):
        raise NotImplementedError("element_loop_eval covers readings R1-R12 only")
    plane = int(_mat(mat, "plane")); thick = _mat(mat, "thickness")
    nel, nen = conn.shape
    nd = dim + 1
    ngp = 2 ** dim
    pts, wts = gauss_points(dim)
    if dim == 1:
        lam, mu = 0.0, 0.0
    else:
        mu = E / (2.0 * (1.0 + nu))
        lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
        if dim == 2 and plane == 0:
            lam = 2.0 * lam * mu / (lam + 2.0 * mu)
    Ke_all = np.zeros((nel, nen * nd, nen * nd))
    fi_all = np.zeros((nel, nen * nd))
    for e in range(nel):
        nodes = conn[e]
        xe = coords[nodes]
        s = e_scale[e]
        for g in range(ngp):
            N, dNdxi = shape_functions(dim, pts[g])
            J = xe.T @ dNdxi
            dNdx = dNdxi @ np.linalg.inv(J)
            wJ = wts[g] * np.linalg.det(J) * (thick if dim < 3 else 1.0)
            u = np.array([[x[n * nd + i] for i in range(dim)] for n in nodes])
            eb = np.array([x[n * nd + dim] for n in nodes])
            grad_u = u.T @ dNdx                         # du_i/dx_j
            eps_t = 0.5 * (grad_u + grad_u.T)
            if dim == 1:
                eeq = eps_t[0, 0]
                Gd = np.ones((1, 1))
                sig = s * E * eps_t
            else:
                t3 = np.zeros((3, 3))
                t3[:dim, :dim] = eps_t
                if dim == 2 and plane == 0:
                    t3[2, 2] = -nu / (1.0 - nu) * (eps_t[0, 0] + eps_t[1, 1])
                eeq, G = equivalent_strain_tensor(t3, k, nu)
                Gd = G[:dim, :dim].copy()
                if dim == 2 and plane == 0:
                    Gd += -nu / (1.0 - nu) * G[2, 2] * np.eye(2)
                sig = s * (lam * np.trace(eps_t) * np.eye(dim) + 2.0 * mu * eps_t)
            ebar = float(N @ eb)
            gb = dNdx.T @ eb
            kap, chi = history(ebar, kappa_n[e * ngp + g], tol_h)
            D, dD = damage(kap, kappa0, alpha, beta, tol_d)
            gv, dg = interaction(D, R, eta)
            D = float(D); dD = float(dD); gv = float(gv); dg = float(dg); chi = float(chi)
            for a in range(nen):
                ra = a * nd
                fi_all[e, ra:ra + dim] += (1.0 - D) * (sig @ dNdx[a]) * wJ
                fi_all[e, ra + dim] += (N[a] * h * (ebar - eeq) + g_dot(dNdx[a], gv * h * c * gb)) * wJ
                for b in range(nen):
                    rb = b * nd
                    for i in range(dim):
                        for j in range(dim):
                            if dim == 1:
                                kij = s * E * dNdx[a, 0] * dNdx[b, 0]
                            else:
                                kij = s * (lam * dNdx[a, i] * dNdx[b, j] + mu * dNdx[a, j] * dNdx[b, i]
                                           + (mu * g_dot(dNdx[a], dNdx[b]) if i == j else 0.0))
                            Ke_all[e, ra + i, rb + j] += (1.0 - D) * kij * wJ
                        Ke_all[e, ra + i, rb + dim] -= (sig @ dNdx[a])[i] * dD * chi * N[b] * wJ
                        Ke_all[e, ra + dim, rb + i] -= N[a] * h * (Gd @ dNdx[b])[i] * wJ
                    Ke_all[e, ra + dim, rb + dim] += (h * N[a] * N[b]
                                                      + h * c * dg * dD * chi * g_dot(dNdx[a], gb) * N[b]
                                                      + gv * h * c * g_dot(dNdx[a], dNdx[b])) * wJ
    return Ke_all, fi_all


def g_dot(a, b):
    return float(np.dot(a, b))


# ---------------------------------------------------------------------------
# sparsity pattern and assembly (Fig. 2 triplets summed into a sparse matrix)
# ---------------------------------------------------------------------------


def csr_pattern_bruteforce(conn, n_nodes, ndpn):
    """CSR pattern of all element-coupled dof pairs from a Python set of node
    pairs (tiny meshes only).  Node-interleaved dofs; columns ascending."""
    nbr = [set() for _ in range(n_nodes)]
    for e in np.asarray(conn):
        for a in e:
            for b in e:
                nbr[int(a)].add(int(b))
    row_ptr = [0]
    cols = []
    for a in range(n_nodes):
        nb = sorted(nbr[a])
        for r in range(ndpn):
            for b in nb:
                for cc in range(ndpn):
                    cols.append(b * ndpn + cc)
            row_ptr.append(len(cols))
    return np.array(row_ptr, dtype=np.int64), np.array(cols, dtype=np.int64)


def csr_pattern_unique(conn, n_nodes, ndpn):
    """Same pattern through np.unique of node-pair keys (large meshes)."""
    conn = np.asarray(conn, dtype=np.int64)
    nen = conn.shape[1]
    a = np.repeat(conn, nen, axis=1).ravel()
    b = np.tile(conn, (1, nen)).ravel()
    keys = np.unique(a * n_nodes + b)
    na = keys // n_nodes
    nb = keys % n_nodes
    deg = np.bincount(na, minlength=n_nodes)
    nstart = np.concatenate([[0], np.cumsum(deg)])
    row_len = deg * ndpn
    rows_per_node = np.repeat(row_len, ndpn)
    row_ptr = np.concatenate([[0], np.cumsum(rows_per_node)]).astype(np.int64)
    cols = np.empty(int(row_ptr[-1]), dtype=np.int64)
    blockcols = (nb[:, None] * ndpn + np.arange(ndpn)[None, :])   # [npairs, ndpn]
    # rows of node a: r = 0..ndpn-1, each row = its neighbours' column blocks in order
    pair_rank = np.arange(len(keys)) - nstart[na]
    for r in range(ndpn):
        base = row_ptr[na * ndpn + r] + pair_rank * ndpn
        for cc in range(ndpn):
            cols[base + cc] = blockcols[:, cc]
    return row_ptr, cols


def assemble(dim, conn, n_nodes, fint, Ke=None):
    """Sum element contributions into global vectors / a CSR matrix (Fig. 2,
    sparse() of concatenated triplets sums duplicates)."""
    nd = dim + 1
    cn = np.asarray(conn, dtype=np.int64)
    ne, nen = cn.shape
    dofs = (cn[:, :, None] * nd + np.arange(nd)).reshape(ne, nen * nd)
    ndof = n_nodes * nd
    f = np.bincount(dofs.ravel(), weights=fint.ravel(), minlength=ndof)
    if Ke is None:
        return f, None
    nl = nen * nd
    rows = np.repeat(dofs, nl, axis=1).ravel()
    cols = np.tile(dofs, (1, nl)).ravel()
    K = sp.coo_matrix((Ke.ravel(), (rows, cols)), shape=(ndof, ndof)).tocsr()
    K.sum_duplicates()
    K.sort_indices()
    return f, K


def apply_dirichlet(K, R, bc_dofs):
    """Reading R8: constrained rows and columns become identity, R_c = 0.
    The pattern is unchanged."""
    K = K.copy()
    n = K.shape[0]
    isbc = np.zeros(n, dtype=bool)
    isbc[bc_dofs] = True
    rows = np.repeat(np.arange(n), np.diff(K.indptr))
    mask = isbc[rows] | isbc[K.indices]
    K.data[mask] = 0.0
    diag = mask & (rows == K.indices) & isbc[rows]
    K.data[diag] = 1.0
    R = R.copy()
    R[bc_dofs] = 0.0
    return K, R


# ---------------------------------------------------------------------------
# the Newton driver (Algorithm 2)
# ---------------------------------------------------------------------------


class Oracle:
    """Incremental-iterative Newton solver of Eq. 11 (Algorithm 2).

    prob: an lgdm_workloads.Problem (or any object with the same fields).
    """

    def __init__(self, prob, coords=None, material=None, h_override=None):
        self.prob = prob
        self.dim = prob.dim
        self.nd = prob.dim + 1
        self.coords = prob.coords if coords is None else coords
        self.conn = np.asarray(prob.conn, dtype=np.int64)
        self.e_scale = np.asarray(prob.e_scale, dtype=np.float64)
        m = material if material is not None else prob.material
        self.mat = dict(m.as_dict() if hasattr(m, "as_dict") else m)
        if h_override is not None:
            self.mat["h"] = h_override
        self.n_nodes = prob.n_nodes
        self.ndof = self.n_nodes * self.nd
        self.ngp = 2 ** self.dim
        self.bc_dofs = (np.asarray(prob.bc_nodes, dtype=np.int64) * self.nd
                        + np.asarray(prob.bc_comps, dtype=np.int64))
        self.bc_vals = np.asarray(prob.bc_values, dtype=np.float64)
        self.loaded = self.bc_dofs[self.bc_vals != 0.0]
        self.x = np.zeros(self.ndof)
        self.kappa_n = np.zeros(prob.n_elems * self.ngp)          # R7: kappa_n(0) = 0
        self.D_n = np.zeros(prob.n_elems * self.ngp)
        self.increment = 0
        self.u_mask = np.ones(self.ndof, dtype=bool)
        self.u_mask[self.dim::self.nd] = False

    # Algorithm 2, "Compute and Assemble K" / "Compute and Assemble F"
    def eval_state(self, x=None, kappa_n=None, want_K=True):
        x = self.x if x is None else x
        kappa_n = self.kappa_n if kappa_n is None else kappa_n
        ev = eval_elements(self.dim, self.coords, self.conn, self.e_scale, self.mat, x,
                           kappa_n, want_K=want_K)
        fint, K = assemble(self.dim, self.conn, self.n_nodes, ev["fint"], ev.get("Ke"))
        fref, _ = assemble(self.dim, self.conn, self.n_nodes,
                           _scatter_e(ev["fref"], self.nd, self.dim))
        R = -fint
        if K is not None:
            K, R = apply_dirichlet(K, R, self.bc_dofs)
        else:
            R[self.bc_dofs] = 0.0
        out = dict(ev)
        out.update(K=K, R=R, fint=fint, fref_vec=fref)
        out["norms"] = self.norms(R, fint, fref)
        out["reaction"] = float(np.sum(fint[self.loaded]))
        return out

    def norms(self, R, fint, fref):
        ru = float(np.linalg.norm(R[self.u_mask]))
        re = float(np.linalg.norm(R[~self.u_mask]))
        fu = float(np.linalg.norm(fint[self.u_mask]))
        fe = float(np.linalg.norm(fref[~self.u_mask]))
        return dict(res_u=ru, res_e=re, ref_u=fu, ref_e=fe)

    @staticmethod
    def converged(nrm, tol, tiny=1e-300):
        """Reading R9, per field.  A non-finite norm (a state that overflowed)
        is never convergence."""
        if not all(np.isfinite(v) for v in nrm.values()):
            return False
        return (nrm["res_u"] <= tol * max(nrm["ref_u"], tiny)
                and nrm["res_e"] <= tol * max(nrm["ref_e"], tiny))

    def solve_increment(self, lam=None, tol=1e-8, max_iter=30):
        """One load increment: set u_c = lam u_ref, Newton to convergence,
        commit kappa (Eq. A.2).  Returns a report dict."""
        if lam is None:
            lam = (self.increment + 1) / self.prob.n_increments
        x_save = self.x.copy()
        self.x[self.bc_dofs] = lam * self.bc_vals                  # R8
        its = 0
        hist = []
        while True:
            st = self.eval_state()
            nrm = st["norms"]
            hist.append(nrm)
            if self.converged(nrm, tol):
                break
            if its >= max_iter:
                self.x = x_save
                return dict(converged=False, iters=its, history=hist)
            dx = spla.splu(st["K"].tocsc()).solve(st["R"])
            self.x = self.x + dx                                   # Algorithm 2 update
            its += 1
        self.kappa_n = st["kappa"].ravel().copy()
        self.D_n = st["D"].ravel().copy()
        self.increment += 1
        return dict(converged=True, iters=its, history=hist, reaction=st["reaction"],
                    lam=lam, D=self.D_n.copy(), kappa=self.kappa_n.copy(), x=self.x.copy(),
                    max_D=float(self.D_n.max()) if self.D_n.size else 0.0)

    def run(self, n_increments=None, tol=1e-8, max_iter=30, callback=None):
        n = self.prob.n_increments if n_increments is None else n_increments
        reps = []
        for _ in range(n):
            rep = self.solve_increment(tol=tol, max_iter=max_iter)
            reps.append(rep)
            if callback is not None:
                callback(rep)
            if not rep["converged"]:
                break
        return reps


def _scatter_e(fref, nd, dim):
    """Place per-node ebar-row values into node-interleaved element vectors."""
    ne, nen = fref.shape
    out = np.zeros((ne, nen * nd))
    out[:, np.arange(nen) * nd + dim] = fref
    return out
