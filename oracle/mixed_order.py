"""LGDM oracle for the mixed-order elements the paper runs in 1D and 2D.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the product
path may import this module.

The paper discretises the displacement with quadratic and the
micro-equivalent strain with linear shape functions (Sec. 2.1, after
Eqs. 9-10), in 1D (Sec. 3.1) and with biquadratic u / bilinear ebar
elements in 2D (Sec. 3.2).  Everything else -- the constitutive functions of
Appendix A, the element integrals of Eqs. 11a-11f, assembly, the Dirichlet
treatment and the Newton iteration of Algorithm 2 -- is that of
oracle.lgdm under the same readings R1-R9, R11 and R12; only the two
interpolations and the quadrature differ.  In the element integrals, N_u and
B_u (the strain-displacement operator) come from the quadratic element and
N_e, grad N_e from the linear one:

  f_u     = int B_u^T (1 - D) s_e C eps
  f_ebar  = int N_e h (ebar - eeq) + grad N_e . (g h c grad ebar)
  K^uu    = int B_u^T (1 - D) s_e C B_u                         (11a)
  K^ue    = -int B_u^T (s_e C eps) D' chi N_e^T                 (11b, R1)
  K^eu    = -int N_e h n^T B_u                                  (11c)
  K^ee    = int h N_e N_e^T + h c g' D' chi (grad N_e . grad ebar) N_e^T
            + g h c grad N_e grad N_e^T                         (11d, R3)

Readings specific to these elements
-----------------------------------
F1  Quadrature: 3-point Gauss-Legendre per direction (points -sqrt(3/5), 0,
    sqrt(3/5), weights 5/9, 8/9, 5/9), Gauss point g = i_xi + 3 i_eta.  The
    paper does not state its rule; this is the full rule of the quadratic
    element (the elastic block of an affine element is integrated exactly).
F2  Geometry is interpolated by the displacement element (isoparametric in
    u); the ebar element shares its Jacobian.
F3  "Biquadratic" is the 9-node Lagrange quadrilateral; the ebar element
    lives on its 4 corner nodes (the 2 end nodes of the 3-node line in 1D),
    so ebar dofs exist at the vertex nodes only.
F4  Local node order: line3 (left end, right end, midpoint); quad9 corners
    counter-clockwise from (-1, -1), mid-side nodes of the edges 0-1, 1-2,
    2-3, 3-0, then the centre.  The ebar element takes the first 2^dim.
F5  The coupling variant (R13) is not defined for these elements.

Dof numbering of this oracle: the plain definition, u of node a component i
at a*dim + i, then ebar of the v-th vertex node (vertex nodes in ascending
node id) at n_nodes*dim + v.  Element vectors and matrices are laid out
[u node-major (nen_u*dim) | ebar (nen_e)].  `to_interleaved` /
`from_interleaved` map to and from the node-interleaved layout
node*(dim+1) + comp used by the workloads (ebar entries of non-vertex nodes
zero there).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .lgdm import (Oracle, _mat, damage, elasticity_matrix, equivalent_strain_tensor,
                   equivalent_strain_voigt, history, interaction, shape_functions,
                   strain_displacement)

__all__ = ["gauss_points_3", "reference_nodes_q", "shape_functions_q", "eval_elements_mixed",
           "element_loop_eval_mixed", "MixedOracle"]


# ---------------------------------------------------------------------------
# quadrature and shape functions (F1, F3, F4)
# ---------------------------------------------------------------------------

def gauss_points_3(dim: int):
    """3-point Gauss-Legendre per direction (F1): points [3^dim, dim] and
    weights [3^dim], point g = i_xi + 3 i_eta."""
    t = (-math.sqrt(0.6), 0.0, math.sqrt(0.6))
    w = (5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0)
    pts, wts = [], []
    for g in range(3 ** dim):
        idx = [(g // 3 ** d) % 3 for d in range(dim)]
        pts.append([t[i] for i in idx])
        wts.append(float(np.prod([w[i] for i in idx])))
    return np.array(pts), np.array(wts)


def reference_nodes_q(dim: int) -> np.ndarray:
    """Reference coordinates of the quadratic element's nodes (F4)."""
    if dim == 1:
        return np.array([[-1.0], [1.0], [0.0]])
    if dim == 2:
        return np.array([[-1.0, -1.0], [1.0, -1.0], [1.0, 1.0], [-1.0, 1.0],
                         [0.0, -1.0], [1.0, 0.0], [0.0, 1.0], [-1.0, 0.0], [0.0, 0.0]])
    raise ValueError("mixed-order elements are defined in 1D and 2D")


def _lagrange2(node: float, t: float):
    """1D quadratic Lagrange function on the nodes {-1, 0, 1} that is 1 at
    `node`, and its derivative, at t."""
    if node < -0.5:
        return 0.5 * t * (t - 1.0), t - 0.5
    if node > 0.5:
        return 0.5 * t * (t + 1.0), t + 0.5
    return 1.0 - t * t, -2.0 * t


def shape_functions_q(dim: int, xi: np.ndarray):
    """Quadratic (1D) / biquadratic Lagrange (2D) shape functions as tensor
    products of _lagrange2: N [nen_u], dN/dxi [nen_u, dim]."""
    nodes = reference_nodes_q(dim)
    nen = len(nodes)
    N = np.ones(nen)
    dN = np.ones((nen, dim))
    for a in range(nen):
        f = [_lagrange2(nodes[a, d], xi[d]) for d in range(dim)]
        for d in range(dim):
            N[a] *= f[d][0]
            for j in range(dim):
                dN[a, j] *= f[d][1] if d == j else f[d][0]
    return N, dN


# ---------------------------------------------------------------------------
# element evaluation, vectorised over elements
# ---------------------------------------------------------------------------

def eval_elements_mixed(dim, coords, conn, e_scale, mat, u_nodal, ebar_vertex, vidx, kappa_n,
                        want_K=True):
    """Gauss-point state, element internal forces and tangents of the
    mixed-order elements (Eqs. 11a-11f with N_u, B_u quadratic and N_e
    linear; readings R1-R3, R5-R7, R11, R12, F1-F4).

    u_nodal [n_nodes, dim]; ebar_vertex [n_vertices]; vidx [n_nodes] the
    vertex index of each node (-1 where the node carries no ebar);
    kappa_n [nel * 3^dim].  Returns fint [ne, nen_u*dim + nen_e], fref
    [ne, nen_e] (int N_e h eeq), Ke [ne, nl, nl] and per-Gauss-point kappa,
    D, eeq, ebar [ne, ngp]."""
    E = _mat(mat, "E"); nu = _mat(mat, "nu"); k = _mat(mat, "k"); h = _mat(mat, "h")
    c = _mat(mat, "c"); R = _mat(mat, "R"); eta = _mat(mat, "eta")
    kappa0 = _mat(mat, "kappa0"); alpha = _mat(mat, "alpha"); beta = _mat(mat, "beta")
    tol_h = _mat(mat, "tol_hist"); tol_d = _mat(mat, "tol_dmg")
    plane = int(_mat(mat, "plane")); thick = _mat(mat, "thickness")
    coupling = int(mat.get("coupling", 0) if isinstance(mat, dict) else getattr(mat, "coupling", 0))
    if coupling:
        raise NotImplementedError("the coupling variant is not defined for mixed-order elements (F5)")
    cn = np.asarray(conn, dtype=np.int64)
    ne, nen = cn.shape
    nene = 2 ** dim
    nu_dofs = nen * dim
    pts, wts = gauss_points_3(dim)
    ngp = len(wts)
    xe = coords[cn]                                   # [ne, nen, dim]
    ue = u_nodal[cn].reshape(ne, nu_dofs)             # node-major u
    vi = vidx[cn[:, :nene]]
    assert np.all(vi >= 0), "ebar element nodes must be vertex nodes"
    ee = ebar_vertex[vi]                              # [ne, nene]
    Cm = elasticity_matrix(dim, plane, E, nu)
    es = np.asarray(e_scale, dtype=np.float64)
    kn = np.asarray(kappa_n).reshape(ne, ngp)
    fu = np.zeros((ne, nu_dofs)); fe = np.zeros((ne, nene)); fr = np.zeros((ne, nene))
    Kuu = np.zeros((ne, nu_dofs, nu_dofs)); Kue = np.zeros((ne, nu_dofs, nene))
    Keu = np.zeros((ne, nene, nu_dofs)); Kee = np.zeros((ne, nene, nene))
    out = {q: np.zeros((ne, ngp)) for q in ("kappa", "D", "eeq", "ebar")}
    for g in range(ngp):
        Nu, dNu = shape_functions_q(dim, pts[g])
        Ne, dNe = shape_functions(dim, pts[g])        # linear Lagrange (the equal-order functions)
        J = np.einsum("ead,aj->edj", xe, dNu)          # F2: geometry from the quadratic element
        detJ = np.linalg.det(J)
        invJ = np.linalg.inv(J)
        dNux = np.einsum("aj,ejd->ead", dNu, invJ)
        dNex = np.einsum("aj,ejd->ead", dNe, invJ)
        B = strain_displacement(dNux)                 # [ne, nstr, nu_dofs]
        eps = np.einsum("esc,ec->es", B, ue)
        eeq, n = equivalent_strain_voigt(dim, plane, k, nu, eps)
        ebar = ee @ Ne
        gradb = np.einsum("ead,ea->ed", dNex, ee)
        kap, chi = history(ebar, kn[:, g], tol_h)
        D, dD = damage(kap, kappa0, alpha, beta, tol_d)
        gv, dg = interaction(D, R, eta)
        wJ = wts[g] * detJ * (thick if dim < 3 else 1.0)
        Cs = es[:, None, None] * Cm
        Ceps = np.einsum("est,et->es", Cs, eps)
        sigma = (1.0 - D)[:, None] * Ceps             # R1
        fu += np.einsum("esc,es->ec", B, sigma) * wJ[:, None]
        fe += (np.outer(h * (ebar - eeq) * wJ, Ne)
               + np.einsum("ead,ed->ea", dNex, (gv * h * c * wJ)[:, None] * gradb))   # R2
        fr += np.outer(h * eeq * wJ, Ne)
        out["kappa"][:, g] = kap; out["D"][:, g] = D; out["eeq"][:, g] = eeq; out["ebar"][:, g] = ebar
        if not want_K:
            continue
        Kuu += np.einsum("esc,est,etd->ecd", B, ((1.0 - D) * wJ)[:, None, None] * Cs, B, optimize=True)
        Kue -= np.einsum("esc,es,a->eca", B, Ceps * (dD * chi * wJ)[:, None], Ne, optimize=True)
        Keu -= np.einsum("a,es,esc->eac", Ne, (h * wJ)[:, None] * n, B, optimize=True)
        Kee += (h * wJ)[:, None, None] * np.outer(Ne, Ne)[None]
        Kee += np.einsum("e,ea,b->eab", h * c * dg * dD * chi * wJ,
                         np.einsum("ead,ed->ea", dNex, gradb), Ne, optimize=True)
        Kee += np.einsum("e,ead,ebd->eab", gv * h * c * wJ, dNex, dNex, optimize=True)
    res = dict(out)
    res["fref"] = fr
    res["fint"] = np.concatenate([fu, fe], axis=1)
    if want_K:
        Ke = np.zeros((ne, nu_dofs + nene, nu_dofs + nene))
        Ke[:, :nu_dofs, :nu_dofs] = Kuu
        Ke[:, :nu_dofs, nu_dofs:] = Kue
        Ke[:, nu_dofs:, :nu_dofs] = Keu
        Ke[:, nu_dofs:, nu_dofs:] = Kee
        res["Ke"] = Ke
    return res


def element_loop_eval_mixed(dim, coords, conn, e_scale, mat, u_nodal, ebar_vertex, vidx, kappa_n):
    """Element-by-element, Gauss-point-by-Gauss-point evaluation in index
    notation (Algorithm 1 structure), used only to cross-check
    eval_elements_mixed on tiny meshes:
      K^uu_{ai,bj} = sum_g w (1-D) s [lam dNa_i dNb_j + mu dNa_j dNb_i
                     + mu delta_ij grad Na . grad Nb]  (1D: s E dNa dNb),
    with lam the plane-stress lam* in plane stress."""
    E = _mat(mat, "E"); nu = _mat(mat, "nu"); k = _mat(mat, "k"); h = _mat(mat, "h")
    c = _mat(mat, "c"); R = _mat(mat, "R"); eta = _mat(mat, "eta")
    kappa0 = _mat(mat, "kappa0"); alpha = _mat(mat, "alpha"); beta = _mat(mat, "beta")
    tol_h = _mat(mat, "tol_hist"); tol_d = _mat(mat, "tol_dmg")
    plane = int(_mat(mat, "plane")); thick = _mat(mat, "thickness")
    nel, nen = conn.shape
    nene = 2 ** dim
    nl = nen * dim + nene
    pts, wts = gauss_points_3(dim)
    if dim == 1:
        lam = mu = 0.0
    else:
        mu = E / (2.0 * (1.0 + nu))
        lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
        if plane == 0:
            lam = 2.0 * lam * mu / (lam + 2.0 * mu)
    Ke_all = np.zeros((nel, nl, nl))
    fi_all = np.zeros((nel, nl))
    for e in range(nel):
        nodes = conn[e]
        xe = coords[nodes]
        s = e_scale[e]
        u = u_nodal[nodes]                                   # [nen, dim]
        eb = np.array([ebar_vertex[vidx[nodes[a]]] for a in range(nene)])
        for g in range(len(wts)):
            Nu, dNu = shape_functions_q(dim, pts[g])
            Ne, dNe = shape_functions(dim, pts[g])
            J = xe.T @ dNu
            Ji = np.linalg.inv(J)
            gu_ = dNu @ Ji                                   # [nen, dim] grad N_u
            ge_ = dNe @ Ji                                   # [nene, dim] grad N_e
            wJ = wts[g] * np.linalg.det(J) * thick
            grad_u = u.T @ gu_
            eps_t = 0.5 * (grad_u + grad_u.T)
            if dim == 1:
                eeq = eps_t[0, 0]
                Gd = np.ones((1, 1))
                sig = s * E * eps_t
            else:
                t3 = np.zeros((3, 3))
                t3[:2, :2] = eps_t
                if plane == 0:
                    t3[2, 2] = -nu / (1.0 - nu) * (eps_t[0, 0] + eps_t[1, 1])
                eeq, G = equivalent_strain_tensor(t3, k, nu)
                Gd = G[:2, :2].copy()
                if plane == 0:
                    Gd += -nu / (1.0 - nu) * G[2, 2] * np.eye(2)
                sig = s * (lam * np.trace(eps_t) * np.eye(2) + 2.0 * mu * eps_t)
            ebar = float(Ne @ eb)
            gb = ge_.T @ eb
            kap, chi = history(ebar, kappa_n[e * len(wts) + g], tol_h)
            D, dD = damage(kap, kappa0, alpha, beta, tol_d)
            gv, dg = interaction(D, R, eta)
            D = float(D); dD = float(dD); gv = float(gv); dg = float(dg); chi = float(chi)
            for a in range(nen):
                for i in range(dim):
                    fi_all[e, a * dim + i] += (1.0 - D) * (sig @ gu_[a])[i] * wJ
                for b in range(nen):
                    for i in range(dim):
                        for j in range(dim):
                            if dim == 1:
                                kij = s * E * gu_[a, 0] * gu_[b, 0]
                            else:
                                kij = s * (lam * gu_[a, i] * gu_[b, j] + mu * gu_[a, j] * gu_[b, i]
                                           + (mu * float(gu_[a] @ gu_[b]) if i == j else 0.0))
                            Ke_all[e, a * dim + i, b * dim + j] += (1.0 - D) * kij * wJ
                for b in range(nene):
                    cb = nen * dim + b
                    for i in range(dim):
                        Ke_all[e, a * dim + i, cb] -= (sig @ gu_[a])[i] * dD * chi * Ne[b] * wJ
            for a in range(nene):
                ra = nen * dim + a
                fi_all[e, ra] += (Ne[a] * h * (ebar - eeq) + float(ge_[a] @ (gv * h * c * gb))) * wJ
                for b in range(nen):
                    for i in range(dim):
                        Ke_all[e, ra, b * dim + i] -= Ne[a] * h * (Gd @ gu_[b])[i] * wJ
                for b in range(nene):
                    Ke_all[e, ra, nen * dim + b] += (h * Ne[a] * Ne[b]
                                                     + h * c * dg * dD * chi * float(ge_[a] @ gb) * Ne[b]
                                                     + gv * h * c * float(ge_[a] @ ge_[b])) * wJ
    return Ke_all, fi_all


# ---------------------------------------------------------------------------
# the Newton driver (Algorithm 2) on the mixed-order layout
# ---------------------------------------------------------------------------

class MixedOracle(Oracle):
    """Algorithm 2 on a mixed-order problem (lgdm_workloads LINE3 / QUAD9).

    x holds u (node-major, n_nodes*dim) then ebar at the vertex nodes.  The
    Newton iteration, convergence test (R9), Dirichlet treatment (R8) and
    history commit (Eq. A.2) are those of Oracle."""

    def __init__(self, prob, coords=None, material=None, h_override=None):
        super().__init__(prob, coords=coords, material=material, h_override=h_override)
        dim = prob.dim
        self.nene = 2 ** dim
        self.vnodes = np.unique(np.asarray(self.conn[:, :self.nene], dtype=np.int64))
        self.vidx = -np.ones(self.n_nodes, dtype=np.int64)
        self.vidx[self.vnodes] = np.arange(len(self.vnodes))
        self.nvert = len(self.vnodes)
        self.ndof = self.n_nodes * dim + self.nvert
        self.ngp = 3 ** dim
        self.bc_dofs = (np.asarray(prob.bc_nodes, dtype=np.int64) * dim
                        + np.asarray(prob.bc_comps, dtype=np.int64))
        self.loaded = self.bc_dofs[self.bc_vals != 0.0]
        self.x = np.zeros(self.ndof)
        self.kappa_n = np.zeros(prob.n_elems * self.ngp)
        self.D_n = np.zeros(prob.n_elems * self.ngp)
        self.u_mask = np.zeros(self.ndof, dtype=bool)
        self.u_mask[:self.n_nodes * dim] = True
        cn = self.conn
        self.edofs = np.concatenate([(cn[:, :, None] * dim + np.arange(dim)).reshape(len(cn), -1),
                                     self.n_nodes * dim + self.vidx[cn[:, :self.nene]]], axis=1)

    # layout maps (node-interleaved node*(dim+1) + comp <-> this oracle's)
    def to_interleaved(self, x):
        dim, nd = self.dim, self.dim + 1
        out = np.zeros(self.n_nodes * nd)
        for i in range(dim):
            out[i::nd] = x[i:self.n_nodes * dim:dim]
        out[self.vnodes * nd + dim] = x[self.n_nodes * dim:]
        return out

    def from_interleaved(self, xi):
        dim, nd = self.dim, self.dim + 1
        out = np.zeros(self.ndof)
        for i in range(dim):
            out[i:self.n_nodes * dim:dim] = xi[i::nd]
        out[self.n_nodes * dim:] = xi[self.vnodes * nd + dim]
        return out

    def interleaved_index(self):
        """Node-interleaved dof of each of this oracle's dofs."""
        dim, nd = self.dim, self.dim + 1
        idx = np.empty(self.ndof, dtype=np.int64)
        nodes = np.arange(self.n_nodes)
        for i in range(dim):
            idx[i:self.n_nodes * dim:dim] = nodes * nd + i
        idx[self.n_nodes * dim:] = self.vnodes * nd + dim
        return idx

    def eval_state(self, x=None, kappa_n=None, want_K=True):
        x = self.x if x is None else x
        kappa_n = self.kappa_n if kappa_n is None else kappa_n
        dim = self.dim
        u = x[:self.n_nodes * dim].reshape(self.n_nodes, dim)
        ev = eval_elements_mixed(dim, self.coords, self.conn, self.e_scale, self.mat, u,
                                 x[self.n_nodes * dim:], self.vidx, kappa_n, want_K=want_K)
        ed = self.edofs
        fint = np.bincount(ed.ravel(), weights=ev["fint"].ravel(), minlength=self.ndof)
        fre = np.zeros_like(ev["fint"])
        fre[:, self.conn.shape[1] * dim:] = ev["fref"]
        fref = np.bincount(ed.ravel(), weights=fre.ravel(), minlength=self.ndof)
        R = -fint
        K = None
        if want_K:
            nl = ed.shape[1]
            rows = np.repeat(ed, nl, axis=1).ravel()
            cols = np.tile(ed, (1, nl)).ravel()
            K = sp.coo_matrix((ev["Ke"].ravel(), (rows, cols)), shape=(self.ndof, self.ndof)).tocsr()
            K.sum_duplicates()
            K.sort_indices()
            from .lgdm import apply_dirichlet
            K, R = apply_dirichlet(K, R, self.bc_dofs)
        else:
            R[self.bc_dofs] = 0.0
        out = dict(ev)
        out.update(K=K, R=R, fint=fint, fref_vec=fref)
        out["norms"] = self.norms(R, fint, fref)
        out["reaction"] = float(np.sum(fint[self.loaded]))
        return out
