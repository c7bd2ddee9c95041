"""Seeded synthetic problem definitions for the LGDM hot path.

This module states *problems* -- geometry, connectivity, per-element stiffness
scale, Dirichlet sets, material parameters and load stepping -- the inputs
named in the paper's problem statement (Algorithms 1 and 2, "Input: Geometry,
Material properties, Loads and boundary conditions").  It holds none of the
method's arithmetic: no shape functions, no constitutive law, no assembly.
Both the HIP path and the CPU oracle consume these definitions; neither
shares any other code.

Meshes are structured:
  node id    = i + (nx+1) * (j + (ny+1) * k)
  element id = i + nx * (j + ny * k)
  local node order: line2 (x0, x1); quad4 counter-clockwise from the
  (i, j) corner; hex8 bottom face counter-clockwise, then the top face in
  the same order.  Mixed-order meshes (line3, quad9) number the nodes of the
  finer node grid the same way and list each element's vertices first.

The problems stand in for the paper's 1D bar (Sec. 3.1, Fig. 10), 2D
side-edge-notch (Sec. 3.2) and 3D notched specimen (Sec. 3.3), whose exact
geometries and reference data are not available; sizes and parameters follow
the workload descriptions the build is measured on.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional

import numpy as np

LINE2, QUAD4, HEX8 = 1, 2, 3
# mixed-order elements (Sec. 2.1: quadratic u, linear ebar): the u element's
# nodes with the ebar element on its vertices
LINE3, QUAD9 = 4, 5
MIXED_ORDER = (LINE3, QUAD9)
PLANE_STRESS, PLANE_STRAIN = 0, 1


@dataclasses.dataclass
class Material:
    """Material and numerical parameters (Eq. 1, Eqs. A.1-A.4).

    E is the undamaged Young's modulus (MPa), nu Poisson's ratio, kappa0 the
    damage threshold, alpha/beta the damage-law parameters (A.1), c the
    gradient parameter (mm^2), R and eta the interaction-function parameters
    (A.4), k the compressive/tensile strength ratio (A.3), h the coupling
    modulus (Eq. 1).  tol_hist / tol_dmg are the tie-break bands of the
    vectorised variable update (Fig. 8b).  thickness is the out-of-plane
    thickness in 2D and the cross-section area in 1D (ignored in 3D).
    """
    E: float
    nu: float
    kappa0: float
    alpha: float
    beta: float
    c: float
    R: float
    eta: float
    k: float
    h: float
    tol_hist: float = 1e-10
    tol_dmg: float = 1e-10
    plane: int = PLANE_STRESS
    thickness: float = 1.0
    coupling: int = 0       # 0: stress (1 - D) C : eps; 1: the stress of Eq. 2 with its h term

    def as_dict(self) -> Dict[str, float]:
        return dataclasses.asdict(self)


@dataclasses.dataclass
class Problem:
    name: str
    dim: int
    elem_type: int
    shape: tuple            # (nx,) / (nx, ny) / (nx, ny, nz)
    coords: np.ndarray      # float64 [n_nodes, dim]
    conn: np.ndarray        # int32 [n_elems, nen]
    e_scale: np.ndarray     # float64 [n_elems] multiplies the elasticity tensor only
    bc_nodes: np.ndarray    # int64 [n_bc]
    bc_comps: np.ndarray    # int64 [n_bc]   displacement component 0..dim-1
    bc_values: np.ndarray   # float64 [n_bc] prescribed value at load factor 1
    material: Material
    n_increments: int

    @property
    def n_nodes(self) -> int:
        return int(self.coords.shape[0])

    @property
    def n_elems(self) -> int:
        return int(self.conn.shape[0])

    @property
    def nen(self) -> int:
        return int(self.conn.shape[1])

    @property
    def ndpn(self) -> int:
        """dofs per node: dim displacement components + the micro-equivalent strain."""
        return self.dim + 1

    @property
    def ndof(self) -> int:
        return self.n_nodes * self.ndpn

    @property
    def ngp(self) -> int:
        """Gauss points per element: 2 per direction for equal-order elements,
        3 per direction for the mixed-order ones."""
        return (3 if self.elem_type in MIXED_ORDER else 2) ** self.dim

    @property
    def nen_e(self) -> int:
        """Nodes of the ebar element: the first 2^dim of each element's list."""
        return 2 ** self.dim

    def ebar_nodes(self) -> np.ndarray:
        """Sorted ids of the nodes that carry an ebar dof (every node for
        equal-order elements, the vertices of the mixed-order elements)."""
        if self.elem_type not in MIXED_ORDER:
            return np.arange(self.n_nodes, dtype=np.int64)
        return np.unique(np.asarray(self.conn[:, :self.nen_e], dtype=np.int64))

    def bc_dofs(self) -> np.ndarray:
        """Node-interleaved dof numbering: dof = node * (dim + 1) + comp."""
        return (self.bc_nodes * self.ndpn + self.bc_comps).astype(np.int64)


# --------------------------------------------------------------------------
# structured meshes
# --------------------------------------------------------------------------

def mesh_line2(nx: int, lx: float):
    x = np.linspace(0.0, lx, nx + 1)
    coords = x.reshape(-1, 1).astype(np.float64)
    i = np.arange(nx)
    conn = np.stack([i, i + 1], axis=1).astype(np.int32)
    return coords, conn


def mesh_quad4(nx: int, ny: int, lx: float, ly: float):
    xs = np.linspace(0.0, lx, nx + 1)
    ys = np.linspace(0.0, ly, ny + 1)
    X, Y = np.meshgrid(xs, ys, indexing="xy")          # [ny+1, nx+1]
    coords = np.stack([X.ravel(), Y.ravel()], axis=1).astype(np.float64)
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    i = i.ravel(); j = j.ravel()
    n = lambda ii, jj: ii + (nx + 1) * jj
    conn = np.stack([n(i, j), n(i + 1, j), n(i + 1, j + 1), n(i, j + 1)], axis=1)
    return coords, conn.astype(np.int32)


def mesh_hex8(nx: int, ny: int, nz: int, lx: float, ly: float, lz: float):
    xs = np.linspace(0.0, lx, nx + 1)
    ys = np.linspace(0.0, ly, ny + 1)
    zs = np.linspace(0.0, lz, nz + 1)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")   # [nz+1, ny+1, nx+1]
    coords = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1).astype(np.float64)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i = i.ravel(); j = j.ravel(); k = k.ravel()
    n = lambda ii, jj, kk: ii + (nx + 1) * (jj + (ny + 1) * kk)
    conn = np.stack([n(i, j, k), n(i + 1, j, k), n(i + 1, j + 1, k), n(i, j + 1, k),
                     n(i, j, k + 1), n(i + 1, j, k + 1), n(i + 1, j + 1, k + 1),
                     n(i, j + 1, k + 1)], axis=1)
    return coords, conn.astype(np.int32)


def mesh_line3(nx: int, lx: float):
    """Quadratic line elements: 2 nx + 1 equally spaced nodes; element e has
    local nodes (left end, right end, midpoint) = (2e, 2e + 2, 2e + 1)."""
    coords = np.linspace(0.0, lx, 2 * nx + 1).reshape(-1, 1).astype(np.float64)
    i = np.arange(nx)
    conn = np.stack([2 * i, 2 * i + 2, 2 * i + 1], axis=1).astype(np.int32)
    return coords, conn


def mesh_quad9(nx: int, ny: int, lx: float, ly: float):
    """Nine-node quadrilaterals on a (2 nx + 1) x (2 ny + 1) node grid, node id
    I + (2 nx + 1) J.  Local order: the corners counter-clockwise from the
    (i, j) corner, the mid-side nodes of edges 0-1, 1-2, 2-3, 3-0, the centre."""
    xs = np.linspace(0.0, lx, 2 * nx + 1)
    ys = np.linspace(0.0, ly, 2 * ny + 1)
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    coords = np.stack([X.ravel(), Y.ravel()], axis=1).astype(np.float64)
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    I = 2 * i.ravel(); J = 2 * j.ravel()
    n = lambda ii, jj: ii + (2 * nx + 1) * jj
    conn = np.stack([n(I, J), n(I + 2, J), n(I + 2, J + 2), n(I, J + 2),
                     n(I + 1, J), n(I + 2, J + 1), n(I + 1, J + 2), n(I, J + 1),
                     n(I + 1, J + 1)], axis=1)
    return coords, conn.astype(np.int32)


def _bc(nodes, comps, values):
    nodes = np.asarray(nodes, dtype=np.int64)
    out_n, out_c, out_v = [], [], []
    for c, v in zip(comps, values):
        out_n.append(nodes)
        out_c.append(np.full(nodes.shape, c, dtype=np.int64))
        out_v.append(np.full(nodes.shape, v, dtype=np.float64))
    n = np.concatenate(out_n); c = np.concatenate(out_c); v = np.concatenate(out_v)
    order = np.lexsort((c, n))
    return n[order], c[order], v[order]


def base_material(E=2.0e4, beta=300.0, nu=0.2, k=10.0, kappa0=1e-4, alpha=0.99,
                  c=4.0, R=0.05, eta=5.0, thickness=1.0, plane=PLANE_STRESS) -> Material:
    # coupling modulus h = E * 1e-9 (the paper's 1D parameter table, Fig. 10)
    return Material(E=E, nu=nu, kappa0=kappa0, alpha=alpha, beta=beta, c=c, R=R,
                    eta=eta, k=k, h=E * 1e-9, plane=plane, thickness=thickness)


# --------------------------------------------------------------------------
# the measured workloads
# --------------------------------------------------------------------------

def bar1d(nx: int = 100, lx: float = 100.0, u_end: float = 0.02, weak_elem: Optional[int] = None,
          weak_factor: float = 0.9, n_increments: int = 100, material: Optional[Material] = None) -> Problem:
    """1D bar in tension: left end fixed, right end displaced; one weakened element."""
    coords, conn = mesh_line2(nx, lx)
    e_scale = np.ones(nx)
    if weak_elem is None:
        weak_elem = nx // 2
    if weak_elem >= 0:
        e_scale[weak_elem] = weak_factor
    bn = np.array([0, nx], dtype=np.int64)
    bc_nodes = bn
    bc_comps = np.zeros(2, dtype=np.int64)
    bc_values = np.array([0.0, u_end])
    return Problem("bar1d_%d" % nx, 1, LINE2, (nx,), coords, conn, e_scale,
                   bc_nodes, bc_comps, bc_values, material or base_material(), n_increments)


def sen2d(nx: int = 200, ny: int = 100, lx: float = 200.0, ly: float = 100.0,
          notch_len: Optional[int] = None, notch_factor: float = 0.01, u_top: float = 0.1,
          n_increments: int = 200, material: Optional[Material] = None) -> Problem:
    """2D plane-stress single-edge-notched plate.

    The notch is a one-element-wide band of weakened elements at row ny/2,
    starting at the left edge.  Bottom edge fixed in x and y; top edge
    displaced in y, free in x.
    """
    coords, conn = mesh_quad4(nx, ny, lx, ly)
    if notch_len is None:
        notch_len = nx // 4
    e_scale = np.ones(nx * ny)
    jn = ny // 2
    e_scale[np.arange(notch_len) + nx * jn] = notch_factor
    bottom = np.arange(nx + 1, dtype=np.int64)
    top = np.arange(nx + 1, dtype=np.int64) + (nx + 1) * ny
    n0, c0, v0 = _bc(bottom, [0, 1], [0.0, 0.0])
    n1, c1, v1 = _bc(top, [1], [u_top])
    n = np.concatenate([n0, n1]); c = np.concatenate([c0, c1]); v = np.concatenate([v0, v1])
    order = np.lexsort((c, n))
    return Problem("sen2d_%dx%d" % (nx, ny), 2, QUAD4, (nx, ny), coords, conn, e_scale,
                   n[order], c[order], v[order], material or base_material(), n_increments)


def beam3d(nx: int = 128, ny: int = 32, nz: int = 16, lx: float = 400.0, ly: float = 100.0,
           lz: float = 50.0, notch_factor: float = 0.01, u_load: float = -0.5,
           n_increments: int = 150, material: Optional[Material] = None) -> Problem:
    """3D notched beam under three-point bending.

    Notch: centre-bottom block of elements spanning x in [lx/2 - w, lx/2 + w]
    (w = lx/128) and y in [0, ly/4], all z, with E scaled by notch_factor
    (2 x 8 x 16 elements on the 128 x 32 x 16 mesh).  Supports: the bottom
    node lines at x = 0 and x = lx, all z, pinned in x, y, z.  Load: the top
    node line at x = lx/2, all z, displaced in y.
    """
    assert nx % 2 == 0
    coords, conn = mesh_hex8(nx, ny, nz, lx, ly, lz)
    half_w = max(1, nx // 128)              # elements each side of the centre line
    i_lo, i_hi = nx // 2 - half_w, nx // 2 + half_w          # [i_lo, i_hi)
    j_hi = max(1, ny // 4)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i = i.ravel(); j = j.ravel()
    notch = (i >= i_lo) & (i < i_hi) & (j < j_hi)
    e_scale = np.where(notch, notch_factor, 1.0)
    node = lambda ii, jj, kk: ii + (nx + 1) * (jj + (ny + 1) * kk)
    ks = np.arange(nz + 1, dtype=np.int64)
    sup = np.concatenate([node(0, 0, ks), node(nx, 0, ks)])
    load = node(nx // 2, ny, ks)
    n0, c0, v0 = _bc(sup, [0, 1, 2], [0.0, 0.0, 0.0])
    n1, c1, v1 = _bc(load, [1], [u_load])
    n = np.concatenate([n0, n1]); c = np.concatenate([c0, c1]); v = np.concatenate([v0, v1])
    order = np.lexsort((c, n))
    return Problem("beam3d_%dx%dx%d" % (nx, ny, nz), 3, HEX8, (nx, ny, nz), coords, conn,
                   e_scale, n[order], c[order], v[order], material or base_material(), n_increments)


def bar1d_quadratic(nx: int = 100, lx: float = 100.0, u_end: float = 0.02,
                    weak_elem: Optional[int] = None, weak_factor: float = 0.9,
                    n_increments: int = 100, material: Optional[Material] = None) -> Problem:
    """The 1D bar of bar1d with quadratic u / linear ebar elements (Sec. 3.1)."""
    coords, conn = mesh_line3(nx, lx)
    e_scale = np.ones(nx)
    if weak_elem is None:
        weak_elem = nx // 2
    if weak_elem >= 0:
        e_scale[weak_elem] = weak_factor
    bc_nodes = np.array([0, 2 * nx], dtype=np.int64)
    return Problem("bar1dq_%d" % nx, 1, LINE3, (nx,), coords, conn, e_scale, bc_nodes,
                   np.zeros(2, dtype=np.int64), np.array([0.0, u_end]),
                   material or base_material(), n_increments)


def sen2d_quadratic(nx: int = 200, ny: int = 100, lx: float = 200.0, ly: float = 100.0,
                    notch_len: Optional[int] = None, notch_factor: float = 0.01, u_top: float = 0.1,
                    n_increments: int = 200, material: Optional[Material] = None) -> Problem:
    """The notched plate of sen2d with biquadratic u / bilinear ebar elements
    (Sec. 3.2): same notch band, bottom edge fixed, top edge displaced in y."""
    coords, conn = mesh_quad9(nx, ny, lx, ly)
    if notch_len is None:
        notch_len = nx // 4
    e_scale = np.ones(nx * ny)
    e_scale[np.arange(notch_len) + nx * (ny // 2)] = notch_factor
    nxn = 2 * nx + 1
    bottom = np.arange(nxn, dtype=np.int64)
    top = np.arange(nxn, dtype=np.int64) + nxn * (2 * ny)
    n0, c0, v0 = _bc(bottom, [0, 1], [0.0, 0.0])
    n1, c1, v1 = _bc(top, [1], [u_top])
    n = np.concatenate([n0, n1]); c = np.concatenate([c0, c1]); v = np.concatenate([v0, v1])
    order = np.lexsort((c, n))
    return Problem("sen2dq_%dx%d" % (nx, ny), 2, QUAD9, (nx, ny), coords, conn, e_scale,
                   n[order], c[order], v[order], material or base_material(), n_increments)


def config(name: str) -> Problem:
    """The named workloads.

    c0  1D bar, 100 line2, E = 20 GPa, centre element E x 0.9, 0.02 mm in 100 increments
    c1  2D plane-stress SEN plate 200 x 100 Q4, notch 50 elements E x 0.01, 0.1 mm in 200 increments
    c2  3D beam 128 x 32 x 16 hex8, 400 x 100 x 50 mm, 0.5 mm in 150 increments
    c3  3D beam 256 x 64 x 32 hex8 (mixed precision workload)
    c3p 3D beam 64 x 16 x 8 hex8 (parity subsample of c3)
    c0q the c0 bar with quadratic u / linear ebar elements (line3)
    c1q the c1 plate with biquadratic u / bilinear ebar elements (quad9)
    """
    if name == "c0":
        return bar1d()
    if name == "c1":
        return sen2d(material=base_material(nu=0.2, k=10.0))
    if name == "c2":
        return beam3d(128, 32, 16)
    if name == "c3":
        return beam3d(256, 64, 32)
    if name == "c3p":
        return beam3d(64, 16, 8)
    if name == "c0q":
        return bar1d_quadratic()
    if name == "c1q":
        return sen2d_quadratic(material=base_material(nu=0.2, k=10.0))
    raise KeyError(name)


# --------------------------------------------------------------------------
# serving stream (continuous batching workload)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    problem: Problem


def serving_stream(n_requests: int = 256, rate_per_s: float = 20.0, seed: int = 0,
                   nx_min: int = 40, nx_max: int = 400, inc_min: int = 50,
                   inc_max: int = 200, first_increments: Optional[int] = None) -> List[Request]:
    """Seeded stream of 2D notched-plate requests with Poisson arrivals.

    Per request, in this draw order from numpy's PCG64 (default_rng(seed)):
    inter-arrival ~ Exp(1/rate); nx uniform over even integers in
    [nx_min, nx_max] (ny = nx/2, plate fixed at 200 x 100 mm); notch fraction
    f ~ U[0.2, 0.5] (length round(f*nx) elements at row ny/2); E ~ U[2e4, 4e4]
    MPa; kappa0 ~ U[5e-5, 2e-4]; beta ~ U[100, 500]; c ~ U[1, 16] mm^2;
    R ~ U[0.005, 0.05]; increments ~ U{inc_min..inc_max}.  Fixed: nu = 0.2,
    alpha = 0.99, eta = 5, k = 10, top displacement 0.1 mm.  first_increments
    (short runs) keeps only the first increments of each request's load path
    (same step size, proportionally smaller final displacement).
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(n_requests):
        t += float(rng.exponential(1.0 / rate_per_s))
        nx = int(rng.integers(nx_min // 2, nx_max // 2 + 1)) * 2
        f = float(rng.uniform(0.2, 0.5))
        E = float(rng.uniform(2.0e4, 4.0e4))
        kappa0 = float(rng.uniform(5e-5, 2e-4))
        beta = float(rng.uniform(100.0, 500.0))
        c = float(rng.uniform(1.0, 16.0))
        R = float(rng.uniform(0.005, 0.05))
        n_inc = int(rng.integers(inc_min, inc_max + 1))
        mat = base_material(E=E, beta=beta, kappa0=kappa0, c=c, R=R)
        u_top, n_run = 0.1, n_inc
        if first_increments is not None and first_increments < n_inc:
            n_run = first_increments
            u_top = 0.1 * n_run / n_inc
        prob = sen2d(nx=nx, ny=nx // 2, notch_len=int(round(f * nx)), n_increments=n_run,
                     u_top=u_top, material=mat)
        prob.name = "req%03d_%dx%d" % (rid, nx, nx // 2)
        out.append(Request(rid, t, prob))
    return out


# --------------------------------------------------------------------------
# injected states (for parity of a single assembly at a chosen state)
# --------------------------------------------------------------------------

def injected_state(prob: Problem, seed: int, load: float = 1.0, noise: float = 0.25,
                   kappa_spread: float = 3.0, ebar_scale: float = 1.0):
    """A seeded state (x, kappa_n) shaped like a mid-load-path state.

    x: the prescribed boundary displacement at load factor `load`
    interpolated linearly through the body, times (1 + noise * U[-1, 1]) per
    dof, plus an ebar field in the same magnitude range as the strains.
    kappa_n: U[0, kappa_spread * kappa0] per Gauss point, so that points fall
    below and above the damage threshold.  ebar_scale scales the ebar field
    (small values keep every point below the threshold).  Returns
    (x [ndof], kappa_n [nel*ngp]).
    """
    rng = np.random.default_rng(seed)
    nd = prob.ndpn
    x = np.zeros(prob.ndof)
    L = prob.coords.max(axis=0) - prob.coords.min(axis=0)
    L = np.where(L > 0, L, 1.0)
    xi = (prob.coords - prob.coords.min(axis=0)) / L            # [0, 1]^dim
    umax = float(np.max(np.abs(prob.bc_values))) * load if prob.bc_values.size else 1e-3
    lref = float(np.max(L))
    for c in range(prob.dim):
        base = umax * xi[:, (c + 1) % prob.dim] * (1.0 if c % 2 == 0 else -0.5)
        x[c::nd] = base * (1.0 + noise * rng.uniform(-1, 1, prob.n_nodes)) \
            + noise * umax * rng.uniform(-1, 1, prob.n_nodes) * 0.1
    strain_scale = umax / lref
    x[prob.dim::nd] = ebar_scale * (strain_scale * rng.uniform(0.2, 2.5, prob.n_nodes)
                                    + prob.material.kappa0 * rng.uniform(0.0, 2.0, prob.n_nodes))
    if prob.elem_type in MIXED_ORDER:             # ebar lives on the vertices only
        keep = np.zeros(prob.n_nodes, dtype=bool)
        keep[prob.ebar_nodes()] = True
        x[prob.dim::nd][~keep] = 0.0
    dofs = prob.bc_dofs()
    x[dofs] = prob.bc_values * load
    kappa_n = prob.material.kappa0 * kappa_spread * rng.uniform(0.0, 1.0, prob.n_elems * prob.ngp)
    return x, kappa_n


def perturbed_coords(prob: Problem, seed: int, amp: float = 0.2) -> np.ndarray:
    """Interior nodes moved by up to amp * element size (distorted-mesh tests)."""
    rng = np.random.default_rng(seed)
    coords = prob.coords.copy()
    h = np.array([(coords[:, d].max() - coords[:, d].min()) / s for d, s in
                  zip(range(prob.dim), prob.shape)])
    lo = coords.min(axis=0); hi = coords.max(axis=0)
    interior = np.all((coords > lo + 1e-9) & (coords < hi - 1e-9), axis=1)
    coords[interior] += amp * h * rng.uniform(-1, 1, (int(interior.sum()), prob.dim))
    return coords
