// Mixed-order elements: quadratic displacement with linear micro-equivalent
// strain (Sec. 2.1, after Eqs. 9-10), the discretisation the paper runs in 1D
// (Sec. 3.1, 3-node lines) and 2D (Sec. 3.2, biquadratic u / bilinear ebar).
//
// Element: the displacement element's nodes (line3: left, right, midpoint;
// quad9: corners counter-clockwise from (-1, -1), mid-side nodes of the
// edges 0-1, 1-2, 2-3, 3-0, centre), the ebar element on its first 2^dim
// nodes (the vertices).  Geometry is interpolated by the quadratic element;
// 3-point Gauss-Legendre per direction, point g = i_xi + 3 i_eta.  The dof
// layout stays node-interleaved with dim + 1 dofs per node; the ebar dof of a
// node that is no element's vertex carries no unknown and is constrained to
// zero like a Dirichlet dof (identity row, zero column, zero residual).
//
// Kernel 1 (q_gp_kernel): one thread per Gauss point, the record of the
//   equal-order kernels (gp_state_record) with the weight w_g folded in.
// Kernel 2 (q_node_kernel): one lane group per node a, lane l owns the
//   neighbour at position l of a's row: for every element of a (ascending id)
//   that contains that neighbour, it sums the (dim+1)x(dim+1) block
//   d f_a / d x_b over the Gauss points (Eqs. 11a-11d with N_u, B_u quadratic
//   and N_e linear) and adds it to the running sum, in element order; lane 0
//   sums the internal force on a (Eqs. 11e-11f) the same way.  No atomics:
//   bitwise repeatable.  Per-workgroup norm partials as the equal-order
//   kernel writes them.
#include "gp_state.h"
#include "lgdm_internal.h"

namespace lgdm {

namespace {

template <int DIM> struct ElemQ {
  static constexpr int NEN = DIM == 1 ? 3 : 9;   // displacement nodes
  static constexpr int NENE = 1 << DIM;          // ebar nodes (the first NENE)
  static constexpr int NGP = DIM == 1 ? 3 : 9;
  static constexpr int ND = DIM + 1;
};

constexpr double GQ = 0.77459666924148337704;   // sqrt(3/5)

// reference coordinate in {-1, 0, 1} of local node a along direction d
template <int DIM> __device__ __forceinline__ int qnode(int a, int d) {
  if (DIM == 1) return a == 0 ? -1 : (a == 1 ? 1 : 0);
  if (a < 4) return d == 0 ? ((a == 1 || a == 2) ? 1 : -1) : (a >= 2 ? 1 : -1);
  if (a == 8) return 0;
  // mid-side nodes of the edges 0-1, 1-2, 2-3, 3-0
  const int m = a - 4;
  if (d == 0) return m == 1 ? 1 : (m == 3 ? -1 : 0);
  return m == 0 ? -1 : (m == 2 ? 1 : 0);
}

// Gauss point coordinate along d and the point's weight
template <int DIM> __device__ __forceinline__ double gq_coord(int g, int d) {
  const int i = d == 0 ? g % 3 : g / 3;
  return (double)(i - 1) * GQ;
}
template <int DIM> __device__ __forceinline__ double gq_weight(int g) {
  const double w0 = (g % 3 == 1) ? 8.0 / 9.0 : 5.0 / 9.0;
  if (DIM == 1) return w0;
  return w0 * ((g / 3 == 1) ? 8.0 / 9.0 : 5.0 / 9.0);
}

// 1D quadratic Lagrange function of the node at n in {-1, 0, 1}, at t
__device__ __forceinline__ void lag2(int n, double t, double& v, double& dv) {
  if (n < 0) {
    v = 0.5 * t * (t - 1.0);
    dv = t - 0.5;
  } else if (n > 0) {
    v = 0.5 * t * (t + 1.0);
    dv = t + 0.5;
  } else {
    v = 1.0 - t * t;
    dv = -2.0 * t;
  }
}

// displacement shape function N_a and dN_a / dxi at Gauss point g
template <int DIM> __device__ __forceinline__ void shape_u(int a, int g, double& N, double dN[DIM]) {
  double v[DIM], dv[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) lag2(qnode<DIM>(a, d), gq_coord<DIM>(g, d), v[d], dv[d]);
  N = 1.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) N *= v[d];
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    double p = dv[j];
#pragma unroll
    for (int d = 0; d < DIM; ++d)
      if (d != j) p *= v[d];
    dN[j] = p;
  }
}

// ebar shape function of local node a (zero unless a is a vertex) at g:
// N_a = prod_d (1 + n_a,d xi_d) / 2
template <int DIM> __device__ __forceinline__ void shape_e(int a, int g, double& N, double dN[DIM]) {
  if (a >= ElemQ<DIM>::NENE) {
    N = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) dN[d] = 0.0;
    return;
  }
  double v[DIM], dv[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const double n = (double)qnode<DIM>(a, d);
    v[d] = 0.5 * (1.0 + n * gq_coord<DIM>(g, d));
    dv[d] = 0.5 * n;
  }
  N = 1.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) N *= v[d];
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    double p = dv[j];
#pragma unroll
    for (int d = 0; d < DIM; ++d)
      if (d != j) p *= v[d];
    dN[j] = p;
  }
}

// ---------------------------------------------------------------------------
// Kernel 1: Gauss-point state and record
// ---------------------------------------------------------------------------
template <int DIM> __global__ void __launch_bounds__(256) q_gp_kernel(GpArgs A, MatParams mp) {
  using E = ElemQ<DIM>;
  using RC = Rec<DIM, false>;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= A.ngauss) return;
  const int64_t e = gid / E::NGP;
  const int g = (int)(gid - e * E::NGP);
  double J[DIM][DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d)
#pragma unroll
    for (int j = 0; j < DIM; ++j) J[d][j] = 0.0;
  double ue[E::NEN][DIM], dNu[E::NEN][DIM];
#pragma unroll
  for (int a = 0; a < E::NEN; ++a) {
    const int64_t n = A.conn[e * E::NEN + a];
    double N, dN[DIM];
    shape_u<DIM>(a, g, N, dN);
#pragma unroll
    for (int j = 0; j < DIM; ++j) dNu[a][j] = dN[j];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const double xd = A.coords[n * DIM + d];
#pragma unroll
      for (int j = 0; j < DIM; ++j) J[d][j] += xd * dN[j];
      ue[a][d] = A.x[n * E::ND + d];
    }
  }
  double Ji[DIM][DIM];
  double detJ;
  if (DIM == 1) {
    detJ = J[0][0];
    Ji[0][0] = 1.0 / detJ;
  } else {
    detJ = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double r = 1.0 / detJ;
    Ji[0][0] = J[1][1] * r;
    Ji[0][1] = -J[0][1] * r;
    Ji[1][0] = -J[1][0] * r;
    Ji[1][1] = J[0][0] * r;
  }
  // displacement gradient from the quadratic element
  double gu[DIM][DIM];
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int d = 0; d < DIM; ++d) gu[i][d] = 0.0;
#pragma unroll
  for (int a = 0; a < E::NEN; ++a) {
    double gx[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < DIM; ++j) s += dNu[a][j] * Ji[j][d];
      gx[d] = s;
    }
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
      for (int d = 0; d < DIM; ++d) gu[i][d] += ue[a][i] * gx[d];
  }
  double eps[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int j = 0; j < DIM; ++j) eps[i][j] = 0.5 * (gu[i][j] + gu[j][i]);
  if (DIM == 2) eps[2][2] = mp.ezz_fac * (eps[0][0] + eps[1][1]);
  // micro-equivalent strain and its gradient from the linear element
  double ebar = 0.0, gb[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) gb[d] = 0.0;
#pragma unroll
  for (int a = 0; a < E::NENE; ++a) {
    const int64_t n = A.conn[e * E::NEN + a];
    const double eb = A.x[n * E::ND + DIM];
    double N, dN[DIM];
    shape_e<DIM>(a, g, N, dN);
    ebar += N * eb;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < DIM; ++j) s += dN[j] * Ji[j][d];
      gb[d] += eb * s;
    }
  }
  double kap, D, eeq;
  gp_state_record<DIM, false>(eps, ebar, gb, Ji, gq_weight<DIM>(g) * detJ * mp.thick, A.e_scale[e],
                              A.kappa_n[gid], mp, A.rec + gid * RC::STRIDE, kap, D, eeq);
  A.kappa_t[gid] = kap;
  A.D_t[gid] = D;
  A.eeq_t[gid] = eeq;
}

// ---------------------------------------------------------------------------
// the block d f_a / d x_b and the force on a at one Gauss point
// ---------------------------------------------------------------------------
template <int DIM>
__device__ __forceinline__ void q_block_force(const double* __restrict__ r, int g, int la, int lb,
                                              const MatParams& mp, bool want_k, bool want_f,
                                              double blk[DIM + 1][DIM + 1], double fa[DIM + 2]) {
  using RC = Rec<DIM, false>;
  double Nua, Nub, Nea, Neb, dua[DIM], dub[DIM], dea[DIM], deb[DIM];
  shape_u<DIM>(la, g, Nua, dua);
  shape_u<DIM>(lb, g, Nub, dub);
  shape_e<DIM>(la, g, Nea, dea);
  shape_e<DIM>(lb, g, Neb, deb);
  double ga[DIM], gbv[DIM], ea[DIM], eb[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      const double jv = r[RC::JINV + j * DIM + d];
      s0 += dua[j] * jv;
      s1 += dub[j] * jv;
      s2 += dea[j] * jv;
      s3 += deb[j] * jv;
    }
    ga[d] = s0;
    gbv[d] = s1;
    ea[d] = s2;
    eb[d] = s3;
  }
  double Sga[DIM];
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) s += r[RC::S + sym_idx<DIM>(i, j)] * ga[j];
    Sga[i] = s;
  }
  double ea_geb = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) ea_geb += ea[d] * r[RC::GB + d];
  if (want_f) {
#pragma unroll
    for (int i = 0; i < DIM; ++i) fa[i] += r[RC::CUU] * Sga[i];
    fa[DIM] += r[RC::RE] * Nea + r[RC::CG] * ea_geb;
    fa[DIM + 1] += r[RC::FR] * Nea;
  }
  if (!want_k) return;
  // uu entries accumulate A = sum_g (1 - D) s_e wJ grad N_a (x) grad N_b;
  // q_finish_uu forms K^uu_ab = lam A + mu A^T + mu tr(A) I (1D: E A)
  const double cuu = r[RC::CUU];
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    const double ca = cuu * ga[i];
#pragma unroll
    for (int j = 0; j < DIM; ++j) blk[i][j] += ca * gbv[j];
  }
  const double cueN = r[RC::CUE] * Neb;
#pragma unroll
  for (int i = 0; i < DIM; ++i) blk[i][DIM] -= cueN * Sga[i];
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    double gg = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) gg += r[RC::GH + sym_idx<DIM>(j, i)] * gbv[i];
    blk[DIM][j] -= Nea * gg;
  }
  double eab = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) eab += ea[d] * eb[d];
  blk[DIM][DIM] += r[RC::CEE] * Nea * Neb + r[RC::CGP] * ea_geb * Neb + r[RC::CG] * eab;
}

template <int DIM> __device__ __forceinline__ void q_finish_uu(double blk[DIM + 1][DIM + 1], const MatParams& mp) {
  if (DIM == 1) {
    blk[0][0] *= mp.E;
    return;
  }
  double a[DIM][DIM], tr = 0.0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    tr += blk[i][i];
#pragma unroll
    for (int j = 0; j < DIM; ++j) a[i][j] = blk[i][j];
  }
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int j = 0; j < DIM; ++j) blk[i][j] = mp.lam * a[i][j] + mp.mu * a[j][i] + (i == j ? mp.mu * tr : 0.0);
}

// ---------------------------------------------------------------------------
// Kernel 2: node-row assembly
// ---------------------------------------------------------------------------
constexpr int QBLOCK = 256;
template <int DIM> struct QNode {
  static constexpr int L = DIM == 1 ? 8 : 32;   // lanes per node: at least the neighbours (5 / 25)
  static constexpr int NPB = QBLOCK / L;        // nodes per workgroup
};

template <int DIM, typename T, bool WANT_K>
__global__ void __launch_bounds__(QBLOCK) q_node_kernel(NodeArgs A, MatParams mp) {
  using E = ElemQ<DIM>;
  using RC = Rec<DIM, false>;
  constexpr int NEN = E::NEN, ND = E::ND, NGP = E::NGP, L = QNode<DIM>::L, NPB = QNode<DIM>::NPB;
  __shared__ double s_red[NORM_SLOTS][NPB];
  const int tid = threadIdx.x;
  const int slot = tid / L, l = tid % L;
  const int64_t a = (int64_t)blockIdx.x * NPB + slot;
  const bool valid = a < A.n_nodes;
  int e0 = 0, ne = 0, nb0 = 0, nnb = 0;
  if (valid) {
    e0 = A.n2e_ptr[a];
    ne = A.n2e_ptr[a + 1] - e0;
    nb0 = A.nbr_ptr[a];
    nnb = A.nbr_ptr[a + 1] - nb0;
  }
  // tangent: lane l, the neighbour at position l
  if (WANT_K && valid && l < nnb) {
    double acc[ND][ND];
#pragma unroll
    for (int i = 0; i < ND; ++i)
#pragma unroll
      for (int j = 0; j < ND; ++j) acc[i][j] = 0.0;
    for (int k = 0; k < ne; ++k) {
      const int ent = A.n2e[e0 + k];
      const int64_t e = ent >> N2E_SHIFT;
      const int la = ent & N2E_MASK;
      int lb = -1;
      for (int b = 0; b < NEN; ++b)
        if (A.pos[(e * NEN + la) * NEN + b] == l) lb = b;
      if (lb < 0) continue;
      double blk[ND][ND], f[DIM + 2];
#pragma unroll
      for (int i = 0; i < ND; ++i)
#pragma unroll
        for (int j = 0; j < ND; ++j) blk[i][j] = 0.0;
      for (int g = 0; g < NGP; ++g)
        q_block_force<DIM>(A.rec + (e * NGP + g) * RC::STRIDE, g, la, lb, mp, true, false, blk, f);
      q_finish_uu<DIM>(blk, mp);
#pragma unroll
      for (int i = 0; i < ND; ++i)
#pragma unroll
        for (int j = 0; j < ND; ++j) acc[i][j] += blk[i][j];
    }
    const int64_t nbn = A.nbr[nb0 + l];
    const int64_t rb = A.row_ptr[a * ND];
    const int64_t rowlen = (int64_t)nnb * ND;
    T* __restrict__ vals = static_cast<T*>(A.vals);
#pragma unroll
    for (int r = 0; r < ND; ++r) {
      const int64_t row = a * ND + r;
      const bool rd = A.flags[row] & 1;
#pragma unroll
      for (int c = 0; c < ND; ++c) {
        const int64_t col = nbn * ND + c;
        double v = acc[r][c];
        if (rd)
          v = (col == row) ? 1.0 : 0.0;
        else if (A.flags[col] & 1)
          v = 0.0;
        vals[rb + r * rowlen + (int64_t)l * ND + c] = (T)v;
      }
    }
  }
  // residual R = -f_int (0 on constrained rows) and norm partials
  double red[NORM_SLOTS] = {0, 0, 0, 0, 0, 0};
  if (valid && l == 0) {
    double facc[DIM + 2];
#pragma unroll
    for (int i = 0; i < DIM + 2; ++i) facc[i] = 0.0;
    for (int k = 0; k < ne; ++k) {
      const int ent = A.n2e[e0 + k];
      const int64_t e = ent >> N2E_SHIFT;
      const int la = ent & N2E_MASK;
      double f[DIM + 2], blk[ND][ND];
#pragma unroll
      for (int i = 0; i < DIM + 2; ++i) f[i] = 0.0;
      for (int g = 0; g < NGP; ++g)
        q_block_force<DIM>(A.rec + (e * NGP + g) * RC::STRIDE, g, la, la, mp, false, true, blk, f);
#pragma unroll
      for (int i = 0; i < DIM + 2; ++i) facc[i] += f[i];
    }
#pragma unroll
    for (int r = 0; r < ND; ++r) {
      const int64_t row = a * ND + r;
      const uint8_t fl = A.flags[row];
      const double fv = facc[r];
      const double rv = (fl & 1) ? 0.0 : -fv;
      A.R[row] = rv;
      if (r < DIM) {
        red[0] += rv * rv;
        red[2] += fv * fv;
        if (fl & 2) red[4] += fv;
      } else {
        red[1] += rv * rv;
      }
      if (!isfinite(fv)) red[5] += 1.0;
    }
    red[3] += facc[DIM + 1] * facc[DIM + 1];
  }
  if (l == 0) {
#pragma unroll
    for (int q = 0; q < NORM_SLOTS; ++q) s_red[q][slot] = red[q];
  }
  __syncthreads();
  if (tid < NORM_SLOTS) {
    double sum = 0.0;
    for (int i = 0; i < NPB; ++i) sum += s_red[tid][i];
    A.partials[blockIdx.x * NORM_SLOTS + tid] = sum;
  }
}

// element blocks for parity checks: one thread per (element, a, b), the
// node-interleaved local layout of the equal-order elements
template <int DIM>
__global__ void q_element_blocks_kernel(int64_t e0, int64_t e1, const double* __restrict__ rec, MatParams mp,
                                        double* __restrict__ Ke, double* __restrict__ fe) {
  using E = ElemQ<DIM>;
  using RC = Rec<DIM, false>;
  constexpr int NEN = E::NEN, ND = E::ND, NL = NEN * ND;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ne = e1 - e0;
  if (t >= ne * NEN * NEN) return;
  const int64_t el = t / (NEN * NEN);
  const int la = (int)((t / NEN) % NEN), lb = (int)(t % NEN);
  const int64_t e = e0 + el;
  double blk[ND][ND], f[DIM + 2];
#pragma unroll
  for (int i = 0; i < ND; ++i)
#pragma unroll
    for (int j = 0; j < ND; ++j) blk[i][j] = 0.0;
#pragma unroll
  for (int i = 0; i < DIM + 2; ++i) f[i] = 0.0;
  for (int g = 0; g < E::NGP; ++g)
    q_block_force<DIM>(rec + (e * E::NGP + g) * RC::STRIDE, g, la, lb, mp, Ke != nullptr, lb == 0, blk, f);
  q_finish_uu<DIM>(blk, mp);
  if (Ke) {
    double* out = Ke + el * NL * NL;
#pragma unroll
    for (int i = 0; i < ND; ++i)
#pragma unroll
      for (int j = 0; j < ND; ++j) out[(la * ND + i) * NL + lb * ND + j] = blk[i][j];
  }
  if (fe && lb == 0) {
#pragma unroll
    for (int i = 0; i < ND; ++i) fe[el * NL + la * ND + i] = f[i];
  }
}

__global__ void zero_flagged_kernel(int64_t n, const uint8_t* __restrict__ flags, uint8_t mask,
                                    double* __restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && (flags[i] & mask)) v[i] = 0.0;
}

}  // namespace

hipError_t launch_zero_flagged(lgdm_ctx* c, double* v, uint8_t mask) {
  const int64_t grid = (c->ndof + 255) / 256;
  if (grid == 0) return hipSuccess;
  zero_flagged_kernel<<<grid, 256, 0, c->stream>>>(c->ndof, c->dof_flags, mask, v);
  return hipGetLastError();
}

int q_node_kernel_nodes_per_block(int dim) { return dim == 1 ? QNode<1>::NPB : QNode<2>::NPB; }

hipError_t launch_q_gp_kernel(lgdm_ctx* c, const MatParams& mp) {
  const int64_t grid = (c->ngauss + 255) / 256;
  if (grid == 0) return hipSuccess;
  const GpArgs A = gp_args(c);
  if (c->dim == 1) q_gp_kernel<1><<<grid, 256, 0, c->stream>>>(A, mp);
  else q_gp_kernel<2><<<grid, 256, 0, c->stream>>>(A, mp);
  return hipGetLastError();
}

hipError_t launch_q_node_kernel(lgdm_ctx* c, const MatParams& mp, bool want_k) {
  const int64_t grid = node_kernel_blocks(c);
  if (grid == 0) return hipSuccess;
  const NodeArgs A = node_args(c);
  const bool mixed = c->precision == LGDM_MIXED;
  if (c->dim == 1) {
    if (!want_k) q_node_kernel<1, double, false><<<grid, QBLOCK, 0, c->stream>>>(A, mp);
    else if (mixed) q_node_kernel<1, float, true><<<grid, QBLOCK, 0, c->stream>>>(A, mp);
    else q_node_kernel<1, double, true><<<grid, QBLOCK, 0, c->stream>>>(A, mp);
  } else {
    if (!want_k) q_node_kernel<2, double, false><<<grid, QBLOCK, 0, c->stream>>>(A, mp);
    else if (mixed) q_node_kernel<2, float, true><<<grid, QBLOCK, 0, c->stream>>>(A, mp);
    else q_node_kernel<2, double, true><<<grid, QBLOCK, 0, c->stream>>>(A, mp);
  }
  return hipGetLastError();
}

hipError_t launch_q_element_blocks(lgdm_ctx* c, const MatParams& mp, int64_t e0, int64_t e1, double* Ke,
                                   double* fe) {
  const int64_t n = (e1 - e0) * c->nen * c->nen;
  const int64_t grid = (n + 255) / 256;
  if (grid == 0) return hipSuccess;
  if (c->dim == 1) q_element_blocks_kernel<1><<<grid, 256, 0, c->stream>>>(e0, e1, c->rec, mp, Ke, fe);
  else q_element_blocks_kernel<2><<<grid, 256, 0, c->stream>>>(e0, e1, c->rec, mp, Ke, fe);
  return hipGetLastError();
}

}  // namespace lgdm
