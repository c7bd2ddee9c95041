// Gauss-point evaluation (H1-H2) and deterministic node-row assembly of the
// element tangents and internal forces (H3-H5) of the localizing gradient
// damage method.
//
// Kernel 1 (gp_kernel): one thread per Gauss point.  Gathers the element's
//   coordinates and nodal (u, ebar), evaluates the Jacobian, the strain, the
//   modified von Mises equivalent strain and its gradient (Eq. A.3), the
//   micro-equivalent strain and its gradient, the history update (Eq. A.2 as
//   the vectorised condition of Fig. 8b), damage (Eq. A.1) and interaction
//   function (Eq. A.4), and writes a compact record of the Gauss point (J^-1
//   and the scalar / tensor coefficients of Eqs. 11a-11f).
//
// Kernel 2 (node_kernel): one lane group per node a.  Lane (k, b) takes the
//   k-th element adjacent to a (ascending element id) and the element's local
//   node b and sums over the Gauss points the (dim+1)x(dim+1) block
//   d f_a / d x_b of Eqs. 11a-11d; the lane of b = 0 also sums the element's
//   internal force on node a (Eqs. 11e-11f).  The blocks are reduced per
//   neighbour position in ascending element order through LDS and written
//   once into the CSR row block of node a (no atomics, bitwise repeatable),
//   with identity rows / zero columns for Dirichlet dofs.  Per-workgroup
//   partial sums of the residual norms follow in a fixed order.
//
// Element law (readings of the paper shared with its executed code, Fig. 2):
//   sigma = (1 - D) s_e C : eps, f_u = int B^T sigma,
//   f_ebar = int N h (ebar - eeq) + grad N . (g h c grad ebar),
//   K^uu = int (1-D) s_e [lam dN_a (x) dN_b + mu dN_b (x) dN_a + mu (dN_a.dN_b) I],
//   K^ue = -int (s_e C:eps dN_a) D' chi N_b,   K^eu = -int N_a h (G dN_b),
//   K^ee = int h N_a N_b + h c g' D' chi (dN_a . grad ebar) N_b + g h c dN_a . dN_b.
#include <cmath>

#include "gp_state.h"
#include "lgdm_internal.h"

namespace lgdm {

namespace {

template <int DIM> struct Elem {
  static constexpr int NEN = 1 << DIM;
  static constexpr int NGP = 1 << DIM;
  static constexpr int ND = DIM + 1;
};

// sign bits of the reference node (bit d set where xi_a,d = +1); the Gauss
// point index g = i_xi + 2 i_eta + 4 i_zeta has bit d set where xi_g,d = +1/sqrt(3)
template <int DIM> __device__ __forceinline__ int node_bits(int a) {
  if (DIM == 1) return a;
  const int x = (a & 1) ^ ((a >> 1) & 1), y = (a >> 1) & 1;
  return DIM == 2 ? (x | (y << 1)) : (x | (y << 1) | (a & 4));
}

// N_a(xi_g) and dN_a/dxi(xi_g) from the factor (1 + xi_a,d xi_g,d)/2, which
// takes (1 +- 1/sqrt(3))/2 when the signs agree / differ
template <int DIM, typename T>
__device__ __forceinline__ void shape_fast(int a, int g, T& N, T dN[DIM]) {
  const T cp = (T)0.78867513459481288225, cm = (T)0.21132486540518711775;
  const int ab = node_bits<DIM>(a);
  T f[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) f[d] = (((ab ^ g) >> d) & 1) ? cm : cp;
  N = (T)1;
#pragma unroll
  for (int d = 0; d < DIM; ++d) N *= f[d];
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    T p = ((ab >> j) & 1) ? (T)0.5 : (T)-0.5;
#pragma unroll
    for (int d = 0; d < DIM; ++d)
      if (d != j) p *= f[d];
    dN[j] = p;
  }
}

// ---------------------------------------------------------------------------
// Kernel 1: Gauss-point state and record
// ---------------------------------------------------------------------------
template <int DIM, bool CPL>
__device__ __forceinline__ void gp_point(int64_t gid, const GpArgs& A, const MatParams& mp) {
  using E = Elem<DIM>;
  using RC = Rec<DIM, CPL>;
  if (gid >= A.ngauss) return;
  const double* __restrict__ coords = A.coords;
  const int32_t* __restrict__ conn = A.conn;
  const double* __restrict__ e_scale = A.e_scale;
  const double* __restrict__ x = A.x;
  const double* __restrict__ kappa_n = A.kappa_n;
  double* __restrict__ rec = A.rec;
  double* __restrict__ kappa_t = A.kappa_t;
  double* __restrict__ D_t = A.D_t;
  const int64_t e = gid / E::NGP;
  const int g = (int)(gid - e * E::NGP);

  double xe[E::NEN][DIM], ue[E::NEN][DIM], eb[E::NEN];
#pragma unroll
  for (int a = 0; a < E::NEN; ++a) {
    const int64_t n = conn[e * E::NEN + a];
#pragma unroll
    for (int d = 0; d < DIM; ++d) xe[a][d] = coords[n * DIM + d];
#pragma unroll
    for (int i = 0; i < DIM; ++i) ue[a][i] = x[n * E::ND + i];
    eb[a] = x[n * E::ND + DIM];
  }
  double N[E::NEN], dNx[E::NEN][DIM];
  double J[DIM][DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d)
#pragma unroll
    for (int j = 0; j < DIM; ++j) J[d][j] = 0.0;
#pragma unroll
  for (int a = 0; a < E::NEN; ++a) {
    double dN[DIM];
    shape_fast<DIM, double>(a, g, N[a], dN);
#pragma unroll
    for (int j = 0; j < DIM; ++j) dNx[a][j] = dN[j];  // reference gradient for now
#pragma unroll
    for (int d = 0; d < DIM; ++d)
#pragma unroll
      for (int j = 0; j < DIM; ++j) J[d][j] += xe[a][d] * dN[j];
  }
  // J^-1 with (J^-1)_{j d} = d xi_j / d x_d
  double Ji[DIM][DIM];
  double detJ;
  if (DIM == 1) {
    detJ = J[0][0];
    Ji[0][0] = 1.0 / detJ;
  } else if (DIM == 2) {
    detJ = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double r = 1.0 / detJ;
    Ji[0][0] = J[1][1] * r;
    Ji[0][1] = -J[0][1] * r;
    Ji[1][0] = -J[1][0] * r;
    Ji[1][1] = J[0][0] * r;
  } else {
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    detJ = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    const double r = 1.0 / detJ;
    // inverse of J (rows j = xi index, cols d = x index)
    Ji[0][0] = c00 * r;
    Ji[1][0] = c01 * r;
    Ji[2][0] = c02 * r;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * r;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * r;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * r;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * r;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * r;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * r;
  }
  // physical gradients dN_a/dx_d = sum_j dN_a/dxi_j (J^-1)_{j d}
#pragma unroll
  for (int a = 0; a < E::NEN; ++a) {
    double t[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < DIM; ++j) s += dNx[a][j] * Ji[j][d];
      t[d] = s;
    }
#pragma unroll
    for (int d = 0; d < DIM; ++d) dNx[a][d] = t[d];
  }
  // displacement gradient, small strain tensor
  double gu[DIM][DIM];
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < E::NEN; ++a) s += ue[a][i] * dNx[a][d];
      gu[i][d] = s;
    }
  double eps[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int j = 0; j < DIM; ++j) eps[i][j] = 0.5 * (gu[i][j] + gu[j][i]);
  if (DIM == 2) eps[2][2] = mp.ezz_fac * (eps[0][0] + eps[1][1]);

  // micro-equivalent strain and its gradient at the Gauss point
  double ebar = 0.0, gb[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) gb[d] = 0.0;
#pragma unroll
  for (int a = 0; a < E::NEN; ++a) {
    ebar += N[a] * eb[a];
#pragma unroll
    for (int d = 0; d < DIM; ++d) gb[d] += eb[a] * dNx[a][d];
  }
  double kap, D, eeq;
  gp_state_record<DIM, CPL>(eps, ebar, gb, Ji, detJ * mp.thick, e_scale[e], kappa_n[gid], mp,
                            rec + gid * RC::STRIDE, kap, D, eeq);
  kappa_t[gid] = kap;
  D_t[gid] = D;
  A.eeq_t[gid] = eeq;
}

template <int DIM, bool CPL>
__global__ void __launch_bounds__(256) gp_kernel(GpArgs A, MatParams mp) {
  gp_point<DIM, CPL>((int64_t)blockIdx.x * blockDim.x + threadIdx.x, A, mp);
}

// slot of workgroup b in a fused launch (slot ranges ascending by first block)
__device__ __forceinline__ int find_slot(const SlotDesc* __restrict__ slots, int nslots, int64_t b,
                                         bool node) {
  int lo = 0, hi = nslots - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int64_t b0 = node ? slots[mid].node_block0 : slots[mid].gp_block0;
    if (b0 <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int DIM>
__global__ void __launch_bounds__(256) gp_fused_kernel(const SlotDesc* __restrict__ slots, int nslots) {
  const int s = find_slot(slots, nslots, blockIdx.x, false);
  const int64_t lb = (int64_t)blockIdx.x - slots[s].gp_block0;
  gp_point<DIM, false>(lb * blockDim.x + threadIdx.x, slots[s].gp, slots[s].mp);
}

// ---------------------------------------------------------------------------
// per-Gauss-point pieces of the node-row assembly
// ---------------------------------------------------------------------------
// record fields in registers in precision T (16-byte loads; records are
// 16-byte aligned)
template <int DIM, bool CPL, typename T>
__device__ __forceinline__ void load_rec(const double* __restrict__ rv, T (&rr)[(Rec<DIM, CPL>::USED + 1) & ~1]) {
  constexpr int RU = (Rec<DIM, CPL>::USED + 1) & ~1;
#pragma unroll
  for (int i = 0; i < RU; i += 2) {
    const double2 t = *reinterpret_cast<const double2*>(rv + i);
    rr[i] = (T)t.x;
    rr[i + 1] = (T)t.y;
  }
}

// gradient of N_a at Gauss point g from the record's J^-1
template <int DIM, typename T>
__device__ __forceinline__ void grad_n(const T* r, const T dNxi[DIM], T out[DIM]) {
  using RC = Rec<DIM>;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    T s = 0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) s += dNxi[j] * r[RC::JINV + j * DIM + d];
    out[d] = s;
  }
}

// Coupling variant (the stress of Eq. 2): adds h (eeq - ebar) G grad N_a to
// the internal force, -h (G grad N_a) N_b to K^{u ebar} (Eq. 11b as
// printed) and h [(G grad N_a)(G grad N_b)^T + (eeq - ebar) d^2 eeq] to K^uu,
// the linearisation of Eq. 2 (G = d eeq / d eps).  The strain variation of
// u_i at node a is sym(e_i (x) grad N_a), plus f (grad N_a)_i e_z (x) e_z in
// plane stress (f = ezz_fac), so with t_a = (1 + f) grad N_a:
//   tr = t_a,i,   d_a : d_b = (delta_ik ga.gb + ga_k gb_i) / 2 + f^2 ga_i gb_k,
//   q : d_a = (q ga)_i + f q_zz ga_i,
//   d_a : d^2 eeq : d_b = al (2 c2^2 tr_a tr_b + c3 (d_a : d_b - tr_a tr_b / 3))
//                         - be (q : d_a)(q : d_b).
template <int DIM, typename T>
__device__ __forceinline__ void coupling_terms(const double* r, const double ga[DIM], const double gb[DIM],
                                               double Nb, const MatParams& mp, bool want_k, bool want_f,
                                               T blk[DIM + 1][DIM + 1], double fa[DIM + 2]) {
  using RC = Rec<DIM, true>;
  double Gga[DIM], Ggb[DIM];
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    double sa = 0.0, sb = 0.0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      sa += r[RC::GU + sym_idx<DIM>(i, j)] * ga[j];
      sb += r[RC::GU + sym_idx<DIM>(i, j)] * gb[j];
    }
    Gga[i] = sa;
    Ggb[i] = sb;
  }
  const double ec = -r[RC::RE];   // wJ h (eeq - ebar)
  if (want_f) {
#pragma unroll
    for (int i = 0; i < DIM; ++i) fa[i] += ec * Gga[i];
  }
  if (!want_k) return;
  const double cee = r[RC::CEE];  // wJ h
#pragma unroll
  for (int i = 0; i < DIM; ++i) blk[i][DIM] -= (T)(cee * Gga[i] * Nb);
  double qa[DIM], qb[DIM];
  const double f = DIM == 2 ? mp.ezz_fac : 0.0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    double sa = 0.0, sb = 0.0;
    if (DIM == 3) {
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        sa += r[RC::Q + sym_idx<3>(i, j)] * ga[j];
        sb += r[RC::Q + sym_idx<3>(i, j)] * gb[j];
      }
    } else if (DIM == 2) {
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        sa += r[RC::Q + sym_idx<2>(i, j)] * ga[j];
        sb += r[RC::Q + sym_idx<2>(i, j)] * gb[j];
      }
      sa += f * r[RC::Q + 3] * ga[i];
      sb += f * r[RC::Q + 3] * gb[i];
    }
    qa[i] = sa;
    qb[i] = sb;
  }
  const double al = r[RC::AL], be = r[RC::BE];
  const double c22 = 2.0 * mp.c2 * mp.c2, c3 = mp.c3, t1 = (1.0 + f) * (1.0 + f);
  double dab = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) dab += ga[d] * gb[d];
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const double trtr = t1 * ga[i] * gb[k];
      const double dd = 0.5 * ((i == k ? dab : 0.0) + ga[k] * gb[i]) + f * f * ga[i] * gb[k];
      const double hess = al * (c22 * trtr + c3 * (dd - trtr / 3.0)) - be * qa[i] * qb[k];
      blk[i][k] += (T)(cee * Gga[i] * Ggb[k] + ec * hess);
    }
}

// tangent block d f_a / d x_b and (want_f) the internal force on node a of
// one element at Gauss point g: one read of the record serves both;
// gradients in FP64, block arithmetic in the working precision T.
//
// Displacement block: with A = sum_g (1 - D) s_e wJ grad N_a (x) grad N_b,
// K^uu_ab = lam A + mu A^T + mu tr(A) I (Eq. 11a for an isotropic C), so the
// Gauss-point loop accumulates A in the block's uu entries (one product per
// entry) and finish_uu applies lam / mu once after the loop.  The coupling
// variant adds its own uu terms per Gauss point and keeps the direct form.
template <int DIM, typename T, bool CPL>
__device__ __forceinline__ void block_and_force(const double* __restrict__ rv, int g, int la, int lb,
                                                const MatParams& mp, bool want_k, bool want_f,
                                                T blk[DIM + 1][DIM + 1], double fa[DIM + 2]) {
  using RC = Rec<DIM, CPL>;
  double r[(RC::USED + 1) & ~1];
  load_rec<DIM, CPL, double>(rv, r);
  double Na, Nb, dNa[DIM], dNb[DIM], ga[DIM], gbv[DIM];
  shape_fast<DIM, double>(la, g, Na, dNa);
  shape_fast<DIM, double>(lb, g, Nb, dNb);
  grad_n<DIM, double>(r, dNa, ga);
  grad_n<DIM, double>(r, dNb, gbv);
  double Sga[DIM];
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) s += r[RC::S + sym_idx<DIM>(i, j)] * ga[j];
    Sga[i] = s;
  }
  double ga_geb = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) ga_geb += ga[d] * r[RC::GB + d];
  if (want_f) {
#pragma unroll
    for (int i = 0; i < DIM; ++i) fa[i] += r[RC::CUU] * Sga[i];
    fa[DIM] += r[RC::RE] * Na + r[RC::CG] * ga_geb;
    fa[DIM + 1] += r[RC::FR] * Na;
  }
  if (!want_k) {
    if constexpr (CPL) coupling_terms<DIM, T>(r, ga, gbv, Nb, mp, false, want_f, blk, fa);
    return;
  }
  const T cuu = (T)r[RC::CUU];
  T ta[DIM], tb[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    ta[d] = (T)ga[d];
    tb[d] = (T)gbv[d];
  }
  T dab = 0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) dab += ta[d] * tb[d];
  if constexpr (!CPL) {
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      const T ca = cuu * ta[i];
#pragma unroll
      for (int j = 0; j < DIM; ++j) blk[i][j] += ca * tb[j];
    }
  } else if (DIM == 1) {
    blk[0][0] += cuu * (T)mp.E * ta[0] * tb[0];
  } else {
    const T lam = (T)mp.lam, mu = (T)mp.mu;
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
      for (int j = 0; j < DIM; ++j)
        blk[i][j] += cuu * (lam * ta[i] * tb[j] + mu * ta[j] * tb[i] + (i == j ? mu * dab : (T)0));
  }
  const T cueN = (T)r[RC::CUE] * (T)Nb;
#pragma unroll
  for (int i = 0; i < DIM; ++i) blk[i][DIM] -= cueN * (T)Sga[i];
  const T tNa = (T)Na;
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    T gg = 0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) gg += (T)r[RC::GH + sym_idx<DIM>(j, i)] * tb[i];
    blk[DIM][j] -= tNa * gg;
  }
  blk[DIM][DIM] += (T)r[RC::CEE] * tNa * (T)Nb + (T)r[RC::CGP] * (T)ga_geb * (T)Nb + (T)r[RC::CG] * dab;
  if constexpr (CPL) coupling_terms<DIM, T>(r, ga, gbv, Nb, mp, want_k, want_f, blk, fa);
}

// after the Gauss-point loop: K^uu_ab = lam A + mu A^T + mu tr(A) I from the
// accumulated A (1D: E A); the coupling variant's blocks are already final
template <int DIM, typename T, bool CPL>
__device__ __forceinline__ void finish_uu(T blk[DIM + 1][DIM + 1], const MatParams& mp) {
  if constexpr (CPL) return;
  if (DIM == 1) {
    blk[0][0] *= (T)mp.E;
    return;
  }
  T a[DIM][DIM];
  T tr = 0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    tr += blk[i][i];
#pragma unroll
    for (int j = 0; j < DIM; ++j) a[i][j] = blk[i][j];
  }
  const T lam = (T)mp.lam, mu = (T)mp.mu;
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int j = 0; j < DIM; ++j) blk[i][j] = lam * a[i][j] + mu * a[j][i] + (i == j ? mu * tr : (T)0);
}

// ---------------------------------------------------------------------------
// Kernel 2: node-row assembly
// ---------------------------------------------------------------------------
constexpr int NODE_BLOCK = 256;

// T: type of the stored CSR values.  The blocks are always formed and summed
// in FP64 and rounded once at the store: FP32 arithmetic would leave absolute
// errors of ~1e-7 of the largest entry in every entry (rigid-body and
// bending modes of the assembled tangent are no longer annihilated to that
// level), which on slender meshes is the size of the smallest eigenvalues.
template <int DIM, typename T, bool CPL> struct NodeLds {
  using E = Elem<DIM>;
  static constexpr int NEN = E::NEN, NGP = E::NGP, ND = E::ND, NB = ND * ND;
  static constexpr int L = NEN * NEN;                 // lanes per node
  static constexpr int NPB = NODE_BLOCK / L;          // nodes per workgroup
  static constexpr int RS = Rec<DIM, CPL>::STRIDE;
  static constexpr int GS = RS + 2;                   // per Gauss point (even: 16-byte aligned)
  // rounds of Gauss points staged through LDS: the coupling variant's hex8
  // records (48 doubles) are staged in two rounds of four points, 52 KB
  // instead of 103 KB, two workgroups per CU instead of one (9.3 -> 6.1 ms
  // on the 256x64x32 beam); the default records stay in one round (two
  // rounds under a 3-wave register bound spill and run 4.7 ms against 3.4)
  static constexpr int NSTAGE = (CPL && NGP > 4) ? 2 : 1;
  static constexpr int GPS = NGP / NSTAGE;            // Gauss points per round
  static constexpr int KS = GPS * GS + 2;             // per element: spreads a node's elements over LDS banks
  static constexpr int REC_D = NPB * NEN * KS;        // phase 1: records, doubles
  static constexpr int BLK_B = NB * NODE_BLOCK * (int)sizeof(double);
  static constexpr int F_B = (DIM + 2) * NODE_BLOCK * 8;
  static constexpr int SLOT_B = NPB * NEN * L * 4;
  static constexpr int P2_D = (BLK_B + F_B + SLOT_B + 7) / 8;   // phase 2, doubles
  static constexpr int SMEM_D = REC_D > P2_D ? REC_D : P2_D;
};

template <int DIM, typename T, bool WANT_K, bool CPL>
__device__ __forceinline__ void node_block(int64_t blk, const NodeArgs& A, const MatParams& mp) {
  const int64_t n_nodes = A.n_nodes;
  const int32_t* __restrict__ n2e_ptr = A.n2e_ptr;
  const int32_t* __restrict__ n2e = A.n2e;
  const int32_t* __restrict__ nbr_ptr = A.nbr_ptr;
  const int32_t* __restrict__ nbr = A.nbr;
  const uint8_t* __restrict__ pos = A.pos;
  const int32_t* __restrict__ row_ptr = A.row_ptr;
  const uint8_t* __restrict__ flags = A.flags;
  const double* __restrict__ rec = A.rec;
  T* __restrict__ vals = static_cast<T*>(A.vals);
  double* __restrict__ R = A.R;
  double* __restrict__ partials = A.partials;
  using E = Elem<DIM>;
  using RC = Rec<DIM, CPL>;
  using LD = NodeLds<DIM, T, CPL>;
  constexpr int NEN = E::NEN, ND = E::ND, NB = ND * ND, NGP = E::NGP;
  constexpr int L = LD::L, NPB = LD::NPB, RS = LD::RS, GS = LD::GS, KS = LD::KS;
  constexpr int FPL = RS / NEN;                // record doubles each lane stages per Gauss point
  static_assert(RS % NEN == 0, "record staging split");
  // phase 1: the Gauss-point records of the node's elements; phase 2 (same
  // memory): element blocks, forces and the position -> local node table
  __shared__ __align__(16) double smem[LD::SMEM_D];
  __shared__ double s_red[NORM_SLOTS][NPB];
  __shared__ int s_chunks;
  double* s_blk = smem;                                                    // [NB][NODE_BLOCK]
  double* s_f = reinterpret_cast<double*>(reinterpret_cast<char*>(smem) + LD::BLK_B);  // [DIM+2][NODE_BLOCK]
  int* s_slot = reinterpret_cast<int*>(reinterpret_cast<char*>(smem) + LD::BLK_B + LD::F_B);  // [NPB][NEN][L]

  const int tid = threadIdx.x;
  const int slot = tid / L;                    // node within the workgroup
  const int l = tid % L;
  const int k = l / NEN, b = l % NEN;
  const int64_t a = blk * NPB + slot;
  const bool valid = a < n_nodes;
  int e0 = 0, ne = 0, nnb = 0, nb0 = 0;
  if (valid) {
    e0 = n2e_ptr[a];
    ne = n2e_ptr[a + 1] - e0;
    nb0 = nbr_ptr[a];
    nnb = nbr_ptr[a + 1] - nb0;
  }
  if (tid == 0) s_chunks = 0;
  __syncthreads();
  if (valid && l == 0) atomicMax(&s_chunks, (ne + NEN - 1) / NEN);
  __syncthreads();
  const int chunks = s_chunks;

  double acc[ND][ND];
#pragma unroll
  for (int i = 0; i < ND; ++i)
#pragma unroll
    for (int j = 0; j < ND; ++j) acc[i][j] = 0.0;
  double facc[DIM + 2];
#pragma unroll
  for (int i = 0; i < DIM + 2; ++i) facc[i] = 0.0;

  for (int ch = 0; ch < chunks; ++ch) {
    const int kk = ch * NEN + k;
    const bool act = valid && kk < ne;
    int p = -1, la = 0;
    int64_t e = 0;
    if (act) {
      const int ent = n2e[e0 + kk];
      e = ent >> N2E_SHIFT;
      la = ent & N2E_MASK;
      p = pos[(e * NEN + la) * NEN + b];
    }
    double blk[ND][ND];
#pragma unroll
    for (int i = 0; i < ND; ++i)
#pragma unroll
      for (int j = 0; j < ND; ++j) blk[i][j] = 0.0;
    double f[DIM + 2];
#pragma unroll
    for (int i = 0; i < DIM + 2; ++i) f[i] = 0.0;
    // phase 1, in LD::NSTAGE rounds of LD::GPS Gauss points: lane (k, b)
    // copies doubles [b*FPL, (b+1)*FPL) of each record of element k, then
    // every lane sums its block over the round's points (ascending g)
    double* srec = smem + (slot * NEN + k) * KS;
#pragma unroll 1
    for (int h = 0; h < LD::NSTAGE; ++h) {
      if (act) {
        const double* src = rec + (e * NGP + h * LD::GPS) * RS + b * FPL;
#pragma unroll
        for (int g = 0; g < LD::GPS; ++g)
#pragma unroll
          for (int q = 0; q < FPL; ++q) srec[g * GS + b * FPL + q] = src[g * RS + q];
      }
      __syncthreads();
      if (act) {
        const bool wf = (b == 0);
#pragma unroll 1
        for (int g = 0; g < LD::GPS; ++g)
          block_and_force<DIM, double, CPL>(srec + g * GS, h * LD::GPS + g, la, b, mp, WANT_K, wf, blk, f);
      }
      __syncthreads();
    }
    if (WANT_K) finish_uu<DIM, double, CPL>(blk, mp);
    // phase 2: blocks to LDS, position -> local node table
#pragma unroll
    for (int q = 0; q < NEN; ++q) s_slot[(slot * NEN + k) * L + b * NEN + q] = -1;
    __syncthreads();
    if (p >= 0) s_slot[(slot * NEN + k) * L + p] = b;
#pragma unroll
    for (int i = 0; i < ND; ++i)
#pragma unroll
      for (int j = 0; j < ND; ++j) s_blk[(i * ND + j) * NODE_BLOCK + tid] = blk[i][j];
#pragma unroll
    for (int i = 0; i < DIM + 2; ++i) s_f[i * NODE_BLOCK + tid] = f[i];
    __syncthreads();
    // lane l owns neighbour position l: sum its blocks in element order
    if (valid && l < nnb) {
      const int base = slot * L;
#pragma unroll
      for (int kq = 0; kq < NEN; ++kq) {
        const int bq = s_slot[(slot * NEN + kq) * L + l];
        if (bq >= 0) {
          const int src = base + kq * NEN + bq;
#pragma unroll
          for (int i = 0; i < ND; ++i)
#pragma unroll
            for (int j = 0; j < ND; ++j) acc[i][j] += s_blk[(i * ND + j) * NODE_BLOCK + src];
        }
      }
    }
    if (valid && l == 0) {
      const int base = slot * L;
      for (int kq = 0; kq < NEN; ++kq) {
#pragma unroll
        for (int i = 0; i < DIM + 2; ++i) facc[i] += s_f[i * NODE_BLOCK + base + kq * NEN];
      }
    }
    __syncthreads();
  }

  // write the CSR row block of node a: rows a*ND + r, positions p, columns c
  if (WANT_K && valid && l < nnb) {
    const int64_t nbn = nbr[nb0 + l];
    const int64_t rb = row_ptr[a * ND];
    const int64_t rowlen = (int64_t)nnb * ND;
#pragma unroll
    for (int r = 0; r < ND; ++r) {
      const int64_t row = a * ND + r;
      const bool rd = flags[row] & 1;
#pragma unroll
      for (int c = 0; c < ND; ++c) {
        const int64_t col = nbn * ND + c;
        double v = acc[r][c];
        if (rd)
          v = (col == row) ? 1.0 : 0.0;
        else if (flags[col] & 1)
          v = 0.0;
        vals[rb + r * rowlen + (int64_t)l * ND + c] = (T)v;
      }
    }
  }
  // residual R = -f_int (0 on Dirichlet rows) and norm partials
  double red[NORM_SLOTS] = {0, 0, 0, 0, 0, 0};
  if (valid && l == 0) {
#pragma unroll
    for (int r = 0; r < ND; ++r) {
      const int64_t row = a * ND + r;
      const uint8_t fl = flags[row];
      const double fv = facc[r];
      const double rv = (fl & 1) ? 0.0 : -fv;
      R[row] = rv;
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
    partials[blk * NORM_SLOTS + tid] = sum;
  }
}

template <int DIM, typename T, bool WANT_K, bool CPL>
__global__ void __launch_bounds__(NODE_BLOCK) node_kernel(NodeArgs A, MatParams mp) {
  node_block<DIM, T, WANT_K, CPL>(blockIdx.x, A, mp);
}

template <int DIM, typename T, bool WANT_K>
__global__ void __launch_bounds__(NODE_BLOCK) node_fused_kernel(const SlotDesc* __restrict__ slots,
                                                                int nslots) {
  const int s = find_slot(slots, nslots, blockIdx.x, true);
  node_block<DIM, T, WANT_K, false>((int64_t)blockIdx.x - slots[s].node_block0, slots[s].node, slots[s].mp);
}

// fixed-order two-stage sums: stage one sums contiguous chunks of the
// per-workgroup partials, stage two (one workgroup) sums the chunk totals
__global__ void __launch_bounds__(256) norm_reduce_kernel(int64_t nblk, int64_t chunk,
                                                          const double* __restrict__ partials,
                                                          double* __restrict__ out) {
  __shared__ double s[NORM_SLOTS][256];
  const int t = threadIdx.x;
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < nblk ? lo + chunk : nblk;
  double acc[NORM_SLOTS] = {0, 0, 0, 0, 0, 0};
  for (int64_t i = lo + t; i < hi; i += 256)
#pragma unroll
    for (int q = 0; q < NORM_SLOTS; ++q) acc[q] += partials[i * NORM_SLOTS + q];
#pragma unroll
  for (int q = 0; q < NORM_SLOTS; ++q) s[q][t] = acc[q];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w)
#pragma unroll
      for (int q = 0; q < NORM_SLOTS; ++q) s[q][t] += s[q][t + w];
    __syncthreads();
  }
  if (t < NORM_SLOTS) out[(int64_t)blockIdx.x * NORM_SLOTS + t] = s[t][0];
}

__global__ void set_dirichlet_kernel(int64_t n, const int32_t* __restrict__ dofs,
                                     const double* __restrict__ vals, double lambda,
                                     double* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[dofs[i]] = lambda * vals[i];
}

__global__ void damage_kernel(int64_t n, const double* __restrict__ kappa, MatParams mp,
                              double* __restrict__ D) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double kap = kappa[i];
  double d = 0.0;
  if (!((kap - mp.kappa0) < mp.tol_dmg)) {
    const double ex = exp(-mp.beta * (kap - mp.kappa0));
    d = 1.0 - mp.kappa0 / kap * (1.0 - mp.alpha + mp.alpha * ex);
  }
  D[i] = d;
}

// element blocks for parity checks: one thread per (element, a, b)
template <int DIM, bool CPL>
__global__ void element_blocks_kernel(int64_t e0, int64_t e1, const double* __restrict__ rec,
                                      MatParams mp, double* __restrict__ Ke,
                                      double* __restrict__ fe) {
  using E = Elem<DIM>;
  using RC = Rec<DIM, CPL>;
  constexpr int NEN = E::NEN, ND = E::ND, NL = NEN * ND;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ne = e1 - e0;
  if (t >= ne * NEN * NEN) return;
  const int64_t el = t / (NEN * NEN);
  const int la = (int)((t / NEN) % NEN), lb = (int)(t % NEN);
  const int64_t e = e0 + el;
  double blk[ND][ND];
#pragma unroll
  for (int i = 0; i < ND; ++i)
#pragma unroll
    for (int j = 0; j < ND; ++j) blk[i][j] = 0.0;
  double f[DIM + 2];
#pragma unroll
  for (int i = 0; i < DIM + 2; ++i) f[i] = 0.0;
  for (int g = 0; g < E::NGP; ++g)
    block_and_force<DIM, double, CPL>(rec + (e * E::NGP + g) * RC::STRIDE, g, la, lb, mp, Ke != nullptr,
                                      lb == 0, blk, f);
  if (Ke) finish_uu<DIM, double, CPL>(blk, mp);
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

__global__ void __launch_bounds__(256) max_reduce_kernel(int64_t n, int64_t chunk,
                                                         const double* __restrict__ v,
                                                         double* __restrict__ out) {
  __shared__ double s[256];
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  double m = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) m = fmax(m, v[i]);
  s[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = s[0];
}

template <int DIM> int node_lanes() { return Elem<DIM>::NEN * Elem<DIM>::NEN; }

}  // namespace

MatParams make_params(const lgdm_material& m, int dim) {
  MatParams p{};
  const double lam = m.E * m.nu / ((1.0 + m.nu) * (1.0 - 2.0 * m.nu));
  const double mu = m.E / (2.0 * (1.0 + m.nu));
  p.mu = mu;
  p.lam = lam;
  p.ezz_fac = 0.0;
  if (dim == 2 && m.plane == LGDM_PLANE_STRESS) {
    p.lam = 2.0 * lam * mu / (lam + 2.0 * mu);
    p.ezz_fac = -m.nu / (1.0 - m.nu);
  }
  p.E = m.E;
  p.nu = m.nu;
  p.kappa0 = m.kappa0;
  p.alpha = m.alpha;
  p.beta = m.beta;
  p.c = m.c;
  p.R = m.R;
  p.eta = m.eta;
  p.h = m.h;
  p.tol_hist = m.tol_hist;
  p.tol_dmg = m.tol_dmg;
  p.k = m.k;
  p.c1 = (m.k - 1.0) / (2.0 * m.k * (1.0 - 2.0 * m.nu));
  p.c2 = (m.k - 1.0) / (1.0 - 2.0 * m.nu);
  p.c3 = 12.0 * m.k / ((1.0 + m.nu) * (1.0 + m.nu));
  p.thick = dim < 3 ? m.thickness : 1.0;
  p.g_den = 1.0 - std::exp(-m.eta);
  p.coupling = m.coupling;
  p.sq_guard = 1e-6 * m.kappa0;
  return p;
}

int64_t node_kernel_blocks(const lgdm_ctx* c) {
  if (c->order2) {
    const int npb = q_node_kernel_nodes_per_block(c->dim);
    return (c->n_nodes + npb - 1) / npb;
  }
  const int L = c->dim == 1 ? node_lanes<1>() : (c->dim == 2 ? node_lanes<2>() : node_lanes<3>());
  const int npb = NODE_BLOCK / L;
  return (c->n_nodes + npb - 1) / npb;
}

GpArgs gp_args(const lgdm_ctx* c) {
  return GpArgs{c->ngauss, c->coords, c->conn, c->e_scale, c->x, c->kappa_n, c->rec, c->kappa_t, c->D_t,
                c->eeq_t};
}

NodeArgs node_args(const lgdm_ctx* c) {
  void* vals = c->precision == LGDM_MIXED ? (void*)c->vals32 : (void*)c->vals;
  return NodeArgs{c->n_nodes, c->n2e_ptr, c->n2e, c->nbr_ptr, c->nbr, c->pos, c->row_ptr, c->dof_flags,
                  c->rec, vals, c->R, c->partials};
}

int64_t gp_kernel_blocks(const lgdm_ctx* c) { return (c->ngauss + 255) / 256; }

hipError_t launch_gp_kernel(lgdm_ctx* c, const MatParams& mp) {
  if (c->order2) return launch_q_gp_kernel(c, mp);
  const int64_t grid = gp_kernel_blocks(c);
  if (grid == 0) return hipSuccess;
  const GpArgs A = gp_args(c);
  const bool cpl = mp.coupling != 0;
  switch (c->dim) {
    case 1:
      if (cpl) gp_kernel<1, true><<<grid, 256, 0, c->stream>>>(A, mp);
      else gp_kernel<1, false><<<grid, 256, 0, c->stream>>>(A, mp);
      break;
    case 2:
      if (cpl) gp_kernel<2, true><<<grid, 256, 0, c->stream>>>(A, mp);
      else gp_kernel<2, false><<<grid, 256, 0, c->stream>>>(A, mp);
      break;
    default:
      if (cpl) gp_kernel<3, true><<<grid, 256, 0, c->stream>>>(A, mp);
      else gp_kernel<3, false><<<grid, 256, 0, c->stream>>>(A, mp);
  }
  return hipGetLastError();
}

template <int DIM, typename T>
static void node_launch(lgdm_ctx* c, const MatParams& mp, bool want_k) {
  const int64_t grid = node_kernel_blocks(c);
  if (grid == 0) return;
  const NodeArgs A = node_args(c);
  if (mp.coupling) {
    if (want_k) node_kernel<DIM, T, true, true><<<grid, NODE_BLOCK, 0, c->stream>>>(A, mp);
    else node_kernel<DIM, T, false, true><<<grid, NODE_BLOCK, 0, c->stream>>>(A, mp);
  } else {
    if (want_k) node_kernel<DIM, T, true, false><<<grid, NODE_BLOCK, 0, c->stream>>>(A, mp);
    else node_kernel<DIM, T, false, false><<<grid, NODE_BLOCK, 0, c->stream>>>(A, mp);
  }
}

hipError_t launch_node_kernel(lgdm_ctx* c, const MatParams& mp, bool want_k) {
  if (c->order2) return launch_q_node_kernel(c, mp, want_k);
  const bool mixed = c->precision == LGDM_MIXED;
  switch (c->dim) {
    case 1:
      if (mixed) node_launch<1, float>(c, mp, want_k);
      else node_launch<1, double>(c, mp, want_k);
      break;
    case 2:
      if (mixed) node_launch<2, float>(c, mp, want_k);
      else node_launch<2, double>(c, mp, want_k);
      break;
    default:
      if (mixed) node_launch<3, float>(c, mp, want_k);
      else node_launch<3, double>(c, mp, want_k);
  }
  return hipGetLastError();
}

// one fused launch of each element kernel over several problems of the same
// dimension and precision (slots: device array, ascending block ranges)
hipError_t launch_fused_assembly(hipStream_t st, int dim, bool mixed, const SlotDesc* slots_dev,
                                 int nslots, int64_t gp_blocks, int64_t node_blocks) {
  if (nslots == 0) return hipSuccess;
  switch (dim) {
    case 1: gp_fused_kernel<1><<<gp_blocks, 256, 0, st>>>(slots_dev, nslots); break;
    case 2: gp_fused_kernel<2><<<gp_blocks, 256, 0, st>>>(slots_dev, nslots); break;
    default: gp_fused_kernel<3><<<gp_blocks, 256, 0, st>>>(slots_dev, nslots);
  }
  switch (dim) {
    case 1:
      if (mixed) node_fused_kernel<1, float, true><<<node_blocks, NODE_BLOCK, 0, st>>>(slots_dev, nslots);
      else node_fused_kernel<1, double, true><<<node_blocks, NODE_BLOCK, 0, st>>>(slots_dev, nslots);
      break;
    case 2:
      if (mixed) node_fused_kernel<2, float, true><<<node_blocks, NODE_BLOCK, 0, st>>>(slots_dev, nslots);
      else node_fused_kernel<2, double, true><<<node_blocks, NODE_BLOCK, 0, st>>>(slots_dev, nslots);
      break;
    default:
      if (mixed) node_fused_kernel<3, float, true><<<node_blocks, NODE_BLOCK, 0, st>>>(slots_dev, nslots);
      else node_fused_kernel<3, double, true><<<node_blocks, NODE_BLOCK, 0, st>>>(slots_dev, nslots);
  }
  return hipGetLastError();
}

hipError_t launch_norm_reduce_on(lgdm_ctx* c, hipStream_t st) {
  const int64_t nblk = node_kernel_blocks(c);
  const int64_t nb1 = nblk < RED_CHUNKS ? nblk : RED_CHUNKS;
  const int64_t chunk = (nblk + nb1 - 1) / nb1;
  norm_reduce_kernel<<<nb1, 256, 0, st>>>(nblk, chunk, c->partials, c->red2);
  norm_reduce_kernel<<<1, 256, 0, st>>>(nb1, nb1, c->red2, c->norms_dev);
  return hipGetLastError();
}

hipError_t launch_norm_reduce(lgdm_ctx* c) { return launch_norm_reduce_on(c, c->stream); }

hipError_t launch_set_dirichlet(lgdm_ctx* c, double lambda) {
  if (c->nbc == 0) return hipSuccess;
  const int64_t grid = (c->nbc + 255) / 256;
  set_dirichlet_kernel<<<grid, 256, 0, c->stream>>>(c->nbc, c->bc_dofs, c->bc_vals, lambda, c->x);
  return hipGetLastError();
}

hipError_t launch_damage_from_kappa(lgdm_ctx* c, const MatParams& mp) {
  const int64_t grid = (c->ngauss + 255) / 256;
  if (grid == 0) return hipSuccess;
  damage_kernel<<<grid, 256, 0, c->stream>>>(c->ngauss, c->kappa_n, mp, c->D_n);
  return hipGetLastError();
}

hipError_t launch_element_blocks(lgdm_ctx* c, const MatParams& mp, int64_t e0, int64_t e1,
                                 double* Ke, double* fe) {
  if (c->order2) return launch_q_element_blocks(c, mp, e0, e1, Ke, fe);
  const int64_t n = (e1 - e0) * c->nen * c->nen;
  const int64_t grid = (n + 255) / 256;
  if (grid == 0) return hipSuccess;
  switch (c->dim) {
    case 1:
      if (mp.coupling) element_blocks_kernel<1, true><<<grid, 256, 0, c->stream>>>(e0, e1, c->rec, mp, Ke, fe);
      else element_blocks_kernel<1, false><<<grid, 256, 0, c->stream>>>(e0, e1, c->rec, mp, Ke, fe);
      break;
    case 2:
      if (mp.coupling) element_blocks_kernel<2, true><<<grid, 256, 0, c->stream>>>(e0, e1, c->rec, mp, Ke, fe);
      else element_blocks_kernel<2, false><<<grid, 256, 0, c->stream>>>(e0, e1, c->rec, mp, Ke, fe);
      break;
    default:
      if (mp.coupling) element_blocks_kernel<3, true><<<grid, 256, 0, c->stream>>>(e0, e1, c->rec, mp, Ke, fe);
      else element_blocks_kernel<3, false><<<grid, 256, 0, c->stream>>>(e0, e1, c->rec, mp, Ke, fe);
  }
  return hipGetLastError();
}

hipError_t launch_max_reduce(lgdm_ctx* c, const double* v, int64_t n, double* out_dev) {
  const int64_t nb1 = (n + 255) / 256 < RED_CHUNKS ? (n + 255) / 256 : RED_CHUNKS;
  const int64_t chunk = (n + nb1 - 1) / nb1;
  max_reduce_kernel<<<nb1, 256, 0, c->stream>>>(n, chunk, v, c->red2);
  max_reduce_kernel<<<1, 256, 0, c->stream>>>(nb1, nb1, c->red2, out_dev);
  return hipGetLastError();
}

}  // namespace lgdm
