// Appendix A at one Gauss point, shared by the equal-order and the
// mixed-order element kernels: from the small-strain tensor (eps_zz already
// set in plane stress), the micro-equivalent strain and its gradient, this
// evaluates the modified von Mises equivalent strain and its gradient
// (Eq. A.3), the history update (Eq. A.2 with the condition vector of
// Fig. 8b), damage (Eq. A.1) and the interaction function (Eq. A.4), and
// writes the Gauss point's record (the coefficients of Eqs. 11a-11f, with the
// weight wJ = w_g det J t folded in).
#pragma once

#include <cmath>

#include "lgdm_internal.h"

namespace lgdm {

// index of the symmetric tensor entry (i, j) in the record ordering
template <int DIM> __device__ __forceinline__ constexpr int sym_idx(int i, int j) {
  if (DIM == 1) return 0;
  if (DIM == 2) return (i == j) ? i : 2;
  if (i == j) return i;
  const int lo = i < j ? i : j, hi = i < j ? j : i;
  return (lo == 0 && hi == 1) ? 3 : ((lo == 1 && hi == 2) ? 4 : 5);
}

template <int DIM, bool CPL>
__device__ __forceinline__ void gp_state_record(const double (&eps)[3][3], double ebar, const double (&gb)[DIM],
                                                const double (&Ji)[DIM][DIM], double wJ, double se, double kn,
                                                const MatParams& mp, double* __restrict__ r, double& kap_out,
                                                double& D_out, double& eeq_out) {
  using RC = Rec<DIM, CPL>;
  // modified von Mises equivalent strain (A.3) and its gradient G = d eeq / d eps
  double eeq;
  double G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double q3[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // coupling variant: ds / deps
  double al = 0.0, be = 0.0;                          // coupling variant: coefficients of d^2 eeq
  if (DIM == 1) {
    eeq = eps[0][0];
    G[0][0] = 1.0;
  } else {
    const double I1 = eps[0][0] + eps[1][1] + eps[2][2];
    double dev[3][3];
    double J2 = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        dev[i][j] = eps[i][j] - (i == j ? I1 / 3.0 : 0.0);
        J2 += dev[i][j] * dev[i][j];
      }
    J2 *= 0.5;
    const double s = mp.c2 * mp.c2 * I1 * I1 + mp.c3 * J2;
    if (CPL) {
      // d^2 eeq / deps^2 = al (2 c2^2 1 (x) 1 + c3 P_dev) - be q (x) q, dropped at the cone point
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) q3[i][j] = (i == j ? 2.0 * mp.c2 * mp.c2 * I1 : 0.0) + mp.c3 * dev[i][j];
      const double sqv = s > 0.0 ? sqrt(s) : 0.0;
      if (sqv > mp.sq_guard) {
        al = 1.0 / (4.0 * mp.k * sqv);
        be = al / (2.0 * s);
      }
    }
    if (s > 0.0) {
      const double sq = sqrt(s);
      eeq = mp.c1 * I1 + sq / (2.0 * mp.k);
      const double f = 1.0 / (4.0 * mp.k * sq);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          G[i][j] = (i == j ? mp.c1 + f * 2.0 * mp.c2 * mp.c2 * I1 : 0.0) + f * mp.c3 * dev[i][j];
    } else {  // minimum-norm subgradient where the root argument vanishes
      eeq = mp.c1 * I1;
#pragma unroll
      for (int i = 0; i < 3; ++i) G[i][i] = mp.c1;
    }
    if (DIM == 2) {  // plane stress: eps_zz depends on the in-plane strains
      G[0][0] += mp.ezz_fac * G[2][2];
      G[1][1] += mp.ezz_fac * G[2][2];
    }
  }
  // history (A.2, condition vector cond1 of Fig. 8b)
  const bool chi = (ebar - kn) > mp.tol_hist;
  const double kap = chi ? ebar : kn;
  // damage (A.1, condition vector cond2 of Fig. 8b)
  double D = 0.0, dD = 0.0;
  if (!((kap - mp.kappa0) < mp.tol_dmg)) {
    const double ex = exp(-mp.beta * (kap - mp.kappa0));
    const double br = 1.0 - mp.alpha + mp.alpha * ex;
    const double q = mp.kappa0 / kap;
    D = 1.0 - q * br;
    dD = q / kap * br + q * mp.alpha * mp.beta * ex;
  }
  // interaction function (A.4)
  const double en = exp(-mp.eta * D);
  const double gv = ((1.0 - mp.R) * en + mp.R - exp(-mp.eta)) / mp.g_den;
  const double dg = -mp.eta * (1.0 - mp.R) * en / mp.g_den;

  // unscaled stress S = C : eps
  double S[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  if (DIM == 1) {
    S[0][0] = mp.E * eps[0][0];
  } else {
    double tr = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) tr += eps[i][i];
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
      for (int j = 0; j < DIM; ++j) S[i][j] = 2.0 * mp.mu * eps[i][j] + (i == j ? mp.lam * tr : 0.0);
  }
  const double chid = chi ? 1.0 : 0.0;

#pragma unroll
  for (int j = 0; j < DIM; ++j)
#pragma unroll
    for (int d = 0; d < DIM; ++d) r[RC::JINV + j * DIM + d] = Ji[j][d];
  r[RC::CUU] = wJ * (1.0 - D) * se;
  r[RC::CUE] = wJ * dD * chid * se;
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int j = i; j < DIM; ++j) {
      r[RC::S + sym_idx<DIM>(i, j)] = S[i][j];
      r[RC::GH + sym_idx<DIM>(i, j)] = wJ * mp.h * G[i][j];
    }
#pragma unroll
  for (int d = 0; d < DIM; ++d) r[RC::GB + d] = gb[d];
  r[RC::CEE] = wJ * mp.h;
  r[RC::CGP] = wJ * mp.h * mp.c * dg * dD * chid;
  r[RC::CG] = wJ * gv * mp.h * mp.c;
  r[RC::RE] = wJ * mp.h * (ebar - eeq);
  r[RC::FR] = wJ * mp.h * eeq;
  if (CPL) {
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
      for (int j = i; j < DIM; ++j) r[RC::GU + sym_idx<DIM>(i, j)] = G[i][j];
    r[RC::AL] = al;
    r[RC::BE] = be;
    if (DIM == 3) {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) r[RC::Q + sym_idx<3>(i, j)] = q3[i][j];
    } else if (DIM == 2) {
      r[RC::Q + 0] = q3[0][0];
      r[RC::Q + 1] = q3[1][1];
      r[RC::Q + 2] = q3[0][1];
      r[RC::Q + 3] = q3[2][2];
    }
  }
#pragma unroll
  for (int f = RC::USED; f < RC::STRIDE; ++f) r[f] = 0.0;
  kap_out = kap;
  D_out = D;
  eeq_out = eeq;
}

}  // namespace lgdm
