// Aggregation multigrid for the linear solve of the Newton system (Eq. 11;
// H6): the right preconditioner LGDM_PRECOND_AMG.
//
// Block-Jacobi leaves the smooth error modes of the elastic and
// micro-equivalent-strain fields to the Krylov method, whose iteration count
// then grows with the number of elements along the longest side.  A
// multigrid cycle removes them on coarser levels:
//
//  - Aggregates (host, once per mesh): greedy over the node graph in node
//    order.  A node whose neighbours are all unaggregated forms an aggregate
//    with them; each node left over joins the aggregate of its first
//    aggregated neighbour, or forms one alone.  On the 27-neighbour graph of
//    a hex8 mesh this gives about 3x3x3-node aggregates.  Coarser levels
//    aggregate the aggregate graph the same way until at most
//    DENSE_MAX_NODES coarse nodes are left.
//  - Coarse basis: on each aggregate the three translations, the three
//    (infinitesimal) rotations about a reference point and a constant
//    micro-equivalent strain, 7 unknowns per coarse node (smoothed-
//    aggregation practice for elasticity: the rigid-body motions are the
//    near-null space of the stiffness).  With d = (x - c_J) / L_{l+1} the
//    offset of a point from the reference point of its aggregate J (L_{l+1} a
//    length of the level's aggregates), a fine node's displacement follows a
//    coarse (T, W, E) as u = T + W x d and its ebar as E; a coarse node of
//    level l >= 1 (unknowns t, w, e) follows t = T + W x d, w = (L_l /
//    L_{l+1}) W, e = E.  Rows of P at Dirichlet dofs are zero, so the cycle
//    leaves them zero as block-Jacobi does (the Newton corrections there
//    must stay exactly zero).  P is never stored: kernels evaluate it from
//    the reference points and the dof flags.
//  - Coarse operators A_{l+1} = P^T A_l P (Galerkin), recomputed for every
//    tangent: one thread per coarse node pair sums, in a fixed order, the
//    fine node pairs that map to it (lists built with the aggregates).
//  - The cycle: on the finest level, additive: out = w D^-1 b + P x_c with
//    x_c the coarse cycle applied to P^T b (no pass over the fine matrix:
//    the Krylov method's own SpMV is the only one per step).  On coarser
//    levels, V(1,1): x = w D^-1 b; r = b - A x; restrict; cycle the next
//    level; x += P x_c; x <- x + w D^-1 (b - A x).  D^-1: the node-block
//    inverses (block-Jacobi), w = 0.7.  The coarsest level is solved with a
//    dense inverse (Gauss-Jordan in LDS, one workgroup).  On the 256 x 64 x
//    32 beam the additive finest level takes about 1.5 times the Krylov
//    steps of a full V(1,1)-cycle at a third of the matrix reads per step:
//    20 % less time per increment.
//  - Values of the coarse operators and their block inverses have the
//    context's matrix type (FP32 in mixed contexts: rounded once from FP64
//    sums); vectors and arithmetic are FP64.  The cycle is a fixed linear
//    map, so IDR(s) takes it as its preconditioner unchanged.
//
// Every reduction has a fixed order (no atomics): results are bitwise
// repeatable.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "lgdm_internal.h"

namespace lgdm {

namespace {

constexpr int BS = 256;
constexpr int NC = 7;                 // unknowns of a coarse node
constexpr int DENSE_MAX_NODES = 13;   // coarsest level: at most this many nodes (91 unknowns)
constexpr int MAX_LEVELS = 12;
constexpr double OMEGA = 0.7;         // block-Jacobi smoothing weight
constexpr int G = 16;                 // lanes per node of the operator kernels
constexpr int MAX_GRID = 4096;

int device_cu_count() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 1;
  }
  return cus;
}

// workgroups for `work` threads of `kernel`: at most the resident ones
template <typename K> int64_t grid_for(K kernel, int64_t work) {
  static int per_cu = 0;
  if (per_cu == 0) {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kernel, BS, 0) != hipSuccess || b < 1) b = 1;
    per_cu = b;
  }
  int64_t cap = (int64_t)per_cu * device_cu_count();
  if (cap > MAX_GRID) cap = MAX_GRID;
  int64_t g = (work + BS - 1) / BS;
  if (g > cap) {
    const int64_t it = (work + cap * BS - 1) / (cap * BS);
    g = (work + it * BS - 1) / (it * BS);
  }
  return g < 1 ? 1 : g;
}

__device__ __forceinline__ bool done(const double* sc) { return sc && sc[KSLOT_DONE] != 0.0; }

// ND consecutive values; 4-wide loads for ND = 4 (node blocks start at
// multiples of 16 values, vectors are 32-byte aligned)
template <typename T, int ND> struct Vals {
  double v[ND];
  __device__ __forceinline__ void load(const T* __restrict__ p) {
#pragma unroll
    for (int c = 0; c < ND; ++c) v[c] = (double)p[c];
  }
};
template <> struct Vals<float, 4> {
  double v[4];
  __device__ __forceinline__ void load(const float* __restrict__ p) {
    const float4 q = *reinterpret_cast<const float4*>(p);
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  }
};
template <> struct Vals<double, 4> {
  double v[4];
  __device__ __forceinline__ void load(const double* __restrict__ p) {
    const double4 q = *reinterpret_cast<const double4*>(p);
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  }
};

// ---------------------------------------------------------------------------
// Galerkin product: for each coarse pair slot s (coarse row I, column J),
// P_a^T A_ab P_b summed over the fine pairs (a, b) of the slot's list, in
// list order, with the structure of P: the translation and ebar columns
// select rows / columns of A_ab, a rotation column m combines the
// displacement ones with e_m x d (and, on coarse levels, adds ratio times
// the rotation unknown m).  Rows and columns of Dirichlet dofs (flags bit 0)
// are left out.

// (e_m x d) . v over the three displacement components
__device__ __forceinline__ double rot_dot(int m, const double (&d)[3], double v0, double v1, double v2) {
  return m == 0 ? d[1] * v2 - d[2] * v1 : (m == 1 ? d[2] * v0 - d[0] * v2 : d[0] * v1 - d[1] * v0);
}

template <typename T, typename TC, int NDF>
__global__ void __launch_bounds__(BS) galerkin_kernel(
    int64_t nslots, const int32_t* __restrict__ slot_row, const int32_t* __restrict__ cnbr,
    const int32_t* __restrict__ cnbr_ptr, const int32_t* __restrict__ crow_ptr,
    const int32_t* __restrict__ gal_ptr, const int32_t* __restrict__ gal, const int32_t* __restrict__ mem_ptr,
    const int32_t* __restrict__ mem, const int32_t* __restrict__ nbr_ptr, const int32_t* __restrict__ nbr,
    const int32_t* __restrict__ row_ptr,
    const T* __restrict__ vals, double se, const uint8_t* __restrict__ flags, const double* __restrict__ cen,
    const double* __restrict__ ccen, double inv_scale, double ratio, TC* __restrict__ cvals) {
  for (int64_t s = (int64_t)blockIdx.x * BS + threadIdx.x; s < nslots; s += (int64_t)gridDim.x * BS) {
    const int32_t I = slot_row[s], J = cnbr[s];
    const double ci[3] = {ccen[3 * (int64_t)I], ccen[3 * (int64_t)I + 1], ccen[3 * (int64_t)I + 2]};
    const double cj[3] = {ccen[3 * (int64_t)J], ccen[3 * (int64_t)J + 1], ccen[3 * (int64_t)J + 2]};
    double acc[NC][NC];
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
      for (int l = 0; l < NC; ++l) acc[k][l] = 0.0;
    // The slot's list holds its fine pairs in fine pair order, i.e. grouped by
    // row node a in ascending order, and the rows are the members of I
    // (ascending).  Walking the members in an outer loop keeps the lanes of
    // one coarse row on the same fine row at the same time (their blocks lie
    // in the same few cache lines) and loads a's row data once; the pairs are
    // still summed in list order.
    int32_t e = gal_ptr[s];
    const int32_t e_end = gal_ptr[s + 1];
    for (int32_t mi = mem_ptr[I]; mi < mem_ptr[I + 1] && e < e_end; ++mi) {
      const int32_t a = mem[mi];
      const int32_t p0 = nbr_ptr[a], p1 = nbr_ptr[a + 1];
      const int64_t len = (int64_t)(p1 - p0) * NDF;
      const T* __restrict__ rowv = vals + row_ptr[(int64_t)a * NDF];
      double da[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) da[i] = (cen[3 * (int64_t)a + i] - ci[i]) * inv_scale;
      for (; e < e_end; ++e) {
        const int32_t p = gal[e];
        if (p >= p1) break;   // the slot's pairs of row a are done
        const int32_t b = nbr[p];
        const T* __restrict__ blk = rowv + (int64_t)(p - p0) * NDF;
        double db[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) db[i] = (cen[3 * (int64_t)b + i] - cj[i]) * inv_scale;
        // the block, ebar row scaled, Dirichlet rows of a / columns of b zeroed
        double A[NDF][NDF];
#pragma unroll
        for (int i = 0; i < NDF; ++i) {
          Vals<T, NDF> row;
          row.load(blk + i * len);
          const double rs = i == NDF - 1 ? se : 1.0;
#pragma unroll
          for (int j = 0; j < NDF; ++j) A[i][j] = row.v[j] * rs;
        }
        if (flags) {
#pragma unroll
          for (int i = 0; i < NDF; ++i) {
            const bool ra = flags[(int64_t)a * NDF + i] & 1, cb = flags[(int64_t)b * NDF + i] & 1;
#pragma unroll
            for (int j = 0; j < NDF; ++j) {
              if (ra) A[i][j] = 0.0;
              if (cb) A[j][i] = 0.0;
            }
          }
        }
        // row k of X = P_a^T A (NDF values), then row k of X P_b
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          double x[NDF];
#pragma unroll
          for (int j = 0; j < NDF; ++j) {
            if (k < 3) x[j] = A[k][j];
            else if (k < 6) {
              x[j] = rot_dot(k - 3, da, A[0][j], A[1][j], A[2][j]);
              if constexpr (NDF == NC) x[j] += ratio * A[k][j];
            } else x[j] = A[NDF - 1][j];
          }
          acc[k][0] += x[0];
          acc[k][1] += x[1];
          acc[k][2] += x[2];
#pragma unroll
          for (int m = 0; m < 3; ++m) {
            double y = rot_dot(m, db, x[0], x[1], x[2]);
            if constexpr (NDF == NC) y += ratio * x[3 + m];
            acc[k][3 + m] += y;
          }
          acc[k][6] += x[NDF - 1];
        }
      }
    }
    const int32_t q0 = cnbr_ptr[I];
    const int64_t clen = (int64_t)(cnbr_ptr[I + 1] - q0) * NC;
    TC* __restrict__ out = cvals + crow_ptr[(int64_t)I * NC] + (int64_t)(s - q0) * NC;
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
      for (int l = 0; l < NC; ++l) out[k * clen + l] = (TC)acc[k][l];
  }
}

// node-block inverses of a coarse level (Gauss-Jordan, partial pivoting); a
// singular block gives the identity
template <typename TC>
__global__ void coarse_bj_kernel(int64_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ dpos,
                                 const TC* __restrict__ vals, TC* __restrict__ minv) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  double m[NC][2 * NC];
  for (int r = 0; r < NC; ++r) {
    const int64_t base = row_ptr[a * NC + r] + (int64_t)dpos[a] * NC;
    for (int c = 0; c < NC; ++c) {
      m[r][c] = (double)vals[base + c];
      m[r][NC + c] = r == c ? 1.0 : 0.0;
    }
  }
  bool ok = true;
  for (int col = 0; col < NC && ok; ++col) {
    int piv = col;
    double best = fabs(m[col][col]);
    for (int r = col + 1; r < NC; ++r)
      if (fabs(m[r][col]) > best) {
        best = fabs(m[r][col]);
        piv = r;
      }
    if (!(best > 0.0) || !isfinite(best)) {
      ok = false;
      break;
    }
    if (piv != col)
      for (int c = 0; c < 2 * NC; ++c) {
        const double t = m[col][c];
        m[col][c] = m[piv][c];
        m[piv][c] = t;
      }
    const double inv = 1.0 / m[col][col];
    for (int c = 0; c < 2 * NC; ++c) m[col][c] *= inv;
    for (int r = 0; r < NC; ++r) {
      if (r == col) continue;
      const double f = m[r][col];
      for (int c = 0; c < 2 * NC; ++c) m[r][c] -= f * m[col][c];
    }
  }
  TC* out = minv + a * NC * NC;
  for (int r = 0; r < NC; ++r)
    for (int c = 0; c < NC; ++c) out[r * NC + c] = ok ? (TC)m[r][NC + c] : (TC)(r == c ? 1.0 : 0.0);
}

// ---------------------------------------------------------------------------
// Operator kernels of a level (node-blocked CSR, G lanes per node, one lane
// per neighbour; the ebar row of a fine node carries the scale se).
// MODE 0: out = b - A x.  MODE 1: out = x + w D^-1 (b - A x).
template <typename T, int ND, int MODE>
__global__ void __launch_bounds__(BS) level_op_kernel(int64_t n_nodes, const int32_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ nbr_ptr,
                                                      const int32_t* __restrict__ nbr, const T* __restrict__ vals,
                                                      double se, const double* __restrict__ x,
                                                      const double* __restrict__ b, const T* __restrict__ minv,
                                                      double* __restrict__ out, const double* __restrict__ sc) {
  if (done(sc)) return;
  const int lane = threadIdx.x % G;
  const int64_t grp = ((int64_t)blockIdx.x * BS + threadIdx.x) / G;
  const int64_t ngrp = (int64_t)gridDim.x * BS / G;
  for (int64_t a = grp; a < n_nodes; a += ngrp) {
    const int32_t p0 = nbr_ptr[a];
    const int nnb = nbr_ptr[a + 1] - p0;
    const int64_t len = (int64_t)nnb * ND;
    const T* __restrict__ rv = vals + row_ptr[a * ND];
    double acc[ND];
#pragma unroll
    for (int r = 0; r < ND; ++r) acc[r] = 0.0;
    for (int q = lane; q < nnb; q += G) {
      Vals<double, ND> xq;
      xq.load(x + (int64_t)nbr[p0 + q] * ND);
#pragma unroll
      for (int r = 0; r < ND; ++r) {
        Vals<T, ND> m;
        m.load(rv + r * len + (int64_t)q * ND);
#pragma unroll
        for (int c = 0; c < ND; ++c) acc[r] += m.v[c] * xq.v[c];
      }
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1)
#pragma unroll
      for (int r = 0; r < ND; ++r) acc[r] += __shfl_xor(acc[r], o, G);
    if (lane < ND) {
      const int64_t o = a * ND;
      double res[ND];
#pragma unroll
      for (int r = 0; r < ND; ++r) res[r] = b[o + r] - acc[r] * (r == ND - 1 ? se : 1.0);
      double mine = res[0];
#pragma unroll
      for (int r = 1; r < ND; ++r)
        if (lane == r) mine = res[r];
      if (MODE == 0) {
        out[o + lane] = mine;
      } else {
        const T* __restrict__ mi = minv + o * ND + (int64_t)lane * ND;
        double z = 0.0;
#pragma unroll
        for (int c = 0; c < ND; ++c) z += (double)mi[c] * res[c];
        out[o + lane] = x[o + lane] + OMEGA * z;
      }
    }
  }
}

// x = w D^-1 b (the pre-smoothing step from a zero start)
template <typename T, int ND>
__global__ void __launch_bounds__(BS) jacobi0_kernel(int64_t n_nodes, const T* __restrict__ minv,
                                                     const double* __restrict__ b, double* __restrict__ x,
                                                     const double* __restrict__ sc) {
  if (done(sc)) return;
  for (int64_t a = (int64_t)blockIdx.x * BS + threadIdx.x; a < n_nodes; a += (int64_t)gridDim.x * BS) {
    Vals<double, ND> bb;
    bb.load(b + a * ND);
    for (int r = 0; r < ND; ++r) {
      Vals<T, ND> m;
      m.load(minv + (a * ND + r) * ND);
      double z = 0.0;
#pragma unroll
      for (int c = 0; c < ND; ++c) z += m.v[c] * bb.v[c];
      x[a * ND + r] = OMEGA * z;
    }
  }
}

// b_c(J) = sum over the members I of J of P_I^T r_I: G lanes per coarse node
template <int NDF>
__global__ void __launch_bounds__(BS) restrict_kernel(int64_t nc, const int32_t* __restrict__ mem_ptr,
                                                      const int32_t* __restrict__ mem,
                                                      const uint8_t* __restrict__ flags,
                                                      const double* __restrict__ cen,
                                                      const double* __restrict__ ccen, double inv_scale,
                                                      double ratio, const double* __restrict__ r,
                                                      double* __restrict__ bc, const double* __restrict__ sc) {
  if (done(sc)) return;
  const int lane = threadIdx.x % G;
  const int64_t grp = ((int64_t)blockIdx.x * BS + threadIdx.x) / G;
  const int64_t ngrp = (int64_t)gridDim.x * BS / G;
  for (int64_t J = grp; J < nc; J += ngrp) {
    double acc[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) acc[k] = 0.0;
    for (int32_t e = mem_ptr[J] + lane; e < mem_ptr[J + 1]; e += G) {
      const int64_t I = mem[e];
      double d[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) d[i] = (cen[3 * I + i] - ccen[3 * J + i]) * inv_scale;
      Vals<double, NDF> v;
      v.load(r + I * NDF);
      if (flags)
#pragma unroll
        for (int i = 0; i < NDF; ++i)
          if (flags[I * NDF + i] & 1) v.v[i] = 0.0;
      // translations: u; rotations: d x u (+ ratio w); ebar
      acc[0] += v.v[0];
      acc[1] += v.v[1];
      acc[2] += v.v[2];
      acc[3] += d[1] * v.v[2] - d[2] * v.v[1];
      acc[4] += d[2] * v.v[0] - d[0] * v.v[2];
      acc[5] += d[0] * v.v[1] - d[1] * v.v[0];
      if (NDF == NC) {
        acc[3] += ratio * v.v[3];
        acc[4] += ratio * v.v[4];
        acc[5] += ratio * v.v[5];
      }
      acc[6] += v.v[NDF - 1];
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1)
#pragma unroll
      for (int k = 0; k < NC; ++k) acc[k] += __shfl_xor(acc[k], o, G);
    if (lane < NC) {
      double mine = acc[0];
#pragma unroll
      for (int k = 1; k < NC; ++k)
        if (lane == k) mine = acc[k];
      bc[J * NC + lane] = mine;
    }
  }
}

// x_I += P_I x_c(agg(I)): u += T + W x d (t likewise; w += ratio W); ebar += E
template <int NDF>
__global__ void __launch_bounds__(BS) prolong_kernel(int64_t n, const int32_t* __restrict__ agg,
                                                     const uint8_t* __restrict__ flags,
                                                     const double* __restrict__ cen,
                                                     const double* __restrict__ ccen, double inv_scale,
                                                     double ratio, const double* __restrict__ xc,
                                                     double* __restrict__ x, const double* __restrict__ sc) {
  if (done(sc)) return;
  for (int64_t I = (int64_t)blockIdx.x * BS + threadIdx.x; I < n; I += (int64_t)gridDim.x * BS) {
    const int64_t J = agg[I];
    double d[3], z[NC];
#pragma unroll
    for (int i = 0; i < 3; ++i) d[i] = (cen[3 * I + i] - ccen[3 * J + i]) * inv_scale;
#pragma unroll
    for (int k = 0; k < NC; ++k) z[k] = xc[J * NC + k];
    double p[NDF];
    p[0] = z[0] + z[4] * d[2] - z[5] * d[1];
    p[1] = z[1] + z[5] * d[0] - z[3] * d[2];
    p[2] = z[2] + z[3] * d[1] - z[4] * d[0];
    if constexpr (NDF == NC) {
      p[3] = ratio * z[3];
      p[4] = ratio * z[4];
      p[5] = ratio * z[5];
    }
    p[NDF - 1] = z[6];
    double* xi = x + I * NDF;
#pragma unroll
    for (int i = 0; i < NDF; ++i)
      if (!(flags && (flags[I * NDF + i] & 1))) xi[i] += p[i];
  }
}

// out = w D^-1 b + P x_c: the finest level of the additive cycle (block-
// Jacobi and the coarse correction side by side, no fine residual)
template <typename T, int NDF>
__global__ void __launch_bounds__(BS) add_level_kernel(int64_t n, const int32_t* __restrict__ agg,
                                                       const uint8_t* __restrict__ flags,
                                                       const double* __restrict__ cen,
                                                       const double* __restrict__ ccen, double inv_scale,
                                                       const T* __restrict__ minv, const double* __restrict__ b,
                                                       const double* __restrict__ xc, double* __restrict__ out,
                                                       const double* __restrict__ sc) {
  if (done(sc)) return;
  for (int64_t I = (int64_t)blockIdx.x * BS + threadIdx.x; I < n; I += (int64_t)gridDim.x * BS) {
    const int64_t J = agg[I];
    double d[3], z[NC];
#pragma unroll
    for (int i = 0; i < 3; ++i) d[i] = (cen[3 * I + i] - ccen[3 * J + i]) * inv_scale;
#pragma unroll
    for (int k = 0; k < NC; ++k) z[k] = xc[J * NC + k];
    double p[NDF];
    p[0] = z[0] + z[4] * d[2] - z[5] * d[1];
    p[1] = z[1] + z[5] * d[0] - z[3] * d[2];
    p[2] = z[2] + z[3] * d[1] - z[4] * d[0];
    p[NDF - 1] = z[6];
    Vals<double, NDF> bb;
    bb.load(b + I * NDF);
#pragma unroll
    for (int r = 0; r < NDF; ++r) {
      Vals<T, NDF> m;
      m.load(minv + (I * NDF + r) * NDF);
      double v = 0.0;
#pragma unroll
      for (int c = 0; c < NDF; ++c) v += m.v[c] * bb.v[c];
      v *= OMEGA;
      if (!(flags && (flags[I * NDF + r] & 1))) v += p[r];
      out[I * NDF + r] = v;
    }
  }
}

// coarsest level: dense A (n x n, FP64) from its node-blocked CSR
template <typename TC>
__global__ void dense_build_kernel(int64_t n_nodes, const int32_t* __restrict__ row_ptr,
                                   const int32_t* __restrict__ nbr_ptr, const int32_t* __restrict__ nbr,
                                   const TC* __restrict__ vals, double* __restrict__ dense) {
  const int64_t n = n_nodes * NC;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double* row = dense + i * n;
    for (int64_t c = 0; c < n; ++c) row[c] = 0.0;
    const int64_t a = i / NC, r = i % NC;
    const int32_t p0 = nbr_ptr[a];
    const int64_t len = (int64_t)(nbr_ptr[a + 1] - p0) * NC;
    for (int32_t p = p0; p < nbr_ptr[a + 1]; ++p) {
      const int64_t b = nbr[p];
      for (int c = 0; c < NC; ++c) row[b * NC + c] = (double)vals[row_ptr[a * NC] + r * len + (p - p0) * NC + c];
    }
  }
}

// Gauss-Jordan with partial pivoting on [A | I] held in LDS by one
// workgroup; the right half becomes A^-1.  A singular matrix gives inv = 0
// (the cycle then skips the coarsest correction).
constexpr int DMAX = NC * DENSE_MAX_NODES;  // largest coarsest size
constexpr int DBS = 1024;
__global__ void __launch_bounds__(DBS) dense_invert_kernel(int n, const double* __restrict__ a,
                                                           double* __restrict__ inv) {
  __shared__ double m[DMAX * 2 * DMAX];
  __shared__ double fac[DMAX];
  __shared__ int piv_s;
  __shared__ int bad;
  const int t = threadIdx.x, w = 2 * n;
  for (int e = t; e < n * w; e += DBS) {
    const int r = e / w, c = e % w;
    m[e] = c < n ? a[r * n + c] : (c - n == r ? 1.0 : 0.0);
  }
  if (t == 0) bad = 0;
  __syncthreads();
  for (int col = 0; col < n; ++col) {
    // pivot: largest |m[r][col]|, lowest row on ties (first wave)
    if (t < 64) {
      double best = -1.0;
      int bi = n;
      for (int r = col + t; r < n; r += 64) {
        const double v = fabs(m[r * w + col]);
        if (v > best) {
          best = v;
          bi = r;
        }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o);
        const int oi = __shfl_xor(bi, o);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (t == 0) {
        if (!(best > 0.0) || !isfinite(best) || bi >= n) bad = 1;
        piv_s = bi;
      }
    }
    __syncthreads();
    if (bad) break;
    const int piv = piv_s;
    if (piv != col)
      for (int c = t; c < w; c += DBS) {
        const double x = m[col * w + c];
        m[col * w + c] = m[piv * w + c];
        m[piv * w + c] = x;
      }
    __syncthreads();
    const double inv_p = 1.0 / m[col * w + col];
    __syncthreads();
    for (int c = t; c < w; c += DBS) m[col * w + c] *= inv_p;
    for (int r = t; r < n; r += DBS) fac[r] = r == col ? 0.0 : m[r * w + col];
    __syncthreads();
    for (int e = t; e < n * w; e += DBS) {
      const int r = e / w, c = e % w;
      if (r != col) m[e] -= fac[r] * m[col * w + c];
    }
    __syncthreads();
  }
  for (int e = t; e < n * n; e += DBS) {
    const int r = e / n, c = e % n;
    inv[e] = bad ? 0.0 : m[r * w + n + c];
  }
}

// x = A^-1 b on the coarsest level (fixed-order row dot products)
__global__ void __launch_bounds__(BS) dense_apply_kernel(int64_t n, const double* __restrict__ inv,
                                                         const double* __restrict__ b, double* __restrict__ x,
                                                         const double* __restrict__ sc) {
  if (done(sc)) return;
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
    double s = 0.0;
    for (int64_t j = 0; j < n; ++j) s += inv[i * n + j] * b[j];
    x[i] = s;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// host side

struct AmgLevel {
  int64_t n = 0;        // nodes
  int nd = 0;           // unknowns per node
  int64_t npairs = 0;
  const int32_t *nbr_ptr = nullptr, *nbr = nullptr, *row_ptr = nullptr, *dpos = nullptr;
  void* vals = nullptr;   // the level's operator (level 0: the context's matrix)
  void* minv = nullptr;   // its node-block inverses
  const double* cen = nullptr;  // reference points [n * 3]
  const uint8_t* flags = nullptr;  // dof flags (bit 0: Dirichlet); level 0 only
  double scale = 1.0;           // L_l
  double *b = nullptr, *x = nullptr, *r = nullptr, *xo = nullptr;
  // transfer to the next level
  int32_t* agg = nullptr;                         // [n]
  int32_t *mem_ptr = nullptr, *mem = nullptr;     // members of each next-level node
  int32_t *gal_ptr = nullptr, *gal = nullptr;     // fine pairs of each next-level pair slot
  int32_t* slot_row = nullptr;                    // (next level) row node of each of its pair slots
};

struct Amg {
  std::vector<AmgLevel> lv;  // lv.back(): the coarsest level (dense inverse)
  bool mixed = false;
  int64_t ndense = 0;
  double* dense = nullptr;   // [ndense * ndense]
  double* dinv = nullptr;    // [ndense * ndense]
  double build_ms = 0.0;
};

namespace {

template <typename V> V* upload(lgdm_ctx* c, const std::vector<V>& h, hipError_t& e) {
  V* d = (V*)dalloc(c, std::max<size_t>(h.size(), 1) * sizeof(V));
  if (!d) {
    e = hipErrorOutOfMemory;
    return nullptr;
  }
  if (!h.empty()) {
    const hipError_t r = hipMemcpyAsync(d, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice, c->stream);
    if (r != hipSuccess) e = r;
  }
  return d;
}

// greedy aggregation of a graph (CSR with the node itself in its list)
int64_t aggregate(int64_t n, const std::vector<int32_t>& ptr, const std::vector<int32_t>& adj,
                  std::vector<int32_t>& agg) {
  agg.assign(n, -1);
  int64_t na = 0;
  for (int64_t a = 0; a < n; ++a) {
    if (agg[a] >= 0) continue;
    bool free_all = true;
    for (int32_t p = ptr[a]; p < ptr[a + 1] && free_all; ++p) free_all = agg[adj[p]] < 0;
    if (!free_all) continue;
    for (int32_t p = ptr[a]; p < ptr[a + 1]; ++p) agg[adj[p]] = (int32_t)na;
    agg[a] = (int32_t)na++;
  }
  for (int64_t a = 0; a < n; ++a) {
    if (agg[a] >= 0) continue;
    int32_t j = -1;
    for (int32_t p = ptr[a]; p < ptr[a + 1] && j < 0; ++p)
      if (adj[p] != a && agg[adj[p]] >= 0) j = agg[adj[p]];
    agg[a] = j >= 0 ? j : (int32_t)na++;
  }
  return na;
}

hipError_t build(lgdm_ctx* c, Amg& m, std::string& msg) {
  hipError_t e = hipSuccess;
  const int64_t n0 = c->n_nodes;
  std::vector<int32_t> ptr(n0 + 1), adj;
  std::vector<double> cen(n0 * 3);
  if ((e = hipMemcpyAsync(ptr.data(), c->nbr_ptr, (n0 + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(c->stream)) != hipSuccess)
    return e;
  adj.resize(ptr[n0]);
  if ((e = hipMemcpyAsync(adj.data(), c->nbr, adj.size() * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(cen.data(), c->coords, n0 * 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(c->stream)) != hipSuccess)
    return e;
  const size_t vsz = m.mixed ? sizeof(float) : sizeof(double);

  AmgLevel L0;
  L0.n = n0;
  L0.nd = c->nd;
  L0.npairs = (int64_t)adj.size();
  L0.nbr_ptr = c->nbr_ptr;
  L0.nbr = c->nbr;
  L0.row_ptr = c->row_ptr;
  L0.dpos = c->dpos;
  L0.vals = m.mixed ? (void*)c->vals32 : (void*)c->vals;
  L0.minv = m.mixed ? (void*)c->minv32 : (void*)c->minv;
  L0.cen = c->coords;
  L0.flags = c->dof_flags;
  L0.scale = 1.0;
  L0.x = (double*)dalloc(c, n0 * c->nd * sizeof(double));
  L0.r = (double*)dalloc(c, n0 * c->nd * sizeof(double));
  if (!L0.x || !L0.r) return hipErrorOutOfMemory;
  m.lv.push_back(L0);

  int64_t n = n0;
  double scale = 1.0;
  while (n > DENSE_MAX_NODES && (int)m.lv.size() < MAX_LEVELS) {
    std::vector<int32_t> agg;
    const int64_t na = aggregate(n, ptr, adj, agg);
    if (na >= n) break;
    // members of each aggregate, ascending
    std::vector<int32_t> mem_ptr(na + 1, 0), mem(n);
    for (int64_t a = 0; a < n; ++a) mem_ptr[agg[a] + 1]++;
    for (int64_t j = 0; j < na; ++j) mem_ptr[j + 1] += mem_ptr[j];
    {
      std::vector<int32_t> fill(mem_ptr.begin(), mem_ptr.end() - 1);
      for (int64_t a = 0; a < n; ++a) mem[fill[agg[a]]++] = (int32_t)a;
    }
    // reference points (member means) and the level's length
    std::vector<double> ccen(na * 3, 0.0);
    for (int64_t j = 0; j < na; ++j) {
      const double k = 1.0 / (mem_ptr[j + 1] - mem_ptr[j]);
      for (int32_t e2 = mem_ptr[j]; e2 < mem_ptr[j + 1]; ++e2)
        for (int i = 0; i < 3; ++i) ccen[j * 3 + i] += cen[(int64_t)mem[e2] * 3 + i] * k;
    }
    double lnext = 0.0;
    for (int64_t a = 0; a < n; ++a) {
      double d2 = 0.0;
      for (int i = 0; i < 3; ++i) {
        const double d = cen[a * 3 + i] - ccen[(int64_t)agg[a] * 3 + i];
        d2 += d * d;
      }
      lnext = std::max(lnext, std::sqrt(d2));
    }
    if (!(lnext > 0.0)) lnext = 1.0;
    // aggregate graph (sorted, with the aggregate itself)
    std::vector<int32_t> cptr(na + 1, 0), cadj, mark(na, -1), tmp;
    for (int64_t j = 0; j < na; ++j) {
      tmp.clear();
      for (int32_t e2 = mem_ptr[j]; e2 < mem_ptr[j + 1]; ++e2) {
        const int32_t a = mem[e2];
        for (int32_t p = ptr[a]; p < ptr[a + 1]; ++p) {
          const int32_t J = agg[adj[p]];
          if (mark[J] != (int32_t)j) {
            mark[J] = (int32_t)j;
            tmp.push_back(J);
          }
        }
      }
      std::sort(tmp.begin(), tmp.end());
      cadj.insert(cadj.end(), tmp.begin(), tmp.end());
      cptr[j + 1] = (int32_t)cadj.size();
    }
    const int64_t cpairs = (int64_t)cadj.size();
    // Galerkin lists: fine pairs of each coarse pair slot, in fine pair order
    std::vector<int32_t> pslot(ptr[n]), gal_ptr(cpairs + 1, 0), gal(ptr[n]), slot_row(cpairs);
    for (int64_t a = 0; a < n; ++a)
      for (int32_t p = ptr[a]; p < ptr[a + 1]; ++p) {
        const int32_t I = agg[a], J = agg[adj[p]];
        const int32_t s = (int32_t)(std::lower_bound(cadj.begin() + cptr[I], cadj.begin() + cptr[I + 1], J) -
                                    cadj.begin());
        pslot[p] = s;
        gal_ptr[s + 1]++;
      }
    for (int64_t s = 0; s < cpairs; ++s) gal_ptr[s + 1] += gal_ptr[s];
    {
      std::vector<int32_t> fill(gal_ptr.begin(), gal_ptr.end() - 1);
      for (int32_t p = 0; p < ptr[n]; ++p) gal[fill[pslot[p]]++] = p;
    }
    for (int64_t j = 0; j < na; ++j)
      for (int32_t s = cptr[j]; s < cptr[j + 1]; ++s) slot_row[s] = (int32_t)j;
    // node-blocked rows of the coarse operator
    std::vector<int32_t> crow(na * NC + 1), cdpos(na);
    int64_t off = 0;
    for (int64_t j = 0; j < na; ++j) {
      const int64_t len = (int64_t)(cptr[j + 1] - cptr[j]) * NC;
      for (int r = 0; r < NC; ++r) {
        crow[j * NC + r] = (int32_t)off;
        off += len;
      }
      cdpos[j] = (int32_t)(std::lower_bound(cadj.begin() + cptr[j], cadj.begin() + cptr[j + 1], (int32_t)j) -
                           (cadj.begin() + cptr[j]));
    }
    if (off >= INT32_MAX) {
      msg = "coarse operator too large for 32-bit offsets";
      return hipErrorInvalidValue;
    }
    crow[na * NC] = (int32_t)off;

    AmgLevel& F = m.lv.back();
    F.agg = upload(c, agg, e);
    F.mem_ptr = upload(c, mem_ptr, e);
    F.mem = upload(c, mem, e);
    F.gal_ptr = upload(c, gal_ptr, e);
    F.gal = upload(c, gal, e);
    AmgLevel C;
    C.n = na;
    C.nd = NC;
    C.npairs = cpairs;
    C.slot_row = upload(c, slot_row, e);
    C.nbr_ptr = upload(c, cptr, e);
    C.nbr = upload(c, cadj, e);
    C.row_ptr = upload(c, crow, e);
    C.dpos = upload(c, cdpos, e);
    C.cen = upload(c, ccen, e);
    C.scale = lnext;
    C.vals = dalloc(c, std::max<int64_t>(off, 1) * vsz);
    C.minv = dalloc(c, na * NC * NC * vsz);
    C.b = (double*)dalloc(c, na * NC * sizeof(double));
    C.x = (double*)dalloc(c, na * NC * sizeof(double));
    C.r = (double*)dalloc(c, na * NC * sizeof(double));
    C.xo = (double*)dalloc(c, na * NC * sizeof(double));
    if (e != hipSuccess) return e;
    if (!F.agg || !F.mem_ptr || !F.mem || !F.gal_ptr || !F.gal || !C.slot_row || !C.nbr_ptr ||
        !C.nbr || !C.row_ptr || !C.dpos || !C.cen || !C.vals || !C.minv || !C.b || !C.x || !C.r || !C.xo)
      return hipErrorOutOfMemory;
    // uploads read these host vectors: finish before they go out of scope
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return e;
    m.lv.push_back(C);
    ptr.swap(cptr);
    adj.swap(cadj);
    cen.swap(ccen);
    n = na;
    scale = lnext;
  }
  (void)scale;
  if (m.lv.size() < 2) {
    msg = "mesh too small for multigrid (no coarse level)";
    return hipErrorInvalidValue;
  }
  if (m.lv.back().n > DENSE_MAX_NODES) {
    msg = "multigrid coarsening stalled above the dense coarsest size";
    return hipErrorInvalidValue;
  }
  m.ndense = m.lv.back().n * NC;
  m.dense = (double*)dalloc(c, m.ndense * m.ndense * sizeof(double));
  m.dinv = (double*)dalloc(c, m.ndense * m.ndense * sizeof(double));
  if (!m.dense || !m.dinv) return hipErrorOutOfMemory;
  return hipSuccess;
}

template <typename T> hipError_t numeric(lgdm_ctx* c, Amg& m) {
  const double se = c->mat.E / c->mat.h;
  hipStream_t st = c->stream;
  for (size_t l = 0; l + 1 < m.lv.size(); ++l) {
    const AmgLevel& F = m.lv[l];
    const AmgLevel& C = m.lv[l + 1];
    const double inv_scale = 1.0 / C.scale, ratio = F.scale / C.scale;
    const int64_t slots = C.npairs;
    if (F.nd == NC) {
      auto k = galerkin_kernel<T, T, NC>;
      k<<<grid_for(k, slots), BS, 0, st>>>(C.npairs, C.slot_row, C.nbr, C.nbr_ptr, C.row_ptr, F.gal_ptr, F.gal,
                                                 F.mem_ptr, F.mem, F.nbr_ptr, F.nbr, F.row_ptr, (const T*)F.vals, 1.0,
                                                 F.flags, F.cen, C.cen, inv_scale, ratio, (T*)C.vals);
    } else {
      auto k = galerkin_kernel<T, T, 4>;
      k<<<grid_for(k, slots), BS, 0, st>>>(C.npairs, C.slot_row, C.nbr, C.nbr_ptr, C.row_ptr, F.gal_ptr, F.gal,
                                                 F.mem_ptr, F.mem, F.nbr_ptr, F.nbr, F.row_ptr, (const T*)F.vals, se,
                                                 F.flags, F.cen, C.cen, inv_scale, ratio, (T*)C.vals);
    }
    if (l + 2 < m.lv.size())
      coarse_bj_kernel<T><<<(C.n + 127) / 128, 128, 0, st>>>(C.n, C.row_ptr, C.dpos, (const T*)C.vals, (T*)C.minv);
  }
  const AmgLevel& D = m.lv.back();
  dense_build_kernel<T><<<(m.ndense + 127) / 128, 128, 0, st>>>(D.n, D.row_ptr, D.nbr_ptr, D.nbr,
                                                                 (const T*)D.vals, m.dense);
  dense_invert_kernel<<<1, DBS, 0, st>>>((int)m.ndense, m.dense, m.dinv);
  return hipGetLastError();
}

// pre-smoothing from zero and the residual
template <typename T, int ND>
void level_ops(const AmgLevel& L, double se, const double* b, double* x, double* r, const double* sc,
               hipStream_t st) {
  auto kj = jacobi0_kernel<T, ND>;
  kj<<<grid_for(kj, L.n), BS, 0, st>>>(L.n, (const T*)L.minv, b, x, sc);
  auto kr = level_op_kernel<T, ND, 0>;
  kr<<<grid_for(kr, L.n * G), BS, 0, st>>>(L.n, L.row_ptr, L.nbr_ptr, L.nbr, (const T*)L.vals, se, x, b, nullptr, r,
                                           sc);
}

// post-smoothing
template <typename T, int ND>
void level_post(const AmgLevel& L, double se, const double* b, const double* x, double* out, const double* sc,
                hipStream_t st) {
  auto ks = level_op_kernel<T, ND, 1>;
  ks<<<grid_for(ks, L.n * G), BS, 0, st>>>(L.n, L.row_ptr, L.nbr_ptr, L.nbr, (const T*)L.vals, se, x, b,
                                           (const T*)L.minv, out, sc);
}

template <typename T>
void vcycle(lgdm_ctx* c, Amg& m, size_t l, const double* b, double* out, const double* sc, hipStream_t st);

// finest level of the additive cycle: restrict b, cycle the coarse levels,
// then out = w D^-1 b + P x_c
template <typename T>
void additive_top(lgdm_ctx* c, Amg& m, const double* b, double* out, const double* sc, hipStream_t st) {
  const AmgLevel& F = m.lv[0];
  const AmgLevel& C = m.lv[1];
  const double inv_scale = 1.0 / C.scale, ratio = F.scale / C.scale;
  auto kr = restrict_kernel<4>;
  kr<<<grid_for(kr, C.n * G), BS, 0, st>>>(C.n, F.mem_ptr, F.mem, F.flags, F.cen, C.cen, inv_scale, ratio, b, C.b, sc);
  vcycle<T>(c, m, 1, C.b, C.xo, sc, st);
  auto ka = add_level_kernel<T, 4>;
  probe_before(c, PROBE_MG_FINEST, st);
  ka<<<grid_for(ka, F.n), BS, 0, st>>>(F.n, F.agg, F.flags, F.cen, C.cen, inv_scale, (const T*)F.minv, b, C.xo, out,
                                       sc);
  probe_after(c, PROBE_MG_FINEST, st);
}

template <typename T>
void vcycle(lgdm_ctx* c, Amg& m, size_t l, const double* b, double* out, const double* sc, hipStream_t st) {
  if (l == 0) {
    additive_top<T>(c, m, b, out, sc, st);
    return;
  }
  if (l + 1 == m.lv.size()) {
    dense_apply_kernel<<<(m.ndense + BS - 1) / BS, BS, 0, st>>>(m.ndense, m.dinv, b, out, sc);
    return;
  }
  const AmgLevel& F = m.lv[l];
  const AmgLevel& C = m.lv[l + 1];
  const double se = l == 0 ? c->mat.E / c->mat.h : 1.0;
  const double inv_scale = 1.0 / C.scale, ratio = F.scale / C.scale;
  if (F.nd == NC) level_ops<T, NC>(F, se, b, F.x, F.r, sc, st);
  else level_ops<T, 4>(F, se, b, F.x, F.r, sc, st);
  if (F.nd == NC) {
    auto k = restrict_kernel<NC>;
    k<<<grid_for(k, C.n * G), BS, 0, st>>>(C.n, F.mem_ptr, F.mem, F.flags, F.cen, C.cen, inv_scale, ratio, F.r, C.b, sc);
  } else {
    auto k = restrict_kernel<4>;
    k<<<grid_for(k, C.n * G), BS, 0, st>>>(C.n, F.mem_ptr, F.mem, F.flags, F.cen, C.cen, inv_scale, ratio, F.r, C.b, sc);
  }
  vcycle<T>(c, m, l + 1, C.b, C.xo, sc, st);
  if (F.nd == NC) {
    auto k = prolong_kernel<NC>;
    k<<<grid_for(k, F.n), BS, 0, st>>>(F.n, F.agg, F.flags, F.cen, C.cen, inv_scale, ratio, C.xo, F.x, sc);
    level_post<T, NC>(F, se, b, F.x, out, sc, st);
  } else {
    auto k = prolong_kernel<4>;
    k<<<grid_for(k, F.n), BS, 0, st>>>(F.n, F.agg, F.flags, F.cen, C.cen, inv_scale, ratio, C.xo, F.x, sc);
    level_post<T, 4>(F, se, b, F.x, out, sc, st);
  }
}

}  // namespace

hipError_t amg_setup(lgdm_ctx* c, std::string& msg) {
  if (c->dim != 3 || c->nd != 4) {
    msg = "multigrid preconditioning is implemented for 3D meshes";
    return hipErrorInvalidValue;
  }
  if (c->amg_unavailable) {
    msg = "the mesh has no usable multigrid hierarchy";
    return hipErrorInvalidValue;
  }
  const bool mixed = c->precision == LGDM_MIXED;
  if (!c->amg) {
    Amg* m = new Amg();
    m->mixed = mixed;
    hipError_t e = build(c, *m, msg);
    if (e != hipSuccess) {
      // its device arrays stay among the context's allocations until the
      // mesh is freed; a mesh without a hierarchy is not tried again
      delete m;
      if (e == hipErrorInvalidValue) c->amg_unavailable = true;
      return e;
    }
    c->amg = m;
  }
  return mixed ? numeric<float>(c, *c->amg) : numeric<double>(c, *c->amg);
}

hipError_t amg_apply(lgdm_ctx* c, const double* in, double* out, const double* sc, hipStream_t st) {
  if (zone_active(c)) return zone_apply(c, in, out, sc, st);
  return amg_cycle(c, in, out, sc, st);
}

hipError_t amg_cycle(lgdm_ctx* c, const double* in, double* out, const double* sc, hipStream_t st) {
  if (!c->amg) return hipErrorInvalidValue;
  if (c->amg->mixed) vcycle<float>(c, *c->amg, 0, in, out, sc, st);
  else vcycle<double>(c, *c->amg, 0, in, out, sc, st);
  return hipGetLastError();
}

void amg_release(lgdm_ctx* c) {
  delete c->amg;
  c->amg = nullptr;
}

void amg_info(const lgdm_ctx* c, AmgInfo& info) {
  info = AmgInfo{};
  if (!c->amg) return;
  info.levels = (int)std::min<size_t>(c->amg->lv.size(), 16);
  for (int l = 0; l < info.levels; ++l) {
    info.nodes[l] = c->amg->lv[l].n;
    info.pairs[l] = c->amg->lv[l].npairs;
  }
}

}  // namespace lgdm

extern "C" lgdm_status lgdm_amg_aggregate(int64_t n, const int32_t* ptr, const int32_t* adj, int32_t* agg,
                                          int64_t* n_agg) {
  if (n < 0 || !ptr || !agg || !n_agg || (n > 0 && !adj && ptr[n] > 0)) return LGDM_ERR_INVALID_ARG;
  if (ptr[0] != 0) return LGDM_ERR_INVALID_ARG;
  for (int64_t a = 0; a < n; ++a) {
    if (ptr[a + 1] < ptr[a]) return LGDM_ERR_INVALID_ARG;
    for (int32_t p = ptr[a]; p < ptr[a + 1]; ++p)
      if (adj[p] < 0 || adj[p] >= n) return LGDM_ERR_INVALID_ARG;
  }
  std::vector<int32_t> P(ptr, ptr + n + 1), A(adj, adj + (n > 0 ? ptr[n] : 0)), out;
  *n_agg = lgdm::aggregate(n, P, A, out);
  std::copy(out.begin(), out.end(), agg);
  return LGDM_OK;
}
