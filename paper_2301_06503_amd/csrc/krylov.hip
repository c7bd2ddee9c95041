// Linear solve of the Newton system (Eq. 11; H6): right-preconditioned
// BiCGSTAB with per-node (dim+1)x(dim+1) block-Jacobi, written for the
// node-blocked CSR the assembly produces.
//
//  - SpMV uses the node graph for its column indices (one int per node pair
//    instead of one per nonzero): row r of node a lists, for each neighbour
//    q of a in ascending order, the nd columns q*nd .. q*nd + nd - 1.  The nd
//    rows of a node share their columns, so a lane group computes them
//    together and gathers each x entry once.
//  - Rows of the micro-equivalent-strain equation carry the coupling
//    modulus h (about 1e-9 of the displacement rows); the solver works on
//    S K with S = diag(1 on u rows, E/h on ebar rows) and S b.  Per-field
//    relative residuals are unchanged by S.
//  - Scalars (rho, alpha, omega, residual norms, done flag) live in device
//    memory; every reduction is a fixed-order sum of per-block partials
//    finished by a one-workgroup scalar kernel next on the stream (no
//    device-scope fences, which write back L2 on every block of a
//    multi-XCD part), so results are bitwise repeatable.  The host reads the
//    scalars every `check_every` iterations.
//  - FP64 contexts run everything in FP64.  Mixed contexts store the matrix
//    and the block-Jacobi inverses in FP32 (the bytes that bound an
//    iteration) and apply them in FP64 arithmetic to FP64 Krylov vectors, so
//    the inner operator is the fixed linear map of the FP32 matrix: an FP32
//    accumulation would make it a noisy map whose rounding, once the Newton
//    residual is smooth, exceeds K p and stalls the refinement.
#include <cmath>
#include <memory>
#include <type_traits>

#include "lgdm_internal.h"

namespace lgdm {

namespace {

constexpr int BS = 256;
constexpr int MAX_GRID = 2048;

// device scalar slots
enum {
  K_RHO = 0, K_RHO_OLD, K_ALPHA, K_OMEGA, K_BETA, K_RU, K_RE, K_BU, K_BE, K_DONE, K_STATUS,
  K_ITER, K_TOL2, K_SE, K_RH2, K_B2, K_BRK, K_NSLOTS = 24
};
// status values
enum { KS_RUN = 0, KS_CONV = 1, KS_BREAK = 2, KS_NAN = 3 };
// a recurrence scalar below this fraction of the norms it is made of is a
// breakdown (~1e2 ulp of the FP64 Krylov vectors)
template <typename T> constexpr double break_rel() { return 1e-14; }
// residual at this fraction of |S b| is at the FP64 precision floor: stop
constexpr double FLOOR_REL2 = 1e-30;
// a field is judged against max(|b_field|, FIELD_FLOOR |b|): the scaled fields
// have comparable magnitudes, and a field whose right-hand side is far below
// the other's cannot be resolved below the operator's rounding of the other
constexpr double FIELD_FLOOR2 = 1e-6;
// iterations without a new best residual after which a solve has stagnated
// (the FP32 operator of a mixed context bounds the attainable residual)
constexpr int STALL_ITERS = 500;

struct Vecs {
  void* r;
  void* rh;
  void* p;
  void* v;
  void* s;
  void* t;
  void* ph;
  void* sh;
};

__device__ __forceinline__ double row_scale(int64_t row, int nd, double se) {
  return (row % nd == nd - 1) ? se : 1.0;
}

// fixed-order block reduction of NQ values; result in lane 0
template <int NQ>
__device__ __forceinline__ void block_sum(double (&v)[NQ], double (*sm)[BS]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < NQ; ++q) sm[q][t] = v[q];
  __syncthreads();
  for (int w = BS / 2; w > 0; w >>= 1) {
    if (t < w)
#pragma unroll
      for (int q = 0; q < NQ; ++q) sm[q][t] += sm[q][t + w];
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] = sm[q][0];
}

// write this block's fixed-order partial sums (the scalar kernel that
// follows on the stream finishes the reduction)
template <int NQ>
__device__ __forceinline__ void write_partials(double (&v)[NQ], double* part, double (*sm)[BS]) {
  block_sum<NQ>(v, sm);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) part[blockIdx.x * NQ + q] = v[q];
}

// y = S A x (+ optional dots).  One group of G lanes per node a computes the
// ND rows of the node together: lane v takes column v of the node's row block
// (neighbour q = v / ND, component c = v % ND), gathers x once and multiplies
// it into the ND rows (coalesced reads of each row), then the group reduces
// its ND sums.  Grid-stride over nodes.
// MODE 0: no dots; 1: dot(rh, y), |y|^2; 2: dot(y, s), |y|^2
template <typename T, int ND, int G, int UNR, int MODE>
__global__ void __launch_bounds__(BS) spmv_kernel(int64_t n_nodes, const int32_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ nbr_ptr,
                                                  const int32_t* __restrict__ nbr,
                                                  const T* __restrict__ vals,
                                                  const double* __restrict__ x,
                                                  double* __restrict__ y, const double* __restrict__ w,
                                                  const double* __restrict__ sc,
                                                  double* __restrict__ part) {
  __shared__ double sm[2][BS];
  if (sc[K_DONE] != 0.0) return;
  const double se = sc[K_SE];
  const int lane = threadIdx.x % G;
  const int64_t grp = ((int64_t)blockIdx.x * BS + threadIdx.x) / G;
  const int64_t ngrp = (int64_t)gridDim.x * BS / G;
  double d0 = 0.0, d1 = 0.0;
  for (int64_t a = grp; a < n_nodes; a += ngrp) {
    const int32_t p0 = nbr_ptr[a];
    const int len = (nbr_ptr[a + 1] - p0) * ND;
    const T* __restrict__ rv = vals + row_ptr[a * ND];
    const int32_t* __restrict__ nb = nbr + p0;
    // stored values of type T (FP32 in mixed contexts), FP64 arithmetic:
    // the operator is the fixed linear map of the stored matrix
    double acc[ND];
#pragma unroll
    for (int r = 0; r < ND; ++r) acc[r] = 0.0;
    for (int v0 = lane; v0 < len; v0 += UNR * G) {
      double xv[UNR];
      T mv[UNR][ND];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int v = v0 + u * G;
        if (v < len) {
          const int q = v / ND, c = v - q * ND;
          xv[u] = x[(int64_t)nb[q] * ND + c];
#pragma unroll
          for (int r = 0; r < ND; ++r) mv[u][r] = rv[r * len + v];
        } else {
          xv[u] = 0.0;
#pragma unroll
          for (int r = 0; r < ND; ++r) mv[u][r] = (T)0;
        }
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u)
#pragma unroll
        for (int r = 0; r < ND; ++r) acc[r] += (double)mv[u][r] * xv[u];
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1)
#pragma unroll
      for (int r = 0; r < ND; ++r) acc[r] += __shfl_xor(acc[r], o, G);
    if (lane < ND) {
      double mine = acc[0];
#pragma unroll
      for (int r = 1; r < ND; ++r)
        if (lane == r) mine = acc[r];
      const int64_t row = a * ND + lane;
      const double yt = mine * (lane == ND - 1 ? se : 1.0);
      y[row] = yt;
      if (MODE == 1) {
        d0 += w[row] * yt;
        d1 += yt * yt;
      }
      if (MODE == 2) {
        d0 += yt * w[row];
        d1 += yt * yt;
      }
    }
  }
  if (MODE == 0) return;
  double v2[2] = {d0, d1};
  write_partials<2>(v2, part, sm);
}

// finishing reductions (one workgroup): fixed-order sums of the partials and
// the BiCGSTAB scalar updates.  KIND 1: alpha; 2: omega; 3: after the x/r
// update (rho, norms, convergence, beta); 4: after init.
template <int KIND, int NQ>
__global__ void __launch_bounds__(BS) scalar_kernel(int nblk, const double* __restrict__ part,
                                                    double* __restrict__ sc) {
  __shared__ double sm[NQ][BS];
  if (KIND != 4 && sc[K_DONE] != 0.0) return;
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  for (int i = threadIdx.x; i < nblk; i += BS)
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] += part[i * NQ + q];
  block_sum<NQ>(acc, sm);
  if (threadIdx.x != 0) return;
  const double tol2 = sc[K_TOL2];
  if (KIND == 1) {  // alpha = rho / (rhat . v)
    const double den = acc[0], vv = acc[1];
    if (!isfinite(den) || !isfinite(vv)) {
      sc[K_STATUS] = KS_NAN;
      sc[K_DONE] = 1.0;
    } else if (den == 0.0 || fabs(den) <= sc[K_BRK] * sqrt(sc[K_RH2] * vv)) {
      sc[K_STATUS] = KS_BREAK;  // rhat (nearly) orthogonal to v
      sc[K_DONE] = 1.0;
    } else {
      sc[K_ALPHA] = sc[K_RHO] / den;
    }
  } else if (KIND == 2) {  // omega = (t . s) / (t . t)
    const double ts = acc[0], tt = acc[1];
    if (!isfinite(ts) || !isfinite(tt)) {
      sc[K_STATUS] = KS_NAN;
      sc[K_DONE] = 1.0;
    } else {
      sc[K_OMEGA] = (tt > 0.0) ? ts / tt : 0.0;
    }
  } else if (KIND == 3) {
    const double rho = acc[0];
    const double al = sc[K_ALPHA], om = sc[K_OMEGA];
    sc[K_RU] = acc[1];
    sc[K_RE] = acc[2];
    sc[K_ITER] += 1.0;
    if (!isfinite(rho) || !isfinite(acc[1]) || !isfinite(acc[2])) {
      sc[K_STATUS] = KS_NAN;
      sc[K_DONE] = 1.0;
      return;
    }
    const double r2 = acc[1] + acc[2];
    if ((acc[1] <= tol2 * sc[K_BU] && acc[2] <= tol2 * sc[K_BE]) || r2 <= FLOOR_REL2 * sc[K_B2]) {
      sc[K_STATUS] = KS_CONV;
      sc[K_DONE] = 1.0;
      return;
    }
    if (om == 0.0 || rho == 0.0 || fabs(rho) <= sc[K_BRK] * sqrt(sc[K_RH2] * r2)) {
      sc[K_STATUS] = KS_BREAK;
      sc[K_DONE] = 1.0;
      return;
    }
    sc[K_BETA] = (rho / sc[K_RHO]) * (al / om);
    sc[K_RHO_OLD] = sc[K_RHO];
    sc[K_RHO] = rho;
  } else {  // KIND 4: after init: rho, |r_u|^2, |r_e|^2, |b_u|^2, |b_e|^2
    const double bu = acc[3], be = acc[4];
    const double btot = bu + be;
    sc[K_BU] = fmax(bu, FIELD_FLOOR2 * btot);
    sc[K_BE] = fmax(be, FIELD_FLOOR2 * btot);
    sc[K_B2] = btot;
    sc[K_RH2] = acc[0];
    sc[K_RHO] = acc[0];
    sc[K_RHO_OLD] = acc[0];
    sc[K_ALPHA] = 1.0;
    sc[K_OMEGA] = 1.0;
    sc[K_BETA] = 0.0;
    sc[K_RU] = acc[1];
    sc[K_RE] = acc[2];
    if (!isfinite(acc[0])) {
      sc[K_STATUS] = KS_NAN;
      sc[K_DONE] = 1.0;
    } else if (btot == 0.0 || (acc[1] <= tol2 * sc[K_BU] && acc[2] <= tol2 * sc[K_BE]) ||
               acc[0] <= FLOOR_REL2 * btot) {
      sc[K_STATUS] = KS_CONV;
      sc[K_DONE] = 1.0;
    } else {
      sc[K_STATUS] = KS_RUN;
      sc[K_DONE] = 0.0;
    }
  }
}

// p = r + beta (p - omega v); ph = M^-1 p    (one thread per node)
template <typename T, int ND>
__global__ void __launch_bounds__(BS) pupdate_kernel(int64_t n_nodes, const T* __restrict__ minv,
                                                     const double* __restrict__ r, double* __restrict__ p,
                                                     const double* __restrict__ v, double* __restrict__ ph,
                                                     const double* __restrict__ sc) {
  if (sc[K_DONE] != 0.0) return;
  const double beta = sc[K_BETA], om = sc[K_OMEGA];
  for (int64_t a = (int64_t)blockIdx.x * BS + threadIdx.x; a < n_nodes; a += (int64_t)gridDim.x * BS) {
    double pv[ND];
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      const int64_t k = a * ND + i;
      pv[i] = r[k] + beta * (p[k] - om * v[k]);
      p[k] = pv[i];
    }
    const T* m = minv + a * ND * ND;
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < ND; ++j) s += (double)m[i * ND + j] * pv[j];
      ph[a * ND + i] = s;
    }
  }
}

// s = r - alpha v; sh = M^-1 s
template <typename T, int ND>
__global__ void __launch_bounds__(BS) supdate_kernel(int64_t n_nodes, const T* __restrict__ minv,
                                                     const double* __restrict__ r, const double* __restrict__ v,
                                                     double* __restrict__ s, double* __restrict__ sh,
                                                     const double* __restrict__ sc) {
  if (sc[K_DONE] != 0.0) return;
  const double al = sc[K_ALPHA];
  for (int64_t a = (int64_t)blockIdx.x * BS + threadIdx.x; a < n_nodes; a += (int64_t)gridDim.x * BS) {
    double sv[ND];
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      const int64_t k = a * ND + i;
      sv[i] = r[k] - al * v[k];
      s[k] = sv[i];
    }
    const T* m = minv + a * ND * ND;
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < ND; ++j) acc += (double)m[i * ND + j] * sv[j];
      sh[a * ND + i] = acc;
    }
  }
}

// x += alpha ph + omega sh; r = s - omega t; partials of rho, |r_u|^2, |r_e|^2
template <int ND>
__global__ void __launch_bounds__(BS) xupdate_kernel(int64_t n, double* __restrict__ x,
                                                     const double* __restrict__ ph, const double* __restrict__ sh,
                                                     const double* __restrict__ s, const double* __restrict__ t,
                                                     double* __restrict__ r, const double* __restrict__ rh,
                                                     const double* __restrict__ sc,
                                                     double* __restrict__ part) {
  __shared__ double sm[3][BS];
  if (sc[K_DONE] != 0.0) return;
  const double al = sc[K_ALPHA], om = sc[K_OMEGA];
  double d[3] = {0.0, 0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
    x[i] += al * ph[i] + om * sh[i];
    const double rd = s[i] - om * t[i];
    r[i] = rd;
    d[0] += rh[i] * rd;
    if (i % ND == ND - 1) d[2] += rd * rd;
    else d[1] += rd * rd;
  }
  write_partials<3>(d, part, sm);
}

// r = S b - y, rh = r, p = v = 0; partials of rho and the field norms of r and S b
template <int ND>
__global__ void __launch_bounds__(BS) init_kernel(int64_t n, const double* __restrict__ b,
                                                  const double* __restrict__ y, int use_y, double* __restrict__ r,
                                                  double* __restrict__ rh, double* __restrict__ p,
                                                  double* __restrict__ v, const double* __restrict__ sc,
                                                  double* __restrict__ part) {
  __shared__ double sm[5][BS];
  const double se = sc[K_SE];
  double d[5] = {0, 0, 0, 0, 0};
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
    const bool fe = (i % ND == ND - 1);
    const double sb = b[i] * (fe ? se : 1.0);
    const double rd = sb - (use_y ? y[i] : 0.0);
    r[i] = rd;
    rh[i] = rd;
    p[i] = 0.0;
    v[i] = 0.0;
    d[0] += rd * rd;
    if (fe) {
      d[2] += rd * rd;
      d[4] += sb * sb;
    } else {
      d[1] += rd * rd;
      d[3] += sb * sb;
    }
  }
  write_partials<5>(d, part, sm);
}

// block-Jacobi: invert the scaled diagonal node blocks (Gauss-Jordan with
// partial pivoting); a singular block falls back to the identity
template <typename T, typename V, int ND>
__global__ void bjacobi_kernel(int64_t n_nodes, const int32_t* __restrict__ row_ptr,
                               const int32_t* __restrict__ dpos, const V* __restrict__ vals,
                               double se, T* __restrict__ minv) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n_nodes) return;
  double m[ND][2 * ND];
#pragma unroll
  for (int r = 0; r < ND; ++r) {
    const double s = (r == ND - 1) ? se : 1.0;
    const int64_t base = row_ptr[a * ND + r] + (int64_t)dpos[a] * ND;
#pragma unroll
    for (int c = 0; c < ND; ++c) {
      m[r][c] = s * (double)vals[base + c];
      m[r][ND + c] = (r == c) ? 1.0 : 0.0;
    }
  }
  bool ok = true;
  for (int col = 0; col < ND; ++col) {
    int piv = col;
    double best = fabs(m[col][col]);
    for (int r = col + 1; r < ND; ++r)
      if (fabs(m[r][col]) > best) {
        best = fabs(m[r][col]);
        piv = r;
      }
    if (!(best > 0.0) || !isfinite(best)) {
      ok = false;
      break;
    }
    if (piv != col)
      for (int c = 0; c < 2 * ND; ++c) {
        const double t = m[col][c];
        m[col][c] = m[piv][c];
        m[piv][c] = t;
      }
    const double inv = 1.0 / m[col][col];
    for (int c = 0; c < 2 * ND; ++c) m[col][c] *= inv;
    for (int r = 0; r < ND; ++r) {
      if (r == col) continue;
      const double f = m[r][col];
      for (int c = 0; c < 2 * ND; ++c) m[r][c] -= f * m[col][c];
    }
  }
  T* out = minv + a * ND * ND;
  for (int r = 0; r < ND; ++r)
    for (int c = 0; c < ND; ++c) out[r * ND + c] = ok ? (T)m[r][ND + c] : (T)(r == c ? 1.0 : 0.0);
}

__global__ void axpy_kernel(int64_t n, double* __restrict__ y, const double* __restrict__ x, double a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}

// |v_u|^2, |v_e|^2 of contiguous chunks (stage one of a fixed-order sum)
__global__ void __launch_bounds__(256) field_norms_kernel(int64_t n, int64_t chunk, int nd,
                                                          const double* __restrict__ v,
                                                          double* __restrict__ out) {
  __shared__ double sm[2][BS];
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  double d[2] = {0.0, 0.0};
  for (int64_t i = lo + threadIdx.x; i < hi; i += BS) {
    const double x = v[i];
    if (i % nd == nd - 1) d[1] += x * x;
    else d[0] += x * x;
  }
  block_sum<2>(d, sm);
  if (threadIdx.x == 0) {
    out[blockIdx.x * 2] = d[0];
    out[blockIdx.x * 2 + 1] = d[1];
  }
}

__global__ void __launch_bounds__(256) pair_sum_kernel(int nblk, const double* __restrict__ in,
                                                       double* __restrict__ out) {
  __shared__ double sm[2][BS];
  double d[2] = {0.0, 0.0};
  for (int i = threadIdx.x; i < nblk; i += BS) {
    d[0] += in[2 * i];
    d[1] += in[2 * i + 1];
  }
  block_sum<2>(d, sm);
  if (threadIdx.x == 0) {
    out[0] = d[0];
    out[1] = d[1];
  }
}

__global__ void set_scalars_kernel(double* sc, double tol2, double se, double brk) {
  if (threadIdx.x == 0) {
    for (int i = 0; i < K_NSLOTS; ++i) sc[i] = 0.0;
    sc[K_TOL2] = tol2;
    sc[K_SE] = se;
    sc[K_BRK] = brk;
  }
}

inline int64_t grid_for(int64_t work) {
  int64_t g = (work + BS - 1) / BS;
  if (g > MAX_GRID) g = MAX_GRID;
  return g < 1 ? 1 : g;
}

template <typename T, int ND>
struct Solver {
  // lanes per node in the SpMV and unroll depth: row blocks hold up to
  // 27 x 4 (hex8), 9 x 3 (quad4) and 3 x 2 (line2) columns, so G * UNR
  // covers a hex8 row block in one unrolled pass (measured on the 3D beam:
  // FP32 values favour a full wave per node, FP64 two nodes per wave)
  static constexpr bool F32 = std::is_same<T, float>::value;
  static constexpr int G = ND == 4 ? (F32 ? 64 : 32) : (ND == 3 ? 8 : 2);
  static constexpr int UNR = ND == 4 ? (F32 ? 2 : 4) : 4;
  lgdm_ctx* c;
  const T* vals;
  const T* minv;
  Vecs V;
  double* sc;
  int64_t n, nn;

  double* vec(void* p) { return static_cast<double*>(p); }

  void spmv(const double* x, double* y, int mode, const double* w) {
    const int64_t g = grid_for(nn * G);
    if (mode == 0) {
      spmv_kernel<T, ND, G, UNR, 0><<<g, BS, 0, c->stream>>>(nn, c->row_ptr, c->nbr_ptr, c->nbr, vals, x, y,
                                                        w, sc, c->kpart);
    } else if (mode == 1) {
      spmv_kernel<T, ND, G, UNR, 1><<<g, BS, 0, c->stream>>>(nn, c->row_ptr, c->nbr_ptr, c->nbr, vals, x, y,
                                                        w, sc, c->kpart);
      scalar_kernel<1, 2><<<1, BS, 0, c->stream>>>((int)g, c->kpart, sc);
    } else {
      spmv_kernel<T, ND, G, UNR, 2><<<g, BS, 0, c->stream>>>(nn, c->row_ptr, c->nbr_ptr, c->nbr, vals, x, y,
                                                        w, sc, c->kpart);
      scalar_kernel<2, 2><<<1, BS, 0, c->stream>>>((int)g, c->kpart, sc);
    }
  }

  void init(const double* b, bool use_y, const double* y) {
    const int64_t g = grid_for(n);
    init_kernel<ND><<<g, BS, 0, c->stream>>>(n, b, y, use_y ? 1 : 0, vec(V.r), vec(V.rh), vec(V.p),
                                             vec(V.v), sc, c->kpart);
    scalar_kernel<4, 5><<<1, BS, 0, c->stream>>>((int)g, c->kpart, sc);
  }

  void iteration(double* x) {
    const int64_t gn = grid_for(nn);
    pupdate_kernel<T, ND><<<gn, BS, 0, c->stream>>>(nn, minv, vec(V.r), vec(V.p), vec(V.v), vec(V.ph), sc);
    spmv(vec(V.ph), vec(V.v), 1, vec(V.rh));
    supdate_kernel<T, ND><<<gn, BS, 0, c->stream>>>(nn, minv, vec(V.r), vec(V.v), vec(V.s), vec(V.sh), sc);
    spmv(vec(V.sh), vec(V.t), 2, vec(V.s));
    const int64_t g = grid_for(n);
    xupdate_kernel<ND><<<g, BS, 0, c->stream>>>(n, x, vec(V.ph), vec(V.sh), vec(V.s), vec(V.t),
                                                vec(V.r), vec(V.rh), sc, c->kpart);
    scalar_kernel<3, 3><<<1, BS, 0, c->stream>>>((int)g, c->kpart, sc);
  }
};

// One linear solve as a state machine: start() enqueues the initial
// residual, then alternately check() (reads the device scalars; decides
// convergence, restart, stagnation) and launch() (enqueues check_every
// iterations) until finished().  Several runs on different streams can be
// interleaved by the host so their kernels overlap on the device.
template <typename T, int ND>
struct KrylovRunImpl final : KrylovRun {
  Solver<T, ND> S;
  lgdm_ctx* c;
  const double* b;
  double* xout;
  lgdm_solver_opts o;
  KrylovResult res{};
  double tol = 0, se = 0;
  int every = 16;
  int64_t done_iters = 0;
  bool true_residual = true;   // the scalars describe b - A x computed directly
  int replacements = 0;
  double* xbest = nullptr;     // best iterate so far (per-field relative residual)
  double best = INFINITY;
  int stall = 0;
  bool have_best = false;
  bool fin = false;

  KrylovRunImpl(lgdm_ctx* ctx, const double* b_, double* x_, const lgdm_solver_opts& o_)
      : c(ctx), b(b_), xout(x_), o(o_) {
    S.c = c;
    S.n = c->ndof;
    S.nn = c->n_nodes;
    const bool mixed = std::is_same<T, float>::value;
    S.vals = mixed ? (const T*)c->vals32 : (const T*)c->vals;
    S.minv = mixed ? (const T*)c->minv32 : (const T*)c->minv;
    void** vp[8] = {&S.V.r, &S.V.rh, &S.V.p, &S.V.v, &S.V.s, &S.V.t, &S.V.ph, &S.V.sh};
    for (int i = 0; i < 8; ++i) *vp[i] = c->kv + (int64_t)i * c->ndof;
    S.sc = c->kscal;
    xbest = c->kv + 8 * c->ndof;
    tol = o.tol_krylov;
    if (mixed && tol < 1e-8) tol = 1e-8;  // FP32 matrix; Newton refines on the FP64 residual
    se = c->mat.E / c->mat.h;
    every = o.check_every > 0 ? o.check_every : 16;
    res.status = LGDM_ERR_NOT_CONVERGED;
  }

  void return_best(int status) {
    if (have_best)
      (void)hipMemcpyAsync(xout, xbest, c->ndof * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
    res.status = status;
    fin = true;
  }

  // restart the recurrences from the current iterate with its true residual
  void restart_from_x() {
    set_scalars_kernel<<<1, 64, 0, c->stream>>>(S.sc, tol * tol, se, break_rel<T>());
    S.spmv(xout, S.vec(S.V.t), 0, nullptr);
    S.init(b, true, S.vec(S.V.t));
  }

  hipError_t start() override {
    set_scalars_kernel<<<1, 64, 0, c->stream>>>(S.sc, tol * tol, se, break_rel<T>());
    hipError_t e = hipMemsetAsync(xout, 0, c->ndof * sizeof(double), c->stream);
    if (e != hipSuccess) return e;
    S.init(b, false, nullptr);
    // read the scalars of the initial residual asynchronously
    return hipMemcpyAsync(c->kscal_host, S.sc, K_NSLOTS * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream);
  }

  hipError_t launch() override {
    if (fin) return hipSuccess;
    for (int i = 0; i < every; ++i) S.iteration(xout);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(c->kscal_host, S.sc, K_NSLOTS * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream);
  }

  // reads the scalars enqueued by the last start()/launch(); restart and
  // replacement kernels are enqueued here and read at the next check
  hipError_t check() override {
    if (fin) return hipSuccess;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return e;
    const double* h = c->kscal_host;
    res.iters = done_iters + (int64_t)h[K_ITER];
    const double bu = h[K_BU] > 0 ? h[K_BU] : 1.0, be = h[K_BE] > 0 ? h[K_BE] : 1.0;
    res.rel_u = std::sqrt(h[K_RU] / bu);
    res.rel_e = std::sqrt(h[K_RE] / be);
    const int st = (int)h[K_STATUS];
    pending_read = false;
    if (h[K_DONE] != 0.0) {
      if (st == KS_CONV) {
        // accept only a converged true residual; a converged recurrence
        // residual is first replaced by the true one (it can drift)
        if (true_residual || replacements >= 4) {
          res.status = LGDM_OK;
          fin = true;
          return hipSuccess;
        }
        replacements++;
        done_iters = res.iters;
        restart_from_x();
        true_residual = true;
        pending_read = true;
        return hipMemcpyAsync(c->kscal_host, S.sc, K_NSLOTS * sizeof(double), hipMemcpyDeviceToHost,
                              c->stream);
      }
      if (st == KS_NAN) {
        if (have_best) return_best(LGDM_ERR_NOT_CONVERGED);
        else {
          res.status = LGDM_ERR_NAN;
          fin = true;
        }
        return hipSuccess;
      }
      // breakdown: restart from the current iterate with the true residual
      if (res.restarts >= o.max_restarts || res.iters >= o.max_krylov) {
        res.status = LGDM_ERR_BREAKDOWN;
        fin = true;
        return hipSuccess;
      }
      res.restarts++;
      done_iters = res.iters;
      restart_from_x();
      true_residual = true;
      pending_read = true;
      return hipMemcpyAsync(c->kscal_host, S.sc, K_NSLOTS * sizeof(double), hipMemcpyDeviceToHost,
                            c->stream);
    }
    true_residual = false;
    const double score = std::max(res.rel_u, res.rel_e);
    if (std::isfinite(score) && score < best * (1.0 - 1e-3)) {
      best = score;
      stall = 0;
      have_best = true;
      e = hipMemcpyAsync(xbest, xout, c->ndof * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
      if (e != hipSuccess) return e;
    } else if ((stall += every) >= STALL_ITERS) {
      return_best(LGDM_ERR_NOT_CONVERGED);
      return hipSuccess;
    }
    if (res.iters >= o.max_krylov) return_best(LGDM_ERR_NOT_CONVERGED);
    return hipSuccess;
  }

  bool pending_read = false;   // a restart's scalars are in flight: check again before launching
  bool needs_check() const override { return pending_read; }
  bool finished() const override { return fin; }
  const KrylovResult& result() const override { return res; }
};

template <typename T, int ND>
std::unique_ptr<KrylovRun> make_run_impl(lgdm_ctx* c, const double* b, double* x,
                                         const lgdm_solver_opts& o) {
  return std::unique_ptr<KrylovRun>(new KrylovRunImpl<T, ND>(c, b, x, o));
}

template <typename T, int ND> hipError_t setup_impl(lgdm_ctx* c) {
  const double se = c->mat.E / c->mat.h;
  const int64_t g = (c->n_nodes + 127) / 128;
  if (c->precision == LGDM_MIXED)
    bjacobi_kernel<float, float, ND><<<g, 128, 0, c->stream>>>(c->n_nodes, c->row_ptr, c->dpos,
                                                               c->vals32, se, c->minv32);
  else
    bjacobi_kernel<double, double, ND><<<g, 128, 0, c->stream>>>(c->n_nodes, c->row_ptr, c->dpos,
                                                                 c->vals, se, c->minv);
  return hipGetLastError();
}

}  // namespace

hipError_t krylov_setup(lgdm_ctx* c) {
  switch (c->nd) {
    case 2: return setup_impl<double, 2>(c);
    case 3: return setup_impl<double, 3>(c);
    default: return setup_impl<double, 4>(c);
  }
}

std::unique_ptr<KrylovRun> make_krylov_run(lgdm_ctx* c, const double* b, double* x,
                                           const lgdm_solver_opts& o) {
  const bool mixed = c->precision == LGDM_MIXED;
  switch (c->nd) {
    case 2: return mixed ? make_run_impl<float, 2>(c, b, x, o) : make_run_impl<double, 2>(c, b, x, o);
    case 3: return mixed ? make_run_impl<float, 3>(c, b, x, o) : make_run_impl<double, 3>(c, b, x, o);
    default: return mixed ? make_run_impl<float, 4>(c, b, x, o) : make_run_impl<double, 4>(c, b, x, o);
  }
}

hipError_t krylov_solve(lgdm_ctx* c, const double* b, double* xout, const lgdm_solver_opts& o,
                        KrylovResult& res) {
  std::unique_ptr<KrylovRun> run = make_krylov_run(c, b, xout, o);
  hipError_t e = run->start();
  while (e == hipSuccess) {
    e = run->check();
    if (e != hipSuccess || run->finished()) break;
    if (!run->needs_check()) e = run->launch();
  }
  res = run->result();
  return e;
}

template <typename T, int ND> hipError_t spmv_only_impl(lgdm_ctx* c, const double* x) {
  Solver<T, ND> S;
  S.c = c;
  S.n = c->ndof;
  S.nn = c->n_nodes;
  const bool mixed = std::is_same<T, float>::value;
  S.vals = mixed ? (const T*)c->vals32 : (const T*)c->vals;
  S.sc = c->kscal;
  set_scalars_kernel<<<1, 64, 0, c->stream>>>(S.sc, 0.0, c->mat.E / c->mat.h, break_rel<T>());
  S.spmv(x, c->kv, 0, nullptr);
  return hipGetLastError();
}

// y = S K x into the Krylov workspace (timing of the SpMV kernel alone)
hipError_t launch_spmv_only(lgdm_ctx* c, const double* x, double*) {
  const bool mixed = c->precision == LGDM_MIXED;
  switch (c->nd) {
    case 2: return mixed ? spmv_only_impl<float, 2>(c, x) : spmv_only_impl<double, 2>(c, x);
    case 3: return mixed ? spmv_only_impl<float, 3>(c, x) : spmv_only_impl<double, 3>(c, x);
    default: return mixed ? spmv_only_impl<float, 4>(c, x) : spmv_only_impl<double, 4>(c, x);
  }
}

hipError_t launch_axpy(lgdm_ctx* c, double* y, const double* x, double a, int64_t n) {
  if (n == 0) return hipSuccess;
  axpy_kernel<<<(n + 255) / 256, 256, 0, c->stream>>>(n, y, x, a);
  return hipGetLastError();
}

hipError_t launch_field_norms(lgdm_ctx* c, const double* v, double* out_dev) {
  const int64_t n = c->ndof;
  const int64_t nb1 = (n + BS - 1) / BS < RED_CHUNKS ? (n + BS - 1) / BS : RED_CHUNKS;
  const int64_t chunk = (n + nb1 - 1) / nb1;
  field_norms_kernel<<<nb1, BS, 0, c->stream>>>(n, chunk, c->nd, v, c->red2);
  pair_sum_kernel<<<1, BS, 0, c->stream>>>((int)nb1, c->red2, out_dev);
  return hipGetLastError();
}

}  // namespace lgdm
