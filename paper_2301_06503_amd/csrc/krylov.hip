// Linear solve of the Newton system (Eq. 11; H6), written for the
// node-blocked CSR the assembly produces: right-preconditioned IDR(s)
// (van Gijzen & Sonneveld 2011; s = 8 by default) or BiCGSTAB (van der Vorst
// 1992), preconditioned by the aggregation multigrid cycle of amg.hip on 3D
// meshes (with the dense process-zone solve of zone.hip) and by per-node
// (dim+1)x(dim+1) block-Jacobi otherwise.
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
#include <algorithm>
#include <cmath>
#include <memory>
#include <type_traits>

#include "lgdm_internal.h"

namespace lgdm {

namespace {

constexpr int BS = 256;
constexpr int MAX_GRID = KPART_BLOCKS;

// device scalar slots
enum {
  K_RHO = 0, K_RHO_OLD, K_ALPHA, K_OMEGA, K_BETA, K_RU, K_RE, K_BU, K_BE, K_DONE, K_STATUS,
  K_ITER, K_TOL2, K_SE, K_RH2, K_B2, K_BRK, K_TOL2E, K_SEED, K_NSLOTS = 24
};
static_assert(K_DONE == KSLOT_DONE, "done slot shared with the multigrid kernels");
// status values
enum { KS_RUN = 0, KS_CONV = 1, KS_BREAK = 2, KS_NAN = 3 };
// a recurrence scalar below this fraction of the norms it is made of is a
// breakdown (~1e2 ulp of the FP64 Krylov vectors)
constexpr double BREAK_REL = 1e-14;
// residual at this fraction of |S b| is at the FP64 precision floor: stop
constexpr double FLOOR_REL2 = 1e-30;
// a recurrence residual grown beyond this multiple of |S b| (squared) has
// left any useful range: a breakdown, restarted from the best iterate
constexpr double GROWTH2 = 1e8;
// a field is judged against max(|b_field|, FIELD_FLOOR |b|): the scaled fields
// have comparable magnitudes, and a field whose right-hand side is far below
// the other's cannot be resolved below the operator's rounding of the other
constexpr double FIELD_FLOOR2 = 1e-6;
// iterations without a new best residual after which a solve has stagnated
// and returns its best iterate.  A solve that has not yet improved on its
// zero start waits as long as it has run (IDR(s) residuals can plateau for
// hundreds of steps before they drop; returning nothing would repeat the
// Newton iteration unchanged).
constexpr int STALL_ITERS = 500;
// IDR(s) minimal-residual step: omega is enlarged until the cosine of the
// angle between t and r it implies is at least this (van Gijzen & Sonneveld)
constexpr double IDR_KAPPA = 0.7;

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
__device__ __forceinline__ void write_partials(double (&v)[NQ], double* part, int64_t blk, double (*sm)[BS]) {
  block_sum<NQ>(v, sm);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) part[blk * NQ + q] = v[q];
}

// Entry j of the q-th IDR shadow vector: a uniform deviate in [-1, 1) from
// the splitmix64 output function (Steele, Lea & Flood, OOPSLA 2014) applied
// to the counter (q + 1) * 2^40 + j.  Computed where it is used, never stored.
__device__ __forceinline__ double shadow_entry(int q, int64_t j) {
  uint64_t z = ((uint64_t)(q + 1) << 40) ^ (uint64_t)j;
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * 0x1.0p-52 - 1.0;
}

// ND consecutive values as one load: 4-wide vectors for the 3D blocks (the
// row blocks of a node start at multiples of 16 values and every vector the
// library allocates is 32-byte aligned), element by element otherwise
template <typename T, int ND> struct Quad {
  T v[ND];
  __device__ __forceinline__ void load(const T* __restrict__ p) {
#pragma unroll
    for (int c = 0; c < ND; ++c) v[c] = p[c];
  }
  __device__ __forceinline__ void store(T* __restrict__ p) const {
#pragma unroll
    for (int c = 0; c < ND; ++c) p[c] = v[c];
  }
};
template <> struct Quad<float, 4> {
  float v[4];
  __device__ __forceinline__ void load(const float* __restrict__ p) {
    const float4 q = *reinterpret_cast<const float4*>(p);
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  }
};
template <> struct Quad<double, 4> {
  double v[4];
  __device__ __forceinline__ void load(const double* __restrict__ p) {
    const double4 q = *reinterpret_cast<const double4*>(p);
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  }
  __device__ __forceinline__ void store(double* __restrict__ p) const {
    *reinterpret_cast<double4*>(p) = make_double4(v[0], v[1], v[2], v[3]);
  }
};

// Sum the ND per-lane values acc over the G lanes of a group.  Returns the
// row this lane holds the total of, or -1.  ND = 4: each of the first two
// butterfly stages exchanges only the half of the values the partner keeps
// (7 exchanges instead of 4 log2 G); rows end in lanes 0, G/4, G/2, 3G/4.
template <int ND, int G>
__device__ __forceinline__ int group_rows(double (&acc)[ND], int lane, double& total) {
  if (ND == 4 && G >= 4) {
    const bool h1 = lane & (G / 2);
    double k0 = h1 ? acc[2] : acc[0], k1 = h1 ? acc[3] : acc[1];
    const double s0 = h1 ? acc[0] : acc[2], s1 = h1 ? acc[1] : acc[3];
    k0 += __shfl_xor(s0, G / 2, G);
    k1 += __shfl_xor(s1, G / 2, G);
    const bool h2 = lane & (G / 4);
    double k = h2 ? k1 : k0;
    const double s = h2 ? k0 : k1;
    k += __shfl_xor(s, G / 4, G);
#pragma unroll
    for (int o = G / 8; o > 0; o >>= 1) k += __shfl_xor(k, o, G);
    total = k;
    return (lane % (G / 4)) == 0 ? (h1 ? 2 : 0) + (h2 ? 1 : 0) : -1;
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1)
#pragma unroll
    for (int r = 0; r < ND; ++r) acc[r] += __shfl_xor(acc[r], o, G);
  total = acc[0];
#pragma unroll
  for (int r = 1; r < ND; ++r)
    if (lane == r) total = acc[r];
  return lane < ND ? lane : -1;
}

// y = S A x (+ optional dots).  One group of G lanes per node a computes the
// ND rows of the node together.  Lane q takes neighbour q of a (ascending):
// it reads the neighbour's ND entries of x and, from each of the node's ND
// rows, the ND values of the (row, neighbour) block (row r of node a lists
// neighbour q's columns at r * len + q * ND), so x is gathered once per
// neighbour and every read is ND values wide.  Grid-stride over nodes.
// MODE 0: no dots; 1: dot(rh, y), |y|^2; 2: dot(y, s), |y|^2;
// 3: the NP shadow-vector dots P_q . y and |y|^2 (IDR)
// workgroup blk of nblk (the kernels below pass their block, the batched
// ones the block within the request)
template <typename T, int ND, int G, int MODE, int NP = 0>
__device__ __forceinline__ void spmv_body(int64_t blk, int64_t nblk, int64_t n_nodes,
                                          const int32_t* __restrict__ row_ptr,
                                          const int32_t* __restrict__ nbr_ptr, const int32_t* __restrict__ nbr,
                                          const T* __restrict__ vals, const double* __restrict__ x,
                                          double* __restrict__ y, const double* __restrict__ w,
                                          const double* __restrict__ sc, double* __restrict__ part) {
  constexpr int NQ = MODE == 3 ? NP + 1 : 2;
  __shared__ double sm[NQ][BS];
  if (sc[K_DONE] != 0.0) return;
  const double se = sc[K_SE];
  const int seed = (int)sc[K_SEED];
  const int lane = threadIdx.x % G;
  const int64_t grp = (blk * BS + threadIdx.x) / G;
  const int64_t ngrp = nblk * BS / G;
  double d[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) d[q] = 0.0;
  for (int64_t a = grp; a < n_nodes; a += ngrp) {
    const int32_t p0 = nbr_ptr[a];
    const int nnb = nbr_ptr[a + 1] - p0;
    const int len = nnb * ND;
    const T* __restrict__ rv = vals + row_ptr[a * ND];
    // stored values of type T (FP32 in mixed contexts), FP64 arithmetic:
    // the operator is the fixed linear map of the stored matrix
    double acc[ND];
#pragma unroll
    for (int r = 0; r < ND; ++r) acc[r] = 0.0;
    for (int q = lane; q < nnb; q += G) {
      Quad<double, ND> xq;
      xq.load(x + (int64_t)nbr[p0 + q] * ND);
#pragma unroll
      for (int r = 0; r < ND; ++r) {
        Quad<T, ND> m;
        m.load(rv + r * len + q * ND);
#pragma unroll
        for (int cc = 0; cc < ND; ++cc) acc[r] += (double)m.v[cc] * xq.v[cc];
      }
    }
    double total;
    const int rr = group_rows<ND, G>(acc, lane, total);
    if (rr >= 0) {
      const int64_t row = a * ND + rr;
      const double yt = total * (rr == ND - 1 ? se : 1.0);
      y[row] = yt;
      if (MODE == 1) {
        d[0] += w[row] * yt;
        d[1] += yt * yt;
      }
      if (MODE == 2) {
        d[0] += yt * w[row];
        d[1] += yt * yt;
      }
      if (MODE == 3) {
#pragma unroll
        for (int q = 0; q < NP; ++q) d[q] += shadow_entry(seed + q, row) * yt;
        d[NP] += yt * yt;
      }
    }
  }
  if (MODE == 0) return;
  write_partials<NQ>(d, part, blk, sm);
}

template <typename T, int ND, int G, int MODE, int NP = 0>
__global__ void __launch_bounds__(BS) spmv_kernel(int64_t n_nodes, const int32_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ nbr_ptr,
                                                  const int32_t* __restrict__ nbr,
                                                  const T* __restrict__ vals,
                                                  const double* __restrict__ x,
                                                  double* __restrict__ y, const double* __restrict__ w,
                                                  const double* __restrict__ sc,
                                                  double* __restrict__ part) {
  spmv_body<T, ND, G, MODE, NP>(blockIdx.x, gridDim.x, n_nodes, row_ptr, nbr_ptr, nbr, vals, x, y, w, sc, part);
}

// The one-workgroup scalar kernels end in one thread's chain of dependent
// reads and writes of the solve's scalars (forward substitutions, breakdown
// tests).  They run on a copy of the scalars in LDS, staged by the whole
// workgroup and written back after: the same arithmetic on the same values,
// without a device-memory round trip per dependent access.
__device__ __forceinline__ void stage_scalars(double* s, const double* __restrict__ sc) {
  for (int i = threadIdx.x; i < KSCAL_DOUBLES; i += BS) s[i] = sc[i];
  __syncthreads();
}
__device__ __forceinline__ void unstage_scalars(double* __restrict__ sc, const double* s) {
  __syncthreads();
  for (int i = threadIdx.x; i < KSCAL_DOUBLES; i += BS) sc[i] = s[i];
}

// finishing reductions (one workgroup): fixed-order sums of the partials and
// the BiCGSTAB scalar updates.  KIND 1: alpha; 2: omega; 3: after the x/r
// update (rho, norms, convergence, beta); 4: after init.
template <int KIND, int NQ>
__device__ __forceinline__ void scalar_body(int nblk, const double* __restrict__ part, double* sc) {
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
    if ((acc[1] <= tol2 * sc[K_BU] && acc[2] <= sc[K_TOL2E] * sc[K_BE]) || r2 <= FLOOR_REL2 * sc[K_B2]) {
      sc[K_STATUS] = KS_CONV;
      sc[K_DONE] = 1.0;
      return;
    }
    if (om == 0.0 || rho == 0.0 || fabs(rho) <= sc[K_BRK] * sqrt(sc[K_RH2] * r2) || r2 > GROWTH2 * sc[K_B2]) {
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
    } else if (btot == 0.0 || (acc[1] <= tol2 * sc[K_BU] && acc[2] <= sc[K_TOL2E] * sc[K_BE]) ||
               acc[0] <= FLOOR_REL2 * btot) {
      sc[K_STATUS] = KS_CONV;
      sc[K_DONE] = 1.0;
    } else {
      sc[K_STATUS] = KS_RUN;
      sc[K_DONE] = 0.0;
    }
  }
}

template <int KIND, int NQ>
__global__ void __launch_bounds__(BS) scalar_kernel(int nblk, const double* __restrict__ part,
                                                    double* __restrict__ sc) {
  __shared__ double s_sc[KSCAL_DOUBLES];
  stage_scalars(s_sc, sc);
  scalar_body<KIND, NQ>(nblk, part, s_sc);
  unstage_scalars(sc, s_sc);
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
  write_partials<3>(d, part, blockIdx.x, sm);
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
  write_partials<5>(d, part, blockIdx.x, sm);
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

// tol2u, tol2e: squared relative tolerances of the u and ebar rows
// seed: index offset of the IDR shadow vectors (a restart draws new ones)
__global__ void set_scalars_kernel(double* sc, double tol2u, double tol2e, double se, double brk, int seed) {
  if (threadIdx.x == 0) {
    for (int i = 0; i < K_NSLOTS; ++i) sc[i] = 0.0;
    sc[K_TOL2] = tol2u;
    sc[K_TOL2E] = tol2e;
    sc[K_SE] = se;
    sc[K_BRK] = brk;
    sc[K_SEED] = (double)seed;
  }
}

// ---------------------------------------------------------------------------
// IDR(s): induced dimension reduction (Sonneveld & van Gijzen, SIAM J. Sci.
// Comput. 31, 2008), in the biorthogonal form of van Gijzen & Sonneveld (ACM
// TOMS 38, 2011), right-preconditioned with the same block-Jacobi and the same
// scaled operator S K as BiCGSTAB (IDR(1) and BiCGSTAB span the same
// spaces).  Each cycle takes s steps that keep the new residual orthogonal to
// s shadow vectors P (generated by shadow_entry, never stored), then one
// minimal-residual step.  State: residual r, s direction pairs (G_k, U_k =
// M^-1-side vectors with G_k = S K U_k), the lower-triangular s x s matrix
// M = P^T G and f = P^T r.  A shadow space of s > 1 vectors replaces the
// single Lanczos shadow vector whose (near-)orthogonality to r breaks
// BiCGSTAB down on the indefinite tangents of the softening branch.
//
// The biorthogonalisation of a new G_k against G_0..G_{k-1} uses one fused
// set of dot products P^T g and a forward substitution with M (the
// coefficients the sequential form computes one at a time).

// scalar slots of IDR(s), after the ones it shares with BiCGSTAB
constexpr int I_OM = 24, I_BETA = 25, I_RR = 26, I_FRESH = 27, I_F = 32, I_C = 40, I_A = 48, I_M = 64;
constexpr int I_LD = 8;  // leading dimension of M in the slots

template <int NQ>
__device__ __forceinline__ void finish_partials(int64_t nblk, const double* __restrict__ part,
                                                double (&acc)[NQ], double (*sm)[BS]) {
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  for (int64_t i = threadIdx.x; i < nblk; i += BS)
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] += part[i * NQ + q];
  block_sum<NQ>(acc, sm);
}

// store the residual norms and decide convergence (one thread)
__device__ __forceinline__ bool idr_norms(double* sc, double ru, double re) {
  sc[K_RU] = ru;
  sc[K_RE] = re;
  sc[I_RR] = ru + re;
  if (!isfinite(ru) || !isfinite(re)) {
    sc[K_STATUS] = KS_NAN;
    sc[K_DONE] = 1.0;
    return true;
  }
  if ((ru <= sc[K_TOL2] * sc[K_BU] && re <= sc[K_TOL2E] * sc[K_BE]) || ru + re <= FLOOR_REL2 * sc[K_B2]) {
    sc[K_STATUS] = KS_CONV;
    sc[K_DONE] = 1.0;
    return true;
  }
  if (ru + re > GROWTH2 * sc[K_B2]) {
    sc[K_STATUS] = KS_BREAK;
    sc[K_DONE] = 1.0;
    return true;
  }
  return false;
}

// c = M[k0:s, k0:s]^-1 f[k0:s] by forward substitution (one thread)
template <int S>
__device__ __forceinline__ void idr_coeffs(double* sc, int k0) {
  for (int j = 0; j < S - k0; ++j) {
    double v = sc[I_F + k0 + j];
    for (int l = 0; l < j; ++l) v -= sc[I_M + (k0 + j) * I_LD + (k0 + l)] * sc[I_C + l];
    sc[I_C + j] = v / sc[I_M + (k0 + j) * I_LD + (k0 + j)];
  }
}

// Each IDR kernel is a device body taking its workgroup blk of nblk, so that
// a single-request kernel (blockIdx.x of gridDim.x) and a batched kernel over
// many requests (the block within its request) run the same code.

// r = S b - y; partials |r_u|^2, |r_e|^2, |(Sb)_u|^2, |(Sb)_e|^2, P^T r
template <int ND, int S>
__device__ __forceinline__ void idr_init_body(int64_t blk, int64_t nblk, int64_t n, const double* __restrict__ b,
                                              const double* __restrict__ y, double* __restrict__ r,
                                              const double* __restrict__ sc, double* __restrict__ part) {
  __shared__ double sm[4 + S][BS];
  const double se = sc[K_SE];
  const int seed = (int)sc[K_SEED];
  double d[4 + S];
#pragma unroll
  for (int q = 0; q < 4 + S; ++q) d[q] = 0.0;
  for (int64_t i = blk * BS + threadIdx.x; i < n; i += nblk * BS) {
    const bool fe = (i % ND == ND - 1);
    const double sb = b[i] * (fe ? se : 1.0);
    const double rd = sb - (y ? y[i] : 0.0);
    r[i] = rd;
    d[fe ? 1 : 0] += rd * rd;
    d[fe ? 3 : 2] += sb * sb;
#pragma unroll
    for (int q = 0; q < S; ++q) d[4 + q] += shadow_entry(seed + q, i) * rd;
  }
  write_partials<4 + S>(d, part, blk, sm);
}

template <int S>
__device__ __forceinline__ void idr_init_scalar_body(int64_t nblk, const double* __restrict__ part,
                                                     double* __restrict__ sc) {
  __shared__ double sm[4 + S][BS];
  double acc[4 + S];
  finish_partials<4 + S>(nblk, part, acc, sm);
  if (threadIdx.x != 0) return;
  const double btot = acc[2] + acc[3];
  sc[K_BU] = fmax(acc[2], FIELD_FLOOR2 * btot);
  sc[K_BE] = fmax(acc[3], FIELD_FLOOR2 * btot);
  sc[K_B2] = btot;
  for (int i = 0; i < I_LD * I_LD; ++i) sc[I_M + i] = (i / I_LD == i % I_LD) ? 1.0 : 0.0;
  for (int q = 0; q < S; ++q) sc[I_F + q] = acc[4 + q];
  sc[I_OM] = 1.0;
  sc[I_FRESH] = 1.0;
  sc[K_STATUS] = KS_RUN;
  sc[K_DONE] = 0.0;
  if (btot == 0.0) {
    sc[K_RU] = sc[K_RE] = 0.0;
    sc[K_STATUS] = KS_CONV;
    sc[K_DONE] = 1.0;
    return;
  }
  if (idr_norms(sc, acc[0], acc[1])) return;
  idr_coeffs<S>(sc, 0);
}

// step K: v = r - sum_j c_j G_{K+j};  U_K = sum_j c_j U_{K+j} + omega M^-1 v.
// In the first cycle after a (re)start every G, U term is zero (the fresh
// flag).  One thread per node; the node's ND entries of each vector are one load.
template <typename T, int ND, int S, int K, int NC>
__device__ __forceinline__ void idr_dir_nodes(int64_t blk, int64_t nblk, int64_t n_nodes,
                                              const T* __restrict__ minv, const double* __restrict__ r,
                                              const double* __restrict__ Gv, double* __restrict__ Uv, int64_t n,
                                              const double* __restrict__ sc) {
  double cc[NC > 0 ? NC : 1];
#pragma unroll
  for (int j = 0; j < NC; ++j) cc[j] = sc[I_C + j];
  const double om = sc[I_OM];
  for (int64_t a = blk * BS + threadIdx.x; a < n_nodes; a += nblk * BS) {
    const int64_t o = a * ND;
    Quad<double, ND> v;
    v.load(r + o);
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      Quad<double, ND> g;
      g.load(Gv + (int64_t)(K + j) * n + o);
#pragma unroll
      for (int i = 0; i < ND; ++i) v.v[i] -= cc[j] * g.v[i];
    }
    Quad<T, ND> m[ND];
#pragma unroll
    for (int i = 0; i < ND; ++i) m[i].load(minv + a * ND * ND + i * ND);
    Quad<double, ND> u;
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      double vh = 0.0;
#pragma unroll
      for (int jj = 0; jj < ND; ++jj) vh += (double)m[i].v[jj] * v.v[jj];
      u.v[i] = om * vh;
    }
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      Quad<double, ND> uj;
      uj.load(Uv + (int64_t)(K + j) * n + o);
#pragma unroll
      for (int i = 0; i < ND; ++i) u.v[i] += cc[j] * uj.v[i];
    }
    u.store(Uv + (int64_t)K * n + o);
  }
}

template <typename T, int ND, int S, int K>
__device__ __forceinline__ void idr_dir_body(int64_t blk, int64_t nblk, int64_t n_nodes,
                                             const T* __restrict__ minv, const double* __restrict__ r,
                                             const double* __restrict__ Gv, double* __restrict__ Uv, int64_t n,
                                             const double* __restrict__ sc) {
  if (sc[K_DONE] != 0.0) return;
  if (sc[I_FRESH] != 0.0)
    idr_dir_nodes<T, ND, S, K, 0>(blk, nblk, n_nodes, minv, r, Gv, Uv, n, sc);
  else
    idr_dir_nodes<T, ND, S, K, S - K>(blk, nblk, n_nodes, minv, r, Gv, Uv, n, sc);
}

// after g = S K U_k with partials P^T g, |g|^2: the biorthogonalisation
// coefficients a (P_i . G_k' = 0 for i < k), column k of M, beta = f_k / M_kk,
// f -= beta M[:, k], and the coefficients c of step k + 1
template <int S>
__device__ __forceinline__ void idr_g_scalar_body(int64_t nblk, const double* __restrict__ part,
                                                  double* __restrict__ sc, int k, double pnorm2) {
  __shared__ double sm[S + 1][BS];
  double acc[S + 1];
  if (sc[K_DONE] != 0.0) return;
  finish_partials<S + 1>(nblk, part, acc, sm);
  if (threadIdx.x != 0) return;
  for (int i = 0; i < k; ++i) {
    double v = acc[i];
    for (int l = 0; l < i; ++l) v -= sc[I_M + i * I_LD + l] * sc[I_A + l];
    sc[I_A + i] = v / sc[I_M + i * I_LD + i];
  }
  for (int l = k; l < S; ++l) {
    double v = acc[l];
    for (int i = 0; i < k; ++i) v -= sc[I_A + i] * sc[I_M + l * I_LD + i];
    sc[I_M + l * I_LD + k] = v;
  }
  sc[K_ITER] += 1.0;
  const double mkk = sc[I_M + k * I_LD + k];
  if (!isfinite(mkk) || !isfinite(acc[S])) {
    sc[K_STATUS] = KS_NAN;
    sc[K_DONE] = 1.0;
    return;
  }
  if (mkk == 0.0 || fabs(mkk) <= sc[K_BRK] * sqrt(acc[S] * pnorm2)) {
    sc[K_STATUS] = KS_BREAK;  // the new direction is (nearly) orthogonal to P_k
    sc[K_DONE] = 1.0;
    return;
  }
  const double beta = sc[I_F + k] / mkk;
  sc[I_BETA] = beta;
  for (int l = k + 1; l < S; ++l) sc[I_F + l] -= beta * sc[I_M + l * I_LD + k];
  if (k + 1 < S) idr_coeffs<S>(sc, k + 1);
}

// G_K -= sum_{i<K} a_i G_i, U_K likewise; r -= beta G_K; x += beta U_K;
// the last step (K = s - 1) also forms v = M^-1 r for the minimal-residual
// step when M is block-Jacobi (minv not null).  Partials |r_u|^2, |r_e|^2.
template <typename T, int ND, int S, int K>
__device__ __forceinline__ void idr_upd_body(int64_t blk, int64_t nblk, int64_t n_nodes,
                                             const T* __restrict__ minv, double* __restrict__ Gv,
                                             double* __restrict__ Uv, double* __restrict__ r,
                                             double* __restrict__ x, double* __restrict__ v, int64_t n,
                                             const double* __restrict__ sc, double* __restrict__ part) {
  constexpr bool LAST = (K == S - 1);
  __shared__ double sm[2][BS];
  if (sc[K_DONE] != 0.0) return;
  double aa[K > 0 ? K : 1];
#pragma unroll
  for (int i = 0; i < K; ++i) aa[i] = sc[I_A + i];
  const double beta = sc[I_BETA];
  double d[2] = {0.0, 0.0};
  for (int64_t a = blk * BS + threadIdx.x; a < n_nodes; a += nblk * BS) {
    const int64_t o = a * ND;
    Quad<double, ND> g, u;
    g.load(Gv + (int64_t)K * n + o);
    u.load(Uv + (int64_t)K * n + o);
    if (K > 0) {
#pragma unroll
      for (int j = 0; j < K; ++j) {
        Quad<double, ND> gj, uj;
        gj.load(Gv + (int64_t)j * n + o);
        uj.load(Uv + (int64_t)j * n + o);
#pragma unroll
        for (int i = 0; i < ND; ++i) {
          g.v[i] -= aa[j] * gj.v[i];
          u.v[i] -= aa[j] * uj.v[i];
        }
      }
      g.store(Gv + (int64_t)K * n + o);
      u.store(Uv + (int64_t)K * n + o);
    }
    Quad<double, ND> rn, xn;
    rn.load(r + o);
    xn.load(x + o);
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      rn.v[i] -= beta * g.v[i];
      xn.v[i] += beta * u.v[i];
      d[i == ND - 1 ? 1 : 0] += rn.v[i] * rn.v[i];
    }
    rn.store(r + o);
    xn.store(x + o);
    if (LAST && minv != nullptr) {
      Quad<T, ND> m[ND];
#pragma unroll
      for (int i = 0; i < ND; ++i) m[i].load(minv + a * ND * ND + i * ND);
      Quad<double, ND> vh;
#pragma unroll
      for (int i = 0; i < ND; ++i) {
        double acc = 0.0;
#pragma unroll
        for (int jj = 0; jj < ND; ++jj) acc += (double)m[i].v[jj] * rn.v[jj];
        vh.v[i] = acc;
      }
      vh.store(v + o);
    }
  }
  write_partials<2>(d, part, blk, sm);
}

// Step K with a preconditioner applied by separate launches (multigrid):
// v = r - sum_j c_j G_{K+j} before it, U_K = sum_j c_j U_{K+j} + omega z
// after it (z = M^-1 v); the first cycle after a (re)start has no G, U terms.
template <int S, int K>
__global__ void __launch_bounds__(BS) idr_formv_kernel(int64_t n, const double* __restrict__ r,
                                                       const double* __restrict__ Gv, double* __restrict__ v,
                                                       const double* __restrict__ sc) {
  if (sc[K_DONE] != 0.0) return;
  const bool fresh = sc[I_FRESH] != 0.0;
  double cc[S - K];
#pragma unroll
  for (int j = 0; j < S - K; ++j) cc[j] = sc[I_C + j];
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
    double x = r[i];
    if (!fresh)
#pragma unroll
      for (int j = 0; j < S - K; ++j) x -= cc[j] * Gv[(int64_t)(K + j) * n + i];
    v[i] = x;
  }
}

template <int S, int K>
__global__ void __launch_bounds__(BS) idr_formu_kernel(int64_t n, const double* __restrict__ z,
                                                       double* __restrict__ Uv, const double* __restrict__ sc) {
  if (sc[K_DONE] != 0.0) return;
  const bool fresh = sc[I_FRESH] != 0.0;
  const double om = sc[I_OM];
  double cc[S - K];
#pragma unroll
  for (int j = 0; j < S - K; ++j) cc[j] = sc[I_C + j];
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
    double u = om * z[i];
    if (!fresh)
#pragma unroll
      for (int j = 0; j < S - K; ++j) u += cc[j] * Uv[(int64_t)(K + j) * n + i];
    Uv[(int64_t)K * n + i] = u;
  }
}

__device__ __forceinline__ void idr_r_scalar_body(int64_t nblk, const double* __restrict__ part,
                                                  double* __restrict__ sc) {
  __shared__ double sm[2][BS];
  double acc[2];
  if (sc[K_DONE] != 0.0) return;
  finish_partials<2>(nblk, part, acc, sm);
  if (threadIdx.x != 0) return;
  idr_norms(sc, acc[0], acc[1]);
}

// omega of the minimal-residual step from t . r and t . t, kept away from
// zero when t and r are far from parallel (the angle safeguard of IDR(s))
__device__ __forceinline__ void idr_om_scalar_body(int64_t nblk, const double* __restrict__ part,
                                                   double* __restrict__ sc) {
  __shared__ double sm[2][BS];
  double acc[2];
  if (sc[K_DONE] != 0.0) return;
  finish_partials<2>(nblk, part, acc, sm);
  if (threadIdx.x != 0) return;
  const double ts = acc[0], tt = acc[1], rr = sc[I_RR];
  sc[K_ITER] += 1.0;
  if (!isfinite(ts) || !isfinite(tt)) {
    sc[K_STATUS] = KS_NAN;
    sc[K_DONE] = 1.0;
    return;
  }
  if (!(tt > 0.0) || ts == 0.0) {
    sc[K_STATUS] = KS_BREAK;
    sc[K_DONE] = 1.0;
    return;
  }
  double om = ts / tt;
  const double cosang = fabs(ts) / sqrt(tt * rr);
  if (cosang < IDR_KAPPA) om *= IDR_KAPPA / cosang;
  sc[I_OM] = om;
}

// r -= omega t; x += omega v; partials |r_u|^2, |r_e|^2, P^T r
template <int ND, int S>
__device__ __forceinline__ void idr_om_body(int64_t blk, int64_t nblk, int64_t n, double* __restrict__ r,
                                            double* __restrict__ x, const double* __restrict__ v,
                                            const double* __restrict__ t, const double* __restrict__ sc,
                                            double* __restrict__ part) {
  __shared__ double sm[2 + S][BS];
  if (sc[K_DONE] != 0.0) return;
  const double om = sc[I_OM];
  const int seed = (int)sc[K_SEED];
  double d[2 + S];
#pragma unroll
  for (int q = 0; q < 2 + S; ++q) d[q] = 0.0;
  for (int64_t i = blk * BS + threadIdx.x; i < n; i += nblk * BS) {
    const double rd = r[i] - om * t[i];
    r[i] = rd;
    x[i] += om * v[i];
    d[(i % ND == ND - 1) ? 1 : 0] += rd * rd;
#pragma unroll
    for (int q = 0; q < S; ++q) d[2 + q] += shadow_entry(seed + q, i) * rd;
  }
  write_partials<2 + S>(d, part, blk, sm);
}

template <int S>
__device__ __forceinline__ void idr_f_scalar_body(int64_t nblk, const double* __restrict__ part,
                                                  double* __restrict__ sc) {
  __shared__ double sm[2 + S][BS];
  double acc[2 + S];
  if (sc[K_DONE] != 0.0) return;
  finish_partials<2 + S>(nblk, part, acc, sm);
  if (threadIdx.x != 0) return;
  sc[I_FRESH] = 0.0;
  if (idr_norms(sc, acc[0], acc[1])) return;
  for (int q = 0; q < S; ++q) sc[I_F + q] = acc[2 + q];
  idr_coeffs<S>(sc, 0);
}

// --- single-request kernels ------------------------------------------------
template <int ND, int S>
__global__ void __launch_bounds__(BS) idr_init_kernel(int64_t n, const double* __restrict__ b,
                                                      const double* __restrict__ y, double* __restrict__ r,
                                                      const double* __restrict__ sc, double* __restrict__ part) {
  idr_init_body<ND, S>(blockIdx.x, gridDim.x, n, b, y, r, sc, part);
}
template <int S>
__global__ void __launch_bounds__(BS) idr_init_scalar(int nblk, const double* __restrict__ part,
                                                      double* __restrict__ sc) {
  __shared__ double s_sc[KSCAL_DOUBLES];
  stage_scalars(s_sc, sc);
  idr_init_scalar_body<S>(nblk, part, s_sc);
  unstage_scalars(sc, s_sc);
}
template <typename T, int ND, int S, int K>
__global__ void __launch_bounds__(BS) idr_dir_kernel(int64_t n_nodes, const T* __restrict__ minv,
                                                     const double* __restrict__ r, const double* __restrict__ Gv,
                                                     double* __restrict__ Uv, int64_t n,
                                                     const double* __restrict__ sc) {
  idr_dir_body<T, ND, S, K>(blockIdx.x, gridDim.x, n_nodes, minv, r, Gv, Uv, n, sc);
}
template <int S>
__global__ void __launch_bounds__(BS) idr_g_scalar(int nblk, const double* __restrict__ part,
                                                   double* __restrict__ sc, int k, double pnorm2) {
  __shared__ double s_sc[KSCAL_DOUBLES];
  stage_scalars(s_sc, sc);
  idr_g_scalar_body<S>(nblk, part, s_sc, k, pnorm2);
  unstage_scalars(sc, s_sc);
}
template <typename T, int ND, int S, int K>
__global__ void __launch_bounds__(BS) idr_upd_kernel(int64_t n_nodes, const T* __restrict__ minv,
                                                     double* __restrict__ Gv, double* __restrict__ Uv,
                                                     double* __restrict__ r, double* __restrict__ x,
                                                     double* __restrict__ v, int64_t n,
                                                     const double* __restrict__ sc, double* __restrict__ part) {
  idr_upd_body<T, ND, S, K>(blockIdx.x, gridDim.x, n_nodes, minv, Gv, Uv, r, x, v, n, sc, part);
}
__global__ void __launch_bounds__(BS) idr_r_scalar(int nblk, const double* __restrict__ part,
                                                   double* __restrict__ sc) {
  __shared__ double s_sc[KSCAL_DOUBLES];
  stage_scalars(s_sc, sc);
  idr_r_scalar_body(nblk, part, s_sc);
  unstage_scalars(sc, s_sc);
}
__global__ void __launch_bounds__(BS) idr_om_scalar(int nblk, const double* __restrict__ part,
                                                    double* __restrict__ sc) {
  __shared__ double s_sc[KSCAL_DOUBLES];
  stage_scalars(s_sc, sc);
  idr_om_scalar_body(nblk, part, s_sc);
  unstage_scalars(sc, s_sc);
}
template <int ND, int S>
__global__ void __launch_bounds__(BS) idr_om_kernel(int64_t n, double* __restrict__ r, double* __restrict__ x,
                                                    const double* __restrict__ v, const double* __restrict__ t,
                                                    const double* __restrict__ sc, double* __restrict__ part) {
  idr_om_body<ND, S>(blockIdx.x, gridDim.x, n, r, x, v, t, sc, part);
}
template <int S>
__global__ void __launch_bounds__(BS) idr_f_scalar(int nblk, const double* __restrict__ part,
                                                   double* __restrict__ sc) {
  __shared__ double s_sc[KSCAL_DOUBLES];
  stage_scalars(s_sc, sc);
  idr_f_scalar_body<S>(nblk, part, s_sc);
  unstage_scalars(sc, s_sc);
}

// --- batched kernels: one launch over the requests of a serving batch -------
// Request j owns the workgroups [blk0[f], blk0[f] + nblk[f]) of a launch of
// family f (per node, SpMV, per dof), sized from its own dimensions only, so
// every reduction of a request has the same order alone and in any mix.
enum { FAM_NODE = 0, FAM_SPMV = 1, FAM_DOF = 2 };

struct KSlot {
  int64_t nn, n;
  const int32_t* row_ptr;
  const int32_t* nbr_ptr;
  const int32_t* nbr;
  const void* vals;
  const void* minv;
  double* x;
  double* r;
  double* v;
  double* t;
  double* G;
  double* U;
  double* sc;
  int64_t blk0[3];
  int64_t nblk[3];
};

__device__ __forceinline__ int find_kslot(const KSlot* __restrict__ ks, int nks, int fam, int64_t blk) {
  int lo = 0, hi = nks - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (ks[mid].blk0[fam] <= blk) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename T, int ND, int S, int K>
__global__ void __launch_bounds__(BS) idr_dir_batch(const KSlot* __restrict__ ks, int nks) {
  const KSlot& q = ks[find_kslot(ks, nks, FAM_NODE, blockIdx.x)];
  idr_dir_body<T, ND, S, K>(blockIdx.x - q.blk0[FAM_NODE], q.nblk[FAM_NODE], q.nn, (const T*)q.minv, q.r, q.G,
                            q.U, q.n, q.sc);
}
template <typename T, int ND, int G, int MODE, int NP>
__global__ void __launch_bounds__(BS) spmv_batch(const KSlot* __restrict__ ks, int nks, int k,
                                                 double* __restrict__ part) {
  const KSlot& q = ks[find_kslot(ks, nks, FAM_SPMV, blockIdx.x)];
  const double* x = MODE == 3 ? q.U + (int64_t)k * q.n : q.v;
  double* y = MODE == 3 ? q.G + (int64_t)k * q.n : q.t;
  spmv_body<T, ND, G, MODE, NP>(blockIdx.x - q.blk0[FAM_SPMV], q.nblk[FAM_SPMV], q.nn, q.row_ptr, q.nbr_ptr,
                                q.nbr, (const T*)q.vals, x, y, MODE == 2 ? q.r : nullptr, q.sc,
                                part + q.blk0[FAM_SPMV] * (MODE == 3 ? NP + 1 : 2));
}
template <int S>
__global__ void __launch_bounds__(BS) idr_g_scalar_batch(const KSlot* __restrict__ ks, int k,
                                                         const double* __restrict__ part) {
  const KSlot& q = ks[blockIdx.x];
  __shared__ double s_sc[KSCAL_DOUBLES];
  stage_scalars(s_sc, q.sc);
  idr_g_scalar_body<S>(q.nblk[FAM_SPMV], part + q.blk0[FAM_SPMV] * (S + 1), s_sc, k, (double)q.n / 3.0);
  unstage_scalars(q.sc, s_sc);
}
template <typename T, int ND, int S, int K>
__global__ void __launch_bounds__(BS) idr_upd_batch(const KSlot* __restrict__ ks, int nks,
                                                    double* __restrict__ part) {
  const KSlot& q = ks[find_kslot(ks, nks, FAM_NODE, blockIdx.x)];
  idr_upd_body<T, ND, S, K>(blockIdx.x - q.blk0[FAM_NODE], q.nblk[FAM_NODE], q.nn, (const T*)q.minv, q.G, q.U,
                            q.r, q.x, q.v, q.n, q.sc, part + q.blk0[FAM_NODE] * 2);
}
__global__ void __launch_bounds__(BS) idr_r_scalar_batch(const KSlot* __restrict__ ks,
                                                         const double* __restrict__ part) {
  const KSlot& q = ks[blockIdx.x];
  __shared__ double s_sc[KSCAL_DOUBLES];
  stage_scalars(s_sc, q.sc);
  idr_r_scalar_body(q.nblk[FAM_NODE], part + q.blk0[FAM_NODE] * 2, s_sc);
  unstage_scalars(q.sc, s_sc);
}
__global__ void __launch_bounds__(BS) idr_om_scalar_batch(const KSlot* __restrict__ ks,
                                                          const double* __restrict__ part) {
  const KSlot& q = ks[blockIdx.x];
  __shared__ double s_sc[KSCAL_DOUBLES];
  stage_scalars(s_sc, q.sc);
  idr_om_scalar_body(q.nblk[FAM_SPMV], part + q.blk0[FAM_SPMV] * 2, s_sc);
  unstage_scalars(q.sc, s_sc);
}
template <int ND, int S>
__global__ void __launch_bounds__(BS) idr_om_batch(const KSlot* __restrict__ ks, int nks,
                                                   double* __restrict__ part) {
  const KSlot& q = ks[find_kslot(ks, nks, FAM_DOF, blockIdx.x)];
  idr_om_body<ND, S>(blockIdx.x - q.blk0[FAM_DOF], q.nblk[FAM_DOF], q.n, q.r, q.x, q.v, q.t, q.sc,
                     part + q.blk0[FAM_DOF] * (2 + S));
}
template <int S>
__global__ void __launch_bounds__(BS) idr_f_scalar_batch(const KSlot* __restrict__ ks,
                                                          const double* __restrict__ part) {
  const KSlot& q = ks[blockIdx.x];
  __shared__ double s_sc[KSCAL_DOUBLES];
  stage_scalars(s_sc, q.sc);
  idr_f_scalar_body<S>(q.nblk[FAM_DOF], part + q.blk0[FAM_DOF] * (2 + S), s_sc);
  unstage_scalars(q.sc, s_sc);
}

// compute units of the current device
inline int device_cus() {
  static int cus[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cus[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v < 1) v = 256;
    cus[dev] = v;
  }
  return cus[dev];
}

// Workgroups of BS threads for `work` threads' worth of items of `kernel`:
// at most the workgroups the device holds at once (a grid-stride kernel
// launched with more leaves a tail round on part of the device) and at most
// MAX_GRID (the partial-sum buffer), with the items spread evenly.
template <typename K> int64_t grid_of(K kernel, int64_t work) {
  static int per_cu = 0;  // per kernel; the kernels' resources do not depend on the device
  if (per_cu == 0) {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kernel, BS, 0) != hipSuccess || b < 1) b = 1;
    per_cu = b;
  }
  int64_t cap = (int64_t)per_cu * device_cus();
  if (cap > MAX_GRID) cap = MAX_GRID;
  int64_t g = (work + BS - 1) / BS;
  if (g > cap) {
    const int64_t iters = (work + cap * BS - 1) / (cap * BS);
    g = (work + iters * BS - 1) / (iters * BS);
  }
  return g < 1 ? 1 : g;
}

template <typename T, int ND>
struct Solver {
  // lanes per node in the SpMV (one per neighbour): nodes have up to 27
  // (hex8), 9 (quad4) and 3 (line2) neighbours; on the 3D beam 16 lanes
  // (two passes, four nodes per wave) beat 32 by a few per cent
  static constexpr bool F32 = std::is_same<T, float>::value;
  static constexpr int G = ND == 4 ? 16 : (ND == 3 ? 16 : 4);
  bool mg = false;  // BiCGSTAB is block-Jacobi preconditioned only
  lgdm_ctx* c;
  hipStream_t st;
  const T* vals;
  const T* minv;
  Vecs V;
  double* sc;
  double* kp;
  int64_t n, nn;

  double* vec(void* p) { return static_cast<double*>(p); }

  void spmv(const double* x, double* y, int mode, const double* w) {
    if (mode == 0) {
      const int64_t g = grid_of(spmv_kernel<T, ND, G, 0>, nn * G);
      spmv_kernel<T, ND, G, 0><<<g, BS, 0, st>>>(nn, c->row_ptr, c->nbr_ptr, c->nbr, vals, x, y,
                                                        w, sc, kp);
    } else if (mode == 1) {
      const int64_t g = grid_of(spmv_kernel<T, ND, G, 1>, nn * G);
      spmv_kernel<T, ND, G, 1><<<g, BS, 0, st>>>(nn, c->row_ptr, c->nbr_ptr, c->nbr, vals, x, y,
                                                        w, sc, kp);
      scalar_kernel<1, 2><<<1, BS, 0, st>>>((int)g, kp, sc);
    } else {
      const int64_t g = grid_of(spmv_kernel<T, ND, G, 2>, nn * G);
      spmv_kernel<T, ND, G, 2><<<g, BS, 0, st>>>(nn, c->row_ptr, c->nbr_ptr, c->nbr, vals, x, y,
                                                        w, sc, kp);
      scalar_kernel<2, 2><<<1, BS, 0, st>>>((int)g, kp, sc);
    }
  }

  void init(const double* b, bool use_y, const double* y) {
    const int64_t g = grid_of(init_kernel<ND>, n);
    init_kernel<ND><<<g, BS, 0, st>>>(n, b, y, use_y ? 1 : 0, vec(V.r), vec(V.rh), vec(V.p),
                                             vec(V.v), sc, kp);
    scalar_kernel<4, 5><<<1, BS, 0, st>>>((int)g, kp, sc);
  }

  void iteration(double* x) {
    pupdate_kernel<T, ND><<<grid_of(pupdate_kernel<T, ND>, nn), BS, 0, st>>>(
        nn, minv, vec(V.r), vec(V.p), vec(V.v), vec(V.ph), sc);
    spmv(vec(V.ph), vec(V.v), 1, vec(V.rh));
    supdate_kernel<T, ND><<<grid_of(supdate_kernel<T, ND>, nn), BS, 0, st>>>(
        nn, minv, vec(V.r), vec(V.v), vec(V.s), vec(V.sh), sc);
    spmv(vec(V.sh), vec(V.t), 2, vec(V.s));
    const int64_t g = grid_of(xupdate_kernel<ND>, n);
    xupdate_kernel<ND><<<g, BS, 0, st>>>(n, x, vec(V.ph), vec(V.sh), vec(V.s), vec(V.t),
                                                vec(V.r), vec(V.rh), sc, kp);
    scalar_kernel<3, 3><<<1, BS, 0, st>>>((int)g, kp, sc);
  }

  // the interface a Krylov run drives
  static constexpr int SPMV_PER_ITER = 2;
  void bind(lgdm_ctx* ctx, hipStream_t stream, double* scal, double* part) {
    c = ctx;
    st = stream;
    n = c->ndof;
    nn = c->n_nodes;
    vals = F32 ? (const T*)c->vals32 : (const T*)c->vals;
    minv = F32 ? (const T*)c->minv32 : (const T*)c->minv;
    void** vp[8] = {&V.r, &V.rh, &V.p, &V.v, &V.s, &V.t, &V.ph, &V.sh};
    for (int i = 0; i < 8; ++i) *vp[i] = c->kv + (int64_t)i * c->ndof;
    sc = scal;
    kp = part;
  }
  void begin(const double* b) { init(b, false, nullptr); }
  void restart(const double* b, const double* x) {
    spmv(x, vec(V.t), 0, nullptr);
    init(b, true, vec(V.t));
  }
  void iterate(double* x, int iters) {
    for (int i = 0; i < iters; ++i) iteration(x);
  }
};

// IDR(s) driver: per cycle, s steps of {direction, SpMV + P^T g, update}
// and one minimal-residual step; scalars as for BiCGSTAB.
template <typename T, int ND, int S>
struct Idr {
  static constexpr bool F32 = std::is_same<T, float>::value;
  static constexpr int G = Solver<T, ND>::G;
  static constexpr int SPMV_PER_ITER = 1;
  lgdm_ctx* c = nullptr;
  hipStream_t st = nullptr;
  const T* vals = nullptr;
  const T* minv = nullptr;
  double* sc = nullptr;
  double* kp = nullptr;
  double *r = nullptr, *v = nullptr, *t = nullptr, *Gv = nullptr, *Uv = nullptr;
  int64_t n = 0, nn = 0;
  bool mg = false;  // multigrid preconditioner (the context's hierarchy) instead of block-Jacobi

  void bind(lgdm_ctx* ctx, hipStream_t stream, double* scal, double* part) {
    c = ctx;
    st = stream;
    n = c->ndof;
    nn = c->n_nodes;
    vals = F32 ? (const T*)c->vals32 : (const T*)c->vals;
    minv = F32 ? (const T*)c->minv32 : (const T*)c->minv;
    r = c->kv;
    v = c->kv + n;
    t = c->kv + 2 * n;
    Gv = c->kv + 3 * n;
    Uv = c->kv + (3 + S) * n;
    sc = scal;
    kp = part;
  }
  int64_t spmv_grid() const { return grid_of(spmv_kernel<T, ND, G, 3, S>, nn * G); }
  void init(const double* b, const double* y) {
    const int64_t g = grid_of(idr_init_kernel<ND, S>, n);
    idr_init_kernel<ND, S><<<g, BS, 0, st>>>(n, b, y, r, sc, kp);
    idr_init_scalar<S><<<1, BS, 0, st>>>((int)g, kp, sc);
  }
  void begin(const double* b) { init(b, nullptr); }
  void restart(const double* b, const double* x) {
    spmv_kernel<T, ND, G, 0><<<grid_of(spmv_kernel<T, ND, G, 0>, nn * G), BS, 0, st>>>(
        nn, c->row_ptr, c->nbr_ptr, c->nbr, vals, x, t, nullptr, sc, kp);
    init(b, t);
  }
  // the s steps of a cycle, each with its compile-time index K
  template <int K> void steps(double* x, int64_t gs, double pnorm2) {
    if constexpr (K < S) {
      if (mg) {
        // v = r - sum c G (in v); z = M^-1 v (in t); U_K from z.  v and t
        // are free until the minimal-residual step at the end of the cycle.
        auto kv = idr_formv_kernel<S, K>;
        kv<<<grid_of(kv, n), BS, 0, st>>>(n, r, Gv, v, sc);
        (void)amg_apply(c, v, t, sc, st);
        auto kf = idr_formu_kernel<S, K>;
        kf<<<grid_of(kf, n), BS, 0, st>>>(n, t, Uv, sc);
      } else {
        auto kd = idr_dir_kernel<T, ND, S, K>;
        kd<<<grid_of(kd, nn), BS, 0, st>>>(nn, minv, r, Gv, Uv, n, sc);
      }
      probe_before(c, PROBE_IDR_SPMV, st);
      spmv_kernel<T, ND, G, 3, S><<<gs, BS, 0, st>>>(nn, c->row_ptr, c->nbr_ptr, c->nbr, vals,
                                                     Uv + (int64_t)K * n, Gv + (int64_t)K * n, nullptr, sc, kp);
      probe_after(c, PROBE_IDR_SPMV, st);
      idr_g_scalar<S><<<1, BS, 0, st>>>((int)gs, kp, sc, K, pnorm2);
      auto ku = idr_upd_kernel<T, ND, S, K>;
      const int64_t gu = grid_of(ku, nn);
      ku<<<gu, BS, 0, st>>>(nn, mg ? nullptr : minv, Gv, Uv, r, x, v, n, sc, kp);
      idr_r_scalar<<<1, BS, 0, st>>>((int)gu, kp, sc);
      if (K == S - 1 && mg) (void)amg_apply(c, r, v, sc, st);  // v = M^-1 r
      steps<K + 1>(x, gs, pnorm2);
    }
  }
  void cycle(double* x) {
    const int64_t gs = spmv_grid();
    const int64_t gm = grid_of(spmv_kernel<T, ND, G, 2>, nn * G), g = grid_of(idr_om_kernel<ND, S>, n);
    const double pnorm2 = (double)n / 3.0;  // E|P_k|^2 of uniform [-1, 1) entries
    steps<0>(x, gs, pnorm2);
    spmv_kernel<T, ND, G, 2><<<gm, BS, 0, st>>>(nn, c->row_ptr, c->nbr_ptr, c->nbr, vals, v, t, r, sc, kp);
    idr_om_scalar<<<1, BS, 0, st>>>((int)gm, kp, sc);
    idr_om_kernel<ND, S><<<g, BS, 0, st>>>(n, r, x, v, t, sc, kp);
    idr_f_scalar<S><<<1, BS, 0, st>>>((int)g, kp, sc);
  }
  // at least `iters` operator applications, in whole cycles of s + 1
  static int cycles_for(int iters) {
    const int ncyc = (iters + S) / (S + 1);
    return ncyc > 0 ? ncyc : 1;
  }
  void iterate(double* x, int iters) {
    for (int i = 0, n_cyc = cycles_for(iters); i < n_cyc; ++i) cycle(x);
  }
};

// The host side of one solve, shared by single and batched runs: reads the
// device scalars after some iterations and decides what happens next.
struct RunControl {
  // RESTART: restart from the current iterate; RESTART_BEST: from the best
  // one (the current one is worse); RETURN_BEST: finish with the best one
  enum Action { NONE, RESTART, RESTART_BEST, RETURN_BEST };
  KrylovResult res{};
  double tol_u = 0, tol_e = 0;
  int64_t done_iters = 0;      // iterations before the last restart
  int replacements = 0;        // restarts that replaced a converged recurrence residual
  double best = INFINITY;      // best per-field residual / tolerance so far
  int64_t stall = 0;
  bool have_best = false;
  bool fin = false;
  int spmv_per_iter = 1;

  void setup(double tu, double te, bool f32, int per_iter) {
    // an FP32 matrix gains nothing below 1e-8; Newton refines on the FP64 residual
    tol_u = f32 && tu < 1e-8 ? 1e-8 : tu;
    tol_e = f32 && te < 1e-8 ? 1e-8 : te;
    spmv_per_iter = per_iter;
    res.status = LGDM_ERR_NOT_CONVERGED;
  }
  double score() const { return std::max(res.rel_u / tol_u, res.rel_e / tol_e); }
  // shadow-vector offset of the current (re)start: every restart of IDR(s)
  // draws shadow vectors it has not used before
  int seed() const { return IDR_SMAX * (res.restarts + replacements); }

  // h: the scalars after `ran` more iterations were enqueued.  save_best is
  // set when the current iterate is the best so far and must be copied.
  Action decide(const double* h, const lgdm_solver_opts& o, int64_t ran, bool& save_best) {
    save_best = false;
    const int64_t it = (int64_t)h[K_ITER];
    res.iters = done_iters + it;
    res.spmv = res.iters * spmv_per_iter + res.restarts + replacements;
    const double bu = h[K_BU] > 0 ? h[K_BU] : 1.0, be = h[K_BE] > 0 ? h[K_BE] : 1.0;
    res.rel_u = std::sqrt(h[K_RU] / bu);
    res.rel_e = std::sqrt(h[K_RE] / be);
    const int st = (int)h[K_STATUS];
    if (h[K_DONE] != 0.0) {
      if (st == KS_CONV) {
        // accept a converged true residual (no iteration since the last
        // (re)start); a converged recurrence residual is first replaced by
        // the true one, which it can drift from
        if (it == 0 || replacements >= 4) {
          res.status = LGDM_OK;
          res.improved = true;
          fin = true;
          return NONE;
        }
        replacements++;
        done_iters = res.iters;
        return RESTART;
      }
      if (st == KS_NAN) {
        fin = true;
        if (have_best) {
          res.status = LGDM_ERR_NOT_CONVERGED;
          return RETURN_BEST;
        }
        res.status = LGDM_ERR_NAN;
        return NONE;
      }
      // breakdown: restart from the current iterate with its true residual
      if (res.restarts >= o.max_restarts || res.iters >= o.max_krylov) {
        res.status = LGDM_ERR_BREAKDOWN;
        fin = true;
        // the current iterate is kept unless an earlier one was better
        if (have_best && !(score() <= best)) return RETURN_BEST;
        res.improved = res.iters > 0 && std::isfinite(score());
        return NONE;
      }
      const bool worse = have_best && !(score() <= best);
      res.restarts++;
      done_iters = res.iters;
      return worse ? RESTART_BEST : RESTART;
    }
    const double sc = score();
    if (std::isfinite(sc) && sc < best * (1.0 - 1e-3)) {
      best = sc;
      stall = 0;
      res.improved = have_best;  // the first best is the zero start itself
      have_best = true;
      save_best = true;
      if (res.iters >= o.max_krylov) {  // the current iterate is the best: keep it
        res.status = LGDM_ERR_NOT_CONVERGED;
        fin = true;
      }
      return NONE;
    }
    stall += ran;
    const int64_t window = res.improved ? STALL_ITERS : std::max<int64_t>(STALL_ITERS, res.iters);
    if (stall >= window || res.iters >= o.max_krylov) {
      res.status = LGDM_ERR_NOT_CONVERGED;
      fin = true;
      return RETURN_BEST;
    }
    return NONE;
  }
};

// One linear solve as a state machine: start() enqueues the initial
// residual, then alternately check() (reads the device scalars; decides
// convergence, restart, stagnation) and launch() (enqueues check_every
// iterations) until finished().  Several runs on different streams can be
// interleaved by the host so their kernels overlap on the device.
template <typename Method>
struct KrylovRunImpl final : KrylovRun {
  Method S;
  lgdm_ctx* c;
  const double* b;
  double* xout;
  lgdm_solver_opts o;
  RunControl rc;
  double se = 0;
  int every = 16;
  double* xbest = nullptr;     // best iterate so far (per-field relative residual)
  bool pending_read = false;   // a restart's scalars are in flight: check again before launching
  int64_t ran = 0;             // iterations enqueued since the last check

  KrylovRunImpl(lgdm_ctx* ctx, const double* b_, double* x_, const lgdm_solver_opts& o_, double tu,
                double te)
      : c(ctx), b(b_), xout(x_), o(o_) {
    S.bind(c, c->stream, c->kscal, c->kpart);
    S.mg = o.precond == LGDM_PRECOND_AMG && c->amg != nullptr;
    xbest = c->kv + (int64_t)(KV_VECS - 1) * c->ndof;
    rc.setup(tu, te, Method::F32, Method::SPMV_PER_ITER);
    se = c->mat.E / c->mat.h;
    every = o.check_every > 0 ? o.check_every : 16;
  }

  hipError_t read_scalars() {
    return hipMemcpyAsync(c->kscal_host, S.sc, K_NSLOTS * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  }

  hipError_t start() override {
    set_scalars_kernel<<<1, 64, 0, c->stream>>>(S.sc, rc.tol_u * rc.tol_u, rc.tol_e * rc.tol_e, se, BREAK_REL,
                                                0);
    hipError_t e = hipMemsetAsync(xout, 0, c->ndof * sizeof(double), c->stream);
    if (e != hipSuccess) return e;
    S.begin(b);
    ran = 0;
    return read_scalars();
  }

  hipError_t launch() override {
    if (rc.fin) return hipSuccess;
    // no further than the solve's iteration limit (IDR(s) runs whole cycles
    // of s + 1 steps, so it can pass the limit by up to s steps)
    const int n = (int)std::max<int64_t>(1, std::min<int64_t>(every, (int64_t)o.max_krylov - rc.res.iters));
    S.iterate(xout, n);
    ran = n;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return read_scalars();
  }

  // reads the scalars enqueued by the last start()/launch(); restart and
  // replacement kernels are enqueued here and read at the next check
  hipError_t check() override {
    if (rc.fin) return hipSuccess;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return e;
    pending_read = false;
    bool save_best = false;
    RunControl::Action a = rc.decide(c->kscal_host, o, ran, save_best);
    ran = 0;
    if (!rc.fin && c->solve_deadline > 0.0 && host_seconds() > c->solve_deadline) {
      // the increment's wall-time bound: stop with the best iterate so far
      rc.fin = true;
      rc.res.status = LGDM_ERR_NOT_CONVERGED;
      a = RunControl::RETURN_BEST;
    }
    if (save_best) {
      e = hipMemcpyAsync(xbest, xout, c->ndof * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
      if (e != hipSuccess) return e;
    }
    if ((a == RunControl::RETURN_BEST || a == RunControl::RESTART_BEST) && rc.have_best) {
      e = hipMemcpyAsync(xout, xbest, c->ndof * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
      if (e != hipSuccess || a == RunControl::RETURN_BEST) return e;
    }
    if (a == RunControl::RESTART || a == RunControl::RESTART_BEST) {
      set_scalars_kernel<<<1, 64, 0, c->stream>>>(S.sc, rc.tol_u * rc.tol_u, rc.tol_e * rc.tol_e, se,
                                                  BREAK_REL, rc.seed());
      S.restart(b, xout);
      pending_read = true;
      return read_scalars();
    }
    return hipSuccess;
  }

  bool needs_check() const override { return pending_read; }
  bool finished() const override { return rc.fin; }
  const KrylovResult& result() const override { return rc.res; }
};

// ---------------------------------------------------------------------------
// Batched IDR(s) over the requests of a serving batch.  Starts and restarts
// of single requests use the single-request kernels; every cycle is one
// launch per kernel over all running requests.  Per-request workgroup counts
// depend only on the request's own size (capped), so its reductions, and
// therefore its results, are the same alone and in any mix.
constexpr int64_t CAP_NODE = 256, CAP_SPMV = 512, CAP_DOF = 256;
constexpr int64_t BATCH_PART_PER_REQUEST = CAP_SPMV * KPART_PER_BLOCK;

template <typename T, int ND, int S>
struct BatchIdr final : BatchRun {
  static constexpr int G = Solver<T, ND>::G;
  hipStream_t st;
  lgdm_solver_opts o;
  BatchSolveBuffers& B;
  std::vector<lgdm_ctx*> ctx;          // by id; null when not in the run
  std::vector<RunControl> rc;
  std::vector<Idr<T, ND, S>> one;
  std::vector<double> se;
  std::vector<int> ended;              // ids whose solves ended, not yet taken
  KSlot* tab_host;
  KSlot* tab_dev;
  int nrun = 0;                        // requests in the device table
  int64_t tot[3] = {0, 0, 0};          // workgroups per launch family
  bool table_stale = true;

  BatchIdr(hipStream_t s, const lgdm_solver_opts& o_, BatchSolveBuffers& buf)
      : st(s), o(o_), B(buf), ctx(buf.max_requests, nullptr), rc(buf.max_requests), one(buf.max_requests),
        se(buf.max_requests, 0.0) {
    tab_host = static_cast<KSlot*>(B.table_host);
    tab_dev = static_cast<KSlot*>(B.table_dev);
  }
  double* sc(int j) { return B.sc_dev + (int64_t)j * KSCAL_DOUBLES; }
  double* xbest(int j) { return ctx[j]->kv + (int64_t)(KV_VECS - 1) * ctx[j]->ndof; }
  int every() const { return o.check_every > 0 ? o.check_every : 16; }
  void set_opts(const lgdm_solver_opts& o_) override { o = o_; }

  void reset_scalars(int j) {
    set_scalars_kernel<<<1, 64, 0, st>>>(sc(j), rc[j].tol_u * rc[j].tol_u, rc[j].tol_e * rc[j].tol_e, se[j],
                                         BREAK_REL, rc[j].seed());
  }

  hipError_t add(int j, lgdm_ctx* c, double tu, double te) override {
    if (j < 0 || j >= B.max_requests || ctx[j]) return hipErrorInvalidValue;
    ctx[j] = c;
    rc[j] = RunControl{};
    rc[j].setup(tu, te, Idr<T, ND, S>::F32, 1);
    se[j] = c->mat.E / c->mat.h;
    one[j].bind(c, st, sc(j), c->kpart);
    reset_scalars(j);
    hipError_t e = hipMemsetAsync(c->delta, 0, c->ndof * sizeof(double), st);
    if (e != hipSuccess) return e;
    one[j].begin(c->R);
    table_stale = true;
    return hipGetLastError();
  }

  // stop a request's solve on the device and drop it from the run
  hipError_t stop(int j) {
    table_stale = true;
    return hipMemcpyAsync(sc(j) + K_DONE, B.one_host, sizeof(double), hipMemcpyHostToDevice, st);
  }
  void remove(int j) override {
    if (j < 0 || j >= B.max_requests || !ctx[j]) return;
    (void)stop(j);
    ctx[j] = nullptr;
  }
  int active() const override {
    int n = 0;
    for (auto* c : ctx) n += c != nullptr;
    return n;
  }
  void take_finished(std::vector<int>& ids, std::vector<KrylovResult>& res) override {
    ids.clear();
    res.clear();
    for (int j : ended) {
      ids.push_back(j);
      res.push_back(rc[j].res);
    }
    ended.clear();
  }

  // device table of the requests in the run
  hipError_t build_table() {
    nrun = 0;
    tot[0] = tot[1] = tot[2] = 0;
    for (int j = 0; j < B.max_requests; ++j) {
      if (!ctx[j]) continue;
      const Idr<T, ND, S>& q = one[j];
      KSlot& k = tab_host[nrun++];
      k.nn = q.nn;
      k.n = q.n;
      k.row_ptr = ctx[j]->row_ptr;
      k.nbr_ptr = ctx[j]->nbr_ptr;
      k.nbr = ctx[j]->nbr;
      k.vals = q.vals;
      k.minv = q.minv;
      k.x = ctx[j]->delta;
      k.r = q.r;
      k.v = q.v;
      k.t = q.t;
      k.G = q.Gv;
      k.U = q.Uv;
      k.sc = q.sc;
      const int64_t nb[3] = {std::min<int64_t>(std::max<int64_t>((q.nn + BS - 1) / BS, 1), CAP_NODE),
                             std::min<int64_t>(std::max<int64_t>((q.nn * G + BS - 1) / BS, 1), CAP_SPMV),
                             std::min<int64_t>(std::max<int64_t>((q.n + BS - 1) / BS, 1), CAP_DOF)};
      for (int f = 0; f < 3; ++f) {
        k.blk0[f] = tot[f];
        k.nblk[f] = nb[f];
        tot[f] += nb[f];
      }
    }
    table_stale = false;
    if (nrun == 0) return hipSuccess;
    return hipMemcpyAsync(tab_dev, tab_host, nrun * sizeof(KSlot), hipMemcpyHostToDevice, st);
  }

  template <int K> void steps() {
    if constexpr (K < S) {
      idr_dir_batch<T, ND, S, K><<<tot[FAM_NODE], BS, 0, st>>>(tab_dev, nrun);
      spmv_batch<T, ND, G, 3, S><<<tot[FAM_SPMV], BS, 0, st>>>(tab_dev, nrun, K, B.part);
      idr_g_scalar_batch<S><<<nrun, BS, 0, st>>>(tab_dev, K, B.part);
      idr_upd_batch<T, ND, S, K><<<tot[FAM_NODE], BS, 0, st>>>(tab_dev, nrun, B.part);
      idr_r_scalar_batch<<<nrun, BS, 0, st>>>(tab_dev, B.part);
      steps<K + 1>();
    }
  }
  void cycle() {
    steps<0>();
    spmv_batch<T, ND, G, 2, 0><<<tot[FAM_SPMV], BS, 0, st>>>(tab_dev, nrun, 0, B.part);
    idr_om_scalar_batch<<<nrun, BS, 0, st>>>(tab_dev, B.part);
    idr_om_batch<ND, S><<<tot[FAM_DOF], BS, 0, st>>>(tab_dev, nrun, B.part);
    idr_f_scalar_batch<S><<<nrun, BS, 0, st>>>(tab_dev, B.part);
  }

  // read every request's scalars and act on them
  hipError_t decide_all(int64_t ran) {
    hipError_t e = hipMemcpyAsync(B.sc_host, B.sc_dev, (size_t)B.max_requests * KSCAL_DOUBLES * sizeof(double),
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    for (int j = 0; j < B.max_requests; ++j) {
      if (!ctx[j]) continue;
      bool save = false;
      const RunControl::Action a = rc[j].decide(B.sc_host + (int64_t)j * KSCAL_DOUBLES, o, ran, save);
      const size_t bytes = ctx[j]->ndof * sizeof(double);
      if (save && (e = hipMemcpyAsync(xbest(j), ctx[j]->delta, bytes, hipMemcpyDeviceToDevice, st)) != hipSuccess)
        return e;
      if ((a == RunControl::RETURN_BEST || a == RunControl::RESTART_BEST) && rc[j].have_best &&
          (e = hipMemcpyAsync(ctx[j]->delta, xbest(j), bytes, hipMemcpyDeviceToDevice, st)) != hipSuccess)
        return e;
      if (a == RunControl::RESTART || a == RunControl::RESTART_BEST) {
        reset_scalars(j);
        one[j].restart(ctx[j]->R, ctx[j]->delta);
      }
      if (rc[j].fin) {
        if ((e = stop(j)) != hipSuccess) return e;
        ctx[j] = nullptr;
        ended.push_back(j);
      }
    }
    return hipGetLastError();
  }

  // requests added since the last round are checked in this round too: the
  // scalars of a request whose start already converged say so with no iteration
  hipError_t advance() override {
    if (table_stale) {
      hipError_t e = build_table();
      if (e != hipSuccess) return e;
    }
    int64_t ran = 0;
    if (nrun > 0) {
      const int ncyc = Idr<T, ND, S>::cycles_for(every());
      for (int i = 0; i < ncyc; ++i) cycle();
      ran = (int64_t)ncyc * (S + 1);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    hipError_t e = decide_all(ran);
    if (e != hipSuccess) return e;
    // the copies enqueued by the decisions land before the caller reads the results
    return hipStreamSynchronize(st);
  }
};

template <typename T, int ND>
std::unique_ptr<BatchRun> make_batch_impl(hipStream_t st, const lgdm_solver_opts& o, BatchSolveBuffers& B) {
  switch (o.idr_s) {
    case 1: return std::unique_ptr<BatchRun>(new BatchIdr<T, ND, 1>(st, o, B));
    case 2: return std::unique_ptr<BatchRun>(new BatchIdr<T, ND, 2>(st, o, B));
    case 8: return std::unique_ptr<BatchRun>(new BatchIdr<T, ND, 8>(st, o, B));
    default: return std::unique_ptr<BatchRun>(new BatchIdr<T, ND, 4>(st, o, B));
  }
}

template <typename T, int ND>
std::unique_ptr<KrylovRun> make_run_impl(lgdm_ctx* c, const double* b, double* x,
                                         const lgdm_solver_opts& o, double tu, double te) {
  if (o.krylov_method == LGDM_KRYLOV_BICGSTAB)
    return std::unique_ptr<KrylovRun>(new KrylovRunImpl<Solver<T, ND>>(c, b, x, o, tu, te));
  switch (o.idr_s) {
    case 1: return std::unique_ptr<KrylovRun>(new KrylovRunImpl<Idr<T, ND, 1>>(c, b, x, o, tu, te));
    case 2: return std::unique_ptr<KrylovRun>(new KrylovRunImpl<Idr<T, ND, 2>>(c, b, x, o, tu, te));
    case 8: return std::unique_ptr<KrylovRun>(new KrylovRunImpl<Idr<T, ND, 8>>(c, b, x, o, tu, te));
    default: return std::unique_ptr<KrylovRun>(new KrylovRunImpl<Idr<T, ND, 4>>(c, b, x, o, tu, te));
  }
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

// defaults of zero-initialised solver options
lgdm_solver_opts fill_opts(const lgdm_solver_opts* o) {
  lgdm_solver_opts r{};
  if (o) r = *o;
  if (r.max_newton <= 0) r.max_newton = 30;
  if (r.max_krylov <= 0) r.max_krylov = 20000;
  if (!(r.tol_newton > 0)) r.tol_newton = 1e-8;
  if (!(r.tol_krylov > 0)) r.tol_krylov = 1e-10;
  if (r.check_every <= 0) r.check_every = 16;
  if (r.max_restarts <= 0) r.max_restarts = 8;
  if (r.krylov_method != LGDM_KRYLOV_BICGSTAB) r.krylov_method = LGDM_KRYLOV_IDRS;
  if (r.forcing != LGDM_FORCING_FIXED) r.forcing = LGDM_FORCING_ADAPTIVE;
  if (r.precond != LGDM_PRECOND_AMG && r.precond != LGDM_PRECOND_BLOCK_JACOBI) r.precond = LGDM_PRECOND_DEFAULT;
  r.idr_s = r.idr_s <= 0 ? 8 : (r.idr_s <= 1 ? 1 : (r.idr_s <= 2 ? 2 : (r.idr_s <= 4 ? 4 : 8)));
  if (!(r.zone_damage > 0.0 && r.zone_damage < 1.0)) r.zone_damage = 0.99;
  if (r.process_zone != LGDM_ZONE_OFF && r.process_zone != LGDM_ZONE_EVERY_TANGENT) r.process_zone = LGDM_ZONE_DEFAULT;
  if (r.line_search != LGDM_LINE_SEARCH_ON) r.line_search = LGDM_LINE_SEARCH_OFF;
  return r;
}

hipError_t krylov_setup(lgdm_ctx* c) {
  switch (c->nd) {
    case 2: return setup_impl<double, 2>(c);
    case 3: return setup_impl<double, 3>(c);
    default: return setup_impl<double, 4>(c);
  }
}

std::unique_ptr<KrylovRun> make_krylov_run(lgdm_ctx* c, const double* b, double* x,
                                           const lgdm_solver_opts& o, double tol_u, double tol_e) {
  const bool mixed = c->precision == LGDM_MIXED;
  switch (c->nd) {
    case 2: return mixed ? make_run_impl<float, 2>(c, b, x, o, tol_u, tol_e)
                         : make_run_impl<double, 2>(c, b, x, o, tol_u, tol_e);
    case 3: return mixed ? make_run_impl<float, 3>(c, b, x, o, tol_u, tol_e)
                         : make_run_impl<double, 3>(c, b, x, o, tol_u, tol_e);
    default: return mixed ? make_run_impl<float, 4>(c, b, x, o, tol_u, tol_e)
                          : make_run_impl<double, 4>(c, b, x, o, tol_u, tol_e);
  }
}

std::unique_ptr<BatchRun> make_batch_run(hipStream_t st, int nd, bool mixed, const lgdm_solver_opts& o,
                                         BatchSolveBuffers& B) {
  if (o.krylov_method == LGDM_KRYLOV_BICGSTAB || B.max_requests <= 0) return nullptr;
  switch (nd) {
    case 2: return mixed ? make_batch_impl<float, 2>(st, o, B) : make_batch_impl<double, 2>(st, o, B);
    case 3: return mixed ? make_batch_impl<float, 3>(st, o, B) : make_batch_impl<double, 3>(st, o, B);
    default: return mixed ? make_batch_impl<float, 4>(st, o, B) : make_batch_impl<double, 4>(st, o, B);
  }
}

// device memory of the batch's solve buffers, through the batch's allocator
static hipError_t bs_alloc(BatchSolveBuffers& B, void** p, size_t bytes) {
  if (!B.alloc_fn) return hipMalloc(p, bytes);
  *p = B.alloc_fn(bytes, B.alloc_user);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
static void bs_free(BatchSolveBuffers& B, void* p) {
  if (!p) return;
  if (B.free_fn) B.free_fn(p, B.alloc_user);
  else (void)hipFree(p);
}

hipError_t batch_solve_alloc(BatchSolveBuffers& B, int max_requests) {
  B.max_requests = max_requests;
  hipError_t e = bs_alloc(B, &B.table_dev, max_requests * sizeof(KSlot));
  if (e == hipSuccess) e = hipHostMalloc(&B.table_host, max_requests * sizeof(KSlot), hipHostMallocDefault);
  if (e == hipSuccess) e = bs_alloc(B, (void**)&B.sc_dev, (size_t)max_requests * KSCAL_DOUBLES * sizeof(double));
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&B.sc_host, (size_t)max_requests * KSCAL_DOUBLES * sizeof(double),
                      hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&B.one_host, sizeof(double), hipHostMallocDefault);
  if (e == hipSuccess)
    e = bs_alloc(B, (void**)&B.part, (size_t)max_requests * BATCH_PART_PER_REQUEST * sizeof(double));
  if (e == hipSuccess) *B.one_host = 1.0;
  return e;
}

void batch_solve_free(BatchSolveBuffers& B) {
  bs_free(B, B.table_dev);
  if (B.table_host) (void)hipHostFree(B.table_host);
  bs_free(B, B.sc_dev);
  if (B.sc_host) (void)hipHostFree(B.sc_host);
  if (B.one_host) (void)hipHostFree(B.one_host);
  bs_free(B, B.part);
  auto af = B.alloc_fn;
  auto ff = B.free_fn;
  void* au = B.alloc_user;
  B = BatchSolveBuffers{};
  B.alloc_fn = af;
  B.free_fn = ff;
  B.alloc_user = au;
}

hipError_t krylov_solve(lgdm_ctx* c, const double* b, double* xout, const lgdm_solver_opts& o,
                        double tol_u, double tol_e, KrylovResult& res) {
  std::unique_ptr<KrylovRun> run = make_krylov_run(c, b, xout, o, tol_u, tol_e);
  hipError_t e = run->start();
  while (e == hipSuccess) {
    e = run->check();
    if (e != hipSuccess || run->finished()) break;
    if (!run->needs_check()) e = run->launch();
  }
  res = run->result();
  return e;
}

// Inexact Newton: the relative tolerances of one Newton correction, per
// field.  A correction needs no smaller linear residual than a fraction of
// what the field may keep at convergence: tol_f = max(eta,
// min(0.5, c * tol_newton * |F_f| / |R_f|)) with eta = tol_krylov, so the
// early corrections solve to tol_krylov and the last one only as far as the
// Newton test needs.  With an
// FP32-stored operator the linear residual left in a correction comes back
// amplified in the next FP64 residual (by up to the FP32 rounding of the
// tangent times its condition number), so mixed contexts keep a tenfold
// margin more (c = 0.01 against 0.1).
void newton_forcing(lgdm_ctx* c, const lgdm_solver_opts& o, double& tol_u, double& tol_e) {
  tol_u = tol_e = o.tol_krylov;
  if (o.forcing == LGDM_FORCING_FIXED) return;
  const double ru = std::sqrt(c->last_norms[0]), re = std::sqrt(c->last_norms[1]);
  const double fu = std::sqrt(c->last_norms[2]), fe = std::sqrt(c->last_norms[3]);
  // an increment still unconverged after ACCURATE_AFTER Newton iterations is
  // strongly nonlinear: its inexact iterates can cycle, so it continues with
  // accurate corrections (the exact-Newton limit)
  constexpr int ACCURATE_AFTER = 8;
  const double eta = c->nw_iter++ >= ACCURATE_AFTER ? std::min(o.tol_krylov, 1e-8) : o.tol_krylov;
  const double margin = c->precision == LGDM_MIXED ? 0.01 : 0.1;
  tol_u = tol_e = eta;
  if (ru > 0) tol_u = std::max(eta, std::min(0.5, margin * o.tol_newton * fu / ru));
  if (re > 0) tol_e = std::max(eta, std::min(0.5, margin * o.tol_newton * fe / re));
}

template <typename T, int ND> hipError_t spmv_only_impl(lgdm_ctx* c, const double* x) {
  // the operator application of an IDR(8) step (SpMV with its eight shadow
  // dot products and |y|^2), the launch that dominates a default solve
  using I = Idr<T, ND, 8>;
  I S;
  S.bind(c, c->stream, c->kscal, c->kpart);
  set_scalars_kernel<<<1, 64, 0, c->stream>>>(S.sc, 0.0, 0.0, c->mat.E / c->mat.h, BREAK_REL, 0);
  spmv_kernel<T, ND, I::G, 3, 8><<<S.spmv_grid(), BS, 0, c->stream>>>(
      S.nn, c->row_ptr, c->nbr_ptr, c->nbr, S.vals, x, S.t, nullptr, S.sc, c->kpart);
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
