// Process-zone solve inside the multigrid preconditioner (H6 on the softening
// branch).
//
// Where damaged Gauss points are loading (the history variable grows in this
// Newton iterate, chi = 1, Eq. A.2) the consistent tangent of Eqs. 11b and
// 11d carries the softening terms D' chi: the element stiffness loses
// positivity there and the scaled system S K acquires eigenvalues that
// neither the block-Jacobi smoother nor the rigid-body coarse space of the
// multigrid cycle represent.  The Krylov method then stalls for thousands of
// steps.  Those modes live on the few elements that are both loading and
// highly damaged, so the preconditioner solves that zone exactly:
//
//   zone    nodes of the elements with a Gauss point that is loading and has
//           trial damage D >= zone_damage (0.99 by default; moved tenfold
//           closer to 1, twice at most, while the zone exceeds the limits
//           below), chosen afresh for every tangent
//   levels  breadth-first level sets of the zone's node graph, each
//           connected component from a pseudo-peripheral node (George & Liu,
//           ACM TOMS 5, 1979): a node's neighbours lie in its own level or
//           the next or previous one, so in level order the zone's block Z of
//           S K is block tridiagonal.  Consecutive levels are merged into
//           groups of at least ZONE_GROUP_MIN unknowns (fewer launches).
//   factor  twisted block LU over the groups 0..L-1, from both ends toward
//           the middle group c = L/2: S_k = Z_kk - Z_k,k-1 S_{k-1}^-1 Z_k-1,k
//           for k < c, S_k = Z_kk - Z_k,k+1 S_{k+1}^-1 Z_k+1,k for k > c, and
//           S_c with both corrections.  Each S_k by LU with partial pivoting
//           and explicit inverse G_k (rocSOLVER getrf, getri), then
//           P_k = G_k Z_k,k-1 and N_k = G_k Z_k,k+1 (rocBLAS gemm); the two
//           chains run on two streams.  A CPU model on the 128x32x16 beam
//           after its peak (zone from D >= 0.99, 5,808 unknowns, condition
//           number 9e8) took 5e9 flops against 4e11 for the dense LU, and
//           its (one-sided) block solve differed from the dense one by 5e-9.
//   apply   x_z = Z^-1 b_z by sweeps from both ends: y_k = G_k b_k -
//           P_k y_{k-1} (k < c) and y_k = G_k b_k - N_k y_{k+1} (k > c) in
//           the same launches, x_c = G_c b_c - P_c y_{c-1} - N_c y_{c+1},
//           then x_k = y_k - N_k x_{k+1} (k < c) and x_k = y_k - P_k x_{k-1}
//           (k > c), again two groups per launch: about L + 1 launches, one
//           wavefront per row of the row-major copies of [G_k | P_k | N_k];
//           r = b - S K x_z (only rows of the zone
//           and its neighbour nodes change); out = x_z + M_mg r, with M_mg
//           the multigrid cycle (multiplicative: the same CPU model needed 64
//           GMRES steps with it, 97 with the additive form x_z + M_mg b, and
//           more than 3000 without a zone)
//
// Within one Newton increment a tangent whose zone has the same nodes as the
// one last factored keeps those factors: the zone's block changes little
// between Newton iterates.  The apply is a fixed linear map for the whole
// solve, so IDR(s) takes it as its preconditioner unchanged.  Every sum has a
// fixed order.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#include "lgdm_internal.h"

namespace lgdm {

namespace {

constexpr int64_t ZONE_GROUP_MIN = 512;           // unknowns per group, at least (but the last)
constexpr int64_t ZONE_MAX_GROUP = 4096;          // unknowns per group, at most
constexpr int64_t ZONE_MAX_PANEL = 320ll << 20;   // doubles of the factor panels P + Q (2.5 GiB)

}  // namespace

struct Zone {
  // host copies of the mesh structure (taken at the first setup)
  std::vector<int32_t> conn, nbr_ptr, nbr;
  std::vector<uint8_t> eflag;
  std::vector<int32_t> zmap_h;              // node -> zone index, -1 outside
  // the zone of the current tangent, in level order
  std::vector<int32_t> nodes, group;        // zone index -> node, group
  std::vector<int64_t> goff, poff, qoff;    // group offsets: unknowns, panel P, panel Q
  int64_t L = 0, mmax = 0;
  // device
  uint8_t* eflag_d = nullptr;               // [n_elems]
  int32_t* zmap = nullptr;                  // [n_nodes]
  int32_t* znodes = nullptr;                // [cap_nodes] zone index -> node
  int32_t* zgroup = nullptr;                // [cap_nodes] zone index -> group
  int64_t* goff_d = nullptr;                // [cap_groups + 1]
  int64_t* poff_d = nullptr;                // [cap_groups + 1]
  int32_t* halo = nullptr;                  // nodes whose rows r = b - S K x_z changes [cap_halo]
  // per group k (m_k unknowns; column major, leading dimension m_k):
  //   panel [Z_k,k-1 | Z_kk -> G_k | Z_k,k+1] in P, [P_k | N_k] in Q
  double* P = nullptr;                      // [cap_p]
  double* Q = nullptr;                      // [cap_q]
  // the sweeps' matrices, row major, in P's layout: per group k the rows of
  // [G_k | P_k | N_k] (m_k + m_{k-1} + m_{k+1} each); FP32 in mixed
  // contexts (t32), FP64 otherwise
  double* T = nullptr;                      // [cap_p] doubles of storage
  bool t32 = false;
  rocblas_int* ipiv = nullptr;              // [cap_m] pivots of the chain from group 0
  rocblas_int* ipiv2 = nullptr;             // [cap_m] pivots of the chain from group L-1
  rocblas_int* info = nullptr;              // [2 cap_groups]
  double* bz = nullptr;                     // [cap_nodes * 4] b at the zone's unknowns
  double* xz = nullptr;                     // [cap_nodes * 4] Z^-1 b_z
  double* r = nullptr;                      // [ndof]
  int64_t cap_nodes = 0, cap_halo = 0, cap_groups = 0, cap_p = 0, cap_q = 0, cap_m = 0;
  void* ws = nullptr;
  void* ws2 = nullptr;
  size_t ws_size = 0;
  rocblas_handle handle = nullptr;          // on the context's stream: chain from group 0, middle group
  rocblas_handle handle2 = nullptr;         // on stream2: chain from group L-1
  hipStream_t stream2 = nullptr;            // default priority
  hipEvent_t ev_built = nullptr, ev_chain2 = nullptr;
  int64_t nz = 0, nh = 0;                   // zone nodes, halo nodes of the current tangent
  bool active = false;
  // the zone whose factors P and Q hold: its nodes (ascending) and the
  // increment it was built in
  std::vector<int32_t> built_nodes;
  int64_t built_serial = -1;
};

namespace {

constexpr int ZBS = 256;

// elements with a loading Gauss point (chi: kappa grew past the band of
// Fig. 8b) whose trial damage is at least dmin; one thread per element
__global__ void zone_flag_kernel(int64_t n_elems, int ngp, const double* __restrict__ kappa_t,
                                 const double* __restrict__ kappa_n, const double* __restrict__ D_t,
                                 double tol_hist, double dmin, uint8_t* __restrict__ flag) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_elems) return;
  uint8_t f = 0;
  for (int g = 0; g < ngp; ++g) {
    const int64_t i = e * ngp + g;
    if (kappa_t[i] - kappa_n[i] > tol_hist && D_t[i] >= dmin) f = 1;
  }
  flag[e] = f;
}

__global__ void zone_zero_kernel(int64_t n, double* __restrict__ p) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// P_g entries of the zone's block of S K: one thread per (zone node,
// neighbour position); the neighbour's group is g - 1, g or g + 1
template <typename T>
__global__ void zone_build_kernel(int64_t nz, int max_nbr, const int32_t* __restrict__ znodes,
                                  const int32_t* __restrict__ zmap, const int32_t* __restrict__ zgroup,
                                  const int64_t* __restrict__ goff, const int64_t* __restrict__ poff,
                                  const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ nbr_ptr,
                                  const int32_t* __restrict__ nbr, const T* __restrict__ vals, double se,
                                  double* __restrict__ P) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nz * max_nbr) return;
  const int64_t za = t / max_nbr;
  const int p = (int)(t % max_nbr);
  const int64_t a = znodes[za];
  const int nb0 = nbr_ptr[a], nnb = nbr_ptr[a + 1] - nb0;
  if (p >= nnb) return;
  const int32_t zq = zmap[nbr[nb0 + p]];
  if (zq < 0) return;
  const int ga = zgroup[za], gq = zgroup[zq];
  const int64_t g0 = goff[ga], m = goff[ga + 1] - g0, mp = ga > 0 ? g0 - goff[ga - 1] : 0;
  // the host checked that neighbouring groups differ by at most one
  const int64_t colbase = gq < ga ? 0 : (gq == ga ? mp : mp + m);
  const int64_t col0 = colbase + 4 * (int64_t)zq - goff[gq], row0 = 4 * za - g0;
  double* Pg = P + poff[ga];
  const int64_t rowlen = (int64_t)nnb * 4, rb = row_ptr[a * 4];
  for (int i = 0; i < 4; ++i) {
    const double s = i == 3 ? se : 1.0;
    for (int j = 0; j < 4; ++j)
      Pg[(row0 + i) + (col0 + j) * m] = s * (double)vals[rb + i * rowlen + (int64_t)p * 4 + j];
  }
}

// bz = b at the zone's unknowns
__global__ void zone_gather_kernel(int64_t nz, const int32_t* __restrict__ znodes, const double* __restrict__ b,
                                   double* __restrict__ bz, const double* __restrict__ sc) {
  if (sc && sc[KSLOT_DONE] != 0.0) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nz * 4) return;
  bz[t] = b[(int64_t)znodes[t / 4] * 4 + (t % 4)];
}

// Row-major copy of a column-major m x n block: out[r * ldo + c0 + c] =
// A[r + c * m], rounded once to TO; one thread per entry
template <typename TO>
__global__ void zone_rowmajor_kernel(int64_t m, int64_t n, const double* __restrict__ A, TO* __restrict__ out,
                                     int64_t ldo, int64_t c0) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m * n) return;
  const int64_t r = t % m, c = t / m;
  out[r * ldo + c0 + c] = (TO)A[t];
}

// One group's step of a sweep: y[r] = sum_c A[r, c] u[c] - sum_c
// A[r, op + c] v[c] - sum_c A[r, on + c] w[c] for r < m (A row major with
// leading dimension lda, element type TA of the kernel; nu, nv or nw may be
// 0), with accumulate y[r] plus that; products and sums in FP64.  One
// wavefront per row; lanes stride the row by 64 (coalesced) and are combined
// by a fixed butterfly, so every apply sums in the same order.
struct SweepOp {
  int64_t m, lda;
  const void* A;   // TA, row major
  const double* u;
  int64_t nu;
  const double* v;
  int64_t nv, op;
  const double* w;
  int64_t nw, on;
  double* y;
  int accumulate;
};
constexpr int SW_ROWS = ZBS / 64;
inline unsigned sweep_blocks(const SweepOp& o) { return (unsigned)((o.m + SW_ROWS - 1) / SW_ROWS); }

// acc += sgn * a[c] * x[c] for c = lane, lane + 64, ... < n, in that order;
// eight loads of each operand are issued before their products are summed
// (one load pair in flight per wavefront left the sweeps latency bound)
template <typename TA>
__device__ __forceinline__ void sweep_dot(const TA* __restrict__ a, const double* __restrict__ x, int64_t n,
                                          int lane, double sgn, double& acc) {
  int64_t c = lane;
  for (; c + 7 * 64 < n; c += 8 * 64) {
    double av[8], xv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      av[j] = (double)a[c + j * 64];
      xv[j] = x[c + j * 64];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) acc += sgn * av[j] * xv[j];
  }
  for (; c < n; c += 64) acc += sgn * (double)a[c] * x[c];
}

// two independent group steps in one launch (the two ends of the twisted
// sweep): blocks [0, nblk_a) take a, the rest take b
template <typename TA>
__global__ void __launch_bounds__(ZBS) zone_sweep_kernel(SweepOp a, SweepOp b, unsigned nblk_a,
                                                         const double* __restrict__ sc) {
  if (sc && sc[KSLOT_DONE] != 0.0) return;
  const bool first = blockIdx.x < nblk_a;
  const SweepOp& o = first ? a : b;
  const int lane = threadIdx.x % 64;
  const int64_t row = (int64_t)(first ? blockIdx.x : blockIdx.x - nblk_a) * SW_ROWS + threadIdx.x / 64;
  if (row >= o.m) return;  // uniform over the wavefront
  const TA* __restrict__ r = static_cast<const TA*>(o.A) + row * o.lda;
  double acc = 0.0;
  sweep_dot<TA>(r, o.u, o.nu, lane, 1.0, acc);
  sweep_dot<TA>(r + o.op, o.v, o.nv, lane, -1.0, acc);
  sweep_dot<TA>(r + o.on, o.w, o.nw, lane, -1.0, acc);
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) o.y[row] = o.accumulate ? o.y[row] + acc : acc;
}

// r = b everywhere (the halo rows are overwritten next)
__global__ void zone_copy_kernel(int64_t n, const double* __restrict__ b, double* __restrict__ r,
                                 const double* __restrict__ sc) {
  if (sc && sc[KSLOT_DONE] != 0.0) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    r[i] = b[i];
}

// r_h = b_h - sum over zone neighbours q of (S K)_{hq} x_z(q), rows of the
// halo nodes: RES_G lanes per halo node, lane l taking neighbour positions
// l, l + RES_G, ...; the four row sums are combined by a fixed butterfly
constexpr int RES_G = 16;
template <typename T>
__global__ void __launch_bounds__(ZBS) zone_residual_kernel(
    int64_t nh, const int32_t* __restrict__ halo, const int32_t* __restrict__ zmap,
    const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ nbr_ptr, const int32_t* __restrict__ nbr,
    const T* __restrict__ vals, double se, const double* __restrict__ b, const double* __restrict__ xz,
    double* __restrict__ r, const double* __restrict__ sc) {
  if (sc && sc[KSLOT_DONE] != 0.0) return;
  const int64_t hi = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / RES_G;
  const int lane = threadIdx.x % RES_G;
  if (hi >= nh) return;  // uniform over the lane group
  const int64_t h = halo[hi];
  const int nb0 = nbr_ptr[h], nnb = nbr_ptr[h + 1] - nb0;
  const int64_t rowlen = (int64_t)nnb * 4, rs = row_ptr[h * 4];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int p = lane; p < nnb; p += RES_G) {
    const int32_t zq = zmap[nbr[nb0 + p]];
    if (zq < 0) continue;
    double x[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = xz[4 * (int64_t)zq + j];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i] += (double)vals[rs + i * rowlen + (int64_t)p * 4 + j] * x[j];
  }
#pragma unroll
  for (int o = RES_G / 2; o > 0; o >>= 1)
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] += __shfl_xor(acc[i], o, RES_G);
  if (lane < 4) {
    double mine = acc[0];
#pragma unroll
    for (int i = 1; i < 4; ++i)
      if (lane == i) mine = acc[i];
    const int64_t row = h * 4 + lane;
    r[row] = b[row] - (lane == 3 ? se : 1.0) * mine;
  }
}

// out += x_z at the zone's unknowns
__global__ void zone_scatter_kernel(int64_t nz, const int32_t* __restrict__ znodes, const double* __restrict__ xz,
                                    double* __restrict__ out, const double* __restrict__ sc) {
  if (sc && sc[KSLOT_DONE] != 0.0) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nz * 4) return;
  out[(int64_t)znodes[t / 4] * 4 + (t % 4)] += xz[t];
}

inline unsigned nblocks(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + ZBS - 1) / ZBS); }

// a rocBLAS / rocSOLVER status as a HIP error, naming the call in msg
hipError_t rb_err(rocblas_status s, const char* what, std::string& msg) {
  if (s == rocblas_status_success) return hipSuccess;
  msg = std::string("process zone: ") + what + " returned " + rocblas_status_to_string(s);
  return hipErrorUnknown;
}

}  // namespace

// Breadth-first levels of the zone's node graph (zone indices 0..nz-1,
// adjacency adj_ptr / adj): every connected component from a
// pseudo-peripheral node, components one after the other.  Fills the level
// of each index and returns the number of levels.
int64_t zone_levels(int64_t nz, const int64_t* adj_ptr, const int32_t* adj, int32_t* level) {
  std::fill(level, level + nz, -1);
  std::vector<int32_t> dist(nz, -1), queue;
  queue.reserve(nz);
  // BFS from s over its component: distances in dist, visit order in queue;
  // returns the eccentricity of s
  auto bfs = [&](int32_t s) {
    queue.clear();
    queue.push_back(s);
    dist[s] = 0;
    int32_t ecc = 0;
    for (size_t h = 0; h < queue.size(); ++h) {
      const int32_t v = queue[h];
      ecc = std::max(ecc, dist[v]);
      for (int64_t p = adj_ptr[v]; p < adj_ptr[v + 1]; ++p)
        if (dist[adj[p]] < 0) {
          dist[adj[p]] = dist[v] + 1;
          queue.push_back(adj[p]);
        }
    }
    return ecc;
  };
  auto reset = [&]() {
    for (int32_t v : queue) dist[v] = -1;
  };
  int64_t base = 0;
  for (int32_t i0 = 0; i0 < (int32_t)nz; ++i0) {
    if (level[i0] >= 0) continue;
    // pseudo-peripheral start: restart from a least-connected node of the
    // last level while the eccentricity grows
    int32_t start = i0;
    int32_t ecc = bfs(start);
    for (int round = 0; round < 8; ++round) {
      int32_t cand = -1;
      int64_t cdeg = 0;
      for (int32_t v : queue)
        if (dist[v] == ecc) {
          const int64_t d = adj_ptr[v + 1] - adj_ptr[v];
          if (cand < 0 || d < cdeg) cand = v, cdeg = d;
        }
      reset();
      const int32_t e2 = bfs(cand);
      if (e2 <= ecc) break;
      start = cand;
      ecc = e2;
    }
    reset();
    ecc = bfs(start);
    for (int32_t v : queue) level[v] = (int32_t)(base + dist[v]);
    reset();
    base += ecc + 1;
  }
  return base;
}

void zone_release(lgdm_ctx* c) {
  if (!c->zone) return;
  Zone& z = *c->zone;
  if (z.handle) (void)rocblas_destroy_handle(z.handle);
  if (z.handle2) (void)rocblas_destroy_handle(z.handle2);
  if (z.ev_built) (void)hipEventDestroy(z.ev_built);
  if (z.ev_chain2) (void)hipEventDestroy(z.ev_chain2);
  if (z.stream2) (void)hipStreamDestroy(z.stream2);
  delete c->zone;
  c->zone = nullptr;
}

// Choose the zone of the current tangent, order it by levels and factor its
// block.  Leaves the zone inactive (plain multigrid) where there is none or
// it does not fit.
hipError_t zone_setup(lgdm_ctx* c, bool allow_alloc, bool reuse, double dmin0, bool* factored, std::string& msg) {
  *factored = false;
  if (c->dim != 3 || c->nd != 4 || c->order2) return hipSuccess;
  if (!c->zone) {
    if (!allow_alloc) return hipErrorNotReady;
    c->zone = new Zone();
  }
  Zone& z = *c->zone;
  z.active = false;
  hipError_t e;
  const int64_t ne = c->n_elems, nn = c->n_nodes;
  if (z.conn.empty()) {
    if (!allow_alloc) return hipErrorNotReady;
    z.conn.resize(ne * c->nen);
    z.nbr_ptr.resize(nn + 1);
    z.nbr.resize(c->npairs);
    z.eflag.resize(ne);
    z.zmap_h.assign(nn, -1);
    if ((e = hipMemcpyAsync(z.conn.data(), c->conn, z.conn.size() * 4, hipMemcpyDeviceToHost, c->stream)) ||
        (e = hipMemcpyAsync(z.nbr_ptr.data(), c->nbr_ptr, z.nbr_ptr.size() * 4, hipMemcpyDeviceToHost, c->stream)) ||
        (e = hipMemcpyAsync(z.nbr.data(), c->nbr, z.nbr.size() * 4, hipMemcpyDeviceToHost, c->stream)))
      return e;
    z.eflag_d = (uint8_t*)dalloc(c, ne);
    z.zmap = (int32_t*)dalloc(c, nn * sizeof(int32_t));
    z.r = (double*)dalloc(c, c->ndof * sizeof(double));
    if (!z.eflag_d || !z.zmap || !z.r) {
      msg = "device allocation failed (process zone)";
      return hipErrorOutOfMemory;
    }
    if (rocblas_create_handle(&z.handle) != rocblas_status_success ||
        rocblas_create_handle(&z.handle2) != rocblas_status_success) {
      msg = "rocblas_create_handle failed";
      return hipErrorUnknown;
    }
    // the second chain of the factorisation runs on a stream of its own
    // (default priority), ordered against the context's stream by events
    if ((e = hipStreamCreateWithFlags(&z.stream2, hipStreamNonBlocking)) ||
        (e = hipEventCreateWithFlags(&z.ev_built, hipEventDisableTiming)) ||
        (e = hipEventCreateWithFlags(&z.ev_chain2, hipEventDisableTiming)))
      return e;
    // no atomics: the factors, and the solves they precondition, are the
    // same bits in every run
    if ((e = rb_err(rocblas_set_atomics_mode(z.handle, rocblas_atomics_not_allowed), "rocblas_set_atomics_mode",
                    msg)) ||
        (e = rb_err(rocblas_set_atomics_mode(z.handle2, rocblas_atomics_not_allowed), "rocblas_set_atomics_mode",
                    msg)) ||
        (e = rb_err(rocblas_set_stream(z.handle2, z.stream2), "rocblas_set_stream", msg)))
      return e;
  }
  if ((e = rb_err(rocblas_set_stream(z.handle, c->stream), "rocblas_set_stream", msg))) return e;
  std::fill(z.zmap_h.begin(), z.zmap_h.end(), -1);
  // the zone: raise the damage threshold until it fits
  std::vector<int32_t> sorted, level, lgroup;
  std::vector<int64_t> adj_ptr;
  std::vector<int32_t> adj;
  // the candidate's layout; it replaces the zone's only once it is built, so
  // that a reused zone keeps the layout its factors were built with
  std::vector<int64_t> goff, poff, qoff;
  int64_t L = 0, mmax = 0;
  bool fits = false;
  for (double dmin : {dmin0, 1.0 - 0.1 * (1.0 - dmin0), 1.0 - 0.01 * (1.0 - dmin0)}) {
    zone_flag_kernel<<<nblocks(ne), ZBS, 0, c->stream>>>(ne, c->ngp, c->kappa_t, c->kappa_n, c->D_t,
                                                         c->mat.tol_hist, dmin, z.eflag_d);
    if ((e = hipMemcpyAsync(z.eflag.data(), z.eflag_d, ne, hipMemcpyDeviceToHost, c->stream)) ||
        (e = hipStreamSynchronize(c->stream)))
      return e;
    sorted.clear();
    for (int64_t el = 0; el < ne; ++el)
      if (z.eflag[el])
        for (int a = 0; a < c->nen; ++a) sorted.push_back(z.conn[el * c->nen + a]);
    std::sort(sorted.begin(), sorted.end());
    sorted.erase(std::unique(sorted.begin(), sorted.end()), sorted.end());
    const int64_t nz = (int64_t)sorted.size();
    if (nz == 0) return hipSuccess;
    // a later tangent of the same increment with the same zone keeps the
    // factors (the halo residual and the cycle read the current tangent)
    if (reuse && c->in_increment && z.built_serial == c->inc_serial && sorted == z.built_nodes) {
      z.active = true;
      return hipSuccess;
    }
    // the zone's node graph and its levels, then the groups
    for (int64_t i = 0; i < nz; ++i) z.zmap_h[sorted[i]] = (int32_t)i;
    adj_ptr.assign(nz + 1, 0);
    adj.clear();
    for (int64_t i = 0; i < nz; ++i) {
      const int32_t a = sorted[i];
      for (int32_t p = z.nbr_ptr[a]; p < z.nbr_ptr[a + 1]; ++p) {
        const int32_t q = z.zmap_h[z.nbr[p]];
        if (q >= 0 && q != i) adj.push_back(q);
      }
      adj_ptr[i + 1] = (int64_t)adj.size();
    }
    for (int32_t a : sorted) z.zmap_h[a] = -1;
    level.resize(nz);
    const int64_t nlev = zone_levels(nz, adj_ptr.data(), adj.data(), level.data());
    std::vector<int64_t> lcount(nlev, 0);
    for (int64_t i = 0; i < nz; ++i) lcount[level[i]] += 4;
    lgroup.assign(nlev, 0);
    goff.assign(1, 0);
    int64_t acc = 0;
    for (int64_t l = 0; l < nlev; ++l) {
      lgroup[l] = (int32_t)(goff.size() - 1);
      acc += lcount[l];
      if (acc >= ZONE_GROUP_MIN || l + 1 == nlev) {
        goff.push_back(goff.back() + acc);
        acc = 0;
      }
    }
    L = (int64_t)goff.size() - 1;
    mmax = 0;
    for (int64_t k = 0; k < L; ++k) mmax = std::max(mmax, goff[k + 1] - goff[k]);
    poff.assign(L + 1, 0);
    qoff.assign(L + 1, 0);
    for (int64_t k = 0; k < L; ++k) {
      const int64_t m = goff[k + 1] - goff[k], mp = k > 0 ? goff[k] - goff[k - 1] : 0,
                    mn = k + 1 < L ? goff[k + 2] - goff[k + 1] : 0;
      poff[k + 1] = poff[k] + m * (mp + m + mn);
      qoff[k + 1] = qoff[k] + m * (mp + mn);
    }
    if (mmax <= ZONE_MAX_GROUP && poff[L] + qoff[L] <= ZONE_MAX_PANEL) {
      fits = true;
      break;
    }
  }
  if (!fits) return hipSuccess;
  // from here on the zone's layout is this candidate's; the factors are
  // valid again only once built
  z.built_serial = -1;
  z.built_nodes.clear();
  z.goff.swap(goff);
  z.poff.swap(poff);
  z.qoff.swap(qoff);
  z.L = L;
  z.mmax = mmax;
  // zone order: by group, ascending node within a group
  z.nz = (int64_t)sorted.size();
  z.nodes.resize(z.nz);
  z.group.resize(z.nz);
  {
    std::vector<int64_t> fill(z.L, 0);
    for (int64_t k = 0; k < z.L; ++k) fill[k] = z.goff[k] / 4;
    for (int64_t i = 0; i < z.nz; ++i) {
      const int32_t g = lgroup[level[i]];
      const int64_t pos = fill[g]++;
      z.nodes[pos] = sorted[i];
      z.group[pos] = g;
    }
  }
  // node -> zone index; the groups of neighbouring zone nodes differ by at
  // most one (levels of a breadth-first search, merged in runs)
  std::fill(z.zmap_h.begin(), z.zmap_h.end(), -1);
  for (int64_t i = 0; i < z.nz; ++i) z.zmap_h[z.nodes[i]] = (int32_t)i;
  for (int64_t i = 0; i < z.nz; ++i)
    for (int32_t p = z.nbr_ptr[z.nodes[i]]; p < z.nbr_ptr[z.nodes[i] + 1]; ++p) {
      const int32_t q = z.zmap_h[z.nbr[p]];
      if (q >= 0 && std::abs(z.group[q] - z.group[i]) > 1) {
        msg = "process zone: neighbouring nodes more than one level apart";
        return hipErrorUnknown;
      }
    }
  // the halo: zone nodes and their neighbours
  std::vector<int32_t> halo;
  std::vector<uint8_t> inh(nn, 0);
  for (int32_t a : z.nodes)
    for (int32_t p = z.nbr_ptr[a]; p < z.nbr_ptr[a + 1]; ++p) inh[z.nbr[p]] = 1;
  for (int64_t a = 0; a < nn; ++a)
    if (inh[a]) halo.push_back((int32_t)a);
  z.nh = (int64_t)halo.size();
  const int64_t np = z.poff[z.L], nq = z.qoff[z.L];
  if (z.nz > z.cap_nodes || z.nh > z.cap_halo || z.L > z.cap_groups || np > z.cap_p || nq > z.cap_q ||
      z.mmax > z.cap_m) {
    if (!allow_alloc) return hipErrorNotReady;
    // grow the buffers to this zone (kept for later tangents); nothing of an
    // earlier factorisation may still run on stream2 when they are freed
    if ((e = hipStreamSynchronize(z.stream2))) return e;
    const int64_t capn = std::max(z.nz, z.cap_nodes), caph = std::max(z.nh, z.cap_halo),
                  capg = std::max(z.L, z.cap_groups), capp = std::max(np, z.cap_p), capq = std::max(nq, z.cap_q),
                  capm = std::max(z.mmax, z.cap_m);
    for (void* p : {(void*)z.P, (void*)z.Q, (void*)z.T, (void*)z.ipiv, (void*)z.ipiv2, (void*)z.info, (void*)z.bz,
                    (void*)z.xz, (void*)z.znodes, (void*)z.zgroup, (void*)z.goff_d, (void*)z.poff_d, (void*)z.halo, z.ws,
                    z.ws2})
      dfree(c, p);
    z.P = (double*)dalloc(c, capp * sizeof(double));
    z.T = (double*)dalloc(c, capp * sizeof(double));
    z.Q = (double*)dalloc(c, std::max<int64_t>(capq, 1) * sizeof(double));
    z.ipiv = (rocblas_int*)dalloc(c, capm * sizeof(rocblas_int));
    z.ipiv2 = (rocblas_int*)dalloc(c, capm * sizeof(rocblas_int));
    z.info = (rocblas_int*)dalloc(c, 2 * capg * sizeof(rocblas_int));
    z.bz = (double*)dalloc(c, capn * 4 * sizeof(double));
    z.xz = (double*)dalloc(c, capn * 4 * sizeof(double));
    z.znodes = (int32_t*)dalloc(c, capn * sizeof(int32_t));
    z.zgroup = (int32_t*)dalloc(c, capn * sizeof(int32_t));
    z.goff_d = (int64_t*)dalloc(c, (capg + 1) * sizeof(int64_t));
    z.poff_d = (int64_t*)dalloc(c, (capg + 1) * sizeof(int64_t));
    z.halo = (int32_t*)dalloc(c, caph * sizeof(int32_t));
    // the workspace of getrf / getri / gemm at the largest group, from the
    // context's allocator; at least 64 MiB (with the size the query
    // reported, a factorization of groups above ~1,500 unknowns was refused)
    size_t ws = 0;
    rocblas_start_device_memory_size_query(z.handle);
    (void)rocsolver_dgetrf(z.handle, (rocblas_int)capm, (rocblas_int)capm, nullptr, (rocblas_int)capm, nullptr,
                           nullptr);
    (void)rocsolver_dgetri(z.handle, (rocblas_int)capm, nullptr, (rocblas_int)capm, nullptr, nullptr);
    {
      const double one = 1.0;
      (void)rocblas_dgemm(z.handle, rocblas_operation_none, rocblas_operation_none, (rocblas_int)capm,
                          (rocblas_int)capm, (rocblas_int)capm, &one, nullptr, (rocblas_int)capm, nullptr,
                          (rocblas_int)capm, &one, nullptr, (rocblas_int)capm);
    }
    rocblas_stop_device_memory_size_query(z.handle, &ws);
    z.ws_size = std::max<size_t>(ws, (size_t)64 << 20);
    z.ws = dalloc(c, z.ws_size);
    z.ws2 = dalloc(c, z.ws_size);
    if (!z.P || !z.Q || !z.T || !z.ipiv || !z.ipiv2 || !z.ws2 || !z.info || !z.bz || !z.xz || !z.znodes || !z.zgroup || !z.goff_d || !z.poff_d ||
        !z.halo || !z.ws) {
      z.cap_nodes = z.cap_halo = z.cap_groups = z.cap_p = z.cap_q = z.cap_m = 0;
      msg = "device allocation failed (process zone factors)";
      return hipErrorOutOfMemory;
    }
    if ((e = rb_err(rocblas_set_workspace(z.handle, z.ws, z.ws_size), "rocblas_set_workspace", msg)) ||
        (e = rb_err(rocblas_set_workspace(z.handle2, z.ws2, z.ws_size), "rocblas_set_workspace", msg)))
      return e;
    z.cap_nodes = capn;
    z.cap_halo = caph;
    z.cap_groups = capg;
    z.cap_p = capp;
    z.cap_q = capq;
    z.cap_m = capm;
  }
  if ((e = hipMemcpyAsync(z.zmap, z.zmap_h.data(), nn * 4, hipMemcpyHostToDevice, c->stream)) ||
      (e = hipMemcpyAsync(z.znodes, z.nodes.data(), z.nz * 4, hipMemcpyHostToDevice, c->stream)) ||
      (e = hipMemcpyAsync(z.zgroup, z.group.data(), z.nz * 4, hipMemcpyHostToDevice, c->stream)) ||
      (e = hipMemcpyAsync(z.goff_d, z.goff.data(), (z.L + 1) * 8, hipMemcpyHostToDevice, c->stream)) ||
      (e = hipMemcpyAsync(z.poff_d, z.poff.data(), (z.L + 1) * 8, hipMemcpyHostToDevice, c->stream)) ||
      (e = hipMemcpyAsync(z.halo, halo.data(), z.nh * 4, hipMemcpyHostToDevice, c->stream)))
    return e;
  // the panels P_k of the zone's block
  zone_zero_kernel<<<std::min<int64_t>(nblocks(np), 4096), ZBS, 0, c->stream>>>(np, z.P);
  const double se = c->mat.E / c->mat.h;
  const int64_t work = z.nz * c->max_nbr;
  if (c->precision == LGDM_MIXED)
    zone_build_kernel<float><<<nblocks(work), ZBS, 0, c->stream>>>(
        z.nz, c->max_nbr, z.znodes, z.zmap, z.zgroup, z.goff_d, z.poff_d, c->row_ptr, c->nbr_ptr, c->nbr, c->vals32,
        se, z.P);
  else
    zone_build_kernel<double><<<nblocks(work), ZBS, 0, c->stream>>>(
        z.nz, c->max_nbr, z.znodes, z.zmap, z.zgroup, z.goff_d, z.poff_d, c->row_ptr, c->nbr_ptr, c->nbr, c->vals,
        se, z.P);
  if ((e = hipGetLastError())) return e;
  // twisted block LU: the chain from group 0 up to the middle group c on the
  // context's stream, the chain from group L-1 down to c on stream2, then c
  const double one = 1.0, mone = -1.0, zero = 0.0;
  const int64_t NG = z.L, mid = z.L / 2;
  auto gsize = [&](int64_t k) { return k >= 0 && k < NG ? z.goff[k + 1] - z.goff[k] : (int64_t)0; };
  // group k's panel pieces: Z_k,k-1 | Z_kk (-> G_k) | Z_k,k+1, and P_k | N_k
  auto Zprev = [&](int64_t k) { return z.P + z.poff[k]; };
  auto Zdiag = [&](int64_t k) { return z.P + z.poff[k] + gsize(k) * gsize(k - 1); };
  auto Znext = [&](int64_t k) { return z.P + z.poff[k] + gsize(k) * (gsize(k - 1) + gsize(k)); };
  auto Pk = [&](int64_t k) { return z.Q + z.qoff[k]; };
  auto Nk = [&](int64_t k) { return z.Q + z.qoff[k] + gsize(k) * gsize(k - 1); };
  // S_k -= Z_k,j X (X: m_j x m_k, the neighbour j's P or N), then G_k, P_k, N_k
  auto factor_group = [&](rocblas_handle h, rocblas_int* piv, int64_t k, bool from_prev, bool from_next,
                          std::string& msg) {
    const rocblas_int im = (rocblas_int)gsize(k), imp = (rocblas_int)gsize(k - 1), imn = (rocblas_int)gsize(k + 1);
    hipError_t r;
    if (from_prev &&
        (r = rb_err(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, im, im, imp, &mone, Zprev(k),
                                  im, Nk(k - 1), imp, &one, Zdiag(k), im),
                    "dgemm (Schur complement)", msg)))
      return r;
    if (from_next &&
        (r = rb_err(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, im, im, imn, &mone, Znext(k),
                                  im, Pk(k + 1), imn, &one, Zdiag(k), im),
                    "dgemm (Schur complement)", msg)))
      return r;
    if ((r = rb_err(rocsolver_dgetrf(h, im, im, Zdiag(k), im, piv, z.info + 2 * k), "dgetrf", msg)) ||
        (r = rb_err(rocsolver_dgetri(h, im, Zdiag(k), im, piv, z.info + 2 * k + 1), "dgetri", msg)))
      return r;
    if (imp > 0 && (r = rb_err(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, im, imp, im, &one,
                                             Zdiag(k), im, Zprev(k), im, &zero, Pk(k), im),
                               "dgemm (P_k)", msg)))
      return r;
    if (imn > 0 && (r = rb_err(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, im, imn, im, &one,
                                             Zdiag(k), im, Znext(k), im, &zero, Nk(k), im),
                               "dgemm (N_k)", msg)))
      return r;
    return hipSuccess;
  };
  if ((e = hipEventRecord(z.ev_built, c->stream)) || (e = hipStreamWaitEvent(z.stream2, z.ev_built, 0))) return e;
  // each chain is thousands of short rocSOLVER launches, so one host thread
  // issuing both is bound by its launch rate: the bottom chain is issued
  // from a second thread (HIP's current device is per thread)
  hipError_t e2 = hipSuccess;
  std::string msg2;
  auto bottom_chain = [&] {
    e2 = hipSetDevice(c->device);
    for (int64_t k = NG - 1; k > mid && e2 == hipSuccess; --k)
      e2 = factor_group(z.handle2, z.ipiv2, k, false, k < NG - 1, msg2);
    if (e2 == hipSuccess) e2 = hipEventRecord(z.ev_chain2, z.stream2);
  };
  std::thread chain2;
  try {
    chain2 = std::thread(bottom_chain);
  } catch (...) {
    bottom_chain();   // no thread available: the same launches from this one
  }
  for (int64_t k = 0; k < mid && e == hipSuccess; ++k) e = factor_group(z.handle, z.ipiv, k, k > 0, false, msg);
  if (chain2.joinable()) chain2.join();
  if (e || e2) {
    // the other chain's launches may still run: finish them before the
    // buffers can be freed or refilled
    (void)hipStreamSynchronize(z.stream2);
    (void)hipStreamSynchronize(c->stream);
    if (e) return e;
    msg = msg2;
    return e2;
  }
  if ((e = hipStreamWaitEvent(c->stream, z.ev_chain2, 0))) return e;
  if ((e = factor_group(z.handle, z.ipiv, mid, mid > 0, mid < NG - 1, msg))) return e;
  // the sweeps read rows of [G_k | P_k | N_k] in row-major order, in FP32
  // in mixed contexts (the matrix values there are FP32 too)
  z.t32 = c->precision == LGDM_MIXED;
  for (int64_t k = 0; k < NG; ++k) {
    const int64_t m = gsize(k), mp = gsize(k - 1), mn = gsize(k + 1), lda = m + mp + mn;
    if (z.t32) {
      float* Tk = reinterpret_cast<float*>(z.T) + z.poff[k];
      zone_rowmajor_kernel<float><<<nblocks(m * m), ZBS, 0, c->stream>>>(m, m, Zdiag(k), Tk, lda, 0);
      if (mp > 0) zone_rowmajor_kernel<float><<<nblocks(m * mp), ZBS, 0, c->stream>>>(m, mp, Pk(k), Tk, lda, m);
      if (mn > 0)
        zone_rowmajor_kernel<float><<<nblocks(m * mn), ZBS, 0, c->stream>>>(m, mn, Nk(k), Tk, lda, m + mp);
    } else {
      double* Tk = z.T + z.poff[k];
      zone_rowmajor_kernel<double><<<nblocks(m * m), ZBS, 0, c->stream>>>(m, m, Zdiag(k), Tk, lda, 0);
      if (mp > 0) zone_rowmajor_kernel<double><<<nblocks(m * mp), ZBS, 0, c->stream>>>(m, mp, Pk(k), Tk, lda, m);
      if (mn > 0)
        zone_rowmajor_kernel<double><<<nblocks(m * mn), ZBS, 0, c->stream>>>(m, mn, Nk(k), Tk, lda, m + mp);
    }
  }
  if ((e = hipGetLastError())) return e;
  std::vector<rocblas_int> info(2 * z.L, 0);
  if ((e = hipMemcpyAsync(info.data(), z.info, info.size() * sizeof(rocblas_int), hipMemcpyDeviceToHost,
                          c->stream)) ||
      (e = hipStreamSynchronize(c->stream)))
    return e;
  *factored = true;
  // an exactly singular group leaves the plain cycle
  z.active = std::all_of(info.begin(), info.end(), [](rocblas_int v) { return v == 0; });
  if (z.active) {
    z.built_nodes.swap(sorted);
    z.built_serial = c->in_increment ? c->inc_serial : -1;
  }
  return hipSuccess;
}

bool zone_active(const lgdm_ctx* c) { return c->zone && c->zone->active; }

void zone_disable(lgdm_ctx* c) {
  if (c->zone) c->zone->active = false;
}

void zone_forget(lgdm_ctx* c) {
  if (c->zone) c->zone->built_serial = -1;
}

int64_t zone_dofs(const lgdm_ctx* c) { return zone_active(c) ? c->zone->nz * 4 : 0; }

// out = x_z + M_mg (b - S K x_z), x_z = Z^-1 b_z
hipError_t zone_apply(lgdm_ctx* c, const double* b, double* out, const double* sc, hipStream_t st) {
  Zone& z = *c->zone;
  const int64_t n = z.nz * 4;
  // the layout must describe the buffers the factors were built in
  if ((int64_t)z.goff.size() != z.L + 1 || (int64_t)z.poff.size() != z.L + 1 || z.goff.back() != n ||
      z.nz > z.cap_nodes || z.nh > z.cap_halo || z.poff[z.L] > z.cap_p || z.L > z.cap_groups)
    return hipErrorInvalidValue;
  zone_gather_kernel<<<nblocks(n), ZBS, 0, st>>>(z.nz, z.znodes, b, z.bz, sc);
  // twisted sweeps: both ends toward the middle group, then back out; the
  // two groups of a step share one launch
  const int64_t L = z.L, mid = z.L / 2;
  auto gsize = [&](int64_t k) { return k >= 0 && k < L ? z.goff[k + 1] - z.goff[k] : (int64_t)0; };
  // y_k (+)= G_k u - P_k v - N_k w over group k's rows
  auto op = [&](int64_t k, const double* u, const double* v, const double* w, int accumulate) {
    const int64_t m = gsize(k), mp = gsize(k - 1), mn = gsize(k + 1);
    SweepOp o;
    o.m = m;
    o.lda = m + mp + mn;
    o.A = z.t32 ? (const void*)(reinterpret_cast<const float*>(z.T) + z.poff[k]) : (const void*)(z.T + z.poff[k]);
    o.u = u;
    o.nu = u ? m : 0;
    o.v = v;
    o.nv = v ? mp : 0;
    o.op = m;
    o.w = w;
    o.nw = w ? mn : 0;
    o.on = m + mp;
    o.y = z.xz + z.goff[k];
    o.accumulate = accumulate;
    return o;
  };
  auto launch = [&](const SweepOp* a, const SweepOp* b) {
    const SweepOp& first = a ? *a : *b;
    const SweepOp& second = a && b ? *b : first;
    const unsigned na = sweep_blocks(first), nb = a && b ? sweep_blocks(second) : 0;
    if (z.t32) zone_sweep_kernel<float><<<na + nb, ZBS, 0, st>>>(first, second, na, sc);
    else zone_sweep_kernel<double><<<na + nb, ZBS, 0, st>>>(first, second, na, sc);
  };
  const int64_t steps = std::max(mid, L - 1 - mid);
  auto xz_at = [&](int64_t k) { return (const double*)(z.xz + z.goff[k]); };
  for (int64_t s = 0; s < steps; ++s) {
    SweepOp a, b;
    const bool ha = s < mid, hb = L - 1 - s > mid;
    if (ha) a = op(s, z.bz + z.goff[s], s > 0 ? xz_at(s - 1) : nullptr, nullptr, 0);
    if (hb) b = op(L - 1 - s, z.bz + z.goff[L - 1 - s], nullptr, L - 1 - s < L - 1 ? xz_at(L - s) : nullptr, 0);
    launch(ha ? &a : nullptr, hb ? &b : nullptr);
  }
  {
    SweepOp m = op(mid, z.bz + z.goff[mid], mid > 0 ? xz_at(mid - 1) : nullptr,
                   mid < L - 1 ? xz_at(mid + 1) : nullptr, 0);
    launch(&m, nullptr);
  }
  for (int64_t s = 0; s < steps; ++s) {
    SweepOp a, b;
    const bool ha = mid - 1 - s >= 0, hb = mid + 1 + s <= L - 1;
    if (ha) a = op(mid - 1 - s, nullptr, nullptr, xz_at(mid - s), 1);
    if (hb) b = op(mid + 1 + s, nullptr, xz_at(mid + s), nullptr, 1);
    launch(ha ? &a : nullptr, hb ? &b : nullptr);
  }
  zone_copy_kernel<<<std::min<int64_t>(nblocks(c->ndof), 2048), ZBS, 0, st>>>(c->ndof, b, z.r, sc);
  const double se = c->mat.E / c->mat.h;
  if (c->precision == LGDM_MIXED)
    zone_residual_kernel<float><<<nblocks(z.nh * RES_G), ZBS, 0, st>>>(z.nh, z.halo, z.zmap, c->row_ptr, c->nbr_ptr,
                                                                   c->nbr, c->vals32, se, b, z.xz, z.r, sc);
  else
    zone_residual_kernel<double><<<nblocks(z.nh * RES_G), ZBS, 0, st>>>(z.nh, z.halo, z.zmap, c->row_ptr, c->nbr_ptr,
                                                                    c->nbr, c->vals, se, b, z.xz, z.r, sc);
  hipError_t e;
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = amg_cycle(c, z.r, out, sc, st)) != hipSuccess) return e;
  zone_scatter_kernel<<<nblocks(n), ZBS, 0, st>>>(z.nz, z.znodes, z.xz, out, sc);
  return hipGetLastError();
}

}  // namespace lgdm

extern "C" lgdm_status lgdm_zone_levels(int64_t n, const int32_t* ptr, const int32_t* adj, int32_t* level,
                                        int64_t* n_levels) {
  if (n < 0 || !ptr || !level || !n_levels || (n > 0 && !adj && ptr[n] > 0)) return LGDM_ERR_INVALID_ARG;
  if (ptr[0] != 0) return LGDM_ERR_INVALID_ARG;
  for (int64_t a = 0; a < n; ++a) {
    if (ptr[a + 1] < ptr[a]) return LGDM_ERR_INVALID_ARG;
    for (int32_t p = ptr[a]; p < ptr[a + 1]; ++p)
      if (adj[p] < 0 || adj[p] >= n) return LGDM_ERR_INVALID_ARG;
  }
  std::vector<int64_t> P(ptr, ptr + n + 1);
  *n_levels = lgdm::zone_levels(n, P.data(), adj, level);
  return LGDM_OK;
}
