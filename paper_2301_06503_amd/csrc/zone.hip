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
//   zone   nodes of the elements with a Gauss point that is loading and has
//          trial damage D >= zone_damage (0.999 by default; moved tenfold
//          closer to 1, twice at most, while the zone exceeds ZONE_MAX_DOFS
//          unknowns), chosen afresh for every tangent
//   Z      the zone's principal block of S K, dense (column major), factored
//          by LU with partial pivoting and inverted (rocSOLVER getrf, getri)
//   apply  x_z = Z^-1 b_z; r = b - S K x_z (only rows of the zone and its
//          neighbour nodes change); out = x_z + M_mg r, with M_mg the
//          multigrid cycle (multiplicative: a CPU model on the 128x32x16
//          beam after its peak, zone from D >= 0.99, needed 64 GMRES steps
//          with it, 97 with the additive form x_z + M_mg b, and more than
//          3000 without a zone)
//
// Within one Newton increment a tangent whose zone has the same nodes as the
// one last factored keeps that inverse: the zone's block changes little
// between Newton iterates, while its factorization costs far more than a
// solve.  The apply is a fixed linear map for the whole solve, so IDR(s)
// takes it as its preconditioner unchanged.  Every sum has a fixed order.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "lgdm_internal.h"

namespace lgdm {

struct Zone {
  // host copies of the mesh structure (taken at the first setup)
  std::vector<int32_t> conn, nbr_ptr, nbr;
  std::vector<uint8_t> eflag;
  std::vector<int32_t> zmap_h;              // node -> zone node, -1 outside
  // device
  uint8_t* eflag_d = nullptr;               // [n_elems]
  int32_t* zmap = nullptr;                  // [n_nodes]
  int32_t* znodes = nullptr;                // [cap_nodes]
  int32_t* halo = nullptr;                  // nodes whose rows r = b - S K x_z changes [cap_halo]
  double* Z = nullptr;                      // [cap_dofs * cap_dofs]
  rocblas_int* ipiv = nullptr;              // [cap_dofs]
  rocblas_int* info = nullptr;              // [1]
  double* bz = nullptr;                     // [cap_dofs] b at the zone's dofs
  double* xz = nullptr;                     // [cap_dofs] Z^-1 b_z
  double* r = nullptr;                      // [ndof]
  int64_t cap_dofs = 0, cap_halo = 0;
  void* ws = nullptr;
  size_t ws_size = 0;
  rocblas_handle handle = nullptr;
  int64_t nz = 0, nh = 0;                   // zone nodes, halo nodes of the current tangent
  bool active = false;
  double damage = 0.0;                      // threshold the current zone was chosen with
  // the zone whose inverse Z holds: its nodes and the increment it was built in
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

// Z[(4 za + i) + (4 zq + j) ld] = (S K)_{4a+i, 4q+j} for zone nodes a, q;
// one thread per (zone node, neighbour position)
template <typename T>
__global__ void zone_build_kernel(int64_t nz, int max_nbr, const int32_t* __restrict__ znodes,
                                  const int32_t* __restrict__ zmap, const int32_t* __restrict__ row_ptr,
                                  const int32_t* __restrict__ nbr_ptr, const int32_t* __restrict__ nbr,
                                  const T* __restrict__ vals, double se, int64_t ld, double* __restrict__ Z) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nz * max_nbr) return;
  const int64_t za = t / max_nbr;
  const int p = (int)(t % max_nbr);
  const int64_t a = znodes[za];
  const int nb0 = nbr_ptr[a], nnb = nbr_ptr[a + 1] - nb0;
  if (p >= nnb) return;
  const int32_t zq = zmap[nbr[nb0 + p]];
  if (zq < 0) return;
  const int64_t rowlen = (int64_t)nnb * 4, rb = row_ptr[a * 4];
  for (int i = 0; i < 4; ++i) {
    const double s = i == 3 ? se : 1.0;
    for (int j = 0; j < 4; ++j)
      Z[(4 * za + i) + (4 * (int64_t)zq + j) * ld] = s * (double)vals[rb + i * rowlen + (int64_t)p * 4 + j];
  }
}

// bz = b at the zone's dofs
__global__ void zone_gather_kernel(int64_t nz, const int32_t* __restrict__ znodes, const double* __restrict__ b,
                                   double* __restrict__ bz, const double* __restrict__ sc) {
  if (sc && sc[KSLOT_DONE] != 0.0) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nz * 4) return;
  bz[t] = b[(int64_t)znodes[t / 4] * 4 + (t % 4)];
}

// r = b everywhere (the halo rows are overwritten next)
__global__ void zone_copy_kernel(int64_t n, const double* __restrict__ b, double* __restrict__ r,
                                 const double* __restrict__ sc) {
  if (sc && sc[KSLOT_DONE] != 0.0) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    r[i] = b[i];
}

// r_h = b_h - sum over zone neighbours q of (S K)_{hq} x_z(q), rows of the
// halo nodes (neighbour order: fixed); one thread per (halo node, row)
template <typename T>
__global__ void zone_residual_kernel(int64_t nh, const int32_t* __restrict__ halo, const int32_t* __restrict__ zmap,
                                     const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ nbr_ptr,
                                     const int32_t* __restrict__ nbr, const T* __restrict__ vals, double se,
                                     const double* __restrict__ b, const double* __restrict__ xz,
                                     double* __restrict__ r, const double* __restrict__ sc) {
  if (sc && sc[KSLOT_DONE] != 0.0) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nh * 4) return;
  const int64_t h = halo[t / 4];
  const int i = (int)(t % 4);
  const int nb0 = nbr_ptr[h], nnb = nbr_ptr[h + 1] - nb0;
  const int64_t rowlen = (int64_t)nnb * 4, rs = row_ptr[h * 4] + i * rowlen;
  double acc = 0.0;
  for (int p = 0; p < nnb; ++p) {
    const int32_t zq = zmap[nbr[nb0 + p]];
    if (zq < 0) continue;
    for (int j = 0; j < 4; ++j) acc += (double)vals[rs + (int64_t)p * 4 + j] * xz[4 * (int64_t)zq + j];
  }
  const int64_t row = h * 4 + i;
  r[row] = b[row] - (i == 3 ? se : 1.0) * acc;
}

// out += x_z at the zone's dofs
__global__ void zone_scatter_kernel(int64_t nz, const int32_t* __restrict__ znodes, const double* __restrict__ xz,
                                    double* __restrict__ out, const double* __restrict__ sc) {
  if (sc && sc[KSLOT_DONE] != 0.0) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nz * 4) return;
  out[(int64_t)znodes[t / 4] * 4 + (t % 4)] += xz[t];
}

inline unsigned nblocks(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + ZBS - 1) / ZBS); }

hipError_t rb_err(rocblas_status s) { return s == rocblas_status_success ? hipSuccess : hipErrorUnknown; }

}  // namespace

void zone_release(lgdm_ctx* c) {
  if (!c->zone) return;
  if (c->zone->handle) (void)rocblas_destroy_handle(c->zone->handle);
  delete c->zone;
  c->zone = nullptr;
}

// Choose the zone of the current tangent and factor its block.  Leaves the
// zone inactive (plain multigrid) where there is none or it does not fit.
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
    z.info = (rocblas_int*)dalloc(c, 64);
    if (!z.eflag_d || !z.zmap || !z.r || !z.info) {
      msg = "device allocation failed (process zone)";
      return hipErrorOutOfMemory;
    }
    if (rocblas_create_handle(&z.handle) != rocblas_status_success) {
      msg = "rocblas_create_handle failed";
      return hipErrorUnknown;
    }
  }
  if (rocblas_set_stream(z.handle, c->stream) != rocblas_status_success) return hipErrorUnknown;
  // the zone: raise the damage threshold until it fits
  std::vector<int32_t> znodes, halo;
  for (double dmin : {dmin0, 1.0 - 0.1 * (1.0 - dmin0), 1.0 - 0.01 * (1.0 - dmin0)}) {
    zone_flag_kernel<<<nblocks(ne), ZBS, 0, c->stream>>>(ne, c->ngp, c->kappa_t, c->kappa_n, c->D_t,
                                                         c->mat.tol_hist, dmin, z.eflag_d);
    if ((e = hipMemcpyAsync(z.eflag.data(), z.eflag_d, ne, hipMemcpyDeviceToHost, c->stream)) ||
        (e = hipStreamSynchronize(c->stream)))
      return e;
    znodes.clear();
    for (int64_t el = 0; el < ne; ++el)
      if (z.eflag[el])
        for (int a = 0; a < c->nen; ++a) znodes.push_back(z.conn[el * c->nen + a]);
    std::sort(znodes.begin(), znodes.end());
    znodes.erase(std::unique(znodes.begin(), znodes.end()), znodes.end());
    z.damage = dmin;
    if ((int64_t)znodes.size() * 4 <= ZONE_MAX_DOFS) break;
  }
  z.nz = (int64_t)znodes.size();
  if (z.nz == 0 || z.nz * 4 > ZONE_MAX_DOFS) return hipSuccess;
  // a later tangent of the same increment with the same zone keeps the
  // inverse (the halo residual and the cycle read the current tangent)
  if (reuse && c->in_increment && z.built_serial == c->inc_serial && znodes == z.built_nodes) {
    z.active = true;
    return hipSuccess;
  }
  z.built_serial = -1;
  // node -> zone index, and the halo: zone nodes and their neighbours
  std::fill(z.zmap_h.begin(), z.zmap_h.end(), -1);
  for (int64_t i = 0; i < z.nz; ++i) z.zmap_h[znodes[i]] = (int32_t)i;
  std::vector<uint8_t> inh(nn, 0);
  for (int32_t a : znodes)
    for (int32_t p = z.nbr_ptr[a]; p < z.nbr_ptr[a + 1]; ++p) inh[z.nbr[p]] = 1;
  for (int64_t a = 0; a < nn; ++a)
    if (inh[a]) halo.push_back((int32_t)a);
  z.nh = (int64_t)halo.size();
  const int64_t n = z.nz * 4;
  if (n > z.cap_dofs || z.nh > z.cap_halo) {
    if (!allow_alloc) return hipErrorNotReady;
    // grow the buffers to this zone (kept for later tangents)
    const int64_t cap = std::max<int64_t>(n, z.cap_dofs), caph = std::max<int64_t>(z.nh, z.cap_halo);
    dfree(c, z.Z);
    dfree(c, z.ipiv);
    dfree(c, z.bz);
    dfree(c, z.xz);
    dfree(c, z.znodes);
    dfree(c, z.halo);
    dfree(c, z.ws);
    z.Z = (double*)dalloc(c, (size_t)cap * cap * sizeof(double));
    z.ipiv = (rocblas_int*)dalloc(c, cap * sizeof(rocblas_int));
    z.bz = (double*)dalloc(c, cap * sizeof(double));
    z.xz = (double*)dalloc(c, cap * sizeof(double));
    z.znodes = (int32_t*)dalloc(c, (cap / 4) * sizeof(int32_t));
    z.halo = (int32_t*)dalloc(c, caph * sizeof(int32_t));
    // rocSOLVER's workspace for getrf / getrs at this size, from the context's allocator
    size_t ws = 0;
    rocblas_start_device_memory_size_query(z.handle);
    (void)rocsolver_dgetrf(z.handle, (rocblas_int)cap, (rocblas_int)cap, nullptr, (rocblas_int)cap, nullptr, nullptr);
    (void)rocsolver_dgetri(z.handle, (rocblas_int)cap, nullptr, (rocblas_int)cap, nullptr, nullptr);
    rocblas_stop_device_memory_size_query(z.handle, &ws);
    z.ws_size = std::max<size_t>(ws, 256);
    z.ws = dalloc(c, z.ws_size);
    if (!z.Z || !z.ipiv || !z.bz || !z.xz || !z.znodes || !z.halo || !z.ws) {
      z.cap_dofs = z.cap_halo = 0;
      msg = "device allocation failed (process zone block)";
      return hipErrorOutOfMemory;
    }
    if (rocblas_set_workspace(z.handle, z.ws, z.ws_size) != rocblas_status_success) return hipErrorUnknown;
    z.cap_dofs = cap;
    z.cap_halo = caph;
  }
  if ((e = hipMemcpyAsync(z.zmap, z.zmap_h.data(), nn * 4, hipMemcpyHostToDevice, c->stream)) ||
      (e = hipMemcpyAsync(z.znodes, znodes.data(), z.nz * 4, hipMemcpyHostToDevice, c->stream)) ||
      (e = hipMemcpyAsync(z.halo, halo.data(), z.nh * 4, hipMemcpyHostToDevice, c->stream)))
    return e;
  // the dense block, leading dimension n
  zone_zero_kernel<<<std::min<int64_t>(nblocks(n * n), 4096), ZBS, 0, c->stream>>>(n * n, z.Z);
  const double se = c->mat.E / c->mat.h;
  const int64_t work = z.nz * c->max_nbr;
  if (c->precision == LGDM_MIXED)
    zone_build_kernel<float><<<nblocks(work), ZBS, 0, c->stream>>>(z.nz, c->max_nbr, z.znodes, z.zmap, c->row_ptr,
                                                                   c->nbr_ptr, c->nbr, c->vals32, se, n, z.Z);
  else
    zone_build_kernel<double><<<nblocks(work), ZBS, 0, c->stream>>>(z.nz, c->max_nbr, z.znodes, z.zmap, c->row_ptr,
                                                                    c->nbr_ptr, c->nbr, c->vals, se, n, z.Z);
  if ((e = hipGetLastError())) return e;
  if ((e = rb_err(rocsolver_dgetrf(z.handle, (rocblas_int)n, (rocblas_int)n, z.Z, (rocblas_int)n, z.ipiv, z.info))))
    return e;
  rocblas_int info = 0;
  if ((e = hipMemcpyAsync(&info, z.info, sizeof(info), hipMemcpyDeviceToHost, c->stream)) ||
      (e = hipStreamSynchronize(c->stream)))
    return e;
  if (info != 0) return hipSuccess;  // an exactly singular block leaves the plain cycle
  // the explicit inverse: each application is then one pass over it (a
  // matrix-vector product), where two triangular solves with one right-hand
  // side are latency-bound
  if ((e = rb_err(rocsolver_dgetri(z.handle, (rocblas_int)n, z.Z, (rocblas_int)n, z.ipiv, z.info)))) return e;
  if ((e = hipMemcpyAsync(&info, z.info, sizeof(info), hipMemcpyDeviceToHost, c->stream)) ||
      (e = hipStreamSynchronize(c->stream)))
    return e;
  z.active = info == 0;  // an exactly singular block leaves the plain cycle
  *factored = true;
  if (z.active) {
    z.built_nodes.swap(znodes);
    z.built_serial = c->in_increment ? c->inc_serial : -1;
  }
  return hipSuccess;
}

bool zone_active(const lgdm_ctx* c) { return c->zone && c->zone->active; }

void zone_disable(lgdm_ctx* c) {
  if (c->zone) c->zone->active = false;
}

int64_t zone_dofs(const lgdm_ctx* c) { return zone_active(c) ? c->zone->nz * 4 : 0; }

// out = x_z + M_mg (b - S K x_z), x_z = Z^-1 b_z
hipError_t zone_apply(lgdm_ctx* c, const double* b, double* out, const double* sc, hipStream_t st) {
  Zone& z = *c->zone;
  const int64_t n = z.nz * 4;
  zone_gather_kernel<<<nblocks(n), ZBS, 0, st>>>(z.nz, z.znodes, b, z.bz, sc);
  if (st != c->stream) (void)rocblas_set_stream(z.handle, st);
  const double one = 1.0, zero = 0.0;
  hipError_t e = rb_err(rocblas_dgemv(z.handle, rocblas_operation_none, (rocblas_int)n, (rocblas_int)n, &one, z.Z,
                                      (rocblas_int)n, z.bz, 1, &zero, z.xz, 1));
  if (st != c->stream) (void)rocblas_set_stream(z.handle, c->stream);
  if (e != hipSuccess) return e;
  zone_copy_kernel<<<std::min<int64_t>(nblocks(c->ndof), 2048), ZBS, 0, st>>>(c->ndof, b, z.r, sc);
  const double se = c->mat.E / c->mat.h;
  if (c->precision == LGDM_MIXED)
    zone_residual_kernel<float><<<nblocks(z.nh * 4), ZBS, 0, st>>>(z.nh, z.halo, z.zmap, c->row_ptr, c->nbr_ptr,
                                                                   c->nbr, c->vals32, se, b, z.xz, z.r, sc);
  else
    zone_residual_kernel<double><<<nblocks(z.nh * 4), ZBS, 0, st>>>(z.nh, z.halo, z.zmap, c->row_ptr, c->nbr_ptr,
                                                                    c->nbr, c->vals, se, b, z.xz, z.r, sc);
  if ((e = amg_cycle(c, z.r, out, sc, st)) != hipSuccess) return e;
  zone_scatter_kernel<<<nblocks(n), ZBS, 0, st>>>(z.nz, z.znodes, z.xz, out, sc);
  return hipGetLastError();
}

}  // namespace lgdm
