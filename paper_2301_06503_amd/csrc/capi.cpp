// C ABI of the LGDM library and the incremental-iterative Newton driver
// (Algorithm 2; H7): argument checks, device memory, the increment state
// machine, convergence test, commit of the history variable and queries.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lgdm_internal.h"

using namespace lgdm;

namespace lgdm {

void* dalloc(lgdm_ctx* c, size_t bytes) {
  if (bytes == 0) bytes = 1;
  bytes = (bytes + 255) & ~(size_t)255;
  void* p = nullptr;
  if (c->alloc_fn) {
    p = c->alloc_fn(bytes, c->alloc_user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  if (p) c->allocs.emplace_back(p, bytes);
  return p;
}

void dfree(lgdm_ctx* c, void* p) {
  if (!p) return;
  for (size_t i = 0; i < c->allocs.size(); ++i)
    if (c->allocs[i].first == p) {
      c->allocs.erase(c->allocs.begin() + i);
      break;
    }
  if (c->free_fn) c->free_fn(p, c->alloc_user);
  else (void)hipFree(p);
}

namespace {

// move finished event pairs into the sum (block: wait for all)
void probe_harvest(KernelProbe& p, bool block) {
  size_t i = 0;
  for (; i < p.pending.size(); ++i) {
    auto& pr = p.pending[i];
    if (block) {
      if (hipEventSynchronize(pr.second) != hipSuccess) break;
    } else if (hipEventQuery(pr.second) != hipSuccess) {
      (void)hipGetLastError();
      break;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
      p.sum_ms += ms;
      p.count += 1;
    }
    p.pool.push_back(pr.first);
    p.pool.push_back(pr.second);
  }
  p.pending.erase(p.pending.begin(), p.pending.begin() + i);
}

void probe_release(lgdm_ctx* c) {
  if (!c->probe) return;
  probe_harvest(*c->probe, true);
  for (auto& pr : c->probe->pending) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  for (auto e : c->probe->pool) (void)hipEventDestroy(e);
  delete c->probe;
  c->probe = nullptr;
}

}  // namespace

void probe_before(lgdm_ctx* c, int kind, hipStream_t st) {
  KernelProbe* p = c->probe;
  if (!p || p->kind != kind) return;
  probe_harvest(*p, false);
  if (p->pool.size() < 2) return;  // all pairs in flight: this launch is not sampled
  p->open1 = p->pool.back();
  p->pool.pop_back();
  p->open0 = p->pool.back();
  p->pool.pop_back();
  if (hipEventRecord(p->open0, st) != hipSuccess) {
    p->pool.push_back(p->open0);
    p->pool.push_back(p->open1);
    p->open0 = p->open1 = nullptr;
  }
}

void probe_after(lgdm_ctx* c, int kind, hipStream_t st) {
  KernelProbe* p = c->probe;
  if (!p || p->kind != kind || !p->open0) return;
  if (hipEventRecord(p->open1, st) == hipSuccess) {
    p->pending.emplace_back(p->open0, p->open1);
  } else {
    p->pool.push_back(p->open0);
    p->pool.push_back(p->open1);
  }
  p->open0 = p->open1 = nullptr;
}

}  // namespace lgdm

namespace {

lgdm_status fail(lgdm_ctx* c, lgdm_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

lgdm_status hip_fail(lgdm_ctx* c, hipError_t e, const char* where) {
  return fail(c, LGDM_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHECK(c, expr, where)                 \
  do {                                           \
    hipError_t e_ = (expr);                      \
    if (e_ != hipSuccess) return hip_fail(c, e_, where); \
  } while (0)

void free_mesh(lgdm_ctx* c) {
  amg_release(c);
  zone_release(c);
  c->amg_unavailable = false;
  // keep pinned host buffers; release every device allocation
  std::vector<std::pair<void*, size_t>> all = c->allocs;
  for (auto& a : all) dfree(c, a.first);
  c->allocs.clear();
  c->coords = nullptr; c->conn = nullptr; c->e_scale = nullptr;
  c->n2e_ptr = c->n2e = c->nbr_ptr = c->nbr = c->dpos = nullptr;
  c->pos = nullptr; c->row_ptr = c->col_idx = nullptr;
  c->dof_flags = nullptr; c->bc_dofs = nullptr; c->bc_vals = nullptr; c->nbc = 0;
  c->x = c->x_save = c->kappa_n = c->D_n = c->kappa_t = c->D_t = c->eeq_t = nullptr;
  c->rec = c->vals = c->R = c->partials = c->norms_dev = c->red2 = nullptr;
  c->vals32 = nullptr;
  c->kv = nullptr; c->minv = nullptr; c->minv32 = nullptr;
  c->kpart = nullptr; c->kscal = nullptr; c->kcount = nullptr; c->delta = nullptr;
  c->dim = 0;
  c->assembled = false;
  c->in_increment = false;
}

bool ready(lgdm_ctx* c) { return c && c->dim > 0 && c->has_mat; }

hipError_t zero(lgdm_ctx* c, void* p, size_t bytes) { return hipMemsetAsync(p, 0, bytes, c->stream); }

// Gauss-point kernel + node-row assembly + norm reduction, then read the
// norms back (the only host synchronisation of an assembly)
lgdm_status assemble_now(lgdm_ctx* c, float* ms) {
  const MatParams mp = make_params(c->mat, c->dim);
  if (ms) HIPCHECK(c, hipEventRecord(c->ev[0], c->stream), "event");
  HIPCHECK(c, launch_gp_kernel(c, mp), "gauss-point kernel");
  HIPCHECK(c, launch_node_kernel(c, mp, true), "assembly kernel");
  HIPCHECK(c, launch_norm_reduce(c), "norm reduction");
  if (ms) HIPCHECK(c, hipEventRecord(c->ev[1], c->stream), "event");
  HIPCHECK(c, hipMemcpyAsync(c->norms_host, c->norms_dev, NORM_SLOTS * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream), "norm readback");
  HIPCHECK(c, hipStreamSynchronize(c->stream), "assembly");
  std::memcpy(c->last_norms, c->norms_host, sizeof(c->last_norms));
  if (ms) HIPCHECK(c, hipEventElapsedTime(ms, c->ev[0], c->ev[1]), "event time");
  c->assembled = true;
  if (c->last_norms[5] != 0.0 || !std::isfinite(c->last_norms[0]) || !std::isfinite(c->last_norms[1]))
    return fail(c, LGDM_ERR_NAN, "non-finite internal force in the assembly");
  return LGDM_OK;
}


void fill_norms(const lgdm_ctx* c, lgdm_increment_report* rep) {
  if (!rep) return;
  rep->res_u = std::sqrt(c->last_norms[0]);
  rep->res_e = std::sqrt(c->last_norms[1]);
  rep->ref_u = std::sqrt(c->last_norms[2]);
  rep->ref_e = std::sqrt(c->last_norms[3]);
  rep->reaction = c->last_norms[4];
}

bool residual_converged(const lgdm_ctx* c, double tol) {
  const double tiny = 1e-300;
  const double ru = std::sqrt(c->last_norms[0]), re = std::sqrt(c->last_norms[1]);
  const double fu = std::sqrt(c->last_norms[2]), fe = std::sqrt(c->last_norms[3]);
  return ru <= tol * std::max(fu, tiny) && re <= tol * std::max(fe, tiny);
}

lgdm_status linear_solve(lgdm_ctx* c, const double* b_dev, double* x_dev, const lgdm_solver_opts& opts,
                         double tol_u, double tol_e, lgdm_increment_report* rep) {
  HIPCHECK(c, krylov_setup(c), "block-Jacobi setup");
  lgdm_solver_opts o = opts;
  if (o.precond == LGDM_PRECOND_DEFAULT)
    o.precond = c->dim == 3 && o.krylov_method == LGDM_KRYLOV_IDRS && !c->amg_unavailable ? LGDM_PRECOND_AMG
                                                                                           : LGDM_PRECOND_BLOCK_JACOBI;
  if (o.precond == LGDM_PRECOND_AMG) {
    if (o.krylov_method != LGDM_KRYLOV_IDRS)
      return fail(c, LGDM_ERR_INVALID_ARG, "the multigrid preconditioner needs IDR(s)");
    std::string msg;
    const hipError_t e = amg_setup(c, msg);
    if (e == hipErrorInvalidValue && opts.precond == LGDM_PRECOND_DEFAULT) {
      // no usable hierarchy for this mesh (too small, or coarsening
      // stalled): the default is block-Jacobi for it from now on
      c->amg_unavailable = true;
      o.precond = LGDM_PRECOND_BLOCK_JACOBI;
    } else if (e != hipSuccess) {
      return msg.empty() ? hip_fail(c, e, "multigrid setup")
                         : fail(c, e == hipErrorInvalidValue ? LGDM_ERR_INVALID_ARG : LGDM_ERR_DEVICE,
                                "multigrid setup: " + msg);
    }
  }
  // the process zone of this tangent, solved densely inside the multigrid cycle
  zone_disable(c);
  const int tier = c->in_increment ? c->inc_zone_tier : 0;
  if (o.precond == LGDM_PRECOND_AMG && o.process_zone != LGDM_ZONE_OFF && tier < 2) {
    std::string msg;
    const double t0 = host_seconds();
    bool factored = false;
    const double dmin = tier == 0 ? o.zone_damage : 1.0 - 0.1 * (1.0 - o.zone_damage);
    const hipError_t e = zone_setup(c, !c->noalloc_call, c->zone_may_reuse && o.process_zone == LGDM_ZONE_DEFAULT,
                                    dmin, &factored, msg);
    if (rep) {
      rep->t_zone_ms += 1e3 * (host_seconds() - t0);
      rep->zone_factorizations += factored ? 1 : 0;
    }
    if (c->in_increment && zone_active(c)) c->inc_zone_used = true;
    if (e == hipErrorNotReady)
      return fail(c, LGDM_ERR_STATE, "the process-zone block of this tangent needs device memory the context has "
                                     "not allocated yet: run lgdm_solve_linear on it first, or turn the zone off");
    if (e == hipErrorUnknown && msg.rfind("process zone:", 0) == 0) {
      // a library call refused the factorization (nothing was launched by
      // it): this solve runs with the plain cycle, the report counts it
      zone_disable(c);
      c->err = msg;
      if (rep) rep->zone_errors += 1;
    } else if (e != hipSuccess) {
      return msg.empty() ? hip_fail(c, e, "process-zone setup") : fail(c, LGDM_ERR_DEVICE, msg);
    }
  }
  KrylovResult kr{};
  HIPCHECK(c, krylov_solve(c, b_dev, x_dev, o, tol_u, tol_e, kr), "Krylov solve");
  const bool out_of_time = c->solve_deadline > 0.0 && host_seconds() > c->solve_deadline;
  if (o.precond == LGDM_PRECOND_AMG && kr.status != LGDM_OK && !kr.improved && kr.iters < o.max_krylov &&
      !out_of_time) {
    // the smoother can amplify where block-Jacobi sees a far-spread spectrum
    // (strongly indefinite tangents): a multigrid solve that made no
    // progress is repeated with block-Jacobi alone, within the iterations
    // left to this solve
    lgdm_solver_opts bj = o;
    bj.precond = LGDM_PRECOND_BLOCK_JACOBI;
    bj.max_krylov = (int32_t)(o.max_krylov - kr.iters);
    const int64_t it0 = kr.iters, sp0 = kr.spmv;
    const int rs0 = kr.restarts;
    HIPCHECK(c, krylov_solve(c, b_dev, x_dev, bj, tol_u, tol_e, kr), "Krylov solve");
    kr.iters += it0;
    kr.spmv += sp0;
    kr.restarts += rs0;
    if (rep) rep->precond_fallbacks += 1;
  }
  c->last_solve_improved = kr.status == LGDM_OK || kr.improved;
  c->inc_krylov += kr.iters;
  if (rep) {
    rep->zone_dofs = std::max<int64_t>(rep->zone_dofs, zone_dofs(c));
    rep->krylov_iters += kr.iters;
    rep->restarts += kr.restarts;
    rep->krylov_status = kr.status;
    rep->krylov_spmv += kr.spmv;
    rep->krylov_rel_u = kr.rel_u;
    rep->krylov_rel_e = kr.rel_e;
    if (kr.status == LGDM_ERR_NOT_CONVERGED || kr.status == LGDM_ERR_BREAKDOWN) rep->inexact_solves += 1;
  }
  if (kr.status == LGDM_ERR_NAN)
    return fail(c, LGDM_ERR_NAN, "non-finite Krylov scalar after " + std::to_string(kr.iters) +
                                     " iterations (" + std::to_string(kr.restarts) + " restarts)");
  if (kr.status == LGDM_ERR_BREAKDOWN)
    return fail(c, LGDM_ERR_BREAKDOWN, "Krylov breakdown persisted after " +
                                           std::to_string(kr.restarts) + " restarts");
  if (kr.status == LGDM_ERR_NOT_CONVERGED)
    return fail(c, LGDM_ERR_NOT_CONVERGED, "Krylov solve stopped short of its tolerance");
  return LGDM_OK;
}

// inside Newton an inexact correction is acceptable: the FP64 residual test
// of the next iteration decides convergence
bool tolerable_in_newton(lgdm_status s) {
  return s == LGDM_OK || s == LGDM_ERR_NOT_CONVERGED || s == LGDM_ERR_BREAKDOWN;
}

}  // namespace

extern "C" {

lgdm_status lgdm_create(lgdm_ctx** out, int32_t device, void* hip_stream, int32_t precision) {
  if (!out) return LGDM_ERR_INVALID_ARG;
  *out = nullptr;
  if (precision != LGDM_FP64 && precision != LGDM_MIXED) return LGDM_ERR_INVALID_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return LGDM_ERR_DEVICE;
  }
  if (hipSetDevice(device) != hipSuccess) return LGDM_ERR_DEVICE;
  // the address of the allocation-free solve's static scratch on this device
  if (noalloc_init(device) != hipSuccess) {
    (void)hipGetLastError();
    return LGDM_ERR_DEVICE;
  }
  lgdm_ctx* c = new (std::nothrow) lgdm_ctx();
  if (!c) return LGDM_ERR_OOM;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->precision = precision;
  if (hipHostMalloc((void**)&c->norms_host, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->kscal_host, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    delete c;
    return LGDM_ERR_OOM;
  }
  for (auto& ev : c->ev)
    if (hipEventCreate(&ev) != hipSuccess) {
      delete c;
      return LGDM_ERR_DEVICE;
    }
  c->events_ready = true;
  *out = c;
  return LGDM_OK;
}

lgdm_status lgdm_destroy(lgdm_ctx* c) {
  if (!c) return LGDM_ERR_INVALID_ARG;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  probe_release(c);
  free_mesh(c);
  if (c->norms_host) (void)hipHostFree(c->norms_host);
  if (c->kscal_host) (void)hipHostFree(c->kscal_host);
  if (c->events_ready)
    for (auto& ev : c->ev) (void)hipEventDestroy(ev);
  delete c;
  return LGDM_OK;
}

const char* lgdm_last_error(const lgdm_ctx* c) { return c ? c->err.c_str() : "null context"; }

lgdm_status lgdm_set_allocator(lgdm_ctx* c, void* (*alloc)(size_t, void*), void (*free_fn)(void*, void*),
                               void* user) {
  if (!c) return LGDM_ERR_INVALID_ARG;
  if (!c->allocs.empty()) return fail(c, LGDM_ERR_STATE, "set the allocator before uploading a mesh");
  if ((alloc == nullptr) != (free_fn == nullptr))
    return fail(c, LGDM_ERR_INVALID_ARG, "alloc and free must both be given or both be NULL");
  c->alloc_fn = alloc;
  c->free_fn = free_fn;
  c->alloc_user = user;
  return LGDM_OK;
}

lgdm_status lgdm_upload_mesh(lgdm_ctx* c, int32_t dim, int32_t elem_type, int64_t n_nodes,
                             const double* coords, int64_t n_elems, const int32_t* conn,
                             const double* e_scale) {
  if (!c) return LGDM_ERR_INVALID_ARG;
  const bool order2 = (elem_type == LGDM_LINE3 && dim == 1) || (elem_type == LGDM_QUAD9 && dim == 2);
  if (dim < 1 || dim > 3 || (elem_type != dim && !order2))
    return fail(c, LGDM_ERR_INVALID_ARG, "dim must be 1, 2 or 3 with element type LINE2, QUAD4, HEX8, "
                                         "or 1 with LINE3, 2 with QUAD9");
  if (n_nodes <= 0 || n_elems <= 0 || !coords || !conn)
    return fail(c, LGDM_ERR_INVALID_ARG, "empty mesh or NULL coords / conn");
  if (n_elems >= ((int64_t)1 << (31 - N2E_SHIFT)) || n_nodes * (dim + 1) >= ((int64_t)1 << 31))
    return fail(c, LGDM_ERR_INVALID_ARG, "mesh too large for int32 indexing");
  if (order2 && c->has_mat && c->mat.coupling != LGDM_COUPLING_EXECUTED)
    return fail(c, LGDM_ERR_INVALID_ARG, "the coupling variant is not available for mixed-order elements");
  (void)hipSetDevice(c->device);
  free_mesh(c);
  c->dim = dim;
  c->order2 = order2;
  c->nen = order2 ? (dim == 1 ? 3 : 9) : 1 << dim;
  c->nen_e = 1 << dim;
  c->ngp = order2 ? (dim == 1 ? 3 : 9) : 1 << dim;
  c->nd = dim + 1;
  c->n_nodes = n_nodes;
  c->n_elems = n_elems;
  c->ndof = n_nodes * c->nd;
  c->ngauss = n_elems * c->ngp;
  c->coords = (double*)dalloc(c, n_nodes * dim * sizeof(double));
  c->conn = (int32_t*)dalloc(c, n_elems * c->nen * sizeof(int32_t));
  c->e_scale = (double*)dalloc(c, n_elems * sizeof(double));
  if (!c->coords || !c->conn || !c->e_scale) {
    free_mesh(c);
    return fail(c, LGDM_ERR_OOM, "device allocation failed (mesh)");
  }
  HIPCHECK(c, hipMemcpyAsync(c->coords, coords, n_nodes * dim * sizeof(double), hipMemcpyDefault, c->stream), "copy coords");
  HIPCHECK(c, hipMemcpyAsync(c->conn, conn, n_elems * c->nen * sizeof(int32_t), hipMemcpyDefault, c->stream), "copy conn");
  if (e_scale) {
    HIPCHECK(c, hipMemcpyAsync(c->e_scale, e_scale, n_elems * sizeof(double), hipMemcpyDefault, c->stream), "copy e_scale");
  } else {
    std::vector<double> ones(n_elems, 1.0);
    HIPCHECK(c, hipMemcpyAsync(c->e_scale, ones.data(), n_elems * sizeof(double), hipMemcpyHostToDevice, c->stream), "copy e_scale");
    HIPCHECK(c, hipStreamSynchronize(c->stream), "copy e_scale");
  }
  std::string msg;
  int status = LGDM_OK;
  hipError_t e = build_pattern(c, msg, status);
  if (e != hipSuccess) {
    free_mesh(c);
    return hip_fail(c, e, "pattern build");
  }
  if (status != LGDM_OK) {
    free_mesh(c);
    return fail(c, status, msg);
  }
  if (order2 && c->max_nbr > (dim == 1 ? 8 : 32)) {
    free_mesh(c);
    return fail(c, LGDM_ERR_INVALID_ARG, "a node has more neighbours than the mixed-order assembly handles");
  }
  // ebar dofs of nodes that are no element's vertex carry no unknown: they
  // are constrained to zero like Dirichlet dofs
  c->base_flags.assign(c->ndof, 0);
  if (order2) {
    std::vector<uint8_t> vert(n_nodes, 0);
    for (int64_t el = 0; el < n_elems; ++el)
      for (int a = 0; a < c->nen_e; ++a) vert[conn[el * c->nen + a]] = 1;
    for (int64_t n = 0; n < n_nodes; ++n)
      if (!vert[n]) c->base_flags[n * c->nd + dim] = 1 | 4;
  }
  // state, assembly and solver buffers
  const int64_t nd = c->ndof, ng = c->ngauss;
  const bool mixed = c->precision == LGDM_MIXED;
  c->x = (double*)dalloc(c, nd * sizeof(double));
  c->x_save = (double*)dalloc(c, nd * sizeof(double));
  c->R = (double*)dalloc(c, nd * sizeof(double));
  c->delta = (double*)dalloc(c, nd * sizeof(double));
  c->kappa_n = (double*)dalloc(c, ng * sizeof(double));
  c->D_n = (double*)dalloc(c, ng * sizeof(double));
  c->kappa_t = (double*)dalloc(c, ng * sizeof(double));
  c->D_t = (double*)dalloc(c, ng * sizeof(double));
  c->eeq_t = (double*)dalloc(c, ng * sizeof(double));
  const int rs = rec_stride(dim, c->has_mat && c->mat.coupling == LGDM_COUPLING_EQ2);
  c->rec = (double*)dalloc(c, ng * rs * sizeof(double));
  c->rec_stride = rs;
  if (mixed) c->vals32 = (float*)dalloc(c, c->nnz * sizeof(float));
  else c->vals = (double*)dalloc(c, c->nnz * sizeof(double));
  c->n_partials = node_kernel_blocks(c);
  c->partials = (double*)dalloc(c, c->n_partials * NORM_SLOTS * sizeof(double));
  c->norms_dev = (double*)dalloc(c, 16 * sizeof(double));
  c->red2 = (double*)dalloc(c, RED_CHUNKS * NORM_SLOTS * sizeof(double));
  c->dof_flags = (uint8_t*)dalloc(c, nd);
  c->kv = (double*)dalloc(c, (size_t)KV_VECS * nd * sizeof(double));
  if (mixed) c->minv32 = (float*)dalloc(c, n_nodes * c->nd * c->nd * sizeof(float));
  else c->minv = (double*)dalloc(c, n_nodes * c->nd * c->nd * sizeof(double));
  c->n_kpart = (int64_t)KPART_BLOCKS * KPART_PER_BLOCK;
  c->kpart = (double*)dalloc(c, c->n_kpart * sizeof(double));
  c->kscal = (double*)dalloc(c, KSCAL_DOUBLES * sizeof(double));
  c->kcount = (unsigned*)dalloc(c, 16 * sizeof(unsigned));
  if (!c->x || !c->x_save || !c->R || !c->delta || !c->kappa_n || !c->D_n || !c->kappa_t || !c->D_t || !c->eeq_t ||
      !c->rec || (!c->vals && !c->vals32) || !c->partials || !c->norms_dev || !c->red2 || !c->dof_flags ||
      !c->kv || (!c->minv && !c->minv32) || !c->kpart || !c->kscal || !c->kcount) {
    free_mesh(c);
    return fail(c, LGDM_ERR_OOM, "device allocation failed (state / matrix / solver)");
  }
  // the SpMV reads blocks of the CSR values and of x as 4-wide vectors
  for (const void* p : {(const void*)c->x, (const void*)c->delta, (const void*)c->kv, (const void*)c->vals,
                        (const void*)c->vals32, (const void*)c->minv, (const void*)c->minv32})
    if (reinterpret_cast<uintptr_t>(p) % 32 != 0) {
      free_mesh(c);
      return fail(c, LGDM_ERR_INVALID_ARG, "the allocator returned memory not aligned to 32 bytes");
    }
  HIPCHECK(c, zero(c, c->x, nd * sizeof(double)), "zero");
  HIPCHECK(c, zero(c, c->x_save, nd * sizeof(double)), "zero");
  HIPCHECK(c, zero(c, c->R, nd * sizeof(double)), "zero");
  HIPCHECK(c, zero(c, c->kappa_n, ng * sizeof(double)), "zero");
  HIPCHECK(c, zero(c, c->D_n, ng * sizeof(double)), "zero");
  HIPCHECK(c, zero(c, c->kappa_t, ng * sizeof(double)), "zero");
  HIPCHECK(c, zero(c, c->D_t, ng * sizeof(double)), "zero");
  HIPCHECK(c, zero(c, c->eeq_t, ng * sizeof(double)), "zero");
  HIPCHECK(c, hipMemcpyAsync(c->dof_flags, c->base_flags.data(), nd, hipMemcpyHostToDevice, c->stream), "flags");
  HIPCHECK(c, zero(c, c->kcount, 16 * sizeof(unsigned)), "zero");
  HIPCHECK(c, hipStreamSynchronize(c->stream), "upload");
  c->increment = 0;
  c->assembled = false;
  c->in_increment = false;
  return LGDM_OK;
}

lgdm_status lgdm_set_material(lgdm_ctx* c, const lgdm_material* m) {
  if (!c || !m) return fail(c, LGDM_ERR_INVALID_ARG, "NULL material");
  if (!(m->E > 0) || !(m->nu > -1.0 && m->nu < 0.5) || !(m->kappa0 > 0) || !(m->k > 0) ||
      !(m->h > 0) || !(m->eta > 0) || !(m->c >= 0) || !(m->thickness > 0) ||
      !(m->tol_hist >= 0) || !(m->tol_dmg >= 0) || (m->plane != 0 && m->plane != 1) ||
      (m->coupling != LGDM_COUPLING_EXECUTED && m->coupling != LGDM_COUPLING_EQ2))
    return fail(c, LGDM_ERR_INVALID_ARG, "material parameter out of range");
  if (c->order2 && m->coupling != LGDM_COUPLING_EXECUTED)
    return fail(c, LGDM_ERR_INVALID_ARG, "the coupling variant is not available for mixed-order elements");
  // the coupling variant's Gauss-point records are longer
  if (c->dim != 0 && c->rec_stride < rec_stride(c->dim, m->coupling == LGDM_COUPLING_EQ2)) {
    const int rs = rec_stride(c->dim, true);
    HIPCHECK(c, hipStreamSynchronize(c->stream), "set_material");
    dfree(c, c->rec);
    c->rec = (double*)dalloc(c, c->ngauss * rs * sizeof(double));
    c->rec_stride = c->rec ? rs : 0;
    if (!c->rec) return fail(c, LGDM_ERR_OOM, "device allocation failed (Gauss-point records)");
  }
  c->mat = *m;
  c->has_mat = true;
  c->assembled = false;
  return LGDM_OK;
}

lgdm_status lgdm_set_dirichlet(lgdm_ctx* c, int64_t n, const int64_t* dofs, const double* ref_values) {
  if (!c) return LGDM_ERR_INVALID_ARG;
  if (c->dim == 0) return fail(c, LGDM_ERR_STATE, "upload a mesh first");
  if (n < 0 || (n > 0 && (!dofs || !ref_values))) return fail(c, LGDM_ERR_INVALID_ARG, "bad Dirichlet arrays");
  std::vector<uint8_t> flags(c->base_flags);
  std::vector<int32_t> d32(n);
  std::vector<double> v(n);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t d = dofs[i];
    if (d < 0 || d >= c->ndof) return fail(c, LGDM_ERR_INVALID_ARG, "Dirichlet dof out of range");
    if (d % c->nd == c->nd - 1)
      return fail(c, LGDM_ERR_INVALID_ARG, "Dirichlet conditions apply to displacement dofs only");
    flags[d] |= 1;
    if (ref_values[i] != 0.0) flags[d] |= 2;
    d32[i] = (int32_t)d;
    v[i] = ref_values[i];
  }
  if (c->bc_dofs) dfree(c, c->bc_dofs);
  if (c->bc_vals) dfree(c, c->bc_vals);
  c->bc_dofs = nullptr;
  c->bc_vals = nullptr;
  c->nbc = n;
  if (n > 0) {
    c->bc_dofs = (int32_t*)dalloc(c, n * sizeof(int32_t));
    c->bc_vals = (double*)dalloc(c, n * sizeof(double));
    if (!c->bc_dofs || !c->bc_vals) return fail(c, LGDM_ERR_OOM, "device allocation failed (Dirichlet)");
    HIPCHECK(c, hipMemcpyAsync(c->bc_dofs, d32.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, c->stream), "copy bc");
    HIPCHECK(c, hipMemcpyAsync(c->bc_vals, v.data(), n * sizeof(double), hipMemcpyHostToDevice, c->stream), "copy bc");
  }
  HIPCHECK(c, hipMemcpyAsync(c->dof_flags, flags.data(), c->ndof, hipMemcpyHostToDevice, c->stream), "copy flags");
  HIPCHECK(c, hipStreamSynchronize(c->stream), "set_dirichlet");
  c->assembled = false;
  return LGDM_OK;
}

lgdm_status lgdm_assemble_tangent_residual(lgdm_ctx* c, double lambda, lgdm_csr_view* K_out, double* R_out) {
  if (!c) return LGDM_ERR_INVALID_ARG;
  if (!ready(c)) return fail(c, LGDM_ERR_STATE, "upload a mesh and set the material first");
  if (lambda >= 0) HIPCHECK(c, launch_set_dirichlet(c, lambda), "set Dirichlet values");
  lgdm_status s = assemble_now(c, nullptr);
  if (s != LGDM_OK && s != LGDM_ERR_NAN) return s;
  if (R_out) {
    HIPCHECK(c, hipMemcpyAsync(R_out, c->R, c->ndof * sizeof(double), hipMemcpyDefault, c->stream), "copy R");
    HIPCHECK(c, hipStreamSynchronize(c->stream), "copy R");
  }
  if (K_out) {
    K_out->nrows = c->ndof;
    K_out->nnz = c->nnz;
    K_out->row_ptr = c->row_ptr;
    K_out->col_idx = c->col_idx;
    K_out->vals = c->vals;
    K_out->vals32 = c->vals32;
  }
  return s;
}

lgdm_status lgdm_solve_linear(lgdm_ctx* c, const double* b, double* delta, const lgdm_solver_opts* o,
                              lgdm_increment_report* rep) {
  if (!c || !b || !delta) return fail(c, LGDM_ERR_INVALID_ARG, "NULL vector");
  if (!ready(c) || !c->assembled) return fail(c, LGDM_ERR_STATE, "assemble before solving");
  const lgdm_solver_opts op = fill_opts(o);
  // stage b in R's sibling buffer to accept host or device input
  HIPCHECK(c, hipMemcpyAsync(c->delta, b, c->ndof * sizeof(double), hipMemcpyDefault, c->stream), "copy b");
  double* bdev = c->delta;
  double* xdev = (double*)dalloc(c, c->ndof * sizeof(double));
  if (!xdev) return fail(c, LGDM_ERR_OOM, "device allocation failed (solution)");
  if (rep) std::memset(rep, 0, sizeof(*rep));
  lgdm_status s = linear_solve(c, bdev, xdev, op, op.tol_krylov, op.tol_krylov, rep);
  if (s == LGDM_OK) {
    hipError_t e = hipMemcpyAsync(delta, xdev, c->ndof * sizeof(double), hipMemcpyDefault, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) s = hip_fail(c, e, "copy solution");
  }
  dfree(c, xdev);
  return s;
}

lgdm_status lgdm_solve_linear_noalloc(lgdm_ctx* c, const double* b, double* delta, const lgdm_solver_opts* o,
                                      lgdm_increment_report* rep) {
  if (!c || !b || !delta) return fail(c, LGDM_ERR_INVALID_ARG, "NULL vector");
  if (!ready(c) || !c->assembled) return fail(c, LGDM_ERR_STATE, "assemble before solving");
  for (const void* p : {(const void*)b, (const void*)delta}) {
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess || a.type != hipMemoryTypeDevice || a.device != c->device) {
      (void)hipGetLastError();
      return fail(c, LGDM_ERR_INVALID_ARG, "b and delta must be device memory of the context's device");
    }
  }
  if (reinterpret_cast<uintptr_t>(delta) % 32 != 0)
    return fail(c, LGDM_ERR_INVALID_ARG, "delta must be aligned to 32 bytes (the SpMV reads it in 4-wide vectors)");
  double* scratch = noalloc_scratch(c->device);
  if (!scratch) return fail(c, LGDM_ERR_DEVICE, "the static scratch of this device is not resolved");
  // the solve's scratch: its reduction partials and its device scalars
  const size_t need = ((size_t)c->n_kpart + KSCAL_DOUBLES) * sizeof(double);
  if (need > LGDM_NOALLOC_SCRATCH_BYTES)
    return fail(c, LGDM_ERR_INVALID_ARG, "the solve needs " + std::to_string(need) +
                                             " bytes of scratch; the static array holds " +
                                             std::to_string((size_t)LGDM_NOALLOC_SCRATCH_BYTES));
  const lgdm_solver_opts op = fill_opts(o);
  const bool amg = (op.precond == LGDM_PRECOND_AMG ||
                    (op.precond == LGDM_PRECOND_DEFAULT && c->dim == 3 && op.krylov_method == LGDM_KRYLOV_IDRS &&
                     !c->amg_unavailable));
  if (amg && !c->amg)
    return fail(c, LGDM_ERR_STATE, "the multigrid hierarchy is allocated at the context's first multigrid solve; "
                                   "run one lgdm_solve_linear first or select block-Jacobi");
  if (rep) std::memset(rep, 0, sizeof(*rep));
  // b is staged in the context's own right-hand-side buffer, as lgdm_solve_linear does
  HIPCHECK(c, hipMemcpyAsync(c->delta, b, c->ndof * sizeof(double), hipMemcpyDeviceToDevice, c->stream), "copy b");
  double* const own_kpart = c->kpart;
  double* const own_kscal = c->kscal;
  c->kpart = scratch;
  c->kscal = scratch + c->n_kpart;
  c->noalloc_call = true;
  // the array keeps the previous call's values: the scalars start at zero
  hipError_t e = launch_fill(c->kscal, KSCAL_DOUBLES, 0.0, c->stream);
  lgdm_status s = e == hipSuccess ? linear_solve(c, c->delta, delta, op, op.tol_krylov, op.tol_krylov, rep)
                                  : hip_fail(c, e, "clear scratch");
  if (e == hipSuccess) {
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess && s == LGDM_OK) s = hip_fail(c, e, "solve");
  }
  c->kpart = own_kpart;
  c->kscal = own_kscal;
  c->noalloc_call = false;
  return s;
}

lgdm_status lgdm_begin_increment(lgdm_ctx* c, double lambda) {
  if (!c) return LGDM_ERR_INVALID_ARG;
  if (!ready(c)) return fail(c, LGDM_ERR_STATE, "upload a mesh and set the material first");
  HIPCHECK(c, hipMemcpyAsync(c->x_save, c->x, c->ndof * sizeof(double), hipMemcpyDeviceToDevice, c->stream), "save x");
  HIPCHECK(c, launch_set_dirichlet(c, lambda), "set Dirichlet values");
  c->in_increment = true;
  c->nw_iter = 0;
  c->nw_stepped = false;
  c->nw_best_phi = HUGE_VAL;
  c->nw_since_best = 0;
  c->inc_lambda = lambda;
  c->inc_serial += 1;
  c->inc_zone_used = false;
  c->inc_zone_tier = 0;
  c->inc_krylov = 0;
  c->inc_t0 = host_seconds();
  return LGDM_OK;
}

lgdm_status lgdm_newton_iteration(lgdm_ctx* c, const lgdm_solver_opts* o, int32_t* converged,
                                  lgdm_increment_report* rep) {
  if (!c || !converged) return fail(c, LGDM_ERR_INVALID_ARG, "NULL argument");
  if (!ready(c) || !c->in_increment) return fail(c, LGDM_ERR_STATE, "begin an increment first");
  const lgdm_solver_opts op = fill_opts(o);
  *converged = 0;
  float t_asm = 0.f, t_sol = 0.f, t_upd = 0.f;
  lgdm_status s = assemble_now(c, &t_asm);
  if (rep) {
    rep->t_assembly_ms += t_asm;
    rep->n_assemblies += 1;
    fill_norms(c, rep);
  }
  if (s != LGDM_OK) return s;
  // line search: a correction that raised the merit more than fourfold is
  // halved (at most four times), each trial assembled like an iterate
  if (op.line_search == LGDM_LINE_SEARCH_ON && c->nw_stepped) {
    while (!residual_converged(c, op.tol_newton) && newton_merit(c) > LS_GROWTH * c->nw_phi &&
           c->nw_cuts < LS_MAX_CUTS) {
      HIPCHECK(c, launch_axpy(c, c->x, c->delta, -0.5 * c->nw_alpha, c->ndof), "line search");
      c->nw_alpha *= 0.5;
      c->nw_cuts += 1;
      s = assemble_now(c, &t_asm);
      if (rep) {
        rep->t_assembly_ms += t_asm;
        rep->n_assemblies += 1;
        rep->backtracks += 1;
        fill_norms(c, rep);
      }
      if (s != LGDM_OK) return s;
    }
  }
  c->nw_stepped = false;
  if (residual_converged(c, op.tol_newton)) {
    *converged = 1;
    return LGDM_OK;
  }
  // Newton with the process zone that no longer reduces the merit restarts
  // the increment from its beginning with a smaller zone (the damage
  // threshold tenfold closer to 1), then without the zone
  const double phi = newton_merit(c);
  if (phi < c->nw_best_phi) {
    c->nw_best_phi = phi;
    c->nw_since_best = 0;
  } else {
    c->nw_since_best += 1;
  }
  if (c->inc_zone_used && c->inc_zone_tier < 2 && c->nw_since_best >= ZONE_PATIENCE) {
    HIPCHECK(c, hipMemcpyAsync(c->x, c->x_save, c->ndof * sizeof(double), hipMemcpyDeviceToDevice, c->stream),
             "restore x");
    HIPCHECK(c, launch_set_dirichlet(c, c->inc_lambda), "set Dirichlet values");
    c->inc_zone_tier += 1;
    c->inc_zone_used = false;
    zone_forget(c);   // factors of the abandoned iterates are not reused
    c->nw_iter = 0;
    c->nw_best_phi = HUGE_VAL;
    c->nw_since_best = 0;
    s = assemble_now(c, &t_asm);
    if (rep) {
      rep->t_assembly_ms += t_asm;
      rep->n_assemblies += 1;
      rep->zone_restarts += 1;
      fill_norms(c, rep);
    }
    if (s != LGDM_OK) return s;
    if (residual_converged(c, op.tol_newton)) {
      *converged = 1;
      return LGDM_OK;
    }
    c->nw_best_phi = newton_merit(c);
  }
  // work bound of the increment: the Krylov iterations and the wall time
  // left to it
  lgdm_solver_opts ob = op;
  if (op.max_increment_krylov > 0) {
    const int64_t left = op.max_increment_krylov - c->inc_krylov;
    if (left <= 0)
      return fail(c, LGDM_ERR_NOT_CONVERGED, "increment work bound reached: " + std::to_string(c->inc_krylov) +
                                                 " Krylov iterations (max_increment_krylov)");
    ob.max_krylov = (int32_t)std::min<int64_t>(op.max_krylov, left);
  }
  c->solve_deadline = 0.0;
  if (op.max_increment_seconds > 0) {
    c->solve_deadline = c->inc_t0 + op.max_increment_seconds;
    if (host_seconds() > c->solve_deadline) {
      c->solve_deadline = 0.0;
      return fail(c, LGDM_ERR_NOT_CONVERGED, "increment work bound reached: wall time above " +
                                                 std::to_string(op.max_increment_seconds) +
                                                 " s (max_increment_seconds)");
    }
  }
  HIPCHECK(c, hipEventRecord(c->ev[2], c->stream), "event");
  double tol_u = op.tol_krylov, tol_e = op.tol_krylov;
  newton_forcing(c, op, tol_u, tol_e);
  c->zone_may_reuse = true;
  s = linear_solve(c, c->R, c->delta, ob, tol_u, tol_e, rep);
  c->zone_may_reuse = false;
  c->solve_deadline = 0.0;
  HIPCHECK(c, hipEventRecord(c->ev[3], c->stream), "event");
  if (!tolerable_in_newton(s)) return s;
  // a correction no better than none would repeat this iteration unchanged:
  // with the process zone in use and a smaller zone (or none) left to try,
  // the next iteration restarts the increment (x is left as it is);
  // otherwise Newton stops here
  if (!c->last_solve_improved) {
    if (c->inc_zone_used && c->inc_zone_tier < 2) {
      c->nw_since_best = ZONE_PATIENCE;
      return LGDM_OK;
    }
    return fail(c, LGDM_ERR_NOT_CONVERGED, "the linear solve made no progress on the Newton system");
  }
  s = LGDM_OK;
  // Algorithm 2: u_i = u_{i-1} + delta u, ebar_i = ebar_{i-1} + delta ebar
  HIPCHECK(c, launch_axpy(c, c->x, c->delta, 1.0, c->ndof), "update");
  c->nw_stepped = true;
  c->nw_phi = newton_merit(c);
  c->nw_alpha = 1.0;
  c->nw_cuts = 0;
  HIPCHECK(c, launch_field_norms(c, c->delta, c->norms_dev + 8), "update norms");
  HIPCHECK(c, hipEventRecord(c->ev[4], c->stream), "event");
  HIPCHECK(c, hipMemcpyAsync(c->norms_host + 8, c->norms_dev + 8, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream), "norms");
  HIPCHECK(c, hipStreamSynchronize(c->stream), "update");
  HIPCHECK(c, hipEventElapsedTime(&t_sol, c->ev[2], c->ev[3]), "event time");
  HIPCHECK(c, hipEventElapsedTime(&t_upd, c->ev[3], c->ev[4]), "event time");
  if (rep) {
    rep->t_solve_ms += t_sol;
    rep->t_update_ms += t_upd;
    rep->newton_iters += 1;
    rep->du_norm = std::sqrt(c->norms_host[8]);
    rep->de_norm = std::sqrt(c->norms_host[9]);
  }
  return LGDM_OK;
}

lgdm_status lgdm_commit_increment(lgdm_ctx* c) {
  if (!c) return LGDM_ERR_INVALID_ARG;
  if (!ready(c) || !c->assembled) return fail(c, LGDM_ERR_STATE, "nothing assembled to commit");
  // Eq. A.2: the history variable becomes the running maximum over converged states
  HIPCHECK(c, hipMemcpyAsync(c->kappa_n, c->kappa_t, c->ngauss * sizeof(double), hipMemcpyDeviceToDevice, c->stream), "commit");
  HIPCHECK(c, hipMemcpyAsync(c->D_n, c->D_t, c->ngauss * sizeof(double), hipMemcpyDeviceToDevice, c->stream), "commit");
  HIPCHECK(c, hipStreamSynchronize(c->stream), "commit");
  c->increment += 1;
  c->in_increment = false;
  return LGDM_OK;
}

lgdm_status lgdm_abort_increment(lgdm_ctx* c) {
  if (!c) return LGDM_ERR_INVALID_ARG;
  if (!ready(c)) return fail(c, LGDM_ERR_STATE, "no mesh");
  if (c->in_increment) {
    HIPCHECK(c, hipMemcpyAsync(c->x, c->x_save, c->ndof * sizeof(double), hipMemcpyDeviceToDevice, c->stream), "restore x");
    HIPCHECK(c, hipStreamSynchronize(c->stream), "restore x");
  }
  c->in_increment = false;
  c->assembled = false;
  return LGDM_OK;
}

lgdm_status lgdm_solve_increment(lgdm_ctx* c, double lambda, const lgdm_solver_opts* o,
                                 lgdm_increment_report* rep) {
  if (!c) return LGDM_ERR_INVALID_ARG;
  const lgdm_solver_opts op = fill_opts(o);
  lgdm_increment_report local{};
  lgdm_increment_report* r = rep ? rep : &local;
  std::memset(r, 0, sizeof(*r));
  lgdm_status s = lgdm_begin_increment(c, lambda);
  if (s != LGDM_OK) return s;
  for (int it = 0;; ++it) {
    int32_t conv = 0;
    s = lgdm_newton_iteration(c, &op, &conv, r);
    if (s != LGDM_OK) {
      std::string msg = c->err;
      lgdm_abort_increment(c);
      c->err = msg;
      return s;
    }
    if (conv) break;
    if (it + 1 > op.max_newton) {
      lgdm_abort_increment(c);
      return fail(c, LGDM_ERR_NOT_CONVERGED, "Newton did not converge within max_newton iterations");
    }
  }
  // max damage of the converged state, then commit
  HIPCHECK(c, launch_max_reduce(c, c->D_t, c->ngauss, c->norms_dev + 12), "max damage");
  HIPCHECK(c, hipMemcpyAsync(c->norms_host + 12, c->norms_dev + 12, sizeof(double), hipMemcpyDeviceToHost, c->stream), "max damage");
  s = lgdm_commit_increment(c);
  if (s != LGDM_OK) return s;
  r->converged = 1;
  r->max_damage = c->norms_host[12];
  return LGDM_OK;
}

lgdm_status lgdm_get_csr(lgdm_ctx* c, int64_t* nrows, int64_t* nnz, const int32_t** row_ptr,
                         const int32_t** col_idx) {
  if (!c) return LGDM_ERR_INVALID_ARG;
  if (c->dim == 0) return fail(c, LGDM_ERR_STATE, "no mesh");
  if (nrows) *nrows = c->ndof;
  if (nnz) *nnz = c->nnz;
  if (row_ptr) *row_ptr = c->row_ptr;
  if (col_idx) *col_idx = c->col_idx;
  return LGDM_OK;
}

lgdm_status lgdm_get_connectivity(lgdm_ctx* c, const int32_t** conn, int64_t* n_elems, int32_t* nen) {
  if (!c) return LGDM_ERR_INVALID_ARG;
  if (c->dim == 0) return fail(c, LGDM_ERR_STATE, "no mesh");
  if (conn) *conn = c->conn;
  if (n_elems) *n_elems = c->n_elems;
  if (nen) *nen = c->nen;
  return LGDM_OK;
}

lgdm_status lgdm_get_sizes(lgdm_ctx* c, int64_t* ndof, int64_t* n_gauss, int64_t* increment) {
  if (!c) return LGDM_ERR_INVALID_ARG;
  if (ndof) *ndof = c->ndof;
  if (n_gauss) *n_gauss = c->ngauss;
  if (increment) *increment = c->increment;
  return LGDM_OK;
}

lgdm_status lgdm_query_state(lgdm_ctx* c, int32_t field, double* out, int64_t n) {
  if (!c || !out) return fail(c, LGDM_ERR_INVALID_ARG, "NULL output");
  if (c->dim == 0) return fail(c, LGDM_ERR_STATE, "no mesh");
  const double* src = nullptr;
  int64_t sz = 0;
  switch (field) {
    case LGDM_FIELD_X: src = c->x; sz = c->ndof; break;
    case LGDM_FIELD_KAPPA: src = c->kappa_n; sz = c->ngauss; break;
    case LGDM_FIELD_DAMAGE: src = c->D_n; sz = c->ngauss; break;
    case LGDM_FIELD_KAPPA_TRIAL: src = c->kappa_t; sz = c->ngauss; break;
    case LGDM_FIELD_DAMAGE_TRIAL: src = c->D_t; sz = c->ngauss; break;
    case LGDM_FIELD_RESIDUAL: src = c->R; sz = c->ndof; break;
    case LGDM_FIELD_EEQ: src = c->eeq_t; sz = c->ngauss; break;
    case LGDM_FIELD_REACTION:
      if (n != 1) return fail(c, LGDM_ERR_INVALID_ARG, "reaction has size 1");
      HIPCHECK(c, hipMemcpy(out, &c->last_norms[4], sizeof(double), hipMemcpyDefault), "copy reaction");
      return LGDM_OK;
    default: return fail(c, LGDM_ERR_INVALID_ARG, "unknown field");
  }
  if (n != sz) return fail(c, LGDM_ERR_INVALID_ARG, "output size does not match the field");
  HIPCHECK(c, hipMemcpyAsync(out, src, sz * sizeof(double), hipMemcpyDefault, c->stream), "copy field");
  HIPCHECK(c, hipStreamSynchronize(c->stream), "copy field");
  return LGDM_OK;
}

lgdm_status lgdm_set_state(lgdm_ctx* c, const double* x, const double* kappa_n, int64_t increment) {
  if (!c) return LGDM_ERR_INVALID_ARG;
  if (!ready(c)) return fail(c, LGDM_ERR_STATE, "upload a mesh and set the material first");
  if (increment < 0) return fail(c, LGDM_ERR_INVALID_ARG, "negative increment");
  if (x) {
    HIPCHECK(c, hipMemcpyAsync(c->x, x, c->ndof * sizeof(double), hipMemcpyDefault, c->stream), "copy x");
    if (c->order2) HIPCHECK(c, launch_zero_flagged(c, c->x, 4), "zero ebar of non-vertex nodes");
  }
  if (kappa_n) {
    HIPCHECK(c, hipMemcpyAsync(c->kappa_n, kappa_n, c->ngauss * sizeof(double), hipMemcpyDefault, c->stream), "copy kappa");
    HIPCHECK(c, launch_damage_from_kappa(c, make_params(c->mat, c->dim)), "damage");
  }
  HIPCHECK(c, hipStreamSynchronize(c->stream), "set_state");
  c->increment = increment;
  c->assembled = false;
  c->in_increment = false;
  return LGDM_OK;
}

lgdm_status lgdm_debug_element_blocks(lgdm_ctx* c, int64_t e0, int64_t e1, double* Ke_out, double* fe_out) {
  if (!c) return LGDM_ERR_INVALID_ARG;
  if (!ready(c) || !c->assembled) return fail(c, LGDM_ERR_STATE, "assemble first");
  if (e0 < 0 || e1 > c->n_elems || e1 < e0) return fail(c, LGDM_ERR_INVALID_ARG, "element range");
  const int64_t ne = e1 - e0;
  if (ne == 0) return LGDM_OK;
  const int64_t nl = (int64_t)c->nen * c->nd;
  double* kd = Ke_out ? (double*)dalloc(c, ne * nl * nl * sizeof(double)) : nullptr;
  double* fd = fe_out ? (double*)dalloc(c, ne * nl * sizeof(double)) : nullptr;
  if ((Ke_out && !kd) || (fe_out && !fd)) {
    dfree(c, kd);
    dfree(c, fd);
    return fail(c, LGDM_ERR_OOM, "device allocation failed (element blocks)");
  }
  if (fd) HIPCHECK(c, zero(c, fd, ne * nl * sizeof(double)), "zero");
  HIPCHECK(c, launch_element_blocks(c, make_params(c->mat, c->dim), e0, e1, kd, fd), "element blocks");
  if (kd) HIPCHECK(c, hipMemcpyAsync(Ke_out, kd, ne * nl * nl * sizeof(double), hipMemcpyDefault, c->stream), "copy Ke");
  if (fd) HIPCHECK(c, hipMemcpyAsync(fe_out, fd, ne * nl * sizeof(double), hipMemcpyDefault, c->stream), "copy fe");
  HIPCHECK(c, hipStreamSynchronize(c->stream), "element blocks");
  dfree(c, kd);
  dfree(c, fd);
  return LGDM_OK;
}

lgdm_status lgdm_kernel_times(lgdm_ctx* c, int32_t reps, double* avg_ms) {
  if (!c || !avg_ms || reps <= 0) return fail(c, LGDM_ERR_INVALID_ARG, "bad arguments");
  if (!ready(c) || !c->assembled) return fail(c, LGDM_ERR_STATE, "assemble first");
  const MatParams mp = make_params(c->mat, c->dim);
  float ms = 0.f;
  for (int k = 0; k < 4; ++k) {
    HIPCHECK(c, hipEventRecord(c->ev[5], c->stream), "event");
    for (int r = 0; r < reps; ++r) {
      hipError_t e = hipSuccess;
      if (k == 0) e = launch_gp_kernel(c, mp);
      else if (k == 1) e = launch_node_kernel(c, mp, true);
      else if (k == 2) e = launch_spmv_only(c, c->x, nullptr);
      else e = krylov_setup(c);
      if (e != hipSuccess) return hip_fail(c, e, "kernel timing");
    }
    HIPCHECK(c, hipEventRecord(c->ev[6], c->stream), "event");
    HIPCHECK(c, hipEventSynchronize(c->ev[6]), "event");
    HIPCHECK(c, hipEventElapsedTime(&ms, c->ev[5], c->ev[6]), "event time");
    avg_ms[k] = ms / reps;
  }
  return LGDM_OK;
}

lgdm_status lgdm_probe_start(lgdm_ctx* c, int32_t kind) {
  if (!c || kind < 0 || kind >= PROBE_KINDS) return fail(c, LGDM_ERR_INVALID_ARG, "bad probe kind");
  probe_release(c);
  auto* p = new KernelProbe();
  p->kind = kind;
  for (int i = 0; i < 128; ++i) {
    // timing-only events: no system-scope fence (cache writeback and
    // invalidation) around the timed launches
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) break;
    p->pool.push_back(e);
  }
  c->probe = p;
  if (p->pool.size() < 2) {
    probe_release(c);
    return fail(c, LGDM_ERR_DEVICE, "could not create probe events");
  }
  return LGDM_OK;
}

lgdm_status lgdm_probe_stop(lgdm_ctx* c, double* avg_ms, int64_t* count) {
  if (!c || !avg_ms || !count) return fail(c, LGDM_ERR_INVALID_ARG, "bad arguments");
  *avg_ms = 0.0;
  *count = 0;
  if (!c->probe) return fail(c, LGDM_ERR_STATE, "no probe running");
  probe_harvest(*c->probe, true);
  *count = c->probe->count;
  *avg_ms = c->probe->count > 0 ? c->probe->sum_ms / c->probe->count : 0.0;
  probe_release(c);
  return LGDM_OK;
}

lgdm_status lgdm_amg_levels(lgdm_ctx* c, int32_t max_levels, int64_t* nodes, int32_t* n_levels) {
  if (!c || !n_levels || max_levels < 0 || (max_levels > 0 && !nodes)) return fail(c, LGDM_ERR_INVALID_ARG, "bad arguments");
  AmgInfo info;
  amg_info(c, info);
  *n_levels = info.levels;
  for (int l = 0; l < info.levels && l < max_levels; ++l) nodes[l] = info.nodes[l];
  return LGDM_OK;
}

lgdm_status lgdm_footprint(lgdm_ctx* c, int64_t* bytes) {
  if (!c || !bytes) return LGDM_ERR_INVALID_ARG;
  int64_t s = 0;
  for (auto& a : c->allocs) s += (int64_t)a.second;
  *bytes = s;
  return LGDM_OK;
}

}  // extern "C"
