// Continuous batching of LGDM simulation requests on one device: slots with
// resident per-request state, admission by HBM footprint, one fused launch of
// each element kernel per tick over all running requests, and one batched
// IDR(s) run over all the requests' linear solves (each kernel one launch
// over every request; BiCGSTAB runs instead go per request on per-slot
// streams, interleaved by the host).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "lgdm_internal.h"

using namespace lgdm;

namespace {

struct Slot {
  lgdm_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  int state = LGDM_SLOT_FREE;
  int64_t n_increments = 0;
  int64_t footprint = 0;
  bool in_increment = false;
  int newton = 0;               // solves in the current increment
  int64_t newton_total = 0, krylov_total = 0, assemblies_total = 0;
  double max_damage = 0.0;
  int last_status = LGDM_OK;
  std::unique_ptr<KrylovRun> run;
  bool solving = false;
  double tol_u = 0.0, tol_e = 0.0;
  KrylovResult kres{};
  // line search: x holds the fraction alpha of the last correction, which
  // started from an iterate of merit phi_prev; halvings so far
  bool stepped = false;
  double phi_prev = 0.0, alpha = 1.0;
  int cuts = 0;
  // the current load step's second attempt, with the line-search setting
  // flipped; load steps retried so far
  bool ls_flip = false;
  int retries = 0;
  // load stepping inside an increment: the committed state sits at the
  // fraction f0 of increment `done` + 1, the step in progress goes to f1;
  // `cuts` halvings of this increment's steps so far
  int64_t done = 0;
  double f0 = 0.0, f1 = 1.0;
  int step_cuts = 0;
  int64_t cutbacks = 0;
};

constexpr int MAX_STEP_CUTS = 3;   // smallest load step: 1/8 of an increment

}  // namespace

struct lgdm_batch {
  int device = 0;
  hipStream_t stream = nullptr;
  int precision = LGDM_FP64;
  int dim = 0;                  // all requests of a batch share the element type
  int64_t budget = 0, used = 0;
  std::vector<Slot> slots;
  SlotDesc* desc_host = nullptr;  // pinned
  SlotDesc* desc_dev = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  BatchSolveBuffers bsolve;     // the batched IDR(s) run's buffers
  std::unique_ptr<BatchRun> run;  // requests whose linear solve is in progress (IDR(s))
  int run_s = 0, run_nd = 0;      // the run's shadow-space dimension and unknowns per node
  std::string err;
  // device allocator of the batch and of every request's context (null:
  // hipMalloc / hipFree)
  void* (*alloc_fn)(size_t, void*) = nullptr;
  void (*free_fn)(void*, void*) = nullptr;
  void* alloc_user = nullptr;
};

namespace {

lgdm_status bfail(lgdm_batch* b, lgdm_status s, const std::string& m) {
  if (b) b->err = m;
  return s;
}

#define BHIP(b, expr, where)                                                              \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return bfail(b, LGDM_ERR_DEVICE, std::string(where) + ": " +   \
                                                             hipGetErrorString(e_));      \
  } while (0)

bool converged(const lgdm_ctx* c, double tol) {
  const double tiny = 1e-300;
  return std::sqrt(c->last_norms[0]) <= tol * std::max(std::sqrt(c->last_norms[2]), tiny) &&
         std::sqrt(c->last_norms[1]) <= tol * std::max(std::sqrt(c->last_norms[3]), tiny);
}


void* batch_dalloc(lgdm_batch* b, size_t bytes) {
  void* p = nullptr;
  if (b->alloc_fn) return b->alloc_fn(bytes, b->alloc_user);
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void batch_dfree(lgdm_batch* b, void* p) {
  if (!p) return;
  if (b->free_fn) b->free_fn(p, b->alloc_user);
  else (void)hipFree(p);
}

void release(lgdm_batch* b, Slot& s) {
  if (s.ctx) {
    lgdm_destroy(s.ctx);
    s.ctx = nullptr;
  }
  if (s.stream) {
    (void)hipStreamDestroy(s.stream);
    s.stream = nullptr;
  }
  b->used -= s.footprint;
  s = Slot();
}

void fail_slot(lgdm_batch* b, int i, lgdm_status st);

// A load step that does not converge is tried once more from its start
// with the line-search setting flipped (full steps converge some load steps
// the line search does not, and the other way round); when that fails too,
// the step is halved (the request's committed state stays where it is), at
// most MAX_STEP_CUTS times per increment; then the request fails.
void retry_or_fail(lgdm_batch* b, int i, lgdm_status st) {
  Slot& s = b->slots[i];
  const bool retry = !s.ls_flip, cut = s.ls_flip && s.step_cuts < MAX_STEP_CUTS;
  if (st != LGDM_ERR_NOT_CONVERGED || !s.ctx || !(retry || cut)) {
    fail_slot(b, i, st);
    return;
  }
  if (s.solving && b->run) b->run->remove(i);
  s.solving = false;
  s.run.reset();
  lgdm_abort_increment(s.ctx);   // restores the committed state
  s.in_increment = false;        // the next tick begins the step again
  if (retry) {
    s.ls_flip = true;
    s.retries += 1;
  } else {
    s.ls_flip = false;
    s.f1 = 0.5 * (s.f0 + s.f1);
    s.step_cuts += 1;
    s.cutbacks += 1;
  }
}

void fail_slot(lgdm_batch* b, int i, lgdm_status st) {
  Slot& s = b->slots[i];
  if (s.solving && b->run) b->run->remove(i);
  s.state = LGDM_SLOT_FAILED;
  s.last_status = st;
  s.solving = false;
  s.run.reset();
  if (s.ctx) lgdm_abort_increment(s.ctx);
  s.in_increment = false;
}

}  // namespace

extern "C" {

lgdm_status lgdm_request_footprint(int32_t dim, int64_t n_nodes, int64_t n_elems, int32_t precision,
                                   int64_t* bytes) {
  if (!bytes || dim < 1 || dim > 3 || n_nodes <= 0 || n_elems <= 0) return LGDM_ERR_INVALID_ARG;
  const int64_t nd = dim + 1, nen = 1 << dim, ngp = 1 << dim;
  int64_t nbr = 1;
  for (int d = 0; d < dim; ++d) nbr *= 3;                       // structured bound
  const int64_t ndof = n_nodes * nd, ng = n_elems * ngp;
  const int64_t nnz = n_nodes * nbr * nd * nd;
  const int64_t sval = precision == LGDM_MIXED ? 4 : 8;
  const int64_t rs = dim == 1 ? Rec<1>::STRIDE : (dim == 2 ? Rec<2>::STRIDE : Rec<3>::STRIDE);
  int64_t s = 0;
  s += n_nodes * dim * 8 + n_elems * nen * 4 + n_elems * 8;     // mesh
  s += (n_nodes + 1) * 4 * 2 + n_elems * nen * 4 + n_nodes * nbr * 4 + n_nodes * 4;  // graph
  s += n_elems * nen * nen;                                     // positions
  s += (ndof + 1) * 4 + nnz * 4 + nnz * sval;                   // CSR
  s += ndof * 8 * (4 + KV_VECS) + ndof;                         // state, Krylov vectors, flags
  s += ng * 8 * 5 + ng * rs * 8;                                // Gauss-point state, records
  s += n_nodes * nd * nd * sval;                                // block-Jacobi
  s += ((int64_t)KPART_BLOCKS * KPART_PER_BLOCK + 1024 * 6 + KSCAL_DOUBLES + 64) * 8;  // partials, scalars
  s += ((n_nodes + 3) / 4 + 1) * 6 * 8;
  *bytes = s + (int64_t)64 * 256;                               // allocation rounding
  return LGDM_OK;
}

lgdm_status lgdm_batch_create(lgdm_batch** out, int32_t device, void* hip_stream, int32_t precision,
                              int32_t max_slots, int64_t hbm_budget_bytes) {
  if (!out || max_slots <= 0 || max_slots > 4096) return LGDM_ERR_INVALID_ARG;
  if (precision != LGDM_FP64 && precision != LGDM_MIXED) return LGDM_ERR_INVALID_ARG;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return LGDM_ERR_DEVICE;
  lgdm_batch* b = new (std::nothrow) lgdm_batch();
  if (!b) return LGDM_ERR_OOM;
  b->device = device;
  b->stream = (hipStream_t)hip_stream;
  b->precision = precision;
  b->slots.resize(max_slots);
  if (hbm_budget_bytes <= 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      delete b;
      return LGDM_ERR_DEVICE;
    }
    hbm_budget_bytes = (int64_t)fr;
  }
  b->budget = hbm_budget_bytes;
  if (hipHostMalloc((void**)&b->desc_host, max_slots * sizeof(SlotDesc), hipHostMallocDefault) != hipSuccess ||
      !(b->desc_dev = (SlotDesc*)batch_dalloc(b, max_slots * sizeof(SlotDesc))) ||
      hipEventCreate(&b->ev0) != hipSuccess || hipEventCreate(&b->ev1) != hipSuccess ||
      batch_solve_alloc(b->bsolve, max_slots) != hipSuccess) {
    lgdm_batch_destroy(b);
    return LGDM_ERR_DEVICE;
  }
  *out = b;
  return LGDM_OK;
}

lgdm_status lgdm_batch_destroy(lgdm_batch* b) {
  if (!b) return LGDM_ERR_INVALID_ARG;
  (void)hipSetDevice(b->device);
  for (auto& s : b->slots)
    if (s.ctx || s.stream) release(b, s);
  if (b->desc_host) (void)hipHostFree(b->desc_host);
  batch_dfree(b, b->desc_dev);
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
  b->run.reset();
  batch_solve_free(b->bsolve);
  delete b;
  return LGDM_OK;
}

const char* lgdm_batch_last_error(const lgdm_batch* b) { return b ? b->err.c_str() : "null batch"; }

lgdm_status lgdm_batch_set_allocator(lgdm_batch* b, void* (*alloc)(size_t, void*), void (*free_fn)(void*, void*),
                                     void* user) {
  if (!b) return LGDM_ERR_INVALID_ARG;
  if ((alloc == nullptr) != (free_fn == nullptr))
    return bfail(b, LGDM_ERR_INVALID_ARG, "alloc and free must both be given or both be NULL");
  for (auto& s : b->slots)
    if (s.state != LGDM_SLOT_FREE) return bfail(b, LGDM_ERR_STATE, "set the allocator before admitting requests");
  BHIP(b, hipSetDevice(b->device), "set device");
  BHIP(b, hipStreamSynchronize(b->stream), "sync");
  // the batch's own device buffers move to the new allocator
  b->run.reset();
  batch_dfree(b, b->desc_dev);
  b->desc_dev = nullptr;
  batch_solve_free(b->bsolve);
  b->alloc_fn = alloc;
  b->free_fn = free_fn;
  b->alloc_user = user;
  b->bsolve.alloc_fn = alloc;
  b->bsolve.free_fn = free_fn;
  b->bsolve.alloc_user = user;
  b->desc_dev = (SlotDesc*)batch_dalloc(b, b->slots.size() * sizeof(SlotDesc));
  if (!b->desc_dev || batch_solve_alloc(b->bsolve, (int)b->slots.size()) != hipSuccess)
    return bfail(b, LGDM_ERR_OOM, "device allocation failed (batch buffers)");
  return LGDM_OK;
}

lgdm_status lgdm_batch_admit(lgdm_batch* b, const lgdm_request* r, int32_t* slot_out) {
  if (!b || !r || !slot_out) return bfail(b, LGDM_ERR_INVALID_ARG, "NULL argument");
  if (b->dim != 0 && r->dim != b->dim) {
    // the slots may have emptied: the batch takes the element type of its next request
    bool any = false;
    for (auto& s : b->slots) any |= s.state != LGDM_SLOT_FREE;
    if (any) return bfail(b, LGDM_ERR_INVALID_ARG, "all requests of a batch share one element type");
  }
  if (r->n_increments <= 0) return bfail(b, LGDM_ERR_INVALID_ARG, "n_increments must be positive");
  if (r->elem_type != r->dim)
    return bfail(b, LGDM_ERR_INVALID_ARG, "the batch serves equal-order elements (LINE2 / QUAD4 / HEX8)");
  int64_t est = 0;
  if (lgdm_request_footprint(r->dim, r->n_nodes, r->n_elems, b->precision, &est) != LGDM_OK)
    return bfail(b, LGDM_ERR_INVALID_ARG, "bad request sizes");
  int free_slot = -1;
  for (int i = 0; i < (int)b->slots.size(); ++i)
    if (b->slots[i].state == LGDM_SLOT_FREE) {
      free_slot = i;
      break;
    }
  if (free_slot < 0) return bfail(b, LGDM_ERR_BUSY, "no free slot");
  if (b->used + est > b->budget) return bfail(b, LGDM_ERR_BUSY, "HBM budget exhausted");
  if (r->material.coupling != LGDM_COUPLING_EXECUTED)
    return bfail(b, LGDM_ERR_INVALID_ARG, "the batch serves the executed-code coupling only");
  Slot& s = b->slots[free_slot];
  BHIP(b, hipSetDevice(b->device), "set device");
  BHIP(b, hipStreamCreate(&s.stream), "slot stream");
  lgdm_status st = lgdm_create(&s.ctx, b->device, s.stream, b->precision);
  if (st == LGDM_OK && b->alloc_fn) st = lgdm_set_allocator(s.ctx, b->alloc_fn, b->free_fn, b->alloc_user);
  if (st == LGDM_OK) st = lgdm_upload_mesh(s.ctx, r->dim, r->elem_type, r->n_nodes, r->coords, r->n_elems,
                                           r->conn, r->e_scale);
  if (st == LGDM_OK) st = lgdm_set_material(s.ctx, &r->material);
  if (st == LGDM_OK) st = lgdm_set_dirichlet(s.ctx, r->n_bc, r->bc_dofs, r->bc_values);
  if (st != LGDM_OK) {
    std::string m = s.ctx ? s.ctx->err : std::string("context creation failed");
    release(b, s);
    return bfail(b, st, "admission: " + m);
  }
  int64_t fp = 0;
  lgdm_footprint(s.ctx, &fp);
  s.footprint = fp;
  b->used += fp;
  s.state = LGDM_SLOT_RUNNING;
  s.n_increments = r->n_increments;
  b->dim = r->dim;
  *slot_out = free_slot;
  return LGDM_OK;
}

lgdm_status lgdm_batch_tick(lgdm_batch* b, const lgdm_solver_opts* o, lgdm_tick_report* rep) {
  if (!b) return LGDM_ERR_INVALID_ARG;
  const auto t0 = std::chrono::steady_clock::now();
  const lgdm_solver_opts op = fill_opts(o);
  const bool idr = op.krylov_method != LGDM_KRYLOV_BICGSTAB;
  lgdm_tick_report R{};
  BHIP(b, hipSetDevice(b->device), "set device");
  // the batched IDR(s) run persists across ticks; it is rebuilt only when
  // it is empty and the options or the element type changed
  if (idr && b->dim != 0 && (!b->run || ((b->run_s != op.idr_s || b->run_nd != b->dim + 1) &&
                                           b->run->active() == 0))) {
    b->run.reset();
    b->run = make_batch_run(b->stream, b->dim + 1, b->precision == LGDM_MIXED, op, b->bsolve);
    b->run_s = op.idr_s;
    b->run_nd = b->dim + 1;
  }
  if (b->run) b->run->set_opts(op);
  // 1. requests between Newton iterations: those between increments start
  //    their next load step
  std::vector<int> act;
  int running = 0;
  for (int i = 0; i < (int)b->slots.size(); ++i) {
    Slot& s = b->slots[i];
    if (s.state != LGDM_SLOT_RUNNING) continue;
    running++;
    if (s.solving) continue;
    if (!s.in_increment) {
      const double lam = ((double)s.done + s.f1) / (double)s.n_increments;
      lgdm_status st = lgdm_begin_increment(s.ctx, lam);
      if (st != LGDM_OK) {
        fail_slot(b, i, st);
        continue;
      }
      s.in_increment = true;
      s.newton = 0;
      s.stepped = false;
    }
    act.push_back(i);
  }
  for (int i : act) BHIP(b, hipStreamSynchronize(b->slots[i].stream), "slot sync");
  R.running = running;
  // 2. one fused launch of each element kernel over those requests
  if (!act.empty()) {
    int64_t gpb = 0, nodeb = 0;
    for (size_t j = 0; j < act.size(); ++j) {
      lgdm_ctx* c = b->slots[act[j]].ctx;
      SlotDesc& d = b->desc_host[j];
      d.gp = gp_args(c);
      d.node = node_args(c);
      d.mp = make_params(c->mat, c->dim);
      d.gp_block0 = gpb;
      d.node_block0 = nodeb;
      gpb += gp_kernel_blocks(c);
      nodeb += node_kernel_blocks(c);
      R.gauss_points += c->ngauss;
    }
    BHIP(b, hipMemcpyAsync(b->desc_dev, b->desc_host, act.size() * sizeof(SlotDesc), hipMemcpyHostToDevice,
                           b->stream), "slot table");
    BHIP(b, hipEventRecord(b->ev0, b->stream), "event");
    BHIP(b, launch_fused_assembly(b->stream, b->dim, b->precision == LGDM_MIXED, b->desc_dev, (int)act.size(),
                                  gpb, nodeb), "fused assembly");
    BHIP(b, hipEventRecord(b->ev1, b->stream), "event");
    for (int i : act) {
      lgdm_ctx* c = b->slots[i].ctx;
      BHIP(b, launch_norm_reduce_on(c, b->stream), "norms");
      BHIP(b, hipMemcpyAsync(c->norms_host, c->norms_dev, NORM_SLOTS * sizeof(double), hipMemcpyDeviceToHost,
                             b->stream), "norms");
    }
    BHIP(b, hipStreamSynchronize(b->stream), "fused assembly");
    float ms = 0.f;
    BHIP(b, hipEventElapsedTime(&ms, b->ev0, b->ev1), "event time");
    R.t_assembly_ms = ms;
  }
  // 3. per-request decisions: commit, fail, or start a solve
  std::vector<int> solve;
  for (int i : act) {
    Slot& s = b->slots[i];
    lgdm_ctx* c = s.ctx;
    std::memcpy(c->last_norms, c->norms_host, sizeof(c->last_norms));
    c->assembled = true;
    s.assemblies_total++;
    if (c->last_norms[5] != 0.0 || !std::isfinite(c->last_norms[0]) || !std::isfinite(c->last_norms[1])) {
      fail_slot(b, i, LGDM_ERR_NAN);
      continue;
    }
    const bool line_search = (op.line_search == LGDM_LINE_SEARCH_ON) != s.ls_flip;
    if (line_search && s.stepped && !converged(c, op.tol_newton) &&
        newton_merit(c) > LS_GROWTH * s.phi_prev && s.cuts < LS_MAX_CUTS) {
      // the correction raised the merit more than fourfold: halve it; the
      // trial is assembled at the next tick like an iterate
      BHIP(b, launch_axpy(c, c->x, c->delta, -0.5 * s.alpha, c->ndof), "line search");
      s.alpha *= 0.5;
      s.cuts += 1;
      continue;
    }
    s.stepped = false;
    if (converged(c, op.tol_newton)) {
      BHIP(b, launch_max_reduce(c, c->D_t, c->ngauss, c->norms_dev + 12), "max damage");
      BHIP(b, hipMemcpyAsync(c->norms_host + 12, c->norms_dev + 12, sizeof(double), hipMemcpyDeviceToHost,
                             c->stream), "max damage");
      lgdm_status st = lgdm_commit_increment(c);   // synchronises the slot stream
      if (st != LGDM_OK) {
        fail_slot(b, i, st);
        continue;
      }
      s.max_damage = c->norms_host[12];
      s.in_increment = false;
      s.ls_flip = false;
      if (s.f1 >= 1.0) {
        // the increment is complete
        s.done += 1;
        s.f0 = 0.0;
        s.f1 = 1.0;
        s.step_cuts = 0;
        R.committed++;
      } else {
        // a sub-step: the next one takes the rest of the increment
        s.f0 = s.f1;
        s.f1 = 1.0;
      }
      if (s.done >= s.n_increments) {
        s.state = LGDM_SLOT_FINISHED;
        R.finished++;
      }
      continue;
    }
    if (s.newton >= op.max_newton) {
      retry_or_fail(b, i, LGDM_ERR_NOT_CONVERGED);
      continue;
    }
    BHIP(b, krylov_setup(c), "block-Jacobi setup");
    double tol_u = op.tol_krylov, tol_e = op.tol_krylov;
    newton_forcing(c, op, tol_u, tol_e);
    s.tol_u = tol_u;
    s.tol_e = tol_e;
    s.solving = true;
    R.solves++;
    solve.push_back(i);
  }
  // 4. the solves
  std::vector<int> done;
  if (idr && b->run) {
    // IDR(s): new solves join the persistent batched run (every kernel one
    // launch over all requests in it); rounds of check_every iterations run
    // until some solve ends, at most MAX_ROUNDS, so that a request's Newton
    // iterations follow its own solves rather than the slowest request's
    constexpr int MAX_ROUNDS = 16;
    for (int i : solve) {
      Slot& s = b->slots[i];
      BHIP(b, hipStreamSynchronize(s.stream), "block-Jacobi setup");
      BHIP(b, b->run->add(i, s.ctx, s.tol_u, s.tol_e), "batched Krylov start");
    }
    std::vector<int> ids;
    std::vector<KrylovResult> res;
    for (int round = 0; round < MAX_ROUNDS && b->run->active() > 0; ++round) {
      BHIP(b, b->run->advance(), "batched Krylov iterations");
      b->run->take_finished(ids, res);
      for (size_t k = 0; k < ids.size(); ++k) {
        b->slots[ids[k]].kres = res[k];
        done.push_back(ids[k]);
      }
      if (!done.empty()) break;
    }
  } else {
    // BiCGSTAB: one run per request on its own stream, interleaved by the host
    for (int i : solve) {
      Slot& s = b->slots[i];
      s.run = make_krylov_run(s.ctx, s.ctx->R, s.ctx->delta, op, s.tol_u, s.tol_e);
      BHIP(b, s.run->start(), "Krylov start");
    }
    bool pending = true;
    while (pending) {
      pending = false;
      for (int i : solve) {
        Slot& s = b->slots[i];
        BHIP(b, s.run->check(), "Krylov check");
        if (s.run->finished()) continue;
        pending = true;
        if (!s.run->needs_check()) BHIP(b, s.run->launch(), "Krylov iterations");
      }
    }
    for (int i : solve) {
      Slot& s = b->slots[i];
      BHIP(b, hipStreamSynchronize(s.stream), "Krylov");
      s.kres = s.run->result();
      s.run.reset();
      done.push_back(i);
    }
  }
  // 5. Newton update of the requests whose solves ended
  for (int i : done) {
    Slot& s = b->slots[i];
    if (!s.solving) continue;
    s.solving = false;
    R.krylov_iters += s.kres.iters;
    s.krylov_total += s.kres.iters;
    if (s.kres.status == LGDM_ERR_NAN) {
      fail_slot(b, i, LGDM_ERR_NAN);
      continue;
    }
    if (s.kres.status != LGDM_OK && !s.kres.improved) {
      // a correction no better than none would repeat this iteration unchanged
      retry_or_fail(b, i, LGDM_ERR_NOT_CONVERGED);
      continue;
    }
    BHIP(b, launch_axpy(s.ctx, s.ctx->x, s.ctx->delta, 1.0, s.ctx->ndof), "update");
    s.stepped = true;
    s.phi_prev = newton_merit(s.ctx);
    s.alpha = 1.0;
    s.cuts = 0;
    s.newton++;
    s.newton_total++;
  }
  for (int i : done)
    if (b->slots[i].stream) BHIP(b, hipStreamSynchronize(b->slots[i].stream), "slot sync");
  R.t_tick_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (rep) *rep = R;
  return LGDM_OK;
}

lgdm_status lgdm_batch_slot_info(lgdm_batch* b, int32_t slot, lgdm_slot_info* info) {
  if (!b || !info || slot < 0 || slot >= (int)b->slots.size()) return bfail(b, LGDM_ERR_INVALID_ARG, "slot");
  const Slot& s = b->slots[slot];
  lgdm_slot_info I{};
  I.state = s.state;
  I.newton_in_increment = s.newton;
  I.increment = s.done;
  I.n_increments = s.n_increments;
  I.newton_total = s.newton_total;
  I.krylov_total = s.krylov_total;
  I.assemblies_total = s.assemblies_total;
  I.n_gauss = s.ctx ? s.ctx->ngauss : 0;
  I.ndof = s.ctx ? s.ctx->ndof : 0;
  I.footprint_bytes = s.footprint;
  I.max_damage = s.max_damage;
  I.last_status = s.last_status;
  I.retries = s.retries;
  I.cutbacks = s.cutbacks;
  *info = I;
  return LGDM_OK;
}

lgdm_status lgdm_batch_query(lgdm_batch* b, int32_t slot, int32_t field, double* out, int64_t n) {
  if (!b || slot < 0 || slot >= (int)b->slots.size()) return bfail(b, LGDM_ERR_INVALID_ARG, "slot");
  Slot& s = b->slots[slot];
  if (!s.ctx) return bfail(b, LGDM_ERR_STATE, "empty slot");
  lgdm_status st = lgdm_query_state(s.ctx, field, out, n);
  if (st != LGDM_OK) b->err = s.ctx->err;
  return st;
}

lgdm_status lgdm_batch_retire(lgdm_batch* b, int32_t slot) {
  if (!b || slot < 0 || slot >= (int)b->slots.size()) return bfail(b, LGDM_ERR_INVALID_ARG, "slot");
  Slot& s = b->slots[slot];
  if (s.state == LGDM_SLOT_FREE) return bfail(b, LGDM_ERR_STATE, "slot is free");
  if (s.state == LGDM_SLOT_RUNNING) return bfail(b, LGDM_ERR_STATE, "request still running");
  release(b, s);
  return LGDM_OK;
}

lgdm_status lgdm_batch_usage(lgdm_batch* b, int64_t* used, int64_t* budget, int32_t* occupied) {
  if (!b) return LGDM_ERR_INVALID_ARG;
  if (used) *used = b->used;
  if (budget) *budget = b->budget;
  if (occupied) {
    int n = 0;
    for (auto& s : b->slots) n += s.state != LGDM_SLOT_FREE;
    *occupied = n;
  }
  return LGDM_OK;
}

}  // extern "C"
