// Internal declarations of the LGDM HIP library: the context, device-side
// parameter structs and the launch wrappers each translation unit exports.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <memory>
#include <string>
#include <cmath>
#include <vector>

#include "lgdm.h"

namespace lgdm {

// Material constants as the kernels need them (Eq. 1, Appendix A).
struct MatParams {
  double lam, mu;        // Lame constants of the element law (plane stress: lambda*)
  double E;              // 1D modulus
  double nu, kappa0, alpha, beta, c, R, eta, h, tol_hist, tol_dmg;
  double c1, c2, c3, k;  // modified von Mises coefficients (A.3)
  double ezz_fac;        // plane stress: eps_zz = ezz_fac (eps_xx + eps_yy); else 0
  double thick;          // thickness (2D) / area (1D); 1 in 3D
  double g_den;          // 1 - exp(-eta)
  double sq_guard;       // coupling variant: no second derivative of A.3 where sqrt(s) <= this
  int coupling;          // LGDM_COUPLING_EXECUTED or LGDM_COUPLING_EQ2
};

// Record layout of one Gauss point written by the Gauss-point kernel and
// read by the node-row assembly kernel.  Tensor components are stored as
// symmetric tensor entries (not engineering shears): 2D (xx, yy, xy),
// 3D (xx, yy, zz, xy, yz, xz).  The coupling variant (CPL: the stress of
// Eq. 2) appends d eeq / d eps unscaled, the two coefficients of the second
// derivative of A.3 and q = ds / deps of its square-root argument s (3D
// tensor entries; in 2D xx, yy, xy, zz).
template <int DIM, bool CPL = false> struct Rec {
  static constexpr int NS = DIM == 1 ? 1 : (DIM == 2 ? 3 : 6);
  static constexpr int JINV = 0;                 // J^-1 [DIM*DIM], (J^-1)_{j d}
  static constexpr int CUU = DIM * DIM;          // wJ (1 - D) s_e
  static constexpr int CUE = CUU + 1;            // wJ D' chi s_e
  static constexpr int S = CUE + 1;              // C : eps (unscaled stress) [NS]
  static constexpr int GH = S + NS;              // wJ h d eeq / d eps [NS]
  static constexpr int GB = GH + NS;             // grad ebar [DIM]
  static constexpr int CEE = GB + DIM;           // wJ h
  static constexpr int CGP = CEE + 1;            // wJ h c g' D' chi
  static constexpr int CG = CGP + 1;             // wJ g h c
  static constexpr int RE = CG + 1;              // wJ h (ebar - eeq)
  static constexpr int FR = RE + 1;              // wJ h eeq
  static constexpr int NQ = DIM == 1 ? 0 : (DIM == 2 ? 4 : 6);
  static constexpr int GU = FR + 1;              // CPL: d eeq / d eps [NS] (plane stress: chained through eps_zz)
  static constexpr int AL = GU + NS;             // CPL: 1 / (4 k sqrt(s)), 0 where sqrt(s) <= guard
  static constexpr int BE = AL + 1;              // CPL: 1 / (8 k s^(3/2)), likewise
  static constexpr int Q = BE + 1;               // CPL: q = 2 c2^2 I1 1 + c3 dev(eps) [NQ]
  static constexpr int USED = CPL ? Q + NQ : FR + 1;
  static constexpr int STRIDE = CPL ? (DIM == 1 ? 16 : (DIM == 2 ? 28 : 48))
                                    : (DIM == 1 ? 12 : (DIM == 2 ? 20 : 32));
  static_assert(USED <= STRIDE, "record stride");
};

// doubles per Gauss-point record of a context
inline int rec_stride(int dim, bool cpl) {
  if (cpl) return dim == 1 ? Rec<1, true>::STRIDE : (dim == 2 ? Rec<2, true>::STRIDE : Rec<3, true>::STRIDE);
  return dim == 1 ? Rec<1>::STRIDE : (dim == 2 ? Rec<2>::STRIDE : Rec<3>::STRIDE);
}

// arguments of the Gauss-point kernel for one problem
struct GpArgs {
  int64_t ngauss;
  const double* coords;
  const int32_t* conn;
  const double* e_scale;
  const double* x;
  const double* kappa_n;
  double* rec;
  double* kappa_t;
  double* D_t;
  double* eeq_t;       // [ngauss] local equivalent strain of A.3 at this assembly
};

// arguments of the node-row assembly kernel for one problem
struct NodeArgs {
  int64_t n_nodes;
  const int32_t* n2e_ptr;
  const int32_t* n2e;
  const int32_t* nbr_ptr;
  const int32_t* nbr;
  const uint8_t* pos;
  const int32_t* row_ptr;
  const uint8_t* flags;
  const double* rec;
  void* vals;          // double* (FP64) or float* (mixed)
  double* R;
  double* partials;
};

// one problem of a fused multi-problem launch: its arguments and the first
// workgroup of its range in the fused grids
struct SlotDesc {
  GpArgs gp;
  NodeArgs node;
  MatParams mp;
  int64_t gp_block0;
  int64_t node_block0;
};

// node -> element list entries: (element << N2E_SHIFT) | local node
constexpr int N2E_SHIFT = 4;
constexpr int N2E_MASK = (1 << N2E_SHIFT) - 1;

constexpr int NORM_SLOTS = 6;  // |R_u|^2, |R_e|^2, |f_u|^2, |fref_e|^2, reaction, non-finite count
constexpr int RED_CHUNKS = 1024;  // stage-one workgroups of the two-stage reductions
// Krylov workspace: IDR(8) needs r, v, t and 8 + 8 direction vectors; the
// last vector holds the best iterate.  BiCGSTAB uses the first 8.
constexpr int IDR_SMAX = 8;
constexpr int KV_VECS = 3 + 2 * IDR_SMAX + 1;
constexpr int KSCAL_DOUBLES = 128;     // device scalar slots of a solve
constexpr int KPART_PER_BLOCK = 16;    // partial sums per workgroup (at most 4 + IDR_SMAX)
constexpr int KPART_BLOCKS = 2048;     // workgroups of a Krylov vector kernel, at most
constexpr int KSLOT_DONE = 9;          // device scalar slot of a solve's done flag

struct Amg;   // aggregation-multigrid hierarchy of a context (amg.hip)
struct Zone;  // process-zone block of the multigrid preconditioner (zone.hip)

// Live timing of one kernel inside the solves: HIP event pairs around its
// launches on the context's stream, harvested without blocking.
enum ProbeKind { PROBE_IDR_SPMV = 0, PROBE_MG_FINEST = 1, PROBE_KINDS = 2 };
struct KernelProbe {
  int kind = -1;
  std::vector<hipEvent_t> pool;                               // free events
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;    // recorded, in launch order
  hipEvent_t open0 = nullptr, open1 = nullptr;                // the launch being recorded
  double sum_ms = 0.0;
  int64_t count = 0;
};

}  // namespace lgdm

struct lgdm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int precision = LGDM_FP64;
  void* (*alloc_fn)(size_t, void*) = nullptr;
  void (*free_fn)(void*, void*) = nullptr;
  void* alloc_user = nullptr;
  std::string err;
  std::vector<std::pair<void*, size_t>> allocs;  // every live device allocation

  // mesh and pattern (H0)
  int dim = 0, nen = 0, ngp = 0, nd = 0;
  bool order2 = false;          // mixed-order elements (line3 / quad9 u, linear ebar on the vertices)
  int nen_e = 0;                // ebar nodes per element (the first nen_e of each element's list)
  std::vector<uint8_t> base_flags;  // per dof: constraints of the mesh itself (ebar of non-vertex nodes)
  int64_t n_nodes = 0, n_elems = 0, ndof = 0, ngauss = 0, nnz = 0, npairs = 0;
  int max_elem_per_node = 0, max_nbr = 0;
  double* coords = nullptr;
  int32_t* conn = nullptr;
  double* e_scale = nullptr;
  int32_t* n2e_ptr = nullptr;   // node -> element list offsets [n_nodes + 1]
  int32_t* n2e = nullptr;       // (element << 3) | local node, ascending element
  int32_t* nbr_ptr = nullptr;   // node graph offsets [n_nodes + 1]
  int32_t* nbr = nullptr;       // neighbour node ids, ascending [npairs]
  int32_t* dpos = nullptr;      // position of the node itself in its neighbour list
  uint8_t* pos = nullptr;       // [n_elems * nen * nen] position of node b in node a's list
  int32_t* row_ptr = nullptr;
  int32_t* col_idx = nullptr;

  // boundary conditions
  uint8_t* dof_flags = nullptr;  // bit0 constrained (Dirichlet, or an ebar dof of a non-vertex node),
                                 // bit1 loaded (nonzero reference value), bit2 ebar dof of a non-vertex node
  int32_t* bc_dofs = nullptr;
  double* bc_vals = nullptr;
  int64_t nbc = 0;

  // material
  lgdm_material mat{};
  bool has_mat = false;

  // state (H2, H7)
  double* x = nullptr;
  double* x_save = nullptr;
  double* kappa_n = nullptr;
  double* D_n = nullptr;
  double* kappa_t = nullptr;
  double* D_t = nullptr;
  int64_t increment = 0;
  bool in_increment = false;
  bool assembled = false;

  // assembly outputs (H3-H5)
  double* rec = nullptr;
  int rec_stride = 0;     // doubles per Gauss-point record in `rec`
  double* vals = nullptr;
  float* vals32 = nullptr;
  double* R = nullptr;
  double* partials = nullptr;
  int64_t n_partials = 0;
  double* norms_dev = nullptr;     // NORM_SLOTS
  double* red2 = nullptr;          // stage-one totals of the two-stage reductions
  double* norms_host = nullptr;    // pinned
  double last_norms[lgdm::NORM_SLOTS] = {0, 0, 0, 0, 0, 0};

  // Krylov workspace (H6)
  double* kv = nullptr;            // KV_VECS FP64 Krylov vectors (the last: best iterate), ndof each
  double* minv = nullptr;          // block-Jacobi inverses [n_nodes * nd * nd]
  float* minv32 = nullptr;
  double* kpart = nullptr;         // per-block partial sums
  int64_t n_kpart = 0;
  double* kscal = nullptr;         // device scalars
  double* kscal_host = nullptr;    // pinned copy
  unsigned int* kcount = nullptr;  // last-block counters
  double* delta = nullptr;
  lgdm::Amg* amg = nullptr;         // multigrid hierarchy (built at the first multigrid solve)
  lgdm::Zone* zone = nullptr;       // process-zone solve of the multigrid preconditioner
  bool noalloc_call = false;        // inside lgdm_solve_linear_noalloc: nothing may be allocated
  lgdm::KernelProbe* probe = nullptr;  // live kernel timing (measurement aid)
  bool amg_unavailable = false;     // the mesh has no usable hierarchy (default: block-Jacobi)
  bool last_solve_improved = true;  // the last linear solve returned a better-than-zero correction
  int nw_iter = 0;                  // Newton corrections of the current increment
  bool nw_stepped = false;          // x holds a correction not yet judged by the line search
  double nw_phi = 0.0;              // merit of the iterate the last correction started from
  double nw_alpha = 1.0;            // fraction of that correction x holds
  int nw_cuts = 0;                  // halvings of it so far
  double nw_best_phi = 0.0;         // smallest merit of the increment's iterates
  int nw_since_best = 0;            // iterates since that one
  double inc_lambda = 0.0;          // load factor of the current increment
  int64_t inc_serial = 0;           // counts lgdm_begin_increment calls
  bool inc_zone_used = false;       // a solve of this increment used the process zone
  int inc_zone_tier = 0;            // restarts of this increment: 0 zone from zone_damage,
                                    // 1 from 1 - (1 - zone_damage) / 10, 2 no zone
  bool zone_may_reuse = false;      // the running solve may keep the zone's inverse
  int64_t inc_krylov = 0;           // Krylov iterations spent in the current increment
  double inc_t0 = 0.0;              // host time the current increment began (lgdm::host_seconds)
  double solve_deadline = 0.0;      // host time a running solve must stop by (0: none)
  double* eeq_t = nullptr;          // [ngauss] equivalent strain (A.3) of the last assembly

  hipEvent_t ev[8] = {};
  bool events_ready = false;
};

namespace lgdm {

// monotonic host clock in seconds (work bounds of an increment)
inline double host_seconds() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// allocation helpers (capi.cpp)
void* dalloc(lgdm_ctx* c, size_t bytes);
void dfree(lgdm_ctx* c, void* p);

// H0 (pattern.hip)
hipError_t build_pattern(lgdm_ctx* c, std::string& msg, int& status);

// H1-H5 (element.hip)
MatParams make_params(const lgdm_material& m, int dim);
hipError_t launch_gp_kernel(lgdm_ctx* c, const MatParams& mp);
hipError_t launch_node_kernel(lgdm_ctx* c, const MatParams& mp, bool want_k);
hipError_t launch_norm_reduce(lgdm_ctx* c);
hipError_t launch_norm_reduce_on(lgdm_ctx* c, hipStream_t st);
hipError_t launch_set_dirichlet(lgdm_ctx* c, double lambda);
hipError_t launch_damage_from_kappa(lgdm_ctx* c, const MatParams& mp);
hipError_t launch_element_blocks(lgdm_ctx* c, const MatParams& mp, int64_t e0, int64_t e1,
                                 double* Ke, double* fe);
hipError_t launch_max_reduce(lgdm_ctx* c, const double* v, int64_t n, double* out_dev);
int64_t node_kernel_blocks(const lgdm_ctx* c);
int64_t gp_kernel_blocks(const lgdm_ctx* c);
GpArgs gp_args(const lgdm_ctx* c);
NodeArgs node_args(const lgdm_ctx* c);
// mixed-order elements (mixed_order.hip)
int q_node_kernel_nodes_per_block(int dim);
hipError_t launch_q_gp_kernel(lgdm_ctx* c, const MatParams& mp);
hipError_t launch_q_node_kernel(lgdm_ctx* c, const MatParams& mp, bool want_k);
hipError_t launch_q_element_blocks(lgdm_ctx* c, const MatParams& mp, int64_t e0, int64_t e1, double* Ke,
                                   double* fe);
hipError_t launch_zero_flagged(lgdm_ctx* c, double* v, uint8_t mask);  // v[d] = 0 where flags[d] & mask
hipError_t launch_fused_assembly(hipStream_t st, int dim, bool mixed, const SlotDesc* slots_dev,
                                 int nslots, int64_t gp_blocks, int64_t node_blocks);

// H6 (krylov.hip)
struct KrylovResult {
  int status;          // LGDM_OK / LGDM_ERR_NAN / LGDM_ERR_BREAKDOWN / LGDM_ERR_NOT_CONVERGED
  int64_t iters;
  int restarts;
  double rel_u, rel_e;
  int64_t spmv;        // operator applications
  bool improved;       // the returned iterate is better than the zero start
};
// one linear solve as a state machine (see krylov.hip)
struct KrylovRun {
  virtual ~KrylovRun() = default;
  virtual hipError_t start() = 0;
  virtual hipError_t launch() = 0;
  virtual hipError_t check() = 0;
  virtual bool needs_check() const = 0;
  virtual bool finished() const = 0;
  virtual const KrylovResult& result() const = 0;
};
std::unique_ptr<KrylovRun> make_krylov_run(lgdm_ctx* c, const double* b, double* x,
                                           const lgdm_solver_opts& o, double tol_u, double tol_e);
// per-field relative tolerances of the next Newton correction
void newton_forcing(lgdm_ctx* c, const lgdm_solver_opts& o, double& tol_u, double& tol_e);
lgdm_solver_opts fill_opts(const lgdm_solver_opts* o);  // defaults for zero fields
// The linear solves of several requests of one serving batch (same element
// type and precision) as one IDR(s) run: every kernel of a cycle is one
// launch over all of them.  Buffers are owned by the batch.
struct BatchSolveBuffers {
  // device allocator of the batch (null: hipMalloc / hipFree)
  void* (*alloc_fn)(size_t, void*) = nullptr;
  void (*free_fn)(void*, void*) = nullptr;
  void* alloc_user = nullptr;
  void* table_dev = nullptr;    // per-request descriptors
  void* table_host = nullptr;   // pinned
  double* sc_dev = nullptr;     // [max_requests][KSCAL_DOUBLES]
  double* sc_host = nullptr;    // pinned
  double* one_host = nullptr;   // pinned constant 1.0
  double* part = nullptr;       // partial sums of a batched launch
  int max_requests = 0;
};
hipError_t batch_solve_alloc(BatchSolveBuffers& B, int max_requests);
void batch_solve_free(BatchSolveBuffers& B);
// A persistent batched run: requests join it with add() (tangent and
// block-Jacobi assembled; b = c->R, x = c->delta) and leave it when their
// solve ends (take_finished) or when removed; every advance() enqueues
// check_every iterations of all of them, reads their scalars and decides.
// Request ids are the batch's slot numbers (< B.max_requests).
struct BatchRun {
  virtual ~BatchRun() = default;
  virtual hipError_t add(int id, lgdm_ctx* c, double tol_u, double tol_e) = 0;
  virtual void remove(int id) = 0;
  virtual hipError_t advance() = 0;
  virtual int active() const = 0;
  // ids whose solves ended since the last call, with their results
  virtual void take_finished(std::vector<int>& ids, std::vector<KrylovResult>& res) = 0;
  virtual void set_opts(const lgdm_solver_opts& o) = 0;
};
// a run for contexts of nd unknowns per node and the given precision; null
// if the options do not select IDR(s)
std::unique_ptr<BatchRun> make_batch_run(hipStream_t st, int nd, bool mixed, const lgdm_solver_opts& o,
                                         BatchSolveBuffers& B);
hipError_t krylov_setup(lgdm_ctx* c);  // block-Jacobi from the assembled matrix
hipError_t krylov_solve(lgdm_ctx* c, const double* b, double* xout, const lgdm_solver_opts& o,
                        double tol_u, double tol_e, KrylovResult& res);
hipError_t launch_spmv_only(lgdm_ctx* c, const double* x, double* scratch);  // y = S K x
hipError_t launch_axpy(lgdm_ctx* c, double* y, const double* x, double a, int64_t n);

// Aggregation multigrid (amg.hip).  amg_setup builds the hierarchy's
// structure on the first call for a mesh (host aggregation of the node graph)
// and, on every call, the coarse operators of the current tangent (after
// krylov_setup).  amg_apply enqueues out = one V-cycle applied to in; it does
// nothing once sc[KSLOT_DONE] is set (sc may be null).  amg_release frees the
// host side (device memory belongs to the context's allocations).
hipError_t amg_setup(lgdm_ctx* c, std::string& msg);
hipError_t amg_apply(lgdm_ctx* c, const double* in, double* out, const double* sc, hipStream_t st);
hipError_t amg_cycle(lgdm_ctx* c, const double* in, double* out, const double* sc, hipStream_t st);
void amg_release(lgdm_ctx* c);
// Line search of the Newton corrections (single contexts and the batch):
// the merit of an assembly is the sum of the squared relative residuals of
// both fields; a correction that raised it more than LS_GROWTH-fold is
// halved, at most LS_MAX_CUTS times.
constexpr double LS_GROWTH = 4.0;
// iterations without a new smallest merit after which Newton with the
// process zone restarts the increment with a smaller zone
constexpr int ZONE_PATIENCE = 4;
constexpr int LS_MAX_CUTS = 4;
inline double newton_merit(const lgdm_ctx* c) {
  const double tiny = 1e-300;
  const double ru = std::sqrt(c->last_norms[0]), re = std::sqrt(c->last_norms[1]);
  const double fu = std::sqrt(c->last_norms[2]), fe = std::sqrt(c->last_norms[3]);
  const double a = ru / std::max(fu, tiny), b = re / std::max(fe, tiny);
  return a * a + b * b;
}
// Process zone (zone.hip): the loading, highly damaged elements of the
// current tangent, solved densely inside the multigrid preconditioner.
// zone_setup chooses and factors it (after amg_setup); with allow_alloc
// false it returns hipErrorNotReady instead of growing its buffers.
// With reuse, a zone whose node set equals the last one built in the same
// increment keeps its inverse; *factored tells whether it was rebuilt.
hipError_t zone_setup(lgdm_ctx* c, bool allow_alloc, bool reuse, double dmin, bool* factored, std::string& msg);
bool zone_active(const lgdm_ctx* c);
int64_t zone_dofs(const lgdm_ctx* c);
void zone_disable(lgdm_ctx* c);
void zone_forget(lgdm_ctx* c);  // the factors are not reused by a later tangent
hipError_t zone_apply(lgdm_ctx* c, const double* in, double* out, const double* sc, hipStream_t st);
void zone_release(lgdm_ctx* c);
// breadth-first levels of a graph (CSR adj_ptr / adj over n nodes), each
// component from a pseudo-peripheral node; returns the number of levels
int64_t zone_levels(int64_t n, const int64_t* adj_ptr, const int32_t* adj, int32_t* level);
struct AmgInfo {
  int levels;
  int64_t nodes[16];
  int64_t pairs[16];
};
void amg_info(const lgdm_ctx* c, AmgInfo& info);
hipError_t launch_field_norms(lgdm_ctx* c, const double* v, double* out_dev);  // |v_u|^2, |v_e|^2

// static scratch of the allocation-free linear solve (noalloc.hip)
hipError_t noalloc_init(int device);       // resolve the scratch address on `device` (current)
double* noalloc_scratch(int device);       // that address, or null before noalloc_init
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t st);

// around a launch of the kernel `kind` on st (no-ops unless that kind is probed)
void probe_before(lgdm_ctx* c, int kind, hipStream_t st);
void probe_after(lgdm_ctx* c, int kind, hipStream_t st);

}  // namespace lgdm
