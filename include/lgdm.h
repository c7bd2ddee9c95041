/*
 * lgdm.h -- C ABI of the MI355X localizing-gradient-damage (LGDM) hot path.
 *
 * The library solves the coupled displacement / micro-equivalent-strain
 * problem of the localizing gradient damage method by the incremental-
 * iterative Newton procedure of the paper's Algorithm 2: each Newton
 * iteration evaluates every Gauss point (Appendix A, Eqs. A.1-A.4), forms the
 * element tangent blocks and internal forces (Eqs. 11a-11f), assembles them
 * into a sparse unsymmetric CSR tangent and residual, solves Eq. 11 and
 * updates the primary fields; converged increments commit the history
 * variable (Eq. A.2).  The calls follow the paper's statement of the
 * problem (Algorithms 1-2, "Input: Geometry, Material properties, Loads and
 * boundary conditions; Output: Damage and Structural response").
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every call returns an lgdm_status; no exception crosses the ABI.
 *    lgdm_last_error(ctx) returns a message for the last failing call.
 *  - Host input arrays are copied; the caller keeps ownership.  Pointer
 *    arguments marked "host or device" may point to either (HIP unified
 *    addressing decides the copy direction).
 *  - Device arrays returned by the library are owned by the context and stay
 *    valid until the next call that changes the mesh or lgdm_destroy.
 *  - All device work is enqueued on the stream given to lgdm_create; calls
 *    that return host values synchronise that stream.
 *  - Indices are 0-based.  Counts in the ABI are int64; the library's CSR
 *    uses int32 indices and rejects meshes with nnz >= 2^31.
 *  - dofs are node-interleaved: dof = node * (dim + 1) + comp, with comp in
 *    [0, dim) the displacement components and comp = dim the
 *    micro-equivalent strain (ebar).
 *  - Gauss-point arrays are indexed element * 2^dim + g with
 *    g = i_xi + 2 i_eta + 4 i_zeta (2-point Gauss-Legendre per direction);
 *    mixed-order elements (LGDM_LINE3 / LGDM_QUAD9) have 3^dim points each.
 *  - One context per host thread.
 */
#ifndef LGDM_H
#define LGDM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lgdm_status;
enum {
  LGDM_OK = 0,
  LGDM_ERR_INVALID_ARG = 1,  /* bad argument or call order; nothing changed   */
  LGDM_ERR_OOM = 2,          /* device allocation failed                       */
  LGDM_ERR_DEVICE = 3,       /* HIP runtime error                              */
  LGDM_ERR_NOT_CONVERGED = 4,/* Newton did not converge; committed state kept  */
  LGDM_ERR_NAN = 5,          /* non-finite residual or solver scalar           */
  LGDM_ERR_BREAKDOWN = 6,    /* Krylov breakdown that restarts did not cure    */
  LGDM_ERR_STATE = 7,        /* call needs a mesh / material / state first     */
  LGDM_ERR_BUSY = 8          /* batch: no free slot or HBM budget right now    */
};

enum { LGDM_FP64 = 0, LGDM_MIXED = 1 };          /* precision of a context      */
/* Element types.  Equal-order elements interpolate u and ebar with the same
 * multilinear functions (2-point Gauss per direction).  The mixed-order
 * elements are the paper's 1D / 2D discretisation (Sec. 2.1 after Eqs. 9-10;
 * Secs. 3.1, 3.2): quadratic u, linear ebar on the element's vertices,
 * geometry from the quadratic element, 3-point Gauss-Legendre per direction
 * (points -sqrt(3/5), 0, sqrt(3/5); weights 5/9, 8/9, 5/9; point
 * g = i_xi + 3 i_eta, so Gauss-point arrays have 3^dim entries per element).
 *  LGDM_LINE3  dim 1: 3 nodes per element (left end, right end, midpoint);
 *              ebar on the two ends.
 *  LGDM_QUAD9  dim 2: 9 nodes (corners counter-clockwise from (-1, -1), the
 *              mid-side nodes of the edges 0-1, 1-2, 2-3, 3-0, the centre);
 *              ebar on the 4 corners.
 * With mixed-order elements the dof layout stays node-interleaved with
 * dim + 1 dofs per node: the ebar dof of a node that is no element's vertex
 * carries no unknown and is held at zero (identity row, zero column, zero
 * residual, like a Dirichlet dof; lgdm_set_state zeroes it).  Mixed-order
 * contexts use the executed-code coupling only, and the batch does not
 * serve them. */
enum { LGDM_LINE2 = 1, LGDM_QUAD4 = 2, LGDM_HEX8 = 3, LGDM_LINE3 = 4, LGDM_QUAD9 = 5 };
enum { LGDM_PLANE_STRESS = 0, LGDM_PLANE_STRAIN = 1 };

/* fields for lgdm_query_state */
enum {
  LGDM_FIELD_X = 0,        /* [ndof]  primary vector (u and ebar, interleaved)    */
  LGDM_FIELD_KAPPA = 1,    /* [nGP]   committed history variable kappa_n (A.2)    */
  LGDM_FIELD_DAMAGE = 2,   /* [nGP]   committed damage D(kappa_n) (A.1)           */
  LGDM_FIELD_KAPPA_TRIAL = 3, /* [nGP] kappa at the last assembly (A.2 update)    */
  LGDM_FIELD_DAMAGE_TRIAL = 4,/* [nGP] D at the last assembly                     */
  LGDM_FIELD_RESIDUAL = 5, /* [ndof]  R = -f_int of the last assembly, R_c = 0    */
  LGDM_FIELD_REACTION = 6, /* [1]     sum of f_int,u over loaded dofs (last asm.) */
  LGDM_FIELD_EEQ = 7       /* [nGP]   local equivalent strain eeq (modified von
                                      Mises, A.3) at the last assembly; after a
                                      converged increment, that of the committed
                                      state                                     */
};

/* Material and numerical parameters (Eq. 1 and Appendix A).
 *  E        undamaged Young's modulus            nu     Poisson's ratio
 *  kappa0   damage threshold (A.1)               alpha, beta  damage law (A.1)
 *  c        gradient parameter (Eq. 1)           R, eta interaction function (A.4)
 *  k        compressive / tensile strength ratio (A.3)
 *  h        coupling modulus (Eq. 1)
 *  tol_hist, tol_dmg  bands of the vectorised history / damage update (Fig. 8b):
 *           kappa <- ebar where ebar - kappa_n > tol_hist; D = 0 where
 *           kappa - kappa0 < tol_dmg.  0 reproduces A.1 / A.2 literally.
 *  plane    LGDM_PLANE_STRESS or LGDM_PLANE_STRAIN (2D only)
 *  coupling LGDM_COUPLING_EXECUTED (0): sigma = (1 - D) C : eps and Eq. 11b
 *           without its h term, the form the paper's executed code (Fig. 2)
 *           assembles.  LGDM_COUPLING_EQ2 (1): the stress of Eq. 2,
 *           sigma = (1 - D) C : eps + h (eeq - ebar) d eeq / d eps, Eq. 11b
 *           as printed, and K^uu of Eq. 11a plus the terms of the consistent
 *           linearisation of Eq. 2, int B^T h [n n^T + (eeq - ebar)
 *           d^2 eeq / d eps^2] B (n = d eeq / d eps; the second derivative of
 *           A.3 is dropped where sqrt(s) <= 1e-6 kappa0, s the square-root
 *           argument).  Single contexts only: the batch rejects it.
 *  thickness  out-of-plane thickness (2D) or cross-section area (1D); 3D ignores it. */
typedef struct lgdm_material {
  double E, nu, kappa0, alpha, beta, c, R, eta, k, h, tol_hist, tol_dmg;
  int32_t plane;
  int32_t coupling;
  double thickness;
} lgdm_material;
enum { LGDM_COUPLING_EXECUTED = 0, LGDM_COUPLING_EQ2 = 1 };

/* Krylov method of the linear solve of the Newton system (Eq. 11).  Both are
 * right-preconditioned (see lgdm_solver_opts.precond: aggregation multigrid
 * by default for IDR(s) on 3D meshes, per-node block-Jacobi otherwise) and
 * work on the same scaled operator; 0 selects the default, LGDM_KRYLOV_IDRS
 * with s = 8.
 *  LGDM_KRYLOV_BICGSTAB  BiCGSTAB (van der Vorst 1992): 2 operator
 *                        applications per iteration.
 *  LGDM_KRYLOV_IDRS      IDR(s) (Sonneveld & van Gijzen 2008, biorthogonal
 *                        variant 2011): one operator application per
 *                        iteration; s shadow vectors instead of BiCGSTAB's
 *                        one, which does not break down on the indefinite
 *                        tangents of the softening branch where BiCGSTAB
 *                        does. */
enum { LGDM_KRYLOV_DEFAULT = 0, LGDM_KRYLOV_BICGSTAB = 1, LGDM_KRYLOV_IDRS = 2 };

/* Right preconditioner of the linear solves of a single context.  0
 * (LGDM_PRECOND_DEFAULT) selects LGDM_PRECOND_AMG for IDR(s) solves on 3D
 * meshes that have a coarse level (more than 13 nodes), block-Jacobi
 * otherwise.  Batch solves always use block-Jacobi.
 *  LGDM_PRECOND_BLOCK_JACOBI  inverse of the (dim+1)x(dim+1) diagonal node
 *                             blocks of the scaled tangent.
 *  LGDM_PRECOND_AMG           one cycle of aggregation multigrid (3D meshes
 *                             with IDR(s) only, else LGDM_ERR_INVALID_ARG):
 *                             node aggregates of the node graph (built once
 *                             per mesh), on each aggregate the rigid-body
 *                             motions and a constant micro-equivalent strain
 *                             as the coarse basis (7 unknowns per coarse
 *                             node), Galerkin coarse operators P^T A P rebuilt
 *                             for every tangent.  Finest level: damped
 *                             block-Jacobi (weight 0.7) plus the coarse
 *                             correction, side by side; coarser levels:
 *                             V(1,1) with the same smoother; a dense inverse
 *                             on the coarsest level.  Block-Jacobi iteration
 *                             counts grow with the mesh size; these stay
 *                             nearly constant. */
enum { LGDM_PRECOND_DEFAULT = 0, LGDM_PRECOND_BLOCK_JACOBI = 1, LGDM_PRECOND_AMG = 2 };

/* Newton / Krylov options.  Zero-initialised fields take the defaults shown. */
typedef struct lgdm_solver_opts {
  int32_t max_newton;      /* 30     Newton iterations per increment                */
  int32_t max_krylov;      /* 20000  Krylov iterations per linear solve             */
  double tol_newton;       /* 1e-8   per-field ||R|| <= tol * max(||F||, tiny)      */
  double tol_krylov;       /* 1e-10  per-field ||r|| <= tol * ||b||                 */
  int32_t check_every;     /* 16     Krylov iterations between host convergence reads */
  int32_t max_restarts;    /* 8      Krylov restarts after breakdown                */
  int32_t krylov_method;   /* LGDM_KRYLOV_IDRS                                      */
  int32_t idr_s;           /* 8      IDR shadow-space dimension: 1, 2, 4 or 8 (other
                                     values round up to the next of these, max 8) */
  int32_t forcing;         /* LGDM_FORCING_ADAPTIVE                                 */
  int32_t precond;         /* LGDM_PRECOND_DEFAULT                                  */
  int32_t process_zone;    /* LGDM_ZONE_DEFAULT: with the multigrid preconditioner,
                              the exact process-zone solve (below)                  */
  int64_t max_increment_krylov;  /* 0 = no bound.  Krylov iterations summed over the
                                    solves of one increment (lgdm_begin_increment to
                                    commit / abort): each solve is limited to what is
                                    left (IDR(s) runs whole cycles of s + 1 steps and
                                    can pass it by up to s), and once it is spent the
                                    next Newton
                                    iteration returns LGDM_ERR_NOT_CONVERGED
                                    (lgdm_solve_increment then restores the
                                    committed state)                               */
  double max_increment_seconds;  /* 0 = no bound.  Host wall time of one increment,
                                    checked before every solve and at every host
                                    read of a solve (check_every iterations): a
                                    solve that runs out returns its best iterate,
                                    and the next Newton iteration returns
                                    LGDM_ERR_NOT_CONVERGED as above               */
  int32_t line_search;     /* LGDM_LINE_SEARCH_OFF: full Newton steps; _ON:
                              backtracking on a correction that blows the
                              residual up (below)                                  */
  double zone_damage;      /* 0.99   trial damage from which a loading element
                              joins the process zone (below); values outside
                              (0, 1) select the default                            */
} lgdm_solver_opts;

/* Tolerance of the linear solves inside Newton (lgdm_newton_iteration,
 * lgdm_solve_increment, the batch):
 *  LGDM_FORCING_ADAPTIVE  per field f, max(tol_krylov, min(0.5, m * tol_newton *
 *                         ||F_f|| / ||R_f||)) with m = 0.1 (FP64) or 0.01
 *                         (mixed): corrections far from convergence solve to
 *                         tol_krylov, the last ones only as far as the Newton
 *                         test needs.  From the 9th Newton iteration of an
 *                         increment on, tol_krylov is replaced by
 *                         min(tol_krylov, 1e-8): the inexact iterates of a
 *                         strongly nonlinear increment can cycle.
 *  LGDM_FORCING_FIXED     every correction to tol_krylov.
 * lgdm_solve_linear always solves to tol_krylov.  Convergence of Newton is
 * judged on the FP64 residual either way. */
enum { LGDM_FORCING_ADAPTIVE = 0, LGDM_FORCING_FIXED = 1 };

/* Process zone of the multigrid preconditioner (3D meshes).  Where damaged
 * Gauss points load in the current Newton iterate, the consistent tangent's
 * softening terms (the D' chi terms of Eqs. 11b and 11d) make S K indefinite
 * on those elements, and neither the smoother nor the rigid-body coarse space
 * of the cycle represents those modes.  With LGDM_ZONE_DEFAULT the
 * preconditioner solves that zone exactly before the cycle:
 *   zone   the nodes of the elements with a loading Gauss point of trial
 *          damage >= zone_damage (raised tenfold closer to 1, twice at most,
 *          while a level group below exceeds 4,096 unknowns or the factor
 *          panels 2.5 GiB; no zone beyond that);
 *   factor the zone's nodes in breadth-first levels (lgdm_zone_levels), which
 *          make its block Z of S K block tridiagonal; consecutive levels form
 *          groups of at least 512 unknowns; twisted block LU from both end
 *          groups toward the middle one, the two chains on two streams
 *          (the second issued from a host thread the library starts for the
 *          factorisation and joins before it returns), each
 *          Schur complement inverted (rocSOLVER getrf/getri) and multiplied
 *          into its off-diagonal blocks (rocBLAS gemm);
 *   apply  x_z = Z^-1 b_z by sweeps from both ends to the middle group and
 *          back out (one launch per pair of groups);
 *          r = b - S K x_z; out = x_z + (multigrid cycle)(r).
 * Inside a Newton increment the factors are rebuilt only when the zone's node
 * set changes (a later tangent of the increment with the same zone keeps
 * them; r and the cycle always use the current tangent);
 * LGDM_ZONE_EVERY_TANGENT rebuilds them for every tangent, and
 * lgdm_solve_linear always does.  Should Newton with the zone stop reducing
 * the merit of the line search (no new smallest value in 4 iterations), or
 * return a correction no better than none, the increment restarts from its
 * beginning with the zone's damage threshold moved tenfold closer to 1, and
 * should that stall too, without the zone (zone_restarts in the report).
 * The factors are allocated through the context's allocator the first time a
 * zone of that size occurs and kept.
 * LGDM_ZONE_OFF: the plain cycle. */
enum { LGDM_ZONE_DEFAULT = 0, LGDM_ZONE_OFF = 1, LGDM_ZONE_EVERY_TANGENT = 2 };

/* Safeguard of the Newton corrections (lgdm_newton_iteration,
 * lgdm_solve_increment, and lgdm_batch_tick, where each halved trial is
 * assembled at the request's next tick).  LGDM_LINE_SEARCH_OFF (the
 * default): full steps, Algorithm 2 as written.  LGDM_LINE_SEARCH_ON: with
 * the merit phi = (||R_u|| / ||F_u||)^2 + (||R_ebar|| / ||F_ebar||)^2 of an
 * assembly, the last correction is halved (x -= alpha/2 delta, one more
 * assembly each) while phi exceeds 4 times its value before that correction,
 * at most 4 times (alpha >= 1/16); the iterate is then kept whatever phi is.
 * A correction that at most doubles the residual is taken whole.  The
 * solution of an increment does not depend on the path to it (the history
 * variable of a trial state is max(kappa_n, eeq(trial)), Eq. A.2), but which
 * increments converge does: on brittle 2D plates of the serving stream the
 * line search converges increments that full steps do not, and on a
 * plane-strain 9-node plate it fails one that full steps converge. */
enum { LGDM_LINE_SEARCH_OFF = 0, LGDM_LINE_SEARCH_ON = 1 };

/* Per-increment / per-iteration report (the paper's time-per-iteration split
 * into assembly, solve and variable update, Sec. 3.1). */
typedef struct lgdm_increment_report {
  int32_t converged;
  int32_t newton_iters;    /* linear solves performed                              */
  int64_t krylov_iters;    /* Krylov iterations (IDR(s) or BiCGSTAB), summed over
                              the solves                                           */
  double res_u, res_e;     /* ||R_u||, ||R_ebar|| at the last assembly             */
  double ref_u, ref_e;     /* ||f_int,u||, ||int N h eeq|| at the last assembly     */
  double du_norm, de_norm; /* ||delta u||, ||delta ebar|| of the last solve        */
  double reaction;         /* sum of f_int,u over loaded dofs                      */
  double max_damage;       /* max over Gauss points of D at the last assembly      */
  double t_assembly_ms;    /* device time in assembly (H1-H5) over the increment   */
  double t_solve_ms;       /* device time in the linear solves                      */
  double t_update_ms;      /* device time in update / norms / commit               */
  int32_t n_assemblies;
  int32_t restarts;        /* Krylov restarts after breakdown, summed               */
  int32_t krylov_status;   /* status of the last linear solve (LGDM_OK, or the
                              NOT_CONVERGED / BREAKDOWN of an inexact correction
                              that Newton accepted)                                */
  int32_t inexact_solves;  /* solves accepted short of tol_krylov                  */
  double krylov_rel_u;     /* last solve: ||(S(b - A x))_u|| / ||(S b)_u||          */
  double krylov_rel_e;     /* last solve: the same for the ebar rows                */
  int64_t krylov_spmv;     /* operator applications (SpMV) in the linear solves     */
  int32_t precond_fallbacks; /* multigrid solves without progress, repeated with
                                block-Jacobi                                        */
  int32_t backtracks;      /* halvings of a Newton correction (line search)         */
  int64_t zone_dofs;       /* largest process zone solved exactly in the solves
                              (unknowns; 0: none), see LGDM_ZONE_DEFAULT           */
  double t_zone_ms;        /* host time choosing and factoring the process zones,
                              part of t_solve_ms                                    */
  int32_t zone_factorizations; /* process-zone blocks factored                      */
  int32_t zone_restarts;   /* restarts of the increment with a smaller zone or
                              none (see LGDM_ZONE_DEFAULT)                          */
  int32_t zone_errors;     /* process-zone factorizations that a rocBLAS / rocSOLVER
                              call refused; those solves ran with the plain cycle
                              (lgdm_last_error holds the call and status)          */
} lgdm_increment_report;

/* View of the assembled tangent.  Device pointers owned by the context. */
typedef struct lgdm_csr_view {
  int64_t nrows, nnz;
  const int32_t* row_ptr;  /* [nrows + 1]                                     */
  const int32_t* col_idx;  /* [nnz], ascending within each row                */
  const double* vals;      /* [nnz] FP64 values (FP64 contexts; else NULL)    */
  const float* vals32;     /* [nnz] FP32 values (mixed contexts; else NULL)   */
} lgdm_csr_view;

typedef struct lgdm_ctx lgdm_ctx;

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  precision: LGDM_FP64 or
 * LGDM_MIXED (FP32 tangent, preconditioner and inner SpMV; FP64 residual,
 * history/damage update, Krylov dot products and Newton update). */
lgdm_status lgdm_create(lgdm_ctx** out, int32_t device, void* hip_stream, int32_t precision);
lgdm_status lgdm_destroy(lgdm_ctx* ctx);
const char* lgdm_last_error(const lgdm_ctx* ctx);

/* Route the context's device allocations through a caller allocator (e.g.
 * PyTorch's caching allocator).  alloc(bytes, user) returns a device pointer
 * aligned to at least 32 bytes, or NULL; free(ptr, user) releases it.  Must
 * be called before lgdm_upload_mesh, which fails with LGDM_ERR_INVALID_ARG if
 * an allocation is not 32-byte aligned.  Without it the library uses
 * hipMalloc / hipFree. */
lgdm_status lgdm_set_allocator(lgdm_ctx* ctx, void* (*alloc)(size_t, void*),
                               void (*free_fn)(void*, void*), void* user);

/* Geometry and connectivity (the "Geometry" input of Algorithm 2) and the
 * once-per-mesh work: dof numbering, node graph, CSR pattern of all
 * element-coupled dof pairs (structural zeros kept), node-to-element lists
 * (Fig. 2 assembly hoisted out of the Newton loop).
 *  dim        1, 2 or 3; elem_type LGDM_LINE2 / LGDM_QUAD4 / LGDM_HEX8 matching dim,
 *             or the mixed-order LGDM_LINE3 (dim 1) / LGDM_QUAD9 (dim 2)
 *  coords     host, [n_nodes * dim] FP64, node-major
 *  conn       host, [n_elems * nen] int32 (nen = 2^dim; 3 / 9 for the mixed-order
 *             types), local node order line2 (x0, x1), quad4 counter-clockwise,
 *             hex8 bottom face then top face; line3 / quad9 as their enum says
 *  e_scale    host, [n_elems] factor on the elasticity tensor only, or NULL (1)
 * Resets the state (x = 0, kappa_n = 0, increment 0).  INVALID_ARG for bad
 * sizes, out-of-range node ids, a node shared by more elements or neighbours
 * than the kernels handle (see lgdm_last_error), or nnz >= 2^31. */
lgdm_status lgdm_upload_mesh(lgdm_ctx* ctx, int32_t dim, int32_t elem_type, int64_t n_nodes,
                             const double* coords, int64_t n_elems, const int32_t* conn,
                             const double* e_scale);

/* Material parameters ("Material properties" input).  INVALID_ARG if
 * E <= 0, nu outside (-1, 0.5), kappa0 <= 0, k <= 0, h <= 0, eta <= 0 or c < 0. */
lgdm_status lgdm_set_material(lgdm_ctx* ctx, const lgdm_material* m);

/* Dirichlet conditions on displacement dofs ("Loads and boundary
 * conditions"): u[dofs[i]] = lambda * ref_values[i] during the increment
 * with load factor lambda.  dofs, ref_values: host, [n].  Constrained rows and
 * columns of the tangent are identity, their residual entries zero.  Dofs
 * with a nonzero ref value are the loaded dofs whose internal forces sum to
 * the reaction.  INVALID_ARG for an ebar dof or an out-of-range dof. */
lgdm_status lgdm_set_dirichlet(lgdm_ctx* ctx, int64_t n, const int64_t* dofs,
                               const double* ref_values);

/* Algorithm 2 "Compute and Assemble K" and "Compute and Assemble F" at the
 * current state (x, kappa_n): Gauss-point update (Eqs. A.1-A.4), element
 * tangents (Eqs. 11a-d) and residual R = -f_int (Eqs. 11e-f), deterministic
 * assembly, Dirichlet rows/columns.  If lambda >= 0 the constrained dofs are
 * first set to lambda * ref.  K_out (nullable) receives a view of the CSR
 * tangent; R_out (nullable, host or device, [ndof]) receives R.  Stores the
 * trial kappa / D and the residual norms of this assembly. */
lgdm_status lgdm_assemble_tangent_residual(lgdm_ctx* ctx, double lambda, lgdm_csr_view* K_out,
                                           double* R_out);

/* Solve the assembled tangent K delta = b (Eq. 11, Algorithm 2 "Solve") with
 * the Krylov method and preconditioner the options select (default: IDR(8),
 * preconditioned by aggregation multigrid on 3D meshes and by per-node
 * block-Jacobi otherwise), to tol_krylov per field.  b, delta: host or
 * device, [ndof].  delta receives the solution; rep (nullable) receives
 * krylov_iters, krylov_spmv, restarts and the reached relative residuals.
 * Needs a prior assembly. */
lgdm_status lgdm_solve_linear(lgdm_ctx* ctx, const double* b, double* delta,
                              const lgdm_solver_opts* o, lgdm_increment_report* rep);

/* For callers that cannot allocate device memory while they run (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same solve as lgdm_solve_linear (same kernels, same preconditioner and
 * options, bitwise the same delta and report), with no device allocation in
 * the call.  lgdm_solve_linear allocates a solution buffer on every call;
 * this variant writes the solution straight into delta, and the solve's
 * scratch (the per-workgroup partial sums of its reductions and its device
 * scalars: 257 KiB, independent of the mesh size) lives in one static device
 * array of LGDM_NOALLOC_SCRATCH_BYTES per GPU, resolved at lgdm_create.
 *  - b, delta: DEVICE memory of ctx's device, [ndof] doubles each, delta
 *    aligned to 32 bytes (host pointers, other devices' memory and a
 *    misaligned delta are rejected with LGDM_ERR_INVALID_ARG).  b is read
 *    only and may alias delta.
 *  - The multigrid hierarchy is allocated at a context's first multigrid
 *    solve.  If the options select multigrid (the 3D default) and the
 *    hierarchy does not exist yet, the call returns LGDM_ERR_STATE and does
 *    nothing: run one lgdm_solve_linear / lgdm_solve_increment /
 *    lgdm_newton_iteration first, or select block-Jacobi.
 *  - The static array is shared by every call on one GPU and keeps the last
 *    call's contents (the call clears its device scalars first).  Calls that
 *    overlap on one GPU (several host threads, or contexts on different
 *    streams) race on it: the caller serialises them.
 *  - Errors as lgdm_solve_linear; LGDM_ERR_INVALID_ARG if the solve would
 *    need more scratch than the static array holds. */
#define LGDM_NOALLOC_SCRATCH_BYTES (1u << 20)
lgdm_status lgdm_solve_linear_noalloc(lgdm_ctx* ctx, const double* b, double* delta,
                                      const lgdm_solver_opts* o, lgdm_increment_report* rep);

/* One load increment of Algorithm 2 with load factor lambda: set the
 * constrained dofs, iterate {assemble, convergence test, solve, update}
 * until the per-field residual test holds, then commit the history variable
 * (Eq. A.2).  On LGDM_ERR_NOT_CONVERGED / NAN / BREAKDOWN the state returns to
 * the last committed increment.  o, rep nullable. */
lgdm_status lgdm_solve_increment(lgdm_ctx* ctx, double lambda, const lgdm_solver_opts* o,
                                 lgdm_increment_report* rep);

/* The same increment split into steps, so one Newton iteration can be
 * driven and timed on its own:
 *  lgdm_begin_increment   saves the committed state, sets u_c = lambda * ref;
 *  lgdm_newton_iteration  assembles; if the residual test holds sets
 *                         *converged = 1 and returns, else solves and
 *                         updates x (Algorithm 2 update of primary variables);
 *  lgdm_commit_increment  commits kappa_n and D from the last assembly;
 *  lgdm_abort_increment   restores the saved committed state. */
lgdm_status lgdm_begin_increment(lgdm_ctx* ctx, double lambda);
lgdm_status lgdm_newton_iteration(lgdm_ctx* ctx, const lgdm_solver_opts* o, int32_t* converged,
                                  lgdm_increment_report* rep);
lgdm_status lgdm_commit_increment(lgdm_ctx* ctx);
lgdm_status lgdm_abort_increment(lgdm_ctx* ctx);

/* Device views of the CSR pattern and connectivity (owned by ctx). */
lgdm_status lgdm_get_csr(lgdm_ctx* ctx, int64_t* nrows, int64_t* nnz, const int32_t** row_ptr,
                         const int32_t** col_idx);
lgdm_status lgdm_get_connectivity(lgdm_ctx* ctx, const int32_t** conn, int64_t* n_elems,
                                  int32_t* nen);
/* Sizes: ndof, number of Gauss points, committed increment count. */
lgdm_status lgdm_get_sizes(lgdm_ctx* ctx, int64_t* ndof, int64_t* n_gauss, int64_t* increment);

/* Copy a field (LGDM_FIELD_*) into out (host or device) of n entries; n must
 * equal the field's size. */
lgdm_status lgdm_query_state(lgdm_ctx* ctx, int32_t field, double* out, int64_t n);

/* Inject a state: x (host or device, [ndof]) and kappa_n (host or device,
 * [nGP]); either may be NULL to keep the current one.  D_n is recomputed
 * from kappa_n (A.1).  increment sets the committed increment counter. */
lgdm_status lgdm_set_state(lgdm_ctx* ctx, const double* x, const double* kappa_n,
                           int64_t increment);

/* Parity aid: element tangents and internal forces of elements [e0, e1) at
 * the last assembled state, in the node-interleaved local order
 * (local dof a * (dim + 1) + comp).  Ke_out: host or device,
 * [(e1 - e0) * (nen (dim+1))^2], row-major; fe_out: [(e1 - e0) * nen (dim+1)].
 * Either may be NULL.  Values are FP64 in both precisions. */
lgdm_status lgdm_debug_element_blocks(lgdm_ctx* ctx, int64_t e0, int64_t e1, double* Ke_out,
                                      double* fe_out);

/* Measurement aid: average device time (ms, HIP events on the context's
 * stream) of `reps` back-to-back launches of each hot kernel at the last
 * assembled state: avg_ms[0] Gauss-point kernel, [1] node-row assembly
 * kernel, [2] one SpMV with the assembled tangent, [3] block-Jacobi setup.
 * Leaves the assembled matrix and state unchanged. */
lgdm_status lgdm_kernel_times(lgdm_ctx* ctx, int32_t reps, double* avg_ms);

/* Measurement aid: live timing of one kernel inside the linear solves.
 * lgdm_probe_start records a pair of HIP events around every launch of that
 * kernel on the context's stream (at most 64 launches in flight are
 * recorded; later ones are skipped until earlier pairs complete);
 * lgdm_probe_stop waits for them and returns the average duration (ms) and
 * the number of launches timed.  Kinds: LGDM_PROBE_IDR_SPMV, the operator
 * application of an IDR(s) step with its shadow-vector dot products;
 * LGDM_PROBE_MG_FINEST, the finest-level kernel of the multigrid cycle
 * (block-Jacobi plus the prolongated coarse correction).  Starting a probe
 * replaces a running one; lgdm_probe_stop without one is LGDM_ERR_STATE. */
enum { LGDM_PROBE_IDR_SPMV = 0, LGDM_PROBE_MG_FINEST = 1 };
lgdm_status lgdm_probe_start(lgdm_ctx* ctx, int32_t kind);
lgdm_status lgdm_probe_stop(lgdm_ctx* ctx, double* avg_ms, int64_t* count);

/* Device bytes held by the context (mesh, pattern, state, matrix, solver). */
lgdm_status lgdm_footprint(lgdm_ctx* ctx, int64_t* bytes);

/* The node aggregation rule of the multigrid preconditioner (host only, no
 * device call).  Graph: CSR over n nodes in host memory, ptr [n + 1] and adj
 * [ptr[n]] with ascending neighbour ids that include the node itself.  In
 * node order, a node whose neighbours are all unaggregated forms a new
 * aggregate with them; then each node left over joins the aggregate of its
 * first (lowest-id) aggregated neighbour, or forms one alone.  Writes agg
 * [n] (aggregate of each node, numbered in order of creation) and *n_agg.
 * INVALID_ARG for NULL pointers or n < 0, or a neighbour id outside [0, n). */
lgdm_status lgdm_amg_aggregate(int64_t n, const int32_t* ptr, const int32_t* adj, int32_t* agg,
                               int64_t* n_agg);

/* The level sets that order the process zone (host only, no device call).
 * Graph: CSR over n nodes in host memory, ptr [n + 1] and adj [ptr[n]],
 * symmetric (b a neighbour of a exactly when a is one of b); self-loops are
 * ignored.  Each connected component, taken in order of its lowest node, is
 * searched breadth-first from a pseudo-peripheral node (George & Liu 1979:
 * from the component's lowest node, restart from a least-connected node of
 * the last level while the number of levels grows); its levels follow those
 * of the components before it.  Writes level [n] and *n_levels; neighbours'
 * levels differ by at most one.  INVALID_ARG for NULL pointers, n < 0, or a
 * neighbour id outside [0, n). */
lgdm_status lgdm_zone_levels(int64_t n, const int32_t* ptr, const int32_t* adj, int32_t* level,
                             int64_t* n_levels);

/* Node counts of the context's multigrid levels (finest first) once a
 * multigrid solve has built them: writes up to max_levels counts to nodes
 * and the number of levels to *n_levels (0 before the first multigrid
 * solve). */
lgdm_status lgdm_amg_levels(lgdm_ctx* ctx, int32_t max_levels, int64_t* nodes, int32_t* n_levels);

/* ------------------------------------------------------------------------
 * Continuous batching of many simulation requests on one device.
 *
 * A batch holds up to max_slots requests.  Each admitted request keeps its
 * mesh, pattern, state (u, ebar, kappa_n) and tangent resident in its own
 * slot.  lgdm_batch_tick advances every running request by one Newton
 * iteration of Algorithm 2: one fused Gauss-point launch and one fused
 * node-row assembly launch cover all running requests; the linear solves of
 * the requests that need one run on per-slot streams and overlap on the
 * device.  Converged increments are committed per request (Eq. A.2) and the
 * request moves to its next load step.  Every reduction belongs to one
 * request and runs in a fixed order, so a request's results do not depend
 * on which other requests share the batch.
 * ------------------------------------------------------------------------ */
typedef struct lgdm_batch lgdm_batch;

/* One request: the problem statement of Algorithm 2 (geometry, material,
 * loads and boundary conditions) plus its number of uniform load steps.
 * Arrays are host pointers, copied at admission. */
typedef struct lgdm_request {
  int32_t dim, elem_type;
  int64_t n_nodes;
  const double* coords;      /* [n_nodes * dim]                    */
  int64_t n_elems;
  const int32_t* conn;       /* [n_elems * 2^dim]                  */
  const double* e_scale;     /* [n_elems] or NULL                  */
  lgdm_material material;
  int64_t n_bc;
  const int64_t* bc_dofs;    /* [n_bc] displacement dofs           */
  const double* bc_values;   /* [n_bc] values at load factor 1     */
  int64_t n_increments;      /* load factor of increment n is n / n_increments */
} lgdm_request;

enum { LGDM_SLOT_FREE = 0, LGDM_SLOT_RUNNING = 1, LGDM_SLOT_FINISHED = 2, LGDM_SLOT_FAILED = 3 };

typedef struct lgdm_slot_info {
  int32_t state;             /* LGDM_SLOT_*                                   */
  int32_t newton_in_increment;
  int64_t increment;         /* committed increments                          */
  int64_t n_increments;
  int64_t newton_total, krylov_total, assemblies_total;
  int64_t n_gauss, ndof, footprint_bytes;
  double max_damage;         /* of the last committed increment               */
  int32_t last_status;       /* lgdm_status of the failure for FAILED slots   */
  int32_t retries;           /* load steps tried a second time, from their start,
                                with the line-search setting flipped           */
  int64_t cutbacks;          /* load steps halved after both tries failed (at
                                most 3 halvings per increment, the smallest
                                step 1/8 of an increment; then the request
                                fails)                                          */
} lgdm_slot_info;

typedef struct lgdm_tick_report {
  int32_t running;           /* requests advanced by this tick                */
  int32_t solves;            /* linear solves performed                       */
  int32_t committed;         /* increments committed                          */
  int32_t finished;          /* requests that completed their load path       */
  int64_t gauss_points;      /* Gauss points assembled by the fused launch    */
  int64_t krylov_iters;
  double t_assembly_ms;      /* device time of the fused assembly launches    */
  double t_tick_ms;          /* host wall time of the tick                    */
} lgdm_tick_report;

/* Create a batch on `device` (fused launches go to hip_stream; each slot gets
 * a stream of its own at default priority).  precision as lgdm_create.
 * hbm_budget_bytes bounds the sum of admitted footprints (0 = free device
 * memory at creation). */
lgdm_status lgdm_batch_create(lgdm_batch** out, int32_t device, void* hip_stream, int32_t precision,
                              int32_t max_slots, int64_t hbm_budget_bytes);
lgdm_status lgdm_batch_destroy(lgdm_batch* b);
const char* lgdm_batch_last_error(const lgdm_batch* b);

/* Route the batch's device allocations (its launch tables and solve
 * buffers) and those of every request it admits through a caller allocator,
 * as lgdm_set_allocator does for one context.  Call it while no request is
 * admitted (else LGDM_ERR_STATE); the batch's buffers are reallocated
 * through the new allocator.  Both NULL returns to hipMalloc / hipFree. */
lgdm_status lgdm_batch_set_allocator(lgdm_batch* b, void* (*alloc)(size_t, void*),
                                     void (*free_fn)(void*, void*), void* user);

/* Upper bound of the device bytes one request of this size holds. */
lgdm_status lgdm_request_footprint(int32_t dim, int64_t n_nodes, int64_t n_elems, int32_t precision,
                                   int64_t* bytes);

/* Admit a request into a free slot if its footprint fits the budget:
 * LGDM_OK and *slot on success, LGDM_ERR_BUSY (nothing changed) when no slot
 * or budget is free; INVALID_ARG for a bad request or a request whose
 * dimension differs from the requests already in the batch. */
lgdm_status lgdm_batch_admit(lgdm_batch* b, const lgdm_request* r, int32_t* slot);

/* One Newton iteration for every running request (see above).  o nullable. */
lgdm_status lgdm_batch_tick(lgdm_batch* b, const lgdm_solver_opts* o, lgdm_tick_report* rep);

lgdm_status lgdm_batch_slot_info(lgdm_batch* b, int32_t slot, lgdm_slot_info* info);

/* lgdm_query_state on the request in `slot`. */
lgdm_status lgdm_batch_query(lgdm_batch* b, int32_t slot, int32_t field, double* out, int64_t n);

/* Release a finished or failed request's slot and device memory. */
lgdm_status lgdm_batch_retire(lgdm_batch* b, int32_t slot);

/* Bytes admitted, the budget, and the number of occupied slots. */
lgdm_status lgdm_batch_usage(lgdm_batch* b, int64_t* used, int64_t* budget, int32_t* occupied);

#ifdef __cplusplus
}
#endif
#endif /* LGDM_H */
