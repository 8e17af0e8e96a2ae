/*
 * rav.h - restricted additive Vanka (RAV) geometric multigrid for Taylor-Hood
 * Q2/Q1 and stabilized Q1-Q1 Stokes systems on MI355X (gfx950).
 *
 * Method: S. Saberi, G. Meschke, A. Vogel, "A restricted additive Vanka
 * smoother for geometric multigrid", arXiv 2103.10127.
 *
 * The library solves L x = b (Sec. 3, eq. 9) for the block system
 * L = [[A, B], [B^T, 0]] of the stationary Stokes problem (Sec. 2, eqs. 1, 6, 7)
 * discretised on a uniform quad (2D) or hex (3D) grid of [0,1]^d, with
 * geometric multigrid V-cycles (Sec. 2, Fig. 1) whose smoother is one of
 *   MV  multiplicative Vanka       (Sec. 3, eq. 11; residual update eq. 15)
 *   AV  additive Vanka             (Sec. 3, eq. 12)
 *   RAV restricted additive Vanka  (Sec. 3, eq. 13; row-limited inverse, Sec. 4.3)
 * each applied as the fixed-point iteration x <- x + S (b - L x) (eq. 10).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Vectors.  A level-l vector has n_total(l) = d (2N_l+1)^d + (N_l+1)^d FP64
 *   entries ordered [u_1; ...; u_d; p] (eq. 6): velocity component c at
 *   half-grid node a in [0,2N]^d at c*(2N+1)^d + sum_k a_k (2N+1)^k (x fastest),
 *   pressure at vertex k in [0,N]^d after all velocity entries.  Velocity
 *   entries on Dirichlet sides are masked: they stay 0 and have residual 0.
 * Levels.  Level 0 is the coarsest, level n_levels-1 the finest;
 *   N_l = n_cells / 2^(n_levels-1-l).
 * Memory.  Arguments named *_dev are device pointers (e.g. from
 *   torch.empty(..., device='cuda', dtype=torch.float64)); the caller owns
 *   them and they must hold n_total(level) doubles.  Arguments named *_host
 *   are host pointers.  Every hierarchy buffer (operators, patch inverses,
 *   coarse inverse, level vectors) is allocated by the library in rav_create /
 *   rav_factor_patches and released by rav_destroy.
 * Streams.  All device work of a context is ordered on the hipStream_t given
 *   to rav_create (NULL = default stream).  Calls that return host values
 *   (norms, iteration counts, exported data) synchronise that stream.
 * Errors.  Every function returns a rav_status; none throws.  Negative values
 *   are hard errors and leave a message retrievable with rav_last_error.
 *   Invalid arguments are rejected before any device work.  A context is not
 *   thread-safe: calls on one context must not overlap.
 */
#ifndef RAV_H
#define RAV_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RAV_OK = 0,
  RAV_NOT_CONVERGED = 1,   /* soft: maxit reached before the tolerance   */
  RAV_EINVAL = -1,         /* invalid argument / descriptor              */
  RAV_ENOMEM = -2,         /* device allocation failed                   */
  RAV_ESINGULAR = -3,      /* zero pivot in a patch or the coarse matrix */
  RAV_EDIVERGED = -4,      /* residual NaN/Inf or > 1e3 x initial        */
  RAV_EDEVICE = -5,        /* HIP runtime error                          */
  RAV_EUNSUPPORTED = -6    /* valid but not implemented combination      */
} rav_status;

typedef enum { RAV_SMOOTHER_RAV = 0, RAV_SMOOTHER_AV = 1, RAV_SMOOTHER_MV = 2 } rav_smoother;

/* Vertex patches: pressure vertex k plus every velocity DoF coupled to it by
 * B^T (Sec. 3): 51 local DoFs in 2D, 376 in 3D (3D: RAV only).  Element
 * patches: the velocity and pressure DoFs of one cell (2D 22, 3D 89). */
typedef enum { RAV_PATCH_VERTEX = 0, RAV_PATCH_ELEMENT = 1 } rav_patch_kind;

/* Storage precision of the patch inverse rows used by RAV (the outer
 * residual, local factorisation and coarse solve are always FP64). */
typedef enum { RAV_FP64 = 0, RAV_FP32 = 1, RAV_BF16 = 2 } rav_precision;

/* How RAV stores the owned rows of each L_i^{-1} (Sec. 4.3).  RAV_ROWS: the
 * owned rows themselves (owned DoFs x patch DoFs).  RAV_FACTORED (vertex
 * patches): the same rows through the block structure of L_i, whose velocity
 * block is the same scalar block K_i for every component and whose pressure
 * block is one unknown: the owned rows of K_i^{-1}, z = K_i^{-1} B_i and the
 * scalar Schur complement inverse, from which the apply forms the owned rows'
 * product with r exactly up to rounding (151 stored values per 2D patch
 * instead of 459, 1,376 per 3D patch instead of 9,400). */
typedef enum { RAV_ROWS = 0, RAV_FACTORED = 1 } rav_inv_format;

/* Discretization of the Stokes system (Sec. 2).  RAV_TAYLOR_HOOD: Q2
 * velocity, Q1 pressure, C = 0 (eq. 6 for an inf-sup stable pair).
 * RAV_Q1Q1_STAB: equal-order Q1 velocity and pressure with the stabilization
 * block of eq. (8), C = -beta sum_e diam_e^2 (grad q, grad p)_e (diam of a
 * d-cube of side h: sqrt(d) h), on the vertices of the grid; vertex patches
 * hold p_k and every velocity DoF at the vertices of the cells around k
 * (2D 19, 3D 82 DoFs) and RAV owns p_k and the velocity at k (Sec. 3, eq. 13).
 * Q1-Q1 vectors have (d+1) (N+1)^d entries [u_1; ...; u_d; p], field f of
 * vertex v at f (N+1)^d + lin(v); it is provided with vertex patches and FP64
 * inverses for RAV (either storage format), AV and MV (full local inverses; MV
 * in the colour order sum_d (k_d mod 4) 4^d, each patch recomputing its residual
 * rows, eq. 15), and FGMRES; batches, the learned weights, profiling markers
 * and rav_export_matrix return RAV_EUNSUPPORTED for it. */
typedef enum { RAV_TAYLOR_HOOD = 0, RAV_Q1Q1_STAB = 1, RAV_Q1Q1_ADAPTIVE = 2 } rav_discretization;

/* Circular (2D: cx, cy, r) or spherical (3D: cx, cy, cz, r) inclusion. */
typedef struct { double cx, cy, cz, r; } rav_inclusion;

typedef struct {
  int dim;                      /* 2 or 3                                        */
  int n_cells;                  /* N of the finest grid, divisible by 2^(n_levels-1) */
  int n_levels;                 /* >= 2                                          */
  unsigned bc_dirichlet_mask;   /* bit 2k: side x_k = 0, bit 2k+1: side x_k = 1 is
                                   Dirichlet (u = 0); other sides natural (eq. 2) */
  double eta_out, eta_in;       /* viscosity outside / inside inclusions, > 0   */
  int n_incl;                   /* number of inclusions (0..64)                  */
  const rav_inclusion* incl;    /* host array, copied by rav_create              */
  rav_patch_kind patch;         /* VERTEX or ELEMENT                             */
  rav_smoother smoother;
  double omega;                 /* damping, > 0 (Sec. 4: 0.66 RAV/MV, 0.1 AV)    */
  int nu_pre, nu_post;          /* smoothing steps, >= 0                         */
  rav_precision inv_precision;  /* RAV only; AV/MV store FP64 full inverses      */
  int coarse_galerkin;          /* 0: every level rediscretised (Sec. 4); 1: the
                                   viscous block of each coarser level is the
                                   Galerkin product P^T A P of the finest one
                                   (cell integrals by the finest grid's Gauss
                                   points; equal to 0 at constant viscosity) */
  rav_inv_format inv_format;    /* RAV storage of the owned inverse rows          */
  rav_discretization discretization;
  double beta;                  /* Q1-Q1 stabilization constant of eq. (8), > 0;
                                   with coarse_galerkin = 1 every level uses the
                                   finest diameter (the Galerkin product P^T C P) */
} rav_problem_desc;

typedef struct rav_ctx rav_ctx;

/* Builds the level hierarchy (Sec. 2): grids, DoF numbering, Dirichlet masks,
 * patch buckets, the rediscretised operator of every level (Sec. 4 assembles
 * the system anew on each grid) in FP64, and the coarse direct solver (Sec. 2:
 * an LU solve, exact up to rounding).  With Dirichlet velocity on every side
 * the coarse solve uses the bordered system [[L_0, e],[e^T, 0]], e = (0, 1_p),
 * i.e. zero-mean pressure.
 * hip_stream: a hipStream_t or NULL.  On success *out owns all device memory.
 * RAV_EINVAL (before any device work) also when the coarsest grid has more than
 * 16383 DoFs: its dense inverse would exceed 2 GB (2D up to 32x32, 3D up to
 * 8x8x8 cells on the coarsest level). */
rav_status rav_create(const rav_problem_desc* desc, void* hip_stream, rav_ctx** out);

/* Factors every local system L_i = R_i L R_i^T (Sec. 3) on every smoothed
 * level in FP64 and stores, for RAV, the owned rows of L_i^{-1} (Sec. 4.3) in
 * the context's precision, for AV/MV the full inverse.  The inverse is formed
 * by block elimination: the velocity block of L_i is the same symmetric
 * positive definite scalar block K_i for every component, so one elimination
 * on K_i (no pivoting) and the Schur complement of the pressure block give
 * L_i^{-1} exactly up to rounding.  RAV_ESINGULAR if a pivot of K_i is not
 * positive or the Schur complement is singular (rav_last_error names level
 * and patch).
 * For RAV it then times the lanes-per-patch variants of the apply on every
 * bucket and keeps the fastest (environment: RAV_AUTOTUNE=0 keeps a size rule,
 * RAV_AUTOTUNE_LOG=1 prints the timings to stderr). */
rav_status rav_factor_patches(rav_ctx* ctx);

/* DoF counts of a level: all entries (including masked) and free entries. */
rav_status rav_dofs(const rav_ctx* ctx, int level, long* n_total, long* n_free);
/* Number of levels and number of patches of a level. */
rav_status rav_n_levels(const rav_ctx* ctx, int* n_levels);
rav_status rav_n_patches(const rav_ctx* ctx, int level, long* n_patches);

/* b_dev = [(f, phi); 0] on the finest level (eq. 5 right-hand side, 3^d Gauss)
 * for the manufactured forcing f = -eta Lap u + grad p.  mms_params (host):
 * 2D: 25 doubles [eta, a(4), m(4), n(4), c(4), r(4), s(4)],
 * 3D: 65 doubles [eta, 3 x (a(4), m(4), n(4), l(4)), c(4), r(4), s(4), t(4)];
 * u from the stream function / vector potential sum_k a_k prod sin^2(w pi x),
 * p = sum_k c_k prod cos(w pi x). */
rav_status rav_assemble_rhs(rav_ctx* ctx, const double* mms_params_host, int n_params, double* b_dev);

/* Driven cavity (Sec. 4.1): b_dev = -L[free, masked] u_D on the finest level,
 * the right-hand side of the lifted problem for no-slip walls and the lid
 * velocity u = (lid_u, 0) on the top side's nodes strictly between the corners
 * (the corners belong to the walls), no forcing.  The solution of L x = b is
 * the velocity minus u_D (masked entries stay 0).  2D only; the top side must
 * be Dirichlet (bit 3 of bc_dirichlet_mask), else RAV_EINVAL. */
rav_status rav_assemble_rhs_lid(rav_ctx* ctx, double lid_u, double* b_dev);

/* r_dev = b_dev - L x_dev on free rows, 0 on masked rows (eq. 10).  If
 * norm_host is non-NULL it receives ||r||_2 (synchronises). */
rav_status rav_residual(rav_ctx* ctx, int level, const double* x_dev, const double* b_dev,
                        double* r_dev, double* norm_host);

/* `sweeps` smoother steps x <- x + S (b - L x) on a level >= 1 (eqs. 10-13),
 * in place on x_dev. */
rav_status rav_smooth(rav_ctx* ctx, int level, int sweeps, double* x_dev, const double* b_dev);

/* Grid transfer between level `level` (fine) and level-1 (coarse): nested
 * Q2/Q1 interpolation P and restriction P^T (Sec. 2).
 * rav_restrict: bc_dev = P^T rf_dev.  rav_prolong_add: xf_dev += P xc_dev. */
rav_status rav_restrict(rav_ctx* ctx, int level, const double* rf_dev, double* bc_dev);
rav_status rav_prolong_add(rav_ctx* ctx, int level, const double* xc_dev, double* xf_dev);

/* Direct solve on level 0 (Sec. 2): x0_dev = L_0^{-1} b0_dev (bordered form
 * for the all-Dirichlet case). */
rav_status rav_coarse_solve(rav_ctx* ctx, const double* b0_dev, double* x0_dev);

/* One V(nu_pre, nu_post) cycle on the finest level, in place on x_dev (Fig. 1). */
rav_status rav_vcycle(rav_ctx* ctx, double* x_dev, const double* b_dev);

/* V-cycles from the given x_dev until ||b - L x||_2 <= rtol ||b - L x_0||_2
 * (Sec. 4: reduction by 1e8) or maxit cycles.  One FP64 norm is read back per
 * cycle.  Returns RAV_OK, RAV_NOT_CONVERGED or RAV_EDIVERGED; *iters and
 * *rel_res (final ||r|| / ||r_0||) are set in every case.  The cycle is
 * captured from the context's stream into a HIP graph on first use and
 * replayed (same launches, same results; RAV_GRAPH=0 in the environment
 * launches directly); rav_set_params and rav_factor_patches drop it. */
rav_status rav_solve(rav_ctx* ctx, double* x_dev, const double* b_dev, double rtol, int maxit,
                     int* iters, double* rel_res);

/* Krylov acceleration (Sec. 4 remarks that the multigrid cycle may equally
 * serve as the preconditioner of a Krylov method): restarted flexible GMRES(restart),
 * right-preconditioned by one V(nu_pre, nu_post) cycle from a zero guess.
 * maxit bounds the number of preconditioner applications (V-cycles); stops
 * when the true residual ||b - L x||_2 <= rtol ||b - L x_0||_2.  Allocates
 * 2*restart+3 work vectors of the finest level on its first call (and on a
 * call with another restart) and keeps them in the context until rav_destroy,
 * so later calls allocate nothing.
 * Serves every context: Taylor-Hood, stabilized Q1-Q1 and adaptive grids
 * (the V-cycle of the context's own smoother).  Same return convention as
 * rav_solve; *iters counts V-cycles. */
rav_status rav_solve_gmres(rav_ctx* ctx, double* x_dev, const double* b_dev, double rtol, int maxit, int restart,
                           int* iters, double* rel_res);

/* For callers that cannot allocate device memory during a solve (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * rav_solve_gmres without any allocation.  Same arguments, arithmetic and
 * results as rav_solve_gmres (bit for bit), but the work vectors live in one
 * library-owned static device array of RAV_NOALLOC_SCRATCH_BYTES per GPU,
 * held from the first call on that GPU until the process ends.  Requires
 * restart <= RAV_NOALLOC_MAX_RESTART and
 * 65536 + (2 restart + 3) * 8 * ceil32(n_total(finest)) <= RAV_NOALLOC_SCRATCH_BYTES
 * (ceil32 rounds up to a multiple of 32); larger requests return RAV_EINVAL
 * with a message before any device work.  Nothing in the array needs to start
 * at zero: every call writes each buffer before reading it.  All calls on one
 * GPU share the array: calls that overlap in time on one GPU (from several
 * threads or streams) race and give wrong results; calls one after another
 * are safe, since each returns after synchronising its stream. */
#define RAV_NOALLOC_SCRATCH_BYTES (64LL * 1024 * 1024)
#define RAV_NOALLOC_MAX_RESTART 64
rav_status rav_solve_gmres_noalloc(rav_ctx* ctx, double* x_dev, const double* b_dev, double rtol, int maxit,
                                   int restart, int* iters, double* rel_res);

/* Change damping and smoothing steps without refactoring. */
rav_status rav_set_params(rav_ctx* ctx, double omega, int nu_pre, int nu_post);

/* Per-patch damping omega_i (the diagonal weighting of eq. 11, one scalar per
 * patch) for `level`: omega_dev holds n_patches(level) floats and must stay
 * valid while used; NULL restores the scalar omega. */
rav_status rav_set_patch_omega(rav_ctx* ctx, int level, const float* omega_dev);

/* Fallback for per-patch weights: during rav_solve, if a cycle reduces the
 * residual by a factor worse than rho_max (||r_k|| > rho_max ||r_{k-1}||)
 * while per-patch weights are set, they are dropped and the solve continues
 * with the scalar omega.  The weights are set again before rav_solve returns,
 * so the next solve starts with them.  rho_max = 0 disables it.  *fell_back
 * (may be NULL) reports whether the previous rav_solve fell back. */
rav_status rav_set_fallback(rav_ctx* ctx, double rho_max, int* fell_back);

/* Host-side patch map of patch `patch` on `level`: its free DoFs in local
 * order (component-major, lexicographic nodes, pressure last) into dofs_host
 * (capacity >= 376), their count into *n, and owned_host[j] = 1 if the DoF is
 * owned by the patch (restricted prolongation of eq. 13), else 0. */
rav_status rav_get_patch_map(const rav_ctx* ctx, int level, long patch, int* dofs_host, int* n,
                             int* owned_host);

/* Host-only versions of the two maps above, computed from the descriptor with
 * the same index code the kernels use; they touch no device and work on a
 * machine without a GPU.  owner_host holds n_total(level) int32. */
rav_status rav_map_patch(const rav_problem_desc* desc, int level, long patch, int* dofs_host, int* n,
                         int* owned_host);
rav_status rav_map_owner(const rav_problem_desc* desc, int level, int* owner_host);

/* Device-computed owner of every DoF (patch index, -1 for masked DoFs) into
 * owner_dev (n_total(level) int32 on the device). */
rav_status rav_get_owner(rav_ctx* ctx, int level, int* owner_dev);

/* Stored inverse rows of one patch, mapped to the patch's free local order:
 * out_host (row-major, *rows x *cols, capacity 128*128 doubles) receives the
 * owned rows of L_i^{-1} (RAV) or the full inverse (AV/MV) as FP64. */
rav_status rav_get_patch_inverse(rav_ctx* ctx, int level, long patch, double* out_host, int* rows,
                                 int* cols);

/* Dense copy of the level operator (free rows/cols, masked ones zero) into
 * out_host (row-major n_total x n_total); only for n_total(level) <= 20000. */
rav_status rav_export_matrix(rav_ctx* ctx, int level, double* out_host);

/* Times `reps` smoother sweeps of `level` with HIP events recorded on the
 * context stream around each kernel: average ms of the residual kernel and of
 * the patch-apply kernel(s) per sweep.  x_dev is updated as by rav_smooth. */
rav_status rav_time_sweep(rav_ctx* ctx, int level, int reps, double* x_dev, const double* b_dev,
                          float* ms_residual, float* ms_apply);

/* Kernel timing during ordinary calls: after rav_profile_begin, every smoother
 * residual launch and patch-apply launch on `level` (up to max_launches of
 * each) is bracketed by HIP events recorded on the context stream (timing-only
 * events without a system-scope cache fence, so they add little to the run).
 * rav_profile_end synchronises, stops recording and returns the average
 * duration in ms of the residual launches, of the apply launches (all buckets
 * of one sweep count as one launch) and how many apply launches were timed. */
rav_status rav_profile_begin(rav_ctx* ctx, int level, int max_launches);
rav_status rav_profile_end(rav_ctx* ctx, float* avg_residual_ms, float* avg_apply_ms, int* n_apply);

/* Plain device copy of n doubles on hip_stream (bandwidth calibration). */
rav_status rav_stream_copy(void* hip_stream, double* dst_dev, const double* src_dev, long n);

/* ---- adaptively refined grids (Sec. 2, Fig. 2; Sec. 4.1-4.2, Tables 1-2) ---
 * Stabilized Q1-Q1 (eq. 8, beta and the viscosity eta_out of the descriptor)
 * on a hierarchy of quadtree grids over a region of the rectangle
 * [0, lattice_x] x [0, lattice_y] (lattice units; lengths in units of the
 * height, a leaf of s units has size s / lattice_y), each grid refining the
 * previous one, with hanging nodes: a leaf corner at the midpoint of a
 * larger neighbour's edge carries no unknown and takes the mean of that edge's
 * endpoints, so the discrete space is the conforming Q1 space (Fig. 2).  The
 * operator of every grid is assembled anew on that grid (Sec. 4) as
 * L = T^T L_leaves T with T the constraint map.  Unknowns: [u_x; u_y; p] over
 * the regular vertices (leaf corners that are not hanging), numbered
 * lexicographically (y slowest).  The region is the union of the coarsest
 * grid's leaves: cells of the rectangle that no leaf covers are holes
 * (obstacles).  Velocity is Dirichlet on the boundary of holes and on the
 * sides of the rectangle whose bit is set in bc_dirichlet_mask (bit 0: x = 0,
 * bit 1: x = lattice_x, bit 2: y = 0, bit 3: y = lattice_y; a vertex on both a
 * Dirichlet and an open side is Dirichlet); on the other sides the velocity
 * is free (the natural outflow condition of the weak form, Sec. 4.2).  Data
 * enter through the lifting (rav_assemble_rhs_lid for the driven cavity,
 * rav_assemble_rhs_dirichlet for any values).  With all four sides Dirichlet
 * the pressure is fixed up to a constant and the coarse solve imposes zero
 * mean; otherwise the coarse matrix is inverted as it is.
 * Vanka patch i (one per regular vertex): p_i and the free velocity at the
 * vertices of the leaves around vertex i, a hanging corner standing for the
 * vertices that constrain it (at most 16 free vertices, else
 * RAV_EUNSUPPORTED); RAV owns p_i and the velocity at i.  MV visits the
 * patches colour by colour (greedy colouring in patch order: a patch takes
 * the smallest colour of no earlier patch whose vertices meet the row pattern
 * of its own vertices), which is the sequential sweep in that order.
 *
 * leaves_host: the leaves of all grids, coarsest first, as int32 triples
 * (x0, y0, s) in lattice units (s a power of two >= 2, x0 and y0 multiples
 * of s, the cell inside the rectangle); n_leaves_host[l] leaves for grid l,
 * l < desc->n_levels.  Copied; the host arrays may be freed on return.  The
 * leaves of a grid must not overlap, every grid must cover the coarsest
 * grid's region, be 2:1 balanced and refine the previous one; the coarsest
 * must have at most 16383 DoFs (dense direct solve).  lattice_x, lattice_y in
 * [2, 2^24].  desc: discretization RAV_Q1Q1_ADAPTIVE, dim 2, n_cells ignored,
 * no inclusions, vertex patches, FP64, coarse_galerkin 0; inv_format is
 * ignored (the owned rows are kept factored: row i of K_i^{-1}, K_i^{-1} b_c
 * and the inverse Schur complement).  RAV_EINVAL with a message (before any
 * device work) for grids that break these rules.  The context then serves
 * rav_factor_patches, rav_dofs, rav_n_levels, rav_n_patches,
 * rav_assemble_rhs_lid, rav_assemble_rhs_dirichlet, rav_residual, rav_smooth, rav_restrict,
 * rav_prolong_add, rav_coarse_solve, rav_vcycle, rav_solve, rav_solve_gmres,
 * rav_solve_gmres_noalloc, rav_set_params, rav_get_patch_map, rav_get_owner,
 * rav_get_patch_inverse, rav_time_sweep and rav_destroy; the others return
 * RAV_EUNSUPPORTED. */
rav_status rav_create_adaptive(const rav_problem_desc* desc, const int* leaves_host, const long* n_leaves_host,
                               long lattice_x, long lattice_y, void* hip_stream, rav_ctx** out);
/* Right-hand side of Dirichlet data on the finest grid of an adaptive
 * context (Sec. 4.2: the parabolic inflow, eq. 14): b_dev = -L_all[:, masked]
 * u_D with L_all the operator before any velocity is masked, masked rows
 * zero, so the solution x holds the free unknowns and u = x + u_D.  ud_host:
 * 2 n host doubles, u_x then u_y of every regular vertex in the library's
 * order (rav_adaptive_host_export what = 4 gives the vertices); only the
 * values at Dirichlet vertices are read.  b_dev: 3 n device doubles.
 * Synchronises.  RAV_EUNSUPPORTED for contexts of uniform grids. */
rav_status rav_assemble_rhs_dirichlet(rav_ctx* ctx, const double* ud_host, double* b_dev);
/* Sizes of grid `level` into info_host[9]: regular vertices, stored operator
 * entries (vertex pairs, padded to 64-vertex slices), stored patch entries
 * (padded likewise), MV colours (0 on the coarsest grid), operator entries
 * and patch entries without the padding, distinct operator value tuples,
 * patch configurations (patches with equal local matrices share one stored
 * factorization; 0 on the coarsest grid), and the entry format (0: one
 * 32-bit word per entry and 16-bit patch offsets; 1: 32-bit columns, ids and
 * patch vertices, used when an offset or id does not fit 16 bits). */
rav_status rav_adaptive_level_info(const rav_ctx* ctx, int level, long* info_host);

/* Host-only (touches no device, works without a GPU): the set-up that
 * rav_create_adaptive performs for grid `level`, written out for checks.
 * what = 0: the operator, dense row-major (*rows = *cols = n_total; masked
 *           rows and columns zero);
 * what = 1: the prolongation from grid level-1 (*rows = n_total(level),
 *           *cols = n_total(level-1); masked velocity rows/columns zero);
 * what = 2: the lid lifting for lid velocity 1 on this grid (*rows = n_total,
 *           *cols = 1; rav_assemble_rhs_lid scales the finest one; needs a
 *           Dirichlet top side);
 * what = 3: the MV colour of every patch (*rows = n_patches, *cols = 1);
 * what = 4: the regular vertices in the library's order (*rows = vertices,
 *           *cols = 3: x and y in lattice units, 1 if the velocity there is
 *           Dirichlet else 0).
 * out_host NULL only reports the shape.  Same validation and errors as
 * rav_create_adaptive. */
rav_status rav_adaptive_host_export(const rav_problem_desc* desc, const int* leaves_host, const long* n_leaves_host,
                                    long lattice_x, long lattice_y, int level, int what, double* out_host, long* rows,
                                    long* cols);

/* Device memory of every buffer the library allocates (hierarchies, patch
 * inverses, work vectors of rav_solve_gmres, batches, networks): by default
 * hipMalloc/hipFree; with this call the caller's functions instead, e.g. a
 * framework's caching allocator.  alloc(bytes, user) returns device memory
 * on the current device aligned to at least 256 bytes, or NULL (the library
 * call then returns RAV_ENOMEM); release(ptr, user) frees it.  Both NULL
 * restores hipMalloc/hipFree.  RAV_EINVAL if only one function is given or
 * while any context, batch or network exists (each buffer is released by the
 * allocator that made it).  Not to be called while another thread uses the
 * library.  rav_solve_gmres_noalloc allocates nothing either way. */
rav_status rav_set_device_allocator(void* (*alloc)(size_t bytes, void* user), void (*release)(void* ptr, void* user),
                                    void* user);

rav_status rav_destroy(rav_ctx* ctx);

/* ---- learned per-patch damping ---------------------------------------------
 * A small network predicts the per-patch weight omega_i (one scalar per
 * subdomain: the diagonal weighting of eq. 11 in its simplest form) from 16
 * local features of each 2D vertex patch: log10(eta/eta_out)/4 sampled at the
 * 3x3 points (k + (a,b)/2) h, a,b in {-1,0,1}; their min, max and mean;
 * boundary flags in x and y; log2(N)/10; 1.  Network 16 -> 64 -> 64 -> 1, ReLU,
 * omega = 0.2 + sigmoid(z), FP32 parameters (5313 floats, flat: W1 64x16, b1,
 * W2 64x64, b2, w3, b3).  Supported for 2D vertex-patch RAV contexts. */
typedef struct rav_mlp rav_mlp;
rav_status rav_mlp_create(const float* theta_host, rav_mlp** out);
/* Copies the parameters and/or the last gradient (FP64) to the host (NULL skips). */
rav_status rav_mlp_get(const rav_mlp* mlp, float* theta_host, double* grad_host);
rav_status rav_mlp_destroy(rav_mlp* mlp);
/* omega_dev (n_patches(level) floats, device) = network output on `level`. */
rav_status rav_learn_patch_omega(rav_ctx* ctx, const rav_mlp* mlp, int level, float* omega_dev);
/* Per-patch weights from the network on every smoothed level (library-owned
 * arrays); mlp = NULL restores the scalar omega. */
rav_status rav_learn_set_omega(rav_ctx* ctx, const rav_mlp* mlp);
/* Two-grid training objective of a 2-level context (FP64 rows, exact coarse
 * solve): J = ||L x_out||^2 / ||L x0||^2 after nu RAV sweeps with the
 * network's weights, the exact coarse correction, nu sweeps, from the error
 * x0_dev (b = 0).  Returns J, dJ/domega_i (grad_omega_dev: n_patches doubles,
 * may be NULL) and dJ/dtheta (grad_theta_host: 5313 doubles, may be NULL),
 * computed by the reverse sweep of the cycle and back-propagation. */
rav_status rav_learn_twogrid(rav_ctx* ctx, const rav_mlp* mlp, const double* x0_dev, int nu, double* loss,
                             double* grad_omega_dev, double* grad_theta_host);
/* rav_learn_twogrid followed by one Adam step (beta1 0.9, beta2 0.999) of size lr. */
rav_status rav_learn_step(rav_ctx* ctx, rav_mlp* mlp, const double* x0_dev, int nu, double lr, double* loss);

/* ---- batched problems -------------------------------------------------------
 * Many independent problems solved together with RAV V-cycles (the additive,
 * order-free sweep of eq. 13 lets the patches of all problems share one
 * launch per V-cycle stage).  All descriptors must share dim, patch kind,
 * smoother (RAV), inverse precision, smoothing steps and the coarsest grid
 * size n_cells / 2^(n_levels-1); grid sizes, level counts, viscosity fields
 * and omega may differ.  x_dev / b_dev are host arrays of n_problems device
 * pointers, each holding that problem's finest-level vector.  Problems stop
 * being updated once converged; iters and rel_res (host arrays of n_problems)
 * receive per-problem results.  The batch owns one context per problem; the
 * coarse matrices of all problems are inverted together at create time
 * (blocked Gauss-Jordan, one launch pair per 32 pivots for the whole batch).
 * rav_batch_factor also times the lanes-per-patch variants of every batched
 * apply launch and keeps the fastest (RAV_AUTOTUNE=0 keeps a size rule);
 * rav_batch_solve replays one captured V-cycle graph per cycle (RAV_GRAPH=0
 * launches directly). */
typedef struct rav_batch rav_batch;
rav_status rav_batch_create(const rav_problem_desc* descs, int n_problems, void* hip_stream, rav_batch** out);
rav_status rav_batch_factor(rav_batch* batch);
rav_status rav_batch_size(const rav_batch* batch, int* n_problems);
rav_status rav_batch_dofs(const rav_batch* batch, int problem, long* n_total, long* n_free);
rav_status rav_batch_assemble_rhs(rav_batch* batch, int problem, const double* mms_params_host, int n_params,
                                  double* b_dev);
rav_status rav_batch_vcycle(rav_batch* batch, double* const* x_dev, const double* const* b_dev);
rav_status rav_batch_solve(rav_batch* batch, double* const* x_dev, const double* const* b_dev, double rtol,
                           int maxit, int* iters, double* rel_res);
/* The same two calls under the names rav_create_batch / rav_solve_batch
 * (identical arguments and behaviour). */
rav_status rav_create_batch(const rav_problem_desc* descs, int n_problems, void* hip_stream, rav_batch** out);
rav_status rav_solve_batch(rav_batch* batch, double* const* x_dev, const double* const* b_dev, double rtol,
                           int maxit, int* iters, double* rel_res);
/* Batched form of rav_solve_gmres (Sec. 4: the multigrid cycle as Krylov
 * preconditioner): restarted flexible GMRES(restart) for every problem, all
 * problems advancing in lockstep so that each preconditioner application is
 * one batched V-cycle and each Gram-Schmidt step one launch per vector
 * operation; a problem leaves the Arnoldi process once its own least-squares
 * residual reaches rtol (checked again on its true residual at the restart).
 * iters[p] counts problem p's V-cycles (<= maxit).  Allocates
 * (2 restart + 3) work vectors per problem for the duration of the call.
 * Returns RAV_OK when every problem converged, else RAV_NOT_CONVERGED or
 * RAV_EDIVERGED (any problem). */
rav_status rav_batch_solve_gmres(rav_batch* batch, double* const* x_dev, const double* const* b_dev, double rtol,
                                 int maxit, int restart, int* iters, double* rel_res);
rav_status rav_batch_destroy(rav_batch* batch);
const char* rav_batch_last_error(const rav_batch* batch);

/* Message of the last hard error on ctx (or of the last failed rav_create
 * when ctx is NULL).  Valid until the next call on the same context. */
const char* rav_last_error(const rav_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* RAV_H */
