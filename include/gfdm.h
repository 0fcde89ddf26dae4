/*
 * gfdm.h -- C ABI of the MI355X (gfx950) library for the meshfree GFDM hot
 * path of "Adaptive coupling of 3D and 2D fluid flow models" (Suchde):
 * neighbourhoods, local PCA transition detection, second-order GFDM stencils,
 * stencil application, the implicit pressure-Poisson solve, the 3D->2D
 * transition, and adjoints of the stencils.
 *
 * Conventions shared by every entry point
 *  - Pointers named as device memory must point to memory on the context's
 *    device (hipMalloc or torch CUDA tensors).  Host pointers are named so.
 *  - The caller owns every buffer it passes.  Opaque handles (gf_ctx,
 *    gf_nbr) own the device memory they allocate and release it in their
 *    *_destroy / *_free call.
 *  - All work is enqueued on the context's stream in order; calls return
 *    without waiting unless stated ("synchronises").
 *  - Particle arrays are in the caller's order (structure of arrays, length
 *    n).  Outputs are in the caller's order too; the Morton/cell order used
 *    internally never leaks out.
 *  - Every call returns a gf_status and never aborts.  On failure
 *    gf_last_error(ctx) describes the cause.  Bad arguments are rejected
 *    before any kernel is launched.  Per-particle numerical problems are not
 *    call failures: they are reported per particle (status arrays).
 *  - Calls that share a context must not run concurrently from several host
 *    threads.
 */
#ifndef GFDM_H
#define GFDM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GF_OK = 0,
  GF_EINVAL = -1,      /* invalid argument or input data (NaN/Inf, h <= 0, bad enum) */
  GF_ENOMEM = -2,      /* device allocation failed */
  GF_EHIP = -3,        /* a HIP runtime call failed */
  GF_ECAPACITY = -4,   /* a documented size limit was exceeded */
  GF_ENOTCONV = -5,    /* iterative solve did not reach its tolerance */
  GF_EBREAKDOWN = -6   /* iterative solve broke down and could not restart */
} gf_status;

typedef enum { GF_F64 = 0, GF_F32 = 1 } gf_dtype;

/* How stencils are computed (gf_gfdm_weights).
 *  GF_PLAIN_F64: one work-item per particle in the caller's order, FP64
 *                throughout, FP64 weights out.
 *  GF_BATCHED:   particles grouped by model and neighbour count, processed
 *                in Morton order by teams of lanes; the per-particle Gram
 *                system is solved in FP64; particles whose condition number
 *                exceeds kappa_max are re-solved by an FP64 Householder QR.
 *                Weights out in FP64 or FP32.  With FP32 output the support
 *                weights w(q) are evaluated in FP32 as well.
 *  GF_F32_QR_FALLBACK64 is another name of GF_BATCHED: FP32 stencils
 *                (storage and support weights), each particle's condition
 *                estimate triggering the FP64 Householder QR fallback. */
typedef enum { GF_PLAIN_F64 = 0, GF_BATCHED = 1, GF_F32_QR_FALLBACK64 = 1 } gf_prec;

enum { GF_OP_DX = 1, GF_OP_DY = 2, GF_OP_DZ = 4, GF_OP_LAP = 8 };

/* particle kinds (Sec. 2.3) and models */
enum { GF_KIND_INTERIOR = 0, GF_KIND_FREE_SURFACE = 1, GF_KIND_WALL = 2 };
enum { GF_MODEL_BULK = 0, GF_MODEL_FILM = 1 };

typedef struct gf_ctx gf_ctx;
typedef struct gf_nbr gf_nbr;

/* Particle cloud, structure of arrays in device memory, length n.
 *  x, y, z, h : positions and support radius h_i (> 0, finite), FP64.
 *  model      : 0 = 3D bulk, 1 = 2D film (Sec. 2.2).
 *  kind       : 0 interior, 1 free surface, 2 wall (Sec. 2.3).  May be NULL
 *               for calls that do not use kinds.
 *  nx, ny, nz : unit wall / film normal; read for wall and film particles
 *               only (may be NULL when there are none). */
typedef struct {
  int64_t n;
  const double *x, *y, *z, *h;
  const int8_t *model;
  const int8_t *kind;
  const double *nx, *ny, *nz;
} gf_particles;

/* ---------------------------------------------------------------- context */
/* Create a context on HIP device `device`.  stream: a hipStream_t to enqueue
 * on, or NULL for the default (null) stream. */
gf_status gf_create(int device, void *stream, gf_ctx **out);
/* Enqueue later calls on `stream`.  The calls of a context share its scratch
 * memory, so the new stream first waits for the work the context enqueued on
 * the previous one (an event; skipped while `stream` is being captured into a
 * graph, where the caller orders the capture).  Does not synchronise. */
gf_status gf_set_stream(gf_ctx *ctx, void *stream);
void gf_destroy(gf_ctx *ctx);
/* Message of the last failed call on ctx ("" if none).  Owned by ctx. */
const char *gf_last_error(const gf_ctx *ctx);
const char *gf_version(void);

/* Per-kernel timing (tracing aid).  While enabled, every kernel the library
 * launches on ctx is bracketed by HIP events on the context stream.
 * gf_profile_read synchronises on those events and writes one line per kernel
 * name, "name launches total_ms", into buf (host, len bytes), then clears the
 * record.  GF_ECAPACITY if buf is too small. */
gf_status gf_profile_enable(gf_ctx *ctx, int on);
gf_status gf_profile_read(gf_ctx *ctx, char *buf, size_t len);

/* LDS budget of the neighbour-tile kernels (stencils, application, PCA,
 * pressure SpMV).  A block stages the distinct neighbours of its tile in LDS
 * when there are at most `entries` of them (further capped by each kernel's
 * own limit, 1024-2048) and otherwise reads them from global memory with the
 * same arithmetic, so the results do not depend on it.  entries <= 0
 * restores the kernels' own limits.  Lets callers trade LDS for occupancy and
 * exercises the unstaged path.  Never fails for a valid ctx. */
gf_status gf_set_tile_capacity(gf_ctx *ctx, int entries);

/* ---------------------------------------------------------- neighbourhoods */
/* Build S_i = { j : |x_j - x_i| <= (h_i + h_j)/2 } for every particle
 * (Sec. 2.2, Eq. Nbd), i in S_i.  cross_model = 0: only particles of the same
 * model (Sec. 6.2: S_i holds neighbours of i's own model); cross_model = 1:
 * all models (used by the smoothing rule of Sec. 4.3).  The predicate is
 * evaluated in FP64 as d2 = (dx*dx + dy*dy) + dz*dz <= r*r, r = 0.5*(h_i+h_j),
 * without fused multiply-adds, so the sets are reproducible bit for bit.
 * Result rows are sorted ascending.  Limit: at most 2048 neighbours per
 * particle (GF_ECAPACITY).  Synchronises (the size of the result is read back).
 * The handle holds the CSR lists, the Morton processing order and the
 * grouping of particles used by the batched kernels.  Scratch: the context's
 * arena grows to about n x 2.1 KB while the rows are staged (512 entries per
 * particle while that stays under 8 GB, else 256, else none) and keeps that
 * size for later calls on the context. */
gf_status gf_build_neighbours(gf_ctx *ctx, const gf_particles *p, int cross_model, gf_nbr **out);
/* Extended neighbourhoods of a cloud whose particles [n_rows, n) are ghost
 * particles (Sec. 6.2): the rows of particles [0, n_rows) hold S_i of
 * Eq. (Nbd) over regular and ghost particles alike (S_i joined with the ghost
 * neighbours S_i^g); no derivatives are taken at ghost particles, so a ghost's
 * own row holds only itself.  0 <= n_rows <= n; n_rows = n is
 * gf_build_neighbours.  Everything else as gf_build_neighbours. */
gf_status gf_build_neighbours_rows(gf_ctx *ctx, const gf_particles *p, int cross_model, int64_t n_rows,
                                   gf_nbr **out);
/* n, nnz and the longest row of a neighbour handle (host outputs, any NULL). */
gf_status gf_nbr_info(const gf_nbr *nbr, int64_t *n, int64_t *nnz, int32_t *max_row);
/* The handle's own CSR lists of Eq. (Nbd) without a copy: *row_ptr
 * ([n+1] int64) and *col ([nnz] int32, user indices, rows ascending) are
 * device pointers owned by the handle, valid until gf_nbr_free; the caller
 * must not write through them.  Any output may be NULL.  Host call, no
 * device work. */
gf_status gf_nbr_view(const gf_nbr *nbr, int64_t *nnz, const int64_t **row_ptr, const int32_t **col);
/* Copy the CSR lists into caller buffers (device): row_ptr [n+1] int64,
 * col [nnz] int32 (user indices, rows ascending).  Either may be NULL. */
gf_status gf_nbr_export(gf_ctx *ctx, const gf_nbr *nbr, int64_t *row_ptr, int32_t *col);
void gf_nbr_free(gf_nbr *nbr);

/* ---------------------------------------------------------- PCA / flags */
typedef struct {
  double eps_lambda_max;  /* 0.15, Sec. 4.1.2 Eq. (EigenvalueLimit)          */
  double theta_star;      /* pi/6, Sec. 4.1.3 Eq. (EigenvectorLimit)         */
  int literal_rule;       /* 0: pass iff |n.w3| >= cos(theta*) (w3 along the
                             depth direction, as the prose and Sec. 7.1
                             require); 1: the inequality exactly as printed,
                             |n.w3| < cos(theta*)                            */
} gf_pca_params;
void gf_pca_params_default(gf_pca_params *p);

/* Local PCA and transition flags (Sec. 4).
 * For every particle: covariance of S_i about its centroid (Sec. 4.1.2),
 * eigenvalues lambda_1 >= lambda_2 >= lambda_3 -> lam_3n [n][3], unit
 * eigenvector of lambda_3 -> w3_3n [n][3] (largest-magnitude component made
 * positive), eps_n = 2 lambda_3 / (lambda_1 + lambda_2) (+inf if the
 * denominator is 0).  Flags flag_n (uint8): 0 none, 1 bulk->film, 2 film->bulk:
 *  3D wall particles follow Alg. 2 (resolution criterion on neighbour kinds,
 *  eigenvalue and eigenvector tests, user criterion); film particles are
 *  flagged when film_height >= h3d (Eq. 2Dto3Dcond) or by the user criterion.
 *  Smoothing (Sec. 4.3): particles with prev_transitioned set are not
 *  flagged; then, if `cross` is given, a flag survives only if another
 *  particle of the cross-model neighbourhood is of the target model or
 *  carries the same flag.
 * same: same-model neighbourhoods (required).  cross, film_height, h3d,
 * prev_transitioned (uint8), user_flag (uint8): optional (NULL).  Outputs
 * lam_3n, w3_3n, eps_n may be NULL; flag_n may be NULL (then only PCA). */
gf_status gf_classify_pca(gf_ctx *ctx, const gf_particles *p, const gf_nbr *same,
                          const gf_nbr *cross, const double *film_height, const double *h3d,
                          const uint8_t *prev_transitioned, const uint8_t *user_flag,
                          const gf_pca_params *params, double *lam_3n, double *w3_3n,
                          double *eps_n, uint8_t *flag_n);

/* ---------------------------------------------------------- GFDM stencils */
typedef struct {
  double alpha_w;    /* support weight w(q) = (e^{-a q^2} - e^{-a}) / (1 - e^{-a}),
                        q = |x_j - x_i| / ((h_i + h_j)/2); default a = 8      */
  double kappa_max;  /* GF_BATCHED: 1-norm condition number of the Gram matrix
                        above which a particle is re-solved by Householder QR
                        (default 1e5)                                         */
} gf_ls_params;
void gf_ls_params_default(gf_ls_params *p);

typedef struct {
  int64_t n_ok, n_fallback, n_rank_deficient, n_too_few;
  double kappa_max_seen;  /* largest Gram-matrix condition estimate */
} gf_ls_stats;

/* Second-order GFDM stencils (Eq. GFDM_Definition, order 2 as in Sec. 2.3).
 * For particle i, with X = (x_j - x_i)/h_i (film: tangent coordinates of a
 * frame built from the normal), monomials [1, X, Y, Z, X^2, Y^2, Z^2, XY, XZ,
 * YZ] (film: [1, U, V, U^2, V^2, UV]) and weights w_j, the stencil is the
 * minimum-norm solution (sum c_j^2 / w_j) of the exactness conditions, i.e.
 * c = W M (M^T W M)^{-1} d.  Output w_out [nnz][4] in `wtype` (FP64 or FP32;
 * GF_PLAIN_F64 requires FP64): physical weights for d/dx, d/dy, d/dz and the
 * Laplacian, aligned with the neighbour CSR; w_out must be 16-byte aligned
 * (else GF_EINVAL: the kernels write whole 16-byte vectors).  Film rows hold the surface
 * gradient as global x, y, z components and the surface Laplacian.
 * status_n (int8, device, may be NULL): 0 ok, 1 solved by the FP64 QR
 * fallback, 2 rank deficient (zero weights), 3 fewer neighbours than
 * monomials (zero weights).  kappa_n (float, device, may be NULL): condition
 * estimate.  stats (host, may be NULL): synchronises and fills counts. */
gf_status gf_gfdm_weights(gf_ctx *ctx, const gf_particles *p, const gf_nbr *nbr, gf_prec prec,
                          const gf_ls_params *params, gf_dtype wtype, void *w_out,
                          int8_t *status_n, float *kappa_n, gf_ls_stats *stats);

/* Apply stencils (Eq. GFDM_Definition) in differenced form:
 *   out[s][i] = sum_{j in S_i, j != i} c_ij^s (u_j - u_i)
 * for each operator s selected in op_mask (bit order dx, dy, dz, lap),
 * stacked [K][n].  Weights of type wtype, 16-byte aligned (else GF_EINVAL);
 * u and out of type io; sums are accumulated in FP64. */
gf_status gf_apply_stencil(gf_ctx *ctx, const gf_nbr *nbr, gf_dtype wtype, const void *w,
                           unsigned op_mask, gf_dtype io, const void *u, void *out);

/* Autotuner for the batched kernels.  For every launch unit of nbr (per
 * model: the tiled rows with at most 128 neighbours, and the rows with more),
 * times the stencil kernel (weights of type wtype) with teams of 4, 8 and 16
 * lanes per particle and the application kernel with 4..64 lanes (median of
 * three runs each) and keeps the fastest team size in ctx (for the stencil
 * kernels 8 lanes unless 4 or 16 is more than 3% faster; 3D rows do not try
 * 4); later calls on ctx use it.  The fused kernel of gf_gfdm_weights_apply (stencils stored and
 * applied to a field) is tuned on its own.  Allocates temporary buffers and
 * synchronises.  team_out (host, may be NULL) receives 24 ints indexed by
 * (model, band): the stencil team sizes (bulk bands 0-3, film bands 0-3; the
 * tiled unit of a model reports in band 2, bands 0-1 keep their previous
 * values), then those of the application kernel, then those of the fused
 * kernel, in the same layout. */
gf_status gf_autotune(gf_ctx *ctx, const gf_particles *p, const gf_nbr *nbr, gf_dtype wtype, int *team_out);

/* Sets the team sizes (lanes per particle) that later calls on ctx use, in
 * the layout of gf_autotune's team_out: 24 ints, the stencil kernel's (bulk
 * bands 0-3, film bands 0-3; a model's tiled rows use band 2), then the
 * application kernel's, then the fused kernel's.  Stencil and fused entries
 * take 4, 8 or 16, application entries 4, 8, 16, 32 or 64; 0 keeps the
 * current size.  teams may be NULL (nothing changes).  previous (host, may be
 * NULL) receives the 24 sizes in effect before the call.  Any other value
 * -> GF_EINVAL and nothing changes.  For reproducible configurations and
 * tests; the results of every size agree to rounding (the team sums run in a
 * different order). */
gf_status gf_set_team_sizes(gf_ctx *ctx, const int *teams, int *previous);

/* Weights and application in one pass: computes the stencils exactly as
 * gf_gfdm_weights (GF_BATCHED) and, while they are in registers, applies them
 * to u (FP64) -> out [K][n] FP64 as gf_apply_stencil does.  w_out may be NULL
 * (stencils used once and discarded). */
gf_status gf_gfdm_weights_apply(gf_ctx *ctx, const gf_particles *p, const gf_nbr *nbr,
                                const gf_ls_params *params, gf_dtype wtype, void *w_out,
                                unsigned op_mask, const double *u, double *out,
                                int8_t *status_n);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, hosts that forbid hipMalloc): the same
 * computation and outputs as gf_gfdm_weights_apply, with every temporary
 * buffer (fallback queue and its counter, QR panels, packed positions) taken
 * from a fixed workspace of gf_noalloc_workspace_bytes() = 128 MiB that the
 * library holds on each device until the process ends.  The call allocates
 * nothing (no hipMalloc / hipFree, no growth of the context's arena); the
 * caller still passes inputs and outputs.  A call whose workspace would exceed
 * the fixed size (about 4 n bytes + 30 KiB per neighbour of the longest row,
 * plus 32 n bytes when rows with more than 128 neighbours exist) returns
 * GF_ECAPACITY before any launch.  Every call on a device shares that device's
 * workspace (it keeps the last call's contents; the call clears its counter
 * itself): calls that overlap on one device, from any context or stream,
 * race and must be ordered by the caller. */
gf_status gf_gfdm_weights_apply_noalloc(gf_ctx *ctx, const gf_particles *p, const gf_nbr *nbr,
                                        const gf_ls_params *params, gf_dtype wtype, void *w_out,
                                        unsigned op_mask, const double *u, double *out,
                                        int8_t *status_n);
size_t gf_noalloc_workspace_bytes(void);

/* ---------------------------------------------------------- pressure solve */
enum { GF_ROW_INTERIOR = 0, GF_ROW_DIRICHLET = 1, GF_ROW_NEUMANN_COMBINED = 2,
       GF_ROW_NEUMANN = 3, GF_ROW_IMPLICIT = 4 };

/* Pressure-system matrix values on the neighbour pattern (implicit pressure
 * Poisson step of the projection scheme, Sec. 2.3; PDE + zeta*BC rows of
 * Sec. 7.2):  row type 0: A_ij = c_ij^lap; 1: A_ij = delta_ij; 2: A_ij =
 * c_ij^lap + (zeta/h_i) n_i . c_ij^grad; 3: A_ij = n_i . c_ij^grad.
 * w64 [nnz][4] FP64 stencils; row_type int8 [n]; val_out FP64 [nnz]. */
gf_status gf_poisson_assemble(gf_ctx *ctx, const gf_particles *p, const gf_nbr *nbr,
                              const double *w64, const int8_t *row_type, double zeta,
                              double *val_out);

typedef struct {
  double rtol;        /* stop when ||b - A x||_2 <= rtol ||b||_2 (FP64 residual), 1e-8 */
  int maxit;          /* iteration limit (inner iterations in mixed mode), 20000 */
  int mixed;          /* 0: FP64 Jacobi-BiCGStab.
                         1: the same iteration with its SpMV on FP32 matrix
                         values (Krylov vectors, dots and updates FP64); the
                         recursive residual is replaced by the FP64 residual
                         b - A x (FP64 matrix) whenever it has fallen 100-fold
                         since the last replacement and before convergence is
                         declared (no restart of the Krylov space).
                         2: iterative refinement with restarts: r = b - A x in
                         FP64, an inner Jacobi-BiCGStab on FP32 values and FP32
                         vectors solves A d = r, x += d. */
  double inner_rtol;  /* mixed = 2: relative reduction per inner solve, 1e-4 (an
                         inner solve never aims below half the overall target) */
  int inner_maxit;    /* mixed = 2: inner iteration limit per refinement, 2000 */
  double zeta;        /* combined Neumann rows, 0.3 (Sec. 7.2) */
  int check_every;    /* iterations between host convergence checks, 4 */
  double implicit_a;  /* a of GF_ROW_IMPLICIT rows, A_ij = delta_ij - a c_ij^lap: one
                         implicit Euler step of a diffusion equation (a = dt kappa), 0 */
} gf_solve_params;
void gf_solve_params_default(gf_solve_params *p);

typedef struct {
  int outer_its;        /* mixed = 1: 1 + residual replacements; mixed = 2:
                           refinement steps; 1 in plain mode */
  int inner_its_total;  /* BiCGStab iterations in total */
  int restarts;         /* restarts from the true residual: after a breakdown, or after a
                           half step that solved the system (t = A shat = 0) */
  int converged;
  double final_rel_res; /* ||b - A x|| / ||b|| in FP64 at exit */
  double seconds;       /* host wall time of the call (it synchronises) */
} gf_solve_stats;

/* Solve A p = rhs with A assembled as in gf_poisson_assemble from FP64
 * stencils w64.  Right-preconditioned BiCGStab with the Jacobi (diagonal)
 * preconditioner.  p_inout: initial guess in, solution out (FP64, device).
 * Synchronises (convergence checks).  Returns GF_ENOTCONV if the tolerance is
 * not reached within maxit, or (FP64 mode) if three restarts after
 * breakdowns in a row fail to cut the true residual by 10% (the tolerance lies
 * below the attainable accuracy); p_inout then holds the last iterate and
 * stats->final_rel_res the residual reached.
 * Ghost particles (Sec. 6.2): rows of type GF_ROW_DIRICHLET whose right-hand
 * side and initial guess hold the known ghost values keep those values, and
 * the regular rows then solve A_rr p_r = rhs_r - A_rg p_g.
 * Besides the row types of gf_poisson_assemble, rows of type GF_ROW_IMPLICIT
 * (A_ij = delta_ij - a c_ij^lap, a = params->implicit_a) give implicit Euler
 * steps of a diffusion equation (gf_poisson_assemble rejects them). */
gf_status gf_poisson_solve(gf_ctx *ctx, const gf_particles *p, const gf_nbr *nbr,
                           const double *w64, const int8_t *row_type, const double *rhs,
                           double *p_inout, const gf_solve_params *params,
                           gf_solve_stats *stats);

/* ---------------------------------------------------------- 3D -> 2D */
/* Transition of flagged 3D wall particles to the film (Sec. 5.1, Alg. 3).
 * flag (uint8 [n], 1 = bulk->film) as from gf_classify_pca.  Candidates are
 * interior / free-surface 3D neighbours of flagged particles; each candidate
 * b is mapped to the nearest wall particle of S_b (smaller index on ties)
 * and deleted iff that wall particle is flagged.  For flagged i with mapped
 * set T_i: rho and phi are averaged over {i} + T_i, m_out = m_i + sum_T m_b,
 * height_out = max_T |(x_b - x_i) . n_i| (0 if T_i is empty), diam_out =
 * (6 m_out / (pi rho_out))^(1/3).  Other kept particles copy m, rho, phi and
 * get height = diam = 0; deleted ones get m_out = 0.  keep_out (uint8) and
 * owner_out (int32, -1 if kept) describe the deletion.  nbr: same-model
 * neighbourhoods.  All arrays device, length n. */
gf_status gf_transition_3d_to_2d(gf_ctx *ctx, const gf_particles *p, const gf_nbr *nbr,
                                 const uint8_t *flag, const double *mass, const double *rho,
                                 const double *phi, double *mass_out, double *rho_out,
                                 double *phi_out, double *height_out, double *diam_out,
                                 uint8_t *keep_out, int32_t *owner_out);

/* ---------------------------------------------------------- coupling layer */
/* Particles created by gf_transition_2d_to_3d or gf_buffer_zone: caller-owned
 * device arrays (structure of arrays) with room for `cap` particles each.
 * x, y, z, h, model, kind, nx, ny, nz, mass and rho are required when cap > 0;
 * phi holds nphi fields, field f at phi[f * cap + t]; height, diam and src
 * (index of the particle a new one was made from) may be NULL. */
typedef struct {
  int64_t cap;
  double *x, *y, *z, *h;
  int8_t *model, *kind;
  double *nx, *ny, *nz;
  double *mass, *rho;
  double *phi;
  double *height, *diam;
  int32_t *src;
} gf_new_particles;

/* largest number of particles a 2D->3D transition adds to one film particle */
enum { GF_MAX_GAMMA = 65536 };

/* Film height of the droplet model (Eq. Height, Sec. 2.4): for every film
 * particle i
 *   H_i = sum_{j in S_i} alpha / (pi h_j^2) exp(-alpha |x_j - x_i|^2 / h_j^2) V_j,
 * V_j = pi d_j^3 / 6, over the same-model neighbourhood `same` (which holds
 * i); 3D particles get 0.  diam [n] FP64: droplet diameters (read for film
 * particles).  alpha > 0: the paper obtains it from a mass-conservation
 * condition of the droplet model it cites; here it is a parameter.
 * height_out [n] FP64. */
gf_status gf_film_height(gf_ctx *ctx, const gf_particles *p, const gf_nbr *same, const double *diam,
                         double alpha, double *height_out);

/* 2D -> 3D transition (Sec. 5.2, Alg. 4) of the film particles i with
 * flag[i] == 2 (film -> bulk, as gf_classify_pca marks them).  With the film
 * height H_i, the inward unit normal n_i and the 3D resolution h3d_i at the
 * particle: psi~ = (r_min h3d_i + r_max h3d_i) / 2 (Eq. psi~), gamma_i =
 * ceil(H_i / psi~) (Eq. gamma; 0 unless H_i > 0) and psi = H_i / gamma_i.
 * Each such particle yields 1 + gamma_i 3D particles in `out`, consecutive
 * and in ascending order of i: first the particle itself as a wall particle,
 * then x_i + (k psi) n_i for k = 1..gamma_i, the last a free-surface particle
 * and the others interior.  All get h = h3d_i, the normal n_i, density rho_i
 * and the nphi fields of i (phi [nphi][n]) copied, the mass m_i / (1 +
 * gamma_i), height = diam = 0 and src = i.  Not part of this call: the wall
 * re-spacing of Alg. 4 and a free-surface check of the added particles
 * (point-cloud management).  r_min > 0, r_max >= r_min: the spacing factors
 * of Sec. 2.3.  *count (host) receives the number of new particles; above
 * out->cap the call returns GF_ECAPACITY and writes nothing.  GF_EINVAL if
 * some gamma_i would exceed GF_MAX_GAMMA.  Synchronises. */
gf_status gf_transition_2d_to_3d(gf_ctx *ctx, const gf_particles *p, const uint8_t *flag,
                                 const double *film_height, const double *h3d, double r_min,
                                 double r_max, const double *mass, const double *rho,
                                 const double *phi, int nphi, gf_new_particles *out,
                                 int64_t *count);

/* Buffer zone, first loop of Alg. 5 (Sec. 6.1): flag_out[i] = 1 iff a
 * particle of the other model lies within the support of i (Eq. Nbd).  The
 * relation is symmetric, so both particles of every cross-model pair are
 * flagged.  same / cross: same-model and cross-model neighbourhoods of p
 * (the flag is whether their rows differ in length).  flag_out uint8 [n]. */
gf_status gf_buffer_flags(gf_ctx *ctx, const gf_particles *p, const gf_nbr *same,
                          const gf_nbr *cross, uint8_t *flag_out);

/* Ghost particles of the buffer zone (Sec. 6.1, Alg. 5).  Each particle
 * flagged by gf_buffer_flags gets a ghost of its own model at its place, and
 * the ghosts then change model:
 *  - 3D ghosts as in Sec. 5.1 with every wall ghost transitioning: an
 *    interior or free-surface ghost b is mapped onto the nearest wall ghost
 *    of its support (smaller index on ties) and deleted; a wall ghost i
 *    becomes a 2D ghost with rho and the fields averaged over i and the ghosts
 *    mapped onto it, the masses lumped, height = max |(x_b - x_i) . n_i|
 *    and diam = (6 m / (pi rho))^(1/3).  Interior or free-surface ghosts with
 *    no wall ghost in their support are dropped.
 *  - 2D ghosts as in gf_transition_2d_to_3d, with h_other as the 3D
 *    resolution.
 * h_other [n]: resolution of the other model at each particle (the h of the
 * ghosts made from it).  film_height [n] (read for film particles), mass,
 * rho [n], phi [nphi][n] FP64.  Ghosts come out in ascending order of their
 * source particle (src), the 1 + gamma ghosts of a film particle in the
 * order of gf_transition_2d_to_3d.  flag_out (uint8 [n], may be NULL)
 * receives the buffer flags.  *count, capacity and errors as in
 * gf_transition_2d_to_3d.  Synchronises.
 * Derivatives with ghosts (Sec. 6.2): append the ghosts to the particles,
 * build gf_build_neighbours_rows with n_rows = the regular count, then
 * compute stencils as usual.  In an implicit solve give ghost rows type
 * GF_ROW_DIRICHLET with the known ghost values as right-hand side and
 * initial guess: the regular rows then solve A_rr p_r = b_r - A_rg p_g. */
gf_status gf_buffer_zone(gf_ctx *ctx, const gf_particles *p, const gf_nbr *same, const gf_nbr *cross,
                         const double *film_height, const double *h_other, double r_min,
                         double r_max, const double *mass, const double *rho, const double *phi,
                         int nphi, gf_new_particles *out, int64_t *count, uint8_t *flag_out);

/* The 3D -> 2D transition applied to the cloud (Sec. 5.1, Alg. 3, including
 * its last loop: the transitioning particles leave the 3D model and join the
 * 2D one).  Deletion sets and data mapping as in gf_transition_3d_to_2d, for
 * density and every one of the nphi fields (phi [nphi][n]).  out receives the
 * new cloud: the particles of p in their order, without the deleted ones;
 * positions and normals copied; flagged particles (flag[i] == 1) become film
 * particles (model 1, kind wall) with h = h_film[i] (the film resolution at
 * their place; h_i if h_film is NULL), lumped mass, averaged density and
 * fields, height = max |(x_b - x_i) . n_i| and diam = (6 m/(pi rho))^(1/3);
 * all others keep h, model, kind, mass, density and fields, and film
 * particles their film_height and diam (either may be NULL: 0; bulk: 0).
 * src = index in p.  nbr: same-model neighbourhoods.  *count, capacity and
 * errors as in gf_transition_2d_to_3d.  Synchronises. */
gf_status gf_transition_3d_to_2d_cloud(gf_ctx *ctx, const gf_particles *p, const gf_nbr *nbr,
                                       const uint8_t *flag, const double *mass, const double *rho,
                                       const double *phi, int nphi, const double *film_height,
                                       const double *diam, const double *h_film,
                                       gf_new_particles *out, int64_t *count);

/* ---------------------------------------------------------- adjoints */
/* Transpose of gf_apply_stencil with respect to u: ubar = C^T ybar, where
 * ybar [K][n] FP64 holds dL/dout; ubar [n] FP64 is overwritten.
 * Deterministic (gathers through the reverse-edge map, no atomics).  With
 * extended neighbourhoods (gf_build_neighbours_rows) the ghost particles,
 * whose rows hold only themselves, receive nothing from the rows that list
 * them; every other term is as for symmetric lists. */
gf_status gf_apply_stencil_adjoint(gf_ctx *ctx, const gf_nbr *nbr, gf_dtype wtype,
                                   const void *w, unsigned op_mask, const double *ybar,
                                   double *ubar);

/* Gradient with respect to particle positions of L(out), out =
 * gf_apply_stencil(gf_gfdm_weights(p), u), given ybar = dL/dout [K][n] FP64
 * and u [n] FP64.  The stencils are recomputed, not stored (FP64 normal
 * equations, LDL^T).  xbar_3n ([n][3] FP64) is accumulated (+=).
 * status_n (int8 [n], device, may be NULL): the statuses the forward
 * gf_gfdm_weights / gf_gfdm_weights_apply call reported; rows with status 2
 * (rank deficient by the QR test) or 3 (fewer neighbours than monomials) have
 * constant zero stencils and contribute nothing.  Without it the rows with
 * fewer neighbours than monomials and those whose Gram matrix has a pivot
 * that is not positive contribute nothing (a nearly rank-deficient row that
 * the forward QR test zeroes may then still contribute: pass the statuses).
 * Each entry (i, j) moves x_i; it moves x_j through the twin entry (j, i), so
 * with extended neighbourhoods (gf_build_neighbours_rows) the ghost
 * particles, whose rows hold only themselves, receive nothing. */
gf_status gf_gfdm_weights_adjoint(gf_ctx *ctx, const gf_particles *p, const gf_nbr *nbr,
                                  const gf_ls_params *params, unsigned op_mask,
                                  const double *u, const double *ybar, const int8_t *status_n,
                                  double *xbar_3n);

#ifdef __cplusplus
}
#endif
#endif /* GFDM_H */
