/*
 * tem.h -- C ABI of libtem: pole-shifted sparse solves for transient EM
 * (rational approximation of the matrix exponential), gfx950 / MI355X.
 *
 * The calls follow the statement of the problem in Boerner, Guettel &
 * Guenther, "Scalable Parallel 3-D TEM Inversion via Rational Approximation
 * of the Matrix Exponential":
 *   - semi-discrete system K u + M du/dt = 0, M u(0) = f  (section "Spatial
 *     discretization");
 *   - u(t_j) ~ 2 Re sum_i alpha_i^[j] (K - xi_i M)^{-1} f  (section "Rational
 *     approximation using RKFIT");
 *   - Algorithm 1 (form A_i = K - xi_i M, factor once, cache, solve g_i);
 *   - d_j = Q u(t_j), data stacked over times (section "The Inverse Problem");
 *   - J v and J^T w through the same cached factors (section "Jacobian
 *     computation");
 *   - the Gauss-Newton step by LSQR on the augmented system (section
 *     "Optimization").
 *
 * Discretisation: uniform hexahedral mesh, lowest-order edge elements, DOF =
 * line integral of E along an edge, tangential E = 0 on the outer boundary.
 * Canonical edge numbering (used by every edge-indexed array of this ABI):
 *   x-edges (i,j,k), i<nx, j<=ny, k<=nz:  i + nx*(j + (ny+1)*k)
 *   y-edges (i,j,k), i<=nx, j<ny, k<=nz:  Ex + i + (nx+1)*(j + ny*k)
 *   z-edges (i,j,k), i<=nx, j<=ny, k<nz:  Ex + Ey + i + (nx+1)*(j + (ny+1)*k)
 * with Ex = nx(ny+1)(nz+1), Ey = (nx+1)ny(nz+1); cells (i,j,k) are numbered
 * i + nx*(j + ny*k).  Boundary (PEC) edges are not unknowns: inputs on them
 * are ignored and outputs on them are zero.
 *
 * Conventions
 *   Ownership: caller buffers are borrowed for the duration of a call; the
 *     library owns K, M, the symbolic structure, the factors, the cached
 *     solutions g_i and all work space, and frees them in tem_destroy.
 *   Memory spaces: every argument says "device" or "host".  Device
 *     pointers must be allocated on the context's device.
 *   Streams: device work is ordered on the context's stream; calls return
 *     once their results are in the caller's buffers (the library
 *     synchronises its stream before returning).  In FP32 mode the
 *     factorisation also runs the pole-independent nodal factor on a private
 *     stream, forked from and joined back into the context's stream within
 *     the call.
 *   Environment (read by tem_create; tuning and test knobs, defaults in
 *     brackets): TEM_PANEL factor panel width, a multiple of 32 [256];
 *     TEM_LEFT_LOOKING panels take earlier panels' updates at once [1];
 *     TEM_UPDATE_TILE "64" | "128x64" | "128" [64]; TEM_UPDATE_3M "f32" |
 *     "f64" | "both" | "none" [f32]; TEM_SWEEP_BLOCK column block of wide
 *     fronts in the sweeps, a multiple of 32 [256]; TEM_SWEEP_BIG_LIMIT
 *     fronts x poles below which an FP64 level counts as wide [1024];
 *     TEM_GRAPHS replay the all-pole sweep from a HIP graph [1].  With FP32
 *     factors and TEM_SWEEP_BLOCK at most 256 the wide fronts' diagonal
 *     blocks are inverted once per factorisation and applied as products.
 *     The autotuner (tem_autotune) overrides the update tile per level.
 *   Errors: a negative tem_status; tem_last_error() describes it.  After an
 *     error the context keeps the last stage that completed.
 *   State machine: create -> assemble -> analyse -> factor_poles ->
 *     {solve_poles | forward} -> {jvp, vjp, gn_step}*.  A new tem_assemble
 *     on the same mesh keeps the symbolic structure and drops factors and
 *     cached solutions; a different mesh also drops the symbolic structure.
 *     Calls out of order return TEM_ESTATE.
 *   Determinism: identical inputs give bitwise identical outputs on the
 *     same device (no floating-point atomics).
 *   Threading: one context per host thread.
 *   Pole convention: A_i = K - xi_i M with Im(xi_i) > 0; the conjugate poles
 *     are implicit through 2 Re (section "Comparison to other numerical
 *     approaches": 42 poles give 21 complex systems).  Complex numbers are
 *     (re, im) pairs of doubles.
 */
#ifndef TEM_H
#define TEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tem_ctx tem_ctx;

typedef enum {
  TEM_OK = 0,
  TEM_EINVAL = -1,   /* bad argument (NULL, size, range, non-finite input) */
  TEM_ENOMEM = -2,   /* device or host allocation failed / budget exceeded */
  TEM_EDEVICE = -3,  /* HIP runtime error */
  TEM_ESTATE = -4,   /* call out of order */
  TEM_EPIVOT = -5,   /* zero or non-finite pivot in the LDL^T factorisation */
  TEM_ENOCONV = -6   /* refinement did not reach the requested tolerance */
} tem_status;

typedef enum {
  TEM_FP64 = 0,     /* complex FP64 factors, FP64 solves, FP64 refinement */
  TEM_FP32_IR = 1   /* complex FP32 factors; classical iterative refinement
                       on FP64 residuals, each FP32 solve followed by the
                       FP64 Galerkin correction on the gradient space
                       z += G (G^T A G)^{-1} G^T (r - A z) (one real nodal
                       factor of G^T M G serves every pole, since K G = 0) */
} tem_precision;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `hip_device`.  `hip_stream` (host value of a
 * hipStream_t, may be NULL) is the stream all device work is ordered on;
 * NULL makes the library create its own.  *out receives the context. */
tem_status tem_create(tem_ctx **out, int hip_device, void *hip_stream);

/* Free every library allocation of ctx.  NULL-safe. */
void tem_destroy(tem_ctx *ctx);

/* Text of the last error on ctx (or, when ctx is NULL, of the calling
 * thread's last failed tem_create).  Valid until the next call on ctx (or
 * the thread's next tem_create). */
const char *tem_last_error(const tem_ctx *ctx);

/* ------------------------------------------------------------- assembly */

typedef struct {
  int32_t nx, ny, nz;  /* cells per axis, each >= 2 */
  double h;            /* cell size (m), > 0 */
  double mu;           /* magnetic permeability (H/m), > 0 */
} tem_mesh;

/* Assemble K (curl-curl stiffness, 1/mu int curl N_a . curl N_b) and
 * M (int sigma N_a . N_b) over the interior edges on the device, FP64
 * (section "Spatial discretization").
 *   sigma_cells  device, nx*ny*nz doubles (S/m), all > 0 and finite.
 *   n_params     number of model parameters P (m = ln sigma on these cells,
 *                section "The Inverse Problem"); 0 disables jvp/vjp.
 *   param_cells  host, P distinct cell ids (any order; parameter p is cell
 *                param_cells[p]).  Copied. */
tem_status tem_assemble(tem_ctx *ctx, const tem_mesh *mesh, const double *sigma_cells,
                        int32_t n_params, const int32_t *param_cells);

/* Set sigma = exp(m) on the parameter cells (m = ln sigma, section "The
 * Inverse Problem"; other cells keep their conductivity) and re-assemble M.
 * Drops factors and cached solutions.
 *   m  device, P doubles (parameter order of tem_assemble), finite. */
tem_status tem_set_model(tem_ctx *ctx, const double *m);

/* Inspection: copy the assembled operators to host memory in the current
 * unknown ordering (after tem_analyse: the nested-dissection ordering).
 * Each output may be NULL.
 *   perm    [N]     perm[q] = unknown index of row q (unknowns numbered in
 *                   increasing canonical edge order)
 *   rowptr  [N+1], col [nnz] (row-sorted), kval [nnz], mval [nnz]
 * nnz is tem_symbolic_info.nnz_a (or call with NULL arrays and read *nnz). */
tem_status tem_export_operators(const tem_ctx *ctx, int64_t *n_unknowns, int64_t *nnz,
                                int32_t *perm, int64_t *rowptr, int32_t *col, double *kval,
                                double *mval);

/* --------------------------------------------------------- symbolic phase */

typedef struct {
  int32_t leaf_max_cells;   /* nested-dissection leaf size (<= 0: 4) */
} tem_analyse_opts;

typedef struct {
  int64_t n_unknowns;       /* N */
  int64_t nnz_a;            /* entries of the CSR pattern of A_i (both triangles) */
  int64_t nnz_l;            /* entries of L incl. diagonal (supernodal) */
  int64_t n_rows_total;     /* sum over supernodes of |U_s| */
  int32_t n_supernodes;
  int32_t n_levels;
  int32_t max_front;        /* max over supernodes of k_s + |U_s| */
  int32_t reserved;
  double flops_per_pole;    /* real flops of one complex partial LDL^T sweep */
} tem_symbolic_info;

/* Nested-dissection ordering and supernodal symbolic factorisation of the
 * common pattern of all A_i (one structure serves every pole: section
 * "Computational performance").  Host work; uploads maps to the device and
 * re-lays K and M out in the new ordering.  info may be NULL. */
tem_status tem_analyse(tem_ctx *ctx, const tem_analyse_opts *opts, tem_symbolic_info *info);

/* Host-only symbolic analysis of an nx*ny*nz mesh without a context or a
 * GPU (same algorithm as tem_analyse).  Outputs, all host and optional
 * (NULL skips):
 *   perm       [N]      perm[new] = unknown index (unknowns numbered in
 *                       increasing canonical edge order)
 *   sn_ptr     [ns+1]   columns of supernode s are new indices
 *                       sn_ptr[s] .. sn_ptr[s+1]-1 (post-order)
 *   sn_parent  [ns]     parent supernode, -1 at the root
 *   rows_ptr   [ns+1]   update rows U_s are rows[rows_ptr[s] .. rows_ptr[s+1]-1]
 *   rows       [n_rows_total]  new indices, increasing within a supernode
 * Call once with NULL arrays to learn the sizes from info. */
tem_status tem_symbolic_host(int32_t nx, int32_t ny, int32_t nz, int32_t leaf_max_cells,
                             tem_symbolic_info *info, int32_t *perm, int32_t *sn_ptr,
                             int32_t *sn_parent, int64_t *rows_ptr, int32_t *rows);

/* ---------------------------------------------------- tetrahedral meshes
 * The paper's discretisation (section "Spatial discretization": lowest-order
 * curl-conforming elements on tetrahedra) and regulariser (section
 * "Regularization": RT0 smoothness with a lumped mass).  A context holds
 * either a hexahedral mesh (tem_assemble) or a tetrahedral one; every
 * single-mesh call after assembly works on either, in both precisions (the
 * gradient-space correction of TEM_FP32_IR uses the interior nodes of the
 * tetrahedra: G^T M G = sum_T sigma_T |T| grad l_i . grad l_j); batches are
 * hexahedral only.
 *
 * Canonical edges of a tetrahedral mesh are the distinct node pairs (a, b),
 * a < b, of its tetrahedra sorted lexicographically and oriented a -> b;
 * sources (tem_forward's F, tem_solve_poles) and receiver columns use this
 * numbering.  The unknowns are the edges on no boundary face (a face of one
 * tetrahedron only), in canonical order. */

typedef struct {
  int64_t n_nodes;      /* >= 4 */
  int64_t n_tets;       /* >= 1, at most 2^31 / 36 - 1 */
  const double *xyz;    /* host, 3 * n_nodes coordinates (m), finite */
  const int32_t *tets;  /* host, 4 * n_tets node ids, distinct per tetrahedron;
                           every tetrahedron of nonzero volume (either
                           orientation); a face belongs to at most two */
  double mu;            /* magnetic permeability (H/m), > 0 */
} tem_tet_mesh;

/* Assemble K (1/mu int curl N_a . curl N_b) and M (int sigma N_a . N_b)
 * over the unknown edges on the device, FP64: element matrices per
 * tetrahedron in one kernel, then a gather of the pattern entries.
 *   sigma_tets   device, n_tets doubles (S/m), > 0 and finite
 *   n_params     P (m = ln sigma on these tetrahedra); 0 disables jvp/vjp
 *   param_tets   host, P distinct tetrahedron ids.  Copied.
 * The mesh arrays are copied.  The regulariser of tem_gn_step and
 * tem_invert is then R = diag(d)^(-1/2) D^T: one row (m_b - m_a) / sqrt(d_f)
 * per face shared by two parameter tetrahedra a < b (faces in increasing
 * order of their sorted node triple), d_f the diagonal of the RT0 mass of
 * the face's unit-flux function over both tetrahedra, so R^T R =
 * D diag(M_div)^-1 D^T with the lumped M_div (no flux through the other
 * faces).  Errors: TEM_EINVAL for invalid meshes (message names the
 * defect), parameters or conductivities. */
tem_status tem_assemble_tet(tem_ctx *ctx, const tem_tet_mesh *mesh, const double *sigma_tets,
                            int32_t n_params, const int32_t *param_tets);

/* Host-only symbolic analysis of a tetrahedral mesh (the ordering
 * tem_analyse computes for it): nested dissection of the unknown graph
 * (unknowns sharing a tetrahedron), each subgraph of more than
 * 3 * leaf_max_cells^3 unknowns split at the median edge midpoint along its
 * longest extent, the separator being a minimum vertex cover of the edges
 * cut by the split.
 * Outputs as tem_symbolic_host (nnz_a is that of the unknown graph). */
tem_status tem_symbolic_tet_host(const tem_tet_mesh *mesh, int32_t leaf_max_cells,
                                 tem_symbolic_info *info, int32_t *perm, int32_t *sn_ptr,
                                 int32_t *sn_parent, int64_t *rows_ptr, int32_t *rows);

/* ---------------------------------------------------------- factorisation */

typedef struct {
  int64_t mem_budget_bytes; /* <= 0: 92% of free device memory */
  int32_t max_group;        /* poles factored together (<= 0: as many as fit) */
  int32_t reserved;
} tem_factor_opts;

/* Form A_i = K - xi_i M and compute A_i = P^T L D L^T P (complex
 * symmetric, no pivoting, no conjugation) for all m poles with a batched
 * multifrontal method; the factors stay cached on the device (Algorithm 1).
 *   xi    host, 2*m doubles (re, im); Im > 0 required.
 *   opts  may be NULL.
 * Poles are factored in groups when the contribution blocks of all poles do
 * not fit beside the factors; the grouping is reported by tem_get_stats.
 * Memory: the factor storage (and, while at least 32 GiB stay free, the
 * contribution-block arenas) remains allocated in the context and is reused
 * by the next call of the same size (a new model in a Gauss-Newton loop);
 * the budget counts it as available.  A different mesh, leaf size or
 * tem_destroy gives it back. */
tem_status tem_factor_poles(tem_ctx *ctx, int32_t m, const double *xi, tem_precision prec,
                            const tem_factor_opts *opts);

/* -------------------------------------------------------------- solves */

typedef struct {
  double rtol;          /* target ||f - A x||_2 / ||f||_2 per system (<= 0: 1e-10) */
  int32_t max_iter;     /* max refinement solves per system (<= 0: 200) */
  int32_t reserved;     /* ignored */
} tem_ir_opts;

typedef struct {
  int32_t *iters;        /* host, m*nrhs or NULL: solves spent per system */
  double *final_rel_res; /* host, m*nrhs or NULL: last residual ratio */
  int32_t n_unconverged; /* systems above rtol after max_iter */
  int32_t reserved;
} tem_ir_stats;

/* g_is = A_i^{-1} f_s for every pole i and right-hand side s, refined in
 * FP64 to ir->rtol (Algorithm 1, the shifted solve of each pole); caches g for
 * tem_jvp / tem_vjp.  Up to 16 right-hand sides share one pass over the
 * factors; more (up to 1024) are solved in equal blocks of at most 16.
 *   nrhs 1..1024.
 *   F    device, n_edges x nrhs doubles, column-major (column s = f_s).
 *   G    device or NULL: m x nrhs x n_edges complex doubles (interleaved
 *        re, im; pole slowest, edge fastest); boundary edges get 0.
 *   ir, stats may be NULL.
 * Returns TEM_ENOCONV (after filling G and stats) if some system missed
 * the tolerance. */
tem_status tem_solve_poles(tem_ctx *ctx, int32_t nrhs, const double *F, double *G,
                           const tem_ir_opts *ir, tem_ir_stats *stats);

/* Forward map: tem_solve_poles for the S sources, then
 * d[s][j][r] = 2 Re sum_i alpha[j][i] (Q g_is)_r  (Algorithm 1's final
 * linear combination followed by the observation operator).
 *   F      device, n_edges x S (as in tem_solve_poles).
 *   Q      host CSR with R rows over canonical edge columns: q_ptr[R+1]
 *          (int64), q_col[nnz] (int32), q_val[nnz] (double).  Copied.
 *   alpha  host, K x m complex (re, im interleaved; time slowest).  Copied.
 *   d      device, S*K*R doubles, layout [s][j][r].
 * Also fixes S, Q and alpha for later tem_jvp / tem_vjp calls.  A call
 * that fails while taking the new Q and alpha or while solving drops the
 * cached survey: tem_jvp, tem_vjp and tem_gn_step return TEM_ESTATE until a
 * tem_forward succeeds (or ends in TEM_ENOCONV, which still fills d). */
tem_status tem_forward(tem_ctx *ctx, int32_t S, const double *F, int32_t R,
                       const int64_t *q_ptr, const int32_t *q_col, const double *q_val,
                       int32_t K, const double *alpha, const tem_ir_opts *ir, double *d,
                       tem_ir_stats *stats);

/* J v with J = d d / d m, m = ln sigma on the parameter cells (section
 * "Jacobian computation"): J v = 2 Re sum_i alpha_i^[j] xi_i Q A_i^{-1}
 * [dM/dm g_i v], through the cached factors.
 *   v   device, P doubles.   jv  device, S*K*R doubles ([s][j][r]). */
tem_status tem_jvp(tem_ctx *ctx, const double *v, double *jv, const tem_ir_opts *ir,
                   tem_ir_stats *stats);

/* J^T w = 2 Re sum_i xi_i [dM/dm g_i]^T A_i^{-1} Q^T (sum_j alpha_i^[j] w_j)
 * (plain transpose: A_i is complex symmetric).
 *   w   device, S*K*R doubles ([s][j][r]).   jtw  device, P doubles. */
tem_status tem_vjp(tem_ctx *ctx, const double *w, double *jtw, const tem_ir_opts *ir,
                   tem_ir_stats *stats);

/* tem_vjp without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and state requirements as tem_vjp
 * (same kernels, launched eagerly: no graph replay, no profiling events).
 * Its work space (right-hand sides, solutions, residuals, sweep and nodal
 * vectors, norm partials) is carved from a static device array of 256 MiB
 * that every GPU the library runs on holds until the process ends; the
 * context's own work buffers are left untouched.  Supports problems whose
 * work space fits (about 8 complex FP64 vectors of m * N * S entries, e.g.
 * a 16^3 mesh with 16 poles and 8 sources); larger ones return TEM_ENOMEM
 * with the sizes in tem_last_error, before any kernel runs on the array
 * region they would have needed.  All calls on one GPU share that GPU's
 * array: calls that overlap in time on one GPU (two threads, or two
 * contexts whose streams run concurrently) race on it and give wrong
 * results.  Each call writes every scratch entry it reads before reading
 * it, so nothing carries over from an earlier call. */
tem_status tem_vjp_noalloc(tem_ctx *ctx, const double *w, double *jtw, const tem_ir_opts *ir,
                           tem_ir_stats *stats);

/* One Gauss-Newton update (section "Optimization"): runs `iters`
 * iterations of LSQR (Paige & Saunders 1982, x0 = 0, no damping) on
 *   min || [W_d J; sqrt(lambda) R] dm + [W_d (d(m) - d_obs); sqrt(lambda) R (m - m_ref)] ||
 * with J v and J^T w through the cached factors (tem_jvp / tem_vjp) and R
 * the first differences m_b - m_a over faces shared by two parameter cells
 * a < b (x-faces, then y-faces, then z-faces, each in increasing cell
 * index of the lower cell): on a uniform hex mesh the section
 * "Regularization"'s RT0 smoothness operator with a lumped mass reduces to
 * these differences up to scale and boundary treatment.  d(m) is the data
 * of the last tem_forward, which must have been run at m.
 *   d_obs, wd   device, S*K*R doubles ([s][j][r]); wd = W_d diagonal
 *   m, m_ref    device, P doubles
 *   dm          device, P doubles (output; the step, m is not updated)
 *   hist        host, iters doubles or NULL: LSQR residual estimate per iteration
 *   ir          refinement options of the inner solves (may be NULL)
 * When the bidiagonalisation ends early (rho = 0, e.g. a zero right-hand
 * side) the iterate is the least-squares solution: LSQR stops there and the
 * remaining hist entries repeat the last estimate.  A refinement that misses
 * its tolerance inside a J v or J^T w returns TEM_ENOCONV. */
tem_status tem_gn_step(tem_ctx *ctx, const double *d_obs, const double *wd, const double *m,
                       const double *m_ref, double lambda, int32_t iters, double *dm,
                       double *hist, const tem_ir_opts *ir);

/* ------------------------------------------------------------ inversion */

typedef struct {
  double lambda0;      /* initial regularisation weight, > 0 */
  double chi2_target;  /* stop once chi^2 = ||W_d (d - d_obs)||^2 / n_data <= this (<= 0: 1) */
  double c1;           /* Armijo constant (<= 0: 1e-4) */
  double eta_min;      /* smallest step length tried (<= 0: 1/32) */
  double conv_rtol;    /* an accepted step that lowers phi by less than conv_rtol * phi
                          halves lambda (<= 0: 1e-2) */
  int32_t max_gn;      /* Gauss-Newton iterations, >= 1 */
  int32_t lsqr_iters;  /* LSQR iterations per step, >= 1 */
} tem_invert_opts;

typedef struct {
  double lambda;         /* regularisation weight of the iteration */
  double chi2;           /* chi^2 at the start of the iteration */
  double phi;            /* phi = ||W_d (d - d_obs)||^2 + lambda ||R (m - m_ref)||^2 there */
  double slope;          /* grad phi^T dm of the Gauss-Newton step dm */
  double eta;            /* step length of the last trial */
  double phi_new;        /* phi after the iteration (= phi when the step was rejected) */
  double seconds;        /* wall time of the iteration: step, line search, restore */
  double factor_seconds; /* of which: factorisations of the trial (and restored) models */
  int32_t accepted;      /* 1: m += eta dm; 0: no trial down to eta_min met the condition */
  int32_t trials;        /* forward runs of the line search */
  int32_t lsqr_iters;    /* LSQR iterations of the step */
  int32_t stop;          /* 1: chi^2 <= chi2_target ended the run (no step taken) */
} tem_invert_record;

/* Gauss-Newton inversion (section "Optimization") from the model of the
 * last tem_forward, whose sources, receivers, residues, poles and
 * precision it keeps using.  Iteration: phi and chi^2 at m (stop when
 * chi^2 <= chi2_target); the step dm from LSQR as in tem_gn_step
 * (lsqr_iters iterations, at the current lambda); a backtracking line
 * search from eta = 1 that refactors every pole at m + eta dm and accepts
 * the first trial with phi(m + eta dm) <= phi(m) + c1 eta grad phi^T dm,
 * the next trial being the minimiser of the quadratic through phi(0), its
 * slope and phi(eta), kept in [eta/10, eta/2]; lambda is halved when no
 * trial down to eta_min is accepted (m stays) or when an accepted step lowers
 * phi by less than conv_rtol * phi (the adaptive cooling of the section).
 *   d_obs, wd   device, S*K*R doubles ([s][j][r]); wd = W_d diagonal
 *   m           device, P doubles: in, the model of the last tem_forward
 *               (m = ln sigma on the parameter cells); out, the final model
 *   m_ref       device, P doubles
 *   ir          refinement options of every solve (may be NULL)
 *   log         host, opts->max_gn records (one per iteration);
 *               *n_records receives how many were written
 * On return the context is factored and solved at the final model. */
tem_status tem_invert(tem_ctx *ctx, const double *d_obs, const double *wd, double *m,
                      const double *m_ref, const tem_invert_opts *opts, const tem_ir_opts *ir,
                      tem_invert_record *log, int32_t *n_records);

/* ------------------------------------------------------ ragged batches
 * Several independent meshes solved together: the per-pole shifted systems
 * of every mesh (the paper's Algorithm 1, repeated per mesh) are merged
 * into one block-diagonal system, so that each level of the multifrontal
 * factorisation and of the sweeps is one launch over the fronts of all
 * meshes and all poles.  Meshes may differ in size, pole count and source
 * count; missing poles of a mesh are not computed.  After
 * tem_assemble_batch the context is in batch mode: tem_analyse (with its
 * usual options) analyses every mesh, then tem_factor_poles_batch,
 * tem_forward_batch and (after tem_set_params_batch) tem_jvp_batch and
 * tem_vjp_batch apply.  tem_set_model, tem_factor_poles,
 * tem_solve_poles, tem_forward, tem_jvp, tem_vjp, tem_gn_step and
 * tem_export_operators return TEM_ESTATE in batch mode; tem_assemble
 * returns the context to single-mesh mode. */

/* Assemble K and M(sigma) of n_mesh meshes (1..4096).
 *   meshes       host, n_mesh descriptions (as in tem_assemble).
 *   sigma_cells  device, concatenated cell conductivities: mesh b's
 *                nx*ny*nz cells follow those of meshes 0..b-1, each block
 *                in tem_assemble's cell order.
 * The same meshes again (same sizes, h and mu) keep the analysis and only
 * refresh the values (a new model); other meshes reset the batch. */
tem_status tem_assemble_batch(tem_ctx *ctx, int32_t n_mesh, const tem_mesh *meshes,
                              const double *sigma_cells);

/* Factor A_bi = K_b - xi_bi M_b for every mesh b and each of its m[b]
 * poles (as tem_factor_poles).
 *   m    host, n_mesh pole counts (1..4096 each).
 *   xi   host, sum(m) complex poles (re, im interleaved), mesh-major:
 *        mesh b's poles follow those of meshes 0..b-1; Im > 0. */
tem_status tem_factor_poles_batch(tem_ctx *ctx, const int32_t *m, const double *xi,
                                  tem_precision prec, const tem_factor_opts *opts);

/* Forward map of every mesh (as tem_forward), with refinement to ir->rtol
 * judged per mesh, pole and source.  Blocks are concatenated mesh-major:
 *   S      host, n_mesh source counts (1..16 each).
 *   F      device, mesh b's n_edges_b x S[b] column-major block follows
 *          those of meshes 0..b-1.
 *   R      host, n_mesh receiver counts (>= 1 each).
 *   q_ptr  host, mesh b's R[b]+1 row pointers (each block starts at 0)
 *          follow those of the previous meshes; q_col / q_val: mesh b's
 *          entries (canonical edge ids of mesh b) follow likewise.
 *   K      number of times (shared by all meshes).
 *   alpha  host, mesh b's K x m[b] complex residues (time slowest) follow
 *          those of the previous meshes.
 *   d      device, mesh b's S[b]*K*R[b] doubles ([s][j][r]) follow those of
 *          the previous meshes.
 *   stats  iters / final_rel_res (if not NULL) hold n_mesh*MP*Smax entries
 *          [mesh][pole][source] with MP = max m, Smax = max S; slots past a
 *          mesh's own poles or sources read 0.
 * Returns TEM_ENOCONV (after filling d and stats) if some system missed
 * the tolerance. */
tem_status tem_forward_batch(tem_ctx *ctx, const int32_t *S, const double *F, const int32_t *R,
                             const int64_t *q_ptr, const int32_t *q_col, const double *q_val,
                             int32_t K, const double *alpha, const tem_ir_opts *ir, double *d,
                             tem_ir_stats *stats);

/* Model parameters of every mesh of a batch (m = ln sigma on the given cells
 * of each mesh, section "The Inverse Problem"); needed by tem_jvp_batch and
 * tem_vjp_batch.  Kept until the batch changes meshes.
 *   n_params     host, n_mesh counts (0..cells of the mesh).
 *   param_cells  host, mesh b's n_params[b] distinct cell ids (its own cell
 *                numbering) after those of meshes 0..b-1.  Copied. */
tem_status tem_set_params_batch(tem_ctx *ctx, const int32_t *n_params, const int32_t *param_cells);

/* J v and J^T w of every mesh of a batch through the cached factors of the
 * last tem_forward_batch (as tem_jvp / tem_vjp per mesh; the adjoint and
 * tangent solves of all meshes and poles run as one merged system).
 *   v    device, mesh b's n_params[b] doubles after those of the previous meshes.
 *   jv   device, mesh b's S[b]*K*R[b] doubles ([s][j][r]) after the previous ones.
 *   w    device, laid out as jv.   jtw  device, laid out as v.
 *   stats  as tem_forward_batch. */
tem_status tem_jvp_batch(tem_ctx *ctx, const double *v, double *jv, const tem_ir_opts *ir,
                         tem_ir_stats *stats);
tem_status tem_vjp_batch(tem_ctx *ctx, const double *w, double *jtw, const tem_ir_opts *ir,
                         tem_ir_stats *stats);

/* ------------------------------------------------------------ autotuning */

typedef struct {
  int32_t n_candidates;       /* update variants timed */
  int32_t n_levels;           /* tree levels of the edge system */
  double candidate_ms[8];     /* per variant: sum over levels of the level's time */
  int32_t candidate_tile[8];  /* variant's output tile: 0 = 64x64, 1 = 128x64, 2 = 128x128 */
  int32_t candidate_m3[8];    /* 1: complex products with three real products, 0: four */
  double tuned_ms;            /* sum over levels of the fastest variant's time */
} tem_autotune_report;

/* Times the front-update kernel variants (FP32: 64x64 and 128x64 output
 * tiles, each with three or four real matrix-core products per complex
 * product; FP64: 64x64 with three or four) level by level on complete
 * factorisations of the given poles, and keeps for each level of the tree
 * the variant that was fastest there.  Every variant is timed twice, in two
 * passes over the list (the second in reverse order); a level's time is the
 * smaller of its two.  Later tem_factor_poles calls of that precision use
 * the choice until the next tem_analyse with other options or another mesh.
 * Leaves the context factored (by the first variant, timed last).
 *   m, xi, prec  as tem_factor_poles;  rep  host, may be NULL.
 * Not available on a batch of meshes. */
tem_status tem_autotune(tem_ctx *ctx, int32_t m, const double *xi, tem_precision prec,
                        tem_autotune_report *rep);

/* The tuned variant of one level (0 = root): tile as candidate_tile, m3 as
 * candidate_m3.  TEM_ESTATE if no tuning is held for that precision. */
tem_status tem_autotune_level(const tem_ctx *ctx, tem_precision prec, int32_t level,
                              int32_t *tile, int32_t *m3);

/* ------------------------------------------------------------ statistics */

typedef struct {
  int32_t n_poles;
  int32_t n_groups;            /* pole groups used by the last factorisation */
  int32_t group_size;
  int32_t precision;           /* tem_precision of the cached factors */
  int64_t factor_bytes;        /* device bytes held by the factors */
  int64_t workspace_bytes;     /* contribution-block arenas etc. */
  int32_t n_tiny_pivots;       /* pivots with |d| below 1e-300 (FP64) / 1e-30 (FP32) */
  int32_t last_solves;         /* refinement solves of the last solve call (max) */
  double factor_ms;            /* device time of the last factorisation */
  double solve_ms;             /* device time of the last solve call */
  /* filled while profiling is enabled (tem_set_profiling), accumulated
     since it was enabled: HIP-event time and algorithmic work of the MFMA
     front-update launches (flops of C -= L D L^T on the lower triangle) and
     of the triangular sweeps (bytes: factors read twice, vectors read and
     written in both passes) */
  double update_ms;
  double update_flops;
  int64_t update_launches;
  double sweep_ms;
  double sweep_bytes;
  int64_t sweeps;
} tem_stats;

tem_status tem_get_stats(const tem_ctx *ctx, tem_stats *out);

/* Enable (1) or disable (0) per-launch HIP-event timing of the front
 * updates and the sweeps, and reset the accumulated figures of tem_stats.
 * For measurement only; adds two events per timed launch. */
tem_status tem_set_profiling(tem_ctx *ctx, int32_t enable);

#ifdef __cplusplus
}
#endif
#endif /* TEM_H */
