/*
 * libsmpm — deflated Schur complement solver for the SMPM discretization of the
 * 2-D Poisson-Neumann problem (Joshi & Diamessis, arXiv 1601.03432), on AMD
 * Instinct MI355X (gfx950).
 *
 * Problem (Sec. 1.2, Eq. poisson): lap u = f on a Cartesian domain split into
 * m_y x m_x rectangular elements with n Gauss-Lobatto-Legendre points per
 * direction, n.grad u = g on the boundary.  The SMPM operator L (Eq.
 * smpm_poisson) is split as L = A + E B (Sec. 1.3) and the interface system
 * S x = b with S = I + B A^{-1} E (Eq. schur_complement_system) is solved by
 * right-preconditioned GMRES with block-Jacobi preconditioning and deflation
 * (Sec. 2, Algorithm 3, Eq. deflated_schur).
 *
 * Sign convention.  Writing the augmented system of Eq. blocksystem as a 2x2
 * block system with A_II = A, A_IG = E, A_GI = B, A_GG = -I, the textbook Schur
 * complement A_GG - A_GI A_II^{-1} A_IG equals -S.  This library uses the
 * paper's S = I + B A^{-1} E throughout.
 *
 * Data layouts (all FP64 unless stated; multi-RHS data is column-blocked, the
 * right-hand-side index outermost: v[i + len*col]):
 *   r-vectors (f, u; r = n^2 m_x m_y): node (p, q) of element e = iy*m_x + ix
 *     at e*n^2 + q*n + p, p the x index.
 *   g (boundary data, 2n(m_x + m_y) per column): south edge (m_x*n values,
 *     x ascending), north edge (m_x*n), west edge (m_y*n, y ascending), east
 *     edge (m_y*n).  g is the outward normal derivative n.grad u.
 *   k-vectors (interface grid Gamma, k = 2 n d): one slot per node of every
 *     inter-element side.  Slot = side_index*n + t, sides numbered
 *     element-major and within an element W, E, S, N (inter-element sides
 *     only); t runs along the side (q for W/E sides, p for S/N sides).  An
 *     element-corner node on two inter-element sides owns two slots.
 *   d-vectors (interfaces): vertical interfaces (between (iy,ix) and
 *     (iy,ix+1)) row-major, then horizontal ones (between (iy,ix), (iy+1,ix)).
 *
 * Discretization (Sec. 1.2, Eq. smpm_poisson).  At the nodes of an element side
 * the row of L adds tau (R u_i - R u_j) across an inter-element side and
 * tau sigma n.grad u_i on a physical side (right-hand side tau sigma g), with
 * the Robin operator R = I + sigma n_i.grad; the values of the element whose row
 * it is serve u_i and u_j alike.  Sec. 1.2 prints R = I + n.grad (sigma = 1) and
 * leaves tau to a heuristic; smpm_robin selects the reading of sigma and tau
 * (omega_0 = 2/(N(N+1)) the GLL end weight, h_perp the element's extent normal to
 * the side, h_e its smaller extent):
 *   SMPM_ROBIN_LITERAL    sigma = 1,          tau = 2 penalty / (omega_0 h_perp)
 *   SMPM_ROBIN_REFERENCE  sigma = h_perp / 2, tau = 2 penalty / (omega_0 h_perp^2)
 *                         (sigma n.grad = the normal derivative in the element's
 *                         reference coordinates [-1,1]^2)
 *   SMPM_ROBIN_MIN        sigma = h_e / 2,    tau = 2 penalty / (omega_0 h_e^2)
 *                         (default; equals REFERENCE on square elements and keeps
 *                         GMRES convergent on elements of aspect ratio up to 8,
 *                         where it is neither the physical nor the reference-
 *                         coordinate derivative)
 * Recommended penalty: 8 (any finite nonzero value is accepted).
 *
 * Ownership and streams.  A context owns its setup data and device workspace;
 * smpm_destroy releases them.  The caller owns every vector argument.  Device
 * pointers must be device memory of the current HIP device; `stream` is a
 * hipStream_t passed as void* (NULL = the default stream).  Apply/project
 * calls are asynchronous and stream-ordered; smpm_setup and smpm_solve
 * synchronize the stream before returning.  A context is used by one host
 * thread at a time.
 *
 * Errors.  Every int-returning call returns SMPM_OK (0) or a negative
 * smpm_status; smpm_last_error(ctx) gives a thread-local message.  A failed call
 * leaves outputs unspecified and the context valid.  Input and output
 * pointers must not alias (smpm_project may run in place).
 */
#ifndef SMPM_H
#define SMPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct smpm_ctx smpm_ctx;

enum smpm_status {
  SMPM_OK = 0,
  SMPM_EINVAL = -1,      /* invalid argument or grid */
  SMPM_ENOMEM = -2,      /* device or host allocation failed */
  SMPM_EHIP = -3,        /* a HIP runtime call failed */
  SMPM_ENOCONV = -4,     /* GMRES / refinement did not reach the tolerance */
  SMPM_ESINGULAR = -5,   /* an element, block or coarse factorization failed */
  SMPM_ENODEVICE = -6    /* the context was built without a device (smpm_plan) */
};

enum smpm_precision {
  SMPM_FP64 = 0,         /* everything in FP64 */
  SMPM_MIXED_FP32 = 1,   /* FP32 Schur/preconditioner applies inside FP64 refinement */
  SMPM_MIXED_BF16 = 2    /* BF16 operators, FP32 accumulation, FP64 refinement */
};

enum smpm_robin {
  SMPM_ROBIN_MIN = 0,        /* sigma = h_e/2 (default)                              */
  SMPM_ROBIN_LITERAL = 1,    /* sigma = 1: R = I + n.grad as printed in Sec. 1.2      */
  SMPM_ROBIN_REFERENCE = 2   /* sigma = h_perp/2: reference-coordinate derivative     */
};

enum smpm_projection {
  SMPM_PROJ_L = 0,       /* r-vector: x - u_L (u_L^T x)            (Eq. regularize_poisson) */
  SMPM_PROJ_S = 1,       /* k-vector: x - u_S (u_S^T x)            (Eq. regularize_schur)   */
  SMPM_PROJ_P = 2,       /* k-vector: x - S Z G Z^T x, G = C^+      (Eq. projection1)        */
  SMPM_PROJ_Q = 3,       /* k-vector: x - Z G Z^T S x               (Eq. projection2)        */
  SMPM_PROJ_MEAN = 4     /* r-vector: x - (w^T x / w^T 1) 1, w = GLL quadrature weights     */
};

enum smpm_export_what {
  SMPM_EXPORT_SCHUR = 0,        /* S, k x k, COO                          */
  SMPM_EXPORT_FLUX_SOLVE = 1,   /* B A^{-1}, k x r, COO                   */
  SMPM_EXPORT_PRECOND_INV = 2,  /* M^{-1}, k x k, COO                     */
  SMPM_EXPORT_COARSE = 3,       /* C = Z^T S Z, d x d dense row-major     */
  SMPM_EXPORT_COARSE_PINV = 4   /* G = C^+ (C^{-1} if C is nonsingular)   */
};

typedef struct smpm_solve_opts {
  double tol;         /* stop when the GMRES least-squares residual (= the Schur residual
                         |b_hat - S x|) <= tol * |b_hat| (default 1e-10); mixed precision:
                         refinement stops when the FP64 true residual meets the same bound  */
  int maxit;          /* maximum GMRES iterations per solve or refinement cycle (default 400)    */
  int precision;      /* smpm_precision (default SMPM_FP64)                                      */
  int transpose;      /* 1: adjoint of the solution map (see smpm_solve; g must be NULL)           */
  int variant;        /* 3: deflated + block-Jacobi (Algorithm 3), 2: block-Jacobi only
                         (Algorithm 2), 1: unpreconditioned (Algorithm 1); default 3               */
  double inner_tol;   /* mixed precision: inner GMRES tolerance of a refinement cycle (default
                         1e-5).  A cycle aims instead for the reduction that finishes the solve
                         (0.3 tol / residual) when one cycle at the current operator precision
                         can attain it (down to 1e-7 with FP32 operators, 1e-6 for block GMRES, 1e-3 with BF16), so
                         two cycles reach 1e-10 where the accuracy of the operators allows     */
  int max_refine;     /* mixed precision: maximum refinement cycles (default 20)                 */
  int graph;          /* 1: the Arnoldi steps run as replays of a captured hipGraph of 8 steps,
                         and the launch sequences before and after them (right-hand side,
                         projections and GMRES start; least squares, recovery of x, FP64 true
                         residual and back-substitution) as replays of two more (each captured
                         once per solve shape and context); 0: launched one by one.
                         (Environment SMPM_PREREDUCE=0/1 forces how the orthogonalization
                         sums are reduced: once per column or in every block;
                         SMPM_STREAM_BASIS=0/1 forces ordinary or non-temporal basis loads.)
                         Results are identical (default 1)                                        */
  int stop_rule;      /* reference of the GMRES stopping test: 0 (default) |b_hat|, the norm the
                         FP64 true residual is accepted against; 1 the initial GMRES residual
                         |P b_hat| (|b_hat| for Algorithms 1 and 2), the rule of Sec. 3.2.  The
                         returned solution is still accepted on its FP64 true residual          */
  int profile;        /* 1: time the solve's phases with HIP events recorded on its stream
                         (smpm_solve_info.phase_ms); 0 (default): no timing.  The environment
                         SMPM_PROFILE=1 turns it on as well                                     */
  int block;          /* 1: step 4 as block GMRES (at most 32 columns; with mixed precision the
                         inner solve of every refinement cycle, its operators FP32 or BF16): all columns
                         share one block Krylov space span{R0, op R0, ...}, R0 the deflated
                         right-hand sides, each column's residual minimized over all of it;
                         the basis is extended by block classical Gram-Schmidt applied twice
                         and Cholesky QR applied twice, and a block column whose part
                         orthogonal to the block's earlier columns is at most 1e-6 of its norm
                         adds no vector (rank deflation).  Iterations count block steps;
                         maxit caps them.  0 (default): each column its own GMRES, batched.
                         opts.graph is not used by the block path                             */
} smpm_solve_opts;

typedef struct smpm_solve_info {
  int iterations;           /* GMRES iterations, summed over refinement cycles, max over columns */
  int refinements;          /* refinement cycles (1 for FP64)                                    */
  double rel_residual;      /* max over columns of the FP64 ||b_hat - S x|| / ||b_hat||          */
  double removed_component; /* column 0: u_L^T (f + T g), the projected-out incompatibility;
                               adjoint: (1^T c)/(w^T 1), the removed multiple of w            */
  int schur_precision;      /* smpm_precision of the Schur operator in the last inner solve:
                               a mixed solve raises it (BF16 -> FP32 -> FP64) when a
                               refinement cycle contracts the residual too little         */
  double cycle_residual[16];  /* mixed precision: max over columns of the FP64 true residual
                                 at the start of refinement cycle i (i < 16; then the final
                                 one); FP64: [0] = the final residual                      */
  int cycle_iterations[16];   /* GMRES iterations of each cycle (max over columns): FP64, the
                                 solve then its correction cycles; mixed, the refinement
                                 cycles (the first 16)                                      */
  int history_len;            /* entries of history (GMRES iterations of the last cycle of
                                 column 0, plus one)                                       */
  double history[1001];       /* column 0, last GMRES cycle: the least-squares residual
                                 estimate |g_j| after j iterations relative to the stopping
                                 reference (history[0] = initial residual / reference)     */
  double phase_ms[4];         /* with opts.profile: [0] right-hand side and projections
                                 (steps 1-3) and, in FP64, the GMRES start; [1] the Arnoldi
                                 iterations (mixed: all refinement cycles); [2] FP64: least
                                 squares, recovery of x (steps 5-8), true residual, step 9
                                 and any correction cycles; mixed: step 9; [3] whole call;
                                 else zeros                                                  */
} smpm_solve_info;

typedef struct smpm_plan_stats {
  int64_t element_classes;        /* distinct element operators (shared by equal elements)      */
  int64_t block_classes;          /* distinct block-Jacobi inverses                             */
  int64_t schur_operator_bytes;   /* FP64 bytes of all distinct Schur side-flux operators        */
  int64_t precond_operator_bytes; /* FP64 bytes of all distinct block-Jacobi inverses            */
  int64_t flux_operator_bytes;    /* FP64 bytes of all distinct B A^{-1} side operators          */
  int64_t coarse_bytes;           /* FP64 bytes of the dense coarse pseudo-inverse (0 if none)   */
  int32_t coarse_singular;        /* 1 if C is singular (pseudo-inverse), 0 otherwise            */
  int32_t has_coarse;             /* 1 if the deflated solve is available                        */
  double null_residual;           /* ||S^T u_S||_2 / ||S|| of the computed left null vector u_S
                                     (||S|| taken as the bound below); -1 before the null
                                     vectors are computed.  Setup accepts <= 1e-12.            */
  int32_t null_iterations;        /* GMRES iterations (over restarts) of the null-vector solve  */
  int32_t pad_;
  double schur_norm_bound;        /* sqrt(||S||_1 ||S||_inf) >= ||S||_2                          */
} smpm_plan_stats;

typedef struct smpm_tune_result {
  int nrhs;                          /* column count the choice was made for (its class:
                                        1, 2-3, 4-7 or >= 8 columns)                         */
  int schur_columns_per_workgroup;   /* right-hand-side columns one Schur workgroup takes     */
  int schur_persistent;              /* Schur kernel: 0 plain matrix-core kernel, 1 persistent
                                        pipelined, 2 warp-specialized persistent, 3 column-
                                        pipelined (one tile, its columns one after another)  */
  int prereduce;                     /* 1: Gram-Schmidt sums reduced once per column; 0: in
                                        every consumer block; -1: not tuned (no coarse space) */
  double schur_us;                   /* measured Schur apply time of the choice               */
  double step_us;                    /* measured time per deflated Arnoldi step of the choice */
} smpm_tune_result;

/* Fills `opts` with the defaults listed above. */
void smpm_default_opts(smpm_solve_opts *opts);

/* Builds the host-side plan only (no device use): GLL grid, element operators,
 * block-Jacobi inverses and the coarse matrix, all FP64 (Secs. 1.2-2).
 * x_breaks (m_x+1) and y_breaks (m_y+1) are host arrays of strictly increasing
 * element breakpoints.  Requires m_x*m_y >= 2, 3 <= n <= 32, penalty finite and
 * nonzero.  The coarse solve with C = Z^T S Z is a dense G = C^+ for up to
 * 4096 interfaces (environment SMPM_DENSE_COARSE_MAX may lower the limit);
 * larger grids solve with C exactly by one level of substructuring: patches of
 * 8 x 8 elements (SMPM_COARSE_PATCH overrides; doubled while the separator
 * system would exceed 8192 unknowns), dense inverses of the patch-interior
 * blocks and of the separator Schur complement (bordered by u_C and tau_hat
 * when C is singular, which yields the Moore-Penrose inverse).
 * The context supports sizes/exports only; device calls on it return
 * SMPM_ENODEVICE.  *out is set only on success. */
int smpm_plan(int m_y, int m_x, int n, const double *x_breaks, const double *y_breaks,
              double penalty, smpm_ctx **out);

/* smpm_plan with a chosen reading of the Robin operator (smpm_robin; smpm_plan uses
 * SMPM_ROBIN_MIN).  SMPM_EINVAL for an unknown mode. */
int smpm_plan_robin(int m_y, int m_x, int n, const double *x_breaks, const double *y_breaks,
                    double penalty, int robin, smpm_ctx **out);

/* smpm_plan + upload to the current device.  Synchronous.  The null vectors
 * u_S (left null vector of S) and u_L (left null vector of L, Sec. 1.4) are
 * computed on first use (smpm_solve, smpm_project L/S, smpm_null_vectors) by a
 * restarted GMRES solve with the transposed Schur complement; that first call
 * returns SMPM_ESINGULAR if ||S^T u_S|| / ||S|| stays above 1e-12 (smpm_stats
 * reports the value). */
int smpm_setup(int m_y, int m_x, int n, const double *x_breaks, const double *y_breaks,
               double penalty, void *stream, smpm_ctx **out);

/* smpm_setup with a chosen reading of the Robin operator (smpm_robin; smpm_setup
 * uses SMPM_ROBIN_MIN). */
int smpm_setup_robin(int m_y, int m_x, int n, const double *x_breaks, const double *y_breaks,
                     double penalty, int robin, void *stream, smpm_ctx **out);

/* Releases everything the context owns (NULL is ignored). */
void smpm_destroy(smpm_ctx *ctx);

/* r = n^2 m_x m_y nodes, k = 2 n d interface slots, d interfaces. */
int smpm_sizes(const smpm_ctx *ctx, int64_t *r, int64_t *k, int64_t *d);

/* Sizes of the setup operators (used for algorithmic byte counts). */
int smpm_stats(const smpm_ctx *ctx, smpm_plan_stats *out);

/* Host array slot_to_node[k]: the node (r-index) each slot sits on (E as a map). */
int smpm_slot_map(const smpm_ctx *ctx, int64_t *slot_to_node);

/* Host arrays x[r], y[r]: node coordinates, as computed by the library. */
int smpm_node_coords(const smpm_ctx *ctx, double *x, double *y);

/* Host array w[r]: GLL quadrature weights omega_p omega_q w_e h_e / 4. */
int smpm_quadrature_weights(const smpm_ctx *ctx, double *w);

/* Host copies of the setup operators for inspection (see smpm_export_what).
 * COO kinds: call with rows/cols/vals NULL to get *count, then again with
 * arrays of that length.  Dense kinds: *count = d*d, vals receives them. */
int smpm_export(const smpm_ctx *ctx, int what, int64_t *count, int64_t *rows, int64_t *cols,
                double *vals);

/* Host copies of the unit null vectors uL[r], uS[k] (either may be NULL),
 * computing them on the default stream if needed.  SMPM_ENODEVICE for a
 * plan-only context. */
int smpm_null_vectors(smpm_ctx *ctx, double *uL, double *uS);

/* Sv = S v (transpose = 0) or S^T v (transpose = 1) for nrhs k-vectors
 * (Eq. schur_complement_system).  Device pointers, column-blocked.  Sv is
 * written with non-temporal stores (it is the caller's result, not reread by
 * the library). */
int smpm_schur_apply(smpm_ctx *ctx, const double *v, double *Sv, int nrhs, int transpose,
                     void *stream);

/* As smpm_schur_apply with the operator precision of a mixed-precision solve:
 * SMPM_MIXED_FP32 / SMPM_MIXED_BF16 use the FP32 / BF16 copies of the element
 * operators with FP32 accumulation (the matrix-core path of the refinement's inner
 * solves); vectors stay FP64.  SMPM_FP64 is smpm_schur_apply. */
int smpm_schur_apply_prec(smpm_ctx *ctx, const double *v, double *Sv, int nrhs, int transpose,
                          int precision, void *stream);

/* y = M^{-1} x (or M^{-T} x): the block-Jacobi preconditioner of Sec. 2 with
 * checkerboard blocks (red element slots plus the neighbours' facing slots). */
int smpm_precond_apply(smpm_ctx *ctx, const double *x, double *y, int nrhs, int transpose,
                       void *stream);

/* One of the projections of smpm_projection on nrhs vectors (r- or k-length).
 * transpose = 1 gives the projections of the adjoint solve: P^T and Q^T; for L
 * and S the orthogonal projection off the null vector of the transposed
 * operator (1/sqrt(r) for L^T, v0/|v0| for S^T); for MEAN the transpose
 * x - w (1^T x)/(w^T 1).  in == out is allowed. */
int smpm_project(smpm_ctx *ctx, int which, const double *in, double *out, int nrhs,
                 int transpose, void *stream);

/* smpm_project without any allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels in the same order as smpm_project (identical results),
 * with their scratch (the Schur product, interface sums, coarse solution and
 * substructured-solve scratch, dot partials) in a static device array of 32 MiB per
 * GPU instead of the context's workspace.  Calls no hipMalloc/hipFree.
 * Limits: SMPM_EINVAL if the call needs more than 32 MiB of scratch (about
 * (k + 2 d) nrhs doubles plus small terms; e.g. up to 3 columns on a 128 x 128,
 * n = 16 grid), and for SMPM_PROJ_L / SMPM_PROJ_S (not transposed) before the null
 * vectors exist (smpm_null_vectors or smpm_solve computes them; that allocates).
 * All contexts on one GPU share the array: calls that overlap on one GPU (other
 * streams, other host threads) race and must be ordered by the caller.  in == out is
 * allowed. */
int smpm_project_noalloc(smpm_ctx *ctx, int which, const double *in, double *out, int nrhs,
                         int transpose, void *stream);

/* Solves L u = f~ for nrhs right-hand sides by Algorithm 3 (Sec. 2):
 * f~ = (I - u_L u_L^T)(f + T g), b_S = B A^{-1} f~ projected out of u_S, GMRES
 * on P S M^{-1}, x = Q M^{-1} x_1 + Z G Z^T b_hat, u = A^{-1}(f~ - E x), and the
 * additive constant fixed by w^T u = 0.  f, u: device r x nrhs; g: device
 * 2n(m_x+m_y) x nrhs or NULL (zero Neumann data).  opts/info may be NULL.
 * Returns SMPM_ENOCONV if some column missed the tolerance (u still holds the
 * last iterate).  Synchronizes the stream. */
int smpm_solve(smpm_ctx *ctx, const double *f, const double *g, double *u, int nrhs,
               const smpm_solve_opts *opts, smpm_solve_info *info, void *stream);
/* With opts->transpose = 1 the same call applies the transpose of that linear
 * solution map u = K (f + T g): f holds a cotangent c (e.g. dLoss/du), g must be
 * NULL, and u receives mu = K^T c, i.e. the solution of L^T mu = c~ with
 * c~ = c - w (1^T c)/(w^T 1) and u_L^T mu = 0.  It runs Algorithm 3 on the
 * transposed system: S^T xi = E^T A^{-T} c~ (projected off v0), deflated GMRES
 * on P'S^T M^{-T} with P' = Q^T, Q' = P^T and G^T, then mu = A^{-T}(c~ - B^T xi).
 * Then dLoss/df = mu and dLoss/dg = T^T mu (smpm_boundary_transpose).  The
 * stopping rule and the precision options are those of the forward solve. */

/* Solves several independent problems concurrently: problem i is smpm_solve(ctxs[i],
 * f[i], g ? g[i] : NULL, u[i], nrhs[i], opts, infos ? &infos[i] : NULL) (same options
 * for all; g[i] may be NULL).  The problems run on streams of their own, each driven by
 * a host thread, ordered after the work already on `stream`, so the kernels of small
 * grids overlap on the device.  The contexts must be distinct and on one device.
 * Workspaces and null vectors are prepared first, in order (this synchronizes the
 * device).  Returns the first hard error (message prefixed with the problem index),
 * else SMPM_ENOCONV if a problem missed the tolerance, else SMPM_OK.  Synchronous. */
int smpm_solve_group(smpm_ctx *const *ctxs, int nproblems, const double *const *f, const double *const *g,
                     double *const *u, const int *nrhs, const smpm_solve_opts *opts,
                     smpm_solve_info *infos, void *stream);

/* Autotuner: times, on `stream`, the candidate launch shapes of the Schur apply
 * (1, 2 or 4 right-hand-side columns per workgroup of the plain matrix-core kernel,
 * the persistent pipelined kernel, the warp-specialized persistent kernel, or the
 * column-pipelined kernel with 2, 4 or 8 columns per workgroup) and the two ways of
 * reducing the Gram-Schmidt
 * sums (24 deflated Arnoldi steps each) for `nrhs` columns on this context's grid,
 * and keeps the fastest for every later call with a column count of the same class.
 * Every candidate computes each column with the same arithmetic in the same order,
 * so results do not change.  Synchronous; allocates the solve workspace for nrhs.
 * out may be NULL. */
int smpm_autotune(smpm_ctx *ctx, int nrhs, void *stream, smpm_tune_result *out);

/* dg = T^T mu for nrhs r-vectors mu: the gradient with respect to the Neumann
 * data (layout of g: south, north, west, east edges, 2n(m_x+m_y) per column)
 * given the gradient mu with respect to f + T g.  T places tau_i g_i on the
 * physical-boundary nodes (Eq. smpm_poisson), so dg_b = tau_b mu[node(b)].
 * Device pointers; mu and dg must not alias. */
int smpm_boundary_transpose(smpm_ctx *ctx, const double *mu, double *dg, int nrhs, void *stream);

/* Text of the last error set on the calling thread ("" if none).  The message is
 * kept per thread, not per context: ctx is accepted for the call shape of the other
 * entry points and may be NULL (errors raised before a context exists, e.g. by a
 * failed smpm_setup, are read the same way). */
const char *smpm_last_error(const smpm_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* SMPM_H */
