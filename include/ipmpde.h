/*
 * libipmpde — interior point method for sparse (L1), box-constrained
 * PDE-constrained optimal control on one AMD Instinct MI355X (gfx950).
 *
 * Problem (Pearson, Porcelli, Stoll, arXiv 1806.05896, Sec. 1, eqs. (pb),
 * (eq:lap), (box), (boxs)), in the finite-difference, unit-mass form of
 * Sec. 2, eq. (pb_fe) with M = D = I:
 *
 *   minimize  1/2 |y - y_d|^2 + alpha/2 |u|^2 + beta |u|_1
 *   s.t.      A y - u = f_hat,  u_a <= u <= u_b,  [y_a <= y <= y_b]
 *
 * where A is the 5-point (2D) or 7-point (3D) Laplacian, or (2D) the
 * upwinded convection-diffusion operator -eps Lap + w.grad with the wind
 * w = (2 x2 (1 - x1^2), -2 x1 (1 - x2^2)) of Sec. 5.2; f_hat = f minus the
 * boundary columns of A applied to the Dirichlet data g.
 *
 * The solver is the path-following method of the Appendix (Algorithm A.1)
 * with the l1 splitting u = w - v (Sec. 2, eq. (split)).  Each Newton system
 * (Sec. 3, eq. (NewtonSystem)) is solved by preconditioned MINRES with the
 * block-diagonal preconditioner P_D, or by FGMRES with the block-triangular
 * P_T (Sec. 4, the last two displayed preconditioners), whose Schur block is
 * the matching approximation S_hat = (A + M_hat)(I + Theta_y)^-1 (A + M_hat)^T
 * (Sec. 4.2, eq. (SchurApprox)) applied with geometric multigrid V-cycles.
 *
 * Conventions for every entry point:
 *   - Grid: N = 2^k - 1 interior points per axis (k >= 2), h = 1/(N+1);
 *     n = N^dim unknowns per field.
 *   - Layout: lexicographic with x1 fastest; node (i1..id) at x = (i1 h, ...).
 *     Boundary data g has (N+2)^dim entries in the same ordering including the
 *     boundary nodes; its interior entries are ignored.
 *   - Host arrays passed to problem_create are copied; the caller keeps
 *     ownership and may free them after the call.  Device arrays passed to
 *     the low-level entry points are owned by the caller.
 *   - All device work is enqueued on the stream argument (NULL = the null
 *     stream); calls that return host results synchronize that stream.
 *   - Return value: IPMPDE_OK or one of the error codes below;
 *     ipmpde_last_error() gives a thread-local message for the last failure.
 *   - A problem handle must not be used by two threads at once.
 */
#ifndef IPMPDE_H
#define IPMPDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* ipmpde_stream; /* a hipStream_t */

enum {
  IPMPDE_OK = 0,
  IPMPDE_EINVAL = 1,        /* bad shape, NaN/Inf input, infeasible bounds, bad option */
  IPMPDE_ENOMEM = 2,        /* device allocation failed */
  IPMPDE_EDEVICE = 3,       /* a HIP runtime error */
  IPMPDE_ENOTCONVERGED = 4, /* IPM iteration limit reached; results are queryable */
  IPMPDE_EKRYLOV = 5,       /* a Krylov solve hit its iteration limit (recorded in stats) */
  IPMPDE_EBREAKDOWN = 6     /* NaN/Inf in the iterates or a collapsed step length */
};

enum { IPMPDE_POISSON = 0, IPMPDE_CONVDIFF = 1, IPMPDE_HEAT = 2 /* ipmpde_heat_create only */,
       IPMPDE_POISSON_Q1 = 3 /* Poisson (2D or 3D) with Q1 finite elements, see ipmpde_problem_create */ };
enum { IPMPDE_MINRES = 0, IPMPDE_FGMRES = 1 };
enum { IPMPDE_PD = 0, IPMPDE_PT = 1, IPMPDE_PPI = 2 };
enum { IPMPDE_FP64 = 0, IPMPDE_FP32 = 1 };
enum { IPMPDE_MU_PAPER = 0, IPMPDE_MU_CENTRAL = 1 };
enum { IPMPDE_MASS_UNIT = 0, IPMPDE_MASS_HD = 1 };
enum { IPMPDE_TILE_AUTO = 0, IPMPDE_TILE_SMALL = 1, IPMPDE_TILE_LARGE = 2 };

/* Fields for ipmpde_query / ipmpde_set_field (each n doubles). */
enum {
  IPMPDE_FIELD_U = 0, IPMPDE_FIELD_Y = 1, IPMPDE_FIELD_P = 2, IPMPDE_FIELD_W = 3, IPMPDE_FIELD_V = 4,
  IPMPDE_FIELD_LAM_YA = 5, IPMPDE_FIELD_LAM_YB = 6, IPMPDE_FIELD_LAM_WA = 7, IPMPDE_FIELD_LAM_WB = 8,
  IPMPDE_FIELD_LAM_VA = 9, IPMPDE_FIELD_LAM_VB = 10,
  IPMPDE_FIELD_DY = 11, IPMPDE_FIELD_DW = 12, IPMPDE_FIELD_DV = 13, IPMPDE_FIELD_DP = 14,
  IPMPDE_FIELD_THETA_Y = 15, IPMPDE_FIELD_THETA_W = 16, IPMPDE_FIELD_THETA_V = 17,
  IPMPDE_FIELD_FHAT = 18
};

typedef struct { int dim; int n; } ipmpde_grid;          /* dim in {2,3}; n = N interior points per axis */
typedef struct { int kind; double eps; } ipmpde_pde;     /* kind IPMPDE_POISSON | IPMPDE_CONVDIFF (2D only), eps > 0 */

/* Solver options.  ipmpde_default_options fills the defaults named here. */
typedef struct {
  double sigma;        /* barrier reduction factor (0,1); default 0.2 (Sec. 5.1) */
  double alpha0;       /* fraction to the boundary; default 0.995 (Sec. 5) */
  double eps_p, eps_d, eps_c; /* stopping tolerances on inf-norms; default 1e-6 (Sec. 5) */
  double mu0;          /* initial barrier parameter; default 1 */
  int ipm_maxit;       /* default 200 */
  int fixed_nli;       /* > 0: take exactly this many IPM steps (parity runs); default 0 */
  int krylov;          /* IPMPDE_MINRES (default) | IPMPDE_FGMRES */
  int precond;         /* IPMPDE_PD (default) | IPMPDE_PT (requires FGMRES) |
                          IPMPDE_PPI, the partial-observation preconditioner of
                          Sec. 4.3 (requires FGMRES) */
  int restart;         /* FGMRES restart length; default 30 */
  double krylov_tol;   /* relative unpreconditioned residual |b - K x| / |b|; default 1e-10 (Sec. 5) */
  int krylov_maxit;    /* default 500 */
  int vcycles;         /* V-cycles per multigrid solve; default 1 */
  int nu_pre, nu_post; /* Jacobi sweeps; default 2, 2 (MINRES needs nu_pre == nu_post) */
  double omega;        /* Jacobi damping; 0 = default (0.8 in 2D, 6/7 in 3D) */
  int mg_precision;    /* IPMPDE_FP64 | IPMPDE_FP32 (default): precision of the V-cycles */
  int chunk;           /* Krylov iterations per device-side batch between host checks; default 8 */
  int use_graphs;      /* capture Krylov chunks in HIP graphs; default 1 */
  int mu_rule;         /* barrier target of the next step: IPMPDE_MU_PAPER (default),
                          mu^{k+1} = sigma mu^k as in Algorithm A.1, or IPMPDE_MU_CENTRAL,
                          sigma times the mean complementarity product of the iterate
                          (the duality measure; equal on the central path, and robust when
                          step lengths collapse) */
  int mass_scaling;    /* IPMPDE_MASS_UNIT (default): the problem divided by the lumped mass
                          w = h^dim of a node (mesh-independent mu and tolerances), or
                          IPMPDE_MASS_HD: the literal weighting of eq. (pb_fe_lin), objective and
                          state equation times w.  Both have the same minimizer, and the HD run
                          takes the UNIT run's steps from mu0 / w with the tolerances divided by
                          w; under HD, mu and the measures in the statistics, the bound
                          multipliers and the Theta fields (query and set_field) and the mu
                          argument of the single-step entry points are in HD units (w times
                          the unit ones).  Stationary problems only (IPMPDE_EINVAL for the heat
                          equation and in an engine). */
  int mg_tile;         /* tile size of the fused 2D Poisson multigrid level kernels:
                          IPMPDE_TILE_AUTO (default: the large tiles when a launch still has
                          at least 2048 workgroups of them), IPMPDE_TILE_SMALL (8 coarse / 16
                          fine nodes per side) or IPMPDE_TILE_LARGE (16 / 32, where the LDS
                          tile fits); no node's arithmetic depends on it */
  int lanes;           /* batches only: the instances are split into this many sub-batches
                          (balanced by node count), each solved on a stream of its own by a host
                          thread of its own, so that the latency-bound multigrid launches of one
                          lane overlap the bandwidth-bound Krylov launches of another; default 1
                          (0 is taken as 1), at most 16, more than the batch's count is clamped to
                          it.  The lanes start after the work queued on the caller's stream,
                          which waits for every lane before the call returns.  No instance's
                          arithmetic depends on it.  Lanes overlap only where their streams
                          hold hardware queues of their own: HIP shares GPU_MAX_HW_QUEUES
                          queues (4 unless set before the runtime starts) among all streams
                          of the process, and lanes on a shared queue run one after another.
                          Ignored by single-problem calls and by the engine. */
} ipmpde_options;

#define IPMPDE_MAX_HIST 256

/* Per-solve statistics.  hist_* hold one entry per IPM iteration k (the
 * measures at the start of iteration k, and for k < nli the Krylov
 * iterations and step lengths of that iteration). */
typedef struct {
  int status;                /* IPMPDE_OK, IPMPDE_ENOTCONVERGED, ... */
  int nli;                   /* IPM iterations taken */
  int krylov_its;            /* total Krylov iterations over the solve */
  int krylov_fail;           /* IPM iterations whose Krylov solve missed krylov_tol */
  double xi_p, xi_d, xi_c;   /* final inf-norm measures */
  double mu;                 /* final barrier parameter */
  double solve_ms;           /* host wall time of the last ipmpde_solve */
  int hist_len;
  int hist_krylov[IPMPDE_MAX_HIST];
  double hist_mu[IPMPDE_MAX_HIST];
  double hist_xi_p[IPMPDE_MAX_HIST], hist_xi_d[IPMPDE_MAX_HIST], hist_xi_c[IPMPDE_MAX_HIST];
  double hist_alpha_p[IPMPDE_MAX_HIST], hist_alpha_d[IPMPDE_MAX_HIST];
  double hist_krylov_relres[IPMPDE_MAX_HIST]; /* true relative residual reached */
} ipmpde_stats;

typedef struct ipmpde_problem ipmpde_problem;

/* Version string of the library. */
const char* ipmpde_version(void);

/* Thread-local description of the last error (never NULL). */
const char* ipmpde_last_error(void);

/* Fill *opts with the defaults documented above. */
int ipmpde_default_options(ipmpde_options* opts);

/* Optional device allocator (e.g. a framework's caching allocator).  Both
 * callbacks NULL restores hipMalloc/hipFree.  Affects problems created
 * afterwards. */
typedef void* (*ipmpde_alloc_fn)(size_t bytes, void* ctx);
typedef void (*ipmpde_free_fn)(void* ptr, void* ctx);
int ipmpde_set_allocator(ipmpde_alloc_fn alloc, ipmpde_free_fn free_, void* ctx);

/* Create a problem instance (Sec. 1 and Sec. 2 data).  u_a, u_b, y_d are
 * required (n values each) with u_a < 0 < u_b elementwise; y_a, y_b are
 * both NULL (no state bounds) or both given with y_a < y_b; f may be NULL
 * (zero); g may be NULL (zero), else (N+2)^dim values.  alpha > 0, beta >= 0.
 * Returns IPMPDE_EINVAL for bad shapes, N != 2^k - 1, NaN/Inf, or bounds
 * that violate the above; IPMPDE_ENOMEM if device memory runs out. */
/* pde->kind = IPMPDE_POISSON_Q1 (dim 2 or 3): the same problem discretized
 * with bilinear (2D) or trilinear (3D) finite elements as in the paper
 * (Sec. 2, eq. (pb_fe_lin); Sec. 5): stiffness L, consistent mass M, lumped
 * mass D = h^dim I, all divided by h^dim (the lumped mass of a node, which
 * leaves the minimizer unchanged):
 *   minimize 1/2 (y - y_d)^T M (y - y_d) + alpha/2 u^T M u + beta |u|_1
 *   s.t. L y - M u = f_hat,  f_hat = M f - L_IB g,
 * with, in 2D, L = (8, -1 x 8) / (3 h^2) and M = (16, 4 x 4, 1 x 4) / 36 as
 * nine-point stencils and, in 3D, L = (8/3, 0 x 6, -1/6 x 12, -1/12 x 8) / h^2
 * and M = (64, 16 x 6, 4 x 12, 1 x 8) / 216 over the node and its face, edge
 * and corner neighbours.  MINRES + P_D, FGMRES + P_D, P_T or P_Pi.  P_D and
 * P_T apply (M + Theta_y)^-1 by 20 steps of Chebyshev
 * semi-iteration with D_M + Theta_y on the spectrum [1/4, 9/4] (2D) or
 * [1/8, 27/8] (3D), alpha M~ + Theta_z by alpha D~_M + Theta_z, M_hat with
 * D_M (Sec. 4.1, 4.2), multigrid on L + M_hat.  With active state bounds the
 * FP32 multigrid loses the Schur approximation late in a solve (Theta_y
 * above ~1e8); mg_precision FP64 solves those instances.  Partial
 * observation (ipmpde_set_observation with one weight per element): the
 * tracking mass is assembled from the observed elements and the solve takes
 * FGMRES + P_Pi (Sec. 4.3) with M_l its lumped diagonal plus Theta_y and
 * M_r the diagonal Sigma of P_D; P_D and P_T are refused then.  Batched only
 * with other Q1 problems; an engine serves them in groups of their own. */
int ipmpde_problem_create(const ipmpde_grid* grid, const ipmpde_pde* pde, double alpha, double beta,
                          const double* u_a, const double* u_b, const double* y_a, const double* y_b,
                          const double* y_d, const double* f, const double* g, ipmpde_problem** out);

/* Heat equation y_t - Lap y = u + f on (0,1)^2 x (0, T], T = nt tau, all
 * time steps at once (Sec. 4.4, eq. (TimeDeptSystem)): backward Euler with
 * step tau gives the block lower bidiagonal state matrix (M + tau L on the
 * diagonal, -M below it).  In the unit-mass form used throughout (M = I, the
 * constraint divided by tau and the objective's rectangle-rule weight tau
 * divided out, which leaves the minimizer unchanged) the problem is the one
 * above with n = N^2 nt space-time unknowns per field and
 *   A = blocks I/tau + A_h on the diagonal, -I/tau below it,
 * A_h the 2D 5-point Laplacian, f_hat = f - A_IB g in every step plus
 * y0/tau in the first.
 * Layout: nt consecutive blocks of N^2 values, block k-1 the time t_k = k tau
 * (k = 1..nt), each block in the 2D layout.  u_a, u_b, y_d (required), y_a,
 * y_b, f (optional) take N^2 nt values; g (optional) (N+2)^2 values, the
 * same at every time step; y0 (optional, zero if NULL) the initial state,
 * N^2 values.  grid->dim must be 2, 1 <= nt <= 65535, tau > 0, N^2 nt <= 1e8;
 * otherwise as ipmpde_problem_create.  The Schur block's solves with
 * L + M_hat (and the transpose) are block forward (backward) substitutions
 * over the time steps with one multigrid solve per step.  P_D and P_T only
 * (P_Pi: IPMPDE_EINVAL at solve).  Heat problems may be batched with other
 * heat problems only (ipmpde_batch_create: IPMPDE_EINVAL for a mix); a batch
 * of more than one needs every time step's hierarchy in the single-workgroup
 * kernel (N <= 63 with FP32, N <= 31 with FP64 V-cycles) and vcycles = 1,
 * else IPMPDE_EINVAL at solve.  Not admitted to an engine (IPMPDE_EINVAL). */
int ipmpde_heat_create(const ipmpde_grid* grid, int nt, double tau, double alpha, double beta,
                       const double* u_a, const double* u_b, const double* y_a, const double* y_b,
                       const double* y_d, const double* f, const double* g, const double* y0,
                       ipmpde_problem** out);

void ipmpde_problem_destroy(ipmpde_problem* prob);

/* Partial observation (Sec. 4.3): the tracking term becomes
 * 1/2 (y - y_d)^T O (y - y_d) with O = diag(weights) (n values, finite and
 * >= 0; 1 = observed), replacing the identity in the (1,1) block of the
 * Newton system.  weights NULL restores full observation.  When some weight
 * is 0 and the problem has no state bounds the (1,1) block is singular and
 * only IPMPDE_PPI (with FGMRES) may be used (other preconditioners give
 * IPMPDE_EINVAL at solve).  Adds n doubles of device memory.
 * Q1 problems take one weight per element instead, count = (N+1)^dim,
 * element (e1, e2[, e3]) spanning [e1 h, (e1+1) h] x ... (x1 fastest): the
 * tracking mass is assembled from the elements with their weights (1 =
 * observed), and only IPMPDE_PPI may be used while weights are set. */
int ipmpde_set_observation(ipmpde_problem* prob, const double* weights, size_t count);

/* Bytes of device memory a problem of this shape holds while it is solved
 * with these options (opts NULL = defaults): data, iterates and barrier
 * diagonals (allocated at create) plus the Newton/Krylov/multigrid
 * workspace (allocated at the first solve, or on admission to an engine).
 * 0 for an invalid grid. */
size_t ipmpde_footprint_bytes(const ipmpde_grid* grid, const ipmpde_pde* pde, int has_state_bounds,
                              const ipmpde_options* opts);

/* Run the interior point method (Algorithm A.1) from the standard starting
 * point (box midpoints, centred multipliers, mu = mu0).  opts NULL means
 * defaults.  Returns IPMPDE_OK on convergence, else an error code; the
 * iterates stay queryable either way. */
int ipmpde_solve(ipmpde_problem* prob, const ipmpde_options* opts, ipmpde_stream stream);

/* Copy a field (n doubles) to host memory; count must equal n. */
int ipmpde_query(const ipmpde_problem* prob, int field, double* host_out, size_t count);

/* Overwrite an iterate field (Y, P, W, V, LAM_*) from host memory, e.g. to
 * continue from a given IPM state; count must equal n. */
int ipmpde_set_field(ipmpde_problem* prob, int field, const double* host_in, size_t count);

/* Reset the iterates to the standard starting point with barrier mu0. */
int ipmpde_reset(ipmpde_problem* prob, const ipmpde_options* opts, ipmpde_stream stream);

/* One IPM iteration from the current iterates with barrier parameter
 * mu_new (Algorithm A.1 loop body): Newton solve, multiplier steps
 * (eqs. (zupdate1)-(zupdate4)), step lengths and update.  The Newton
 * direction stays queryable (FIELD_DY..DP).  alpha_p/alpha_d/krylov_its/
 * relres may be NULL. */
int ipmpde_ipm_step(ipmpde_problem* prob, const ipmpde_options* opts, double mu_new, ipmpde_stream stream,
                    double* alpha_p, double* alpha_d, int* krylov_its, double* relres);

/* Solve only the Newton system eq. (NewtonSystem) at the current iterates
 * and barrier mu_new; the direction is queryable as FIELD_DY..DP. */
int ipmpde_newton_direction(ipmpde_problem* prob, const ipmpde_options* opts, double mu_new,
                            ipmpde_stream stream, int* krylov_its, double* relres);

/* Feasibility and complementarity measures of the current iterates
 * (inf-norms of eq. (prdu) and of the products of eq. (gap)). */
int ipmpde_measures(ipmpde_problem* prob, ipmpde_stream stream, double* xi_p, double* xi_d, double* xi_c);

/* ipmpde_measures without any device allocation, for callers that cannot
 * allocate (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same kernel and results (bit for bit) as
 * ipmpde_measures; its scratch (launch descriptor, reduction partials and
 * tickets, results) is a 4 MiB device array of the library that each GPU
 * holds until the process ends.  The iterates must already be set (by
 * ipmpde_reset or ipmpde_solve, which allocate), else IPMPDE_EINVAL; at most
 * 44,648,448 nodes (N^dim, times nt for the heat equation), else
 * IPMPDE_EINVAL.  Runs on the current device, which must be the problem's.
 * Every call on a GPU shares that GPU's scratch: calls that overlap on one
 * GPU (from several threads or streams) race. */
int ipmpde_measures_noalloc(ipmpde_problem* prob, ipmpde_stream stream, double* xi_p, double* xi_d, double* xi_c);

int ipmpde_get_stats(const ipmpde_problem* prob, ipmpde_stats* out);

/* ---- low-level operators on caller-owned device arrays (FP64) ---- */

/* y = A x (transpose = 0) or y = A^T x (transpose = 1), n values each. */
int ipmpde_apply_operator(const ipmpde_problem* prob, int transpose, const double* x_dev, double* y_dev,
                          ipmpde_stream stream);

/* y = K x for the 4n saddle matrix of eq. (NewtonSystem) at the current
 * barrier diagonals (set by the last Newton setup); blocks [y; w; v; p]. */
int ipmpde_apply_saddle(ipmpde_problem* prob, const double* x_dev, double* y_dev, ipmpde_stream stream);

/* y = P^-1 x for the preconditioner selected by opts (P_D or P_T) at the
 * current barrier diagonals; 4n values each. */
int ipmpde_apply_precond(ipmpde_problem* prob, const ipmpde_options* opts, const double* x_dev, double* y_dev,
                         ipmpde_stream stream);

/* Prepare barrier diagonals, preconditioner data and the Newton right-hand
 * side at barrier mu_new (needed before apply_saddle/apply_precond). */
int ipmpde_newton_setup(ipmpde_problem* prob, const ipmpde_options* opts, double mu_new, ipmpde_stream stream);

/* Copy the current Newton right-hand side (4n doubles) to host memory. */
int ipmpde_query_rhs(const ipmpde_problem* prob, double* host_out, size_t count);

/* Time one hot-path kernel over `reps` back-to-back launches on `stream`
 * with HIP events; *avg_ms receives the mean duration per launch and
 * *bytes the algorithmic bytes one launch moves.  Requires a Newton setup
 * (ipmpde_newton_setup or a solve) in the same multigrid precision.
 * kernel ids: 0 saddle matvec, 2 Lanczos vector + exact (1,1)-block inverse,
 * 3 one 2D V-cycle, 4 finest-level descent kernel (2D), 5 finest-level
 * ascent kernel (2D), 6 MINRES update + saddle matvec + dot products,
 * 7 the single-workgroup coarse-grid kernel. */
int ipmpde_time_kernel(ipmpde_problem* prob, const ipmpde_options* opts, int kernel, int reps,
                       ipmpde_stream stream, double* avg_ms, double* bytes);

/* ---- batches: many instances advanced by the same kernel launches ---- */

/* A batch of `count` existing problems of the same dimension (sizes,
 * operators and parameters may differ).  The batch references the
 * problems; they must outlive it and must not be used concurrently with
 * it.  Every kernel launch of a batched solve serves all instances (one
 * grid z-slice per instance), so small and medium problems share the GPU
 * instead of paying the launch latency one by one. */
typedef struct ipmpde_batch ipmpde_batch;
int ipmpde_batch_create(ipmpde_problem* const* probs, int count, ipmpde_batch** out);
void ipmpde_batch_destroy(ipmpde_batch* batch);

/* Run Algorithm A.1 on every problem of the batch in lockstep; each
 * instance stops on its own test (then its blocks exit at once).  opts:
 * NULL (defaults), one options struct (per_problem = 0), or an array of
 * `count` structs (per_problem = 1) whose IPM fields (sigma, alpha0,
 * tolerances, mu0, iteration limits) may differ while the Krylov and
 * multigrid fields must agree (else IPMPDE_EINVAL).  Returns IPMPDE_OK
 * once every instance has finished; each problem's outcome is in its
 * stats (ipmpde_get_stats) and its iterates are queryable. */
int ipmpde_batch_solve(ipmpde_batch* batch, const ipmpde_options* opts, int per_problem, ipmpde_stream stream);

/* Autotuner of the multigrid schedule (the batching form's tile and
 * smoother schedules): times whole batched solves of this batch for each
 * candidate (V-cycles and Jacobi sweeps per solve in {1 x 1+1, 1 x 2+2,
 * 1 x 3+3, 2 x 1+1, 2 x 2+2}, for 2D Poisson batches both tile sizes of the
 * level kernels, with IPMPDE_TUNE_PRECISION in flags also the other V-cycle
 * precision) and returns in *best the options `base` (NULL = defaults) with
 * the fastest candidate's vcycles, nu_pre, nu_post, mg_precision, mg_tile and lanes
 * among those that solve every instance (IPMPDE_ENOTCONVERGED if none does);
 * each candidate is also timed with the instances split into 2, 4 and 8 lanes
 * (as many as the batch has instances), and *best carries the fastest lanes.
 * Each candidate costs two batched solves, so the problems' iterates hold the
 * last candidate's result afterwards.  cache_path (may be NULL) names a JSON
 * file of earlier results keyed by the GPU architecture and the batch's shape
 * (dimension, PDE kinds, largest N and nt, count, Krylov method,
 * preconditioner, state bounds, restart, precision unless tuned, and the
 * process's hardware queue count GPU_MAX_HW_QUEUES); a hit
 * returns the stored pick without solving (*from_cache = 1), a miss tunes and
 * adds the result to the file.  best_ms (may be NULL) receives the winner's
 * solve time in milliseconds; from_cache may be NULL. */
enum { IPMPDE_TUNE_PRECISION = 1 };
int ipmpde_batch_autotune(ipmpde_batch* batch, const ipmpde_options* base, int flags, const char* cache_path,
                          ipmpde_stream stream, ipmpde_options* best, double* best_ms, int* from_cache);

/* ipmpde_time_kernel for a whole batch: one launch serves every instance;
 * *bytes sums the instances' algorithmic bytes.  Requires a Newton setup by
 * this batch in one lane (a batch solve with lanes = 1) in the same
 * multigrid precision (IPMPDE_EINVAL otherwise); kernel 0 (the saddle matvec
 * on explicit vectors) is for single problems only. */
int ipmpde_batch_time_kernel(ipmpde_batch* batch, const ipmpde_options* opts, int kernel, int reps,
                             ipmpde_stream stream, double* avg_ms, double* bytes);

/* ---- serving engine: continuous batching of solves ----------------------
 *
 * A request is a problem (created as above) plus options.  Requests queue in
 * arrival order and are admitted while fewer than max_slots run and the sum
 * of the admitted requests' ipmpde_footprint_bytes stays within
 * hbm_budget_bytes; admission allocates the problem's Newton/Krylov/multigrid
 * workspace (from the registered allocator) and retirement frees it, while
 * the problem's data and iterates stay on the device.  Each
 * ipmpde_engine_step advances every admitted request by one iteration of
 * Algorithm A.1 (Appendix); requests with equal Krylov and multigrid options
 * (and dimension) share the same kernel launches, each at its own IPM
 * iteration, and requests admitted at a step join at that step.  A
 * request's arithmetic is that of its solo ipmpde_solve, so its result does
 * not depend on the other requests in flight.  Once a request is done its
 * problem can be queried and reused (its stats hold the outcome).  While a
 * problem is queued or running, every other entry point on it fails with
 * IPMPDE_EINVAL; destroying it then is undefined.  An engine is not
 * thread-safe.  ipmpde_engine_step runs the groups of different solver
 * options concurrently, each on a stream of the engine's own (default
 * priority) driven by a host thread of its own; they start after the work
 * queued on the stream passed, that stream waits for all of them, and every
 * group's stream has been synchronised when the call returns. */
typedef struct ipmpde_engine ipmpde_engine;

enum { IPMPDE_REQ_QUEUED = 0, IPMPDE_REQ_RUNNING = 1, IPMPDE_REQ_DONE = 2 };

typedef struct {
  int state;              /* IPMPDE_REQ_* */
  int status;             /* the solve's result code once done, else -1 */
  int nli;                /* IPM iterations so far */
  int krylov_its;         /* Krylov iterations so far */
  double queue_ms;        /* submission to admission (to now while queued) */
  double latency_ms;      /* submission to completion (to now while not done) */
  size_t footprint_bytes; /* HBM bytes accounted for the request */
} ipmpde_request_info;

typedef struct {
  int running, queued, groups;
  size_t bytes_in_use, peak_bytes, budget_bytes;
  long steps;
} ipmpde_engine_info;

/* hbm_budget_bytes > 0, 1 <= max_slots <= 4096; EINVAL otherwise. */
int ipmpde_engine_create(size_t hbm_budget_bytes, int max_slots, ipmpde_engine** out);
/* Frees the engine; requests still queued or running are dropped (their
 * workspace freed, their problems usable again). */
void ipmpde_engine_destroy(ipmpde_engine* engine);
/* Queues a request; *ticket identifies it.  opts NULL = defaults.  ENOMEM
 * when the request alone exceeds the budget; EINVAL for bad options or a
 * problem already in an engine. */
int ipmpde_engine_submit(ipmpde_engine* engine, ipmpde_problem* problem, const ipmpde_options* opts,
                         uint64_t* ticket);
/* Admits what fits, then runs one IPM iteration of every admitted request
 * and retires the finished ones.  running/queued (may be NULL) receive the
 * counts after the step.  A request's own failure (breakdown, iteration
 * limit) is its status, not the step's; the step fails only on EDEVICE or
 * ENOMEM for engine structures. */
int ipmpde_engine_step(ipmpde_engine* engine, ipmpde_stream stream, int* running, int* queued);
/* State of a request; EINVAL for an unknown ticket. */
int ipmpde_engine_poll(const ipmpde_engine* engine, uint64_t ticket, ipmpde_request_info* info);
/* Forgets a finished request (its ticket becomes unknown). */
int ipmpde_engine_release(ipmpde_engine* engine, uint64_t ticket);
int ipmpde_engine_get_info(const ipmpde_engine* engine, ipmpde_engine_info* info);

#ifdef __cplusplus
}
#endif
#endif /* IPMPDE_H */
