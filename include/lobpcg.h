/*
 * liblobpcg: mixed-precision LOBPCG for the k smallest eigenpairs of a real
 * symmetric positive definite matrix on one AMD Instinct MI355X (gfx950).
 *
 * Method: Kressner, Ma, Shao, "A mixed precision LOBPCG algorithm" (2023),
 * Algorithm 3, working-precision loop (lines 2-17).  Working precision is
 * IEEE double; the preconditioner T = (L L^T)^{-1} of section 5.1 uses a
 * Cholesky factor L held in single (FP32) or double (FP64) precision and is
 * applied by two triangular solves in the factor's precision (section 3.1);
 * the block W is orthonormalised with Algorithm 2 (section 3.2).
 *
 * Conventions shared by every entry point
 *  - Dense blocks are row-major (C order): element (i, j) of an n x c block
 *    with leading dimension ld is at p[i*ld + j].
 *  - "device" pointers are HIP device memory on the current device; "host"
 *    pointers are ordinary host memory.  The caller owns every buffer it
 *    passes; the library owns (and frees in lobpcg_destroy) what it allocates.
 *  - All GPU work is enqueued on the stream bound at setup (NULL = default
 *    stream).  Functions that return results to the host synchronise it.
 *  - No function throws or aborts across the ABI: each returns a status.
 *    lobpcg_last_error() gives a message for the last failure on the thread.
 *  - A context must not be used from two host threads at once.
 */
#ifndef LOBPCG_H
#define LOBPCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lobpcg_ctx_s* lobpcg_ctx;

typedef enum {
  LOBPCG_OK = 0,
  LOBPCG_NOT_CONVERGED = 1,        /* maxit reached; best Ritz pairs returned */
  LOBPCG_ERR_INVALID_ARG = 2,      /* argument check failed, nothing enqueued */
  LOBPCG_ERR_FACTOR_BREAKDOWN = 3, /* non-positive pivot in the Cholesky factor */
  LOBPCG_ERR_ORTHO_BREAKDOWN = 4,  /* Algorithm 2 failed and its FP64 retry too */
  LOBPCG_ERR_NONFINITE = 5,        /* NaN/Inf in inputs or residual norms */
  LOBPCG_ERR_ALLOC = 6,            /* device or host allocation failed */
  LOBPCG_ERR_HIP = 7,              /* a HIP runtime call failed */
  LOBPCG_ERR_STATE = 8             /* call out of order (e.g. backward before solve) */
} lobpcg_status;

typedef enum { LOBPCG_FP64 = 0, LOBPCG_FP32 = 1 } lobpcg_precision;

typedef enum {
  LOBPCG_STOP_PAPER = 0,  /* eq. (stop): ||r_j|| <= tol (||A||_2 + |theta_j|) ||x_j|| */
  LOBPCG_STOP_NORMA = 1   /* ||r_j|| <= tol ||A||_2 ||x_j|| */
} lobpcg_stop_rule;

/* The matrix A (section 1: Hermitian positive definite; real here).
 * CSR: full symmetric pattern (both triangles), column indices sorted and
 *      unique within each row, int32 indices, FP64 values.
 * Dense: n x n FP64, row-major with leading dimension ld (A symmetric, so
 *      row- and column-major coincide).
 * grid: optional geometry of a structured grid, node p = (i0*g1 + i1)*g2 + i2
 *      with 0 <= i_d < grid[d]; used by nested dissection; zeros = none.
 * All pointers are HOST pointers; setup copies what it needs. */
typedef struct {
  int32_t format;            /* 0 = CSR, 1 = dense */
  int32_t grid[3];
  int64_t n;
  int64_t nnz;               /* CSR only */
  const int32_t* rowptr;     /* CSR, n+1 */
  const int32_t* colind;     /* CSR, nnz */
  const double* val;         /* CSR, nnz */
  const double* dense;       /* dense, n*ld */
  int64_t ld;                /* dense leading dimension (>= n) */
} lobpcg_matrix;

/* LOBPCG_FLAG_GRAPH: run each steady-state iteration (Algorithm 3 lines 9-16) as one
 * replay of a HIP graph captured on a private stream of the context (two graphs, one per
 * buffer parity, captured on first use and kept until lobpcg_destroy).  Results are bitwise
 * identical to the eager launches; the per-step GPU timings of lobpcg_info are then zero. */
#define LOBPCG_FLAG_GRAPH 1
/* LOBPCG_FLAG_AUTOTUNE: at setup, time the candidate launch shapes on this context's own
 * buffers and keep the fastest: the split target of the triangular-solve plan (levels
 * with fewer output tiles split their reduction ranges until they have about 256, 1024,
 * 2048 or 4096 tile items) and the rows per reduction chunk of the
 * instance-segmented Gram and norm kernels (512 to 8192).  If the environment variable
 * LOBPCG_TUNE_CACHE names a file, results are appended to it keyed by device architecture
 * and problem structure, and later setups with the same key read them instead of timing.
 * The choice changes the order of floating-point reductions, so results may differ in the
 * last bits from an untuned context. */
#define LOBPCG_FLAG_AUTOTUNE 2
/* LOBPCG_FLAG_FORCE_FP64_REDO: treat every FP32-step-1 Algorithm 2 of the iteration loop as if its
 * step-3 Cholesky had broken down, so that each iteration takes the recovery path (at the next
 * synchronisation the iteration is redone from its saved inputs with step 1 in FP64).  For testing
 * that path: the results equal those of qr_lower = 0 (step 1 in FP64 throughout), and
 * lobpcg_info.fallbacks counts the redone iterations; the start block's Algorithm 2 (and that of
 * lobpcg_pinvit) then runs with step 1 in FP64 directly.  No effect when qr_lower = 0. */
#define LOBPCG_FLAG_FORCE_FP64_REDO 4

/* Device memory of a context from the caller (section 8 of the boundary: the caller's framework owns
 * every device byte).  alloc(bytes, user) returns device memory on the current device, aligned to at
 * least 256 bytes, or NULL on failure (setup then returns ALLOC); free(ptr, user) takes it back.
 * Both are called only from the host thread inside lobpcg_setup, lobpcg_solve, lobpcg_backward and
 * lobpcg_destroy; the library synchronises its streams before the frees in lobpcg_destroy, so the
 * memory is idle when it is returned.  The library may use a block on streams other than the one bound
 * at setup (its factorization side stream, its graph stream); an allocator that hands a freed block to
 * other work must not do so before free() is called. */
typedef struct {
  void* (*alloc)(size_t bytes, void* user);
  void (*free)(void* ptr, void* user);
  void* user;
} lobpcg_allocator;

/* Optional tuning of setup (pass NULL for defaults). */
typedef struct {
  int32_t leaf_size;         /* nested-dissection leaf volume; 0 (default) = 256 for a 3D grid hint, 64 otherwise */
  int32_t stop_rule;         /* lobpcg_stop_rule (default LOBPCG_STOP_PAPER) */
  int32_t qr_lower;          /* 1 = Algorithm 2 step 1 in FP32 (default), 0 = in FP64 */
  int32_t flags;             /* bit field of LOBPCG_FLAG_* (default 0) */
  double norm_a;             /* > 0: use this ||A||_2 instead of the section 5.1 estimate */
  double eig_tol;            /* > 0: also require ||r_j||^2 <= eig_tol |theta_j| (theta_m - theta_j) */
  /* Launch plan of the triangular solves (section 5.1's two solves): 0 = automatic (the whole
   * supernodal tree in one workgroup when its panels are small, otherwise one launch sequence per
   * level), -1 = one launch sequence per level always, L > 0 = the bottom L levels as subtrees of
   * one workgroup each.  Results agree to rounding; the choice only moves work between kernels. */
  int32_t subtree_levels;
  /* Factorization: fronts with at least this many 64-row tiles below their diagonal block apply
   * the Schur complement on 128 x 128 blocks (0 = default, 8).  Same arithmetic per entry. */
  int32_t schur_wide_tiles;
  /* > 0: Algorithm 3 line 1 - before the working-precision loop, a LOBPCG run in single precision
   * (FP32 blocks, single(A), FP32 products, Gram matrices, updates, residual, preconditioner output
   * and QR; the small Rayleigh-Ritz and Cholesky matrices in FP64) from single(X0) until the test of
   * eq. (stop) holds with this tolerance (section 5.1 uses 5e-6), whose X then starts the loop with
   * P = [].  0 = off (default).  Also for batched contexts, per problem. */
  double stage1_tol;
  /* NULL: device memory from hipMalloc/hipFree.  Otherwise every device allocation of the context goes
   * through it (the struct is copied at setup; user must stay valid until lobpcg_destroy). */
  const lobpcg_allocator* allocator;
} lobpcg_options;

typedef struct {
  int32_t iters;             /* outer iterations of Algorithm 3 */
  int32_t n_conv;            /* n_c at exit */
  int32_t fallbacks;         /* Algorithm 2 retries in FP64: an FP32 step 1 whose step-3 Cholesky broke
                                down is redone with step 1 in FP64 (in the loop: the whole iteration's
                                lines 11-16, at the next synchronisation) */
  int32_t nlevels;           /* levels of the supernodal elimination tree */
  double norm_a;             /* ||A||_2 used by the convergence test */
  double t_symbolic;         /* s, host ordering + symbolic analysis (setup) */
  double t_factor;           /* s, numeric factorization on the GPU */
  double t_solve;            /* s, lobpcg_solve wall time */
  double nnz_factor;         /* stored entries of the supernodal factor */
  double factor_flops;       /* flops of the numeric factorization */
  double* resid;             /* host array of k final normalised residuals, nullable */
  /* GPU time measured with HIP events on the context's stream during this solve
   * (lobpcg_solve only; zero for batched solves and backward): */
  double t_precond_gpu;      /* s, sum over the preconditioner applications (lines 9-10) */
  double t_spmm_gpu;         /* s, sum over the products A W (line 13) */
  int32_t n_precond;         /* number of preconditioner applications timed */
  int32_t n_spmm;            /* number of products A W timed */
  /* First stage (lobpcg_options.stage1_tol > 0; zero otherwise).  iters above counts the
   * working-precision loop only. */
  int32_t stage1_iters;      /* outer iterations of the single-precision LOBPCG */
  int32_t stage1_exit;       /* 1 its test held, 2 iteration cap, 3 ended early (its FP32 QR broke
                                down or a residual was not finite: the previous X was kept) */
  double t_stage1;           /* s, wall time of the first stage (included in t_solve) */
} lobpcg_info;

/* Set up a solver for the k smallest eigenpairs with block size m (Algorithm 3
 * REQUIRE: k <= m), tolerance tol for the test selected in opts.
 * Performs ordering (a fill-reducing symmetric permutation Pi, section 5.1),
 * symbolic analysis on the host, uploads and permutes A on the GPU once
 * (section 5.1: Pi is applied to A, not to R in every iteration), computes the
 * factor Pi^T A Pi = L L^T in factor_precision on the GPU, and estimates
 * ||A||_2 by ||A Omega||_F / ||Omega||_F with a seeded Gaussian Omega (n x m).
 * Errors: INVALID_ARG (k < 1, k > m, 3m > n, tol <= 0, bad pattern, non-finite
 * values), FACTOR_BREAKDOWN, ALLOC, HIP.  On error *out is NULL. */
lobpcg_status lobpcg_setup(const lobpcg_matrix* A, int32_t k, int32_t m, double tol,
                           lobpcg_precision factor_precision, void* hip_stream,
                           const lobpcg_options* opts, lobpcg_ctx* out);

/* Replace A's values by vals (CSR order of the setup pattern, device or host
 * per vals_on_device) plus diag(shift) if shift != NULL (device, n, original
 * order), then refactor.  Used for potentials A = A0 + diag(V). */
lobpcg_status lobpcg_update_values(lobpcg_ctx ctx, const double* vals, int32_t vals_on_device,
                                   const double* shift);

/* Numeric refactorization of the current values (setup already does one). */
lobpcg_status lobpcg_factor(lobpcg_ctx ctx);

/* Run Algorithm 3 lines 2-17 from X0 (device, n x m row-major, original
 * ordering; NULL = seeded N(0,1) block).  Writes evals (device, k, ascending)
 * and evecs (device, n x k row-major, original ordering, unit 2-norm).
 * Returns OK, NOT_CONVERGED (outputs still written), NONFINITE,
 * ORTHO_BREAKDOWN or HIP.  Synchronises the stream. */
lobpcg_status lobpcg_solve(lobpcg_ctx ctx, const double* X0, int32_t maxit,
                           double* evals, double* evecs, lobpcg_info* info);

/* Algorithm 1 (section 3.1): mixed-precision block PINVIT on the context's
 * matrix, factor and preconditioner.  Per iteration: X = Q of X~ (the QR is
 * Algorithm 2), Theta = X^T A X, R = A X - X Theta, return once the k leading
 * columns pass the test of lobpcg_solve (eq. (stop)), W = working(f_T(lower(R))),
 * X~ = X - W.  Theta is diagonalised every iteration (X <- X C, A X <- A X C
 * with Theta = C D C^T; the span of X and hence the iteration are unchanged)
 * so that the test and the outputs are per Ritz pair.  X0, maxit, evals, evecs
 * and info as lobpcg_solve; theta_hist (host, nullable) receives the k
 * smallest Ritz values of every iteration, k per row, maxit rows (rows after
 * the last iteration are left untouched).  Single-problem contexts only
 * (INVALID_ARG otherwise).  Returns OK, NOT_CONVERGED (outputs still
 * written), NONFINITE, ORTHO_BREAKDOWN or HIP.  Synchronises the stream;
 * afterwards lobpcg_backward needs a new lobpcg_solve. */
lobpcg_status lobpcg_pinvit(lobpcg_ctx ctx, const double* X0, int32_t maxit, double* evals,
                            double* evecs, lobpcg_info* info, double* theta_hist);

/* Batched setup: count independent problems A[0..count-1] (CSR, each with its
 * own n_b and grid hint) sharing k, m, tol and the factor precision; each is
 * solved by Algorithm 3 exactly as lobpcg_solve would (batching is an addition
 * to the method, not part of it).  They are stored as one
 * block-diagonal matrix: one ordering (each problem's rows stay contiguous),
 * one factorization and one product with A per iteration over all of them;
 * the dense block steps run per problem.  ||A_b||_2 is estimated per problem.
 * Dense matrices are not batched.  Errors as lobpcg_setup (INVALID_ARG also
 * for count < 1 or more than 2^31 nonzeros in total). */
lobpcg_status lobpcg_setup_batched(const lobpcg_matrix* A, int32_t count, int32_t k, int32_t m,
                                   double tol, lobpcg_precision factor_precision, void* hip_stream,
                                   const lobpcg_options* opts, lobpcg_ctx* out);

/* Algorithm 3 lines 2-17 for every problem of a batched context.  X0 (host
 * array of count device pointers, each n_b x m; NULL array or NULL entry =
 * seeded N(0,1) block), evals[b] (device, k), evecs[b] (device, n_b x k), and
 * infos (host array of count, nullable).  Each problem stops at its own
 * convergence (eq. (stop)) and is then frozen; the iteration ends when none is
 * active.  Returns OK when all converged, otherwise the first non-OK status
 * by problem index (outputs of converged and NOT_CONVERGED problems are
 * written).  Synchronises the stream. */
lobpcg_status lobpcg_solve_batched(lobpcg_ctx ctx, const double* const* X0, int32_t maxit,
                                   double* const* evals, double* const* evecs, lobpcg_info* infos);

/* Complex Hermitian positive definite A (section 1; the paper's complex dense and 2D-Laplace tests of
 * sections 5.4-5.5).  A->format 2: CSR as for format 0 but val holds 2 nnz doubles (real and imaginary
 * part of each entry, interleaved), full Hermitian pattern; format 3: dense n x n complex, row-major,
 * interleaved (2 ld doubles per row).  Host pointers; a grid hint (g0, g1, 1) is used for ordering.
 * The context holds the real symmetric positive definite embedding M = [[B, -C], [C, B]] of
 * A = B + iC (order 2n): each eigenvalue of A is a double eigenvalue of M, so the loop runs with 2k
 * wanted pairs and block 2m, and the preconditioner is the Cholesky factor of M (nested dissection on
 * M's graph), held in factor_precision.  Requires 1 <= k <= m <= 32 and 6m <= 2n; dense n <= 8192.  Errors as
 * lobpcg_setup (INVALID_ARG also for a matrix that is not Hermitian). */
lobpcg_status lobpcg_setup_hermitian(const lobpcg_matrix* A, int32_t k, int32_t m, double tol,
                                     lobpcg_precision factor_precision, void* hip_stream,
                                     const lobpcg_options* opts, lobpcg_ctx* out);

/* Algorithm 3 for a Hermitian context: X0 (device, n x m complex, row-major, interleaved re/im; NULL =
 * seeded complex Gaussian block), evals (device, k, ascending), evecs (device, n x k complex, row-major,
 * interleaved; unit 2-norm, each determined up to a complex phase).  Eigenvector j is read from the first
 * real Ritz vector of pair j of the embedding, and the k vectors are then made orthonormal in complex
 * arithmetic (a Cholesky QR: X <- X L^{-H} with X^H X = L L^H; the vectors read from the pairs are
 * orthonormal up to about residual / gap already, so this changes them by that much).  For an eigenvalue
 * of A that is itself multiple the pairs must separate for the vectors to span its eigenspace.  info as
 * lobpcg_solve (iters, residuals of the k pairs before the QR, n_conv counted in pairs).  lobpcg_solve,
 * lobpcg_pinvit, lobpcg_backward and lobpcg_update_values reject Hermitian contexts. */
lobpcg_status lobpcg_solve_hermitian(lobpcg_ctx ctx, const double* X0, int32_t maxit, double* evals,
                                     double* evecs, lobpcg_info* info);

/* Number of problems held by ctx (1 for lobpcg_setup). */
int32_t lobpcg_batch_count(lobpcg_ctx ctx);

/* Gradient of a loss L(theta_1..k, x_1..k) with respect to a diagonal
 * potential added to A, given d_evals = dL/dtheta (device, k, nullable) and
 * d_evecs = dL/dX (device, n x k row-major, nullable):
 *   g = sum_i dtheta_i (x_i o x_i) - sum_i y_i o x_i,
 *   (A - theta_i I) y_i = (I - x_i x_i^T) dX_i,  y_i orthogonal to x_i,
 * solved by projected preconditioned CG in FP64 with the factor as
 * preconditioner.  Writes d_diag (device, n, original ordering).
 * Errors: STATE (no successful solve), NOT_CONVERGED (adjoint solve). */
lobpcg_status lobpcg_backward(lobpcg_ctx ctx, const double* d_evals, const double* d_evecs,
                              double* d_diag);

/* Iterations of the projected preconditioned CG in the latest lobpcg_backward on ctx (0 before
 * the first one, or for a NULL ctx). */
int32_t lobpcg_backward_iters(lobpcg_ctx ctx);

lobpcg_status lobpcg_destroy(lobpcg_ctx ctx);
const char* lobpcg_status_string(lobpcg_status s);
const char* lobpcg_last_error(void);

/* ---- Per-step entry points (each one step of the hot path, for tests and
 * measurement).  Blocks are in the permuted ordering of the context. ---- */

/* Host-only symbolic analysis (no GPU use): the fill-reducing ordering and
 * supernode partition setup would build for A.  perm_host (n, nullable)
 * receives perm[new] = old; stats (nullable, 8 doubles) receives
 * {supernodes, levels, stored factor entries (lower), factorization flops,
 *  largest front rows, largest supernode columns, update-matrix entries,
 *  panel entries}. */
lobpcg_status lobpcg_symbolic(const lobpcg_matrix* A, int32_t leaf_size, int32_t* perm_host, double* stats);

/* Host-only: entries of the exact Cholesky factor L of Pi^T A Pi (diagonal included) for the ordering
 * lobpcg_symbolic builds, counted on the elimination tree without forming L (section 5.1's factor
 * without the supernodes' explicit zeros; the dense format gives n(n+1)/2).  *nnz_exact (host) receives
 * it.  Work O(nnz(L)) on the host; no GPU use.  Errors: INVALID_ARG. */
lobpcg_status lobpcg_exact_fill(const lobpcg_matrix* A, int32_t leaf_size, double* nnz_exact);

/* Launch shapes in use: out3 = {split target of the triangular-solve plan, rows per reduction
 * chunk, 0 = defaults / 1 = tuned at setup / 2 = read from the tuning cache}. */
lobpcg_status lobpcg_get_tuning(lobpcg_ctx ctx, int32_t* out3);

/* Host copy of the permutation: perm[new] = old (n entries). */
lobpcg_status lobpcg_get_permutation(lobpcg_ctx ctx, int32_t* perm_host);

/* Y = A X for the permuted A of ctx: X, Y device n x c (ld >= c), c <= 256.
 * (Algorithm 3 line 13, A S; section 4's fl(Ax).) */
lobpcg_status lobpcg_apply_a(lobpcg_ctx ctx, const double* X, int64_t ldx, double* Y, int64_t ldy,
                             int32_t c);

/* W = working(f_T(lower(R))) with T = (L L^T)^{-1} of ctx, in the factor's
 * precision (Algorithm 3 lines 9-10): R, W device n x m, ld = m. */
lobpcg_status lobpcg_apply_precond(lobpcg_ctx ctx, const double* R, double* W);

/* Algorithm 2 in place on W (device, n x c row-major, c <= ldw < 2^22, c <= 64):
 * W <- Q; R (device, c x c row-major, nullable) <- upper triangular factor.
 * lower_step1 = 1: step 1 in FP32, else FP64.  Returns ORTHO_BREAKDOWN if the
 * step-3 Cholesky fails. */
lobpcg_status lobpcg_mixed_qr(double* W, int64_t n, int32_t c, int64_t ldw, int32_t lower_step1,
                              double* R, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): lobpcg_mixed_qr with the same arguments, kernels and
 * results, whose scratch (plans, TSQR tree, R factors, Gram partial sums, breakdown flag) lives in
 * one fixed device array of LOBPCG_NOALLOC_SCRATCH_BYTES per GPU that the library holds until the
 * process ends; the call allocates nothing (no hipMalloc, hipFree or allocating library routine).
 * The caller passes W and R as for lobpcg_mixed_qr.  Sizes whose scratch would exceed the array
 * return INVALID_ARG before any work (n <= 262,144 fits for c <= 32, n <= 65,536 for c <= 64).
 * Every call on one GPU uses that GPU's array and leaves it holding its own intermediates: calls
 * that overlap on one GPU (two host threads, or two streams whose work overlaps) race. */
#define LOBPCG_NOALLOC_SCRATCH_BYTES (32u << 20)
lobpcg_status lobpcg_mixed_qr_noalloc(double* W, int64_t n, int32_t c, int64_t ldw, int32_t lower_step1,
                                      double* R, void* hip_stream);

/* G = X^T Y (device; X n x c1, Y n x c2, row-major; G c1 x c2 row-major),
 * deterministic two-stage reduction.  c1, c2 <= 256; ldx, ldy <= 32768 (INVALID_ARG otherwise). */
lobpcg_status lobpcg_gram(const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t n,
                          int32_t c1, int32_t c2, double* G, void* hip_stream);

/* Symmetric eigensolver for a small c x c FP64 matrix (device, row-major,
 * symmetrised as (H + H^T)/2): the nev smallest eigenpairs, evals ascending
 * (device, nev), evecs (device, c x c row-major; column j < nev =
 * eigenvector j, the other columns are not written).  1 <= nev <= c <= 192.
 * (Algorithm 3 line 14.) */
lobpcg_status lobpcg_syev_small(const double* H, int32_t c, int32_t nev, double* evals, double* evecs,
                                void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* LOBPCG_H */
