/*
 * acr.h -- C ABI of the MI355X (gfx950) Accelerated Cyclic Reduction library.
 *
 * Method: Chavez, Turkiyyah, Keyes, "A Direct Elliptic Solver Based on
 * Hierarchically Low-rank Schur Complements" (arXiv:1604.00617).  The solver
 * takes a block-tridiagonal system A u = f, A = tridiag(E_i, D_i, F_i)
 * (Section 3, Eq. "system"), runs block cyclic reduction on its even/odd
 * permutation (Eq. "sche", Eq. "fund"), holds every block that arises as a
 * HODLR matrix (H-matrix with weak admissibility) whose off-diagonal blocks
 * are truncated to a relative accuracy eps, and solves by forward reduction of
 * the right-hand side and back-substitution.
 *
 * Conventions shared by every entry point
 *  - All array arguments are DEVICE pointers on the current HIP device,
 *    unless a parameter says "host".  Sizes are element counts.
 *  - The operator is given in 5-point stencil form (D_i tridiagonal, E_i and
 *    F_i diagonal, Section 3): N = nx*ny unknowns, index i*nx + j with i the
 *    block (grid row) and j the position inside the block; each stencil array
 *    has N FP64 values.  Couplings leaving the grid (west at j=0, east at
 *    j=nx-1, south at i=0, north at i=ny-1) are ignored.
 *  - Vectors are FP64, column-major N x nrhs with leading dimension N.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *    on it; entry points that must read device results (acr_factor,
 *    acr_solve_refined, acr_solve_krylov) synchronise that stream before
 *    returning.
 *  - Every entry point returns an acr_status; on error no output is valid and
 *    acr_last_error() describes the failure (thread-local text).
 *  - The library allocates its own device memory (factor storage and
 *    workspace) with hipMalloc through an internal caching pool.
 */
#ifndef ACR_H
#define ACR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ACR_OK = 0,
  ACR_ERR_INVALID_ARG = 1,  /* bad size, pointer, option or unsupported block size */
  ACR_ERR_OOM = 2,          /* device allocation failed */
  ACR_ERR_SINGULAR = 3,     /* a zero or non-finite pivot in a dense leaf inverse */
  ACR_ERR_NOT_CONVERGED = 4,/* refinement did not reach the tolerance in maxit steps */
  ACR_ERR_DEVICE = 5,       /* a HIP runtime call failed */
  ACR_ERR_INTERNAL = 6
} acr_status;

typedef enum {
  ACR_FP64 = 0,        /* every H-arithmetic step in FP64 */
  ACR_MIXED_FP32 = 1   /* factor and solve in FP32; leaf and capacitance inverses
                          in FP64 (rounded to FP32 for storage); refinement
                          residuals in FP64 */
} acr_precision;

/* The block-tridiagonal operator (Section 3, Eq. "system") in stencil form.
 * Owned by the caller; read during acr_factor (and acr_solve_refined /
 * acr_residual), never retained. */
typedef struct {
  int32_t nx;            /* block size s (unknowns per block), >= 1 */
  int32_t ny;            /* number of blocks, >= 1 */
  const double* diag;    /* [N] main diagonal of D_i */
  const double* west;    /* [N] sub-diagonal of D_i   (couples j to j-1) */
  const double* east;    /* [N] super-diagonal of D_i (couples j to j+1) */
  const double* south;   /* [N] diagonal of E_i (couples block i to i-1) */
  const double* north;   /* [N] diagonal of F_i (couples block i to i+1) */
} acr_operator;

/* Factorisation options.
 * The block size nx must be leaf' * 2^L for the HODLR split to be exact: a
 * cluster of size s > leaf is split into two halves of size s/2 (so s must be
 * even at every split); nx <= leaf gives a single dense leaf (exact BCR).
 * Otherwise ACR_ERR_INVALID_ARG. */
typedef struct {
  int32_t leaf;          /* maximum dense leaf size, 1..128 */
  double eps;            /* truncation tolerance: keep singular values
                            s_t > eps * s_1 of each off-diagonal block, >= 0 */
  int32_t precision;     /* acr_precision */
  int32_t max_rank;      /* cap on every off-diagonal rank, 0 = none */
  double inner_eps;      /* tolerance for intermediate truncations of the
                            products inside one Schur update (0 = accumulate
                            exactly, truncate once per stored block) */
} acr_options;

/* Summary of a factorisation. */
typedef struct {
  int32_t nx, ny, leaf, depth;  /* depth = HODLR levels L (leaf' = nx / 2^L) */
  int32_t levels;               /* cyclic-reduction levels */
  int32_t precision;
  double eps;
  int64_t factor_bytes;         /* device bytes of the stored factor */
  int32_t max_rank;             /* max stored off-diagonal rank over all levels */
  int32_t level_max_rank[40];   /* per CR level (stored X, E, F blocks) */
  double factor_flops;          /* algorithmic flops of the factorisation, counted
                                   from the shapes actually processed */
  double solve_bytes;           /* stored-factor bytes one solve pass reads */
  double solve_flops_per_rhs;   /* flops of one solve pass per right-hand side */
} acr_info;

typedef struct acr_handle_s* acr_handle;   /* opaque; owned by the library */

/* Factor A (Section 3, reduction phase): level by level, invert the even
 * diagonal blocks (HODLR inverse), form P_k = X_k E_k and Q_k = X_k F_k, and
 * the odd Schur updates D'_j = D_i - E_i Q_{i-1} - F_i P_{i+1},
 * E'_j = -E_i P_{i-1}, F'_j = -F_i Q_{i+1} (i = 2j+1), every stored block cut
 * to eps; repeat until one block is left and invert it.
 * op, opt: host structs (op's arrays on the device).  *out: host, receives a
 * new handle on success.  Blocks until the factorisation has finished on
 * `stream`.  ACR_ERR_SINGULAR if a dense leaf or capacitance inverse meets a
 * zero or non-finite pivot (there is no pivoting across blocks). */
acr_status acr_factor(const acr_operator* op, const acr_options* opt, void* stream,
                      acr_handle* out);

/* X = M^{-1} B with M the stored ACR factor (Section 3: forward reduction of
 * f, Eq. "fund", then back-substitution u_k = X_k (f_k - E_k u_{k-1} - F_k
 * u_{k+1})).  B, X: N x nrhs FP64, column-major, ld = N; X may alias B.
 * In ACR_MIXED_FP32 the pass runs in FP32 (B rounded on entry).  Asynchronous
 * on `stream` (no host synchronisation), so it may be captured in a graph
 * after a first call with the same nrhs has sized the workspace. */
acr_status acr_solve(acr_handle h, const double* B, double* X, int32_t nrhs, void* stream);

/* Iterative refinement with ACR as the preconditioner (Section 4, closing
 * paragraph): x_0 = 0, r = B - A x in FP64, x += M^{-1} r, until
 * max_col ||r||_2/||B||_2 <= tol or maxit corrections.  op must be the
 * operator that was factored.  iters, relres: host outputs (may be NULL).
 * ACR_ERR_NOT_CONVERGED (X holds the last iterate) if tol is not reached. */
acr_status acr_solve_refined(acr_handle h, const acr_operator* op, const double* B, double* X,
                             int32_t nrhs, double tol, int32_t maxit, int32_t* iters,
                             double* relres, void* stream);

/* Restarted flexible GMRES, right-preconditioned by the ACR factor (ACR as
 * a preconditioner of tunable accuracy, Section 4, closing paragraph; the
 * Krylov alternative to acr_solve_refined where its contraction is slow or
 * fails): per column b of B, x_0 = 0; each restart cycle builds up to
 * `restart` (1..64) FP64 basis vectors v_j (classical Gram-Schmidt applied
 * twice), z_j = M^{-1} v_j with acr_solve's pass, and sets x += Z y with y
 * the least-squares solution of the Hessenberg system (Givens rotations on
 * the host).  Stops when the true relative residual ||b - A x||/||b|| <= tol
 * or after maxit applications of M^{-1}.  op must be the factored operator.
 * B, X: N x nrhs FP64 column-major (ld = N); X must not alias B.  iters,
 * relres: host outputs (may be NULL): the largest preconditioner count and
 * relative residual over the columns.  Workspace: (2 restart + 3) N doubles.
 * ACR_ERR_NOT_CONVERGED (X holds the last iterate) if tol is not reached.
 * Synchronises `stream` (the small Hessenberg problem lives on the host). */
acr_status acr_solve_krylov(acr_handle h, const acr_operator* op, const double* B, double* X,
                            int32_t nrhs, double tol, int32_t maxit, int32_t restart,
                            int32_t* iters, double* relres, void* stream);

/* R = B - A X in FP64 for the stencil operator (N x nrhs, ld = N). */
acr_status acr_residual(const acr_operator* op, const double* X, const double* B, double* R,
                        int32_t nrhs, void* stream);

/* Fill *out (host) with the factor summary. */
acr_status acr_get_info(acr_handle h, acr_info* out);

/* Copy out the stored blocks of one CR level for inspection (FP64, host
 * buffers, dense): which = 0 -> X_k of even block k (level < levels) or the
 * last inverse (level == levels, k = 0); 1 -> E_k; 2 -> F_k.  dense: host
 * [nx*nx] column-major.  Synchronises `stream`.  Intended for tests. */
acr_status acr_get_block(acr_handle h, int32_t level, int32_t which, int32_t k, double* dense,
                         void* stream);

/* Release every device allocation of the handle (synchronises its stream). */
acr_status acr_destroy(acr_handle h);

/* Static description of a status code. */
const char* acr_status_string(acr_status s);

/* Text of the last error raised on the calling thread ("" if none). */
const char* acr_last_error(void);

/* Kernel classes of the event profiler. */
typedef enum {
  ACR_KC_GEMM = 0,     /* batched GEMM over (matrix, cluster) problems */
  ACR_KC_INVERSE = 1,  /* dense leaf / capacitance inverses (FP64) */
  ACR_KC_QR = 2,       /* Householder R factors (recompression) */
  ACR_KC_APPLYQ = 3,   /* Q [J; 0] products (recompression) */
  ACR_KC_SVD = 4,      /* one-sided Jacobi SVD of the recompression cores */
  ACR_KC_MATVEC = 5,   /* HODLR multi-vector products of the solve */
  ACR_KC_COPY = 6,     /* stacking copies, scalings */
  ACR_KC_OTHER = 7,    /* layout, residual, reductions */
  ACR_KC_COUNT = 8
} acr_kernel_class;

/* Start timing every launch of the classes in class_mask (bit c = class c)
 * with HIP events recorded on each launch's stream; clears earlier records.
 * A mask of 0 stops recording.  For benchmarking and diagnostics. */
acr_status acr_profile_start(uint32_t class_mask);

/* Totals for one class since acr_profile_start (host outputs, any may be
 * NULL): launches, summed event time in ms, algorithmic flops and bytes of
 * those launches (counted from their shapes; for the Jacobi SVD the pair
 * inner products of the sweeps actually run).  Waits for the recorded events. */
acr_status acr_profile_read(int32_t cls, int64_t* launches, double* total_ms, double* flops,
                            double* bytes);

/* Text report of the launches recorded since acr_profile_start, one
 * tab-separated line per group:
 *   "stage  <stage> <level> <class> <launches> <ms> <flops> <bytes>"  per
 *       (stage, level, kernel class); stages are the factorisation and solve
 *       steps ("inverse", "products P,Q", "recompress D',E',F'", "solve
 *       forward", ...), level the cyclic-reduction level (-1 outside the loop);
 *   "kernel <name> <class> <launches> <ms> <flops> <bytes>"  per kernel, with
 *       the name as kernel statistics of rocprofv3 print it ("k_gqr<float>");
 *   "stagekernel <stage> <name> <launches> <ms> <flops> <bytes>"  per (stage,
 *       kernel) over all levels.
 * flops and bytes are the algorithmic counts of those launches.  Writes at
 * most len bytes including the terminating NUL into buf (host memory, owned
 * by the caller; may be NULL with len 0); *needed (may be NULL) receives the
 * full length.  Waits for the recorded events. */
acr_status acr_profile_report(char* buf, int64_t len, int64_t* needed);

/* Release the library's cached (unused) device memory. */
acr_status acr_trim_pool(void);

#ifdef __cplusplus
}
#endif
#endif
