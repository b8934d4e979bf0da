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
 *  - Device memory (factor storage and workspace) comes from an internal
 *    caching pool, which takes it from hipMalloc or, after
 *    acr_set_allocator, from the caller's allocator.  A block freed by work
 *    of one host thread on one stream is reused only by later work of the
 *    same thread on the same stream (or after a device synchronisation), so
 *    calls on different streams never share a buffer that is still in use.
 *  - Threads: each host thread has its own launch queue and descriptor
 *    arena, so different threads may call the library at the same time on
 *    different handles.  Calls that use the same handle from two threads at
 *    once are not supported (the handle is read-only after acr_factor, but
 *    acr_destroy must not overlap any other call on it).
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

/* The block-tridiagonal operator given by dense blocks (Section 3, Eq.
 * "system", general blocks), for small problems and tests: D_i, E_i, F_i of
 * block row i are nx x nx column-major FP64 device arrays at D + i*nx*nx etc.
 * (E_0 and F_(ny-1) are ignored).  Owned by the caller, read during
 * acr_factor_dense only. */
typedef struct {
  int32_t nx;            /* block size s, >= 1 */
  int32_t ny;            /* number of blocks, >= 1 */
  const double* D;       /* [ny][nx][nx] */
  const double* E;       /* [ny][nx][nx] */
  const double* F;       /* [ny][nx][nx] */
} acr_dense_operator;

/* A 3-D operator (Section 4, closing remarks: 3-D discretisations are block
 * tridiagonal with one block per plane) as a 7-point stencil on an
 * nx x ny x nz grid, unknown index (k*ny + i)*nx + j (k the plane):
 *   (A u) = diag u + west u[j-1] + east u[j+1] + south u[i-1] + north u[i+1]
 *           + down u[k-1] + up u[k+1].
 * Block k is plane k (s = nx*ny unknowns): D_k its five-point operator,
 * E_k = diag(down), F_k = diag(up); nz blocks.  Couplings that would leave
 * the grid (west at j = 0, east at j = nx-1, south at i = 0, north at
 * i = ny-1, down at k = 0, up at k = nz-1) are ignored.  Owned by the
 * caller, read during the call only. */
typedef struct {
  int32_t nx;            /* row length of a plane, >= 1 */
  int32_t ny;            /* rows per plane, >= 1 */
  int32_t nz;            /* planes (blocks), >= 1 */
  const double* diag;    /* [N] */
  const double* west;    /* [N] couples j to j-1 */
  const double* east;    /* [N] couples j to j+1 */
  const double* south;   /* [N] couples i to i-1 (inside a plane) */
  const double* north;   /* [N] couples i to i+1 (inside a plane) */
  const double* down;    /* [N] couples plane k to k-1 */
  const double* up;      /* [N] couples plane k to k+1 */
} acr_operator3d;

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
  int32_t stop_blocks;   /* early stop of the recursion (Section 3: it may end
                            once the system is small enough): levels run while
                            more than stop_blocks blocks remain (0 or 1: down
                            to one block); the remaining m blocks are inverted
                            as one dense (m*nx)^2 matrix in FP64 (m <= 16 and
                            m*nx <= 1024, else ACR_ERR_INVALID_ARG) */
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
  /* Ranks are stored padded: every block of one (set, HODLR depth) holds the
   * set's largest rank, the extra columns zero.  The figures below count the
   * blocks at their own numerical ranks instead. */
  double factor_bytes_ranked;   /* stored factor without the padding columns */
  double solve_bytes_ranked;    /* solve_bytes without the padding columns */
  double level_mean_rank[40];   /* per CR level: mean numerical rank of the
                                   stored off-diagonal blocks of X, E, F */
  int64_t factor_launches;      /* kernel launches of the factorisation */
  int32_t stop_blocks;          /* blocks of the dense remainder (1 = none) */
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

/* acr_factor for an operator of dense blocks: every block is first held as a
 * HODLR matrix with each off-diagonal block cut to eps (the block taken as
 * U = block, V = I and recompressed as in the factorisation), then the same
 * level recursion runs with general (non-diagonal) E_i and F_i from level 0.
 * The handle works with acr_solve / acr_solve_batched / acr_get_block /
 * acr_get_info (the refinement entry points take stencil operators only).
 * Costs O(nx^3) per block to compress; meant for small problems. */
acr_status acr_factor_dense(const acr_dense_operator* op, const acr_options* opt, void* stream, acr_handle* out);

/* acr_factor for a 3-D operator: the block size is the plane, s = nx*ny, and
 * each D_k enters as its exact HODLR form (a leaf holds the plane operator
 * restricted to it; an off-diagonal block is rank nx where the two clusters
 * hold whole rows of the plane (the y couplings across the split) and rank 1
 * inside a row (the x coupling)).  Needs s = leaf' * 2^L and, at every depth,
 * clusters that split on row boundaries or inside one row (s/2^d a multiple
 * of nx, or nx a multiple of s/2^(d-1)); ACR_ERR_INVALID_ARG otherwise.  The
 * off-diagonal ranks of the inverses grow with the plane's side, which makes
 * the method superlinear in 3-D; a coarse eps with acr_solve_krylov_3d uses
 * the factor as a preconditioner of tunable accuracy.  The handle works with
 * acr_solve, acr_get_block, acr_get_info and the _3d refinement calls. */
acr_status acr_factor_3d(const acr_operator3d* op, const acr_options* opt, void* stream, acr_handle* out);

/* Factor `count` independent problems at once (the even blocks of every
 * level are independent, Section 3; so are separate systems): ops[p] is the
 * p-th operator (host array of count structs, their arrays on the device;
 * block sizes and counts may differ), opt applies to all.  The problems run
 * in lockstep over the cyclic-reduction levels and each step of a level is
 * one set of grouped kernel launches for all of them.  Every kernel variant
 * is picked by the shape of its own problem, so out[p] (host array of count
 * handles, each destroyed with acr_destroy) holds the same factor, bit for
 * bit, as acr_factor(&ops[p], opt, ...).  On any error no handle is
 * returned; ACR_ERR_SINGULAR / ACR_ERR_INVALID_ARG name the problem in
 * acr_last_error().  acr_get_info of each handle reports the flops and
 * launches of the whole batch.  Blocks until done on `stream`. */
acr_status acr_factor_batched(const acr_operator* ops, const acr_options* opt, int32_t count, void* stream,
                              acr_handle* out);

/* X[p] = M_p^{-1} B[p] for count handles at once (host arrays of count device
 * pointers, FP64 N_p x nrhs[p] column-major, ld N_p): the forward and back
 * substitution steps of all problems with at most 8 right-hand sides share
 * their launches (per precision); problems with more right-hand sides are
 * solved one after the other.  Results equal acr_solve's bit for bit.  X[p]
 * may alias B[p]; X[p] must not overlap X[q] or B[q] for q != p
 * (ACR_ERR_INVALID_ARG).  Asynchronous on `stream`. */
acr_status acr_solve_batched(const acr_handle* hs, const double* const* B, double* const* X, const int32_t* nrhs,
                             int32_t count, void* stream);

/* X = M^{-1} B with M the stored ACR factor (Section 3: forward reduction of
 * f, Eq. "fund", then back-substitution u_k = X_k (f_k - E_k u_{k-1} - F_k
 * u_{k+1})).  B, X: N x nrhs FP64, column-major, ld = N; X may alias B.
 * In ACR_MIXED_FP32 the pass runs in FP32 (B rounded on entry).  Asynchronous
 * on `stream` (no host synchronisation); its workspace comes from the pool on
 * every call, so the call is not meant for stream capture.  With at most 8
 * right-hand sides each matvec step of the pass is two grouped launches
 * (projections, then rows) by default, from descriptors and a workspace the
 * handle keeps on the device after the first such solve (see
 * acr_set_solve_mode); acr_set_solve_mode can select a persistent launch for
 * part or all of the pass instead. */
acr_status acr_solve(acr_handle h, const double* B, double* X, int32_t nrhs, void* stream);

/* acr_solve without any device allocation, for callers that cannot allocate
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results (bit for bit) and kernels as
 * acr_solve; its workspace and job descriptors live in a fixed scratch array
 * of 64 MiB that the library holds on every GPU it runs on until the process
 * ends (60 MiB of workspace, 4 MiB of descriptors).  A solve that needs more
 * (it grows with N * nrhs: about 24 N nrhs bytes in FP32 factors, twice that
 * in FP64) is rejected with ACR_ERR_INVALID_ARG before any work is issued.
 * The call issues no hipMalloc, hipFree, allocating library routine or
 * profiler event.  All calls on one GPU share that GPU's scratch and the
 * scratch keeps the last call's contents: calls that overlap in time on one
 * GPU (other threads or other streams) race and are not allowed.  The
 * handle must exist (acr_factor allocates) and its factor is read only.  It
 * runs the pass as grouped launches per step (acr_set_solve_mode's mode 1),
 * whose results equal the persistent pass's bit for bit. */
acr_status acr_solve_noalloc(acr_handle h, const double* B, double* X, int32_t nrhs, void* stream);

/* Iterative refinement with ACR as the preconditioner (Section 4, closing
 * paragraph): x_0 = 0, r = B - A x in FP64, x += M^{-1} r, until
 * max_col ||r||_2/||B||_2 <= tol or maxit corrections.  op must be the
 * operator that was factored.  B, X: N x nrhs FP64 column-major (ld = N);
 * X must not overlap B (B is read by every residual): ACR_ERR_INVALID_ARG.
 * iters, relres: host outputs (may be NULL).
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
 * B, X: N x nrhs FP64 column-major (ld = N); X must not overlap B.  iters,
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

/* acr_residual, acr_solve_refined and acr_solve_krylov for a 3-D operator
 * factored with acr_factor_3d (same arguments and rules; N = nx*ny*nz). */
acr_status acr_residual_3d(const acr_operator3d* op, const double* X, const double* B, double* R,
                           int32_t nrhs, void* stream);
acr_status acr_solve_refined_3d(acr_handle h, const acr_operator3d* op, const double* B, double* X,
                                int32_t nrhs, double tol, int32_t maxit, int32_t* iters,
                                double* relres, void* stream);
acr_status acr_solve_krylov_3d(acr_handle h, const acr_operator3d* op, const double* B, double* X,
                               int32_t nrhs, double tol, int32_t maxit, int32_t restart,
                               int32_t* iters, double* relres, void* stream);

/* Fill *out (host) with the factor summary. */
acr_status acr_get_info(acr_handle h, acr_info* out);

/* Copy out the stored blocks of one CR level for inspection (FP64, host
 * buffers, dense): which = 0 -> X_k of even block k (level < levels) or the
 * last inverse (level == levels, k = 0; after an early stop at m > 1 blocks,
 * block (i, j) of the dense remainder inverse for k = i*m + j); 1 -> E_k;
 * 2 -> F_k.  dense: host
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
 *       kernel) over all levels;
 *   "path <name> <problems>"  per kernel path (variant and operand class,
 *       e.g. "qr.reg.p>128"): the number of batched problems planned on it.
 * flops and bytes are the algorithmic counts of those launches.  Writes at
 * most len bytes including the terminating NUL into buf (host memory, owned
 * by the caller; may be NULL with len 0); *needed (may be NULL) receives the
 * full length.  Waits for the recorded events. */
acr_status acr_profile_report(char* buf, int64_t len, int64_t* needed);

/* ---------------------------------------------------------------- serving
 * A server keeps the factors of registered operators resident in device
 * memory under a byte budget and solves requests A x = b (FP64 right-hand
 * sides) by iterative refinement with the factor as preconditioner (Section
 * 4, closing paragraph), to the relative residual `tol` of its config.  One
 * worker thread and one stream per server.  A request whose operator has no
 * resident factor waits until the factor fits next to the resident ones
 * (idle factors are evicted least recently used first; a factor larger than
 * the whole budget is admitted alone), then its operator is factored,
 * together with every other operator admitted at that moment (one batched
 * factorisation).  Active requests advance together one refinement step at a
 * time (residuals, norms, corrections and updates of all of them in shared
 * launches); requests that arrive meanwhile join at the next step.  A
 * request's arithmetic does not depend on the other requests, so its X is
 * the same bits alone and in any mix. */
typedef struct acr_server_s* acr_server;

typedef struct {
  int64_t memory_budget;   /* device bytes the resident factors may take (> 0) */
  double tol;              /* refinement target: max_col ||b - A x|| / ||b|| <= tol */
  int32_t maxit;           /* refinement corrections at most (>= 0) */
} acr_server_config;

typedef struct {
  int64_t requests, rhs, steps;        /* completed requests / right-hand sides, refinement steps */
  int64_t factorizations, evictions;   /* factors computed / evicted */
  int64_t resident_bytes, peak_resident_bytes;
  double seconds;                      /* first submit to last completion */
  double requests_per_s, rhs_per_s;
  double latency_p50_ms, latency_p99_ms, latency_max_ms;   /* submit to completion */
  double busy_s;                       /* worker time spent admitting and stepping */
} acr_server_info;

/* Start a server on the current device (config: host struct).  *out: host. */
acr_status acr_server_create(const acr_server_config* cfg, acr_server* out);

/* Register an operator with its factorisation options; the server keeps its
 * own device copy of the operator (op's arrays may be freed afterwards).
 * *op_id (host) identifies it in acr_server_submit.  Synchronises the
 * device.  No factorisation happens before the first request. */
acr_status acr_server_add_operator(acr_server s, const acr_operator* op, const acr_options* opt, int32_t* op_id);

/* Queue X = A^{-1} B for operator op_id: B, X device arrays N x nrhs FP64
 * (column-major, ld N), X must not overlap B; both must stay valid until
 * acr_server_wait returns for this request.  The server's stream waits for
 * the work enqueued so far on `stream` before it reads B.  *request (host)
 * receives the request id.  Returns at once. */
acr_status acr_server_submit(acr_server s, int32_t op_id, const double* B, double* X, int32_t nrhs,
                             void* stream, int64_t* request);

/* Block until the request completes; then X holds the solution (device work
 * done).  iters, relres, latency_ms (host, may be NULL): refinement
 * corrections, final relative residual, submit-to-completion time.
 * ACR_ERR_NOT_CONVERGED if tol was not reached in maxit corrections.  Each
 * request is waited for once. */
acr_status acr_server_wait(acr_server s, int64_t request, int32_t* iters, double* relres, double* latency_ms);

/* Statistics of the requests completed since the last reset (reset != 0
 * starts a new window after filling *out). */
acr_status acr_server_stats(acr_server s, int32_t reset, acr_server_info* out);

/* Finish every queued request, stop the worker and free the server. */
acr_status acr_server_destroy(acr_server s);

/* ------------------------------------------------------------- autotuner
 * Kernel-variant choices per shape key, measured on the device: the tile
 * shape of the grouped GEMM per (precision, M, N, K size class, problem-count
 * size class) -- every tile gives the same bits -- and the Householder QR
 * form (one wave, registers, LDS) per (precision, panel rows, columns), whose
 * forms differ in rounding.  Keys hold a problem's own shapes only, so with
 * any fixed table a problem's result is the same whatever it is batched
 * with.  Without a table the built-in choices apply. */
/* Start (on != 0) or stop noting the shape keys the library meets. */
acr_status acr_tune_record(int32_t on);
/* Measure every noted key that has no table entry yet (micro-benchmarks on
 * synthetic operands on `stream`; synchronises it) and add the fastest
 * choice; *added (host, may be NULL): entries added.  Tuning is off while it
 * measures; the table's use afterwards follows acr_tune_enable. */
acr_status acr_tune_run(void* stream, int32_t* added);
/* Use (on != 0) or ignore the table. */
acr_status acr_tune_enable(int32_t on);
/* Write the table as JSON {"arch": <device architecture>, "entries": {key: choice}}. */
acr_status acr_tune_save(const char* path);
/* Replace the table by the file's entries and use it; ACR_ERR_INVALID_ARG if
 * the file was written for another architecture or is malformed. */
acr_status acr_tune_load(const char* path);
/* Drop the table and the noted keys; built-in choices from now on. */
acr_status acr_tune_clear(void);

/* How solve passes with at most 8 right-hand sides and no early stop run
 * (process-wide; the levels of the pass are those of Section 3's
 * back-substitution).
 *   mode 0 (default): two grouped launches per matvec step (projections,
 *     then rows), ordered by the stream.  For a single handle the steps'
 *     descriptors and the pass's workspace are laid out and copied to the
 *     device on the first solve with a given nrhs on a given stream and host
 *     thread (that call synchronises `stream` once) and kept with the handle
 *     (about 16 N nrhs bytes in FP32; at most 16 such passes per handle, later
 *     combinations plan on every call) until acr_destroy, so a pass only
 *     enqueues its launches.  acr_solve_batched and the serving loop, whose
 *     handles and nrhs change from call to call, plan on every call as in
 *     mode 3.
 *   mode 1: the levels of at most 16 blocks, the last block and their
 *     back-substitution as one persistent launch; the wider levels as in
 *     mode 0.
 *   mode 2: the whole pass as one persistent launch.
 *   mode 3: as mode 0, with the steps laid out and their descriptors copied
 *     on every call (nothing kept).
 * In a persistent launch the matvecs are tasks (some projection units, or
 * 256 output rows, of one block).  Workgroups take them in an order in
 * which each task follows the tasks it reads from, wait (polling a counter,
 * bounded) until those are done, run, and count themselves done; the waits
 * cannot deadlock whatever number of workgroups is resident.  The task list
 * is built on a handle's first persistent solve with a given nrhs (that call
 * synchronises `stream` once) and kept with the handle.  Every mode computes
 * every value with the same device code in the same order, so results are
 * equal bit for bit across modes.  wait_limit > 0: polls a
 * task makes on one counter before it gives up; 0: the default, 2^22 polls
 * (seconds); < 0: every task that reads another task's output gives up (this
 * forces the failure path).  Once a task gives up, every later wait of the
 * launch gives up at once, every workgroup still runs to the end of the task
 * list, and the pass's solution X is set to NaN.  ACR_ERR_INVALID_ARG for
 * another mode. */
acr_status acr_set_solve_mode(int32_t mode, int64_t wait_limit);

/* Number of kernel launches (and device fills) the calling thread has
 * issued through the library so far (for launch counts per step). */
int64_t acr_launch_count(void);

/* Release the library's cached (unused) device memory: the blocks cached for
 * the calling thread and the idle ones. */
acr_status acr_trim_pool(void);

/* Device memory source of the library (the boundary's allocator hook, for
 * callers such as PyTorch that own device memory).  alloc(bytes, stream)
 * returns a device pointer (NULL on failure, reported as ACR_ERR_OOM) whose
 * memory may be used on `stream` (a hipStream_t); free(ptr, stream) returns
 * it.  Passing NULL for both restores hipMalloc / hipFree.  Allowed only
 * while the library holds no live device allocation (no handle exists):
 * otherwise ACR_ERR_INVALID_ARG.  Cached blocks of the previous source are
 * returned to it first.  The callbacks may be called from any library call
 * of any thread, between the calls' kernel launches. */
acr_status acr_set_allocator(void* (*alloc_fn)(size_t bytes, void* stream),
                             void (*free_fn)(void* ptr, void* stream));

#ifdef __cplusplus
}
#endif
#endif
