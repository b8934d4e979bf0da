// Host launchers of the ACR device kernels (gfx950).  Every launcher enqueues
// on `st` and checks the launch.  Problems of a batched call are indexed
// p = m*ncl + c (matrix m, cluster c) unless stated otherwise.
#pragma once

#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace acr {

// ------------------------------------------------------------ grouped jobs
// A grouped launch runs a list of independent jobs (each a batch of uniform
// problems) in one kernel; workgroups [block0, next block0) belong to a job.
constexpr int kMaxSeg = 16;

// C = alpha * sum_s op(A_s) op(B_s) + beta * C over the problems (m, c) of a
// job; segment s contributes a K_s-deep product (a K-concatenated GEMM).
struct GSeg {
  BOp A, B;
  int K = 0, pad = 0;
  double scale = 1.0;   // multiplies this segment's product
};
struct GJob {
  long long block0 = 0;
  int M = 0, N = 0, nmat = 0, ncl = 0;
  int tilesM = 0, tilesN = 0, seg0 = 0, nseg = 0;
  int kind = 0, pad = 0;   // kernel kind (set by the launcher)
  double alpha = 1.0, beta = 0.0;
  BOp C;
};

// Householder R (and optionally reflectors) of p x k panels, one workgroup
// per problem; R at R + prob*c*k (c = min(p, k), ld c), reflectors at
// Vref + prob*p*c, tau + prob*c; ws = global scratch when the panel does not
// fit in LDS (p*k per problem).
struct QJob {
  long long block0 = 0;
  int p = 0, k = 0, nmat = 0, ncl = 0;
  BOp A;
  void* R = nullptr;
  void* Vref = nullptr;
  void* tau = nullptr;
  void* ws = nullptr;
  int lds = 0, pad = 0;
};

// Rank-revealing SVD of c x c cores (see brsvd).
struct SJob {
  long long block0 = 0;
  int c = 0, nprob = 0;
  void* K = nullptr;
  void* X = nullptr;
  void* J = nullptr;
  void* sig = nullptr;
  void* UK = nullptr;
  int* rank = nullptr;
  double* flops = nullptr;
  double eps = 0.0;
  int maxrank = 0, lds = 0;   // lds: K, X and J staged in LDS
  int* redo = nullptr;        // register path: per-problem "left to the general kernel" flags
};

// Y_(m,c) = Q_(m,c) [Z_(m, c^zxor); 0] with reflectors of a QJob.
struct AJob {
  long long block0 = 0;
  int p = 0, c = 0, t = 0, nmat = 0, ncl = 0, zxor = 0, lds = 0, pad = 0;
  int wslot = 0, pad2 = 0;
  const void* Vref = nullptr;
  const void* tau = nullptr;
  const void* Z = nullptr;
  long long sZ = 0;
  BOp Y;
};

// dst_(m,c) (= or +=) alpha * diag? * src_(m,c), rows x cols each; optional
// scale vector: element (r, q) is multiplied by
// scale[(smul*m + soff)*sstride + c*scl + (sside ? q : r)].
struct CJob {
  long long block0 = 0;
  int rows = 0, cols = 0, nmat = 0, ncl = 0, chunks = 0, accumulate = 0;
  double alpha = 1.0;
  BOp src, dst;
  const void* scale = nullptr;
  int smul = 1, soff = 0, sside = 0;
  int vec = 0;   // set by the launcher: 16-byte accesses
  long long sstride = 0, scl = 0;
};

// Multi-term HODLR matvec for a few right-hand sides (solve path):
//   out_m = beta * C0_m + sum_t alpha_t op_t(m) y_t(m)
// with op_t a HODLR matrix of a set or a diagonal.  Every job has its own
// block size s, leaf b, depth L and number of right-hand sides (<= 8), so the
// jobs of several independent problems share the launches.  Vector blocks are
// s x nrhs, column-major, block stride s*nrhs; block index of matrix m is
// mul*m + off for every operand.  The output may not overlap any input.
constexpr int kMvMaxDepth = 15;
struct MVTerm {
  int type = 0;               // 0 HODLR, 1 diagonal
  int mmul = 1, moff = 0;     // operator index
  int ymul = 1, yoff = 0;     // y block index
  int pad = 0;
  double alpha = 1.0;
  const void* y = nullptr;
  const void* lv = nullptr;   // leaves [cnt][2^L][b][b] (HODLR) or diagonals [cnt][s]
  const void* U[kMvMaxDepth + 1] = {};
  const void* V[kMvMaxDepth + 1] = {};
  int k[kMvMaxDepth + 1] = {};    // allocated columns per depth (matrix stride k*s)
  int kc[kMvMaxDepth + 1] = {};   // used columns
  // set by the launcher: projections V_d[node]^T y[node] of matrix m at
  // tbase + m * tstride + toff[d] + (node * kc[d] + column) * NR + rhs;
  // s and nrhs of the job the term belongs to
  long long tbase = 0;
  int tstride = 0, s = 0, nrhs = 0, pad2 = 0;
  int toff[kMvMaxDepth + 1] = {};
  // host only (algorithmic counts): mean numerical rank of the depth-d blocks
  // (<= kc[d]; the padding columns up to kc[d] are zeros)
  float kmean[kMvMaxDepth + 1] = {};
};
struct MVRed {                    // projections of one term (launcher-internal)
  long long block0 = 0;           // first wave
  int term = 0, upm = 0;          // term index, waves per matrix
};
struct MVJob {
  long long block0 = 0;
  int nmat = 0, nterm = 0, term0 = 0;
  int omul = 1, ooff = 0, cmul = 1, coff = 0;
  int s = 0, b = 0, L = 0, nrhs = 0;   // shapes of this job's operands
  double beta = 0.0;
  const void* C0 = nullptr;       // null: out = sum of terms
  void* out = nullptr;
};

// Jobs keep their own s, b, L and nrhs (1..8).
template <typename T>
void ghmv(hipStream_t st, std::vector<MVJob> jobs, const std::vector<MVTerm>& terms);
// ghmv in two halves, for a caller that keeps a step's descriptors in device
// memory and launches it many times: hmv_plan lays out the step (the
// descriptors to copy to the device, the grid sizes, the projection buffer
// size tsize and the algorithmic counts); hmv_launch enqueues its two
// launches with the device copies of reds, terms and jobs.
struct HmvStep {
  std::vector<MVRed> reds;
  std::vector<MVTerm> terms;
  std::vector<MVJob> jobs;
  long long rows = 0, units = 0, tsize = 0;
  int NR = 1;
  bool w64 = true;
  double flr = 0, byr = 0, fla = 0, bya = 0;
};
template <typename T>
HmvStep hmv_plan(std::vector<MVJob> jobs, const std::vector<MVTerm>& terms);
template <typename T>
void hmv_launch(hipStream_t st, const HmvStep& h, const MVRed* reds, const MVTerm* terms, const MVJob* jobs, T* tbuf);
// All jobs with the same shapes.
template <typename T>
void ghmv(hipStream_t st, int s, int b, int L, int nrhs, std::vector<MVJob> jobs,
          const std::vector<MVTerm>& terms);

// Block-major <-> column-major vector layouts for several problems at once:
// V[i][q][j] = B[(i*s + j) + q*ld] for the nblk blocks of each job.
struct VJob {
  long long block0 = 0;   // first workgroup
  int s = 0, nblk = 0, nrhs = 0, per = 0;
  long long ld = 0;
  const void* src = nullptr;
  void* dst = nullptr;
};
template <typename T>
void gto_blocks(hipStream_t st, std::vector<VJob> jobs);     // src double, dst T
template <typename T>
void gfrom_blocks(hipStream_t st, std::vector<VJob> jobs);   // src T, dst double

// ------------------------------------------------- persistent solve pass
// A solve pass as one launch over a task list.  A task is either some
// projection units of one (term, matrix) of a matvec step (kind 0) or up to
// 256 output rows of one output block (kind 1).  Workgroups take the tasks
// in list order; a task first waits until the counters of the tasks whose
// outputs it reads have reached their totals (ndep pairs counter, total),
// then runs and adds one to its own counter.  Every task follows the tasks
// it waits for in the list.  In the jobs and terms of a pass the vector
// operands (y, C0, out) are byte offsets into the pass's workspace, and the
// projection buffer lies at tbuf_off in it; factor operands are device
// addresses.  Counters start at zero.
constexpr int kPMaxDep = 5;
struct PTask {
  int kind = 0;        // 0 projections, 1 output rows
  int idx = 0;         // term (kind 0) or job (kind 1), indices of the pass
  int m = 0;           // matrix of the term or job
  int u0 = 0, u1 = 0;  // units [u0, u1) of the matrix, or rows [u0, u1) of the block
  int done = 0;        // counter this task adds one to
  int ndep = 0, pad = 0;
  int dep[kPMaxDep] = {};
  int need[kPMaxDep] = {};
};
struct PInst {              // one pass of a launch
  long long task0 = 0;      // ticket of its first task (set by the launcher)
  const PTask* tasks = nullptr;
  const MVJob* jobs = nullptr;
  const MVTerm* terms = nullptr;
  char* ws = nullptr;       // the pass's workspace
  int* ctr = nullptr;       // its counters, zero at the start
  long long tbuf_off = 0;   // projection buffer in the workspace (bytes)
  int ntasks = 0, pad = 0;
};
// Task list of a sequence of matvec steps, each given as to ghmv (vector
// operands as workspace offsets).  NR: the right-hand-side slots of the
// projections (1, 2, 4 or 8, at least every job's nrhs).
struct PBuilder {
  explicit PBuilder(int nr) : NR(nr) {}
  int NR = 1;
  bool w64 = true;      // every job's leaf size is a multiple of 64
  std::vector<PTask> tasks;
  std::vector<MVJob> jobs;
  std::vector<MVTerm> terms;
  long long tsize = 0;  // projection buffer elements
  int nctr = 0;
  double flops = 0, bytes = 0;   // algorithmic counts (numerical ranks)
  template <typename T>
  void step(std::vector<MVJob> jobs, const std::vector<MVTerm>& terms);
  // Checks the list (ACR_ERR_INTERNAL otherwise): counters in range, and
  // every counter a task waits for reaches the awaited total from tasks
  // listed before it alone, so no wait depends on a later task.
  void check() const;
 private:
  std::map<long long, std::pair<int, int>> prod_;   // output block offset -> (counter, total)
};
// Runs the passes `insts` (built with the same NR and row form) in one launch
// on st; then, if a wait gave up, sets the final unknowns `fin` (the sources
// of the block-to-vector copies that follow) to NaN.  ctl: two ints of device
// memory, zero (ticket, abort word).
template <typename T>
void psolve_run(hipStream_t st, std::vector<PInst> insts, int NR, bool w64, int* ctl, const std::vector<VJob>& fin,
                double flops, double bytes);
// Process-wide solve-pass settings: mode 0 grouped launches per step, 1 the
// levels of few blocks as one persistent launch, 2 the whole pass as one
// persistent launch; wait limit in polls per dependency (< 0: every task
// with dependencies gives up).
struct SolveMode {
  std::atomic<int> mode{0};
  std::atomic<long long> limit{1LL << 22};
  static SolveMode& get() {
    static SolveMode m;
    return m;
  }
};

// Level-0 ingest of the five-point operator, grouped over problems: job j
// covers matrices m = 0..nmat-1 of one problem, which use block row
// bmul*m + boff of that problem's stencil arrays (diag, west = D[i][i-1],
// east = D[i][i+1]).  `per` and block0 are set by the launchers.
struct OpJob {
  long long block0 = 0;
  int s = 0, b = 0, L = 0, nmat = 0, bmul = 1, boff = 0, per = 1, zblk = -1;
  int pnx = 0;                     // 3-D operators: row length of a plane (0: five-point)
  const double* diag = nullptr;
  const double* west = nullptr;
  const double* east = nullptr;
  const double* south = nullptr;   // 3-D: in-plane couplings to r - pnx and r + pnx
  const double* north = nullptr;
  const double* src = nullptr;     // ggather_diag: the stencil array gathered
  void* out = nullptr;             // leaves [nmat][2^L][b][b] or gathered diagonals [nmat][s]
  void* U[kMvMaxDepth + 1] = {};   // depth-d factors, matrix m at U[d] + m*s (one column)
  void* V[kMvMaxDepth + 1] = {};
  int* flag = nullptr;             // gtridiag_inverse: set to 1 on a breakdown
};
// Leaves: the tridiagonal band restricted to each b x b diagonal leaf of D_i
// (3-D, pnx > 0: the plane's five-point operator, x couplings cut at the ends
// of each row of pnx unknowns).
template <typename T>
void gleaves_tridiag(hipStream_t st, std::vector<OpJob> jobs);
// Exact factors of the off-diagonal blocks of a plane operator D_k (3-D,
// pnx > 0) at every depth d = 1..L: where the children of a cluster hold whole
// rows of the plane (s/2^d a multiple of pnx) the block couples the last pnx
// unknowns of the first child to the first pnx of the second (rank pnx, the
// y couplings); inside one row it is the single x coupling (rank 1).
int plane_rank(int s, int d, int pnx);
template <typename T>
void gplane_factors(hipStream_t st, std::vector<OpJob> jobs);
// Depth-d rank-one factors of D_i for every depth d = 1..L (Section 3:
// tridiagonal D_i has exact rank-1 off-diagonal blocks).
template <typename T>
void grank1_factors(hipStream_t st, std::vector<OpJob> jobs);
// out[m][r] = src[(bmul*m + boff)*s + r], zero for block row zblk (E_0 and
// F_(ny-1) couple to rows outside the grid).
template <typename T>
void ggather_diag(hipStream_t st, std::vector<OpJob> jobs);
// X_m = D^{-1} for the tridiagonal D of block row bmul*m + boff, written
// directly in HODLR form (leaves in out, rank-one factors in U/V); *flag = 1
// when the elimination without pivoting breaks down (the caller then uses the
// general H-inverse).  Needs s <= 3072.
template <typename T>
void gtridiag_inverse(hipStream_t st, std::vector<OpJob> jobs);

// *flag = 1 if any of a[0..n) is NaN or infinite, per job.
struct NFJob {
  long long block0 = 0;
  long long n = 0;
  const double* a = nullptr;
  int* flag = nullptr;
  int per = 1, pad = 0;
};
void gflag_nonfinite(hipStream_t st, std::vector<NFJob> jobs);


// force_tile (0..4) / force_form (4 one wave, 2 registers, 0 LDS) bypass the
// tuned or built-in choice (tuning runs).
template <typename T>
void ggemm(hipStream_t st, std::vector<GJob> jobs, const std::vector<GSeg>& segs, int force_tile = -1);
template <typename T>
void gqr(hipStream_t st, std::vector<QJob> jobs, int force_form = -1);

// Full-rank HODLR form of dense s x s blocks (the dense operator ingest):
// for matrix m (at A + m*s*s, column-major): leaves = the diagonal b x b
// blocks; at depth d the block A[tau, sib tau] is stored as U_tau = that
// block (sd columns, rows of tau) and V_tau = I (rows of sib tau).  U[d], V[d]
// have sd columns per matrix (k[d] = sd).
struct HJob {
  long long block0 = 0;
  int s = 0, b = 0, L = 0, nmat = 0, per = 1, zm = -1;   // matrix zm is taken as zero
  const double* A = nullptr;
  void* lv = nullptr;
  void* U[kMvMaxDepth + 1] = {};
  void* V[kMvMaxDepth + 1] = {};
};
template <typename T>
void gdense_to_hodlr(hipStream_t st, std::vector<HJob> jobs);

// Dense assembly of one s x s block of a block-tridiagonal system (early
// stop): out[r + c*ld] (FP64) = entry (r, c) of matrix midx of a HODLR set
// (type 0: leaves lv, factors U/V as in MVTerm) or diag(d) with d = lv + midx*s
// (type 1).  `per` workgroups per block (set by the launcher).
struct DenseJob {
  long long block0 = 0;
  int type = 0, s = 0, b = 0, L = 0, midx = 0, per = 1;
  const void* lv = nullptr;
  const void* U[kMvMaxDepth + 1] = {};
  const void* V[kMvMaxDepth + 1] = {};
  int k[kMvMaxDepth + 1] = {};
  int kc[kMvMaxDepth + 1] = {};
  double* out = nullptr;
  long long ld = 0;
};
template <typename T>
void gdense_blocks(hipStream_t st, std::vector<DenseJob> jobs);

// Kernel-variant table of the autotuner (see kernels.hip): key -> choice.
struct Tuner {
  std::mutex mu;
  std::map<std::string, int> table;        // measured choices
  std::map<std::string, long long> seen;   // keys met while recording (largest problem count)
  bool active = false;                     // use the table
  bool recording = false;                  // note the keys met
  static Tuner& get();
  int lookup(const std::string& key);
  void note(const std::string& key, long long nprob);
};
// Measure every recorded key that has no entry yet; returns how many were added.
int tune_run(hipStream_t st);
template <typename T>
void grsvd(hipStream_t st, std::vector<SJob> jobs);
template <typename T>
void gapply_q(hipStream_t st, std::vector<AJob> jobs);
template <typename T>
void gcopy(hipStream_t st, std::vector<CJob> jobs);

// C_p = alpha * op(A_p) op(B_p) + beta * C_p, all problems M x N x K.
// beta == 0 overwrites C without reading it.
template <typename T>
void bgemm(hipStream_t st, int M, int N, int K, int nmat, int ncl, T alpha, const BOp& A,
           const BOp& B, T beta, const BOp& C);

// Grouped small dense inverses: job j inverts its nprob matrices of size n
// (A at A + p*sA, X at X + p*sX, ld n) as binverse does; jobs of one call may
// have different sizes.  ws / use_lds are set by the launcher.
struct IJob {
  long long block0 = 0;
  int n = 0, nprob = 0;
  const void* A = nullptr;
  long long sA = 0;
  void* X = nullptr;
  long long sX = 0;
  int* status = nullptr;
  double* ws = nullptr;
  int use_lds = 0;
  // capacitance mode (cap_k > 0, n = 2 cap_k): matrix p is not read from A
  // but formed from the cores c_(2p), c_(2p+1) (cap_k x cap_k each, contiguous)
  // as [[I, c_(2p+1)], [c_(2p), I]]
  int cap_k = 0;
  const void* cores = nullptr;
};
template <typename Tin, typename Tout>
void ginverse(hipStream_t st, std::vector<IJob> jobs);

// X_p = A_p^{-1} (n x n, Gauss-Jordan with partial pivoting, computed in FP64).
// A_p at A + p*sA (ld n), X_p at X + p*sX (ld n).  *status set to 1 on a zero
// or non-finite pivot.
template <typename Tin, typename Tout>
void binverse(hipStream_t st, int n, int nprob, const Tin* A, long long sA, Tout* X,
              long long sX, int* status);

// R factor of the Householder QR of each p x k operand A_(m,c):
// R_p = c x k upper trapezoidal, c = min(p, k), column-major ld = c, at R + p*c*k.
// If Vref is given, the reflectors are kept: v_j (p values, zero above row j,
// v_j[j] = 1) at Vref + (p_idx*c + j)*p and tau_j at tau + p_idx*c + j, so that
// Q = H_0 H_1 ... H_(c-1), H_j = I - tau_j v_j v_j^T.
template <typename T>
void bqr_r(hipStream_t st, int p, int k, int nmat, int ncl, const BOp& A, T* R, T* Vref = nullptr,
           T* tau = nullptr);

// Y_(m,c) = Q_(m,c) [Z; 0] with the reflectors of a bqr_r call (same p, c
// and problem order); Z of problem (m, c) is the c x t block at
// Z + (m*ncl + (c ^ zxor)) * sZ (ld c).
template <typename T>
void bapply_q(hipStream_t st, int p, int c, int t, int nmat, int ncl, const T* Vref, const T* tau,
              const T* Z, long long sZ, int zxor, const BOp& Y);

// Rank-revealing SVD of each c x c core K_p (at K + p*c*c, ld c; overwritten):
// column-pivoted QR stopped at 0.1*eps of the largest column, one-sided Jacobi
// on the thin transposed triangle, left singular vectors U_K = Q_K [J; 0].
// Outputs per problem: sig[c] sorted decreasing, UK (c x c, columns = left
// singular vectors in that order, zero past the numerical rank), rank_p =
// #{sig > eps*sig_1} capped by maxrank (> 0).
template <typename T>
void brsvd(hipStream_t st, int c, int nprob, T* K, T* sig, T* UK, int* rank, double eps, int maxrank);


// dst_m = alpha * src_m (rows x cols each; ld / stride per matrix / maps in
// the BOps; cluster fields ignored).
template <typename T>
void bcopy(hipStream_t st, int rows, int cols, int nmat, T alpha, const BOp& src, const BOp& dst);
// dst_m += alpha * src_m
template <typename T>
void badd(hipStream_t st, int rows, int cols, int nmat, T alpha, const BOp& src, const BOp& dst);

// Fill n values with v.
template <typename T>
void fill(hipStream_t st, T* p, size_t n, T v);

// Scale rows (side 0) or columns (side 1) of per-matrix / per-cluster blocks:
// X_(m,c)[r, q] *= alpha * vec[(vmul*m+voff)*vstride + c*vcl + (side ? q : r)].
// The operand uses the cluster fields of X (sc_pair/sc_odd).
template <typename T>
void bscale(hipStream_t st, int rows, int cols, int nmat, int ncl, const BOp& X, const T* vec,
            int vmul, int voff, long long vstride, long long vcl, int side, T alpha);

// Block-major <-> column-major vector layouts.  V[i][q][j] = B[(i*s + j) + q*ld].
template <typename T>
void to_blocks(hipStream_t st, int s, int nblk, int nrhs, const double* B, long long ld, T* V);
template <typename T>
void from_blocks(hipStream_t st, int s, int nblk, int nrhs, const T* V, double* B, long long ld);

// y = y + alpha * diag(d_(bmul*j+boff)) * x_j  for vectors in block-major form
// (nmat blocks of s x nrhs).  Rows scaled by d.
template <typename T>
void bdiag_axpy(hipStream_t st, int s, int nrhs, int nmat, T alpha, const T* d, int dmul, int doff,
                const T* x, int xmul, int xoff, T* y, int ymul, int yoff);

// R = B - A X (FP64 5-point stencil); N = nx*ny, columns nrhs, ld N.
void stencil_residual(hipStream_t st, int nx, int ny, int nrhs, const double* diag,
                      const double* west, const double* east, const double* south,
                      const double* north, const double* X, const double* B, double* R);

// Refinement vector work of several problems in one launch: job j covers
// nrhs columns of N = nx*ny FP64 values (column q at offset q*N).
//   gresidual:  R = B - A X with the job's five-point stencil;
//   gcol_sumsq: out[q] = sum_i R[i + q*N]^2 (fixed chunking per N, fixed
//               summation order: the same bits whatever the batch);
//   gaxpy:      R += B (X += D with R = X, B = D).
struct RJob {
  long long block0 = 0;
  int nx = 0, ny = 0, nrhs = 0, per = 0;
  const double* diag = nullptr;
  const double* west = nullptr;
  const double* east = nullptr;
  const double* south = nullptr;
  const double* north = nullptr;
  const double* X = nullptr;
  const double* B = nullptr;
  double* R = nullptr;
  double* part = nullptr;   // set by gcol_sumsq
  double* out = nullptr;
};
void gresidual(hipStream_t st, std::vector<RJob> jobs);
// R = B - A X for a 7-point operator (3-D; nx*ny*nz FP64 values per column).
void stencil_residual3d(hipStream_t st, int nx, int ny, int nz, int nrhs, const double* const* a7,
                        const double* X, const double* B, double* R);
void gcol_sumsq(hipStream_t st, std::vector<RJob> jobs);
void gaxpy(hipStream_t st, std::vector<RJob> jobs);

// out[q] = sum_i A[i + q*n]^2  (n rows, ncol columns), FP64.
void col_sumsq(hipStream_t st, long long n, int ncol, const double* A, double* out);


// Diagnostics: whether a[0..n) holds a NaN/Inf and the largest finite |a|.
// Synchronises st.
template <typename T>
void scan_values(hipStream_t st, long long n, const T* a, bool* bad, double* amax);

// X += D (both N x nrhs FP64).
void axpy_d(hipStream_t st, long long n, const double* D, double* X);
// Krylov vector kernels (FP64): out[i] = V_i . w for i < nvec (V_i at V + i*ldv,
// deterministic two-stage sum); w = a w + sc * sum_i c_i V_i with c on the device.
void mdot(hipStream_t st, long long n, int nvec, const double* V, long long ldv, const double* w, double* out);
void maxpy(hipStream_t st, long long n, int nvec, double a, double sc, const double* c, const double* V,
           long long ldv, double* w);

}  // namespace acr
