// Batched HODLR (weak-admissibility H-matrix) sets on the device and the
// H-arithmetic of one cyclic-reduction level (Section 3 of the paper).
//
// A set holds `cnt` HODLR matrices of size s sharing one cluster tree: a
// cluster of size > leaf is halved, L times, down to leaves of size b = s/2^L.
// Storage ("flat" per depth, column-major):
//   lv     : [cnt][2^L][b][b]   dense diagonal leaves
//   U[d]   : [cnt][k[d]][s]     depth d = 1..L: rows of cluster tau (size s/2^d)
//                               hold U_tau of the block A[tau, sib(tau)] = U_tau V_tau^T
//   V[d]   : [cnt][k[d]][s]     rows of cluster sib(tau) hold V_tau
// so every depth is one s x k[d] matrix per HODLR, and all clusters of all
// depths and of several independent operations are processed by a few
// grouped launches.  Ranks are padded to the set maximum per depth (padding
// columns are zero).
#pragma once

#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace acr {

template <typename T>
struct HSet {
  int cnt = 0, s = 0, b = 0, L = 0;
  std::vector<int> k;    // allocated columns per depth (index 0 unused)
  std::vector<int> kc;   // filled columns per depth
  // sum over the cnt * 2^d blocks of depth d of their numerical ranks, once
  // known (after a truncation); -1 = every block has kc[d] columns
  std::vector<double> rsum;
  DBuf<T> lv;
  std::vector<DBuf<T>> U, V;

  int nleaf() const { return 1 << L; }
  int sd(int d) const { return s >> d; }
  long long leaf_stride() const { return (long long)nleaf() * b * b; }
  // allocate cnt_ matrices; with zero_from >= 0 the matrices [zero_from, cnt_)
  // are set to zero (the others are written by the caller)
  void alloc(hipStream_t st, int cnt_, int s_, int b_, int L_, const std::vector<int>& k_,
             int zero_from);
  size_t bytes() const;
  int max_rank() const;
  // sum of the ranks of the depth-d blocks of all matrices, and their mean
  double rank_sum(int d) const {
    return (d < (int)rsum.size() && rsum[d] >= 0.0) ? rsum[d] : (double)kc[d] * cnt * (1 << d);
  }
  double rank_mean(int d) const { return cnt ? rank_sum(d) / ((double)cnt * (1 << d)) : 0.0; }
  // bytes of the stored factor at the blocks' numerical ranks (no padding)
  double bytes_ranked() const;
};

// A HODLR operand: set + matrix index map (matrix m of an operation uses
// entry mmul*m + moff of the set).
template <typename T>
struct HV {
  const HSet<T>* h = nullptr;
  int mmul = 1, moff = 0;
};

// Flat operand: one s x ncol column-major matrix per matrix index.
template <typename T>
struct Flat {
  T* p = nullptr;
  int ld = 0;
  long long sm = 0;
  int mmul = 1, moff = 0;
};

// Jobs of one grouped GEMM launch.
struct GemmPlan {
  std::vector<GJob> jobs;
  std::vector<GSeg> segs;
  void add(int M, int N, int nmat, int ncl, double alpha, double beta, const BOp& C,
           const std::vector<GSeg>& sg);
  template <typename T>
  void run(hipStream_t st);
  bool empty() const { return jobs.empty(); }
};

// HODLR multi-vector product alpha * op(Hdiag) Y with Hdiag the block-diagonal
// part of H at depth dfrom (leaves + off-diagonal blocks of depth > dfrom;
// dfrom = 0 is the whole matrix).  Adds the per-depth reductions
// T_d = F_d[cl]^T Y[cl] to `red` and returns the K-segments whose sum, per
// leaf row block, is the product (leaf block times Y, then every depth's
// U_d[rows] T_d[sibling ancestor]).  Temporaries are appended to `keep`.
template <typename T>
std::vector<GSeg> plan_hmul(GemmPlan& red, std::vector<DBuf<T>>& keep, HV<T> H, int nmat,
                            int dfrom, bool trans, int ncol, double alpha, Flat<T> Y);

// Operand of rows (cluster c of size sc) of a flat matrix.
template <typename T>
BOp flat_op(const Flat<T>& f, long long sc, int col0 = 0);

// out_m = alpha op(Hdiag_m) Y_m + beta out_m (two grouped launches).
template <typename T>
void hmul(hipStream_t st, HV<T> H, int nmat, int dfrom, bool trans, int ncol, T alpha, Flat<T> Y,
          T beta, Flat<T> out);

// One product term coef * A_m B_m of a sum of products.
template <typename T>
struct PTerm {
  double coef = 1.0;
  HV<T> A, B;
};

// C_m = D_m (optional) + sum_t coef_t A_t,m B_t,m, accumulated exactly in
// low-rank form (ranks add, no truncation).  C gets cnt_alloc >= nmat
// entries (extra entries zero).
template <typename T>
struct POut {
  HSet<T>* C = nullptr;
  int cnt_alloc = 0, nmat = 0;
  bool has_d = false;
  HV<T> D;
  std::vector<PTerm<T>> terms;
};

// All outputs are planned together: three grouped GEMM stages and two grouped
// copies, whatever the number of outputs, terms and depths.
template <typename T>
void hprod_multi(hipStream_t st, std::vector<POut<T>>& outs);

// X_m = M_m^{-1}, exact in exact arithmetic (bottom-up Sherman-Morrison-
// Woodbury over the depths; the capacitance and leaf inverses in FP64).
// Several inversions (of sets of different shapes) are planned together:
// their steps share launches, counted from the bottom depth of each tree.
template <typename T>
struct HInvJob {
  HSet<T>* X = nullptr;
  HV<T> M;
  int nmat = 0;
  int* status = nullptr;   // set to 1 on a zero or non-finite pivot
};
template <typename T>
void hinv_multi(hipStream_t st, std::vector<HInvJob<T>>& jobs);
template <typename T>
void hinv(hipStream_t st, HSet<T>& X, HV<T> M, int nmat, int* status);

// Level-0 operations with diagonal E/F (scalings): see acr.hip.
// C_m = diag(rows_(rmul*m+roff))? * coef * H_m  (copy with optional row scale)
// or, with cols set, H_m diag(cols_(cmul*m+coff)).
template <typename T>
struct ScaleTerm {
  HV<T> h;
  double coef = 1.0;
  const T* rows = nullptr;
  int rmul = 1, roff = 0;
};

// C_m = sum_t coef_t diag(rows_t) H_t,m (stack of scaled sets), for several
// outputs at once.
template <typename T>
struct StackOut {
  HSet<T>* C = nullptr;
  int cnt_alloc = 0, nmat = 0;
  std::vector<ScaleTerm<T>> terms;
};
template <typename T>
void hstack_multi(hipStream_t st, std::vector<StackOut<T>>& outs);

// C_m = H_m diag(cols_(cmul*m+coff)) for several outputs at once.
template <typename T>
struct ColScale {
  HSet<T>* C = nullptr;
  int cnt_alloc = 0, nmat = 0;
  HV<T> H;
  const T* cols = nullptr;
  int cmul = 1, coff = 0;
};
template <typename T>
void hscale_cols_multi(hipStream_t st, std::vector<ColScale<T>>& outs);

// T_eps of every off-diagonal block of every matrix of every set (in place):
// QR of the stacked U and V, rank-revealing SVD of R_U R_V^T, keep
// s_t > eps * s_1.  One synchronisation for all sets and depths.
template <typename T>
void recompress_multi(hipStream_t st, const std::vector<HSet<T>*>& sets, double eps, int maxrank);

// Dense copy of matrix m (host, column-major s x s, FP64).  Synchronises st.
template <typename T>
void densify_to_host(hipStream_t st, const HSet<T>& H, int m, double* out);

// Algorithmic work counters of the factorisation (host side, from shapes).
struct Work {
  double gemm_flops = 0, qr_flops = 0, svd_flops = 0, inv_flops = 0;
  double total() const { return gemm_flops + qr_flops + svd_flops + inv_flops; }
};
Work& work();

}  // namespace acr
