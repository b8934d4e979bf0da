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
// so every depth is one s x k[d] matrix per HODLR, and all clusters of a depth
// are processed by one batched launch.  Ranks are padded to the set maximum
// per depth (padding columns are zero).
#pragma once

#include <vector>

#include "common.hpp"

namespace acr {

template <typename T>
struct HSet {
  int cnt = 0, s = 0, b = 0, L = 0;
  std::vector<int> k;    // allocated columns per depth (index 0 unused)
  std::vector<int> kc;   // filled columns per depth
  DBuf<T> lv;
  std::vector<DBuf<T>> U, V;

  int nleaf() const { return 1 << L; }
  int sd(int d) const { return s >> d; }
  long long leaf_stride() const { return (long long)nleaf() * b * b; }
  void alloc(hipStream_t st, int cnt_, int s_, int b_, int L_, const std::vector<int>& k_,
             bool zero);
  size_t bytes() const;
  int max_rank() const;
};

// A HODLR operand: set + matrix index map (matrix m of an operation uses
// entry mmul*m + moff of the set).
template <typename T>
struct HV {
  const HSet<T>* h;
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

// out_m = alpha * op(Hdiag_m) Y_m + beta * out_m, where Hdiag_m is the
// block-diagonal part of H_m at depth dfrom (leaves plus off-diagonal blocks
// of depth > dfrom; dfrom = 0 is the whole matrix) and op = transpose if trans.
template <typename T>
void hmul(hipStream_t st, HV<T> H, int nmat, int dfrom, bool trans, int ncol, T alpha, Flat<T> Y,
          T beta, Flat<T> out);

// C_m = alpha * A_m B_m with exact low-rank accumulation (no truncation).
// C is allocated with cnt_alloc >= nmat entries (extra entries zero).
template <typename T>
void hprod(hipStream_t st, HSet<T>& C, int cnt_alloc, HV<T> A, HV<T> B, int nmat, T alpha);

// X_m = M_m^{-1}, exact in exact arithmetic (bottom-up Sherman-Morrison-
// Woodbury over the depths; the capacitance and leaf inverses in FP64).
template <typename T>
void hinv(hipStream_t st, HSet<T>& X, HV<T> M, int nmat, int* status);

// One term of a stacked sum: coef * diag(rows)? * H_m; `rows` (optional) is a
// per-matrix vector of s values at rows + (rmul*m + roff)*s.
template <typename T>
struct STerm {
  HV<T> h;
  T coef = T(1);
  const T* rows = nullptr;
  int rmul = 1, roff = 0;
};

// C_m = sum_t terms: factors stacked side by side (ranks add), leaves summed.
template <typename T>
void hstack(hipStream_t st, HSet<T>& C, int cnt_alloc, const std::vector<STerm<T>>& terms,
            int nmat);

// C_m = H_m diag(cols_(cmul*m+coff)) (column scaling: leaves' columns and V rows).
template <typename T>
void hscale_cols(hipStream_t st, HSet<T>& C, int cnt_alloc, HV<T> H, const T* cols, int cmul,
                 int coff, int nmat);

// T_eps of every off-diagonal block of every matrix in the set (in place):
// QR of the stacked U and V, SVD of R_U R_V^T, keep s_t > eps * s_1.
template <typename T>
void recompress(hipStream_t st, HSet<T>& H, double eps, int maxrank);

// Dense copy of matrix m (host, column-major s x s, FP64).  Synchronises st.
template <typename T>
void densify_to_host(hipStream_t st, const HSet<T>& H, int m, double* out);

// Algorithmic work counters of the batched primitives (host side, from the
// shapes launched): flops and the name of the calling phase.
struct Work {
  double gemm_flops = 0, qr_flops = 0, svd_flops = 0, inv_flops = 0;
  double total() const { return gemm_flops + qr_flops + svd_flops + inv_flops; }
};
Work& work();

}  // namespace acr
