// Accelerated Cyclic Reduction driver and the extern "C" entry points.
//
// Factor (Section 3): level by level over the current m blocks, with the
// even block indices k eliminated and the odd ones i = 2j+1 kept,
//   X_k = T(D_k^{-1}), P_k = T(X_k E_k), Q_k = T(X_k F_k),
//   D'_j = T(D_i - E_i Q_{i-1} - F_i P_{i+1}), E'_j = T(-E_i P_{i-1}),
//   F'_j = T(-F_i Q_{i+1}),
// until one block remains (its inverse is stored too).  At level 0 the E_i
// and F_i are diagonal and the products are scalings.  All blocks of one
// level are processed together by each batched launch.
// Solve: forward reduction g_k = X_k f_k, f'_j = f_i - E_i g_{i-1} - F_i g_{i+1};
// final u = X f; back-substitution u_k = X_k (f_k - E_k u_{k-1} - F_k u_{k+1}).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "hodlr.hpp"
#include "kernels.hpp"

namespace acr {

namespace {

thread_local std::string g_last_error;

struct FactorBase {
  virtual ~FactorBase() = default;
  virtual void solve(const double* B, double* X, int nrhs, hipStream_t st) = 0;
  virtual void info(acr_info* out) const = 0;
  virtual void block(int level, int which, int k, double* dense, hipStream_t st) const = 0;
};

template <typename T>
struct Level {
  int m = 0;        // blocks at this level
  int nreal = 0;    // even blocks (ceil(m/2))
  int ne = 0;       // even slots incl. a zero dummy when m is even (floor(m/2)+1)
  HSet<T> X;        // nreal inverses
  bool diag = false;
  DBuf<T> e0, f0;   // level 0: diagonals of E_i, F_i ([m][s])
  HSet<T> E, F;     // level >= 1: m HODLR blocks each
};

template <typename T>
struct Factor final : FactorBase {
  int nx = 0, ny = 0, leaf = 0, b = 0, L = 0, precision = 0;
  double eps = 0;
  std::vector<Level<T>> lev;
  HSet<T> Xlast;
  Work work_done;
  std::vector<int> lev_rank;

  size_t bytes() const {
    size_t t = Xlast.bytes();
    for (const auto& l : lev) {
      t += l.X.bytes() + l.E.bytes() + l.F.bytes() + l.e0.bytes() + l.f0.bytes();
    }
    return t;
  }

  void info(acr_info* o) const override {
    std::memset(o, 0, sizeof(*o));
    o->nx = nx; o->ny = ny; o->leaf = leaf; o->depth = L; o->levels = (int)lev.size();
    o->precision = precision; o->eps = eps;
    o->factor_bytes = (int64_t)bytes();
    int mr = Xlast.max_rank();
    for (size_t i = 0; i < lev.size() && i < 40; ++i) {
      o->level_max_rank[i] = lev_rank[i];
      mr = std::max(mr, lev_rank[i]);
    }
    o->max_rank = mr;
    o->factor_flops = work_done.total();
    // one solve pass reads every stored X twice (forward and back) and every
    // stored E/F once
    double sb = 2.0 * Xlast.bytes();
    double fl = 0;
    for (const auto& l : lev) {
      sb += 2.0 * l.X.bytes() + l.E.bytes() + l.F.bytes() + l.e0.bytes() + l.f0.bytes();
    }
    o->solve_bytes = sb;
    // two flops per stored multiply-add entry read
    fl = 2.0 * sb / sizeof(T);
    o->solve_flops_per_rhs = fl;
  }

  void block(int level, int which, int k, double* dense, hipStream_t st) const override {
    const int s = nx;
    if (level == (int)lev.size()) {
      if (which != 0 || k != 0) fail(ACR_ERR_INVALID_ARG, "last level holds only X_0");
      densify_to_host(st, Xlast, 0, dense);
      return;
    }
    if (level < 0 || level > (int)lev.size()) fail(ACR_ERR_INVALID_ARG, "level out of range");
    const Level<T>& l = lev[level];
    if (which == 0) {
      if (k < 0 || k >= l.m || (k & 1)) fail(ACR_ERR_INVALID_ARG, "X_k needs an even k < m");
      densify_to_host(st, l.X, k / 2, dense);
      return;
    }
    if (which != 1 && which != 2) fail(ACR_ERR_INVALID_ARG, "which must be 0, 1 or 2");
    if (k < 0 || k >= l.m) fail(ACR_ERR_INVALID_ARG, "block index out of range");
    if (l.diag) {
      std::vector<T> d(s);
      const DBuf<T>& src = which == 1 ? l.e0 : l.f0;
      read_to_host(d.data(), src.get() + (size_t)k * s, s * sizeof(T), st);
      for (size_t e = 0; e < (size_t)s * s; ++e) dense[e] = 0.0;
      for (int r = 0; r < s; ++r) dense[(size_t)r * (s + 1)] = (double)d[r];
    } else {
      densify_to_host(st, which == 1 ? l.E : l.F, k, dense);
    }
  }

  void solve(const double* B, double* Xout, int nrhs, hipStream_t st) override;
  void solve_fused(const double* B, double* Xout, int nrhs, hipStream_t st);
  void solve_gemm(const double* B, double* Xout, int nrhs, hipStream_t st);
  bool fused_ok(int nrhs) const;
};

template <typename T>
Flat<T> vflat(T* p, int s, int nrhs, int mmul = 1, int moff = 0) {
  Flat<T> f;
  f.p = p; f.ld = s; f.sm = (long long)s * nrhs; f.mmul = mmul; f.moff = moff;
  return f;
}

template <typename T>
MVTerm mv_hodlr(const HSet<T>& H, int mmul, int moff, const T* y, int ymul, int yoff, double alpha) {
  MVTerm M;
  M.type = 0;
  M.mmul = mmul; M.moff = moff; M.ymul = ymul; M.yoff = yoff; M.alpha = alpha; M.y = y;
  M.lv = H.lv.get();
  for (int d = 1; d <= H.L; ++d) {
    M.U[d] = H.U[d].get(); M.V[d] = H.V[d].get(); M.k[d] = H.k[d]; M.kc[d] = H.kc[d];
  }
  return M;
}

template <typename T>
MVTerm mv_diag(const T* dg, int mmul, int moff, const T* y, int ymul, int yoff, double alpha) {
  MVTerm M;
  M.type = 1;
  M.mmul = mmul; M.moff = moff; M.ymul = ymul; M.yoff = yoff; M.alpha = alpha; M.y = y; M.lv = dg;
  return M;
}

template <typename T>
MVJob mv_job(int nmat, T* out, int omul, int ooff, int term0, int nterm, const T* C0 = nullptr, int cmul = 1,
             int coff = 0, double beta = 1.0) {
  MVJob J;
  J.nmat = nmat; J.out = out; J.omul = omul; J.ooff = ooff; J.term0 = term0; J.nterm = nterm;
  J.C0 = C0; J.cmul = cmul; J.coff = coff; J.beta = beta;
  return J;
}

template <typename T>
bool Factor<T>::fused_ok(int nrhs) const {
  return nrhs <= 8 && L <= kMvMaxDepth;
}

template <typename T>
void Factor<T>::solve(const double* B, double* Xout, int nrhs, hipStream_t st) {
  if (fused_ok(nrhs)) solve_fused(B, Xout, nrhs, st);
  else solve_gemm(B, Xout, nrhs, st);
}

// Few right-hand sides: every step of a level is one multi-term matvec.
// U[l] holds the level-l unknowns with one zero pad block at each end.
template <typename T>
void Factor<T>::solve_fused(const double* B, double* Xout, int nrhs, hipStream_t st) {
  const int s = nx;
  const int nl = (int)lev.size();
  const size_t blk = (size_t)s * nrhs;
  std::vector<DBuf<T>> F(nl + 1), G(nl), U(nl + 1);
  F[0].resize((size_t)ny * blk);
  to_blocks<T>(st, s, ny, nrhs, B, (long long)nx * ny, F[0].get());
  for (int l = 0; l < nl; ++l) {
    PhaseScope ph("solve forward", l);
    const Level<T>& Lv = lev[l];
    const int m = Lv.m, nodd = m / 2;
    G[l].resize((size_t)Lv.ne * blk);
    {  // g_k = X_k f_(2k); the dummy slot (m even) is zero
      std::vector<MVTerm> tm{mv_hodlr<T>(Lv.X, 1, 0, F[l].get(), 2, 0, 1.0)};
      std::vector<MVJob> jb{mv_job<T>(Lv.nreal, G[l].get(), 1, 0, 0, 1),
                            mv_job<T>(Lv.ne - Lv.nreal, G[l].get(), 1, Lv.nreal, 0, 0)};
      ghmv<T>(st, s, b, L, nrhs, jb, tm);
    }
    F[l + 1].resize((size_t)nodd * blk);
    if (nodd > 0) {  // f'_j = f_(2j+1) - E_(2j+1) g_j - F_(2j+1) g_(j+1)
      std::vector<MVTerm> tm;
      if (Lv.diag) {
        tm.push_back(mv_diag<T>(Lv.e0.get(), 2, 1, G[l].get(), 1, 0, -1.0));
        tm.push_back(mv_diag<T>(Lv.f0.get(), 2, 1, G[l].get(), 1, 1, -1.0));
      } else {
        tm.push_back(mv_hodlr<T>(Lv.E, 2, 1, G[l].get(), 1, 0, -1.0));
        tm.push_back(mv_hodlr<T>(Lv.F, 2, 1, G[l].get(), 1, 1, -1.0));
      }
      std::vector<MVJob> jb{mv_job<T>(nodd, F[l + 1].get(), 1, 0, 0, 2, F[l].get(), 2, 1, 1.0)};
      ghmv<T>(st, s, b, L, nrhs, jb, tm);
    }
  }
  U[nl].resize(3 * blk);
  {
    std::vector<MVTerm> tm{mv_hodlr<T>(Xlast, 1, 0, F[nl].get(), 1, 0, 1.0)};
    std::vector<MVJob> jb{mv_job<T>(1, U[nl].get(), 1, 1, 0, 1), mv_job<T>(2, U[nl].get(), 2, 0, 0, 0)};
    ghmv<T>(st, s, b, L, nrhs, jb, tm);
  }
  for (int l = nl - 1; l >= 0; --l) {
    PhaseScope ph("solve backward", l);
    const Level<T>& Lv = lev[l];
    const int m = Lv.m, nodd = m / 2;
    U[l].resize((size_t)(m + 2) * blk);
    DBuf<T> tmp((size_t)Lv.nreal * blk);
    {  // tmp_k = E_(2k) u_(2k-1) + F_(2k) u_(2k+1): level-(l+1) unknowns k-1 and k (padded k, k+1)
      std::vector<MVTerm> tm;
      if (Lv.diag) {
        tm.push_back(mv_diag<T>(Lv.e0.get(), 2, 0, U[l + 1].get(), 1, 0, 1.0));
        tm.push_back(mv_diag<T>(Lv.f0.get(), 2, 0, U[l + 1].get(), 1, 1, 1.0));
      } else {
        tm.push_back(mv_hodlr<T>(Lv.E, 2, 0, U[l + 1].get(), 1, 0, 1.0));
        tm.push_back(mv_hodlr<T>(Lv.F, 2, 0, U[l + 1].get(), 1, 1, 1.0));
      }
      std::vector<MVJob> jb{mv_job<T>(Lv.nreal, tmp.get(), 1, 0, 0, 2)};
      ghmv<T>(st, s, b, L, nrhs, jb, tm);
    }
    {  // u_(2k) = g_k - X_k tmp_k; odd unknowns from level l+1; zero pads
      std::vector<MVTerm> tm{mv_hodlr<T>(Lv.X, 1, 0, tmp.get(), 1, 0, -1.0)};
      std::vector<MVJob> jb{mv_job<T>(Lv.nreal, U[l].get(), 2, 1, 0, 1, G[l].get(), 1, 0, 1.0),
                            mv_job<T>(nodd, U[l].get(), 2, 2, 0, 0, U[l + 1].get(), 1, 1, 1.0),
                            mv_job<T>(1, U[l].get(), 1, 0, 0, 0),
                            mv_job<T>(1, U[l].get(), 1, m + 1, 0, 0)};
      ghmv<T>(st, s, b, L, nrhs, jb, tm);
    }
  }
  from_blocks<T>(st, s, ny, nrhs, U[0].get() + blk, Xout, (long long)nx * ny);
}

template <typename T>
void Factor<T>::solve_gemm(const double* B, double* Xout, int nrhs, hipStream_t st) {
  const int s = nx;
  const int nl = (int)lev.size();
  const size_t blk = (size_t)s * nrhs;
  std::vector<DBuf<T>> F(nl + 1), G(nl), U(nl + 1);
  F[0].resize((size_t)ny * blk);
  to_blocks<T>(st, s, ny, nrhs, B, (long long)nx * ny, F[0].get());
  for (int l = 0; l < nl; ++l) {
    const Level<T>& L_ = lev[l];
    const int m = L_.m, nodd = m / 2;
    G[l].resize((size_t)L_.ne * blk);
    // g_k = X_k f_(2k)
    hmul<T>(st, HV<T>{&L_.X, 1, 0}, L_.nreal, 0, false, nrhs, T(1), vflat(F[l].get(), s, nrhs, 2, 0),
            T(0), vflat(G[l].get(), s, nrhs));
    if (L_.ne > L_.nreal) fill<T>(st, G[l].get() + (size_t)L_.nreal * blk, blk, T(0));
    // f'_j = f_(2j+1) - E_(2j+1) g_j - F_(2j+1) g_(j+1)
    F[l + 1].resize((size_t)nodd * blk);
    bcopy<T>(st, (int)blk, 1, nodd, T(1), with_map(bop(F[l].get(), 1, (long long)blk), 2, 1),
             bop(F[l + 1].get(), 1, (long long)blk));
    if (L_.diag) {
      bdiag_axpy<T>(st, s, nrhs, nodd, T(-1), L_.e0.get(), 2, 1, G[l].get(), 1, 0, F[l + 1].get(), 1, 0);
      bdiag_axpy<T>(st, s, nrhs, nodd, T(-1), L_.f0.get(), 2, 1, G[l].get(), 1, 1, F[l + 1].get(), 1, 0);
    } else {
      hmul<T>(st, HV<T>{&L_.E, 2, 1}, nodd, 0, false, nrhs, T(-1), vflat(G[l].get(), s, nrhs, 1, 0), T(1),
              vflat(F[l + 1].get(), s, nrhs));
      hmul<T>(st, HV<T>{&L_.F, 2, 1}, nodd, 0, false, nrhs, T(-1), vflat(G[l].get(), s, nrhs, 1, 1), T(1),
              vflat(F[l + 1].get(), s, nrhs));
    }
  }
  // final block; U[l] holds level-l unknowns with one zero pad block at each end
  U[nl].resize(3 * blk);
  fill<T>(st, U[nl].get(), 3 * blk, T(0));
  hmul<T>(st, HV<T>{&Xlast, 1, 0}, 1, 0, false, nrhs, T(1), vflat(F[nl].get(), s, nrhs), T(0),
          vflat(U[nl].get() + blk, s, nrhs));
  for (int l = nl - 1; l >= 0; --l) {
    const Level<T>& L_ = lev[l];
    const int m = L_.m, nodd = m / 2;
    U[l].resize((size_t)(m + 2) * blk);
    fill<T>(st, U[l].get(), blk, T(0));
    fill<T>(st, U[l].get() + (size_t)(m + 1) * blk, blk, T(0));
    bcopy<T>(st, (int)blk, 1, nodd, T(1), with_map(bop(U[l + 1].get(), 1, (long long)blk), 1, 1),
             with_map(bop(U[l].get(), 1, (long long)blk), 2, 2));
    DBuf<T> tmp((size_t)L_.nreal * blk);
    // tmp_k = E_(2k) u_(2k-1) + F_(2k) u_(2k+1)   (padded indices 2k and 2k+2)
    if (L_.diag) {
      fill<T>(st, tmp.get(), tmp.size(), T(0));
      bdiag_axpy<T>(st, s, nrhs, L_.nreal, T(1), L_.e0.get(), 2, 0, U[l].get(), 2, 0, tmp.get(), 1, 0);
      bdiag_axpy<T>(st, s, nrhs, L_.nreal, T(1), L_.f0.get(), 2, 0, U[l].get(), 2, 2, tmp.get(), 1, 0);
    } else {
      hmul<T>(st, HV<T>{&L_.E, 2, 0}, L_.nreal, 0, false, nrhs, T(1), vflat(U[l].get(), s, nrhs, 2, 0), T(0),
              vflat(tmp.get(), s, nrhs));
      hmul<T>(st, HV<T>{&L_.F, 2, 0}, L_.nreal, 0, false, nrhs, T(1), vflat(U[l].get(), s, nrhs, 2, 2), T(1),
              vflat(tmp.get(), s, nrhs));
    }
    // u_(2k) = g_k - X_k tmp_k   (padded index 2k+1)
    bcopy<T>(st, (int)blk, 1, L_.nreal, T(1), bop(G[l].get(), 1, (long long)blk),
             with_map(bop(U[l].get(), 1, (long long)blk), 2, 1));
    hmul<T>(st, HV<T>{&L_.X, 1, 0}, L_.nreal, 0, false, nrhs, T(-1), vflat(tmp.get(), s, nrhs), T(1),
            vflat(U[l].get(), s, nrhs, 2, 1));
  }
  from_blocks<T>(st, s, ny, nrhs, U[0].get() + blk, Xout, (long long)nx * ny);
}

int hodlr_depth(int s, int leaf) {
  int L = 0;
  while (s > leaf) {
    if (s & 1) return -1;
    s >>= 1;
    ++L;
  }
  return L;
}

// Opt-in stage checks (environment ACR_DEBUG_CHECKS=1): after each stage of
// the factorisation, synchronise and fail with the stage name if a pivot was
// bad or a stored value is not finite.
bool debug_checks() {
  static const bool on = [] {
    const char* e = std::getenv("ACR_DEBUG_CHECKS");
    return e && e[0] == '1';
  }();
  return on;
}

template <typename T>
void stage_check(hipStream_t st, const HSet<T>& H, const int* status, const char* what, int level) {
  if (!debug_checks()) return;
  int bad = 0;
  read_to_host(&bad, status, sizeof(int), st);
  std::string msg;
  bool nf = false;
  double mx = 0, m1 = 0;
  scan_values<T>(st, (long long)H.cnt * H.leaf_stride(), H.lv.get(), &nf, &m1);
  if (nf) msg += " leaves";
  mx = m1;
  for (int d = 1; d <= H.L; ++d) {
    bool b1 = false, b2 = false;
    double a1 = 0, a2 = 0;
    scan_values<T>(st, (long long)H.cnt * H.k[d] * H.s, H.U[d].get(), &b1, &a1);
    scan_values<T>(st, (long long)H.cnt * H.k[d] * H.s, H.V[d].get(), &b2, &a2);
    if (b1) msg += " U" + std::to_string(d);
    if (b2) msg += " V" + std::to_string(d);
    mx = std::max(mx, std::max(a1, a2));
  }
  std::fprintf(stderr, "[acr check] level %d %-10s cnt %d ranks", level, what, H.cnt);
  for (int d = 1; d <= H.L; ++d) std::fprintf(stderr, " %d", H.kc[d]);
  std::fprintf(stderr, " max|.| %.3e%s%s\n", mx, bad ? " BAD-PIVOT" : "", msg.empty() ? "" : (" NONFINITE:" + msg).c_str());
  if (bad || !msg.empty())
    fail(bad ? ACR_ERR_SINGULAR : ACR_ERR_INTERNAL,
         std::string("stage check failed at level ") + std::to_string(level) + " " + what + msg);
}

template <typename T>
std::unique_ptr<FactorBase> factor_impl(const acr_operator& op, const acr_options& opt, hipStream_t st) {
  auto f = std::make_unique<Factor<T>>();
  const int s = op.nx, ny = op.ny;
  f->nx = s; f->ny = ny; f->leaf = opt.leaf; f->eps = opt.eps; f->precision = opt.precision;
  const int L = hodlr_depth(s, opt.leaf);
  f->L = L;
  const int b = s >> L;
  f->b = b;
  const double eps = opt.eps;
  const double ieps = opt.inner_eps;
  const int mr = opt.max_rank;
  work() = Work();
  DBuf<int> status(1);
  memset_async(status.get(), 0, sizeof(int), st);
  {
    DBuf<int> nonfin(1);
    memset_async(nonfin.get(), 0, sizeof(int), st);
    const long long n = (long long)s * ny;
    for (const double* a : {op.diag, op.west, op.east, op.south, op.north}) flag_nonfinite(st, n, a, nonfin.get());
    int bad = 0;
    read_to_host(&bad, nonfin.get(), sizeof(int), st);
    if (bad) fail(ACR_ERR_INVALID_ARG, "the operator holds a NaN or infinite coefficient");
  }

  // level-0 operator: D_i as exact rank-1 HODLR, E_i/F_i diagonal
  HSet<T> D;
  {
    std::vector<int> k1(L + 1, 1);
    D.alloc(st, ny, s, b, L, k1, false);
    build_leaves_tridiag<T>(st, s, b, ny, 1, 0, op.diag, op.west, op.east, D.lv.get());
    for (int d = 1; d <= L; ++d) {
      build_rank1_factors<T>(st, s, s >> d, ny, 1, 0, op.west, op.east, D.U[d].get(), D.V[d].get());
      D.kc[d] = 1;
    }
  }
  HSet<T> E, F;
  DBuf<T> e0((size_t)ny * s), f0((size_t)ny * s);
  gather_diag<T>(st, s, ny, 1, 0, op.south, e0.get());
  gather_diag<T>(st, s, ny, 1, 0, op.north, f0.get());
  // E_0 and F_(ny-1) are outside the grid: exact zeros
  fill<T>(st, e0.get(), s, T(0));
  fill<T>(st, f0.get() + (size_t)(ny - 1) * s, s, T(0));

  int m = ny;
  bool diag = true;
  while (m > 1) {
    Level<T> lv;
    lv.m = m;
    lv.nreal = (m + 1) / 2;
    lv.ne = m / 2 + 1;
    lv.diag = diag;
    const int nodd = m / 2;
    PhaseScope lvl("level", (int)f->lev.size());
    // X_k = T(D_k^{-1}) for even k
    stage_check(st, D, status.get(), "D", (int)f->lev.size());
    bool closed = false;   // level 0: D_k tridiagonal, its inverse in closed form (exact rank 1)
    {
      PhaseScope ph("inverse");
      if (diag && s <= 3072) {
        std::vector<int> k1(L + 1, 1);
        lv.X.alloc(st, lv.nreal, s, b, L, k1, false);
        TriInvOut to;
        for (int d = 1; d <= L; ++d) {
          to.U[d] = lv.X.U[d].get();
          to.V[d] = lv.X.V[d].get();
          lv.X.kc[d] = 1;
        }
        DBuf<int> fb(1);
        memset_async(fb.get(), 0, sizeof(int), st);
        tridiag_inverse<T>(st, s, b, L, lv.nreal, 2, 0, op.diag, op.west, op.east, lv.X.lv.get(), to, fb.get());
        int fbh = 0;
        read_to_host(&fbh, fb.get(), sizeof(int), st);
        closed = fbh == 0;
      }
      if (!closed) hinv<T>(st, lv.X, HV<T>{&D, 2, 0}, lv.nreal, status.get());
    }
    stage_check(st, lv.X, status.get(), "inv", (int)f->lev.size());
    if (!closed) {   // the closed form is exact with rank-one blocks: T_eps leaves it unchanged
      PhaseScope ph("recompress X");
      recompress_multi<T>(st, {&lv.X}, eps, mr);
    }
    stage_check(st, lv.X, status.get(), "X", (int)f->lev.size());
    HSet<T> P, Q;
    HSet<T> Dn, En, Fn;
    if (diag) {
      // P_k = X_k diag(e_2k), Q_k = X_k diag(f_2k)
      std::vector<ColScale<T>> cs(2);
      cs[0].C = &P; cs[0].cnt_alloc = lv.ne; cs[0].nmat = lv.nreal; cs[0].H = HV<T>{&lv.X, 1, 0};
      cs[0].cols = e0.get(); cs[0].cmul = 2; cs[0].coff = 0;
      cs[1] = cs[0];
      cs[1].C = &Q; cs[1].cols = f0.get();
      {
        PhaseScope ph("products P,Q");
        hscale_cols_multi<T>(st, cs);
      }
      {
        PhaseScope ph("recompress P,Q");
        recompress_multi<T>(st, {&P, &Q}, eps, mr);
      }
      PhaseScope ph("products D',E',F'");
      // D'_j = D_i - diag(e_i) Q_j - diag(f_i) P_(j+1);  E'_j = -diag(e_i) P_j;  F'_j = -diag(f_i) Q_(j+1)
      std::vector<ScaleTerm<T>> terms(3);
      terms[0].h = HV<T>{&D, 2, 1};
      terms[1].h = HV<T>{&Q, 1, 0}; terms[1].coef = -1.0; terms[1].rows = e0.get(); terms[1].rmul = 2; terms[1].roff = 1;
      terms[2].h = HV<T>{&P, 1, 1}; terms[2].coef = -1.0; terms[2].rows = f0.get(); terms[2].rmul = 2; terms[2].roff = 1;
      hstack<T>(st, Dn, nodd, terms, nodd);
      std::vector<ScaleTerm<T>> te(1), tf(1);
      te[0].h = HV<T>{&P, 1, 0}; te[0].coef = -1.0; te[0].rows = e0.get(); te[0].rmul = 2; te[0].roff = 1;
      tf[0].h = HV<T>{&Q, 1, 1}; tf[0].coef = -1.0; tf[0].rows = f0.get(); tf[0].rmul = 2; tf[0].roff = 1;
      hstack<T>(st, En, nodd, te, nodd);
      hstack<T>(st, Fn, nodd, tf, nodd);
      lv.e0 = std::move(e0);
      lv.f0 = std::move(f0);
    } else {
      // P_k = X_k E_2k, Q_k = X_k F_2k
      std::vector<POut<T>> pq(2);
      pq[0].C = &P; pq[0].cnt_alloc = lv.ne; pq[0].nmat = lv.nreal;
      pq[0].terms = {PTerm<T>{1.0, HV<T>{&lv.X, 1, 0}, HV<T>{&E, 2, 0}}};
      pq[1].C = &Q; pq[1].cnt_alloc = lv.ne; pq[1].nmat = lv.nreal;
      pq[1].terms = {PTerm<T>{1.0, HV<T>{&lv.X, 1, 0}, HV<T>{&F, 2, 0}}};
      {
        PhaseScope ph("products P,Q");
        hprod_multi<T>(st, pq);
      }
      {
        PhaseScope ph("recompress P,Q");
        recompress_multi<T>(st, {&P, &Q}, eps, mr);
      }
      PhaseScope ph("products D',E',F'");
      std::vector<POut<T>> up(3);
      up[1].C = &En; up[1].cnt_alloc = nodd; up[1].nmat = nodd;
      up[1].terms = {PTerm<T>{-1.0, HV<T>{&E, 2, 1}, HV<T>{&P, 1, 0}}};
      up[2].C = &Fn; up[2].cnt_alloc = nodd; up[2].nmat = nodd;
      up[2].terms = {PTerm<T>{-1.0, HV<T>{&F, 2, 1}, HV<T>{&Q, 1, 1}}};
      HSet<T> EQ, FP;
      if (ieps > 0) {
        // intermediate truncation of the two Schur products, then the sum
        up[0].C = &EQ; up[0].cnt_alloc = nodd; up[0].nmat = nodd;
        up[0].terms = {PTerm<T>{1.0, HV<T>{&E, 2, 1}, HV<T>{&Q, 1, 0}}};
        up.push_back(POut<T>());
        up[3].C = &FP; up[3].cnt_alloc = nodd; up[3].nmat = nodd;
        up[3].terms = {PTerm<T>{1.0, HV<T>{&F, 2, 1}, HV<T>{&P, 1, 1}}};
        hprod_multi<T>(st, up);
        PhaseScope ph2("recompress EQ,FP");
        recompress_multi<T>(st, {&EQ, &FP}, ieps, 0);
        std::vector<ScaleTerm<T>> terms(3);
        terms[0].h = HV<T>{&D, 2, 1};
        terms[1].h = HV<T>{&EQ, 1, 0}; terms[1].coef = -1.0;
        terms[2].h = HV<T>{&FP, 1, 0}; terms[2].coef = -1.0;
        hstack<T>(st, Dn, nodd, terms, nodd);
      } else {
        // D'_j = D_i - E_i Q_j - F_i P_(j+1), accumulated exactly, one truncation
        up[0].C = &Dn; up[0].cnt_alloc = nodd; up[0].nmat = nodd;
        up[0].has_d = true; up[0].D = HV<T>{&D, 2, 1};
        up[0].terms = {PTerm<T>{-1.0, HV<T>{&E, 2, 1}, HV<T>{&Q, 1, 0}},
                       PTerm<T>{-1.0, HV<T>{&F, 2, 1}, HV<T>{&P, 1, 1}}};
        hprod_multi<T>(st, up);
      }
      lv.E = std::move(E);
      lv.F = std::move(F);
    }
    stage_check(st, P, status.get(), "P", (int)f->lev.size());
    stage_check(st, Q, status.get(), "Q", (int)f->lev.size());
    stage_check(st, Dn, status.get(), "D'-exact", (int)f->lev.size());
    {
      PhaseScope ph("recompress D',E',F'");
      recompress_multi<T>(st, {&Dn, &En, &Fn}, eps, mr);
    }
    stage_check(st, Dn, status.get(), "D'", (int)f->lev.size());
    stage_check(st, En, status.get(), "E'", (int)f->lev.size());
    stage_check(st, Fn, status.get(), "F'", (int)f->lev.size());
    int r = lv.X.max_rank();
    r = std::max(r, lv.E.max_rank());
    r = std::max(r, lv.F.max_rank());
    f->lev_rank.push_back(r);
    f->lev.push_back(std::move(lv));
    D = std::move(Dn);
    E = std::move(En);
    F = std::move(Fn);
    m = nodd;
    diag = false;
  }
  {
    PhaseScope ph("last inverse", (int)f->lev.size());
    hinv<T>(st, f->Xlast, HV<T>{&D, 1, 0}, 1, status.get());
    recompress_multi<T>(st, {&f->Xlast}, eps, mr);
  }
  int bad = 0;
  read_to_host(&bad, status.get(), sizeof(int), st);
  if (bad) fail(ACR_ERR_SINGULAR, "zero or non-finite pivot in a dense leaf or capacitance inverse");
  f->work_done = work();
  return f;
}

}  // namespace
}  // namespace acr

struct acr_handle_s {
  std::unique_ptr<acr::FactorBase> f;
  int precision = 0;
  int nx = 0, ny = 0;
};

using namespace acr;

namespace {

acr_status guard(const std::function<void()>& fn) {
  try {
    g_last_error.clear();
    fn();
    Queue::get().flush();   // everything recorded by this call is on the caller's stream now
    return ACR_OK;
  } catch (const Error& e) {
    Queue::get().discard();
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc& e) {
    Queue::get().discard();
    g_last_error = "host allocation failed";
    return ACR_ERR_OOM;
  } catch (const std::exception& e) {
    Queue::get().discard();
    g_last_error = e.what();
    return ACR_ERR_INTERNAL;
  }
}

void check_op(const acr_operator* op) {
  if (!op) fail(ACR_ERR_INVALID_ARG, "operator is NULL");
  if (op->nx < 1 || op->ny < 1) fail(ACR_ERR_INVALID_ARG, "nx and ny must be >= 1");
  if ((long long)op->nx * op->ny > (1LL << 31)) fail(ACR_ERR_INVALID_ARG, "N too large");
  if (!op->diag || !op->west || !op->east || !op->south || !op->north)
    fail(ACR_ERR_INVALID_ARG, "a stencil array is NULL");
}

}  // namespace

extern "C" {

acr_status acr_factor(const acr_operator* op, const acr_options* opt, void* stream, acr_handle* out) {
  return guard([&] {
    check_op(op);
    if (!opt || !out) fail(ACR_ERR_INVALID_ARG, "options or output handle is NULL");
    if (opt->leaf < 1 || opt->leaf > 128) fail(ACR_ERR_INVALID_ARG, "leaf must be in 1..128");
    if (!(opt->eps >= 0.0) || !std::isfinite(opt->eps)) fail(ACR_ERR_INVALID_ARG, "eps must be finite and >= 0");
    if (!(opt->inner_eps >= 0.0)) fail(ACR_ERR_INVALID_ARG, "inner_eps must be >= 0");
    if (opt->precision != ACR_FP64 && opt->precision != ACR_MIXED_FP32)
      fail(ACR_ERR_INVALID_ARG, "unknown precision");
    if (opt->max_rank < 0) fail(ACR_ERR_INVALID_ARG, "max_rank must be >= 0");
    if (hodlr_depth(op->nx, opt->leaf) < 0)
      fail(ACR_ERR_INVALID_ARG, "block size must be leaf' * 2^L (halving exact down to the leaf)");
    hipStream_t st = static_cast<hipStream_t>(stream);
    auto h = std::make_unique<acr_handle_s>();
    h->precision = opt->precision;
    h->nx = op->nx; h->ny = op->ny;
    if (opt->precision == ACR_FP64) h->f = factor_impl<double>(*op, *opt, st);
    else h->f = factor_impl<float>(*op, *opt, st);
    *out = h.release();
  });
}

acr_status acr_solve(acr_handle h, const double* B, double* X, int32_t nrhs, void* stream) {
  return guard([&] {
    if (!h || !B || !X) fail(ACR_ERR_INVALID_ARG, "NULL argument");
    if (nrhs < 1) fail(ACR_ERR_INVALID_ARG, "nrhs must be >= 1");
    h->f->solve(B, X, nrhs, static_cast<hipStream_t>(stream));
  });
}

acr_status acr_residual(const acr_operator* op, const double* X, const double* B, double* R,
                        int32_t nrhs, void* stream) {
  return guard([&] {
    check_op(op);
    if (!X || !B || !R || nrhs < 1) fail(ACR_ERR_INVALID_ARG, "bad vector arguments");
    stencil_residual(static_cast<hipStream_t>(stream), op->nx, op->ny, nrhs, op->diag, op->west, op->east,
                     op->south, op->north, X, B, R);
  });
}

acr_status acr_solve_refined(acr_handle h, const acr_operator* op, const double* B, double* X,
                             int32_t nrhs, double tol, int32_t maxit, int32_t* iters, double* relres,
                             void* stream) {
  int its = 0;
  double rel = INFINITY;
  acr_status st0 = guard([&] {
    check_op(op);
    if (!h || !B || !X || nrhs < 1 || maxit < 0) fail(ACR_ERR_INVALID_ARG, "bad arguments");
    if (op->nx != h->nx || op->ny != h->ny) fail(ACR_ERR_INVALID_ARG, "operator shape differs from the factor");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const long long n = (long long)op->nx * op->ny;
    DBuf<double> R((size_t)n * nrhs), D((size_t)n * nrhs), nb(nrhs), nr(nrhs);
    std::vector<double> hb(nrhs), hr(nrhs);
    col_sumsq(st, n, nrhs, B, nb.get());
    memset_async(X, 0, (size_t)n * nrhs * sizeof(double), st);
    copy_d2d_async(R.get(), B, (size_t)n * nrhs * sizeof(double), st);
    read_to_host(hb.data(), nb.get(), nrhs * sizeof(double), st);
    for (its = 0;; ++its) {
      if (its > 0) {
        stencil_residual(st, op->nx, op->ny, nrhs, op->diag, op->west, op->east, op->south, op->north, X, B,
                         R.get());
      }
      col_sumsq(st, n, nrhs, R.get(), nr.get());
      read_to_host(hr.data(), nr.get(), nrhs * sizeof(double), st);
      rel = 0.0;
      for (int q = 0; q < nrhs; ++q) {
        const double v = hb[q] > 0 ? std::sqrt(hr[q] / hb[q]) : std::sqrt(hr[q]);
        rel = std::max(rel, v);
      }
      if (!(rel > tol) || its >= maxit || !std::isfinite(rel)) break;
      h->f->solve(R.get(), D.get(), nrhs, st);
      axpy_d(st, n * nrhs, D.get(), X);
    }
    if (!(rel <= tol)) fail(ACR_ERR_NOT_CONVERGED, "refinement stopped at relative residual " + std::to_string(rel));
  });
  if (iters) *iters = its;
  if (relres) *relres = rel;
  return st0;
}

acr_status acr_solve_krylov(acr_handle h, const acr_operator* op, const double* B, double* X, int32_t nrhs,
                            double tol, int32_t maxit, int32_t restart, int32_t* iters, double* relres,
                            void* stream) {
  int its_all = 0;
  double rel_all = 0.0;
  acr_status st0 = guard([&] {
    check_op(op);
    if (!h || !B || !X || nrhs < 1 || maxit < 0) fail(ACR_ERR_INVALID_ARG, "bad arguments");
    if (restart < 1 || restart > 64) fail(ACR_ERR_INVALID_ARG, "restart must be in 1..64");
    if (X == B) fail(ACR_ERR_INVALID_ARG, "X must not alias B");
    if (op->nx != h->nx || op->ny != h->ny) fail(ACR_ERR_INVALID_ARG, "operator shape differs from the factor");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const long long n = (long long)op->nx * op->ny;
    const int m = restart;
    DBuf<double> V((size_t)(m + 1) * n), Z((size_t)m * n), R(n), zero(n), dv(2 * (m + 1) + 1);
    memset_async(zero.get(), 0, (size_t)n * sizeof(double), st);
    std::vector<double> hv(2 * (m + 1) + 1);
    auto norm2 = [&](const double* v) {
      col_sumsq(st, n, 1, v, dv.get());
      double r = 0.0;
      read_to_host(&r, dv.get(), sizeof(double), st);
      return std::sqrt(r);
    };
    auto Aop = [&](const double* x, const double* b, double* r) {   // r = b - A x
      stencil_residual(st, op->nx, op->ny, 1, op->diag, op->west, op->east, op->south, op->north, x, b, r);
    };
    for (int q = 0; q < nrhs; ++q) {
      const double* b = B + (size_t)q * n;
      double* x = X + (size_t)q * n;
      memset_async(x, 0, (size_t)n * sizeof(double), st);
      const double bn = norm2(b);
      int its = 0;
      double rel = 0.0;
      std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
      for (;;) {
        Aop(x, b, R.get());
        const double beta = norm2(R.get());
        rel = bn > 0.0 ? beta / bn : beta;
        if (!(rel > tol) || its >= maxit || !std::isfinite(rel)) break;
        // V_0 = r / beta
        copy_d2d_async(V.get(), R.get(), (size_t)n * sizeof(double), st);
        maxpy(st, n, 0, 1.0 / beta, 0.0, nullptr, nullptr, 0, V.get());
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;   // columns of the Hessenberg matrix built in this cycle
        for (int j = 0; j < m && its < maxit; ++j) {
          double* vj = V.get() + (size_t)j * n;
          double* zj = Z.get() + (size_t)j * n;
          double* w = V.get() + (size_t)(j + 1) * n;
          h->f->solve(vj, zj, 1, st);   // z_j = M^{-1} v_j
          ++its;
          Aop(zj, zero.get(), w);        // w = -A z_j
          // classical Gram-Schmidt twice: d = V^T w, w = -w + V d (= A z_j - V h);
          // e = V^T w, w = w - V e; h = -d + e
          mdot(st, n, j + 1, V.get(), n, w, dv.get());
          maxpy(st, n, j + 1, -1.0, 1.0, dv.get(), V.get(), n, w);
          mdot(st, n, j + 1, V.get(), n, w, dv.get() + (m + 1));
          maxpy(st, n, j + 1, 1.0, -1.0, dv.get() + (m + 1), V.get(), n, w);
          col_sumsq(st, n, 1, w, dv.get() + 2 * (m + 1));
          read_to_host(hv.data(), dv.get(), hv.size() * sizeof(double), st);
          double* hc = H.data() + (size_t)j * (m + 1);   // column j
          for (int i = 0; i <= j; ++i) hc[i] = -hv[i] + hv[m + 1 + i];
          const double hn = std::sqrt(std::max(hv[2 * (m + 1)], 0.0));
          hc[j + 1] = hn;
          for (int i = 0; i < j; ++i) {   // earlier rotations
            const double a = cs[i] * hc[i] + sn[i] * hc[i + 1];
            hc[i + 1] = -sn[i] * hc[i] + cs[i] * hc[i + 1];
            hc[i] = a;
          }
          const double den = std::hypot(hc[j], hc[j + 1]);
          cs[j] = den > 0.0 ? hc[j] / den : 1.0;
          sn[j] = den > 0.0 ? hc[j + 1] / den : 0.0;
          hc[j] = den;
          hc[j + 1] = 0.0;
          g[j + 1] = -sn[j] * g[j];
          g[j] = cs[j] * g[j];
          k = j + 1;
          if (hn > 0.0) maxpy(st, n, 0, 1.0 / hn, 0.0, nullptr, nullptr, 0, w);   // v_(j+1)
          const double est = bn > 0.0 ? std::fabs(g[j + 1]) / bn : std::fabs(g[j + 1]);
          if (!(est > tol) || !(hn > 0.0)) break;
        }
        // y = H^{-1} g (upper triangular k x k), x += Z y
        for (int i = k - 1; i >= 0; --i) {
          double v = g[i];
          for (int l = i + 1; l < k; ++l) v -= H[(size_t)l * (m + 1) + i] * y[l];
          const double d = H[(size_t)i * (m + 1) + i];
          y[i] = d != 0.0 ? v / d : 0.0;
        }
        if (k > 0) {
          const double* yd = static_cast<const double*>(DescArena::get().put(y.data(), k * sizeof(double), st));
          maxpy(st, n, k, 1.0, 1.0, yd, Z.get(), n, x);
        }
      }
      its_all = std::max(its_all, its);
      rel_all = std::max(rel_all, rel);
    }
    if (!(rel_all <= tol))
      fail(ACR_ERR_NOT_CONVERGED, "FGMRES stopped at relative residual " + std::to_string(rel_all));
  });
  if (iters) *iters = its_all;
  if (relres) *relres = rel_all;
  return st0;
}

acr_status acr_get_info(acr_handle h, acr_info* out) {
  return guard([&] {
    if (!h || !out) fail(ACR_ERR_INVALID_ARG, "NULL argument");
    h->f->info(out);
  });
}

acr_status acr_get_block(acr_handle h, int32_t level, int32_t which, int32_t k, double* dense, void* stream) {
  return guard([&] {
    if (!h || !dense) fail(ACR_ERR_INVALID_ARG, "NULL argument");
    h->f->block(level, which, k, dense, static_cast<hipStream_t>(stream));
  });
}

acr_status acr_destroy(acr_handle h) {
  return guard([&] {
    if (!h) return;
    (void)hipDeviceSynchronize();
    delete h;
  });
}

const char* acr_status_string(acr_status s) {
  switch (s) {
    case ACR_OK: return "ok";
    case ACR_ERR_INVALID_ARG: return "invalid argument";
    case ACR_ERR_OOM: return "out of device memory";
    case ACR_ERR_SINGULAR: return "singular pivot";
    case ACR_ERR_NOT_CONVERGED: return "refinement did not converge";
    case ACR_ERR_DEVICE: return "HIP runtime error";
    case ACR_ERR_INTERNAL: return "internal error";
  }
  return "unknown status";
}

const char* acr_last_error(void) { return g_last_error.c_str(); }

acr_status acr_profile_start(uint32_t class_mask) {
  return guard([&] { Profiler::get().start(class_mask); });
}

acr_status acr_profile_read(int32_t cls, int64_t* launches, double* total_ms, double* flops,
                            double* bytes) {
  return guard([&] {
    if (cls < 0 || cls >= KC_COUNT) fail(ACR_ERR_INVALID_ARG, "unknown kernel class");
    Profiler& P = Profiler::get();
    std::lock_guard<std::mutex> g(P.mu());
    int64_t n = 0;
    double ms = 0, fl = 0, by = 0;
    for (auto& r : P.recs()) {
      if (r.cls != cls) continue;
      ACR_HIP(hipEventSynchronize(r.b));
      float e = 0;
      ACR_HIP(hipEventElapsedTime(&e, r.a, r.b));
      ++n;
      ms += e;
      by += r.bytes;
      fl += r.flops;
      if (r.dev_flops) {
        std::vector<double> f(r.nprob);
        ACR_HIP(hipMemcpy(f.data(), r.dev_flops, r.nprob * sizeof(double), hipMemcpyDeviceToHost));
        for (double v : f) fl += v;
      }
      if (r.dev_sweeps) {
        std::vector<int> sw(r.nprob);
        ACR_HIP(hipMemcpy(sw.data(), r.dev_sweeps, r.nprob * sizeof(int), hipMemcpyDeviceToHost));
        const double per = 3.0 * (double)r.c * r.c * (r.c - 1);   // pair dot products per sweep
        for (int v : sw) fl += per * v;
      }
    }
    if (launches) *launches = n;
    if (total_ms) *total_ms = ms;
    if (flops) *flops = fl;
    if (bytes) *bytes = by;
  });
}

acr_status acr_profile_report(char* buf, int64_t len, int64_t* needed) {
  return guard([&] {
    Profiler& P = Profiler::get();
    std::lock_guard<std::mutex> g(P.mu());
    struct Agg { int cls = 0; int64_t n = 0; double ms = 0, flops = 0, bytes = 0; };
    std::vector<std::pair<std::string, Agg>> rows;
    std::map<std::string, size_t> index;
    auto add = [&](const std::string& key, int cls, float ms, double fl, double by) {
      auto it = index.find(key);
      if (it == index.end()) {
        index[key] = rows.size();
        rows.push_back({key, Agg()});
        it = index.find(key);
      }
      Agg& a = rows[it->second].second;
      a.cls = cls; a.n += 1; a.ms += ms; a.flops += fl; a.bytes += by;
    };
    static const char* names[KC_COUNT] = {"gemm", "inverse", "qr", "applyq", "svd", "matvec", "copy", "other"};
    for (auto& r : P.recs()) {
      ACR_HIP(hipEventSynchronize(r.b));
      float e = 0;
      ACR_HIP(hipEventElapsedTime(&e, r.a, r.b));
      double fl = r.flops;
      if (r.dev_flops) {
        std::vector<double> f(r.nprob);
        ACR_HIP(hipMemcpy(f.data(), r.dev_flops, r.nprob * sizeof(double), hipMemcpyDeviceToHost));
        for (double v : f) fl += v;
      }
      add(std::string("stage\t") + (r.phase ? r.phase : "-") + "\t" + std::to_string(r.level) + "\t" +
              names[r.cls], r.cls, e, fl, r.bytes);
      add(std::string("kernel\t") + (r.kname ? r.kname : "-") + "\t" + names[r.cls], r.cls, e, fl, r.bytes);
      add(std::string("stagekernel\t") + (r.phase ? r.phase : "-") + "\t" + (r.kname ? r.kname : "-"), r.cls, e, fl,
          r.bytes);
    }
    std::string out;
    for (auto& kv : rows) {
      char line[512];
      std::snprintf(line, sizeof line, "%s\t%lld\t%.6f\t%.6e\t%.6e\n", kv.first.c_str(),
                    (long long)kv.second.n, kv.second.ms, kv.second.flops, kv.second.bytes);
      out += line;
    }
    if (needed) *needed = (int64_t)out.size() + 1;
    if (buf && len > 0) {
      const size_t n = std::min<size_t>(out.size(), (size_t)len - 1);
      std::memcpy(buf, out.data(), n);
      buf[n] = 0;
    }
  });
}

acr_status acr_trim_pool(void) {
  return guard([&] { Pool::get().trim(); });
}

}  // extern "C"
