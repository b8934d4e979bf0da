// The stored ACR factorisation of one problem and the entry-point helpers
// shared by the library's C ABI files (acr.hip, serve.hip).
#pragma once

#include <cmath>
#include <functional>
#include <map>
#include <mutex>
#include <memory>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "hodlr.hpp"
#include "kernels.hpp"

namespace acr {

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

// The persistent solve pass of one factor for one number of right-hand
// sides: its task list in device memory (built once, read-only afterwards)
// and the layout of the workspace every pass allocates (byte offsets; the
// first 256 bytes are unused, so that no operand offset is zero).
// A matvec step run as a grouped launch (the levels before the persistent
// part): jobs and terms as for ghmv, vector operands as workspace offsets.
struct HostStep {
  int level = 0;
  std::vector<MVJob> jobs;
  std::vector<MVTerm> terms;
};
// In the deep-level persistent mode, levels with more blocks than this run
// as grouped launches and the rest of the pass (deep levels, last block,
// their back-substitution) as one persistent launch.
constexpr int kPersistBlocks = 16;
struct PPlan {
  int NR = 1, ntasks = 0, nctr = 0, l0 = 0;
  std::vector<HostStep> pre, post;   // forward steps of levels < l0; backward ones
  bool w64 = true;
  size_t ws_bytes = 0;
  long long f0_off = 0, u0_off = 0, tbuf_off = 0;   // F_0 blocks, U_0 (with its leading pad block)
  DBuf<char> dev;                                   // tasks | jobs | terms
  const PTask* tasks = nullptr;
  const MVJob* jobs = nullptr;
  const MVTerm* terms = nullptr;
  double flops = 0, bytes = 0;
};

// A grouped solve pass kept on the device for one (right-hand-side count,
// stream, host thread): the workspace of the plan's layout, a projection
// buffer for the largest step, and every step's descriptors; a pass only
// enqueues the steps' launches.
struct GPass {
  DBuf<char> ws, tb, desc;
  long long f0_off = 0, u0_off = 0;
  std::vector<HmvStep> steps;
  std::vector<const MVRed*> reds;
  std::vector<const MVTerm*> terms;
  std::vector<const MVJob*> jobs;
};

constexpr int kMaxKeptPasses = 16;   // kept solve passes per handle

template <typename T>
struct Factor final : FactorBase {
  int nx = 0, ny = 0, leaf = 0, b = 0, L = 0, precision = 0;
  double eps = 0;
  std::vector<Level<T>> lev;
  HSet<T> Xlast;
  // early stop (stop_blocks): the inverse of the remaining block-tridiagonal
  // system of mstop > 1 blocks, dense (mstop*nx)^2 column-major
  int mstop = 1;
  DBuf<T> Xd;
  Work work_done;
  std::vector<int> lev_rank;
  std::vector<double> lev_mean;
  long long launches = 0;
  int batch = 1;   // problems factored together (work and launches are of the batch)

  size_t bytes() const {
    size_t t = Xlast.bytes() + Xd.bytes();
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
    double sb = 2.0 * Xlast.bytes() + Xd.bytes();
    double fl = 0;
    for (const auto& l : lev) {
      sb += 2.0 * l.X.bytes() + l.E.bytes() + l.F.bytes() + l.e0.bytes() + l.f0.bytes();
    }
    o->solve_bytes = sb;
    // two flops per stored multiply-add entry read
    fl = 2.0 * sb / sizeof(T);
    o->solve_flops_per_rhs = fl;
    double fr = Xlast.bytes_ranked() + Xd.bytes(), sr = 2.0 * Xlast.bytes_ranked() + Xd.bytes();
    for (const auto& l : lev) {
      const double x = l.X.bytes_ranked(), ef = l.E.bytes_ranked() + l.F.bytes_ranked() + l.e0.bytes() + l.f0.bytes();
      fr += x + ef;
      sr += 2.0 * x + ef;
    }
    o->factor_bytes_ranked = fr;
    o->solve_bytes_ranked = sr;
    for (size_t i = 0; i < lev_mean.size() && i < 40; ++i) o->level_mean_rank[i] = lev_mean[i];
    o->factor_launches = launches;
    o->stop_blocks = mstop;
  }

  void block(int level, int which, int k, double* dense, hipStream_t st) const override {
    const int s = nx;
    if (level == (int)lev.size()) {
      if (mstop > 1) {   // block (k / mstop, k % mstop) of the dense remainder inverse
        if (which != 0 || k < 0 || k >= mstop * mstop) fail(ACR_ERR_INVALID_ARG, "last level: k = i*mstop + j");
        const int i = k / mstop, j = k % mstop, n = mstop * s;
        std::vector<T> h((size_t)n * s);
        read_to_host(h.data(), Xd.get() + (size_t)j * s * n, h.size() * sizeof(T), st);
        for (int c = 0; c < s; ++c)
          for (int r = 0; r < s; ++r) dense[r + (size_t)c * s] = (double)h[(size_t)i * s + r + (size_t)c * n];
        return;
      }
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

  // persistent solve plans by (right-hand sides, largest grouped-level size)
  mutable std::mutex plan_mu;
  mutable std::map<std::pair<int, int>, std::unique_ptr<PPlan>> plans;
  mutable std::map<std::tuple<int, hipStream_t, std::thread::id>, std::unique_ptr<GPass>> gpasses;
  const PPlan& plan(int nrhs, int max_blocks, hipStream_t st) const;   // max_blocks < 0: all grouped
  const PPlan& plan_locked(int nrhs, int max_blocks, hipStream_t st) const;
  const GPass& gpass(int nrhs, hipStream_t st) const;
  bool may_keep(int nrhs, hipStream_t st) const;

  void solve(const double* B, double* Xout, int nrhs, hipStream_t st) override;
  void solve_fused(const double* B, double* Xout, int nrhs, hipStream_t st);
  void solve_gemm(const double* B, double* Xout, int nrhs, hipStream_t st);
  bool fused_ok(int nrhs) const;
};

// Factor the problems ops[0..] together (see acr.hip).
// With `dense` (then ops holds one entry giving nx, ny only) the single
// problem's blocks come from the dense operator instead of a stencil.  With
// `op3` the single problem is a 3-D operator: ops[0] then holds its block
// form (nx = plane size, ny = planes, diag/west/east of the planes,
// south/north = down/up) and op3 supplies the row length and the in-plane
// y couplings.
template <typename T>
std::vector<std::unique_ptr<Factor<T>>> factor_many(const std::vector<acr_operator>& ops, const acr_options& opt,
                                                    hipStream_t st, const acr_dense_operator* dense = nullptr,
                                                    const acr_operator3d* op3 = nullptr);

// X_p = M_p^{-1} B_p for several factors with <= 8 right-hand sides each, in
// shared launches (see acr.hip).  keep: a single factor may use (and build)
// its kept grouped pass; the batched and serving callers pass false, since
// their handles and right-hand-side counts change from call to call.
template <typename T>
void solve_fused_many(const std::vector<const Factor<T>*>& fs, const std::vector<const double*>& Bs,
                      const std::vector<double*>& Xs, const std::vector<int>& nrs, hipStream_t st,
                      bool keep = false);

// max(a, b) that keeps a NaN (a NaN residual norm must stop a solver as
// not converged, never read as zero).
inline double nan_max(double a, double b) {
  if (std::isnan(a)) return a;
  if (std::isnan(b)) return b;
  return b > a ? b : a;
}

// HODLR depth of block size s for a leaf bound (-1 if the halving is not exact).
int hodlr_depth(int s, int leaf);

// Runs an entry point body: flushes its launches at the end, turns
// exceptions into status codes and the thread's last-error text.
acr_status guard(const std::function<void()>& fn);
void set_last_error(const std::string& msg);

// Argument checks shared by the entry points (ACR_ERR_INVALID_ARG).
void check_op(const acr_operator* op);
void check_op3(const acr_operator3d* op);
void check_options(const acr_options* opt);
bool overlap2(const double* a, size_t na, const double* b, size_t nb);

}  // namespace acr

struct acr_handle_s {
  std::unique_ptr<acr::FactorBase> f;
  int precision = 0;
  int nx = 0, ny = 0;
};
