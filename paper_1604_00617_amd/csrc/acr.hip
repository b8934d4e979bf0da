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
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "factor.hpp"

namespace acr {

namespace {
thread_local std::string g_last_error;
}  // namespace

void set_last_error(const std::string& msg) { g_last_error = msg; }

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
    M.kmean[d] = (float)H.rank_mean(d);
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

// Last step after an early stop: output block i (padded position i + 1) of
// U = Xd F, with F the m blocks of s x nrhs (block-major) and Xd the dense
// (m s)^2 inverse: one K-segmented GEMM job, cluster = output block, segment
// = input block.
template <typename T>
void plan_dense_last(GemmPlan& plan, const Factor<T>& f, const T* F, T* U, int nrhs) {
  const int m = f.mstop, s = f.nx, n = m * s;
  const long long blk = (long long)s * nrhs;
  if (m > kMaxSeg) fail(ACR_ERR_INVALID_ARG, "early stop keeps at most 16 blocks");
  std::vector<GSeg> sg;
  for (int j = 0; j < m; ++j) {
    GSeg g;
    g.A = bop(f.Xd.get() + (size_t)j * s * n, n, 0, s);   // rows of output block i, columns of block j
    g.B = bop(F + j * blk, s, 0, 0);
    g.K = s;
    sg.push_back(g);
  }
  plan.add(s, nrhs, 1, m, 1.0, 0.0, bop(U + blk, s, 0, blk), sg);
}

// The persistent pass of this factor for nrhs right-hand sides: the same
// matvec steps as the grouped solve below (forward reduction level by level,
// the last block, back-substitution), as one task list.  Vector operands are
// workspace offsets: F_l, G_l, U_l (with one zero pad block at each end) and
// tmp_l for every level, then the projection buffer.
template <typename T>
const PPlan& Factor<T>::plan(int nrhs, int max_blocks, hipStream_t st) const {
  std::lock_guard<std::mutex> g(plan_mu);
  return plan_locked(nrhs, max_blocks, st);
}

template <typename T>
const PPlan& Factor<T>::plan_locked(int nrhs, int max_blocks, hipStream_t st) const {
  const auto key = std::make_pair(nrhs, max_blocks);
  auto found = plans.find(key);
  if (found != plans.end()) return *found->second;
  if (mstop > 1 || !fused_ok(nrhs)) fail(ACR_ERR_INTERNAL, "persistent solve: unsupported factor");
  auto P = std::make_unique<PPlan>();
  P->NR = nrhs <= 1 ? 1 : nrhs <= 2 ? 2 : nrhs <= 4 ? 4 : 8;
  PBuilder pb(P->NR);
  const int s = nx, nl = (int)lev.size();
  const size_t blk = (size_t)s * nrhs * sizeof(T);
  size_t off = 256;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  std::vector<size_t> F(nl + 1), G(nl), U(nl + 1), Tm(nl);
  F[0] = take((size_t)ny * blk);
  for (int l = 0; l < nl; ++l) {
    F[l + 1] = take((size_t)(lev[l].m / 2) * blk);
    G[l] = take((size_t)lev[l].ne * blk);
    U[l] = take((size_t)(lev[l].m + 2) * blk);
    Tm[l] = take((size_t)lev[l].nreal * blk);
  }
  U[nl] = take(3 * blk);
  auto at = [](size_t o) { return reinterpret_cast<T*>(o); };
  auto job = [&](int nmat, size_t out, int omul, int ooff, int term0, int nterm, const T* C0 = nullptr,
                 int cmul = 1, int coff = 0) {
    MVJob J = mv_job<T>(nmat, at(out), omul, ooff, term0, nterm, C0, cmul, coff, 1.0);
    J.s = s; J.b = b; J.L = L; J.nrhs = nrhs;
    return J;
  };
  // levels with more blocks than kPersistBlocks run as grouped launches
  // before (forward) and after (backward) the persistent launch
  int l0 = 0;
  while (l0 < nl && lev[l0].m > max_blocks) ++l0;
  if (max_blocks < 0) l0 = nl + 1;   // every step grouped, the last block's too
  P->l0 = l0;
  int cur = 0;   // level of the steps being added
  bool fwd = true;
  auto add = [&](std::vector<MVJob> jb, std::vector<MVTerm> tm) {
    if (cur >= l0) {
      pb.step<T>(std::move(jb), tm);
    } else {
      (fwd ? P->pre : P->post).push_back(HostStep{cur, std::move(jb), std::move(tm)});
    }
  };
  for (int l = 0; l < nl; ++l) {
    const Level<T>& Lv = lev[l];
    cur = l;
    {  // g_k = X_k f_(2k); the dummy slot (m even) is zero
      std::vector<MVTerm> tm{mv_hodlr<T>(Lv.X, 1, 0, at(F[l]), 2, 0, 1.0)};
      add({job(Lv.nreal, G[l], 1, 0, 0, 1), job(Lv.ne - Lv.nreal, G[l], 1, Lv.nreal, 0, 0)}, tm);
    }
    const int nodd = Lv.m / 2;
    if (nodd > 0) {  // f'_j = f_(2j+1) - E_(2j+1) g_j - F_(2j+1) g_(j+1)
      std::vector<MVTerm> tm;
      if (Lv.diag) {
        tm.push_back(mv_diag<T>(Lv.e0.get(), 2, 1, at(G[l]), 1, 0, -1.0));
        tm.push_back(mv_diag<T>(Lv.f0.get(), 2, 1, at(G[l]), 1, 1, -1.0));
      } else {
        tm.push_back(mv_hodlr<T>(Lv.E, 2, 1, at(G[l]), 1, 0, -1.0));
        tm.push_back(mv_hodlr<T>(Lv.F, 2, 1, at(G[l]), 1, 1, -1.0));
      }
      add({job(nodd, F[l + 1], 1, 0, 0, 2, at(F[l]), 2, 1)}, tm);
    }
  }
  cur = nl;
  {  // u = X f on the last block; zero pads
    std::vector<MVTerm> tm{mv_hodlr<T>(Xlast, 1, 0, at(F[nl]), 1, 0, 1.0)};
    add({job(1, U[nl], 1, 1, 0, 1), job(2, U[nl], 2, 0, 0, 0)}, tm);
  }
  fwd = false;
  for (int l = nl - 1; l >= 0; --l) {
    const Level<T>& Lv = lev[l];
    const int m = Lv.m, nodd = m / 2;
    cur = l;
    {  // tmp_k = E_(2k) u_(2k-1) + F_(2k) u_(2k+1)
      std::vector<MVTerm> tm;
      if (Lv.diag) {
        tm.push_back(mv_diag<T>(Lv.e0.get(), 2, 0, at(U[l + 1]), 1, 0, 1.0));
        tm.push_back(mv_diag<T>(Lv.f0.get(), 2, 0, at(U[l + 1]), 1, 1, 1.0));
      } else {
        tm.push_back(mv_hodlr<T>(Lv.E, 2, 0, at(U[l + 1]), 1, 0, 1.0));
        tm.push_back(mv_hodlr<T>(Lv.F, 2, 0, at(U[l + 1]), 1, 1, 1.0));
      }
      add({job(Lv.nreal, Tm[l], 1, 0, 0, 2)}, tm);
    }
    {  // u_(2k) = g_k - X_k tmp_k; odd unknowns from level l+1; zero pads
      std::vector<MVTerm> tm{mv_hodlr<T>(Lv.X, 1, 0, at(Tm[l]), 1, 0, -1.0)};
      add({job(Lv.nreal, U[l], 2, 1, 0, 1, at(G[l]), 1, 0), job(nodd, U[l], 2, 2, 0, 0, at(U[l + 1]), 1, 1),
           job(1, U[l], 1, 0, 0, 0), job(1, U[l], 1, m + 1, 0, 0)},
          tm);
    }
  }
  pb.check();
  P->tbuf_off = (long long)take((size_t)pb.tsize * sizeof(T));
  P->ws_bytes = off;
  P->f0_off = (long long)F[0];
  P->u0_off = (long long)U[0];
  P->w64 = pb.w64;
  P->ntasks = (int)pb.tasks.size();
  P->nctr = pb.nctr;
  P->flops = pb.flops;
  P->bytes = pb.bytes;
  const size_t bt = pb.tasks.size() * sizeof(PTask), bj = pb.jobs.size() * sizeof(MVJob),
               bm = pb.terms.size() * sizeof(MVTerm);
  const size_t oj = (bt + 255) & ~size_t(255), om = oj + ((bj + 255) & ~size_t(255));
  std::vector<char> h(om + bm);
  std::memcpy(h.data(), pb.tasks.data(), bt);
  std::memcpy(h.data() + oj, pb.jobs.data(), bj);
  std::memcpy(h.data() + om, pb.terms.data(), bm);
  P->dev.resize(h.size());
  if (!h.empty()) {   // one upload, complete before any stream reads the plan
    Queue::get().flush();
    ACR_HIP(hipMemcpyAsync(P->dev.get(), h.data(), h.size(), hipMemcpyHostToDevice, st));
    ACR_HIP(hipStreamSynchronize(st));
    Queue::get().device_idle();
  }
  P->tasks = reinterpret_cast<const PTask*>(P->dev.get());
  P->jobs = reinterpret_cast<const MVJob*>(P->dev.get() + oj);
  P->terms = reinterpret_cast<const MVTerm*>(P->dev.get() + om);
  const PPlan& r = *P;
  plans[key] = std::move(P);
  return r;
}

// The grouped solve pass of this factor for nrhs right-hand sides on the
// calling thread and stream, with its workspace and every step's
// descriptors kept on the device: built on first use from the plan's steps
// (all grouped), then each pass only enqueues its launches.
template <typename T>
const GPass& Factor<T>::gpass(int nrhs, hipStream_t st) const {
  std::lock_guard<std::mutex> g(plan_mu);
  const auto key = std::make_tuple(nrhs, st, std::this_thread::get_id());
  auto found = gpasses.find(key);
  if (found != gpasses.end()) return *found->second;
  const PPlan& P = plan_locked(nrhs, -1, st);
  auto G = std::make_unique<GPass>();
  G->ws.resize(P.ws_bytes);
  G->f0_off = P.f0_off;
  G->u0_off = P.u0_off;
  const uintptr_t base = reinterpret_cast<uintptr_t>(G->ws.get());
  std::vector<char> blob;
  auto put = [&](const void* p, size_t n) {
    const size_t o = (blob.size() + 255) & ~size_t(255);
    blob.resize(o + n);
    if (n) std::memcpy(blob.data() + o, p, n);
    return o;
  };
  std::vector<std::array<size_t, 3>> offs;
  long long tmax = 1;
  for (const auto* list : {&P.pre, &P.post})
    for (const HostStep& hs : *list) {
      std::vector<MVTerm> tm = hs.terms;
      std::vector<MVJob> jb = hs.jobs;
      for (MVTerm& M : tm) M.y = reinterpret_cast<const void*>(base + reinterpret_cast<uintptr_t>(M.y));
      for (MVJob& J : jb) {
        J.out = reinterpret_cast<void*>(base + reinterpret_cast<uintptr_t>(J.out));
        if (J.C0) J.C0 = reinterpret_cast<const void*>(base + reinterpret_cast<uintptr_t>(J.C0));
      }
      HmvStep h = hmv_plan<T>(std::move(jb), tm);
      if (h.rows <= 0) continue;
      offs.push_back({put(h.reds.data(), h.reds.size() * sizeof(MVRed)), put(h.terms.data(), h.terms.size() * sizeof(MVTerm)),
                      put(h.jobs.data(), h.jobs.size() * sizeof(MVJob))});
      tmax = std::max(tmax, h.tsize);
      G->steps.push_back(std::move(h));
    }
  G->tb.resize((size_t)tmax * sizeof(T));
  G->desc.resize(blob.size());
  if (!blob.empty()) {   // one upload, complete before the first pass reads it
    Queue::get().flush();
    ACR_HIP(hipMemcpyAsync(G->desc.get(), blob.data(), blob.size(), hipMemcpyHostToDevice, st));
    ACR_HIP(hipStreamSynchronize(st));
    Queue::get().device_idle();
  }
  for (const auto& o : offs) {
    G->reds.push_back(reinterpret_cast<const MVRed*>(G->desc.get() + o[0]));
    G->terms.push_back(reinterpret_cast<const MVTerm*>(G->desc.get() + o[1]));
    G->jobs.push_back(reinterpret_cast<const MVJob*>(G->desc.get() + o[2]));
  }
  const GPass& r = *G;
  gpasses[key] = std::move(G);
  return r;
}

// A kept pass exists, or may still be added, for (nrhs, stream, thread):
// a handle keeps at most kMaxKeptPasses (a caller that solves on many
// streams or threads gets per-call planning beyond that).
template <typename T>
bool Factor<T>::may_keep(int nrhs, hipStream_t st) const {
  std::lock_guard<std::mutex> g(plan_mu);
  return gpasses.size() < (size_t)kMaxKeptPasses ||
         gpasses.count(std::make_tuple(nrhs, st, std::this_thread::get_id())) > 0;
}

// X = M^{-1} B by the kept grouped pass: block layout in, the steps' launches
// (no planning, no descriptor copies), block layout out.
template <typename T>
void solve_kept(const Factor<T>& f, const double* B, double* Xout, int nrhs, hipStream_t st) {
  const GPass& G = f.gpass(nrhs, st);
  VJob J;
  J.s = f.nx; J.nblk = f.ny; J.nrhs = nrhs; J.ld = (long long)f.nx * f.ny;
  J.src = B; J.dst = G.ws.get() + G.f0_off;
  gto_blocks<T>(st, {J});
  {
    PhaseScope ph("solve pass");
    T* tb = reinterpret_cast<T*>(G.tb.get());
    for (size_t i = 0; i < G.steps.size(); ++i) hmv_launch<T>(st, G.steps[i], G.reds[i], G.terms[i], G.jobs[i], tb);
  }
  J.src = G.ws.get() + G.u0_off + (long long)f.nx * nrhs * sizeof(T); J.dst = Xout;
  gfrom_blocks<T>(st, {J});
}

// X_p = M_p^{-1} B_p as one persistent launch per group of passes with the
// same projection slots and row form, after one block-layout copy in and
// before one copy out; the counters of all passes are cleared by one fill.
template <typename T>
void solve_persistent_many(const std::vector<const Factor<T>*>& fs, const std::vector<const double*>& Bs,
                           const std::vector<double*>& Xs, const std::vector<int>& nrs, int max_blocks,
                           hipStream_t st) {
  const int P = (int)fs.size();
  std::vector<const PPlan*> pl(P);
  size_t nctr = 0;
  for (int p = 0; p < P; ++p) {
    pl[p] = &fs[p]->plan(nrs[p], max_blocks, st);
    nctr += (size_t)pl[p]->nctr;
  }
  std::vector<DBuf<char>> ws(P);
  DBuf<int> ctr(nctr + 2 * 8 + 1);   // pass counters, then (ticket, abort word) per launch group
  memset_async(ctr.get(), 0, ctr.bytes(), st);
  std::vector<VJob> tb, fb;
  std::vector<PInst> in(P);
  size_t c0 = 0;
  for (int p = 0; p < P; ++p) {
    const Factor<T>& f = *fs[p];
    ws[p].resize(pl[p]->ws_bytes);
    VJob J;
    J.s = f.nx; J.nblk = f.ny; J.nrhs = nrs[p]; J.ld = (long long)f.nx * f.ny;
    J.src = Bs[p]; J.dst = ws[p].get() + pl[p]->f0_off;
    tb.push_back(J);
    J.src = ws[p].get() + pl[p]->u0_off + (long long)f.nx * nrs[p] * sizeof(T); J.dst = Xs[p];
    fb.push_back(J);
    PInst& I = in[p];
    I.tasks = pl[p]->tasks; I.jobs = pl[p]->jobs; I.terms = pl[p]->terms; I.ntasks = pl[p]->ntasks;
    I.ws = ws[p].get(); I.ctr = ctr.get() + c0; I.tbuf_off = pl[p]->tbuf_off;
    c0 += (size_t)pl[p]->nctr;
  }
  gto_blocks<T>(st, tb);
  // grouped steps of the wide levels, merged over the problems step by step
  // (every plan lists its steps of one direction in the same level order)
  auto grouped = [&](bool pre) {
    size_t most = 0;
    for (int p = 0; p < P; ++p) most = std::max(most, (pre ? pl[p]->pre : pl[p]->post).size());
    for (size_t i = 0; i < most; ++i) {
      std::vector<MVJob> jb;
      std::vector<MVTerm> tm;
      for (int p = 0; p < P; ++p) {
        const auto& list = pre ? pl[p]->pre : pl[p]->post;
        // backward steps are aligned at level 0 (the last ones of every list)
        const long long k = pre ? (long long)i : (long long)i - (long long)(most - list.size());
        if (k < 0 || k >= (long long)list.size()) continue;
        const HostStep& h = list[(size_t)k];
        const uintptr_t base = reinterpret_cast<uintptr_t>(ws[p].get());
        const int t0 = (int)tm.size();
        for (MVTerm M : h.terms) {
          M.y = reinterpret_cast<const void*>(base + reinterpret_cast<uintptr_t>(M.y));
          tm.push_back(M);
        }
        for (MVJob J : h.jobs) {
          J.out = reinterpret_cast<void*>(base + reinterpret_cast<uintptr_t>(J.out));
          if (J.C0) J.C0 = reinterpret_cast<const void*>(base + reinterpret_cast<uintptr_t>(J.C0));
          J.term0 += t0;
          jb.push_back(J);
        }
      }
      PhaseScope ph(pre ? "solve forward" : "solve backward");
      ghmv<T>(st, jb, tm);
    }
  };
  grouped(true);
  // one launch per (NR, row form) group
  int grp = 0;
  for (int nr : {1, 2, 4, 8})
    for (int w : {1, 0}) {
      std::vector<PInst> gi;
      std::vector<VJob> gf;
      double fl = 0, by = 0;
      for (int p = 0; p < P; ++p)
        if (pl[p]->NR == nr && (int)pl[p]->w64 == w) {
          gi.push_back(in[p]);
          gf.push_back(fb[p]);
          fl += pl[p]->flops;
          by += pl[p]->bytes;
        }
      if (gi.empty()) continue;
      PhaseScope ph("solve persistent", -1);
      psolve_run<T>(st, gi, nr, w == 1, ctr.get() + nctr + 2 * grp, gf, fl, by);
      ++grp;
    }
  grouped(false);
  gfrom_blocks<T>(st, fb);
}

// Few right-hand sides (<= 8 per problem): every step of a level is one
// multi-term matvec, for all problems at once (levels counted from the top
// going down, from each problem's last level going up).  U[l] holds the
// level-l unknowns with one zero pad block at each end.
template <typename T>
void solve_fused_many(const std::vector<const Factor<T>*>& fs, const std::vector<const double*>& Bs,
                      const std::vector<double*>& Xs, const std::vector<int>& nrs, hipStream_t st, bool keep) {
  const int P = (int)fs.size();
  {   // a kept grouped pass for one problem, or the deep levels or the whole
      // pass as one persistent launch when asked for
    const int mode = SolveMode::get().mode.load();
    bool ok = !Bump::cur() && !Queue::get().dry();
    for (int p = 0; p < P && ok; ++p) ok = fs[p]->mstop == 1 && fs[p]->fused_ok(nrs[p]);
    if (ok && (mode == 1 || mode == 2)) {
      solve_persistent_many<T>(fs, Bs, Xs, nrs, mode == 2 ? INT32_MAX : kPersistBlocks, st);
      return;
    }
    if (ok && mode == 0 && keep && P == 1 && fs[0]->may_keep(nrs[0], st)) {
      solve_kept<T>(*fs[0], Bs[0], Xs[0], nrs[0], st);
      return;
    }
  }
  struct PV {
    std::vector<DBuf<T>> F, G, U;
    size_t blk = 0;
    int nl = 0;
  };
  std::vector<PV> pv(P);
  int maxl = 0;
  auto job = [&](int p, int nmat, T* out, int omul, int ooff, int term0, int nterm, const T* C0 = nullptr,
                 int cmul = 1, int coff = 0) {
    MVJob J = mv_job<T>(nmat, out, omul, ooff, term0, nterm, C0, cmul, coff, 1.0);
    J.s = fs[p]->nx; J.b = fs[p]->b; J.L = fs[p]->L; J.nrhs = nrs[p];
    return J;
  };
  {
    std::vector<VJob> tb;
    for (int p = 0; p < P; ++p) {
      const Factor<T>& f = *fs[p];
      PV& v = pv[p];
      v.nl = (int)f.lev.size();
      maxl = std::max(maxl, v.nl);
      v.blk = (size_t)f.nx * nrs[p];
      v.F.resize(v.nl + 1);
      v.G.resize(v.nl);
      v.U.resize(v.nl + 1);
      v.F[0].resize((size_t)f.ny * v.blk);
      VJob J;
      J.s = f.nx; J.nblk = f.ny; J.nrhs = nrs[p]; J.ld = (long long)f.nx * f.ny; J.src = Bs[p]; J.dst = v.F[0].get();
      tb.push_back(J);
    }
    gto_blocks<T>(st, tb);
  }
  for (int l = 0; l < maxl; ++l) {
    PhaseScope ph("solve forward", l);
    {  // g_k = X_k f_(2k); the dummy slot (m even) is zero
      std::vector<MVTerm> tm;
      std::vector<MVJob> jb;
      for (int p = 0; p < P; ++p) {
        PV& v = pv[p];
        if (l >= v.nl) continue;
        const Level<T>& Lv = fs[p]->lev[l];
        v.G[l].resize((size_t)Lv.ne * v.blk);
        const int t = (int)tm.size();
        tm.push_back(mv_hodlr<T>(Lv.X, 1, 0, v.F[l].get(), 2, 0, 1.0));
        jb.push_back(job(p, Lv.nreal, v.G[l].get(), 1, 0, t, 1));
        jb.push_back(job(p, Lv.ne - Lv.nreal, v.G[l].get(), 1, Lv.nreal, t, 0));
      }
      ghmv<T>(st, jb, tm);
    }
    {  // f'_j = f_(2j+1) - E_(2j+1) g_j - F_(2j+1) g_(j+1)
      std::vector<MVTerm> tm;
      std::vector<MVJob> jb;
      for (int p = 0; p < P; ++p) {
        PV& v = pv[p];
        if (l >= v.nl) continue;
        const Level<T>& Lv = fs[p]->lev[l];
        const int nodd = Lv.m / 2;
        v.F[l + 1].resize((size_t)nodd * v.blk);
        if (nodd <= 0) continue;
        const int t = (int)tm.size();
        if (Lv.diag) {
          tm.push_back(mv_diag<T>(Lv.e0.get(), 2, 1, v.G[l].get(), 1, 0, -1.0));
          tm.push_back(mv_diag<T>(Lv.f0.get(), 2, 1, v.G[l].get(), 1, 1, -1.0));
        } else {
          tm.push_back(mv_hodlr<T>(Lv.E, 2, 1, v.G[l].get(), 1, 0, -1.0));
          tm.push_back(mv_hodlr<T>(Lv.F, 2, 1, v.G[l].get(), 1, 1, -1.0));
        }
        jb.push_back(job(p, nodd, v.F[l + 1].get(), 1, 0, t, 2, v.F[l].get(), 2, 1));
      }
      ghmv<T>(st, jb, tm);
    }
  }
  {
    PhaseScope ph("solve last", -1);
    std::vector<MVTerm> tm;
    std::vector<MVJob> jb;
    GemmPlan dense;
    for (int p = 0; p < P; ++p) {
      PV& v = pv[p];
      const Factor<T>& f = *fs[p];
      if (f.mstop > 1) {   // u = Xd f over the remaining blocks; zero pads
        v.U[v.nl].resize((size_t)(f.mstop + 2) * v.blk);
        plan_dense_last<T>(dense, f, v.F[v.nl].get(), v.U[v.nl].get(), nrs[p]);
        jb.push_back(job(p, 1, v.U[v.nl].get(), 1, 0, 0, 0));
        jb.push_back(job(p, 1, v.U[v.nl].get(), 1, f.mstop + 1, 0, 0));
        continue;
      }
      v.U[v.nl].resize(3 * v.blk);
      const int t = (int)tm.size();
      tm.push_back(mv_hodlr<T>(f.Xlast, 1, 0, v.F[v.nl].get(), 1, 0, 1.0));
      jb.push_back(job(p, 1, v.U[v.nl].get(), 1, 1, t, 1));
      jb.push_back(job(p, 2, v.U[v.nl].get(), 2, 0, t, 0));
    }
    ghmv<T>(st, jb, tm);
    dense.run<T>(st);
  }
  for (int l = maxl - 1; l >= 0; --l) {
    PhaseScope ph("solve backward", l);
    std::vector<DBuf<T>> tmp(P);
    {  // tmp_k = E_(2k) u_(2k-1) + F_(2k) u_(2k+1): level-(l+1) unknowns k-1 and k (padded k, k+1)
      std::vector<MVTerm> tm;
      std::vector<MVJob> jb;
      for (int p = 0; p < P; ++p) {
        PV& v = pv[p];
        if (l >= v.nl) continue;
        const Level<T>& Lv = fs[p]->lev[l];
        v.U[l].resize((size_t)(Lv.m + 2) * v.blk);
        tmp[p].resize((size_t)Lv.nreal * v.blk);
        const int t = (int)tm.size();
        if (Lv.diag) {
          tm.push_back(mv_diag<T>(Lv.e0.get(), 2, 0, v.U[l + 1].get(), 1, 0, 1.0));
          tm.push_back(mv_diag<T>(Lv.f0.get(), 2, 0, v.U[l + 1].get(), 1, 1, 1.0));
        } else {
          tm.push_back(mv_hodlr<T>(Lv.E, 2, 0, v.U[l + 1].get(), 1, 0, 1.0));
          tm.push_back(mv_hodlr<T>(Lv.F, 2, 0, v.U[l + 1].get(), 1, 1, 1.0));
        }
        jb.push_back(job(p, Lv.nreal, tmp[p].get(), 1, 0, t, 2));
      }
      ghmv<T>(st, jb, tm);
    }
    {  // u_(2k) = g_k - X_k tmp_k; odd unknowns from level l+1; zero pads
      std::vector<MVTerm> tm;
      std::vector<MVJob> jb;
      for (int p = 0; p < P; ++p) {
        PV& v = pv[p];
        if (l >= v.nl) continue;
        const Level<T>& Lv = fs[p]->lev[l];
        const int m = Lv.m, nodd = m / 2;
        const int t = (int)tm.size();
        tm.push_back(mv_hodlr<T>(Lv.X, 1, 0, tmp[p].get(), 1, 0, -1.0));
        jb.push_back(job(p, Lv.nreal, v.U[l].get(), 2, 1, t, 1, v.G[l].get(), 1, 0));
        jb.push_back(job(p, nodd, v.U[l].get(), 2, 2, t, 0, v.U[l + 1].get(), 1, 1));
        jb.push_back(job(p, 1, v.U[l].get(), 1, 0, t, 0));
        jb.push_back(job(p, 1, v.U[l].get(), 1, m + 1, t, 0));
      }
      ghmv<T>(st, jb, tm);
    }
  }
  {
    std::vector<VJob> fb;
    for (int p = 0; p < P; ++p) {
      const Factor<T>& f = *fs[p];
      VJob J;
      J.s = f.nx; J.nblk = f.ny; J.nrhs = nrs[p]; J.ld = (long long)f.nx * f.ny;
      J.src = pv[p].U[0].get() + pv[p].blk; J.dst = Xs[p];
      fb.push_back(J);
    }
    gfrom_blocks<T>(st, fb);
  }
}

template <typename T>
void Factor<T>::solve_fused(const double* B, double* Xout, int nrhs, hipStream_t st) {
  solve_fused_many<T>({this}, {B}, {Xout}, {nrhs}, st, true);
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
  // final block(s); U[l] holds level-l unknowns with one zero pad block at each end
  if (mstop > 1) {
    U[nl].resize((size_t)(mstop + 2) * blk);
    fill<T>(st, U[nl].get(), (size_t)(mstop + 2) * blk, T(0));
    GemmPlan dense;
    plan_dense_last<T>(dense, *this, F[nl].get(), U[nl].get(), nrhs);
    dense.run<T>(st);
  } else {
    U[nl].resize(3 * blk);
    fill<T>(st, U[nl].get(), 3 * blk, T(0));
    hmul<T>(st, HV<T>{&Xlast, 1, 0}, 1, 0, false, nrhs, T(1), vflat(F[nl].get(), s, nrhs), T(0),
            vflat(U[nl].get() + blk, s, nrhs));
  }
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

// The factorisation of one or many independent problems.  The problems run
// in lockstep over the cyclic-reduction levels: every H-arithmetic step of a
// level (inverses, products, truncations) is planned for all problems that
// still have more than one block and issued as one set of grouped launches,
// so a batch of problems costs the launches of one.  Each problem keeps its
// own HODLR sets (its own padding), and every kernel variant is chosen by the
// shape of its problem alone, so a problem's factor is the same bits whether
// it is factored alone or in a batch.
template <typename T>
std::vector<std::unique_ptr<Factor<T>>> factor_many(const std::vector<acr_operator>& ops, const acr_options& opt,
                                                    hipStream_t st, const acr_dense_operator* dense,
                                                    const acr_operator3d* op3) {
  const int P = (int)ops.size();
  const double eps = opt.eps;
  const double ieps = opt.inner_eps;
  const int mr = opt.max_rank;
  work() = Work();
  const long long launches0 = launch_count();
  struct PS {
    Factor<T>* f = nullptr;
    const acr_operator* op = nullptr;
    int s = 0, ny = 0, L = 0, b = 0, m = 0;
    int pnx = 0;                           // 3-D: a block is a plane of rows of pnx unknowns
    const double* ys = nullptr;            // 3-D: in-plane couplings to r - pnx, r + pnx
    const double* yn = nullptr;
    HSet<T> D, E, F;
    DBuf<T> e0, f0;
  };
  std::vector<std::unique_ptr<Factor<T>>> out(P);
  std::vector<PS> ps(P);
  const int stop = std::max(opt.stop_blocks, 1);
  for (int p = 0; p < P; ++p) {
    int m = ops[p].ny;
    while (m > stop) m /= 2;
    if (m > 1 && ((long long)m * ops[p].nx > 1024 || m > kMaxSeg))
      fail(ACR_ERR_INVALID_ARG, "stop_blocks leaves a dense remainder of " + std::to_string(m) + " blocks of " +
                                    std::to_string(ops[p].nx) + " (at most 16 blocks and 1024 unknowns)" +
                                    (P > 1 ? " in problem " + std::to_string(p) : std::string()));
  }
  for (int p = 0; p < P; ++p) {
    out[p] = std::make_unique<Factor<T>>();
    Factor<T>& f = *out[p];
    PS& q = ps[p];
    q.f = &f;
    q.op = &ops[p];
    q.s = ops[p].nx;
    q.ny = ops[p].ny;
    q.L = hodlr_depth(q.s, opt.leaf);
    q.b = q.s >> q.L;
    q.m = q.ny;
    f.nx = q.s; f.ny = q.ny; f.leaf = opt.leaf; f.eps = eps; f.precision = opt.precision;
    f.L = q.L; f.b = q.b;
  }
  if (op3) {
    ps[0].pnx = op3->nx;
    ps[0].ys = op3->south;
    ps[0].yn = op3->north;
  }
  DBuf<int> status(P);   // per problem: a bad pivot in one of its inverses
  memset_async(status.get(), 0, (size_t)P * sizeof(int), st);
  if (dense) {
    // dense blocks: full-rank HODLR form, each off-diagonal block cut to eps;
    // E_i and F_i are general matrices from level 0 on
    PS& q = ps[0];
    const size_t nb = (size_t)q.ny * q.s * q.s;
    {
      DBuf<int> nonfin(1);
      memset_async(nonfin.get(), 0, sizeof(int), st);
      std::vector<NFJob> nf;
      for (const double* a : {dense->D, dense->E, dense->F}) {
        NFJob J;
        J.n = (long long)nb; J.a = a; J.flag = nonfin.get();
        nf.push_back(J);
      }
      gflag_nonfinite(st, nf);
      int bad = 0;
      read_to_host(&bad, nonfin.get(), sizeof(int), st);
      if (bad) fail(ACR_ERR_INVALID_ARG, "the dense operator holds a NaN or infinite coefficient");
    }
    std::vector<HJob> hj;
    std::vector<int> kfull(q.L + 1, 0);
    for (int d = 1; d <= q.L; ++d) kfull[d] = q.s >> d;
    HSet<T>* sets[3] = {&q.D, &q.E, &q.F};
    const double* src[3] = {dense->D, dense->E, dense->F};
    const int zm[3] = {-1, 0, q.ny - 1};
    for (int i = 0; i < 3; ++i) {
      HSet<T>& H = *sets[i];
      H.alloc(st, q.ny, q.s, q.b, q.L, kfull, -1);
      HJob J;
      J.s = q.s; J.b = q.b; J.L = q.L; J.nmat = q.ny; J.A = src[i]; J.zm = zm[i];
      J.lv = H.lv.get();
      for (int d = 1; d <= q.L; ++d) {
        J.U[d] = H.U[d].get();
        J.V[d] = H.V[d].get();
        H.kc[d] = kfull[d];
      }
      hj.push_back(J);
    }
    gdense_to_hodlr<T>(st, hj);
    {
      PhaseScope ph("compress blocks");
      recompress_multi<T>(st, {&q.D, &q.E, &q.F}, eps, mr);
    }
  } else {
  {
    DBuf<int> nonfin(P);
    memset_async(nonfin.get(), 0, (size_t)P * sizeof(int), st);
    std::vector<NFJob> nf;
    for (int p = 0; p < P; ++p) {
      const acr_operator& op = ops[p];
      for (const double* a : {op.diag, op.west, op.east, op.south, op.north, ps[p].ys, ps[p].yn}) {
        if (!a) continue;
        NFJob J;
        J.n = (long long)op.nx * op.ny; J.a = a; J.flag = nonfin.get() + p;
        nf.push_back(J);
      }
    }
    gflag_nonfinite(st, nf);
    std::vector<int> bad(P);
    read_to_host(bad.data(), nonfin.get(), (size_t)P * sizeof(int), st);
    for (int p = 0; p < P; ++p)
      if (bad[p])
        fail(ACR_ERR_INVALID_ARG, "the operator" + (P > 1 ? " of problem " + std::to_string(p) : std::string()) +
                                      " holds a NaN or infinite coefficient");
  }
  // level-0 operators: D_i as exact rank-1 HODLR (3-D: the plane operator,
  // exact ranks pnx or 1 by depth), E_i/F_i diagonal (E_0 and F_(ny-1) are
  // outside the grid: exact zeros)
  {
    std::vector<OpJob> lj, rj, pj, gj;
    for (PS& q : ps) {
      std::vector<int> k1(q.L + 1, 1);
      if (q.pnx > 0)
        for (int d = 1; d <= q.L; ++d) k1[d] = plane_rank(q.s, d, q.pnx);
      q.D.alloc(st, q.ny, q.s, q.b, q.L, k1, -1);
      OpJob J;
      J.s = q.s; J.b = q.b; J.L = q.L; J.nmat = q.ny;
      J.diag = q.op->diag; J.west = q.op->west; J.east = q.op->east;
      J.pnx = q.pnx; J.south = q.ys; J.north = q.yn;
      J.out = q.D.lv.get();
      lj.push_back(J);
      if (q.L > 0) {
        OpJob R = J;
        R.out = nullptr;
        for (int d = 1; d <= q.L; ++d) {
          R.U[d] = q.D.U[d].get();
          R.V[d] = q.D.V[d].get();
          q.D.kc[d] = k1[d];
        }
        (q.pnx > 0 ? pj : rj).push_back(R);
      }
      q.e0.resize((size_t)q.ny * q.s);
      q.f0.resize((size_t)q.ny * q.s);
      OpJob G;
      G.s = q.s; G.nmat = q.ny;
      G.src = q.op->south; G.out = q.e0.get(); G.zblk = 0;
      gj.push_back(G);
      G.src = q.op->north; G.out = q.f0.get(); G.zblk = q.ny - 1;
      gj.push_back(G);
    }
    gleaves_tridiag<T>(st, lj);
    grank1_factors<T>(st, rj);
    gplane_factors<T>(st, pj);
    ggather_diag<T>(st, gj);
  }
  }

  bool diag = dense == nullptr;   // level 0 of a stencil: E_i, F_i diagonal
  for (int lvl = 0;; ++lvl) {
    std::vector<int> act;   // problems with more than max(stop_blocks, 1) blocks left
    for (int p = 0; p < P; ++p)
      if (ps[p].m > stop) act.push_back(p);
    if (act.empty()) break;
    const int na = (int)act.size();
    PhaseScope lph("level", lvl);
    std::vector<Level<T>> lv(na);
    for (int a = 0; a < na; ++a) {
      const PS& q = ps[act[a]];
      lv[a].m = q.m;
      lv[a].nreal = (q.m + 1) / 2;
      lv[a].ne = q.m / 2 + 1;
      lv[a].diag = diag;
      stage_check(st, q.D, status.get() + act[a], "D", lvl);
    }
    // X_k = T(D_k^{-1}) for even k
    std::vector<char> closed(na, 0);   // level 0: D_k tridiagonal, inverse in closed form (exact rank 1)
    {
      PhaseScope ph("inverse");
      if (diag) {
        std::vector<OpJob> tj;
        std::vector<int> ta;
        for (int a = 0; a < na; ++a) {
          const PS& q = ps[act[a]];
          if (q.s > 3072 || q.pnx > 0) continue;   // closed form: tridiagonal D only
          std::vector<int> k1(q.L + 1, 1);
          lv[a].X.alloc(st, lv[a].nreal, q.s, q.b, q.L, k1, -1);
          OpJob J;
          J.s = q.s; J.b = q.b; J.L = q.L; J.nmat = lv[a].nreal; J.bmul = 2; J.boff = 0;
          J.diag = q.op->diag; J.west = q.op->west; J.east = q.op->east;
          J.out = lv[a].X.lv.get();
          for (int d = 1; d <= q.L; ++d) {
            J.U[d] = lv[a].X.U[d].get();
            J.V[d] = lv[a].X.V[d].get();
            lv[a].X.kc[d] = 1;
          }
          tj.push_back(J);
          ta.push_back(a);
        }
        if (!tj.empty()) {
          DBuf<int> fb(tj.size());
          memset_async(fb.get(), 0, tj.size() * sizeof(int), st);
          for (size_t i = 0; i < tj.size(); ++i) tj[i].flag = fb.get() + i;
          gtridiag_inverse<T>(st, tj);
          std::vector<int> fbh(tj.size());
          read_to_host(fbh.data(), fb.get(), tj.size() * sizeof(int), st);
          for (size_t i = 0; i < tj.size(); ++i) closed[ta[i]] = fbh[i] == 0;
        }
      }
      std::vector<HInvJob<T>> hj;
      for (int a = 0; a < na; ++a)
        if (!closed[a]) hj.push_back(HInvJob<T>{&lv[a].X, HV<T>{&ps[act[a]].D, 2, 0}, lv[a].nreal, status.get() + act[a]});
      hinv_multi<T>(st, hj);
    }
    {   // the closed form is exact with rank-one blocks: T_eps leaves it unchanged
      PhaseScope ph("recompress X");
      std::vector<HSet<T>*> xs;
      for (int a = 0; a < na; ++a) {
        stage_check(st, lv[a].X, status.get() + act[a], "inv", lvl);
        if (!closed[a]) xs.push_back(&lv[a].X);
      }
      recompress_multi<T>(st, xs, eps, mr);
    }
    std::vector<HSet<T>> P_(na), Q_(na), Dn(na), En(na), Fn(na), EQ(na), FP(na);
    if (diag) {
      // P_k = X_k diag(e_2k), Q_k = X_k diag(f_2k)
      std::vector<ColScale<T>> cs;
      for (int a = 0; a < na; ++a) {
        PS& q = ps[act[a]];
        ColScale<T> c;
        c.C = &P_[a]; c.cnt_alloc = lv[a].ne; c.nmat = lv[a].nreal; c.H = HV<T>{&lv[a].X, 1, 0};
        c.cols = q.e0.get(); c.cmul = 2; c.coff = 0;
        cs.push_back(c);
        c.C = &Q_[a]; c.cols = q.f0.get();
        cs.push_back(c);
      }
      {
        PhaseScope ph("products P,Q");
        hscale_cols_multi<T>(st, cs);
      }
      {
        PhaseScope ph("recompress P,Q");
        std::vector<HSet<T>*> sets;
        for (int a = 0; a < na; ++a) { sets.push_back(&P_[a]); sets.push_back(&Q_[a]); }
        recompress_multi<T>(st, sets, eps, mr);
      }
      PhaseScope ph("products D',E',F'");
      // D'_j = D_i - diag(e_i) Q_j - diag(f_i) P_(j+1);  E'_j = -diag(e_i) P_j;  F'_j = -diag(f_i) Q_(j+1)
      std::vector<StackOut<T>> so;
      for (int a = 0; a < na; ++a) {
        PS& q = ps[act[a]];
        const int nodd = q.m / 2;
        StackOut<T> d;
        d.C = &Dn[a]; d.cnt_alloc = nodd; d.nmat = nodd;
        d.terms.resize(3);
        d.terms[0].h = HV<T>{&q.D, 2, 1};
        d.terms[1].h = HV<T>{&Q_[a], 1, 0}; d.terms[1].coef = -1.0; d.terms[1].rows = q.e0.get(); d.terms[1].rmul = 2; d.terms[1].roff = 1;
        d.terms[2].h = HV<T>{&P_[a], 1, 1}; d.terms[2].coef = -1.0; d.terms[2].rows = q.f0.get(); d.terms[2].rmul = 2; d.terms[2].roff = 1;
        so.push_back(d);
        StackOut<T> e;
        e.C = &En[a]; e.cnt_alloc = nodd; e.nmat = nodd;
        e.terms.resize(1);
        e.terms[0].h = HV<T>{&P_[a], 1, 0}; e.terms[0].coef = -1.0; e.terms[0].rows = q.e0.get(); e.terms[0].rmul = 2; e.terms[0].roff = 1;
        so.push_back(e);
        StackOut<T> fo;
        fo.C = &Fn[a]; fo.cnt_alloc = nodd; fo.nmat = nodd;
        fo.terms.resize(1);
        fo.terms[0].h = HV<T>{&Q_[a], 1, 1}; fo.terms[0].coef = -1.0; fo.terms[0].rows = q.f0.get(); fo.terms[0].rmul = 2; fo.terms[0].roff = 1;
        so.push_back(fo);
      }
      hstack_multi<T>(st, so);
      for (int a = 0; a < na; ++a) {
        lv[a].e0 = std::move(ps[act[a]].e0);
        lv[a].f0 = std::move(ps[act[a]].f0);
      }
    } else {
      // P_k = X_k E_2k, Q_k = X_k F_2k
      std::vector<POut<T>> pq;
      for (int a = 0; a < na; ++a) {
        PS& q = ps[act[a]];
        POut<T> o;
        o.C = &P_[a]; o.cnt_alloc = lv[a].ne; o.nmat = lv[a].nreal;
        o.terms = {PTerm<T>{1.0, HV<T>{&lv[a].X, 1, 0}, HV<T>{&q.E, 2, 0}}};
        pq.push_back(o);
        o.C = &Q_[a];
        o.terms = {PTerm<T>{1.0, HV<T>{&lv[a].X, 1, 0}, HV<T>{&q.F, 2, 0}}};
        pq.push_back(o);
      }
      {
        PhaseScope ph("products P,Q");
        hprod_multi<T>(st, pq);
      }
      {
        PhaseScope ph("recompress P,Q");
        std::vector<HSet<T>*> sets;
        for (int a = 0; a < na; ++a) { sets.push_back(&P_[a]); sets.push_back(&Q_[a]); }
        recompress_multi<T>(st, sets, eps, mr);
      }
      PhaseScope ph("products D',E',F'");
      std::vector<POut<T>> up;
      for (int a = 0; a < na; ++a) {
        PS& q = ps[act[a]];
        const int nodd = q.m / 2;
        POut<T> e;
        e.C = &En[a]; e.cnt_alloc = nodd; e.nmat = nodd;
        e.terms = {PTerm<T>{-1.0, HV<T>{&q.E, 2, 1}, HV<T>{&P_[a], 1, 0}}};
        up.push_back(e);
        POut<T> fo;
        fo.C = &Fn[a]; fo.cnt_alloc = nodd; fo.nmat = nodd;
        fo.terms = {PTerm<T>{-1.0, HV<T>{&q.F, 2, 1}, HV<T>{&Q_[a], 1, 1}}};
        up.push_back(fo);
        if (ieps > 0) {
          // intermediate truncation of the two Schur products, then the sum
          POut<T> x;
          x.C = &EQ[a]; x.cnt_alloc = nodd; x.nmat = nodd;
          x.terms = {PTerm<T>{1.0, HV<T>{&q.E, 2, 1}, HV<T>{&Q_[a], 1, 0}}};
          up.push_back(x);
          x.C = &FP[a];
          x.terms = {PTerm<T>{1.0, HV<T>{&q.F, 2, 1}, HV<T>{&P_[a], 1, 1}}};
          up.push_back(x);
        } else {
          // D'_j = D_i - E_i Q_j - F_i P_(j+1), accumulated exactly, one truncation
          POut<T> d;
          d.C = &Dn[a]; d.cnt_alloc = nodd; d.nmat = nodd;
          d.has_d = true; d.D = HV<T>{&q.D, 2, 1};
          d.terms = {PTerm<T>{-1.0, HV<T>{&q.E, 2, 1}, HV<T>{&Q_[a], 1, 0}},
                     PTerm<T>{-1.0, HV<T>{&q.F, 2, 1}, HV<T>{&P_[a], 1, 1}}};
          up.push_back(d);
        }
      }
      hprod_multi<T>(st, up);
      if (ieps > 0) {
        {
          PhaseScope ph2("recompress EQ,FP");
          std::vector<HSet<T>*> sets;
          for (int a = 0; a < na; ++a) { sets.push_back(&EQ[a]); sets.push_back(&FP[a]); }
          recompress_multi<T>(st, sets, ieps, 0);
        }
        std::vector<StackOut<T>> so;
        for (int a = 0; a < na; ++a) {
          PS& q = ps[act[a]];
          const int nodd = q.m / 2;
          StackOut<T> d;
          d.C = &Dn[a]; d.cnt_alloc = nodd; d.nmat = nodd;
          d.terms.resize(3);
          d.terms[0].h = HV<T>{&q.D, 2, 1};
          d.terms[1].h = HV<T>{&EQ[a], 1, 0}; d.terms[1].coef = -1.0;
          d.terms[2].h = HV<T>{&FP[a], 1, 0}; d.terms[2].coef = -1.0;
          so.push_back(d);
        }
        hstack_multi<T>(st, so);
      }
      for (int a = 0; a < na; ++a) {
        lv[a].E = std::move(ps[act[a]].E);
        lv[a].F = std::move(ps[act[a]].F);
      }
    }
    for (int a = 0; a < na; ++a) {
      stage_check(st, P_[a], status.get() + act[a], "P", lvl);
      stage_check(st, Q_[a], status.get() + act[a], "Q", lvl);
      stage_check(st, Dn[a], status.get() + act[a], "D'-exact", lvl);
    }
    {
      PhaseScope ph("recompress D',E',F'");
      std::vector<HSet<T>*> sets;
      for (int a = 0; a < na; ++a) { sets.push_back(&Dn[a]); sets.push_back(&En[a]); sets.push_back(&Fn[a]); }
      recompress_multi<T>(st, sets, eps, mr);
    }
    for (int a = 0; a < na; ++a) {
      PS& q = ps[act[a]];
      Factor<T>& f = *q.f;
      stage_check(st, Dn[a], status.get() + act[a], "D'", lvl);
      stage_check(st, En[a], status.get() + act[a], "E'", lvl);
      stage_check(st, Fn[a], status.get() + act[a], "F'", lvl);
      Level<T>& L_ = lv[a];
      int r = L_.X.max_rank();
      r = std::max(r, L_.E.max_rank());
      r = std::max(r, L_.F.max_rank());
      f.lev_rank.push_back(r);
      {   // mean numerical rank of the stored off-diagonal blocks of this level
        double rs = 0.0, nb = 0.0;
        for (const HSet<T>* H : {&L_.X, &L_.E, &L_.F})
          for (int d = 1; d <= H->L; ++d) {
            rs += H->rank_sum(d);
            nb += (double)H->cnt * (1 << d);
          }
        f.lev_mean.push_back(nb > 0 ? rs / nb : 0.0);
      }
      f.lev.push_back(std::move(L_));
      q.D = std::move(Dn[a]);
      q.E = std::move(En[a]);
      q.F = std::move(Fn[a]);
      q.m = q.m / 2;
    }
    diag = false;
  }
  {
    PhaseScope ph("last inverse", -1);
    std::vector<HInvJob<T>> hj;
    std::vector<HSet<T>*> xs;
    std::vector<DenseJob> dj;
    std::vector<IJob> ij;
    std::vector<DBuf<double>> dense;
    for (int p = 0; p < P; ++p) {
      PS& q = ps[p];
      if (q.m == 1) {
        hj.push_back(HInvJob<T>{&q.f->Xlast, HV<T>{&q.D, 1, 0}, 1, status.get() + p});
        xs.push_back(&q.f->Xlast);
        continue;
      }
      // early stop: the remaining block-tridiagonal system, dense, inverted in FP64
      const int m = q.m, s = q.s, n = m * s;
      const bool at0 = q.f->lev.empty();   // no level ran: E, F are the level-0 diagonals
      dense.emplace_back((size_t)n * n);
      double* A = dense.back().get();
      memset_async(A, 0, (size_t)n * n * sizeof(double), st);
      auto hodlr_job = [&](const HSet<T>& H, int idx, double* o) {
        DenseJob J;
        J.type = 0; J.s = s; J.b = H.b; J.L = H.L; J.midx = idx; J.lv = H.lv.get(); J.out = o; J.ld = n;
        for (int d = 1; d <= H.L; ++d) {
          J.U[d] = H.U[d].get(); J.V[d] = H.V[d].get(); J.k[d] = H.k[d]; J.kc[d] = H.kc[d];
        }
        return J;
      };
      auto diag_job = [&](const DBuf<T>& v, int idx, double* o) {
        DenseJob J;
        J.type = 1; J.s = s; J.midx = idx; J.lv = v.get(); J.out = o; J.ld = n;
        return J;
      };
      for (int i = 0; i < m; ++i) {
        double* di = A + (size_t)i * s + (size_t)i * s * n;
        dj.push_back(hodlr_job(q.D, i, di));
        if (i > 0) dj.push_back(at0 ? diag_job(q.e0, i, di - (size_t)s * n) : hodlr_job(q.E, i, di - (size_t)s * n));
        if (i + 1 < m) dj.push_back(at0 ? diag_job(q.f0, i, di + (size_t)s * n) : hodlr_job(q.F, i, di + (size_t)s * n));
      }
      q.f->mstop = m;
      q.f->Xd.resize((size_t)n * n);
      IJob I;
      I.n = n; I.nprob = 1; I.A = A; I.sA = (long long)n * n; I.X = q.f->Xd.get(); I.sX = (long long)n * n;
      I.status = status.get() + p;
      ij.push_back(I);
      work().inv_flops += 2.0 * (double)n * n * n;
    }
    gdense_blocks<T>(st, dj);
    ginverse<double, T>(st, ij);
    hinv_multi<T>(st, hj);
    recompress_multi<T>(st, xs, eps, mr);
  }
  std::vector<int> bad(P);
  read_to_host(bad.data(), status.get(), (size_t)P * sizeof(int), st);
  for (int p = 0; p < P; ++p)
    if (bad[p])
      fail(ACR_ERR_SINGULAR, "zero or non-finite pivot in a dense leaf or capacitance inverse" +
                                 (P > 1 ? " (problem " + std::to_string(p) + ")" : std::string()));
  const Work w = work();
  const long long nl = launch_count() - launches0;
  for (int p = 0; p < P; ++p) {
    out[p]->work_done = w;
    out[p]->launches = nl;
    out[p]->batch = P;
  }
  return out;
}

#define ACR_INST(T)                                                                                      \
  template struct Factor<T>;                                                                             \
  template std::vector<std::unique_ptr<Factor<T>>> factor_many<T>(const std::vector<acr_operator>&,      \
                                                                  const acr_options&, hipStream_t,       \
                                                                  const acr_dense_operator*,             \
                                                                  const acr_operator3d*);                \
  template void solve_fused_many<T>(const std::vector<const Factor<T>*>&, const std::vector<const double*>&, \
                                    const std::vector<double*>&, const std::vector<int>&, hipStream_t, bool);
ACR_INST(float)
ACR_INST(double)
#undef ACR_INST

}  // namespace acr

namespace acr {
namespace {

// Scratch of the allocation-free solve (acr_solve_noalloc): the workspace of
// one call, then its job descriptors.  Each GPU the library runs on holds its
// own copy of the array until the process ends.
constexpr size_t kNoAllocBytes = size_t(64) << 20;
constexpr size_t kNoAllocDescBytes = size_t(4) << 20;
constexpr size_t kNoAllocWorkBytes = kNoAllocBytes - kNoAllocDescBytes;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// Device address of `scratch` on device `dev` (the host-side name is only a
// stand-in): looked up once per device, with that device current.
char* scratch_on_device(int dev) {
  static std::mutex mu;
  static std::map<int, char*> ptrs;
  std::lock_guard<std::mutex> g(mu);
  auto it = ptrs.find(dev);
  if (it != ptrs.end()) return it->second;
  void* p = nullptr;
  ACR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) fail(ACR_ERR_DEVICE, "no device address for the allocation-free scratch");
  ptrs[dev] = static_cast<char*>(p);
  return static_cast<char*>(p);
}

// Installs the scratch as the calling thread's memory and descriptor source.
struct NoAllocScope {
  Bump bump;
  DescArena::External ext;
  NoAllocScope(char* base, bool count_only) {
    bump.base = base;
    bump.cap = kNoAllocWorkBytes;
    bump.count_only = count_only;
    ext.dev = base + kNoAllocWorkBytes;
    ext.cap = kNoAllocDescBytes;
    ext.count_only = count_only;
    Bump::cur() = &bump;
    DescArena::External::cur() = &ext;
    Queue::get().set_dry(count_only);
  }
  ~NoAllocScope() {
    Queue::get().set_dry(false);
    Bump::cur() = nullptr;
    DescArena::External::cur() = nullptr;
  }
};

}  // namespace
}  // namespace acr


using namespace acr;

namespace acr {

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

// Whether [a, a+na) and [b, b+nb) (doubles) share an element.
bool overlap2(const double* a, size_t na, const double* b, size_t nb) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + nb * sizeof(double) && y < x + na * sizeof(double);
}

void check_options(const acr_options* opt) {
  if (!opt) fail(ACR_ERR_INVALID_ARG, "options are NULL");
  if (opt->leaf < 1 || opt->leaf > 128) fail(ACR_ERR_INVALID_ARG, "leaf must be in 1..128");
  if (!(opt->eps >= 0.0) || !std::isfinite(opt->eps)) fail(ACR_ERR_INVALID_ARG, "eps must be finite and >= 0");
  if (!(opt->inner_eps >= 0.0)) fail(ACR_ERR_INVALID_ARG, "inner_eps must be >= 0");
  if (opt->precision != ACR_FP64 && opt->precision != ACR_MIXED_FP32) fail(ACR_ERR_INVALID_ARG, "unknown precision");
  if (opt->max_rank < 0) fail(ACR_ERR_INVALID_ARG, "max_rank must be >= 0");
  if (opt->stop_blocks < 0) fail(ACR_ERR_INVALID_ARG, "stop_blocks must be >= 0");
}

void check_op(const acr_operator* op) {
  if (!op) fail(ACR_ERR_INVALID_ARG, "operator is NULL");
  if (op->nx < 1 || op->ny < 1) fail(ACR_ERR_INVALID_ARG, "nx and ny must be >= 1");
  if ((long long)op->nx * op->ny > (1LL << 31)) fail(ACR_ERR_INVALID_ARG, "N too large");
  if (!op->diag || !op->west || !op->east || !op->south || !op->north)
    fail(ACR_ERR_INVALID_ARG, "a stencil array is NULL");
}

void check_op3(const acr_operator3d* op) {
  if (!op) fail(ACR_ERR_INVALID_ARG, "operator is NULL");
  if (op->nx < 1 || op->ny < 1 || op->nz < 1) fail(ACR_ERR_INVALID_ARG, "nx, ny and nz must be >= 1");
  if ((long long)op->nx * op->ny * op->nz > (1LL << 31) || (long long)op->nx * op->ny > (1LL << 30))
    fail(ACR_ERR_INVALID_ARG, "N too large");
  if (!op->diag || !op->west || !op->east || !op->south || !op->north || !op->down || !op->up)
    fail(ACR_ERR_INVALID_ARG, "a stencil array is NULL");
}

}  // namespace acr

namespace {

bool overlap(const double* a, const double* b, size_t n) { return overlap2(a, n, b, n); }

// Iterative refinement with the factor of h as M (the body of the
// acr_solve_refined entry points): resid(X, B, R, nrhs) sets R = B - A X.
template <typename Resid>
void refine_body(acr_handle h, long long n, const double* B, double* X, int nrhs, double tol, int maxit,
                 hipStream_t st, int& its, double& rel, Resid resid) {
  if (!h || !B || !X || nrhs < 1 || maxit < 0) fail(ACR_ERR_INVALID_ARG, "bad arguments");
  StreamScope ss(st);
  if (overlap(X, B, (size_t)n * nrhs)) fail(ACR_ERR_INVALID_ARG, "X must not overlap B");
  DBuf<double> R((size_t)n * nrhs), D((size_t)n * nrhs), nb(nrhs), nr(nrhs);
  std::vector<double> hb(nrhs), hr(nrhs);
  col_sumsq(st, n, nrhs, B, nb.get());
  memset_async(X, 0, (size_t)n * nrhs * sizeof(double), st);
  copy_d2d_async(R.get(), B, (size_t)n * nrhs * sizeof(double), st);
  read_to_host(hb.data(), nb.get(), nrhs * sizeof(double), st);
  for (its = 0;; ++its) {
    if (its > 0) {
      resid(X, B, R.get(), nrhs);
    }
    col_sumsq(st, n, nrhs, R.get(), nr.get());
    read_to_host(hr.data(), nr.get(), nrhs * sizeof(double), st);
    rel = 0.0;
    for (int q = 0; q < nrhs; ++q) {
      const double v = hb[q] > 0 ? std::sqrt(hr[q] / hb[q]) : std::sqrt(hr[q]);
      rel = nan_max(rel, v);
    }
    if (!(rel > tol) || its >= maxit || !std::isfinite(rel)) break;
    h->f->solve(R.get(), D.get(), nrhs, st);
    axpy_d(st, n * nrhs, D.get(), X);
  }
  if (!(rel <= tol)) fail(ACR_ERR_NOT_CONVERGED, "refinement stopped at relative residual " + std::to_string(rel));
}

// Restarted FGMRES right-preconditioned by the factor of h (the body of the
// acr_solve_krylov entry points): resid(x, b, r) sets r = b - A x (one column).
template <typename Resid>
void krylov_body(acr_handle h, long long n, const double* B, double* X, int nrhs, double tol, int maxit,
                 int restart, hipStream_t st, int& its_all, double& rel_all, Resid resid) {
  if (!h || !B || !X || nrhs < 1 || maxit < 0) fail(ACR_ERR_INVALID_ARG, "bad arguments");
  if (restart < 1 || restart > 64) fail(ACR_ERR_INVALID_ARG, "restart must be in 1..64");
  StreamScope ss(st);
  if (overlap(X, B, (size_t)n * nrhs)) fail(ACR_ERR_INVALID_ARG, "X must not overlap B");
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
  auto Aop = resid;   // r = b - A x
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
        const double* yd = static_cast<const double*>(desc_put(y.data(), k * sizeof(double), st));
        maxpy(st, n, k, 1.0, 1.0, yd, Z.get(), n, x);
      }
    }
    its_all = std::max(its_all, its);
    rel_all = nan_max(rel_all, rel);
  }
  if (!(rel_all <= tol))
    fail(ACR_ERR_NOT_CONVERGED, "FGMRES stopped at relative residual " + std::to_string(rel_all));
}

// Architecture name of the current device (the tuning table's key).
std::string device_arch() {
  int dev = 0;
  ACR_HIP(hipGetDevice(&dev));
  hipDeviceProp_t pr;
  ACR_HIP(hipGetDeviceProperties(&pr, dev));
  return std::string(pr.gcnArchName);
}

template <typename T>
void solve_batched_t(const acr_handle* hs, const double* const* B, double* const* X, const int32_t* nrhs,
                     int count, int precision, hipStream_t st) {
  std::vector<const Factor<T>*> fs;
  std::vector<const double*> bs;
  std::vector<double*> xs;
  std::vector<int> nr;
  for (int p = 0; p < count; ++p) {
    if (hs[p]->precision != precision) continue;
    auto* f = static_cast<Factor<T>*>(hs[p]->f.get());
    if (f->fused_ok(nrhs[p])) {
      fs.push_back(f);
      bs.push_back(B[p]);
      xs.push_back(X[p]);
      nr.push_back(nrhs[p]);
    } else {
      f->solve_gemm(B[p], X[p], nrhs[p], st);   // many right-hand sides: one problem at a time
    }
  }
  if (!fs.empty()) solve_fused_many<T>(fs, bs, xs, nr, st);
}

}  // namespace

extern "C" {

acr_status acr_factor(const acr_operator* op, const acr_options* opt, void* stream, acr_handle* out) {
  return guard([&] {
    check_op(op);
    if (!out) fail(ACR_ERR_INVALID_ARG, "output handle is NULL");
    check_options(opt);
    if (hodlr_depth(op->nx, opt->leaf) < 0)
      fail(ACR_ERR_INVALID_ARG, "block size must be leaf' * 2^L (halving exact down to the leaf)");
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamScope ss(st);
    auto h = std::make_unique<acr_handle_s>();
    h->precision = opt->precision;
    h->nx = op->nx; h->ny = op->ny;
    std::vector<acr_operator> ops{*op};
    if (opt->precision == ACR_FP64) h->f = std::move(factor_many<double>(ops, *opt, st)[0]);
    else h->f = std::move(factor_many<float>(ops, *opt, st)[0]);
    *out = h.release();
  });
}

acr_status acr_factor_3d(const acr_operator3d* op, const acr_options* opt, void* stream, acr_handle* out) {
  return guard([&] {
    check_op3(op);
    if (!out) fail(ACR_ERR_INVALID_ARG, "output handle is NULL");
    check_options(opt);
    const int s = op->nx * op->ny;
    const int L = hodlr_depth(s, opt->leaf);
    if (L < 0) fail(ACR_ERR_INVALID_ARG, "plane size nx*ny must be leaf' * 2^L (halving exact down to the leaf)");
    for (int d = 1; d <= L; ++d) {   // every split on a row boundary or inside one row
      const int sd = s >> d;
      if (sd % op->nx != 0 && op->nx % (2 * sd) != 0)
        fail(ACR_ERR_INVALID_ARG, "the HODLR split of a plane must fall on row boundaries or inside a row "
                                  "(s/2^d a multiple of nx, or nx a multiple of s/2^(d-1))");
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamScope ss(st);
    acr_operator blk{};   // block form: one block per plane, z couplings as E_k / F_k
    blk.nx = s;
    blk.ny = op->nz;
    blk.diag = op->diag; blk.west = op->west; blk.east = op->east;
    blk.south = op->down; blk.north = op->up;
    std::vector<acr_operator> v{blk};
    auto h = std::make_unique<acr_handle_s>();
    h->precision = opt->precision;
    h->nx = s;
    h->ny = op->nz;
    if (opt->precision == ACR_FP64) h->f = std::move(factor_many<double>(v, *opt, st, nullptr, op)[0]);
    else h->f = std::move(factor_many<float>(v, *opt, st, nullptr, op)[0]);
    *out = h.release();
  });
}

acr_status acr_factor_dense(const acr_dense_operator* op, const acr_options* opt, void* stream, acr_handle* out) {
  return guard([&] {
    if (!op || !out) fail(ACR_ERR_INVALID_ARG, "NULL argument");
    if (op->nx < 1 || op->ny < 1) fail(ACR_ERR_INVALID_ARG, "nx and ny must be >= 1");
    if ((long long)op->nx * op->nx * op->ny > (1LL << 31)) fail(ACR_ERR_INVALID_ARG, "operator too large");
    if (!op->D || !op->E || !op->F) fail(ACR_ERR_INVALID_ARG, "a block array is NULL");
    check_options(opt);
    if (hodlr_depth(op->nx, opt->leaf) < 0)
      fail(ACR_ERR_INVALID_ARG, "block size must be leaf' * 2^L (halving exact down to the leaf)");
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamScope ss(st);
    acr_operator shape{};
    shape.nx = op->nx;
    shape.ny = op->ny;
    std::vector<acr_operator> v{shape};
    auto h = std::make_unique<acr_handle_s>();
    h->precision = opt->precision;
    h->nx = op->nx;
    h->ny = op->ny;
    if (opt->precision == ACR_FP64) h->f = std::move(factor_many<double>(v, *opt, st, op)[0]);
    else h->f = std::move(factor_many<float>(v, *opt, st, op)[0]);
    *out = h.release();
  });
}

acr_status acr_factor_batched(const acr_operator* ops, const acr_options* opt, int32_t count, void* stream,
                              acr_handle* out) {
  return guard([&] {
    if (count < 1 || !ops || !out) fail(ACR_ERR_INVALID_ARG, "count must be >= 1 with non-NULL ops and out");
    check_options(opt);
    std::vector<acr_operator> v(ops, ops + count);
    for (int p = 0; p < count; ++p) {
      check_op(&v[p]);
      if (hodlr_depth(v[p].nx, opt->leaf) < 0)
        fail(ACR_ERR_INVALID_ARG, "problem " + std::to_string(p) +
                                      ": block size must be leaf' * 2^L (halving exact down to the leaf)");
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamScope ss(st);
    std::vector<std::unique_ptr<acr_handle_s>> hs(count);
    if (opt->precision == ACR_FP64) {
      auto fs = factor_many<double>(v, *opt, st);
      for (int p = 0; p < count; ++p) {
        hs[p] = std::make_unique<acr_handle_s>();
        hs[p]->f = std::move(fs[p]);
      }
    } else {
      auto fs = factor_many<float>(v, *opt, st);
      for (int p = 0; p < count; ++p) {
        hs[p] = std::make_unique<acr_handle_s>();
        hs[p]->f = std::move(fs[p]);
      }
    }
    for (int p = 0; p < count; ++p) {
      hs[p]->precision = opt->precision;
      hs[p]->nx = v[p].nx;
      hs[p]->ny = v[p].ny;
    }
    for (int p = 0; p < count; ++p) out[p] = hs[p].release();
  });
}

acr_status acr_solve_batched(const acr_handle* hs, const double* const* B, double* const* X, const int32_t* nrhs,
                             int32_t count, void* stream) {
  return guard([&] {
    if (count < 1 || !hs || !B || !X || !nrhs) fail(ACR_ERR_INVALID_ARG, "NULL argument or count < 1");
    for (int p = 0; p < count; ++p) {
      if (!hs[p] || !B[p] || !X[p]) fail(ACR_ERR_INVALID_ARG, "NULL handle or vector in the batch");
      if (nrhs[p] < 1) fail(ACR_ERR_INVALID_ARG, "nrhs must be >= 1");
      const size_t n = (size_t)hs[p]->nx * hs[p]->ny * nrhs[p];
      for (int q = 0; q < count; ++q) {
        const size_t nq = (size_t)hs[q]->nx * hs[q]->ny * nrhs[q];
        if (q < p && overlap2(X[p], n, X[q], nq)) fail(ACR_ERR_INVALID_ARG, "outputs of the batch overlap");
        if (q != p && overlap2(X[p], n, B[q], nq))
          fail(ACR_ERR_INVALID_ARG, "an output of the batch overlaps another problem's right-hand side");
      }
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamScope ss(st);
    solve_batched_t<double>(hs, B, X, nrhs, count, ACR_FP64, st);
    solve_batched_t<float>(hs, B, X, nrhs, count, ACR_MIXED_FP32, st);
  });
}

acr_status acr_solve(acr_handle h, const double* B, double* X, int32_t nrhs, void* stream) {
  return guard([&] {
    if (!h || !B || !X) fail(ACR_ERR_INVALID_ARG, "NULL argument");
    if (nrhs < 1) fail(ACR_ERR_INVALID_ARG, "nrhs must be >= 1");
    StreamScope ss(static_cast<hipStream_t>(stream));
    h->f->solve(B, X, nrhs, static_cast<hipStream_t>(stream));
  });
}

acr_status acr_solve_noalloc(acr_handle h, const double* B, double* X, int32_t nrhs, void* stream) {
  return guard([&] {
    if (!h || !B || !X) fail(ACR_ERR_INVALID_ARG, "NULL argument");
    if (nrhs < 1) fail(ACR_ERR_INVALID_ARG, "nrhs must be >= 1");
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamScope ss(st);
    queue_flush();   // nothing of an earlier call may be issued from the scratch
    int dev = 0;
    ACR_HIP(hipGetDevice(&dev));
    char* base = scratch_on_device(dev);
    size_t need_work = 0, need_desc = 0;
    {   // planning pass: the memory the call takes, nothing issued
      NoAllocScope ns(base, true);
      h->f->solve(B, X, nrhs, st);
      need_work = ns.bump.off;
      need_desc = ns.ext.off;
    }
    if (need_work > kNoAllocWorkBytes || need_desc > kNoAllocDescBytes)
      fail(ACR_ERR_INVALID_ARG, "acr_solve_noalloc: this solve needs " + std::to_string(need_work >> 20) +
                                    " MiB of workspace and " + std::to_string(need_desc >> 10) +
                                    " KiB of descriptors; the maximum is " + std::to_string(kNoAllocWorkBytes >> 20) +
                                    " MiB and " + std::to_string(kNoAllocDescBytes >> 10) + " KiB (use acr_solve)");
    NoAllocScope ns(base, false);
    h->f->solve(B, X, nrhs, st);
    queue_flush();   // issue everything while the scratch is still the descriptor source
  });
}

acr_status acr_residual(const acr_operator* op, const double* X, const double* B, double* R,
                        int32_t nrhs, void* stream) {
  return guard([&] {
    check_op(op);
    if (!X || !B || !R || nrhs < 1) fail(ACR_ERR_INVALID_ARG, "bad vector arguments");
    StreamScope ss(static_cast<hipStream_t>(stream));
    stencil_residual(static_cast<hipStream_t>(stream), op->nx, op->ny, nrhs, op->diag, op->west, op->east,
                     op->south, op->north, X, B, R);
  });
}

acr_status acr_residual_3d(const acr_operator3d* op, const double* X, const double* B, double* R,
                           int32_t nrhs, void* stream) {
  return guard([&] {
    check_op3(op);
    if (!X || !B || !R || nrhs < 1) fail(ACR_ERR_INVALID_ARG, "bad vector arguments");
    StreamScope ss(static_cast<hipStream_t>(stream));
    const double* a7[7] = {op->diag, op->west, op->east, op->south, op->north, op->down, op->up};
    stencil_residual3d(static_cast<hipStream_t>(stream), op->nx, op->ny, op->nz, nrhs, a7, X, B, R);
  });
}

acr_status acr_solve_refined(acr_handle h, const acr_operator* op, const double* B, double* X,
                             int32_t nrhs, double tol, int32_t maxit, int32_t* iters, double* relres,
                             void* stream) {
  int its = 0;
  double rel = INFINITY;
  acr_status st0 = guard([&] {
    check_op(op);
    if (op->nx != (h ? h->nx : op->nx) || op->ny != (h ? h->ny : op->ny))
      fail(ACR_ERR_INVALID_ARG, "operator shape differs from the factor");
    hipStream_t st = static_cast<hipStream_t>(stream);
    refine_body(h, (long long)op->nx * op->ny, B, X, nrhs, tol, maxit, st, its, rel,
                [&](const double* x, const double* b, double* r, int nr) {
                  stencil_residual(st, op->nx, op->ny, nr, op->diag, op->west, op->east, op->south, op->north,
                                   x, b, r);
                });
  });
  if (iters) *iters = its;
  if (relres) *relres = rel;
  return st0;
}

acr_status acr_solve_refined_3d(acr_handle h, const acr_operator3d* op, const double* B, double* X,
                                int32_t nrhs, double tol, int32_t maxit, int32_t* iters, double* relres,
                                void* stream) {
  int its = 0;
  double rel = INFINITY;
  acr_status st0 = guard([&] {
    check_op3(op);
    if (h && (op->nx * op->ny != h->nx || op->nz != h->ny))
      fail(ACR_ERR_INVALID_ARG, "operator shape differs from the factor");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const double* a7[7] = {op->diag, op->west, op->east, op->south, op->north, op->down, op->up};
    refine_body(h, (long long)op->nx * op->ny * op->nz, B, X, nrhs, tol, maxit, st, its, rel,
                [&](const double* x, const double* b, double* r, int nr) {
                  stencil_residual3d(st, op->nx, op->ny, op->nz, nr, a7, x, b, r);
                });
  });
  if (iters) *iters = its;
  if (relres) *relres = rel;
  return st0;
}

acr_status acr_solve_krylov(acr_handle h, const acr_operator* op, const double* B, double* X, int32_t nrhs,
                            double tol, int32_t maxit, int32_t restart, int32_t* iters, double* relres,
                            void* stream) {
  int its = 0;
  double rel = 0.0;
  acr_status st0 = guard([&] {
    check_op(op);
    if (op->nx != (h ? h->nx : op->nx) || op->ny != (h ? h->ny : op->ny))
      fail(ACR_ERR_INVALID_ARG, "operator shape differs from the factor");
    hipStream_t st = static_cast<hipStream_t>(stream);
    krylov_body(h, (long long)op->nx * op->ny, B, X, nrhs, tol, maxit, restart, st, its, rel,
                [&](const double* x, const double* b, double* r) {
                  stencil_residual(st, op->nx, op->ny, 1, op->diag, op->west, op->east, op->south, op->north,
                                   x, b, r);
                });
  });
  if (iters) *iters = its;
  if (relres) *relres = rel;
  return st0;
}

acr_status acr_solve_krylov_3d(acr_handle h, const acr_operator3d* op, const double* B, double* X,
                               int32_t nrhs, double tol, int32_t maxit, int32_t restart, int32_t* iters,
                               double* relres, void* stream) {
  int its = 0;
  double rel = 0.0;
  acr_status st0 = guard([&] {
    check_op3(op);
    if (h && (op->nx * op->ny != h->nx || op->nz != h->ny))
      fail(ACR_ERR_INVALID_ARG, "operator shape differs from the factor");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const double* a7[7] = {op->diag, op->west, op->east, op->south, op->north, op->down, op->up};
    krylov_body(h, (long long)op->nx * op->ny * op->nz, B, X, nrhs, tol, maxit, restart, st, its, rel,
                [&](const double* x, const double* b, double* r) {
                  stencil_residual3d(st, op->nx, op->ny, op->nz, 1, a7, x, b, r);
                });
  });
  if (iters) *iters = its;
  if (relres) *relres = rel;
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
    StreamScope ss(static_cast<hipStream_t>(stream));
    h->f->block(level, which, k, dense, static_cast<hipStream_t>(stream));
  });
}

acr_status acr_destroy(acr_handle h) {
  return guard([&] {
    if (!h) return;
    (void)hipDeviceSynchronize();
    Pool::IdleScope idle;   // the factor's blocks are idle: any stream may reuse them
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
    for (auto& kv : P.paths()) out += "path\t" + kv.first + "\t" + std::to_string(kv.second) + "\n";
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

int64_t acr_launch_count(void) { return (int64_t)launch_count(); }

acr_status acr_set_solve_mode(int32_t mode, int64_t wait_limit) {
  return guard([&] {
    if (mode < 0 || mode > 3) fail(ACR_ERR_INVALID_ARG, "solve mode must be 0, 1, 2 or 3");
    SolveMode::get().mode = mode;
    SolveMode::get().limit = wait_limit == 0 ? (1LL << 22) : wait_limit;
  });
}

acr_status acr_tune_record(int32_t on) {
  return guard([&] { Tuner::get().recording = on != 0; });
}

acr_status acr_tune_run(void* stream, int32_t* added) {
  return guard([&] {
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamScope ss(st);
    const int n = tune_run(st);
    if (added) *added = n;
  });
}

acr_status acr_tune_enable(int32_t on) {
  return guard([&] { Tuner::get().active = on != 0; });
}

acr_status acr_tune_save(const char* path) {
  return guard([&] {
    if (!path) fail(ACR_ERR_INVALID_ARG, "NULL path");
    Tuner& t = Tuner::get();
    std::string out = "{\n  \"arch\": \"" + device_arch() + "\",\n  \"entries\": {";
    {
      std::lock_guard<std::mutex> g(t.mu);
      bool first = true;
      for (auto& kv : t.table) {
        out += std::string(first ? "\n" : ",\n") + "    \"" + kv.first + "\": " + std::to_string(kv.second);
        first = false;
      }
    }
    out += "\n  }\n}\n";
    FILE* f = std::fopen(path, "w");
    if (!f) fail(ACR_ERR_INVALID_ARG, std::string("cannot write ") + path);
    const size_t w = std::fwrite(out.data(), 1, out.size(), f);
    std::fclose(f);
    if (w != out.size()) fail(ACR_ERR_INVALID_ARG, std::string("short write to ") + path);
  });
}

acr_status acr_tune_load(const char* path) {
  return guard([&] {
    if (!path) fail(ACR_ERR_INVALID_ARG, "NULL path");
    FILE* f = std::fopen(path, "r");
    if (!f) fail(ACR_ERR_INVALID_ARG, std::string("cannot read ") + path);
    std::string txt;
    char buf[4096];
    size_t r;
    while ((r = std::fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, r);
    std::fclose(f);
    // a flat JSON object: "arch": "<name>", "entries": {"<key>": <int>, ...}
    auto str_after = [&](size_t pos, size_t* end) {
      const size_t a = txt.find('"', pos);
      const size_t b = a == std::string::npos ? a : txt.find('"', a + 1);
      if (b == std::string::npos) fail(ACR_ERR_INVALID_ARG, "malformed tuning file");
      *end = b + 1;
      return txt.substr(a + 1, b - a - 1);
    };
    const size_t ka = txt.find("\"arch\"");
    if (ka == std::string::npos) fail(ACR_ERR_INVALID_ARG, "tuning file without \"arch\"");
    size_t e = 0;
    const std::string arch = str_after(txt.find(':', ka) + 1, &e);
    if (arch != device_arch())
      fail(ACR_ERR_INVALID_ARG, "tuning file is for " + arch + ", this device is " + device_arch());
    const size_t ke = txt.find("\"entries\"");
    if (ke == std::string::npos) fail(ACR_ERR_INVALID_ARG, "tuning file without \"entries\"");
    size_t pos = txt.find('{', ke);
    const size_t close = txt.find('}', pos);
    if (pos == std::string::npos || close == std::string::npos) fail(ACR_ERR_INVALID_ARG, "malformed tuning file");
    std::map<std::string, int> table;
    for (;;) {
      const size_t q = txt.find('"', pos);
      if (q == std::string::npos || q > close) break;
      const std::string key = str_after(q, &e);
      const size_t colon = txt.find(':', e);
      if (colon == std::string::npos || colon > close) fail(ACR_ERR_INVALID_ARG, "malformed tuning file");
      table[key] = std::atoi(txt.c_str() + colon + 1);
      pos = colon + 1;
    }
    Tuner& t = Tuner::get();
    std::lock_guard<std::mutex> g(t.mu);
    t.table.swap(table);
    t.active = true;
  });
}

acr_status acr_tune_clear(void) {
  return guard([&] {
    Tuner& t = Tuner::get();
    std::lock_guard<std::mutex> g(t.mu);
    t.table.clear();
    t.seen.clear();
    t.active = false;
  });
}

acr_status acr_trim_pool(void) {
  return guard([&] { Pool::get().trim(); });
}

acr_status acr_set_allocator(void* (*alloc_fn)(size_t, void*), void (*free_fn)(void*, void*)) {
  return guard([&] {
    if ((alloc_fn == nullptr) != (free_fn == nullptr))
      fail(ACR_ERR_INVALID_ARG, "give both callbacks or neither");
    queue_flush();
    Profiler::get().start(0);   // drops the profiler's device buffers (and its records)
    Pool& P = Pool::get();
    if (P.live() != 0) fail(ACR_ERR_INVALID_ARG, "the library holds live device memory (destroy every handle first)");
    ACR_HIP(hipDeviceSynchronize());
    P.release_all_cached();
    Allocator::get().alloc = alloc_fn;
    Allocator::get().free = free_fn;
  });
}

}  // extern "C"
