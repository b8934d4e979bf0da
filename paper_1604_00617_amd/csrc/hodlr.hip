// H-arithmetic on batched HODLR sets, planned as grouped launches: every
// operation below collects the independent batched problems of all clusters,
// depths and operands it needs into a few job lists and launches each list
// once (see kernels.hpp for the job kinds).
#include "hodlr.hpp"

#include <algorithm>

namespace acr {

Work& work() {
  static thread_local Work w;
  return w;
}

// ------------------------------------------------------------------ HSet
template <typename T>
void HSet<T>::alloc(hipStream_t st, int cnt_, int s_, int b_, int L_, const std::vector<int>& k_,
                    int zero_from) {
  cnt = cnt_; s = s_; b = b_; L = L_;
  k.assign(L + 1, 0);
  kc.assign(L + 1, 0);
  rsum.assign(L + 1, -1.0);
  for (int d = 1; d <= L; ++d) k[d] = d < (int)k_.size() ? k_[d] : 0;
  lv.resize((size_t)cnt * leaf_stride());
  U.clear(); V.clear();
  U.resize(L + 1); V.resize(L + 1);
  for (int d = 1; d <= L; ++d) {
    U[d].resize((size_t)cnt * k[d] * s);
    V[d].resize((size_t)cnt * k[d] * s);
  }
  if (zero_from >= 0 && zero_from < cnt) {   // matrices [zero_from, cnt) start as zeros
    const size_t nz = (size_t)(cnt - zero_from);
    memset_async(lv.get() + (size_t)zero_from * leaf_stride(), 0, nz * leaf_stride() * sizeof(T), st);
    for (int d = 1; d <= L; ++d) {
      const size_t per = (size_t)k[d] * s;
      memset_async(U[d].get() + (size_t)zero_from * per, 0, nz * per * sizeof(T), st);
      memset_async(V[d].get() + (size_t)zero_from * per, 0, nz * per * sizeof(T), st);
    }
  }
}

template <typename T>
size_t HSet<T>::bytes() const {
  size_t t = (size_t)cnt * leaf_stride() * sizeof(T);
  for (int d = 1; d <= L; ++d) t += 2 * (size_t)cnt * kc[d] * s * sizeof(T);
  return t;
}

template <typename T>
double HSet<T>::bytes_ranked() const {
  // depth d: 2^d blocks per matrix of sd = s/2^d rows each, U and V
  double t = (double)cnt * leaf_stride() * sizeof(T);
  for (int d = 1; d <= L; ++d) t += 2.0 * rank_sum(d) * sd(d) * sizeof(T);
  return t;
}

template <typename T>
int HSet<T>::max_rank() const {
  int r = 0;
  for (int d = 1; d <= L; ++d) r = std::max(r, kc[d]);
  return r;
}

// ------------------------------------------------------------- operands
namespace {

template <typename T>
BOp leaves_op(HV<T> H) {
  BOp o = bop(H.h->lv.get(), H.h->b, H.h->leaf_stride(), (long long)H.h->b * H.h->b);
  return with_map(o, H.mmul, H.moff);
}

// Depth-d factor (U or V) of a set as a flat operand; cluster stride = rows sc.
template <typename T>
BOp factor_op(HV<T> H, const DBuf<T>& F, int d, long long sc) {
  BOp o = bop(F.get(), H.h->s, (long long)H.h->k[d] * H.h->s, sc);
  return with_map(o, H.mmul, H.moff);
}

template <typename T>
Flat<T> flat_set(HV<T> H, const DBuf<T>& F, int d) {
  Flat<T> f;
  f.p = F.get();
  f.ld = H.h->s;
  f.sm = (long long)H.h->k[d] * H.h->s;
  f.mmul = H.mmul;
  f.moff = H.moff;
  return f;
}

GSeg seg(const BOp& A, const BOp& B, int K, double scale = 1.0) {
  GSeg g;
  g.A = A; g.B = B; g.K = K; g.scale = scale;
  return g;
}

CJob copy_job(int rows, int cols, int nmat, double alpha, const BOp& src, const BOp& dst,
              int ncl = 1, int accumulate = 0) {
  CJob J;
  J.rows = rows; J.cols = cols; J.nmat = nmat; J.ncl = ncl; J.alpha = alpha;
  J.src = src; J.dst = dst; J.accumulate = accumulate;
  return J;
}

}  // namespace

template <typename T>
BOp flat_op(const Flat<T>& f, long long sc, int col0) {
  BOp o = bop(f.p + (long long)col0 * f.ld, f.ld, f.sm, sc);
  return with_map(o, f.mmul, f.moff);
}

// ------------------------------------------------------------- GemmPlan
void GemmPlan::add(int M, int N, int nmat, int ncl, double alpha, double beta, const BOp& C,
                   const std::vector<GSeg>& sg) {
  if (M <= 0 || N <= 0 || nmat <= 0 || ncl <= 0 || sg.empty()) return;
  if ((int)sg.size() > kMaxSeg) fail(ACR_ERR_INTERNAL, "too many GEMM segments");
  GJob J;
  J.M = M; J.N = N; J.nmat = nmat; J.ncl = ncl; J.alpha = alpha; J.beta = beta; J.C = C;
  J.seg0 = (int)segs.size();
  J.nseg = (int)sg.size();
  double K = 0;
  for (const auto& g : sg) {
    segs.push_back(g);
    K += g.K;
  }
  work().gemm_flops += 2.0 * M * N * K * nmat * ncl;
  jobs.push_back(J);
}

template <typename T>
void GemmPlan::run(hipStream_t st) {
  if (!jobs.empty()) ggemm<T>(st, jobs, segs);
  jobs.clear();
  segs.clear();
}

// ------------------------------------------------------------------- hmul
template <typename T>
std::vector<GSeg> plan_hmul(GemmPlan& red, std::vector<DBuf<T>>& keep, HV<T> H, int nmat,
                            int dfrom, bool trans, int ncol, double alpha, Flat<T> Y) {
  const HSet<T>& h = *H.h;
  const int b = h.b, L = h.L;
  std::vector<GSeg> out;
  BOp A = leaves_op(H);
  A.trans = trans ? 1 : 0;
  out.push_back(seg(A, flat_op(Y, b), b, alpha));
  for (int d = std::max(dfrom + 1, 1); d <= L; ++d) {
    const int w = h.kc[d];
    if (w == 0) continue;
    const int ncl = 1 << d, sd = h.sd(d);
    keep.emplace_back((size_t)nmat * ncl * w * ncol);
    // T_d[c] = F_d[rows c]^T Y[rows c]   (F = V, or U for the transpose)
    BOp Tc = bop(keep.back().get(), w, (long long)ncl * w * ncol, (long long)w * ncol);
    red.add(w, ncol, nmat, ncl, 1.0, 0.0, Tc,
            {seg(transposed(factor_op(H, trans ? h.U[d] : h.V[d], d, sd)), flat_op(Y, sd), sd)});
    // rows of leaf l: G_d[rows l] T_d[sibling of the depth-d ancestor of l]
    out.push_back(seg(factor_op(H, trans ? h.V[d] : h.U[d], d, b), ancestor(Tc, L - d, 1), w, alpha));
  }
  return out;
}

template <typename T>
void hmul(hipStream_t st, HV<T> H, int nmat, int dfrom, bool trans, int ncol, T alpha, Flat<T> Y,
          T beta, Flat<T> out) {
  if (nmat <= 0 || ncol <= 0) return;
  GemmPlan red, exp;
  std::vector<DBuf<T>> keep;
  auto sg = plan_hmul<T>(red, keep, H, nmat, dfrom, trans, ncol, (double)alpha, Y);
  exp.add(H.h->b, ncol, nmat, H.h->nleaf(), 1.0, (double)beta, flat_op(out, H.h->b), sg);
  red.run<T>(st);
  exp.run<T>(st);
}

// ------------------------------------------------------------ hprod_multi
// For every output C = D + sum_t coef_t A_t B_t (exact low-rank accumulation):
//   depth-d block of A B = A[t,t] B[t,s] + A[t,s] B[s,s] + ancestor terms
//                        = (Adiag_{>d} U^B_d) V^B_d^T + U^A_d (Bdiag_{>d}^T V^A_d)^T + ...
// The products Adiag_{>d} U^B_d of all depths d are one pass over A's leaves:
// with Y = [U^B_1 | ... | U^B_L] (column block d), the depth-e reduction
// T_e = V^A_e[cl]^T Y[cl] is kept only for the column blocks d < e (the rest
// stays zero), and out = leaves(A) Y + sum_e U^A_e[rows] T_e[sibling ancestor]
// holds every Adiag_{>d} U^B_d in its column block d.  Same for the
// transposed side.  Stages: copies in, reductions + cores, ancestor parts,
// expansions + leaves, copies out.
template <typename T>
void hprod_multi(hipStream_t st, std::vector<POut<T>>& outs) {
  GemmPlan s1, s2, s3;
  // copies: cin = everything that reads only the operands (stacked inputs,
  // and the parts of C taken over unchanged), before the products; cout =
  // everything that reads products (ancestor parts, expanded factors), after
  std::vector<CJob> cin, cout;
  std::vector<DBuf<T>> keep;
  struct Anc {
    int w = 0;
    const T* up = nullptr;
    long long ups = 0;
    int upm = 1, upo = 0;
    const T* vp = nullptr;
    long long vps = 0;
    int vpm = 1, vpo = 0;
  };
  // reduction outputs of all terms live in one zero-initialised buffer
  size_t tsize = 0;
  for (auto& O : outs) {
    const HSet<T>& g = O.terms.empty() ? *O.D.h : *O.terms[0].A.h;
    for (auto& tm : O.terms) {
      int NA = 0, NB = 0;
      for (int d = 1; d <= g.L; ++d) { NA += tm.A.h->kc[d]; NB += tm.B.h->kc[d]; }
      for (int e = 1; e <= g.L; ++e)
        tsize += (size_t)O.nmat * ((size_t)1 << e) * ((size_t)tm.A.h->kc[e] * NB + (size_t)tm.B.h->kc[e] * NA);
    }
  }
  DBuf<T> tbuf(tsize);
  memset_async(tbuf.get(), 0, tsize * sizeof(T), st);
  size_t toff = 0;
  for (auto& O : outs) {
    const int nmat = O.nmat;
    const HSet<T>& g = O.terms.empty() ? *O.D.h : *O.terms[0].A.h;
    const int L = g.L, s = g.s, b = g.b, nleaf = g.nleaf();
    std::vector<std::vector<Anc>> anc(O.terms.size(), std::vector<Anc>(L + 1));
    std::vector<const T*> outA(O.terms.size(), nullptr), outB(O.terms.size(), nullptr);
    std::vector<std::vector<int>> cAo(O.terms.size()), cBo(O.terms.size());
    for (size_t t = 0; t < O.terms.size(); ++t) {
      const double coef = O.terms[t].coef;
      const HV<T> A = O.terms[t].A, B = O.terms[t].B;
      const HSet<T>& a = *A.h;
      const HSet<T>& bb = *B.h;
      // ancestor terms (see the block comment above)
      for (int d = 1; d <= L; ++d) {
        const int kA = a.kc[d], kB = bb.kc[d];
        if (kA == 0 || kB == 0) continue;
        const int ncl = 1 << d, sd = g.sd(d);
        keep.emplace_back((size_t)nmat * ncl * kA * kB);
        BOp Wc = bop(keep.back().get(), kA, (long long)ncl * kA * kB, (long long)kA * kB);
        s1.add(kA, kB, nmat, ncl, 1.0, 0.0, Wc,
               {seg(transposed(factor_op(A, a.V[d], d, sd)), factor_op(B, bb.U[d], d, sd), sd)});
        Anc& an = anc[t][d];
        if (kB <= kA) {
          keep.emplace_back((size_t)nmat * kB * s);
          s2.add(sd, kB, nmat, ncl, 1.0, 0.0, bop(keep.back().get(), s, (long long)kB * s, sd),
                 {seg(factor_op(A, a.U[d], d, sd), swapped(Wc), kA)});
          an.w = kB;
          an.up = keep.back().get(); an.ups = (long long)kB * s; an.upm = 1; an.upo = 0;
          an.vp = bb.V[d].get(); an.vps = (long long)bb.k[d] * s; an.vpm = B.mmul; an.vpo = B.moff;
        } else {
          keep.emplace_back((size_t)nmat * kA * s);
          s2.add(sd, kA, nmat, ncl, 1.0, 0.0, bop(keep.back().get(), s, (long long)kA * s, sd),
                 {seg(factor_op(B, bb.V[d], d, sd), transposed(swapped(Wc)), kB)});
          an.w = kA;
          an.up = a.U[d].get(); an.ups = (long long)a.k[d] * s; an.upm = A.mmul; an.upo = A.moff;
          an.vp = keep.back().get(); an.vps = (long long)kA * s; an.vpm = 1; an.vpo = 0;
        }
      }
      // stacked inputs Y = [U^B_1 | ... | U^B_L], Y' = [V^A_1 | ... | V^A_L]
      std::vector<int>& cB = cBo[t];
      std::vector<int>& cA = cAo[t];
      cB.assign(L + 2, 0);
      cA.assign(L + 2, 0);
      for (int d = 1; d <= L; ++d) { cB[d + 1] = cB[d] + bb.kc[d]; cA[d + 1] = cA[d] + a.kc[d]; }
      const int NB = cB[L + 1], NA = cA[L + 1];
      if (NB > 0) {
        keep.emplace_back((size_t)nmat * NB * s);
        T* Y = keep.back().get();
        for (int d = 1; d <= L; ++d)
          if (bb.kc[d])
            cin.push_back(copy_job(s, bb.kc[d], nmat, 1.0, factor_op(B, bb.U[d], d, 0),
                                   bop(Y + (size_t)cB[d] * s, s, (long long)NB * s)));
        keep.emplace_back((size_t)nmat * NB * s);
        T* Oa = keep.back().get();
        outA[t] = Oa;
        // reductions: T_e = V^A_e[cl]^T Y[cl] on the column blocks d < e
        BOp leafA = leaves_op(A);
        std::vector<GSeg> ex{seg(leafA, bop(Y, s, (long long)NB * s, b), b, coef)};
        for (int e = 1; e <= L; ++e) {
          const int w = a.kc[e];
          const int ncl = 1 << e, sd = g.sd(e);
          if (w == 0) continue;
          T* Te = tbuf.get() + toff;
          toff += (size_t)nmat * ncl * w * NB;
          BOp Tc = bop(Te, w, (long long)ncl * w * NB, (long long)w * NB);
          if (cB[e] > 0)
            s1.add(w, cB[e], nmat, ncl, 1.0, 0.0, Tc,
                   {seg(transposed(factor_op(A, a.V[e], e, sd)), bop(Y, s, (long long)NB * s, sd), sd)});
          ex.push_back(seg(factor_op(A, a.U[e], e, b), ancestor(Tc, L - e, 1), w, coef));
        }
        s3.add(b, NB, nmat, nleaf, 1.0, 0.0, bop(Oa, s, (long long)NB * s, b), ex);
      }
      if (NA > 0) {
        keep.emplace_back((size_t)nmat * NA * s);
        T* Y = keep.back().get();
        for (int d = 1; d <= L; ++d)
          if (a.kc[d])
            cin.push_back(copy_job(s, a.kc[d], nmat, 1.0, factor_op(A, a.V[d], d, 0),
                                   bop(Y + (size_t)cA[d] * s, s, (long long)NA * s)));
        keep.emplace_back((size_t)nmat * NA * s);
        T* Ob = keep.back().get();
        outB[t] = Ob;
        BOp leafB = leaves_op(B);
        leafB.trans = 1;
        std::vector<GSeg> ex{seg(leafB, bop(Y, s, (long long)NA * s, b), b, 1.0)};
        for (int e = 1; e <= L; ++e) {
          const int w = bb.kc[e];
          const int ncl = 1 << e, sd = g.sd(e);
          if (w == 0) continue;
          T* Te = tbuf.get() + toff;
          toff += (size_t)nmat * ncl * w * NA;
          BOp Tc = bop(Te, w, (long long)ncl * w * NA, (long long)w * NA);
          if (cA[e] > 0)
            s1.add(w, cA[e], nmat, ncl, 1.0, 0.0, Tc,
                   {seg(transposed(factor_op(B, bb.U[e], e, sd)), bop(Y, s, (long long)NA * s, sd), sd)});
          ex.push_back(seg(factor_op(B, bb.V[e], e, b), ancestor(Tc, L - e, 1), w, 1.0));
        }
        s3.add(b, NA, nmat, nleaf, 1.0, 0.0, bop(Ob, s, (long long)NA * s, b), ex);
      }
    }
    std::vector<int> kC(L + 1, 0);
    for (int d = 1; d <= L; ++d) {
      if (O.has_d) kC[d] += O.D.h->kc[d];
      for (size_t t = 0; t < O.terms.size(); ++t) {
        kC[d] += O.terms[t].A.h->kc[d] + O.terms[t].B.h->kc[d];
        for (int e = 1; e < d; ++e) kC[d] += anc[t][e].w;
      }
    }
    HSet<T>& C = *O.C;
    C.alloc(st, O.cnt_alloc, s, b, L, kC, O.cnt_alloc > nmat ? nmat : -1);
    for (int d = 1; d <= L; ++d) {
      int col = 0;
      auto cu = [&](int c0) { return bop(C.U[d].get() + (size_t)c0 * s, s, (long long)C.k[d] * s); };
      auto cv = [&](int c0) { return bop(C.V[d].get() + (size_t)c0 * s, s, (long long)C.k[d] * s); };
      if (O.has_d && O.D.h->kc[d]) {
        const int w = O.D.h->kc[d];
        cin.push_back(copy_job(s, w, nmat, 1.0, factor_op(O.D, O.D.h->U[d], d, 0), cu(col)));
        cin.push_back(copy_job(s, w, nmat, 1.0, factor_op(O.D, O.D.h->V[d], d, 0), cv(col)));
        col += w;
      }
      for (size_t t = 0; t < O.terms.size(); ++t) {
        const double coef = O.terms[t].coef;
        const HV<T> A = O.terms[t].A, B = O.terms[t].B;
        const HSet<T>& a = *A.h;
        const HSet<T>& bb = *B.h;
        const int kA = a.kc[d], kB = bb.kc[d];
        if (kB > 0) {   // (Adiag U^B) V^B^T: column block d of the A-side pass
          const int NB = cBo[t][L + 1];
          cout.push_back(copy_job(s, kB, nmat, 1.0, bop(outA[t] + (size_t)cBo[t][d] * s, s, (long long)NB * s), cu(col)));
          cin.push_back(copy_job(s, kB, nmat, 1.0, factor_op(B, bb.V[d], d, 0), cv(col)));
          col += kB;
        }
        if (kA > 0) {   // U^A (Bdiag^T V^A)^T: column block d of the transposed pass
          const int NA = cAo[t][L + 1];
          cin.push_back(copy_job(s, kA, nmat, coef, factor_op(A, a.U[d], d, 0), cu(col)));
          cout.push_back(copy_job(s, kA, nmat, 1.0, bop(outB[t] + (size_t)cAo[t][d] * s, s, (long long)NA * s), cv(col)));
          col += kA;
        }
        for (int e = 1; e < d; ++e) {
          const Anc& an = anc[t][e];
          if (!an.w) continue;
          cout.push_back(copy_job(s, an.w, nmat, coef, with_map(bop(an.up, s, an.ups), an.upm, an.upo), cu(col)));
          cout.push_back(copy_job(s, an.w, nmat, 1.0, with_map(bop(an.vp, s, an.vps), an.vpm, an.vpo), cv(col)));
          col += an.w;
        }
      }
      C.kc[d] = col;
    }
    // leaves: C_l = D_l + sum_t coef_t (A_l B_l + sum_e Upart_e[l] Vpart_e[l]^T)
    std::vector<GSeg> ls;
    for (size_t t = 0; t < O.terms.size(); ++t) {
      const double coef = O.terms[t].coef;
      ls.push_back(seg(leaves_op(O.terms[t].A), leaves_op(O.terms[t].B), b, coef));
      for (int e = 1; e <= L; ++e) {
        const Anc& an = anc[t][e];
        if (!an.w) continue;
        ls.push_back(seg(with_map(bop(an.up, s, an.ups, b), an.upm, an.upo),
                         with_map(bop(an.vp, s, an.vps, b, 1), an.vpm, an.vpo), an.w, coef));
      }
    }
    const BOp CL = bop(C.lv.get(), b, C.leaf_stride(), (long long)b * b);
    if (O.has_d)
      cin.push_back(copy_job((int)O.D.h->leaf_stride(), 1, nmat, 1.0,
                              with_map(bop(O.D.h->lv.get(), 1, O.D.h->leaf_stride()), O.D.mmul, O.D.moff),
                              bop(C.lv.get(), 1, C.leaf_stride())));
    if (!ls.empty()) s3.add(b, b, nmat, nleaf, 1.0, O.has_d ? 1.0 : 0.0, CL, ls);
  }
  gcopy<T>(st, cin);
  s1.run<T>(st);
  s2.run<T>(st);
  s3.run<T>(st);
  gcopy<T>(st, cout);
  Queue::get().flush();   // let the device start while the host plans the next step
}

// ------------------------------------------------------------------- hinv
template <typename T>
void hinv_multi(hipStream_t st, std::vector<HInvJob<T>>& jobs) {
  std::vector<HInvJob<T>> js;
  for (auto& J : jobs)
    if (J.nmat > 0) js.push_back(J);
  if (js.empty()) return;
  int maxL = 0;
  {
    std::vector<CJob> cp;
    std::vector<IJob> ij;
    for (auto& J : js) {
      const HSet<T>& mm = *J.M.h;
      const int L = mm.L, s = mm.s, b = mm.b, nleaf = mm.nleaf();
      maxL = std::max(maxL, L);
      std::vector<int> kX(L + 1, 0);
      for (int d = 1; d <= L; ++d)
        for (int e = 1; e <= d; ++e) kX[d] += mm.kc[e];
      J.X->alloc(st, J.nmat, s, b, L, kX, -1);
      // leaves: X_l = M_l^{-1}
      cp.push_back(copy_job((int)mm.leaf_stride(), 1, J.nmat, 1.0,
                            with_map(bop(mm.lv.get(), 1, mm.leaf_stride()), J.M.mmul, J.M.moff),
                            bop(J.X->lv.get(), 1, J.X->leaf_stride())));
      IJob I;
      I.n = b; I.nprob = J.nmat * nleaf; I.A = J.X->lv.get(); I.sA = (long long)b * b;
      I.X = J.X->lv.get(); I.sX = (long long)b * b; I.status = J.status;
      ij.push_back(I);
      work().inv_flops += 2.0 * b * b * b * J.nmat * nleaf;
    }
    gcopy<T>(st, cp);
    ginverse<T, T>(st, ij);
  }
  // Sherman-Morrison-Woodbury, bottom-up: step i handles depth L - i of every tree
  for (int step = 0; step < maxL; ++step) {
    struct Part {
      HInvJob<T>* J;
      int d, k, ncl, sd;
      DBuf<T> abuf, bbuf, wbuf, cores, G;
    };
    std::vector<Part> parts;
    for (auto& J : js) {
      const int d = J.M.h->L - step;
      if (d < 1) continue;
      const int k = J.M.h->kc[d];
      if (k == 0) continue;
      Part pt;
      pt.J = &J; pt.d = d; pt.k = k; pt.ncl = 1 << d; pt.sd = J.M.h->sd(d);
      parts.push_back(std::move(pt));
    }
    if (parts.empty()) continue;
    std::vector<DBuf<T>> keep;
    GemmPlan red, exp;
    for (auto& pt : parts) {
      const HInvJob<T>& J = *pt.J;
      const HSet<T>& mm = *J.M.h;
      const int s = mm.s, b = mm.b, nleaf = mm.nleaf(), k = pt.k, d = pt.d, nmat = J.nmat;
      pt.abuf.resize((size_t)nmat * k * s);
      pt.bbuf.resize((size_t)nmat * k * s);
      pt.wbuf.resize((size_t)nmat * k * s);
      Flat<T> fa; fa.p = pt.abuf.get(); fa.ld = s; fa.sm = (long long)k * s;
      Flat<T> fb; fb.p = pt.bbuf.get(); fb.ld = s; fb.sm = (long long)k * s;
      // a = Xdiag U^M (children inverses applied), bb = Xdiag^T V^M
      HV<T> XV{J.X, 1, 0};
      auto sa = plan_hmul<T>(red, keep, XV, nmat, d, false, k, 1.0, flat_set(J.M, mm.U[d], d));
      auto sb = plan_hmul<T>(red, keep, XV, nmat, d, true, k, 1.0, flat_set(J.M, mm.V[d], d));
      exp.add(b, k, nmat, nleaf, 1.0, 0.0, flat_op(fa, b), sa);
      exp.add(b, k, nmat, nleaf, 1.0, 0.0, flat_op(fb, b), sb);
    }
    red.run<T>(st);
    exp.run<T>(st);
    // cores c_sigma = V^M[sigma]^T a[sigma]
    GemmPlan cp;
    for (auto& pt : parts) {
      const HInvJob<T>& J = *pt.J;
      const HSet<T>& mm = *J.M.h;
      const int s = mm.s, k = pt.k, d = pt.d, nmat = J.nmat, ncl = pt.ncl;
      Flat<T> fa; fa.p = pt.abuf.get(); fa.ld = s; fa.sm = (long long)k * s;
      pt.cores.resize((size_t)nmat * ncl * k * k);
      cp.add(k, k, nmat, ncl, 1.0, 0.0, bop(pt.cores.get(), k, (long long)ncl * k * k, (long long)k * k),
             {seg(transposed(factor_op(J.M, mm.V[d], d, pt.sd)), flat_op(fa, pt.sd), pt.sd)});
      const int npairs = nmat * ncl / 2, n2 = 2 * k;
      pt.G.resize((size_t)npairs * n2 * n2);
    }
    cp.run<T>(st);
    {   // G_q^{-1}, with G_q = [[I, c_(2q+1)], [c_(2q), I]] formed from the cores as it is read
      std::vector<IJob> ij;
      for (auto& pt : parts) {
        const int npairs = pt.J->nmat * pt.ncl / 2, n2 = 2 * pt.k;
        IJob I;
        I.n = n2; I.nprob = npairs; I.A = nullptr; I.sA = (long long)n2 * n2;
        I.cap_k = pt.k; I.cores = pt.cores.get();
        I.X = pt.G.get(); I.sX = (long long)n2 * n2; I.status = pt.J->status;
        ij.push_back(I);
        work().inv_flops += 2.0 * n2 * n2 * n2 * npairs;
      }
      ginverse<T, T>(st, ij);
    }
    GemmPlan gp, lp;
    std::vector<CJob> cj;
    for (auto& pt : parts) {
      HInvJob<T>& J = *pt.J;
      HSet<T>& X = *J.X;
      const HSet<T>& mm = *J.M.h;
      const int s = mm.s, b = mm.b, L = mm.L, nleaf = mm.nleaf(), k = pt.k, d = pt.d, nmat = J.nmat, ncl = pt.ncl;
      const int n2 = 2 * k;
      Flat<T> fa; fa.p = pt.abuf.get(); fa.ld = s; fa.sm = (long long)k * s;
      Flat<T> fw; fw.p = pt.wbuf.get(); fw.ld = s; fw.sm = (long long)k * s;
      // diagonal block of G^{-1} for cluster t: (t&1) selects (0,0) or (1,1)
      BOp Gd;
      Gd.p = pt.G.get(); Gd.ld = n2; Gd.sm = (long long)(ncl / 2) * n2 * n2;
      Gd.sc_pair = (long long)n2 * n2; Gd.sc_odd = (long long)k + (long long)k * n2;
      BOp Go = Gd;
      Go.p = pt.G.get() + (size_t)k * n2;              // (0,1) block for a first child
      Go.sc_odd = (long long)k - (long long)k * n2;    // (1,0) block for a second child
      // U^X_d = -a[t] Gdiag(t);  W = a[t] Goff(t)
      gp.add(pt.sd, k, nmat, ncl, -1.0, 0.0, bop(X.U[d].get(), s, (long long)X.k[d] * s, pt.sd),
             {seg(flat_op(fa, pt.sd), Gd, k)});
      gp.add(pt.sd, k, nmat, ncl, 1.0, 0.0, flat_op(fw, pt.sd), {seg(flat_op(fa, pt.sd), Go, k)});
      // V^X_d = bb; X[t,t] -= W[t] bb[t]^T pushed to every depth below d
      cj.push_back(copy_job(s, k, nmat, 1.0, bop(pt.bbuf.get(), s, (long long)k * s),
                            bop(X.V[d].get(), s, (long long)X.k[d] * s)));
      X.kc[d] = k;
      for (int e = d + 1; e <= L; ++e) {
        cj.push_back(copy_job(s, k, nmat, -1.0, bop(pt.wbuf.get(), s, (long long)k * s),
                              bop(X.U[e].get() + (size_t)X.kc[e] * s, s, (long long)X.k[e] * s)));
        cj.push_back(copy_job(s, k, nmat, 1.0, bop(pt.bbuf.get(), s, (long long)k * s),
                              bop(X.V[e].get() + (size_t)X.kc[e] * s, s, (long long)X.k[e] * s)));
        X.kc[e] += k;
      }
      lp.add(b, b, nmat, nleaf, 1.0, 1.0, bop(X.lv.get(), b, X.leaf_stride(), (long long)b * b),
             {seg(bop(pt.wbuf.get(), s, (long long)k * s, b), bop(pt.bbuf.get(), s, (long long)k * s, b, 1), k, -1.0)});
    }
    gp.run<T>(st);
    gcopy<T>(st, cj);
    lp.run<T>(st);
  }
  Queue::get().flush();   // let the device start while the host plans the next step
}

template <typename T>
void hinv(hipStream_t st, HSet<T>& X, HV<T> M, int nmat, int* status) {
  std::vector<HInvJob<T>> js{HInvJob<T>{&X, M, nmat, status}};
  hinv_multi<T>(st, js);
}

// ------------------------------------------------------------- level 0
template <typename T>
void hstack_multi(hipStream_t st, std::vector<StackOut<T>>& outs) {
  // the first term of every output is a plain (scaled) copy; every further
  // term accumulates into the leaves, one launch per term index so that the
  // accumulations of one output are ordered
  std::vector<CJob> first;
  std::vector<std::vector<CJob>> rest;
  for (auto& O : outs) {
    if (O.terms.empty()) continue;
    const HSet<T>& h0 = *O.terms[0].h.h;
    const int L = h0.L, s = h0.s, b = h0.b, nmat = O.nmat;
    std::vector<int> kC(L + 1, 0);
    for (const auto& t : O.terms)
      for (int d = 1; d <= L; ++d) kC[d] += t.h.h->kc[d];
    HSet<T>& C = *O.C;
    C.alloc(st, O.cnt_alloc, s, b, L, kC, O.cnt_alloc > nmat ? nmat : -1);
    const long long ls = C.leaf_stride();
    std::vector<int> col(L + 1, 0);
    for (size_t ti = 0; ti < O.terms.size(); ++ti) {
      const auto& t = O.terms[ti];
      const HSet<T>& h = *t.h.h;
      // leaves (rows of leaf c are rows c*b.. of the scale vector)
      CJob lj = copy_job(b, b, nmat, t.coef, leaves_op(t.h), bop(C.lv.get(), b, ls, (long long)b * b), h.nleaf(),
                         ti > 0 ? 1 : 0);
      if (t.rows) { lj.scale = t.rows; lj.smul = t.rmul; lj.soff = t.roff; lj.sstride = s; lj.scl = b; lj.sside = 0; }
      if (ti == 0) first.push_back(lj);
      else {
        if (rest.size() < ti) rest.resize(ti);
        rest[ti - 1].push_back(lj);
      }
      for (int d = 1; d <= L; ++d) {
        const int w = h.kc[d];
        if (!w) continue;
        CJob uj = copy_job(s, w, nmat, t.coef, factor_op(t.h, h.U[d], d, 0),
                           bop(C.U[d].get() + (size_t)col[d] * s, s, (long long)C.k[d] * s));
        if (t.rows) { uj.scale = t.rows; uj.smul = t.rmul; uj.soff = t.roff; uj.sstride = s; uj.scl = 0; uj.sside = 0; }
        first.push_back(uj);
        first.push_back(copy_job(s, w, nmat, 1.0, factor_op(t.h, h.V[d], d, 0),
                                 bop(C.V[d].get() + (size_t)col[d] * s, s, (long long)C.k[d] * s)));
        col[d] += w;
      }
    }
    for (int d = 1; d <= L; ++d) C.kc[d] = col[d];
  }
  gcopy<T>(st, first);
  for (auto& r : rest) gcopy<T>(st, r);
  Queue::get().flush();   // let the device start while the host plans the next step
}

template <typename T>
void hscale_cols_multi(hipStream_t st, std::vector<ColScale<T>>& outs) {
  std::vector<CJob> cj;
  for (auto& O : outs) {
    const HSet<T>& h = *O.H.h;
    const int L = h.L, s = h.s, b = h.b, nmat = O.nmat;
    std::vector<int> kC(L + 1, 0);
    for (int d = 1; d <= L; ++d) kC[d] = h.kc[d];
    HSet<T>& C = *O.C;
    C.alloc(st, O.cnt_alloc, s, b, L, kC, O.cnt_alloc > nmat ? nmat : -1);
    const long long ls = C.leaf_stride();
    CJob lj = copy_job(b, b, nmat, 1.0, leaves_op(O.H), bop(C.lv.get(), b, ls, (long long)b * b), h.nleaf());
    lj.scale = O.cols; lj.smul = O.cmul; lj.soff = O.coff; lj.sstride = s; lj.scl = b; lj.sside = 1;
    cj.push_back(lj);
    for (int d = 1; d <= L; ++d) {
      const int w = h.kc[d];
      if (!w) continue;
      cj.push_back(copy_job(s, w, nmat, 1.0, factor_op(O.H, h.U[d], d, 0), bop(C.U[d].get(), s, (long long)C.k[d] * s)));
      // (H diag(c))[t, sib t] = U_t (diag(c_sib) V_t)^T: scale V rows
      CJob vj = copy_job(s, w, nmat, 1.0, factor_op(O.H, h.V[d], d, 0), bop(C.V[d].get(), s, (long long)C.k[d] * s));
      vj.scale = O.cols; vj.smul = O.cmul; vj.soff = O.coff; vj.sstride = s; vj.scl = 0; vj.sside = 0;
      cj.push_back(vj);
      C.kc[d] = w;
    }
  }
  gcopy<T>(st, cj);
  Queue::get().flush();   // let the device start while the host plans the next step
}

// ------------------------------------------------------------- recompress
template <typename T>
void recompress_multi(hipStream_t st, const std::vector<HSet<T>*>& sets, double eps, int maxrank) {
  struct Item {
    HSet<T>* H = nullptr;
    int d = 0, sd = 0, kcol = 0, c = 0, ncl = 0, nprob = 0, kout = 0;
    long long roff = 0;   // this item's ranks in the shared rank buffer
    DBuf<T> Ru, Rv, Uref, Utau, K, sig, UK, Un, Vn, Cv;
  };
  std::vector<Item> items;
  for (HSet<T>* H : sets)
    for (int d = 1; d <= H->L; ++d) {
      // a block of rank <= 1 is already T_eps-truncated (up to a zero column)
      if (H->kc[d] <= 1 || H->cnt == 0) continue;
      Item it;
      it.H = H; it.d = d; it.sd = H->sd(d); it.kcol = H->kc[d];
      it.c = std::min(it.sd, it.kcol); it.ncl = 1 << d; it.nprob = H->cnt * it.ncl;
      items.push_back(std::move(it));
    }
  if (items.empty()) return;
  // QR of the stacked U (reflectors kept) and V (R only) of every block,
  // cores K_t = Ru_t Rv_(sib t)^T, their rank-revealing SVDs and ranks
  std::vector<QJob> qj;
  GemmPlan kp;
  std::vector<SJob> sj;
  long long nrank = 0;
  for (auto& it : items) {
    it.roff = nrank;
    nrank += it.nprob;
  }
  DBuf<int> ranks((size_t)nrank);
  for (size_t i = 0; i < items.size(); ++i) {
    Item& it = items[i];
    HV<T> HH{it.H, 1, 0};
    const size_t np = it.nprob, c = it.c, kc = it.kcol;
    it.Ru.resize(np * c * kc); it.Rv.resize(np * c * kc);
    it.Uref.resize(np * it.sd * c); it.Utau.resize(np * c);
    QJob qu;
    qu.p = it.sd; qu.k = it.kcol; qu.nmat = it.H->cnt; qu.ncl = it.ncl;
    qu.A = factor_op(HH, it.H->U[it.d], it.d, it.sd);
    qu.R = it.Ru.get(); qu.Vref = it.Uref.get(); qu.tau = it.Utau.get();
    QJob qv = qu;
    qv.A = factor_op(HH, it.H->V[it.d], it.d, it.sd);
    qv.R = it.Rv.get(); qv.Vref = nullptr; qv.tau = nullptr;
    qj.push_back(qu);
    qj.push_back(qv);
    {
      const double p = it.sd, k = it.kcol, r = it.c;
      work().qr_flops += 2.0 * np * (2.0 * p * k * r - (p + k) * r * r + 2.0 / 3.0 * r * r * r);
    }
    it.K.resize(np * c * c);
    BOp Rub = bop(it.Ru.get(), it.c, (long long)it.ncl * c * kc, (long long)c * kc);
    BOp Rvb = bop(it.Rv.get(), it.c, (long long)it.ncl * c * kc, (long long)c * kc);
    kp.add(it.c, it.c, it.H->cnt, it.ncl, 1.0, 0.0, bop(it.K.get(), it.c, (long long)it.ncl * c * c, (long long)c * c),
           {seg(Rub, transposed(swapped(Rvb)), it.kcol)});
    it.sig.resize(np * c); it.UK.resize(np * c * c);
    SJob sv;
    sv.c = it.c; sv.nprob = it.nprob; sv.K = it.K.get(); sv.sig = it.sig.get(); sv.UK = it.UK.get();
    sv.rank = ranks.get() + it.roff; sv.eps = eps; sv.maxrank = maxrank;
    sj.push_back(sv);
    work().svd_flops += 6.0 * (double)c * c * c * np;
  }
  gqr<T>(st, qj);
  kp.run<T>(st);
  grsvd<T>(st, sj);
  // every block's numerical rank, one copy; the set's rank per depth is their maximum
  std::vector<int> hr((size_t)nrank);
  read_to_host(hr.data(), ranks.get(), (size_t)nrank * sizeof(int), st);
  std::vector<long long> rsum(items.size(), 0);
  for (size_t i = 0; i < items.size(); ++i) {
    int mx = 0;
    for (int q = 0; q < items[i].nprob; ++q) {
      const int r = hr[(size_t)items[i].roff + q];
      mx = std::max(mx, r);
      rsum[i] += r;
    }
    items[i].kout = mx;
  }
  // Keep s_t > eps s_1:  K = U_K S J^T, with the SVD's U_K already zero past
  // each block's rank (t columns kept: the set's maximum rank),
  //   U_new = Q_U [U_K,t; 0]          (orthonormal columns)
  //   V_new = V Ru^T U_K,t            (= Q_V J_t S_t, no inverse)
  std::vector<AJob> aj;
  GemmPlan cvp, vnp;
  for (size_t i = 0; i < items.size(); ++i) {
    Item& it = items[i];
    if (it.kout == 0) continue;
    HV<T> HH{it.H, 1, 0};
    const int s = it.H->s, c = it.c, ko = it.kout, kc = it.kcol;
    const size_t np = it.nprob;
    it.Un.resize((size_t)it.H->cnt * ko * s);
    it.Vn.resize((size_t)it.H->cnt * ko * s);
    AJob a;
    a.p = it.sd; a.c = c; a.t = ko; a.nmat = it.H->cnt; a.ncl = it.ncl; a.zxor = 0;
    a.Vref = it.Uref.get(); a.tau = it.Utau.get(); a.Z = it.UK.get(); a.sZ = (long long)c * c;
    a.Y = bop(it.Un.get(), s, (long long)ko * s, it.sd);
    aj.push_back(a);
    work().qr_flops += 4.0 * it.sd * c * ko * np;
    it.Cv.resize(np * kc * ko);
    BOp Rub = bop(it.Ru.get(), c, (long long)it.ncl * c * kc, (long long)c * kc);
    BOp Cvb = bop(it.Cv.get(), kc, (long long)it.ncl * kc * ko, (long long)kc * ko);
    cvp.add(kc, ko, it.H->cnt, it.ncl, 1.0, 0.0, Cvb,
            {seg(transposed(Rub), bop(it.UK.get(), c, (long long)it.ncl * c * c, (long long)c * c), c)});
    vnp.add(it.sd, ko, it.H->cnt, it.ncl, 1.0, 0.0, bop(it.Vn.get(), s, (long long)ko * s, it.sd),
            {seg(factor_op(HH, it.H->V[it.d], it.d, it.sd), swapped(Cvb), kc)});
  }
  gapply_q<T>(st, aj);
  cvp.run<T>(st);
  vnp.run<T>(st);
  for (size_t i = 0; i < items.size(); ++i) {
    Item& it = items[i];
    it.H->U[it.d] = std::move(it.Un);
    it.H->V[it.d] = std::move(it.Vn);
    it.H->k[it.d] = it.H->kc[it.d] = it.kout;
    it.H->rsum[it.d] = (double)rsum[i];
  }
  Queue::get().flush();   // let the device start while the host plans the next step
}

template <typename T>
void densify_to_host(hipStream_t st, const HSet<T>& H, int m, double* out) {
  const int s = H.s, b = H.b;
  std::vector<T> lv((size_t)H.leaf_stride());
  Queue::get().flush();
  ACR_HIP(hipMemcpyAsync(lv.data(), H.lv.get() + (size_t)m * H.leaf_stride(), lv.size() * sizeof(T),
                         hipMemcpyDeviceToHost, st));
  std::vector<std::vector<T>> U(H.L + 1), V(H.L + 1);
  for (int d = 1; d <= H.L; ++d) {
    U[d].resize((size_t)H.kc[d] * s);
    V[d].resize((size_t)H.kc[d] * s);
    if (H.kc[d]) {
      ACR_HIP(hipMemcpyAsync(U[d].data(), H.U[d].get() + (size_t)m * H.k[d] * s, U[d].size() * sizeof(T),
                             hipMemcpyDeviceToHost, st));
      ACR_HIP(hipMemcpyAsync(V[d].data(), H.V[d].get() + (size_t)m * H.k[d] * s, V[d].size() * sizeof(T),
                             hipMemcpyDeviceToHost, st));
    }
  }
  ACR_HIP(hipStreamSynchronize(st));
  for (size_t e = 0; e < (size_t)s * s; ++e) out[e] = 0.0;
  for (int l = 0; l < H.nleaf(); ++l)
    for (int c = 0; c < b; ++c)
      for (int r = 0; r < b; ++r)
        out[(size_t)(l * b + r) + (size_t)(l * b + c) * s] = (double)lv[(size_t)l * b * b + r + (size_t)c * b];
  for (int d = 1; d <= H.L; ++d) {
    const int sd = H.sd(d), w = H.kc[d];
    for (int t = 0; t < (1 << d); ++t) {
      const int sg = t ^ 1;
      for (int c = 0; c < sd; ++c)
        for (int r = 0; r < sd; ++r) {
          double v = 0.0;
          for (int q = 0; q < w; ++q)
            v += (double)U[d][(size_t)q * s + t * sd + r] * (double)V[d][(size_t)q * s + sg * sd + c];
          out[(size_t)(t * sd + r) + (size_t)(sg * sd + c) * s] = v;
        }
    }
  }
}

#define INST(T)                                                                                    \
  template struct HSet<T>;                                                                         \
  template void GemmPlan::run<T>(hipStream_t);                                                     \
  template BOp flat_op<T>(const Flat<T>&, long long, int);                                         \
  template std::vector<GSeg> plan_hmul<T>(GemmPlan&, std::vector<DBuf<T>>&, HV<T>, int, int, bool, \
                                          int, double, Flat<T>);                                   \
  template void hmul<T>(hipStream_t, HV<T>, int, int, bool, int, T, Flat<T>, T, Flat<T>);          \
  template void hprod_multi<T>(hipStream_t, std::vector<POut<T>>&);                                \
  template void hinv<T>(hipStream_t, HSet<T>&, HV<T>, int, int*);                                  \
  template void hinv_multi<T>(hipStream_t, std::vector<HInvJob<T>>&);                              \
  template void hstack_multi<T>(hipStream_t, std::vector<StackOut<T>>&);                           \
  template void hscale_cols_multi<T>(hipStream_t, std::vector<ColScale<T>>&);                      \
  template void recompress_multi<T>(hipStream_t, const std::vector<HSet<T>*>&, double, int);       \
  template void densify_to_host<T>(hipStream_t, const HSet<T>&, int, double*);

INST(float)
INST(double)
#undef INST

}  // namespace acr
