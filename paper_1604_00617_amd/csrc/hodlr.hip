// H-arithmetic on batched HODLR sets: every operation is a short sequence of
// batched launches over (matrix, cluster) problems of one depth.
#include "hodlr.hpp"

#include <algorithm>

#include "kernels.hpp"

namespace acr {

Work& work() {
  static thread_local Work w;
  return w;
}

// ------------------------------------------------------------------ HSet
template <typename T>
void HSet<T>::alloc(hipStream_t st, int cnt_, int s_, int b_, int L_, const std::vector<int>& k_,
                    bool zero) {
  cnt = cnt_; s = s_; b = b_; L = L_;
  k.assign(L + 1, 0);
  kc.assign(L + 1, 0);
  for (int d = 1; d <= L; ++d) k[d] = d < (int)k_.size() ? k_[d] : 0;
  lv.resize((size_t)cnt * leaf_stride());
  U.clear(); V.clear();
  U.resize(L + 1); V.resize(L + 1);
  for (int d = 1; d <= L; ++d) {
    U[d].resize((size_t)cnt * k[d] * s);
    V[d].resize((size_t)cnt * k[d] * s);
  }
  if (zero) {
    if (lv.bytes()) ACR_HIP(hipMemsetAsync(lv.get(), 0, lv.bytes(), st));
    for (int d = 1; d <= L; ++d) {
      if (U[d].bytes()) ACR_HIP(hipMemsetAsync(U[d].get(), 0, U[d].bytes(), st));
      if (V[d].bytes()) ACR_HIP(hipMemsetAsync(V[d].get(), 0, V[d].bytes(), st));
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
int HSet<T>::max_rank() const {
  int r = 0;
  for (int d = 1; d <= L; ++d) r = std::max(r, kc[d]);
  return r;
}

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
BOp flat_op(const Flat<T>& f, long long sc, int col0 = 0) {
  BOp o = bop(f.p + (long long)col0 * f.ld, f.ld, f.sm, sc);
  return with_map(o, f.mmul, f.moff);
}

template <typename T>
Flat<T> flat_of(const HSet<T>& H, const DBuf<T>& F, int d, int col0 = 0) {
  Flat<T> f;
  f.p = F.get() + (size_t)col0 * H.s;
  f.ld = H.s;
  f.sm = (long long)H.k[d] * H.s;
  return f;
}

template <typename T>
void count_gemm(long long M, long long N, long long K, long long nprob) {
  work().gemm_flops += 2.0 * M * N * K * nprob;
}

}  // namespace

// ------------------------------------------------------------------- hmul
template <typename T>
void hmul(hipStream_t st, HV<T> H, int nmat, int dfrom, bool trans, int ncol, T alpha, Flat<T> Y,
          T beta, Flat<T> out) {
  const HSet<T>& h = *H.h;
  if (nmat <= 0 || ncol <= 0) return;
  const int b = h.b;
  // dense leaves
  BOp A = leaves_op(H);
  A.trans = trans ? 1 : 0;
  bgemm<T>(st, b, ncol, b, nmat, h.nleaf(), alpha, A, flat_op(Y, b), beta, flat_op(out, b));
  count_gemm<T>(b, ncol, b, (long long)nmat * h.nleaf());
  for (int d = std::max(dfrom + 1, 1); d <= h.L; ++d) {
    const int w = h.kc[d];
    if (w == 0) continue;
    const int ncl = 1 << d, sd = h.sd(d);
    DBuf<T> tmp((size_t)nmat * ncl * w * ncol);
    // tmp_c = (V or U)[rows c]^T Y[rows c]
    BOp Ain = factor_op(H, trans ? h.U[d] : h.V[d], d, sd);
    Ain.trans = 1;
    BOp Tc = bop(tmp.get(), w, (long long)ncl * w * ncol, (long long)w * ncol);
    bgemm<T>(st, w, ncol, sd, nmat, ncl, T(1), Ain, flat_op(Y, sd), T(0), Tc);
    // out[rows c] += alpha * (U or V)[rows c] tmp_(sib c)
    BOp Aout = factor_op(H, trans ? h.V[d] : h.U[d], d, sd);
    bgemm<T>(st, sd, ncol, w, nmat, ncl, alpha, Aout, swapped(Tc), T(1), flat_op(out, sd));
    count_gemm<T>(2LL * sd, ncol, w, (long long)nmat * ncl);
  }
}

// ------------------------------------------------------------------ hprod
template <typename T>
void hprod(hipStream_t st, HSet<T>& C, int cnt_alloc, HV<T> A, HV<T> B, int nmat, T alpha) {
  const HSet<T>& a = *A.h;
  const HSet<T>& bb = *B.h;
  const int L = a.L, s = a.s, b = a.b;
  const int nleaf = a.nleaf();
  // Ancestor terms: for depth d'' the block A[p, q] B[q, p] (q = sib p) is
  // U^A_p (V^A_p^T U^B_q) V^B_q^T; it restricts to every block below p.
  // Stored as (Upart, Vpart) flat pairs of width min(kA, kB).
  std::vector<int> wanc(L + 1, 0);
  std::vector<DBuf<T>> Up(L + 1), Vp(L + 1);
  std::vector<const T*> Upp(L + 1, nullptr), Vpp(L + 1, nullptr);
  std::vector<long long> Ups(L + 1, 0), Vps(L + 1, 0);
  std::vector<int> Upm(L + 1, 1), Upo(L + 1, 0), Vpm(L + 1, 1), Vpo(L + 1, 0);
  for (int d = 1; d <= L; ++d) {
    const int kA = a.kc[d], kB = bb.kc[d];
    if (kA == 0 || kB == 0) continue;
    const int ncl = 1 << d, sd = a.sd(d);
    DBuf<T> W((size_t)nmat * ncl * kA * kB);
    BOp Wc = bop(W.get(), kA, (long long)ncl * kA * kB, (long long)kA * kB);
    bgemm<T>(st, kA, kB, sd, nmat, ncl, T(1), transposed(factor_op(A, a.V[d], d, sd)),
             factor_op(B, bb.U[d], d, sd), T(0), Wc);
    count_gemm<T>(kA, kB, sd, (long long)nmat * ncl);
    if (kB <= kA) {
      // Upart = U^A (.) W_(sib), Vpart = V^B
      wanc[d] = kB;
      Up[d].resize((size_t)nmat * kB * s);
      BOp Z = bop(Up[d].get(), s, (long long)kB * s, sd);
      bgemm<T>(st, sd, kB, kA, nmat, ncl, T(1), factor_op(A, a.U[d], d, sd), swapped(Wc), T(0), Z);
      count_gemm<T>(sd, kB, kA, (long long)nmat * ncl);
      Upp[d] = Up[d].get(); Ups[d] = (long long)kB * s; Upm[d] = 1; Upo[d] = 0;
      Vpp[d] = bb.V[d].get(); Vps[d] = (long long)bb.k[d] * s; Vpm[d] = B.mmul; Vpo[d] = B.moff;
    } else {
      // Upart = U^A, Vpart = V^B (.) W_(sib)^T
      wanc[d] = kA;
      Vp[d].resize((size_t)nmat * kA * s);
      BOp Z = bop(Vp[d].get(), s, (long long)kA * s, sd);
      bgemm<T>(st, sd, kA, kB, nmat, ncl, T(1), factor_op(B, bb.V[d], d, sd),
               transposed(swapped(Wc)), T(0), Z);
      count_gemm<T>(sd, kA, kB, (long long)nmat * ncl);
      Upp[d] = a.U[d].get(); Ups[d] = (long long)a.k[d] * s; Upm[d] = A.mmul; Upo[d] = A.moff;
      Vpp[d] = Vp[d].get(); Vps[d] = (long long)kA * s; Vpm[d] = 1; Vpo[d] = 0;
    }
  }
  std::vector<int> kC(L + 1, 0);
  for (int d = 1; d <= L; ++d) {
    kC[d] = a.kc[d] + bb.kc[d];
    for (int e = 1; e < d; ++e) kC[d] += wanc[e];
  }
  C.alloc(st, cnt_alloc, s, b, L, kC, cnt_alloc > nmat);
  // leaves: C_l = A_l B_l + sum over ancestors of Upart[l] Vpart[l]^T
  bgemm<T>(st, b, b, b, nmat, nleaf, alpha, leaves_op(A), leaves_op(B), T(0),
           bop(C.lv.get(), b, C.leaf_stride(), (long long)b * b));
  count_gemm<T>(b, b, b, (long long)nmat * nleaf);
  for (int e = 1; e <= L; ++e) {
    if (!wanc[e]) continue;
    BOp Ua = with_map(bop(Upp[e], s, Ups[e], b), Upm[e], Upo[e]);
    BOp Va = with_map(bop(Vpp[e], s, Vps[e], b, 1), Vpm[e], Vpo[e]);
    bgemm<T>(st, b, b, wanc[e], nmat, nleaf, alpha, Ua, Va, T(1),
             bop(C.lv.get(), b, C.leaf_stride(), (long long)b * b));
    count_gemm<T>(b, b, wanc[e], (long long)nmat * nleaf);
  }
  for (int d = 1; d <= L; ++d) {
    int col = 0;
    const int kA = a.kc[d], kB = bb.kc[d];
    if (kB > 0) {   // A[t,t] B[t,s] = (Adiag U^B) V^B^T
      Flat<T> Y; Y.p = bb.U[d].get(); Y.ld = s; Y.sm = (long long)bb.k[d] * s; Y.mmul = B.mmul; Y.moff = B.moff;
      hmul<T>(st, A, nmat, d, false, kB, alpha, Y, T(0), flat_of(C, C.U[d], d, col));
      bcopy<T>(st, s, kB, nmat, T(1), with_map(bop(bb.V[d].get(), s, (long long)bb.k[d] * s), B.mmul, B.moff),
               bop(C.V[d].get() + (size_t)col * s, s, (long long)C.k[d] * s));
      col += kB;
    }
    if (kA > 0) {   // A[t,s] B[s,s] = U^A (Bdiag^T V^A)^T
      bcopy<T>(st, s, kA, nmat, alpha, with_map(bop(a.U[d].get(), s, (long long)a.k[d] * s), A.mmul, A.moff),
               bop(C.U[d].get() + (size_t)col * s, s, (long long)C.k[d] * s));
      Flat<T> Y; Y.p = a.V[d].get(); Y.ld = s; Y.sm = (long long)a.k[d] * s; Y.mmul = A.mmul; Y.moff = A.moff;
      hmul<T>(st, B, nmat, d, true, kA, T(1), Y, T(0), flat_of(C, C.V[d], d, col));
      col += kA;
    }
    for (int e = 1; e < d; ++e) {
      if (!wanc[e]) continue;
      bcopy<T>(st, s, wanc[e], nmat, alpha, with_map(bop(Upp[e], s, Ups[e]), Upm[e], Upo[e]),
               bop(C.U[d].get() + (size_t)col * s, s, (long long)C.k[d] * s));
      bcopy<T>(st, s, wanc[e], nmat, T(1), with_map(bop(Vpp[e], s, Vps[e]), Vpm[e], Vpo[e]),
               bop(C.V[d].get() + (size_t)col * s, s, (long long)C.k[d] * s));
      col += wanc[e];
    }
    C.kc[d] = col;
  }
}

// ------------------------------------------------------------------- hinv
template <typename T>
void hinv(hipStream_t st, HSet<T>& X, HV<T> M, int nmat, int* status) {
  const HSet<T>& mm = *M.h;
  const int L = mm.L, s = mm.s, b = mm.b, nleaf = mm.nleaf();
  std::vector<int> kX(L + 1, 0);
  for (int d = 1; d <= L; ++d)
    for (int e = 1; e <= d; ++e) kX[d] += mm.kc[e];
  X.alloc(st, nmat, s, b, L, kX, false);
  // leaves: X_l = M_l^{-1}
  bcopy<T>(st, b * nleaf * b, 1, nmat, T(1), with_map(bop(mm.lv.get(), 1, mm.leaf_stride()), M.mmul, M.moff),
           bop(X.lv.get(), 1, X.leaf_stride()));
  binverse<T, T>(st, b, nmat * nleaf, X.lv.get(), (long long)b * b, X.lv.get(), (long long)b * b,
                 status);
  work().inv_flops += 2.0 * b * b * b * nmat * nleaf;
  HV<T> XV{&X, 1, 0};
  for (int d = L; d >= 1; --d) {
    const int k = mm.kc[d];
    if (k == 0) continue;
    const int ncl = 1 << d, sd = mm.sd(d);
    DBuf<T> abuf((size_t)nmat * k * s), bbuf((size_t)nmat * k * s), wbuf((size_t)nmat * k * s);
    Flat<T> fa; fa.p = abuf.get(); fa.ld = s; fa.sm = (long long)k * s;
    Flat<T> fb; fb.p = bbuf.get(); fb.ld = s; fb.sm = (long long)k * s;
    Flat<T> fw; fw.p = wbuf.get(); fw.ld = s; fw.sm = (long long)k * s;
    Flat<T> Um; Um.p = mm.U[d].get(); Um.ld = s; Um.sm = (long long)mm.k[d] * s; Um.mmul = M.mmul; Um.moff = M.moff;
    Flat<T> Vm = Um; Vm.p = mm.V[d].get();
    // a = Xdiag U^M (children inverses applied), bb = Xdiag^T V^M
    hmul<T>(st, XV, nmat, d, false, k, T(1), Um, T(0), fa);
    hmul<T>(st, XV, nmat, d, true, k, T(1), Vm, T(0), fb);
    // cores c_sigma = V^M[sigma]^T a[sigma]
    DBuf<T> cores((size_t)nmat * ncl * k * k);
    bgemm<T>(st, k, k, sd, nmat, ncl, T(1), transposed(factor_op(M, mm.V[d], d, sd)), flat_op(fa, sd),
             T(0), bop(cores.get(), k, (long long)ncl * k * k, (long long)k * k));
    count_gemm<T>(k, k, sd, (long long)nmat * ncl);
    const int npairs = nmat * ncl / 2, n2 = 2 * k;
    DBuf<T> G((size_t)npairs * n2 * n2);
    build_capacitance<T>(st, k, npairs, cores.get(), G.get());
    binverse<T, T>(st, n2, npairs, G.get(), (long long)n2 * n2, G.get(), (long long)n2 * n2, status);
    work().inv_flops += 2.0 * n2 * n2 * n2 * npairs;
    // diagonal block of G^{-1} for cluster t: (t&1) selects (0,0) or (1,1)
    BOp Gd;
    Gd.p = G.get(); Gd.ld = n2; Gd.sm = (long long)(ncl / 2) * n2 * n2;
    Gd.sc_pair = (long long)n2 * n2; Gd.sc_odd = (long long)k + (long long)k * n2;
    BOp Go = Gd;
    Go.p = G.get() + (size_t)k * n2;              // (0,1) block for a first child
    Go.sc_odd = (long long)k - (long long)k * n2;  // (1,0) block for a second child
    // U^X_d = -a[t] Gdiag(t), V^X_d = bb
    bgemm<T>(st, sd, k, k, nmat, ncl, T(-1), flat_op(fa, sd), Gd, T(0),
             bop(X.U[d].get(), s, (long long)X.k[d] * s, sd));
    bcopy<T>(st, s, k, nmat, T(1), bop(bbuf.get(), s, (long long)k * s),
             bop(X.V[d].get(), s, (long long)X.k[d] * s));
    X.kc[d] = k;
    // W = a[t] Goff(t): X[t,t] -= W[t] bb[t]^T pushed below depth d
    bgemm<T>(st, sd, k, k, nmat, ncl, T(1), flat_op(fa, sd), Go, T(0), flat_op(fw, sd));
    count_gemm<T>(2LL * sd, k, k, (long long)nmat * ncl);
    for (int e = d + 1; e <= L; ++e) {
      bcopy<T>(st, s, k, nmat, T(-1), bop(wbuf.get(), s, (long long)k * s),
               bop(X.U[e].get() + (size_t)X.kc[e] * s, s, (long long)X.k[e] * s));
      bcopy<T>(st, s, k, nmat, T(1), bop(bbuf.get(), s, (long long)k * s),
               bop(X.V[e].get() + (size_t)X.kc[e] * s, s, (long long)X.k[e] * s));
      X.kc[e] += k;
    }
    bgemm<T>(st, b, b, k, nmat, nleaf, T(-1), bop(wbuf.get(), s, (long long)k * s, b),
             bop(bbuf.get(), s, (long long)k * s, b, 1), T(1),
             bop(X.lv.get(), b, X.leaf_stride(), (long long)b * b));
    count_gemm<T>(b, b, k, (long long)nmat * nleaf);
  }
}

// ----------------------------------------------------------------- hstack
template <typename T>
void hstack(hipStream_t st, HSet<T>& C, int cnt_alloc, const std::vector<STerm<T>>& terms, int nmat) {
  const HSet<T>& h0 = *terms[0].h.h;
  const int L = h0.L, s = h0.s, b = h0.b;
  std::vector<int> kC(L + 1, 0);
  for (const auto& t : terms)
    for (int d = 1; d <= L; ++d) kC[d] += t.h.h->kc[d];
  C.alloc(st, cnt_alloc, s, b, L, kC, cnt_alloc > nmat);
  const long long ls = C.leaf_stride();
  bool first = true;
  std::vector<int> col(L + 1, 0);
  for (const auto& t : terms) {
    const HSet<T>& h = *t.h.h;
    // leaves: C += coef * diag(rows) * H_leaves
    DBuf<T> tmp;
    const T* src = h.lv.get();
    int smul = t.h.mmul, soff = t.h.moff;
    long long sstr = h.leaf_stride();
    if (t.rows) {
      tmp.resize((size_t)nmat * ls);
      bcopy<T>(st, (int)ls, 1, nmat, T(1), with_map(bop(h.lv.get(), 1, h.leaf_stride()), t.h.mmul, t.h.moff),
               bop(tmp.get(), 1, ls));
      bscale<T>(st, b, b, nmat, h.nleaf(), bop(tmp.get(), b, ls, (long long)b * b), t.rows, t.rmul,
                t.roff, s, b, 0, T(1));
      src = tmp.get(); smul = 1; soff = 0; sstr = ls;
    }
    if (first)
      bcopy<T>(st, (int)ls, 1, nmat, t.coef, with_map(bop(src, 1, sstr), smul, soff), bop(C.lv.get(), 1, ls));
    else
      badd<T>(st, (int)ls, 1, nmat, t.coef, with_map(bop(src, 1, sstr), smul, soff), bop(C.lv.get(), 1, ls));
    first = false;
    for (int d = 1; d <= L; ++d) {
      const int w = h.kc[d];
      if (!w) continue;
      T* ud = C.U[d].get() + (size_t)col[d] * s;
      T* vd = C.V[d].get() + (size_t)col[d] * s;
      bcopy<T>(st, s, w, nmat, t.coef, with_map(bop(h.U[d].get(), s, (long long)h.k[d] * s), t.h.mmul, t.h.moff),
               bop(ud, s, (long long)C.k[d] * s));
      if (t.rows)
        bscale<T>(st, s, w, nmat, 1, bop(ud, s, (long long)C.k[d] * s), t.rows, t.rmul, t.roff, s, 0, 0, T(1));
      bcopy<T>(st, s, w, nmat, T(1), with_map(bop(h.V[d].get(), s, (long long)h.k[d] * s), t.h.mmul, t.h.moff),
               bop(vd, s, (long long)C.k[d] * s));
      col[d] += w;
    }
  }
  for (int d = 1; d <= L; ++d) C.kc[d] = col[d];
}

template <typename T>
void hscale_cols(hipStream_t st, HSet<T>& C, int cnt_alloc, HV<T> H, const T* cols, int cmul, int coff,
                 int nmat) {
  const HSet<T>& h = *H.h;
  const int L = h.L, s = h.s, b = h.b;
  std::vector<int> kC(L + 1, 0);
  for (int d = 1; d <= L; ++d) kC[d] = h.kc[d];
  C.alloc(st, cnt_alloc, s, b, L, kC, cnt_alloc > nmat);
  const long long ls = C.leaf_stride();
  bcopy<T>(st, (int)ls, 1, nmat, T(1), with_map(bop(h.lv.get(), 1, h.leaf_stride()), H.mmul, H.moff),
           bop(C.lv.get(), 1, ls));
  bscale<T>(st, b, b, nmat, h.nleaf(), bop(C.lv.get(), b, ls, (long long)b * b), cols, cmul, coff, s, b, 1,
            T(1));
  for (int d = 1; d <= L; ++d) {
    const int w = h.kc[d];
    if (!w) continue;
    bcopy<T>(st, s, w, nmat, T(1), with_map(bop(h.U[d].get(), s, (long long)h.k[d] * s), H.mmul, H.moff),
             bop(C.U[d].get(), s, (long long)C.k[d] * s));
    bcopy<T>(st, s, w, nmat, T(1), with_map(bop(h.V[d].get(), s, (long long)h.k[d] * s), H.mmul, H.moff),
             bop(C.V[d].get(), s, (long long)C.k[d] * s));
    // (H diag(c))[t, sib t] = U_t (diag(c_sib) V_t)^T: scale V rows
    bscale<T>(st, s, w, nmat, 1, bop(C.V[d].get(), s, (long long)C.k[d] * s), cols, cmul, coff, s, 0, 0, T(1));
    C.kc[d] = w;
  }
}

// ------------------------------------------------------------- recompress
template <typename T>
void recompress(hipStream_t st, HSet<T>& H, double eps, int maxrank) {
  const int s = H.s, cnt = H.cnt;
  if (cnt <= 0) return;
  DBuf<int> dmax(1);
  for (int d = 1; d <= H.L; ++d) {
    const int kcol = H.kc[d];
    if (kcol == 0) continue;
    const int ncl = 1 << d, sd = H.sd(d), c = std::min(sd, kcol);
    const int nprob = cnt * ncl;
    HV<T> HH{&H, 1, 0};
    DBuf<T> Ru((size_t)nprob * c * kcol), Rv((size_t)nprob * c * kcol);
    DBuf<T> Vref((size_t)nprob * sd * c), tau((size_t)nprob * c);
    bqr_r<T>(st, sd, kcol, cnt, ncl, factor_op(HH, H.U[d], d, sd), Ru.get());
    bqr_r<T>(st, sd, kcol, cnt, ncl, factor_op(HH, H.V[d], d, sd), Rv.get(), Vref.get(), tau.get());
    {
      const double p = sd, k = kcol, r = c;
      work().qr_flops += 2.0 * nprob * (2.0 * p * k * r - (p + k) * r * r + 2.0 / 3.0 * r * r * r);
    }
    BOp Rub = bop(Ru.get(), c, (long long)ncl * c * kcol, (long long)c * kcol);
    BOp Rvb = bop(Rv.get(), c, (long long)ncl * c * kcol, (long long)c * kcol);
    DBuf<T> K((size_t)nprob * c * c);
    bgemm<T>(st, c, c, kcol, cnt, ncl, T(1), Rub, transposed(swapped(Rvb)), T(0),
             bop(K.get(), c, (long long)ncl * c * c, (long long)c * c));
    count_gemm<T>(c, c, kcol, nprob);
    DBuf<T> sig((size_t)nprob * c), Usc((size_t)nprob * c * c), J((size_t)nprob * c * c);
    DBuf<int> rank(nprob);
    bsvd<T>(st, c, nprob, K.get(), sig.get(), Usc.get(), J.get(), rank.get(), eps, maxrank);
    work().svd_flops += 8.0 * 6.0 * (double)c * c * c / 2.0 * nprob;   // nominal 8 sweeps
    bmax_int(st, rank.get(), nprob, dmax.get());
    int kout = 0;
    ACR_HIP(hipMemcpyAsync(&kout, dmax.get(), sizeof(int), hipMemcpyDeviceToHost, st));
    ACR_HIP(hipStreamSynchronize(st));
    DBuf<T> Un, Vn;
    if (kout > 0) {
      // K = Ru Rv^T = Usc J^T with Usc = Ut S.  Kept part:
      //   U_new = Q_U Usc_t = U Rv^T J_t   (no inverse: U Rv^T = Q_U K)
      //   V_new = Q_V J_t                  (reflectors of the V factor)
      DBuf<T> Jt((size_t)nprob * c * kout);
      btrunc_coef<T>(st, c, kout, nprob, J.get(), rank.get(), Jt.get());
      DBuf<T> Cu((size_t)nprob * kcol * kout);
      BOp Cub = bop(Cu.get(), kcol, (long long)ncl * kcol * kout, (long long)kcol * kout);
      bgemm<T>(st, kcol, kout, c, cnt, ncl, T(1), transposed(swapped(Rvb)),
               bop(Jt.get(), c, (long long)ncl * c * kout, (long long)c * kout), T(0), Cub);
      count_gemm<T>(kcol, kout, c, nprob);
      Un.resize((size_t)cnt * kout * s);
      Vn.resize((size_t)cnt * kout * s);
      bgemm<T>(st, sd, kout, kcol, cnt, ncl, T(1), factor_op(HH, H.U[d], d, sd), Cub, T(0),
               bop(Un.get(), s, (long long)kout * s, sd));
      count_gemm<T>(sd, kout, kcol, nprob);
      // V_new[rows sig] = Q_V(sig) [Jt_(sib sig); 0]
      bapply_q<T>(st, sd, c, kout, cnt, ncl, Vref.get(), tau.get(), Jt.get(), (long long)c * kout, 1,
                  bop(Vn.get(), s, (long long)kout * s, sd));
      work().qr_flops += 4.0 * sd * c * kout * nprob;
    }
    H.U[d] = std::move(Un);
    H.V[d] = std::move(Vn);
    H.k[d] = H.kc[d] = kout;
  }
}

template <typename T>
void densify_to_host(hipStream_t st, const HSet<T>& H, int m, double* out) {
  const int s = H.s, b = H.b;
  std::vector<T> lv((size_t)H.leaf_stride());
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
  template void hmul<T>(hipStream_t, HV<T>, int, int, bool, int, T, Flat<T>, T, Flat<T>);          \
  template void hprod<T>(hipStream_t, HSet<T>&, int, HV<T>, HV<T>, int, T);                        \
  template void hinv<T>(hipStream_t, HSet<T>&, HV<T>, int, int*);                                  \
  template void hstack<T>(hipStream_t, HSet<T>&, int, const std::vector<STerm<T>>&, int);          \
  template void hscale_cols<T>(hipStream_t, HSet<T>&, int, HV<T>, const T*, int, int, int);        \
  template void recompress<T>(hipStream_t, HSet<T>&, double, int);                                 \
  template void densify_to_host<T>(hipStream_t, const HSet<T>&, int, double*);

INST(float)
INST(double)
#undef INST

}  // namespace acr
