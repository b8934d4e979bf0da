// Device kernels of the ACR library for gfx950 (CDNA4, 64-wide wavefronts).
//
// The H-arithmetic of every cyclic-reduction level is expressed as batched
// operations over (matrix, cluster) problems of uniform shape; this file holds
// the batched primitives: a tiled batched GEMM, dense inverses (leaves and
// capacitance matrices), Householder R factors and one-sided Jacobi SVDs for
// recompression, plus the elementwise, layout and residual kernels.
#include "kernels.hpp"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <vector>

namespace acr {

namespace {

constexpr int WAVE = 64;
constexpr size_t kMaxLds = 65536;   // dynamic + static LDS budget per workgroup

template <typename T>
__device__ __forceinline__ const T* optr(const BOp& o, int m, int c) {
  const int cc = c ^ o.cxor;
  return static_cast<const T*>(o.p) + (long long)(o.mmul * m + o.moff) * o.sm +
         (long long)(cc >> 1) * o.sc_pair + (long long)(cc & 1) * o.sc_odd;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

template <typename T>
__device__ __forceinline__ T group_sum(T v, int g) {   // sum within aligned groups of g lanes
  for (int off = g / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// Block-wide sum over 256 threads (4 waves); every thread gets the result.
template <typename T>
__device__ T block_sum256(T v, T* red) {
  v = wave_sum(v);
  const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  T r = red[0] + red[1] + red[2] + red[3];
  return r;
}

template <typename T> struct Eps;
template <> struct Eps<float> { static constexpr double v = 5.9604644775390625e-8; };
template <> struct Eps<double> { static constexpr double v = 1.1102230246251565e-16; };

// ------------------------------------------------------------------ GEMM
// Tile TM x TN per workgroup, TK deep, each thread RM x RN outputs.
template <typename T, int TM, int TN, int TK, int RM, int RN>
__global__ __launch_bounds__((TM / RM) * (TN / RN)) void k_bgemm(int M, int N, int K, int ncl,
                                                                int tilesM, int tilesN, T alpha,
                                                                BOp A, BOp B, T beta, BOp C) {
  constexpr int TX = TM / RM, TY = TN / RN, NT = TX * TY;
  __shared__ T As[TK][TM + 1];
  __shared__ T Bs[TK][TN + 1];
  const int tiles = tilesM * tilesN;
  const long long bid = blockIdx.x;
  const int prob = (int)(bid / tiles);
  const int t = (int)(bid % tiles);
  const int tm = t % tilesM, tn = t / tilesM;
  const int m = prob / ncl, c = prob % ncl;
  const T* Ap = optr<T>(A, m, c);
  const T* Bp = optr<T>(B, m, c);
  T* Cp = const_cast<T*>(optr<T>(C, m, c));
  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const int i0 = tm * TM, j0 = tn * TN;
  T acc[RM][RN];
#pragma unroll
  for (int r = 0; r < RM; ++r)
#pragma unroll
    for (int q = 0; q < RN; ++q) acc[r][q] = T(0);

  for (int k0 = 0; k0 < K; k0 += TK) {
    for (int e = tid; e < TM * TK; e += NT) {
      int i, kk;
      if (!A.trans) { i = e % TM; kk = e / TM; } else { kk = e % TK; i = e / TK; }
      const int gi = i0 + i, gk = k0 + kk;
      T v = T(0);
      if (gi < M && gk < K) v = A.trans ? Ap[gk + (long long)gi * A.ld] : Ap[gi + (long long)gk * A.ld];
      As[kk][i] = v;
    }
    for (int e = tid; e < TK * TN; e += NT) {
      int kk, j;
      if (!B.trans) { kk = e % TK; j = e / TK; } else { j = e % TN; kk = e / TN; }
      const int gk = k0 + kk, gj = j0 + j;
      T v = T(0);
      if (gk < K && gj < N) v = B.trans ? Bp[gj + (long long)gk * B.ld] : Bp[gk + (long long)gj * B.ld];
      Bs[kk][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      T a[RM], b[RN];
#pragma unroll
      for (int r = 0; r < RM; ++r) a[r] = As[kk][tx + r * TX];
#pragma unroll
      for (int q = 0; q < RN; ++q) b[q] = Bs[kk][ty + q * TY];
#pragma unroll
      for (int r = 0; r < RM; ++r)
#pragma unroll
        for (int q = 0; q < RN; ++q) acc[r][q] = fma(a[r], b[q], acc[r][q]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < RM; ++r) {
    const int gi = i0 + tx + r * TX;
    if (gi >= M) continue;
#pragma unroll
    for (int q = 0; q < RN; ++q) {
      const int gj = j0 + ty + q * TY;
      if (gj >= N) continue;
      T* cp = Cp + gi + (long long)gj * C.ld;
      T v = alpha * acc[r][q];
      if (beta != T(0)) v = fma(beta, *cp, v);
      *cp = v;
    }
  }
}

template <typename T, int TM, int TN, int RM, int RN>
void launch_gemm(hipStream_t st, int M, int N, int K, int nprob, int ncl, T alpha, const BOp& A,
                 const BOp& B, T beta, const BOp& C) {
  const int tilesM = (M + TM - 1) / TM, tilesN = (N + TN - 1) / TN;
  const long long blocks = (long long)nprob * tilesM * tilesN;
  constexpr int NT = (TM / RM) * (TN / RN);
  if (blocks <= 0) return;
  if (blocks > 0x7fffffffLL) fail(ACR_ERR_INVALID_ARG, "bgemm: grid too large");
  hipLaunchKernelGGL((k_bgemm<T, TM, TN, 16, RM, RN>), dim3((unsigned)blocks), dim3(NT), 0, st, M,
                     N, K, ncl, tilesM, tilesN, alpha, A, B, beta, C);
  ACR_CHECK_LAUNCH();
}

// ---------------------------------------------------------------- inverse
// Gauss-Jordan on the augmented matrix [A | I] (row-major n x 2n) in FP64.
template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void k_inverse(int n, const Tin* A, long long sA, Tout* X,
                                                 long long sX, double* ws, int use_lds,
                                                 int* status) {
  extern __shared__ double smem[];
  const int p = blockIdx.x;
  const int n2 = 2 * n;
  __shared__ double colj_s[128];
  double* W = use_lds ? smem : ws + (size_t)p * n * n2;
  double* colj = n <= 128 ? colj_s : ws + (size_t)gridDim.x * n * n2 + (size_t)p * n;
  __shared__ int piv;
  __shared__ double pval;
  __shared__ int bad;
  const Tin* Ap = A + (long long)p * sA;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  for (int e = tid; e < n * n2; e += blockDim.x) {
    const int r = e / n2, c = e % n2;
    W[e] = c < n ? (double)Ap[r + (long long)c * n] : (c - n == r ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (tid < WAVE) {
      double best = -1.0;
      int bi = j;
      for (int r = j + tid; r < n; r += WAVE) {
        const double v = fabs(W[(size_t)r * n2 + j]);
        if (v > best) { best = v; bi = r; }
      }
      for (int off = WAVE / 2; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, WAVE);
        const int oi = __shfl_xor(bi, off, WAVE);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (tid == 0) {
        piv = bi;
        pval = W[(size_t)bi * n2 + j];
        if (!(best > 0.0) || !isfinite(best)) bad = 1;
      }
    }
    __syncthreads();
    const int pr = piv;
    const double inv = (pval != 0.0) ? 1.0 / pval : 0.0;
    for (int c = tid; c < n2; c += blockDim.x) {
      const double a = W[(size_t)j * n2 + c];
      const double b = W[(size_t)pr * n2 + c];
      if (pr != j) W[(size_t)pr * n2 + c] = a;
      W[(size_t)j * n2 + c] = b * inv;
    }
    __syncthreads();
    for (int r = tid; r < n; r += blockDim.x) colj[r] = W[(size_t)r * n2 + j];
    __syncthreads();
    const int w = n2 - j;
    for (int e = tid; e < n * w; e += blockDim.x) {
      const int r = e / w, c = j + e % w;
      if (r != j) W[(size_t)r * n2 + c] -= colj[r] * W[(size_t)j * n2 + c];
    }
    __syncthreads();
  }
  Tout* Xp = X + (long long)p * sX;
  for (int e = tid; e < n * n; e += blockDim.x) {
    const int r = e % n, c = e / n;
    Xp[r + (long long)c * n] = (Tout)W[(size_t)r * n2 + n + c];
  }
  if (tid == 0 && bad) status[0] = 1;
}

// In-place Gauss-Jordan with partial pivoting, n x n row-major in LDS (FP64):
// pivot j: a_jj <- 1/p, row j scaled, column j <- -a_rj/p, rank-1 update of the
// rest; the row swaps are undone as column swaps in reverse order at the end.
template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void k_inverse_lds(int n, const Tin* A, long long sA, Tout* X,
                                                     long long sX, int* status) {
  extern __shared__ double W[];
  __shared__ int perm[128];
  __shared__ double colj[128];
  __shared__ int piv;
  __shared__ double pinv;
  __shared__ int bad;
  const int p = blockIdx.x, tid = threadIdx.x;
  const Tin* Ap = A + (long long)p * sA;
  if (tid == 0) bad = 0;
  for (int e = tid; e < n * n; e += 256) {
    const int r = e % n, c = e / n;
    W[r * n + c] = (double)Ap[e];
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (tid < WAVE) {
      double best = -1.0;
      int bi = j;
      for (int r = j + tid; r < n; r += WAVE) {
        const double v = fabs(W[r * n + j]);
        if (v > best) { best = v; bi = r; }
      }
      for (int off = WAVE / 2; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, WAVE);
        const int oi = __shfl_xor(bi, off, WAVE);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (tid == 0) {
        piv = bi;
        perm[j] = bi;
        if (!(best > 0.0) || !isfinite(best)) bad = 1;
      }
    }
    __syncthreads();
    const int pr = piv;
    if (pr != j)
      for (int c = tid; c < n; c += 256) {
        const double a = W[j * n + c];
        W[j * n + c] = W[pr * n + c];
        W[pr * n + c] = a;
      }
    __syncthreads();
    for (int r = tid; r < n; r += 256) colj[r] = W[r * n + j];
    if (tid == 0) {
      const double pv = W[j * n + j];
      pinv = pv != 0.0 ? 1.0 / pv : 0.0;
    }
    __syncthreads();
    const double inv = pinv;
    for (int c = tid; c < n; c += 256) W[j * n + c] = (c == j) ? inv : W[j * n + c] * inv;
    __syncthreads();
    for (int e = tid; e < n * n; e += 256) {
      const int r = e / n, c = e % n;
      if (r == j) continue;
      W[r * n + c] = (c == j) ? -colj[r] * inv : fma(-colj[r], W[j * n + c], W[r * n + c]);
    }
    __syncthreads();
  }
  for (int j = n - 1; j >= 0; --j) {
    const int pc = perm[j];
    if (pc != j)
      for (int r = tid; r < n; r += 256) {
        const double a = W[r * n + j];
        W[r * n + j] = W[r * n + pc];
        W[r * n + pc] = a;
      }
    __syncthreads();
  }
  Tout* Xp = X + (long long)p * sX;
  for (int e = tid; e < n * n; e += 256) {
    const int r = e % n, c = e / n;
    Xp[e] = (Tout)W[r * n + c];
  }
  if (tid == 0 && bad) status[0] = 1;
}

// ------------------------------------------------------------ QR (R only)
// Householder QR of a p x k panel; one workgroup of 256 threads per problem.
// The panel is copied to LDS when it fits, else to a global scratch copy.
template <typename T>
__global__ __launch_bounds__(256) void k_qr_r(int p, int k, int ncl, BOp A, T* R, T* ws,
                                              int use_lds, T* Vref, T* taus) {
  extern __shared__ unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  __shared__ double red[4];
  __shared__ T s_beta, s_tau;
  __shared__ double s_v0;
  const int prob = blockIdx.x;
  const int m = prob / ncl, c = prob % ncl;
  const T* Ap = optr<T>(A, m, c);
  T* v = sm;                                  // Householder vector, p entries
  T* W = use_lds ? sm + p : ws + (size_t)prob * p * k;
  const int tid = threadIdx.x, wv = tid / WAVE, lane = tid % WAVE;
  for (int e = tid; e < p * k; e += 256) {
    const int r = e % p, q = e / p;
    W[e] = Ap[r + (long long)q * A.ld];
  }
  __syncthreads();
  const int kr = min(p, k);
  for (int j = 0; j < kr; ++j) {
    // norm of W[j:p, j] (accumulated in FP64)
    double ss = 0.0;
    for (int r = j + 1 + tid; r < p; r += 256) {
      const double x = (double)W[r + (size_t)j * p];
      ss += x * x;
    }
    const double tail = block_sum256(ss, red);
    if (tid == 0) {
      const double alpha = (double)W[j + (size_t)j * p];
      const double nrm = sqrt(alpha * alpha + tail);
      const double beta = alpha >= 0.0 ? -nrm : nrm;
      if (tail == 0.0 || nrm == 0.0) {
        s_tau = T(0);
        s_beta = (T)alpha;
      } else {
        s_tau = (T)((beta - alpha) / beta);
        s_beta = (T)beta;
        s_v0 = alpha - beta;                        // |v0| >= nrm >= |x_r|
      }
    }
    __syncthreads();
    const T tau = s_tau;
    if (tau != T(0)) {
      // v = x / v0 formed in FP64: |v_r| <= 1 even when the column is far
      // below 1/FLT_MAX (columns of inverses decay exponentially), where an
      // FP32 reciprocal of v0 would overflow.
      const double v0 = s_v0;
      for (int r = j + tid; r < p; r += 256)
        v[r] = (r == j) ? T(1) : (T)((double)W[r + (size_t)j * p] / v0);
      __syncthreads();
      if (Vref) {
        T* vo = Vref + (size_t)prob * p * kr + (size_t)j * p;
        for (int r = tid; r < p; r += 256) vo[r] = r < j ? T(0) : v[r];
      }
      // apply (I - tau v v^T) to columns j+1..k-1: one wave per column
      for (int q = j + 1 + wv; q < k; q += 4) {
        T* col = W + (size_t)q * p;
        T d = T(0);
        for (int r = j + lane; r < p; r += WAVE) d = fma(v[r], col[r], d);
        d = wave_sum(d) * tau;
        for (int r = j + lane; r < p; r += WAVE) col[r] = fma(-d, v[r], col[r]);
      }
    }
    if (Vref && tau == T(0)) {
      T* vo = Vref + (size_t)prob * p * kr + (size_t)j * p;
      for (int r = tid; r < p; r += 256) vo[r] = T(0);
    }
    if (Vref && tid == 0) taus[(size_t)prob * kr + j] = tau;
    __syncthreads();
    if (tid == 0) W[j + (size_t)j * p] = s_beta;
    __syncthreads();
  }
  // R = upper trapezoid of W[0:kr, 0:k]
  T* Rp = R + (size_t)prob * kr * k;
  for (int e = tid; e < kr * k; e += 256) {
    const int r = e % kr, q = e / kr;
    Rp[e] = (r <= q) ? W[r + (size_t)q * p] : T(0);
  }
}

// Y = Q [Z; 0] for the Householder Q of a QR with reflectors (v_j, tau_j):
// Y is p x t (column-major, ld = Y.ld, in place), Z is c x t (ld c).
template <typename T>
__global__ __launch_bounds__(256) void k_apply_q(int p, int c, int t, int ncl, const T* Vref,
                                                 const T* taus, const T* Z, long long sZ, int zxor,
                                                 BOp Y) {
  const int prob = blockIdx.x;
  const int m = prob / ncl, cl = prob % ncl;
  T* y = const_cast<T*>(optr<T>(Y, m, cl));
  const T* z = Z + (size_t)(m * ncl + (cl ^ zxor)) * sZ;
  const T* vr = Vref + (size_t)prob * p * c;
  const T* ta = taus + (size_t)prob * c;
  const int tid = threadIdx.x, wv = tid / WAVE, lane = tid % WAVE;
  for (int e = tid; e < p * t; e += 256) {
    const int r = e % p, q = e / p;
    y[r + (long long)q * Y.ld] = r < c ? z[r + (size_t)q * c] : T(0);
  }
  __syncthreads();
  for (int j = c - 1; j >= 0; --j) {
    const T tau = ta[j];
    if (tau != T(0)) {
      const T* v = vr + (size_t)j * p;
      for (int q = wv; q < t; q += 4) {
        T* col = y + (long long)q * Y.ld;
        T d = T(0);
        for (int r = j + lane; r < p; r += WAVE) d = fma(v[r], col[r], d);
        d = wave_sum(d) * tau;
        for (int r = j + lane; r < p; r += WAVE) col[r] = fma(-d, v[r], col[r]);
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------- one-sided Jacobi
template <typename T>
__global__ __launch_bounds__(256) void k_svd(int c, T* Kall, T* Jall, T* sig, T* Usc, T* Jout,
                                             int* rank, double eps, int maxrank, int* sweeps) {
  __shared__ int nrot;
  __shared__ double red[4];
  __shared__ T snorm[512];
  __shared__ int spos[512];
  const int prob = blockIdx.x;
  T* Ak = Kall + (size_t)prob * c * c;
  T* J = Jall + (size_t)prob * c * c;
  const int tid = threadIdx.x;
  for (int e = tid; e < c * c; e += 256) J[e] = (e % c == e / c) ? T(1) : T(0);
  // Frobenius norm for the negligible-column test
  double ss = 0.0;
  for (int e = tid; e < c * c; e += 256) ss += (double)Ak[e] * (double)Ak[e];
  const double fro2 = block_sum256(ss, red);
  const double negl2 = fro2 * Eps<T>::v * Eps<T>::v;
  const double tol = Eps<T>::v * 4.0;
  const int cp = (c + 1) & ~1;          // players (one bye if c is odd)
  const int npairs = cp / 2;
  int g = 256 / max(npairs, 1);         // threads per pair (power of two, <= 64)
  int gp = 1;
  while (gp * 2 <= g && gp * 2 <= WAVE) gp *= 2;
  g = gp;
  const int slots = 256 / g;            // pairs processed concurrently
  const int gl = tid % g;
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) nrot = 0;
    __syncthreads();
    for (int rnd = 0; rnd < cp - 1; ++rnd) {
      for (int pb = 0; pb < npairs; pb += slots) {
        const int pk = pb + tid / g;
        int i = -1, j = -1;
        if (pk < npairs) {
          const int a = (pk == 0) ? 0 : ((rnd + pk - 1) % (cp - 1)) + 1;
          const int b = ((rnd + (cp - 1 - pk) - 1) % (cp - 1)) + 1;
          i = min(a, b); j = max(a, b);
          if (j >= c) { i = -1; j = -1; }
        }
        double al = 0.0, be = 0.0, ga = 0.0;
        if (i >= 0) {
          const T* ai = Ak + (size_t)i * c;
          const T* aj = Ak + (size_t)j * c;
          for (int r = gl; r < c; r += g) {
            const double x = ai[r], y = aj[r];
            al += x * x; be += y * y; ga += x * y;
          }
        }
        al = group_sum(al, g); be = group_sum(be, g); ga = group_sum(ga, g);
        if (i >= 0 && fabs(ga) > tol * sqrt(al * be) && fmax(al, be) > negl2) {
          const double zeta = (be - al) / (2.0 * ga);
          const double az = fabs(zeta);
          double t = (az > 1e15) ? 0.5 / az : 1.0 / (az + sqrt(1.0 + az * az));
          t = copysign(t, zeta);
          const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
          T* ai = Ak + (size_t)i * c;
          T* aj = Ak + (size_t)j * c;
          T* ji = J + (size_t)i * c;
          T* jj = J + (size_t)j * c;
          for (int r = gl; r < c; r += g) {
            const double x = ai[r], y = aj[r];
            ai[r] = (T)(cs * x - sn * y);
            aj[r] = (T)(sn * x + cs * y);
            const double u = ji[r], w = jj[r];
            ji[r] = (T)(cs * u - sn * w);
            jj[r] = (T)(sn * u + cs * w);
          }
          if (gl == 0) atomicAdd(&nrot, 1);
        }
        __syncthreads();
      }
    }
    __syncthreads();
    const int done = (nrot == 0);
    __syncthreads();
    if (sweeps && tid == 0) sweeps[prob] = sweep + 1;
    if (done) break;
  }
  // column norms, sort descending (ties by index), emit
  for (int q = tid; q < c; q += 256) {
    double s2 = 0.0;
    const T* aq = Ak + (size_t)q * c;
    for (int r = 0; r < c; ++r) s2 += (double)aq[r] * (double)aq[r];
    snorm[q] = (T)sqrt(s2);
  }
  __syncthreads();
  for (int q = tid; q < c; q += 256) {
    const T v = snorm[q];
    int pos = 0;
    for (int o = 0; o < c; ++o) pos += (snorm[o] > v) || (snorm[o] == v && o < q);
    spos[q] = pos;
  }
  __syncthreads();
  T* so = sig + (size_t)prob * c;
  T* uo = Usc + (size_t)prob * c * c;
  T* jo = Jout + (size_t)prob * c * c;
  for (int e = tid; e < c * c; e += 256) {
    const int r = e % c, q = e / c;
    const int d = spos[q];
    uo[r + (size_t)d * c] = Ak[e];
    jo[r + (size_t)d * c] = J[e];
  }
  for (int q = tid; q < c; q += 256) so[spos[q]] = snorm[q];
  __syncthreads();
  if (tid == 0) {
    T smax = T(0);
    for (int q = 0; q < c; ++q) smax = snorm[q] > smax ? snorm[q] : smax;
    int t = 0;
    if (smax > T(0)) {
      const double thr = eps * (double)smax;
      for (int q = 0; q < c; ++q) t += ((double)snorm[q] > thr);
    }
    if (maxrank > 0 && t > maxrank) t = maxrank;
    rank[prob] = t;
  }
}

template <typename T>
__global__ void k_trunc_coef(int c, int kout, const T* J, const int* rank, T* Jt) {
  const int prob = blockIdx.y;
  const long long n = (long long)c * kout;
  const int t = rank[prob];
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(e % c), q = (int)(e / c);
    Jt[(size_t)prob * n + e] = (q < t && q < c) ? J[(size_t)prob * c * c + r + (size_t)q * c] : T(0);
  }
}

__global__ void k_max_int(const int* v, int n, int* out) {
  __shared__ int sm[256];
  int mx = 0;
  for (int i = threadIdx.x; i < n; i += 256) mx = max(mx, v[i]);
  sm[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sm[threadIdx.x] = max(sm[threadIdx.x], sm[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sm[0];
}

template <typename T>
__global__ void k_bcopy(int rows, int cols, T alpha, BOp src, BOp dst, int accumulate) {
  const int m = blockIdx.y;
  const T* s = optr<T>(src, m, 0);
  T* d = const_cast<T*>(optr<T>(dst, m, 0));
  const long long n = (long long)rows * cols;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(e % rows), q = (int)(e / rows);
    T* dp = d + r + (long long)q * dst.ld;
    const T v = alpha * s[r + (long long)q * src.ld];
    *dp = accumulate ? *dp + v : v;
  }
}

template <typename T>
__global__ void k_fill(T* p, size_t n, T v) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    p[e] = v;
}

template <typename T>
__global__ void k_bscale(int rows, int cols, int ncl, BOp X, const T* vec, int vmul, int voff,
                         long long vstride, long long vcl, int side, T alpha) {
  const int prob = blockIdx.y;
  const int m = prob / ncl, c = prob % ncl;
  T* x = const_cast<T*>(optr<T>(X, m, c));
  const T* v = vec + (long long)(vmul * m + voff) * vstride + (long long)c * vcl;
  const long long n = (long long)rows * cols;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(e % rows), q = (int)(e / rows);
    x[r + (long long)q * X.ld] *= alpha * v[side ? q : r];
  }
}

template <typename T>
__global__ void k_build_cap(int k, int npairs, const T* cores, T* G) {
  const int q = blockIdx.y;
  const int n = 2 * k;
  const T* c0 = cores + (size_t)(2 * q) * k * k;
  const T* c1 = cores + (size_t)(2 * q + 1) * k * k;
  T* g = G + (size_t)q * n * n;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n * n; e += gridDim.x * blockDim.x) {
    const int r = e % n, col = e / n;
    T v;
    if ((r < k) == (col < k)) v = (r == col) ? T(1) : T(0);
    else if (r < k) v = c1[r + (size_t)(col - k) * k];      // upper-right: c_(2q+1)
    else v = c0[(r - k) + (size_t)col * k];                  // lower-left: c_(2q)
    g[e] = v;
  }
}

template <typename T>
__global__ void k_leaves_tridiag(int s, int b, int bmul, int boff, const double* diag,
                                 const double* west, const double* east, T* leaves) {
  const int m = blockIdx.y;
  const int blk = bmul * m + boff;
  const int nleaf = s / b;
  const long long n = (long long)nleaf * b * b;
  T* lv = leaves + (size_t)m * n;
  const double* dg = diag + (size_t)blk * s;
  const double* we = west + (size_t)blk * s;
  const double* ea = east + (size_t)blk * s;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const int lam = (int)(e / ((long long)b * b));
    const int rem = (int)(e % ((long long)b * b));
    const int r = rem % b, c = rem / b;
    const int gr = lam * b + r;
    double v = 0.0;
    if (c == r) v = dg[gr];
    else if (c == r - 1) v = we[gr];
    else if (c == r + 1) v = ea[gr];
    lv[e] = (T)v;
  }
}

template <typename T>
__global__ void k_rank1(int s, int sd, int bmul, int boff, const double* west, const double* east,
                        T* U, T* V) {
  const int m = blockIdx.y;
  const int blk = bmul * m + boff;
  const double* we = west + (size_t)blk * s;
  const double* ea = east + (size_t)blk * s;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < s; r += gridDim.x * blockDim.x) {
    const int cl = r / sd, loc = r % sd;
    T u = T(0), v = T(0);
    if ((cl & 1) == 0 && loc == sd - 1) { u = (T)ea[r]; v = T(1); }
    if ((cl & 1) == 1 && loc == 0) { u = (T)we[r]; v = T(1); }
    U[(size_t)m * s + r] = u;
    V[(size_t)m * s + r] = v;
  }
}

template <typename T>
__global__ void k_gather_diag(int s, int bmul, int boff, const double* src, T* dst) {
  const int m = blockIdx.y;
  const int blk = bmul * m + boff;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < s; r += gridDim.x * blockDim.x)
    dst[(size_t)m * s + r] = (T)src[(size_t)blk * s + r];
}

template <typename T>
__global__ void k_to_blocks(int s, int nblk, int nrhs, const double* B, long long ld, T* V) {
  const long long n = (long long)s * nblk * nrhs;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(e % s);
    const long long t = e / s;
    const int q = (int)(t % nrhs);
    const int i = (int)(t / nrhs);
    V[e] = (T)B[(long long)i * s + j + (long long)q * ld];
  }
}

template <typename T>
__global__ void k_from_blocks(int s, int nblk, int nrhs, const T* V, double* B, long long ld) {
  const long long n = (long long)s * nblk * nrhs;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(e % s);
    const long long t = e / s;
    const int q = (int)(t % nrhs);
    const int i = (int)(t / nrhs);
    B[(long long)i * s + j + (long long)q * ld] = (double)V[e];
  }
}

template <typename T>
__global__ void k_bdiag_axpy(int s, int nrhs, T alpha, const T* d, int dmul, int doff, const T* x,
                             int xmul, int xoff, T* y, int ymul, int yoff) {
  const int m = blockIdx.y;
  const T* dd = d + (size_t)(dmul * m + doff) * s;
  const T* xx = x + (size_t)(xmul * m + xoff) * s * nrhs;
  T* yy = y + (size_t)(ymul * m + yoff) * s * nrhs;
  const int n = s * nrhs;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x)
    yy[e] = fma(alpha * dd[e % s], xx[e], yy[e]);
}

__global__ void k_residual(int nx, int ny, const double* diag, const double* west,
                           const double* east, const double* south, const double* north,
                           const double* X, const double* B, double* R) {
  const long long N = (long long)nx * ny;
  const int q = blockIdx.y;
  const double* x = X + q * N;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < N;
       e += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(e % nx);
    const int i = (int)(e / nx);
    double ax = diag[e] * x[e];
    if (j > 0) ax += west[e] * x[e - 1];
    if (j + 1 < nx) ax += east[e] * x[e + 1];
    if (i > 0) ax += south[e] * x[e - nx];
    if (i + 1 < ny) ax += north[e] * x[e + nx];
    R[e + q * N] = B[e + q * N] - ax;
  }
}

// Partial sums of squares: block (x, q) covers a contiguous chunk of column q.
__global__ void k_col_sumsq_part(long long n, long long chunk, const double* A, double* part) {
  __shared__ double red[4];
  const int q = blockIdx.y;
  const long long lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
  double s = 0.0;
  for (long long i = lo + threadIdx.x; i < hi; i += 256) {
    const double v = A[i + q * n];
    s += v * v;
  }
  s = block_sum256(s, red);
  if (threadIdx.x == 0) part[(size_t)q * gridDim.x + blockIdx.x] = s;
}

__global__ void k_col_sumsq_final(int nparts, const double* part, double* out) {
  __shared__ double red[4];
  const int q = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 256) s += part[(size_t)q * nparts + i];
  s = block_sum256(s, red);
  if (threadIdx.x == 0) out[q] = s;
}

template <typename T>
__global__ void k_scan_values(long long n, const T* a, int* bad, double* amax) {
  __shared__ double red[4];
  double mx = 0.0;
  int b = 0;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const double v = (double)a[e];
    if (!isfinite(v)) b = 1;
    else mx = fmax(mx, fabs(v));
  }
  if (b) bad[0] = 1;
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, WAVE));
  if (threadIdx.x % WAVE == 0) red[threadIdx.x / WAVE] = mx;
  __syncthreads();
  if (threadIdx.x == 0) amax[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

__global__ void k_count_nonfinite(long long n, const double* a, int* out) {
  int bad = 0;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    bad |= !isfinite(a[e]);
  if (bad) out[0] = 1;
}

__global__ void k_axpy_d(long long n, const double* D, double* X) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    X[e] += D[e];
}

inline unsigned grid1(long long n, int bs = 256, long long cap = 65535) {
  long long g = (n + bs - 1) / bs;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

// ================================================================ launchers
template <typename T>
void bgemm(hipStream_t st, int M, int N, int K, int nmat, int ncl, T alpha, const BOp& A,
           const BOp& B, T beta, const BOp& C) {
  if (M <= 0 || N <= 0 || nmat <= 0 || ncl <= 0) return;
  const int nprob = nmat * ncl;
  ProfScope ps(KC_GEMM, st, 2.0 * M * N * K * nprob,
               (double)sizeof(T) * nprob * ((double)M * K + (double)K * N + (double)M * N * (beta != T(0) ? 2 : 1)));
  // pick the tile shape with the least padded area (bigger tiles preferred)
  struct Cfg { int tm, tn; double eff; };
  const Cfg cfgs[] = {{64, 64, 1.0}, {64, 16, 0.8}, {16, 64, 0.8}, {32, 32, 0.8}, {16, 16, 0.55}};
  int best = 0;
  double bc = 1e300;
  for (int i = 0; i < 5; ++i) {
    const double pm = (double)((M + cfgs[i].tm - 1) / cfgs[i].tm) * cfgs[i].tm;
    const double pn = (double)((N + cfgs[i].tn - 1) / cfgs[i].tn) * cfgs[i].tn;
    const double cost = pm * pn / cfgs[i].eff;
    if (cost < bc) { bc = cost; best = i; }
  }
  switch (best) {
    case 0: launch_gemm<T, 64, 64, 4, 4>(st, M, N, K, nprob, ncl, alpha, A, B, beta, C); break;
    case 1: launch_gemm<T, 64, 16, 4, 4>(st, M, N, K, nprob, ncl, alpha, A, B, beta, C); break;
    case 2: launch_gemm<T, 16, 64, 4, 4>(st, M, N, K, nprob, ncl, alpha, A, B, beta, C); break;
    case 3: launch_gemm<T, 32, 32, 4, 4>(st, M, N, K, nprob, ncl, alpha, A, B, beta, C); break;
    default: launch_gemm<T, 16, 16, 2, 2>(st, M, N, K, nprob, ncl, alpha, A, B, beta, C); break;
  }
}

template <typename Tin, typename Tout>
void binverse(hipStream_t st, int n, int nprob, const Tin* A, long long sA, Tout* X, long long sX,
              int* status) {
  if (n <= 0 || nprob <= 0) return;
  ProfScope ps(KC_INVERSE, st, 2.0 * n * n * n * nprob, 2.0 * n * n * nprob * sizeof(Tin));
  if (n <= 88) {   // in place: n*n doubles of LDS (+1.6 KB static) within 64 KB
    hipLaunchKernelGGL((k_inverse_lds<Tin, Tout>), dim3(nprob), dim3(256), (size_t)n * n * sizeof(double),
                       st, n, A, sA, X, sX, status);
    ACR_CHECK_LAUNCH();
    return;
  }
  const size_t lds = (size_t)n * 2 * n * sizeof(double);
  const bool use_lds = lds + 2048 <= kMaxLds;
  DBuf<double> ws;
  if (!use_lds || n > 128) ws.resize((size_t)nprob * n * (2 * n + 1));
  hipLaunchKernelGGL((k_inverse<Tin, Tout>), dim3(nprob), dim3(256), use_lds ? lds : 0, st, n, A,
                     sA, X, sX, ws.get(), use_lds ? 1 : 0, status);
  ACR_CHECK_LAUNCH();
}

template <typename T>
void bqr_r(hipStream_t st, int p, int k, int nmat, int ncl, const BOp& A, T* R, T* Vref, T* tau) {
  if (p <= 0 || k <= 0 || nmat <= 0) return;
  const int nprob = nmat * ncl;
  const double kr = std::min(p, k);
  ProfScope ps(KC_QR, st,
               nprob * (p >= k ? 2.0 * k * k * (p - k / 3.0) : 2.0 * p * p * (k - p / 3.0)),
               (double)sizeof(T) * nprob * ((double)p * k + kr * k + (Vref ? (double)p * kr : 0.0)));
  const size_t panel = (size_t)p * k * sizeof(T);
  const size_t vbytes = (size_t)p * sizeof(T);
  const bool use_lds = panel + vbytes + 1024 <= kMaxLds;
  DBuf<T> ws;
  if (!use_lds) ws.resize((size_t)nprob * p * k);
  hipLaunchKernelGGL((k_qr_r<T>), dim3(nprob), dim3(256), use_lds ? panel + vbytes : vbytes, st, p,
                     k, ncl, A, R, ws.get(), use_lds ? 1 : 0, Vref, tau);
  ACR_CHECK_LAUNCH();
}

template <typename T>
void bapply_q(hipStream_t st, int p, int c, int t, int nmat, int ncl, const T* Vref, const T* tau,
              const T* Z, long long sZ, int zxor, const BOp& Y) {
  if (p <= 0 || t <= 0 || nmat <= 0) return;
  ProfScope ps(KC_APPLYQ, st, 4.0 * nmat * ncl * t * ((double)p * c - 0.5 * c * c),
               (double)sizeof(T) * nmat * ncl * ((double)p * c + (double)c * t + (double)p * t));
  hipLaunchKernelGGL((k_apply_q<T>), dim3(nmat * ncl), dim3(256), 0, st, p, c, t, ncl, Vref, tau, Z,
                     sZ, zxor, Y);
  ACR_CHECK_LAUNCH();
}

template <typename T>
void bsvd(hipStream_t st, int c, int nprob, T* K, T* sig, T* Usc, T* J, int* rank, double eps,
          int maxrank) {
  if (c <= 0 || nprob <= 0) return;
  if (c > 512) fail(ACR_ERR_INVALID_ARG, "bsvd: core larger than 512");
  DBuf<T> Jw((size_t)nprob * c * c);
  int* sweeps = nullptr;
  Profiler& P = Profiler::get();
  if (P.on(KC_SVD)) {
    std::lock_guard<std::mutex> g(P.mu());
    P.owned().emplace_back((size_t)nprob);
    sweeps = P.owned().back().get();
  }
  ProfScope ps(KC_SVD, st, 0.0, 3.0 * (double)c * c * nprob * sizeof(T));
  ps.r.dev_sweeps = sweeps; ps.r.nprob = nprob; ps.r.c = c;
  hipLaunchKernelGGL((k_svd<T>), dim3(nprob), dim3(256), 0, st, c, K, Jw.get(), sig, Usc, J, rank,
                     eps, maxrank, sweeps);
  ACR_CHECK_LAUNCH();
}

template <typename T>
void btrunc_coef(hipStream_t st, int c, int kout, int nprob, const T* J, const int* rank, T* Jt) {
  if (c <= 0 || kout <= 0 || nprob <= 0) return;
  dim3 g(grid1((long long)c * kout, 256, 64), nprob);
  hipLaunchKernelGGL((k_trunc_coef<T>), g, dim3(256), 0, st, c, kout, J, rank, Jt);
  ACR_CHECK_LAUNCH();
}

void bmax_int(hipStream_t st, const int* rank, int n, int* out) {
  hipLaunchKernelGGL(k_max_int, dim3(1), dim3(256), 0, st, rank, n, out);
  ACR_CHECK_LAUNCH();
}

template <typename T>
void bcopy(hipStream_t st, int rows, int cols, int nmat, T alpha, const BOp& src, const BOp& dst) {
  if (rows <= 0 || cols <= 0 || nmat <= 0) return;
  ProfScope ps(KC_COPY, st, 0.0, 2.0 * rows * cols * nmat * sizeof(T));
  dim3 g(grid1((long long)rows * cols, 256, 1024), nmat);
  hipLaunchKernelGGL((k_bcopy<T>), g, dim3(256), 0, st, rows, cols, alpha, src, dst, 0);
  ACR_CHECK_LAUNCH();
}

template <typename T>
void badd(hipStream_t st, int rows, int cols, int nmat, T alpha, const BOp& src, const BOp& dst) {
  if (rows <= 0 || cols <= 0 || nmat <= 0) return;
  ProfScope ps(KC_COPY, st, (double)rows * cols * nmat, 3.0 * rows * cols * nmat * sizeof(T));
  dim3 g(grid1((long long)rows * cols, 256, 1024), nmat);
  hipLaunchKernelGGL((k_bcopy<T>), g, dim3(256), 0, st, rows, cols, alpha, src, dst, 1);
  ACR_CHECK_LAUNCH();
}

template <typename T>
void fill(hipStream_t st, T* p, size_t n, T v) {
  if (!n) return;
  hipLaunchKernelGGL((k_fill<T>), dim3(grid1((long long)n, 256, 16384)), dim3(256), 0, st, p, n, v);
  ACR_CHECK_LAUNCH();
}

template <typename T>
void bscale(hipStream_t st, int rows, int cols, int nmat, int ncl, const BOp& X, const T* vec,
            int vmul, int voff, long long vstride, long long vcl, int side, T alpha) {
  if (rows <= 0 || cols <= 0 || nmat <= 0) return;
  ProfScope ps(KC_COPY, st, (double)rows * cols * nmat * ncl, 2.0 * rows * cols * nmat * ncl * sizeof(T));
  dim3 g(grid1((long long)rows * cols, 256, 256), nmat * ncl);
  hipLaunchKernelGGL((k_bscale<T>), g, dim3(256), 0, st, rows, cols, ncl, X, vec, vmul, voff,
                     vstride, vcl, side, alpha);
  ACR_CHECK_LAUNCH();
}

template <typename T>
void build_capacitance(hipStream_t st, int k, int npairs, const T* cores, T* G) {
  if (k <= 0 || npairs <= 0) return;
  dim3 g(grid1(4LL * k * k, 256, 64), npairs);
  hipLaunchKernelGGL((k_build_cap<T>), g, dim3(256), 0, st, k, npairs, cores, G);
  ACR_CHECK_LAUNCH();
}

template <typename T>
void build_leaves_tridiag(hipStream_t st, int s, int b, int nmat, int bmul, int boff,
                          const double* diag, const double* west, const double* east, T* leaves) {
  if (nmat <= 0) return;
  dim3 g(grid1((long long)s * b, 256, 256), nmat);
  hipLaunchKernelGGL((k_leaves_tridiag<T>), g, dim3(256), 0, st, s, b, bmul, boff, diag, west, east,
                     leaves);
  ACR_CHECK_LAUNCH();
}

template <typename T>
void build_rank1_factors(hipStream_t st, int s, int sd, int nmat, int bmul, int boff,
                         const double* west, const double* east, T* U, T* V) {
  if (nmat <= 0) return;
  dim3 g(grid1(s, 256, 64), nmat);
  hipLaunchKernelGGL((k_rank1<T>), g, dim3(256), 0, st, s, sd, bmul, boff, west, east, U, V);
  ACR_CHECK_LAUNCH();
}

template <typename T>
void gather_diag(hipStream_t st, int s, int nmat, int bmul, int boff, const double* src, T* dst) {
  if (nmat <= 0) return;
  dim3 g(grid1(s, 256, 64), nmat);
  hipLaunchKernelGGL((k_gather_diag<T>), g, dim3(256), 0, st, s, bmul, boff, src, dst);
  ACR_CHECK_LAUNCH();
}

template <typename T>
void to_blocks(hipStream_t st, int s, int nblk, int nrhs, const double* B, long long ld, T* V) {
  const long long n = (long long)s * nblk * nrhs;
  if (n <= 0) return;
  ProfScope ps(KC_OTHER, st, 0.0, (double)n * (8 + sizeof(T)));
  hipLaunchKernelGGL((k_to_blocks<T>), dim3(grid1(n, 256, 16384)), dim3(256), 0, st, s, nblk, nrhs,
                     B, ld, V);
  ACR_CHECK_LAUNCH();
}

template <typename T>
void from_blocks(hipStream_t st, int s, int nblk, int nrhs, const T* V, double* B, long long ld) {
  const long long n = (long long)s * nblk * nrhs;
  if (n <= 0) return;
  ProfScope ps(KC_OTHER, st, 0.0, (double)n * (8 + sizeof(T)));
  hipLaunchKernelGGL((k_from_blocks<T>), dim3(grid1(n, 256, 16384)), dim3(256), 0, st, s, nblk,
                     nrhs, V, B, ld);
  ACR_CHECK_LAUNCH();
}

template <typename T>
void bdiag_axpy(hipStream_t st, int s, int nrhs, int nmat, T alpha, const T* d, int dmul, int doff,
                const T* x, int xmul, int xoff, T* y, int ymul, int yoff) {
  if (nmat <= 0) return;
  ProfScope ps(KC_MATVEC, st, 2.0 * s * nrhs * nmat, (double)sizeof(T) * nmat * (3.0 * s * nrhs + s));
  dim3 g(grid1((long long)s * nrhs, 256, 256), nmat);
  hipLaunchKernelGGL((k_bdiag_axpy<T>), g, dim3(256), 0, st, s, nrhs, alpha, d, dmul, doff, x, xmul,
                     xoff, y, ymul, yoff);
  ACR_CHECK_LAUNCH();
}

void stencil_residual(hipStream_t st, int nx, int ny, int nrhs, const double* diag,
                      const double* west, const double* east, const double* south,
                      const double* north, const double* X, const double* B, double* R) {
  const long long N = (long long)nx * ny;
  ProfScope ps(KC_OTHER, st, 10.0 * N * nrhs, 8.0 * N * (5.0 + 3.0 * nrhs));
  dim3 g(grid1(N, 256, 8192), nrhs);
  hipLaunchKernelGGL(k_residual, g, dim3(256), 0, st, nx, ny, diag, west, east, south, north, X, B,
                     R);
  ACR_CHECK_LAUNCH();
}

void col_sumsq(hipStream_t st, long long n, int ncol, const double* A, double* out) {
  const int nparts = (int)std::min<long long>(512, std::max<long long>(1, (n + 4095) / 4096));
  const long long chunk = (n + nparts - 1) / nparts;
  DBuf<double> part((size_t)nparts * ncol);
  hipLaunchKernelGGL(k_col_sumsq_part, dim3(nparts, ncol), dim3(256), 0, st, n, chunk, A, part.get());
  ACR_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_col_sumsq_final, dim3(ncol), dim3(256), 0, st, nparts, part.get(), out);
  ACR_CHECK_LAUNCH();
}

void flag_nonfinite(hipStream_t st, long long n, const double* a, int* flag) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_count_nonfinite, dim3(grid1(n, 256, 4096)), dim3(256), 0, st, n, a, flag);
  ACR_CHECK_LAUNCH();
}

template <typename T>
void scan_values(hipStream_t st, long long n, const T* a, bool* bad, double* amax) {
  *bad = false;
  *amax = 0.0;
  if (n <= 0) return;
  const unsigned g = grid1(n, 256, 1024);
  DBuf<int> flag(1);
  DBuf<double> mx(g);
  ACR_HIP(hipMemsetAsync(flag.get(), 0, sizeof(int), st));
  hipLaunchKernelGGL((k_scan_values<T>), dim3(g), dim3(256), 0, st, n, a, flag.get(), mx.get());
  ACR_CHECK_LAUNCH();
  int hb = 0;
  std::vector<double> hm(g);
  ACR_HIP(hipMemcpyAsync(&hb, flag.get(), sizeof(int), hipMemcpyDeviceToHost, st));
  ACR_HIP(hipMemcpyAsync(hm.data(), mx.get(), g * sizeof(double), hipMemcpyDeviceToHost, st));
  ACR_HIP(hipStreamSynchronize(st));
  *bad = hb != 0;
  for (double v : hm) *amax = std::max(*amax, v);
}
template void scan_values<float>(hipStream_t, long long, const float*, bool*, double*);
template void scan_values<double>(hipStream_t, long long, const double*, bool*, double*);

void axpy_d(hipStream_t st, long long n, const double* D, double* X) {
  hipLaunchKernelGGL(k_axpy_d, dim3(grid1(n, 256, 16384)), dim3(256), 0, st, n, D, X);
  ACR_CHECK_LAUNCH();
}

#define INST(T)                                                                                   \
  template void bgemm<T>(hipStream_t, int, int, int, int, int, T, const BOp&, const BOp&, T,      \
                         const BOp&);                                                             \
  template void bqr_r<T>(hipStream_t, int, int, int, int, const BOp&, T*, T*, T*);                \
  template void bapply_q<T>(hipStream_t, int, int, int, int, int, const T*, const T*, const T*,   \
                            long long, int, const BOp&);                                          \
  template void bsvd<T>(hipStream_t, int, int, T*, T*, T*, T*, int*, double, int);                \
  template void btrunc_coef<T>(hipStream_t, int, int, int, const T*, const int*, T*);             \
  template void bcopy<T>(hipStream_t, int, int, int, T, const BOp&, const BOp&);                  \
  template void badd<T>(hipStream_t, int, int, int, T, const BOp&, const BOp&);                   \
  template void fill<T>(hipStream_t, T*, size_t, T);                                              \
  template void bscale<T>(hipStream_t, int, int, int, int, const BOp&, const T*, int, int,        \
                          long long, long long, int, T);                                          \
  template void build_capacitance<T>(hipStream_t, int, int, const T*, T*);                        \
  template void build_leaves_tridiag<T>(hipStream_t, int, int, int, int, int, const double*,      \
                                        const double*, const double*, T*);                        \
  template void build_rank1_factors<T>(hipStream_t, int, int, int, int, int, const double*,       \
                                       const double*, T*, T*);                                    \
  template void gather_diag<T>(hipStream_t, int, int, int, int, const double*, T*);               \
  template void to_blocks<T>(hipStream_t, int, int, int, const double*, long long, T*);           \
  template void from_blocks<T>(hipStream_t, int, int, int, const T*, double*, long long);         \
  template void bdiag_axpy<T>(hipStream_t, int, int, int, T, const T*, int, int, const T*, int,   \
                              int, T*, int, int);

INST(float)
INST(double)
#undef INST

template void binverse<double, double>(hipStream_t, int, int, const double*, long long, double*,
                                       long long, int*);
template void binverse<float, float>(hipStream_t, int, int, const float*, long long, float*,
                                     long long, int*);

}  // namespace acr
