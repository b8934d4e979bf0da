// Device kernels of the ACR library for gfx950 (CDNA4, 64-wide wavefronts).
//
// The H-arithmetic of every cyclic-reduction level is expressed as batched
// operations over (matrix, cluster) problems of uniform shape; this file holds
// the batched primitives: a tiled batched GEMM, dense inverses (leaves and
// capacitance matrices), Householder R factors and one-sided Jacobi SVDs for
// recompression, plus the elementwise, layout and residual kernels.
#include "kernels.hpp"

#include <algorithm>
#include <cctype>
#include <cfloat>
#include <cmath>
#include <mutex>
#include <set>
#include <string>
#include <vector>

namespace acr {

namespace {

constexpr int WAVE = 64;
constexpr size_t kMaxLds = 65536;        // LDS budget of a workgroup that shares its CU
constexpr size_t kMaxLdsLarge = 163840;  // all the LDS a gfx950 workgroup may hold
constexpr size_t kMaxDynLarge = kMaxLdsLarge - 16384;   // dynamic part next to <= 16 KB static
constexpr long long kSmallLaunch = 1024;   // workgroups below which shape variants share a launch
constexpr int kApplyRows = 8;        // Q application in registers: rows per lane (p <= 512)
constexpr int kApplyCols = 8;        // and output columns per wave (t <= 32)

// Device pointers taken from job descriptors reach a kernel as generic
// pointers, for which the compiler emits FLAT accesses; a FLAT access also
// counts against the LDS and scalar-load wait counter, so each wait for an LDS
// read or a descriptor load (and the wait ahead of every barrier) would also
// wait for the global loads and stores in flight.  gmem() restates such a
// pointer in the global address space (every descriptor pointer is device
// memory), so that the compiler emits global loads and stores, which only the
// vector-memory counter tracks.
template <typename T>
__device__ __forceinline__ T* gmem(T* p) {
  return (T*)(__attribute__((address_space(1))) T*)(uintptr_t)p;
}

template <typename T>
__device__ __forceinline__ const T* optr(const BOp& o, int m, int c) {
  const int cc = (c >> o.cshift) ^ o.cxor;
  return gmem(static_cast<const T*>(o.p)) + (long long)(o.mmul * m + o.moff) * o.sm +
         (long long)(cc >> 1) * o.sc_pair + (long long)(cc & 1) * o.sc_odd;
}

// Job owning workgroup `bid` in a grouped launch (jobs sorted by block0).
template <typename J>
__device__ __forceinline__ int job_of(const J* jobs, int n, long long bid) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].block0 <= bid) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Cross-lane moves with DPP (data-parallel primitives: register operand
// modifiers of VALU instructions, no LDS round trip).  Lanes whose source is
// out of range or masked off read 0.
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ float dpp_mov(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROWMASK, 0xf, false));
}
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ double dpp_mov(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWMASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, ROWMASK, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float lane_read(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ double lane_read(double x, int l) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)v, l);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <int CTRL>
__device__ __forceinline__ int dpp_mov_i(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xf, 0xf, false);
}

// 64-bit lane move with DPP (out-of-range sources read the lane's own value).
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_mov_u64(unsigned long long x) {
  const int lo = (int)(unsigned)x, hi = (int)(unsigned)(x >> 32);
  const int l2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, false);
  const int h2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, false);
  return ((unsigned long long)(unsigned)h2 << 32) | (unsigned)l2;
}
__device__ __forceinline__ unsigned long long lane_read_u64(unsigned long long x, int l) {
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)x, l);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(x >> 32), l);
  return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}
// Maximum of a 64-bit key over aligned groups of N lanes (N = 8, 16, 32, 64),
// returned to every lane of the group: quad and mirror DPP steps give the
// maximum of each row of 16 to all its lanes, lane reads combine rows.
template <int N>
__device__ __forceinline__ unsigned long long group_max_u64(unsigned long long k) {
  auto mx = [](unsigned long long a, unsigned long long b) { return a > b ? a : b; };
  k = mx(k, dpp_mov_u64<0xb1>(k));     // quad_perm [1,0,3,2]
  k = mx(k, dpp_mov_u64<0x4e>(k));     // quad_perm [2,3,0,1]
  if constexpr (N >= 8) k = mx(k, dpp_mov_u64<0x141>(k));    // row_half_mirror
  if constexpr (N >= 16) k = mx(k, dpp_mov_u64<0x140>(k));   // row_mirror
  if constexpr (N == 32) {
    const unsigned long long a = mx(lane_read_u64(k, 15), lane_read_u64(k, 31));
    const unsigned long long b = mx(lane_read_u64(k, 47), lane_read_u64(k, 63));
    k = (threadIdx.x % WAVE) < 32 ? a : b;
  } else if constexpr (N == 64) {
    k = mx(mx(lane_read_u64(k, 15), lane_read_u64(k, 31)), mx(lane_read_u64(k, 47), lane_read_u64(k, 63)));
  }
  return k;
}

// Sum over the 64 lanes of a wave, returned to every lane: quad sums
// (quad_perm), row-of-16 sums (row_shr 4, 8: the last lane of each row holds
// its row's total), then row_bcast 15 / 31 carry the row totals into lane 63,
// which is read back as a scalar.  Every lane of the wave must be active.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  v += dpp_mov<0xb1>(v);        // quad_perm [1,0,3,2]
  v += dpp_mov<0x4e>(v);        // quad_perm [2,3,0,1]
  v += dpp_mov<0x114>(v);       // row_shr:4
  v += dpp_mov<0x118>(v);       // row_shr:8
  v += dpp_mov<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_mov<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return lane_read(v, 63);
}

// Sum within aligned groups of g lanes (g a power of two <= 64), returned to
// every lane of the group: quad_perm swaps, then the half-row and row
// mirrors (each step adds the partner half, so every lane of a group ends
// with the same value); groups of 32 and 64 combine the four row totals
// read as scalars.  Every lane of the wave must be active.
template <typename T>
__device__ __forceinline__ T group_sum(T v, int g) {
  if (g >= 2) v += dpp_mov<0xb1>(v);    // quad_perm [1,0,3,2]
  if (g >= 4) v += dpp_mov<0x4e>(v);    // quad_perm [2,3,0,1]
  if (g >= 8) v += dpp_mov<0x141>(v);   // row_half_mirror
  if (g >= 16) v += dpp_mov<0x140>(v);  // row_mirror
  if (g >= 32) {
    const T r0 = lane_read(v, 0), r1 = lane_read(v, 16), r2 = lane_read(v, 32), r3 = lane_read(v, 48);
    if (g == 32) v = (threadIdx.x % WAVE) < 32 ? r0 + r1 : r2 + r3;
    else v = (r0 + r1) + (r2 + r3);
  }
  return v;
}

// Largest value over the wave, ties to the smallest index; the pair is
// returned to every lane.  Same DPP steps as group_sum.  Every lane of the
// wave must be active.
__device__ __forceinline__ void wave_argmax(double& best, int& bi) {
  auto step = [&](double ob, int oi) {
    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
  };
  step(dpp_mov<0xb1>(best), dpp_mov_i<0xb1>(bi));
  step(dpp_mov<0x4e>(best), dpp_mov_i<0x4e>(bi));
  step(dpp_mov<0x141>(best), dpp_mov_i<0x141>(bi));
  step(dpp_mov<0x140>(best), dpp_mov_i<0x140>(bi));
  double b0 = lane_read(best, 0);
  int i0 = __builtin_amdgcn_readlane(bi, 0);
  for (int r = 16; r < WAVE; r += 16) {
    const double ob = lane_read(best, r);
    const int oi = __builtin_amdgcn_readlane(bi, r);
    if (ob > b0 || (ob == b0 && oi < i0)) { b0 = ob; i0 = oi; }
  }
  best = b0;
  bi = i0;
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

// Sum over the NW waves of a workgroup; every thread gets the result.
template <int NW, typename T>
__device__ T block_sum_n(T v, T* red) {
  if (NW == 1) return wave_sum(v);
  v = wave_sum(v);
  const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  T r = red[0];
  for (int i = 1; i < NW; ++i) r += red[i];
  return r;
}

template <typename T> struct Eps;
template <> struct Eps<float> { static constexpr double v = 5.9604644775390625e-8; };
template <> struct Eps<double> { static constexpr double v = 1.1102230246251565e-16; };

// ------------------------------------------------------------------ GEMM
// Grouped, K-segmented batched GEMM.  A workgroup computes one TM x TN tile
// of one problem of one job, accumulating over every segment of the job;
// each thread holds RM x RN outputs, operands are staged through LDS in TK
// slices.
template <typename T, int TM, int TN, int TK, int RM, int RN>
__device__ __forceinline__ void ggemm_body(const GJob* __restrict__ jobs,
                                                                int njobs,
                                                                const GSeg* __restrict__ segs, long long bid) {
  constexpr int TX = TM / RM, TY = TN / RN, NT = TX * TY;
  __shared__ T As[TK][TM + 1];
  __shared__ T Bs[TK][TN + 1];
  
  const GJob& J = jobs[job_of(jobs, njobs, bid)];
  const int tilesM = J.tilesM;
  const int tiles = tilesM * J.tilesN;
  const long long local = bid - J.block0;
  const int prob = (int)(local / tiles);
  const int t = (int)(local % tiles);
  const int tm = t % tilesM, tn = t / tilesM;
  const int m = prob / J.ncl, c = prob % J.ncl;
  const int M = J.M, N = J.N;
  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const int i0 = tm * TM, j0 = tn * TN;
  T acc[RM][RN];
#pragma unroll
  for (int r = 0; r < RM; ++r)
#pragma unroll
    for (int q = 0; q < RN; ++q) acc[r][q] = T(0);
  for (int sg = 0; sg < J.nseg; ++sg) {
    const GSeg& S = segs[J.seg0 + sg];
    const int K = S.K;
    const int lda = S.A.ld, ldb = S.B.ld, ta = S.A.trans, tb = S.B.trans;
    const T sscale = (T)S.scale;
    const T* Ap = optr<T>(S.A, m, c);
    const T* Bp = optr<T>(S.B, m, c);
    // the next K slice is loaded into registers while the current one is
    // multiplied out of LDS (same values, same product order)
    constexpr int LA = (TM * TK + NT - 1) / NT, LB = (TK * TN + NT - 1) / NT;
    T ra[LA], rb[LB];
    auto fetch = [&](int k0) {
#pragma unroll
      for (int u = 0; u < LA; ++u) {
        const int e = tid + u * NT;
        int i, kk;
        if (!ta) { i = e % TM; kk = e / TM; } else { kk = e % TK; i = e / TK; }
        const int gi = i0 + i, gk = k0 + kk;
        T v = T(0);
        if (e < TM * TK && gi < M && gk < K) v = ta ? Ap[gk + (long long)gi * lda] : Ap[gi + (long long)gk * lda];
        ra[u] = v * sscale;
      }
#pragma unroll
      for (int u = 0; u < LB; ++u) {
        const int e = tid + u * NT;
        int kk, jj;
        if (!tb) { kk = e % TK; jj = e / TK; } else { jj = e % TN; kk = e / TN; }
        const int gk = k0 + kk, gj = j0 + jj;
        T v = T(0);
        if (e < TK * TN && gk < K && gj < N) v = tb ? Bp[gj + (long long)gk * ldb] : Bp[gk + (long long)gj * ldb];
        rb[u] = v;
      }
    };
    if (K > 0) fetch(0);
    for (int k0 = 0; k0 < K; k0 += TK) {
#pragma unroll
      for (int u = 0; u < LA; ++u) {
        const int e = tid + u * NT;
        if (e >= TM * TK) break;
        int i, kk;
        if (!ta) { i = e % TM; kk = e / TM; } else { kk = e % TK; i = e / TK; }
        As[kk][i] = ra[u];
      }
#pragma unroll
      for (int u = 0; u < LB; ++u) {
        const int e = tid + u * NT;
        if (e >= TK * TN) break;
        int kk, jj;
        if (!tb) { kk = e % TK; jj = e / TK; } else { jj = e % TN; kk = e / TN; }
        Bs[kk][jj] = rb[u];
      }
      __syncthreads();
      if (k0 + TK < K) fetch(k0 + TK);
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
  }
  T* Cp = const_cast<T*>(optr<T>(J.C, m, c));
  const int ldc = J.C.ld;
  const T alpha = (T)J.alpha, beta = (T)J.beta;
#pragma unroll
  for (int r = 0; r < RM; ++r) {
    const int gi = i0 + tx + r * TX;
    if (gi >= M) continue;
#pragma unroll
    for (int q = 0; q < RN; ++q) {
      const int gj = j0 + ty + q * TY;
      if (gj >= N) continue;
      T* cp = Cp + gi + (long long)gj * ldc;
      T v = alpha * acc[r][q];
      if (beta != T(0)) v = fma(beta, *cp, v);
      *cp = v;
    }
  }
}

template <typename T, int TM, int TN, int TK, int RM, int RN>
__global__ __launch_bounds__((TM / RM) * (TN / RN)) void k_ggemm(const GJob* __restrict__ jobs, int njobs,
    const GSeg* __restrict__ segs) {
  ggemm_body<T, TM, TN, TK, RM, RN>(jobs, njobs, segs, blockIdx.x);
}

// The FP32 tile GEMM on the matrix cores (v_mfma_f32_16x16x4f32): the same
// jobs, tiles and LDS staging as ggemm_body, but a wave owns BM x BN output
// blocks of 16 x 16 and each K step of four is one MFMA per block.  Lane l
// feeds A[i0 + l % 16][k + l / 16] and B[k + l / 16][j0 + l % 16] and holds
// rows 4 (l / 16) .. 4 (l / 16) + 3 of column l % 16 of the block.  Every
// output sums its K terms four at a time in K order whatever the tile, so the
// five tile shapes give the same bits (as the vector tiles do among
// themselves in FP64).  LDS rows are padded to 16 banks apart so that the two
// 16-lane halves of a 32-lane LDS access read disjoint banks.
typedef float v4f32 __attribute__((ext_vector_type(4)));

template <int TM, int TN, int WM, int WN, int TK = 16>
__device__ __forceinline__ void ggemm_mfma_body(const GJob* __restrict__ jobs, int njobs,
                                                const GSeg* __restrict__ segs, long long bid) {
  constexpr int NT = WM * WN * WAVE;
  constexpr int BM = TM / (16 * WM), BN = TN / (16 * WN);
  constexpr int LA = TM % 32 == 0 ? TM + 16 : TM, LB = TN % 32 == 0 ? TN + 16 : TN;
  static_assert(BM >= 1 && BN >= 1 && BM * 16 * WM == TM && BN * 16 * WN == TN, "tile");
  __shared__ float As[TK][LA];
  __shared__ float Bs[TK][LB];

  const GJob& J = jobs[job_of(jobs, njobs, bid)];
  const int tilesM = J.tilesM;
  const int tiles = tilesM * J.tilesN;
  const long long local = bid - J.block0;
  const int prob = (int)(local / tiles);
  const int t = (int)(local % tiles);
  const int tm = t % tilesM, tn = t / tilesM;
  const int m = prob / J.ncl, c = prob % J.ncl;
  const int M = J.M, N = J.N;
  const int tid = threadIdx.x;
  const int lane = tid % WAVE;
  const int w = __builtin_amdgcn_readfirstlane(tid / WAVE);
  const int wm = w % WM, wn = w / WM;
  const int i0 = tm * TM, j0 = tn * TN;
  const int lr = lane % 16, lk = lane / 16;
  v4f32 acc[BM][BN];
#pragma unroll
  for (int r = 0; r < BM; ++r)
#pragma unroll
    for (int q = 0; q < BN; ++q) acc[r][q] = v4f32{0.f, 0.f, 0.f, 0.f};
  for (int sg = 0; sg < J.nseg; ++sg) {
    const GSeg& S = segs[J.seg0 + sg];
    const int K = S.K;
    const int lda = S.A.ld, ldb = S.B.ld, ta = S.A.trans, tb = S.B.trans;
    const float sscale = (float)S.scale;
    const float* Ap = optr<float>(S.A, m, c);
    const float* Bp = optr<float>(S.B, m, c);
    for (int k0 = 0; k0 < K; k0 += TK) {
      for (int e = tid; e < TM * TK; e += NT) {
        int i, kk;
        if (!ta) { i = e % TM; kk = e / TM; } else { kk = e % TK; i = e / TK; }
        const int gi = i0 + i, gk = k0 + kk;
        float v = 0.f;
        if (gi < M && gk < K) v = ta ? Ap[gk + (long long)gi * lda] : Ap[gi + (long long)gk * lda];
        As[kk][i] = v * sscale;
      }
      for (int e = tid; e < TK * TN; e += NT) {
        int kk, jj;
        if (!tb) { kk = e % TK; jj = e / TK; } else { jj = e % TN; kk = e / TN; }
        const int gk = k0 + kk, gj = j0 + jj;
        float v = 0.f;
        if (gk < K && gj < N) v = tb ? Bp[gj + (long long)gk * ldb] : Bp[gk + (long long)gj * ldb];
        Bs[kk][jj] = v;
      }
      __syncthreads();
#pragma unroll
      for (int kq = 0; kq < TK; kq += 4) {
        float a[BM], b[BN];
#pragma unroll
        for (int r = 0; r < BM; ++r) a[r] = As[kq + lk][(wm * BM + r) * 16 + lr];
#pragma unroll
        for (int q = 0; q < BN; ++q) b[q] = Bs[kq + lk][(wn * BN + q) * 16 + lr];
#pragma unroll
        for (int r = 0; r < BM; ++r)
#pragma unroll
          for (int q = 0; q < BN; ++q) acc[r][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r], b[q], acc[r][q], 0, 0, 0);
      }
      __syncthreads();
    }
  }
  float* Cp = const_cast<float*>(optr<float>(J.C, m, c));
  const int ldc = J.C.ld;
  const float alpha = (float)J.alpha, beta = (float)J.beta;
#pragma unroll
  for (int q = 0; q < BN; ++q) {
    const int gj = j0 + (wn * BN + q) * 16 + lr;
    if (gj >= N) continue;
#pragma unroll
    for (int r = 0; r < BM; ++r)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int gi = i0 + (wm * BM + r) * 16 + 4 * lk + u;
        if (gi >= M) continue;
        float* cp = Cp + gi + (long long)gj * ldc;
        float v = alpha * acc[r][q][u];
        if (beta != 0.f) v = fmaf(beta, *cp, v);
        *cp = v;
      }
  }
}

template <int TM, int TN, int WM, int WN, int TK>
__global__ __launch_bounds__(WM * WN * WAVE) void k_ggemm_mfma(const GJob* __restrict__ jobs, int njobs,
                                                              const GSeg* __restrict__ segs) {
  ggemm_mfma_body<TM, TN, WM, WN, TK>(jobs, njobs, segs, blockIdx.x);
}

// Reduction GEMM C = sum_s scale_s A_s^T B_s with long K (A_s: K x M, B_s:
// K x N, both column-major).  A workgroup owns an 8 x 8 output tile; its four
// waves split K (wave w takes k = 64 w + lane, step 256), every lane keeps the
// 64 partial sums of the tile (coalesced loads, each element read once), a
// butterfly transpose-reduction leaves lane l with output l of its wave, and
// the four waves are summed through LDS.
template <typename T>
__device__ __forceinline__ void gemm_dot_body(const GJob* __restrict__ jobs, int njobs,
                                                 const GSeg* __restrict__ segs, long long bid) {
  __shared__ T red[4][64];
  
  const GJob& J = jobs[job_of(jobs, njobs, bid)];
  const int tilesM = J.tilesM;
  const int tiles = tilesM * J.tilesN;
  const long long local = bid - J.block0;
  const int prob = (int)(local / tiles);
  const int t = (int)(local % tiles);
  const int tm = t % tilesM, tn = t / tilesM;
  const int m = prob / J.ncl, c = prob % J.ncl;
  const int M = J.M, N = J.N;
  const int lane = threadIdx.x % WAVE;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const int i0 = tm * 8, j0 = tn * 8;
  T acc[64];
#pragma unroll
  for (int q = 0; q < 64; ++q) acc[q] = T(0);
  for (int sg = 0; sg < J.nseg; ++sg) {
    const GSeg& S = segs[J.seg0 + sg];
    const int K = S.K, lda = S.A.ld, ldb = S.B.ld;
    const T sc = (T)S.scale;
    const T* Ap = optr<T>(S.A, m, c);
    const T* Bp = optr<T>(S.B, m, c);
    for (int k = wv * WAVE + lane; k < K; k += 4 * WAVE) {
      T a[8], bv[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) a[r] = (i0 + r < M) ? Ap[k + (long long)(i0 + r) * lda] * sc : T(0);
#pragma unroll
      for (int q = 0; q < 8; ++q) bv[q] = (j0 + q < N) ? Bp[k + (long long)(j0 + q) * ldb] : T(0);
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[r * 8 + q] = fma(a[r], bv[q], acc[r * 8 + q]);
    }
  }
  // butterfly transpose-reduction: after step h (partner lane ^ (32 >> h)) a
  // lane keeps the half of its values selected by that lane bit; at the end
  // lane l holds the wave's sum for output l
#pragma unroll
  for (int h = 0; h < 6; ++h) {
    const int half = 32 >> h;
    const bool hi = (lane & half) != 0;
#pragma unroll
    for (int q = 0; q < half; ++q) {
      const T send = hi ? acc[q] : acc[q + half];
      const T keep = hi ? acc[q + half] : acc[q];
      acc[q] = keep + __shfl_xor(send, half, WAVE);
    }
  }
  red[wv][lane] = acc[0];
  __syncthreads();
  if (wv == 0) {
    const T v0 = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
    const int gi = i0 + lane / 8, gj = j0 + lane % 8;
    if (gi < M && gj < N) {
      T* cp = const_cast<T*>(optr<T>(J.C, m, c)) + gi + (long long)gj * J.C.ld;
      T v = (T)J.alpha * v0;
      if (J.beta != 0.0) v = fma((T)J.beta, *cp, v);
      *cp = v;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_gemm_dot(const GJob* __restrict__ jobs, int njobs,
    const GSeg* __restrict__ segs) {
  gemm_dot_body<T>(jobs, njobs, segs, blockIdx.x);
}

// Short-K reduction GEMM C = sum_s scale_s A_s^T B_s with outputs up to
// 16 x 16 per workgroup: 64-deep K slices of A^T and B are staged through LDS
// with loads coalesced along K, then thread t accumulates output
// (t % 16, t / 16) of the tile.
template <typename T>
__device__ __forceinline__ void gemm_small_body(const GJob* __restrict__ jobs, int njobs,
                                                   const GSeg* __restrict__ segs, long long bid) {
  constexpr int KS = 64;
  __shared__ T As[KS][17];
  __shared__ T Bs[KS][17];
  
  const GJob& J = jobs[job_of(jobs, njobs, bid)];
  const int tilesM = J.tilesM;
  const int tiles = tilesM * J.tilesN;
  const long long local = bid - J.block0;
  const int prob = (int)(local / tiles);
  const int t = (int)(local % tiles);
  const int tm = t % tilesM, tn = t / tilesM;
  const int m = prob / J.ncl, c = prob % J.ncl;
  const int M = J.M, N = J.N;
  const int tid = threadIdx.x;
  const int i0 = tm * 16, j0 = tn * 16;
  const int oi = tid % 16, oj = tid / 16;
  T acc = T(0);
  for (int sg = 0; sg < J.nseg; ++sg) {
    const GSeg& S = segs[J.seg0 + sg];
    const int K = S.K, lda = S.A.ld, ldb = S.B.ld;
    const T sc = (T)S.scale;
    const T* Ap = optr<T>(S.A, m, c);
    const T* Bp = optr<T>(S.B, m, c);
    for (int k0 = 0; k0 < K; k0 += KS) {
      for (int e = tid; e < KS * 16; e += 256) {
        const int kk = e % KS, q = e / KS;
        const int k = k0 + kk;
        As[kk][q] = (k < K && i0 + q < M) ? Ap[k + (long long)(i0 + q) * lda] * sc : T(0);
        Bs[kk][q] = (k < K && j0 + q < N) ? Bp[k + (long long)(j0 + q) * ldb] : T(0);
      }
      __syncthreads();
#pragma unroll 16
      for (int kk = 0; kk < KS; ++kk) acc = fma(As[kk][oi], Bs[kk][oj], acc);
      __syncthreads();
    }
  }
  const int gi = i0 + oi, gj = j0 + oj;
  if (gi < M && gj < N) {
    T* cp = const_cast<T*>(optr<T>(J.C, m, c)) + gi + (long long)gj * J.C.ld;
    T v = (T)J.alpha * acc;
    if (J.beta != 0.0) v = fma((T)J.beta, *cp, v);
    *cp = v;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_gemm_small(const GJob* __restrict__ jobs, int njobs,
    const GSeg* __restrict__ segs) {
  gemm_small_body<T>(jobs, njobs, segs, blockIdx.x);
}

// Row GEMM C = sum_s scale_s op(A_s) B_s for tall outputs with few columns
// (N <= NMAX): every wave owns one tile of 64 output rows (one per lane) and
// the whole K range, so the waves of a workgroup (four consecutive tiles of
// the job) never wait for each other.  Per chunk of 32 columns of A a lane
// issues its 32 loads at once; the matching rows of B are staged, scaled, in
// the wave's own slice of LDS and read back as broadcasts.
template <typename T, int NMAX>
__device__ __forceinline__ void gemm_rows_body(const GJob* __restrict__ jobs, int njobs,
                                                  const GSeg* __restrict__ segs, long long bid) {
  constexpr int KC = 32;
  __shared__ T bsh[4][KC * NMAX];
  const GJob& J = jobs[job_of(jobs, njobs, bid)];
  const int lane = threadIdx.x % WAVE;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const long long tile = (bid - J.block0) * 4 + wv;
  if (tile >= (long long)J.nmat * J.ncl * J.tilesM) return;   // no barriers below
  const int prob = (int)(tile / J.tilesM), tm = (int)(tile % J.tilesM);
  const int m = prob / J.ncl, c = prob % J.ncl;
  const int M = J.M, N = J.N;
  const int i = tm * 64 + lane;
  const bool live = i < M;
  T* const bw = bsh[wv];
  T acc[NMAX];
#pragma unroll
  for (int q = 0; q < NMAX; ++q) acc[q] = T(0);
  for (int sg = 0; sg < J.nseg; ++sg) {
    const GSeg& S = segs[J.seg0 + sg];
    const T* Ap = optr<T>(S.A, m, c);
    const T* Bp = optr<T>(S.B, m, c);
    const long long lda = S.A.ld, ldb = S.B.ld;
    const bool ta = S.A.trans;
    const T sc = (T)S.scale;
    const int K = S.K;
    const T* arow = ta ? Ap + (long long)i * lda : Ap + i;   // A(i, k) = arow[k * astep]
    const long long astep = ta ? 1 : lda;
    for (int k0 = 0; k0 < K; k0 += KC) {
      const int kn = min(KC, K - k0);
      T a[KC];
#pragma unroll
      for (int u = 0; u < KC; ++u) a[u] = (live && u < kn) ? arow[(long long)(k0 + u) * astep] : T(0);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");   // earlier reads of bw are done
      for (int e = lane; e < KC * NMAX; e += WAVE) {
        const int kk = e / NMAX, q = e % NMAX;
        bw[e] = (kk < kn && q < N) ? sc * Bp[(k0 + kk) + (long long)q * ldb] : T(0);
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");   // bw visible to every lane
#pragma unroll
      for (int u = 0; u < KC; ++u) {
        if (u < kn) {
          const T* br = bw + u * NMAX;
#pragma unroll
          for (int q = 0; q < NMAX; ++q) acc[q] = fma(a[u], br[q], acc[q]);
        }
      }
    }
  }
  if (!live) return;
  T* Cp = const_cast<T*>(optr<T>(J.C, m, c));
  const long long ldc = J.C.ld;
  const T alpha = (T)J.alpha, beta = (T)J.beta;
#pragma unroll
  for (int q = 0; q < NMAX; ++q) {
    if (q >= N) break;
    T* cp = Cp + i + (long long)q * ldc;
    T v = alpha * acc[q];
    if (beta != T(0)) v = fma(beta, *cp, v);
    *cp = v;
  }
}

template <typename T, int NMAX>
__global__ __launch_bounds__(256) void k_gemm_rows(const GJob* __restrict__ jobs, int njobs,
    const GSeg* __restrict__ segs) {
  gemm_rows_body<T, NMAX>(jobs, njobs, segs, blockIdx.x);
}

// Every GEMM kind in one launch (the job's kind selects the body; the narrow
// tile shapes run as 64 x 64 tiles): used when a grouped GEMM is too small to
// fill the GPU, where one launch per kind would only add their latencies.
template <typename T>
__global__ __launch_bounds__(256) void k_gemm_any(const GJob* __restrict__ jobs, int njobs,
                                                 const GSeg* __restrict__ segs) {
  const long long bid = blockIdx.x;
  switch (jobs[job_of(jobs, njobs, bid)].kind) {
    case 5: gemm_dot_body<T>(jobs, njobs, segs, bid); break;
    case 6: gemm_rows_body<T, 16>(jobs, njobs, segs, bid); break;
    case 7: gemm_rows_body<T, sizeof(T) == 4 ? 32 : 16>(jobs, njobs, segs, bid); break;
    case 8: gemm_rows_body<T, 4>(jobs, njobs, segs, bid); break;
    case 9: gemm_small_body<T>(jobs, njobs, segs, bid); break;
    case 10:
      if constexpr (sizeof(T) == 4) ggemm_mfma_body<64, 64, 2, 2, 16>(jobs, njobs, segs, bid);
      break;
    default: ggemm_body<T, 64, 64, 16, 4, 4>(jobs, njobs, segs, bid); break;
  }
}

// ------------------------------------------------------------ HODLR matvec
// out = beta * C0 + sum_t alpha_t op_t y_t for a batch of blocks, in two
// steps.  The projection step computes, for every HODLR term, matrix, depth d
// and node tau of that depth, the projections V_d[tau]^T y[tau] (one wave per
// node and chunk of up to 16 columns, written to a small buffer).  The row
// step then gives every output row to one thread: the row of the leaf times y
// on the leaf's rows, plus U_d[row] times the projection of the sibling of the
// row's depth-d ancestor, for every depth; no barriers, the leaf and U loads
// are independent and coalesced over the rows of a wave.  Both steps run as
// grouped launches (k_hmv_reduce, k_hmv_apply) or as tasks of the persistent
// solve pass (k_psolve); the arithmetic is the same device code in both.
//
// Operand addresses y, C0 and out are taken relative to `ws` (ws = 0: they
// are device addresses); factor addresses are device addresses.
template <typename T>
__device__ __forceinline__ T* wsp(const void* p, const char* ws) {
  return gmem(reinterpret_cast<T*>(reinterpret_cast<uintptr_t>(ws) + reinterpret_cast<uintptr_t>(p)));
}

// Projection unit `rem` (depth, node, 16-column chunk) of matrix m of term M,
// by one whole wave.
template <typename T, int NR>
__device__ __forceinline__ void hmv_reduce_unit(const MVTerm& M, int m, int rem, const char* ws,
                                                T* __restrict__ tbuf, int lane) {
  constexpr int CH = 16;                               // columns per unit
  constexpr int RB = NR <= 1 ? 4 : NR <= 2 ? 2 : 1;    // rows per lane per batch
  const int s = M.s, nrhs = M.nrhs;
  int d = 1;
  for (;; ++d) {
    const int units = (1 << d) * ((M.kc[d] + CH - 1) / CH);
    if (rem < units) break;
    rem -= units;
  }
  const int w = M.kc[d], nch = (w + CH - 1) / CH;
  const int node = rem / nch, q0 = (rem % nch) * CH;
  const int sd = s >> d;
  const long long vs = (long long)s * nrhs;
  const T* Vb = gmem(static_cast<const T*>(M.V[d])) + (long long)(M.mmul * m + M.moff) * M.k[d] * s +
                (long long)q0 * s + (long long)node * sd;
  const T* yb = wsp<const T>(M.y, ws) + (long long)(M.ymul * m + M.yoff) * vs + (long long)node * sd;
  T pr[CH][NR];
#pragma unroll
  for (int c = 0; c < CH; ++c)
#pragma unroll
    for (int q = 0; q < NR; ++q) pr[c][q] = T(0);
  for (int i0 = 0; i0 < sd; i0 += WAVE * RB) {
    T vv[RB][CH], yv[RB][NR];
#pragma unroll
    for (int e = 0; e < RB; ++e) {
      const int i = i0 + e * WAVE + lane;
      const bool ok = i < sd;
#pragma unroll
      for (int q = 0; q < NR; ++q) yv[e][q] = (ok && q < nrhs) ? yb[i + (long long)q * s] : T(0);
#pragma unroll
      for (int c = 0; c < CH; ++c) vv[e][c] = (ok && q0 + c < w) ? Vb[i + (long long)c * s] : T(0);
    }
#pragma unroll
    for (int e = 0; e < RB; ++e)
#pragma unroll
      for (int c = 0; c < CH; ++c)
#pragma unroll
        for (int q = 0; q < NR; ++q) pr[c][q] = fma(vv[e][c], yv[e][q], pr[c][q]);
  }
  // value v = c * NR + q (column q0 + c, right-hand side q) is stored by lane
  // v mod 64
  constexpr int NV = (CH * NR + WAVE - 1) / WAVE;
  T mine[NV];
#pragma unroll
  for (int h = 0; h < NV; ++h) mine[h] = T(0);
#pragma unroll
  for (int c = 0; c < CH; ++c)
    if (q0 + c < w)
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        const T tot = wave_sum(pr[c][q]);
        if (lane == (c * NR + q) % WAVE) mine[(c * NR + q) / WAVE] = tot;
      }
  T* const to = tbuf + M.tbase + (long long)m * M.tstride + M.toff[d] + (long long)(node * w + q0) * NR;
#pragma unroll
  for (int h = 0; h < NV; ++h) {
    const int v = h * WAVE + lane;
    if (v < CH * NR && q0 + v / NR < w) to[v] = mine[h];
  }
}

// Output row `row` of matrix m of job J, by one thread.  W64: every wave lies
// inside one leaf column block (b and s multiples of 64, rows in whole waves),
// so the wave loads y on 64 leaf columns at once and broadcasts each value
// with a lane read.
template <typename T, int NR, bool W64>
__device__ __forceinline__ void hmv_apply_row(const MVJob& J, const MVTerm* __restrict__ terms, int m, int row,
                                              int lane, const char* ws, const T* __restrict__ tbuf) {
  const int s = J.s, b = J.b, L = J.L, nrhs = J.nrhs;
  const int l = row / b, r = row % b, nleaf = 1 << L;
  const long long vs = (long long)s * nrhs;
  T acc[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) acc[q] = T(0);
  if (J.C0) {
    const T* c0 = wsp<const T>(J.C0, ws) + (long long)(J.cmul * m + J.coff) * vs + row;
#pragma unroll
    for (int q = 0; q < NR; ++q)
      if (q < nrhs) acc[q] = (T)J.beta * c0[(long long)q * s];
  }
  for (int t = 0; t < J.nterm; ++t) {
    const MVTerm& M = terms[J.term0 + t];
    const int mm = M.mmul * m + M.moff;
    const T* y = wsp<const T>(M.y, ws) + (long long)(M.ymul * m + M.yoff) * vs;
    T ta[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) ta[q] = T(0);
    if (M.type == 1) {   // diagonal
      const T dv = gmem(static_cast<const T*>(M.lv))[(long long)mm * s + row];
#pragma unroll
      for (int q = 0; q < NR; ++q)
        if (q < nrhs) ta[q] = dv * y[row + (long long)q * s];
    } else {
      const T* lf = gmem(static_cast<const T*>(M.lv)) + ((long long)mm * nleaf + l) * b * b + r;
      const T* yl = y + (long long)l * b;
      if (W64) {
        // all loads of a slice of leaf columns are issued before its products
        // (64 columns in FP32, 32 in FP64); the products keep column order
        constexpr int SL = sizeof(T) == 4 ? WAVE : WAVE / 2;
        for (int cb = 0; cb < b; cb += WAVE) {
          T yw[NR];
#pragma unroll
          for (int q = 0; q < NR; ++q) yw[q] = q < nrhs ? yl[cb + lane + (long long)q * s] : T(0);
#pragma unroll
          for (int c0 = 0; c0 < WAVE; c0 += SL) {
            T av[SL];
#pragma unroll
            for (int c = 0; c < SL; ++c) av[c] = lf[(long long)(cb + c0 + c) * b];
#pragma unroll
            for (int c = 0; c < SL; ++c)
#pragma unroll
              for (int q = 0; q < NR; ++q) ta[q] = fma(av[c], lane_read(yw[q], c0 + c), ta[q]);
          }
        }
      } else {
#pragma unroll 8
        for (int c = 0; c < b; ++c) {
          const T a = lf[(long long)c * b];
#pragma unroll
          for (int q = 0; q < NR; ++q)
            if (q < nrhs) ta[q] = fma(a, yl[c + (long long)q * s], ta[q]);
        }
      }
      const T* tb = tbuf + M.tbase + (long long)m * M.tstride;
      for (int d = 1; d <= L; ++d) {
        const int w = M.kc[d];
        if (w == 0) continue;
        const int sib = (l >> (L - d)) ^ 1;
        const T* tv = tb + M.toff[d] + (long long)sib * w * NR;
        const T* Ud = gmem(static_cast<const T*>(M.U[d])) + (long long)mm * M.k[d] * s + row;
        // eight U columns loaded at once, products in column order
        for (int q0 = 0; q0 < w; q0 += 8) {
          T uv[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) uv[e] = q0 + e < w ? Ud[(long long)(q0 + e) * s] : T(0);
#pragma unroll
          for (int e = 0; e < 8; ++e)
            if (q0 + e < w)
#pragma unroll
              for (int q = 0; q < NR; ++q) ta[q] = fma(uv[e], tv[(q0 + e) * NR + q], ta[q]);
        }
      }
    }
    const T al = (T)M.alpha;
#pragma unroll
    for (int q = 0; q < NR; ++q) acc[q] = fma(al, ta[q], acc[q]);
  }
  T* out = wsp<T>(J.out, ws) + (long long)(J.omul * m + J.ooff) * vs + row;
#pragma unroll
  for (int q = 0; q < NR; ++q)
    if (q < nrhs) out[(long long)q * s] = acc[q];
}

template <typename T, int NR>
__global__ __launch_bounds__(256) void k_hmv_reduce(const MVRed* __restrict__ reds, int nred,
                                                    const MVTerm* __restrict__ terms, long long nunits,
                                                    T* __restrict__ tbuf) {
  const long long u = (long long)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  if (u >= nunits) return;   // uniform over the wave; no barriers below
  const MVRed& R = reds[job_of(reds, nred, u)];
  const long long local = u - R.block0;
  hmv_reduce_unit<T, NR>(terms[R.term], (int)(local / R.upm), (int)(local % R.upm), nullptr, tbuf,
                         threadIdx.x % WAVE);
}

// One thread per output row (rows of all jobs' blocks numbered in order, a
// job's rows from block0).
template <typename T, int NR, bool W64>
__global__ __launch_bounds__(64) void k_hmv_apply(const MVJob* __restrict__ jobs, int njobs,
                                                  const MVTerm* __restrict__ terms, long long nrows,
                                                  const T* __restrict__ tbuf) {
  const long long g = (long long)blockIdx.x * WAVE + threadIdx.x;
  if (g >= nrows) return;   // never with W64: the rows fill whole waves
  const MVJob& J = jobs[job_of(jobs, njobs, g)];
  const long long local = g - J.block0;
  hmv_apply_row<T, NR, W64>(J, terms, (int)(local / J.s), (int)(local % J.s), threadIdx.x, nullptr, tbuf);
}

// ------------------------------------------------- persistent solve pass
// One launch runs the whole task list of one or more solve passes (see
// PTask).  Workgroups take tickets in order from one counter; ticket t is
// task t - task0 of the instance holding it.  Thread 0 waits until every
// counter the task depends on has reached its total (polling with a sleep,
// at most `limit` polls per counter), then the workgroup runs the task and
// adds one to the task's own counter.
//   * Visibility: after the workgroup barrier that follows the task, thread
//     0 increments with release order at device scope; the waiting thread
//     fences with acquire order at device scope before the barrier that
//     releases its workgroup to read the inputs.  Each such release and
//     acquire writes back or invalidates the non-coherent cache lines of the
//     chip's L2 slices, which is why only the levels with few blocks (few
//     tasks) run this way.
//   * Termination: tasks are listed so that each one follows every task it
//     waits for, and a workgroup holds one task at a time, so the earliest
//     unfinished task that has been taken has all its inputs done.  A wait
//     that runs out of polls (or finds the abort word set) gives up: the
//     workgroup sets the abort word, and every later wait of the launch gives
//     up at once, so every workgroup reaches the end of the ticket range.
//     Tasks that gave up leave their outputs unwritten; the pass then writes
//     NaN to its whole solution (k_pcheck).
constexpr int kPRows = 256;   // output rows per row task (4 waves)
constexpr int kPUnits = 8;    // projection units per projection task

__device__ __forceinline__ int pinst_of(const PInst* insts, int n, long long t) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (insts[mid].task0 <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename T, int NR, bool W64>
__global__ __launch_bounds__(256) void k_psolve(const PInst* __restrict__ insts, int ninst, long long ntask,
                                                int* __restrict__ ticket, int* __restrict__ abort_word,
                                                long long limit) {
  __shared__ long long s_t;
  __shared__ int s_go;
  const int tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
  for (;;) {
    if (tid == 0) s_t = __hip_atomic_fetch_add(ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const long long t = s_t;
    if (t >= ntask) break;   // uniform over the workgroup
    const PInst& I = insts[pinst_of(insts, ninst, t)];
    const PTask& K = I.tasks[t - I.task0];
    if (tid == 0) {
      int go = 1;
      if (limit < 0 && K.ndep > 0) {   // forced give-up (tests of the failure path)
        __hip_atomic_store(abort_word, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        go = 0;
      }
      for (int e = 0; e < K.ndep && go; ++e) {
        const int* c = I.ctr + K.dep[e];
        long long polls = 0;
        while (__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < K.need[e]) {
          if (__hip_atomic_load(abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || ++polls > limit) {
            __hip_atomic_store(abort_word, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            go = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // inputs written by finished tasks are visible
      s_go = go;
    }
    __syncthreads();
    if (s_go) {
      const char* ws = I.ws;
      T* tbuf = reinterpret_cast<T*>(I.ws + I.tbuf_off);
      if (K.kind == 0) {
        const MVTerm& M = I.terms[K.idx];
        for (int u = K.u0 + wv; u < K.u1; u += 4) hmv_reduce_unit<T, NR>(M, K.m, u, ws, tbuf, lane);
      } else {
        const MVJob& J = I.jobs[K.idx];
        const int row = K.u0 + tid;
        // W64: u1 - u0 is a multiple of 64, so whole waves take part or none
        if (row < K.u1) hmv_apply_row<T, NR, W64>(J, I.terms, K.m, row, lane, ws, tbuf);
      }
    }
    __syncthreads();   // the workgroup's stores are done before thread 0 releases them
    if (tid == 0 && s_go) __hip_atomic_fetch_add(I.ctr + K.done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// After a persistent pass: if a wait gave up, the final unknowns of every
// instance (the sources of the block-to-vector copy that follows) are set to
// NaN, since some task outputs were never written.
template <typename T>
__global__ __launch_bounds__(256) void k_pcheck(const VJob* __restrict__ jobs, int njobs,
                                                const int* __restrict__ abort_word) {
  if (__hip_atomic_load(abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) return;
  const VJob& J = jobs[job_of(jobs, njobs, blockIdx.x)];
  const long long part = blockIdx.x - J.block0;
  const long long n = (long long)J.s * J.nblk * J.nrhs;
  T* V = gmem(static_cast<T*>(const_cast<void*>(J.src)));
  for (long long e = part * 256 + threadIdx.x; e < n; e += (long long)J.per * 256) V[e] = T(NAN);
}

// ---------------------------------------------------------------- inverse
// Small inverses (n <= N <= 64): Gauss-Jordan with partial pivoting in FP64,
// one row per lane.  A wave holds 64/N matrices (lane group g, row r = lane
// mod N) with the working row in registers.  Rows are neither swapped nor
// normalised during the elimination: at step j the pivot row p_j (largest
// |entry| in column j among the rows not yet used) is published in LDS, every
// other row subtracts its multiple of it, and the in-place storage turns
// column j into column p_j of the accumulated transformation M (M A = D P,
// D the pivots).  At the end each row is divided by its pivot and the inverse
// is read back as X[j, p_j'] = W[p_j, j'] / d_(p_j).  The current column is
// kept at a compile-time register position by rotating the row by 8 columns
// after every 8 steps.
// Entry (r, c) of matrix p of an inverse job: from A, or in capacitance
// mode formed from the two cores of the pair p.
template <typename Tin>
__device__ __forceinline__ double inv_entry(const IJob& J, long long p, int r, int c) {
  if (J.cap_k > 0) {
    const int k = J.cap_k;
    if ((r < k) == (c < k)) return r == c ? 1.0 : 0.0;
    const Tin* cores = gmem(static_cast<const Tin*>(J.cores));
    if (r < k) return (double)cores[(size_t)(2 * p + 1) * k * k + r + (size_t)(c - k) * k];   // c_(2p+1)
    return (double)cores[(size_t)(2 * p) * k * k + (r - k) + (size_t)c * k];                  // c_(2p)
  }
  return (double)gmem(static_cast<const Tin*>(J.A))[p * J.sA + r + (long long)c * J.n];
}

template <typename Tin, typename Tout, int N>
__global__ __launch_bounds__(256) void k_inverse_wave(const IJob* __restrict__ jobs, int njobs) {
  constexpr int G = WAVE / N;
  constexpr int JB = N < 8 ? N : 8;
  __shared__ int piv_row[4][WAVE];
  __shared__ double prow[4][WAVE];
  const IJob& Jb = jobs[job_of(jobs, njobs, blockIdx.x)];
  const int n = Jb.n, nprob = Jb.nprob;
  const Tin* __restrict__ A = gmem(static_cast<const Tin*>(Jb.A));
  Tout* __restrict__ X = gmem(static_cast<Tout*>(Jb.X));
  const long long sA = Jb.sA, sX = Jb.sX;
  int* const status = gmem(Jb.status);
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
  const int g = lane / N, r = lane % N;
  const long long p = ((long long)(blockIdx.x - Jb.block0) * 4 + wv) * G + g;
  const bool valid = p < nprob;
  (void)A;
  (void)sA;
  double a[N];
#pragma unroll
  for (int c = 0; c < N; ++c)
    a[c] = (valid && r < n && c < n) ? inv_entry<Tin>(Jb, p, r, c) : (r == c ? 1.0 : 0.0);
  bool used = false, bad = false;
  int mystep = r;
  double mypiv = 1.0;
  double* pr = &prow[wv][g * N];
  for (int jb = 0; jb < n; jb += JB) {
#pragma unroll
    for (int jj = 0; jj < JB; ++jj) {
      const int j = jb + jj;
      if (j < n) {
        const double f = a[jj];
        // pivot: largest |f| over the unused rows, ties to the lowest row; the
        // key is |f|'s bit pattern (monotone for non-negative doubles) with its
        // 6 lowest bits replaced by 63 - row
        const unsigned long long key =
            used ? 0ull : ((__double_as_longlong(fabs(f)) & ~63ull) | (unsigned long long)(63 - r));
        const unsigned long long kmax = group_max_u64<N>(key);
        const int bi = 63 - (int)(kmax & 63ull);
        const double best = __longlong_as_double((long long)(kmax & ~63ull));
        if (!(best > 0.0) || !isfinite(best)) bad = true;
        const bool is_piv = r == bi;
        if (is_piv) {
          used = true;
          mystep = j;
          mypiv = f;
          if constexpr (N != WAVE) {
#pragma unroll
            for (int c = 0; c < N; ++c) pr[c] = a[c];
          }
        }
        if constexpr (N == WAVE) {
          // one matrix per wave: every lane reads the pivot row from the pivot
          // lane's registers (bi is uniform), outside any branch, before any
          // lane updates its row
          const double pv = lane_read(a[jj], bi);
          const double qq = is_piv ? 0.0 : f / pv;
#pragma unroll
          for (int c = 0; c < N; ++c) a[c] = fma(-qq, lane_read(a[c], bi), a[c]);
          a[jj] = is_piv ? 1.0 : -qq;
        } else {
          // the other lanes of the group read what the pivot lane wrote: a
          // wavefront-scope fence orders the accesses (LDS is in order per wave)
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          const double qq = is_piv ? 0.0 : f / pr[jj];
#pragma unroll
          for (int c = 0; c < N; ++c) a[c] = fma(-qq, pr[c], a[c]);
          a[jj] = is_piv ? 1.0 : -qq;
        }
        if (r == 0) piv_row[wv][g * N + j] = bi;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      }
    }
    double t[JB];
#pragma unroll
    for (int c = 0; c < JB; ++c) t[c] = a[c];
#pragma unroll
    for (int c = 0; c < N - JB; ++c) a[c] = a[c + JB];
#pragma unroll
    for (int c = 0; c < JB; ++c) a[N - JB + c] = t[c];
  }
  __syncthreads();
  if (valid && r < n) {
    const double inv = 1.0 / mypiv;
    const int R = ((n + JB - 1) / JB) * JB;   // total rotation: register c holds column (c + R) mod N
    Tout* Xp = X + p * sX;
#pragma unroll
    for (int c = 0; c < N; ++c) {
      const int L = (c + R) % N;
      if (L < n) {
        const int pc = piv_row[wv][g * N + L];   // < n unless the matrix is singular (then flagged)
        if (pc < n) Xp[mystep + (long long)pc * n] = (Tout)(a[c] * inv);
      }
    }
    if (r == 0 && bad) status[0] = 1;
  }
}

// Gauss-Jordan on the augmented matrix [A | I] (row-major n x 2n) in FP64.
template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void k_inverse(const IJob* __restrict__ jobs, int njobs) {
  extern __shared__ double smem[];
  const IJob& Jb = jobs[job_of(jobs, njobs, blockIdx.x)];
  const int n = Jb.n;
  const Tin* A = gmem(static_cast<const Tin*>(Jb.A));
  Tout* X = gmem(static_cast<Tout*>(Jb.X));
  const long long sA = Jb.sA, sX = Jb.sX;
  double* ws = gmem(Jb.ws);
  const int use_lds = Jb.use_lds;
  int* const status = gmem(Jb.status);
  const int p = (int)(blockIdx.x - Jb.block0);
  const int n2 = 2 * n;
  __shared__ double colj_s[128];
  double* W = use_lds ? smem : ws + (size_t)p * n * n2;
  double* colj = n <= 128 ? colj_s : ws + (size_t)Jb.nprob * n * n2 + (size_t)p * n;
  __shared__ int piv;
  __shared__ double pval;
  __shared__ int bad;
  (void)A;
  (void)sA;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  for (int e = tid; e < n * n2; e += blockDim.x) {
    const int r = e / n2, c = e % n2;
    W[e] = c < n ? inv_entry<Tin>(Jb, p, r, c) : (c - n == r ? 1.0 : 0.0);
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
      wave_argmax(best, bi);
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
__global__ __launch_bounds__(256) void k_inverse_lds(const IJob* __restrict__ jobs, int njobs) {
  extern __shared__ double W[];
  __shared__ int perm[128];
  __shared__ double colj[128];
  __shared__ int piv;
  __shared__ double pinv;
  __shared__ int bad;
  const IJob& Jb = jobs[job_of(jobs, njobs, blockIdx.x)];
  const int n = Jb.n;
  const Tin* A = gmem(static_cast<const Tin*>(Jb.A));
  Tout* X = gmem(static_cast<Tout*>(Jb.X));
  const long long sA = Jb.sA, sX = Jb.sX;
  int* const status = gmem(Jb.status);
  const int p = (int)(blockIdx.x - Jb.block0), tid = threadIdx.x;
  (void)A;
  (void)sA;
  if (tid == 0) bad = 0;
  for (int e = tid; e < n * n; e += 256) {
    const int r = e % n, c = e / n;
    W[r * n + c] = inv_entry<Tin>(Jb, p, r, c);
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
      wave_argmax(best, bi);
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

// ------------------------------------ rank-revealing SVD, core in registers
// Same computation and outputs as k_grsvd for cores of size c <= 64 whose
// numerical rank (the number of pivoted Householder steps before the stop
// test) is at most SV_TP: the column-pivoted QR runs with the core in
// registers (wave w owns the physical columns q = w + 4u, lane = row; no
// column swaps: the pivot column is processed in place and R is recorded by
// physical column), then one wave runs the one-sided Jacobi iteration on
// X = R_top^T with X and J in registers (cyclic pair order) and forms
// U_K = Q_K [J; 0].  A problem whose rank exceeds SV_TP is flagged in redo[]
// and left to k_grsvd.
constexpr int SV_TP = 16;
template <typename T>
__global__ __launch_bounds__(256) void k_grsvd_reg(const SJob* __restrict__ jobs, int njobs) {
  constexpr int SL = 16;   // column slots per wave (c <= 64)
  __shared__ T Rt[64][65];
  __shared__ T Vk[64][64];
  __shared__ T tk[64];
  __shared__ double cval[2][4];
  __shared__ int cidx[2][4];
  __shared__ double cfro[4];
  const SJob& Jb = jobs[job_of(jobs, njobs, blockIdx.x)];
  const int prob = (int)(blockIdx.x - Jb.block0);
  const int c = Jb.c, maxrank = Jb.maxrank;
  const double eps = Jb.eps;
  const T* Kp = gmem(static_cast<const T*>(Jb.K)) + (size_t)prob * c * c;
  const int tid = threadIdx.x, lane = tid % WAVE;
  const int wv = __builtin_amdgcn_readfirstlane(tid / WAVE);
  T w[SL];
  bool used[SL];
#pragma unroll
  for (int u = 0; u < SL; ++u) {
    const int q = wv + 4 * u;
    w[u] = (lane < c && q < c) ? Kp[lane + (size_t)q * c] : T(0);
    used[u] = false;
  }
  double delta2 = 0.0, fl = 0.0;
  int tp = 0;
  for (int j = 0; j < c; ++j) {
    const int cb = j & 1;
    // this wave's best unused column: squared norm of rows >= j
    double best = -1.0, fro = 0.0;
    int bq = 0x7fffffff;
#pragma unroll
    for (int u = 0; u < SL; ++u) {
      const int q = wv + 4 * u;
      if (q < c && !used[u]) {
        const double xv = (double)w[u];
        const double nn = wave_sum((lane >= j && lane < c) ? xv * xv : 0.0);
        fro += nn;
        if (nn > best) { best = nn; bq = q; }
      }
    }
    if (lane == 0) {
      cval[cb][wv] = best;
      cidx[cb][wv] = bq;
      if (j == 0) cfro[wv] = fro;
    }
    __syncthreads();
    double gb = -1.0;
    int pc = 0x7fffffff;
    for (int o = 0; o < 4; ++o) {
      const double v = cval[cb][o];
      const int qq = cidx[cb][o];
      if (v > gb || (v == gb && qq < pc)) { gb = v; pc = qq; }
    }
    if (j == 0) {   // stop rule of k_grsvd
      const double fl2 = 16.0 * Eps<T>::v * Eps<T>::v * (cfro[0] + cfro[1] + cfro[2] + cfro[3]);
      delta2 = eps > 0.0 ? fmax((0.01 * eps * eps) * gb / c, fl2) : 0.0;
    }
    if (gb <= delta2 || !(gb > 0.0)) break;   // same decision in every thread
    if (wv == (pc & 3)) {
      const int slot = pc >> 2;
      T x = T(0);
#pragma unroll
      for (int u = 0; u < SL; ++u)
        if (u == slot) x = w[u];
      const double xv = (double)x;
      const double tail = wave_sum((lane > j && lane < c) ? xv * xv : 0.0);
      const double alpha = wave_sum(lane == j ? xv : 0.0);
      const double nr = sqrt(alpha * alpha + tail);
      const double beta = alpha >= 0.0 ? -nr : nr;
      const bool refl = !(tail == 0.0 || nr == 0.0);
      const double v0 = alpha - beta;
      T vv = T(0);
      if (refl && lane >= j && lane < c) vv = (lane == j) ? T(1) : (T)(xv / v0);
      Vk[j][lane] = vv;
      if (lane == 0) tk[j] = refl ? (T)((beta - alpha) / beta) : T(0);
      const T diag = refl ? (T)beta : (T)alpha;
#pragma unroll
      for (int u = 0; u < SL; ++u)
        if (u == slot) {
          if (lane == j) w[u] = diag;
          else if (lane > j) w[u] = T(0);
        }
    }
#pragma unroll
    for (int u = 0; u < SL; ++u)
      if (wv + 4 * u == pc) used[u] = true;
    __syncthreads();
    const T tau = tk[j];
    if (tau != T(0)) {
      const T v = Vk[j][lane];
#pragma unroll
      for (int u = 0; u < SL; ++u) {
        const int q = wv + 4 * u;
        if (q < c && !used[u]) {
          const T d = wave_sum(v * w[u]) * tau;
          w[u] = fma(-d, v, w[u]);
        }
      }
    }
    if (lane == j)
#pragma unroll
      for (int u = 0; u < SL; ++u) {
        const int q = wv + 4 * u;
        if (q < c) Rt[j][q] = w[u];
      }
    tp = j + 1;
    fl += 6.0 * (double)(c - j) * (c - j);
  }
  __syncthreads();
  if (tp > SV_TP) {
    if (tid == 0) gmem(Jb.redo)[prob] = 1;
    return;
  }
  if (wv != 0) return;
  // one-sided Jacobi on X = R_top^T (c x tp): lane = row of X; J (tp x tp): lane = row
  T x[SV_TP], jr[SV_TP];
#pragma unroll
  for (int i = 0; i < SV_TP; ++i) {
    x[i] = (i < tp && lane < c) ? Rt[i][lane] : T(0);
    jr[i] = (lane == i) ? T(1) : T(0);
  }
  double ssf = 0.0;
#pragma unroll
  for (int i = 0; i < SV_TP; ++i) ssf += (double)x[i] * (double)x[i];
  const double negl2 = wave_sum(ssf) * Eps<T>::v * Eps<T>::v;
  // a pair counts as orthogonal once |cos| <= sqrt(c) u: rounding the rotated
  // columns to the working precision leaves cosines of that size
  const double tol = fmax(4.0, sqrt((double)c)) * Eps<T>::v;
  for (int sweep = 0; sweep < 60 && tp > 1; ++sweep) {
    int nrot = 0;
#pragma unroll
    for (int p0 = 0; p0 < SV_TP; ++p0)
#pragma unroll
      for (int q0 = p0 + 1; q0 < SV_TP; ++q0) {
        if (q0 < tp) {
          const double xa = x[p0], xb = x[q0];
          const double al = wave_sum(xa * xa), be = wave_sum(xb * xb), ga = wave_sum(xa * xb);
          if (fabs(ga) > tol * sqrt(al * be) && fmax(al, be) > negl2) {
            const double zeta = (be - al) / (2.0 * ga);
            const double az = fabs(zeta);
            double t = (az > 1e15) ? 0.5 / az : 1.0 / (az + sqrt(1.0 + az * az));
            t = copysign(t, zeta);
            const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
            x[p0] = (T)(cs * xa - sn * xb);
            x[q0] = (T)(sn * xa + cs * xb);
            const double ja = jr[p0], jb = jr[q0];
            jr[p0] = (T)(cs * ja - sn * jb);
            jr[q0] = (T)(sn * ja + cs * jb);
            ++nrot;
          }
        }
      }
    fl += 3.0 * (double)tp * (tp - 1) * c + (double)nrot * (6.0 * c + 6.0 * tp);
    if (nrot == 0) break;
  }
  // singular values (column norms of X), their order (descending, ties by index)
  T sv[SV_TP];
#pragma unroll
  for (int i = 0; i < SV_TP; ++i) {
    const double s2 = wave_sum((double)x[i] * (double)x[i]);
    sv[i] = i < tp ? (T)sqrt(s2) : T(0);
  }
  int pos[SV_TP];
#pragma unroll
  for (int i = 0; i < SV_TP; ++i) {
    int ps = 0;
#pragma unroll
    for (int o = 0; o < SV_TP; ++o) ps += (o < tp) && (sv[o] > sv[i] || (sv[o] == sv[i] && o < i));
    pos[i] = ps;
  }
  // U_K = Q_K [J; 0]: reflectors applied in reverse order to the columns of J
  T y[SV_TP];
#pragma unroll
  for (int i = 0; i < SV_TP; ++i) y[i] = (lane < tp) ? jr[i] : T(0);
  for (int j = tp - 1; j >= 0; --j) {
    const T tau = tk[j];
    if (tau == T(0)) continue;
    const T v = lane < c ? Vk[j][lane] : T(0);
#pragma unroll
    for (int i = 0; i < SV_TP; ++i)
      if (i < tp) {
        const T d = wave_sum(v * y[i]) * tau;
        y[i] = fma(-d, v, y[i]);
      }
  }
  // numerical rank (every lane holds every sv): keep s_i > eps s_1, capped
  T smax = T(0);
#pragma unroll
  for (int i = 0; i < SV_TP; ++i) smax = sv[i] > smax ? sv[i] : smax;
  int t = 0;
  if (smax > T(0)) {
    const double thr = eps * (double)smax;
#pragma unroll
    for (int i = 0; i < SV_TP; ++i) t += (i < tp) && ((double)sv[i] > thr);
  }
  if (maxrank > 0 && t > maxrank) t = maxrank;
  // U_K in sorted order, columns past the rank zero (the truncated factor)
  T* Y = gmem(static_cast<T*>(Jb.UK)) + (size_t)prob * c * c;
  if (lane < c) {
#pragma unroll
    for (int i = 0; i < SV_TP; ++i)
      if (i < tp) Y[lane + (size_t)pos[i] * c] = pos[i] < t ? y[i] : T(0);
    for (int q = tp; q < c; ++q) Y[lane + (size_t)q * c] = T(0);
  }
  T* so = gmem(static_cast<T*>(Jb.sig)) + (size_t)prob * c;
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < SV_TP; ++i)
      if (i < tp) so[pos[i]] = sv[i];
    for (int q = tp; q < c; ++q) so[q] = T(0);
    gmem(Jb.rank)[prob] = t;
    fl += 4.0 * (double)c * tp * tp;
    if (Jb.flops) gmem(Jb.flops)[prob] = fl;
  }
}

// ------------------------------------------------- QR, one wave per panel
// Value of lane `src` (any lane, per-lane index) through the LDS crossbar
// (ds_bpermute: no LDS storage, no barrier).
__device__ __forceinline__ float lane_fetch(float v, int src) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}
__device__ __forceinline__ double lane_fetch(double v, int src) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)x);
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(x >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Reflector of column j in the one-wave QR layout (below), from this lane's
// entries x of that column (those of the owner lane row, j & 3, count): the
// norm in FP64 (as in the other QR kernels) over the owner row by group_sum,
// alpha by readlane, the same scalars formed in every lane, and this lane's
// rows of v fetched from the owner row (ds_bpermute).  v = x / v0 is formed in
// FP64, so |v_r| <= 1 also for columns far below the FP32 normal range.
template <typename T, int RPL>
__device__ __forceinline__ void wave_reflector(const T (&x)[RPL], int j, int p, int rg, T& tau, T& diag, T (&v)[RPL]) {
  const int jo = j & 3, ji = j >> 4;
  double ss = 0.0;
  T xj = T(0);
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int r = rg + 16 * i;
    const double xv = (double)x[i];
    if (r > j && r < p) ss += xv * xv;
    if (i == ji) xj = x[i];
  }
  const double tail = lane_read(group_sum(ss, 16), 16 * jo);
  const double alpha = (double)lane_read(xj, 16 * jo + (j & 15));
  const double nrm = sqrt(alpha * alpha + tail);
  const double beta = alpha >= 0.0 ? -nrm : nrm;
  const bool refl = !(tail == 0.0 || nrm == 0.0);
  tau = refl ? (T)((beta - alpha) / beta) : T(0);
  diag = refl ? (T)beta : (T)alpha;
  const double rv = refl ? 1.0 / (alpha - beta) : 0.0;
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int r = rg + 16 * i;
    const T got = lane_fetch((T)((double)x[i] * rv), 16 * jo + rg);
    v[i] = (refl && r >= j && r < p) ? ((r == j) ? T(1) : got) : T(0);
  }
}

// Householder QR of a p x k panel (p <= 16*RPL, k <= 4*CPL) held by one wave:
// lane l keeps rows rg + 16 i (rg = l mod 16, i < RPL) of the columns
// cg + 4 u (cg = l / 16, u < CPL).  The entries of a column then lie in one
// DPP row of 16 lanes, so each dot product takes RPL in-lane products and the
// four in-row DPP steps of group_sum, and the panel needs neither LDS storage
// nor barriers.  Step j applies reflector j to the columns q > j; column j+1
// is updated first and its reflector formed right away, so that the latency
// of forming it overlaps the update of the other columns.  Column j keeps its
// old entries (only R's diagonal, stored at once, is needed from it).  Same
// outputs as k_gqr.
template <typename T, int RPL, int CPL>
__device__ __forceinline__ void gqr_wave_body(const QJob& Jb, int prob) {
  const int p = Jb.p, k = Jb.k, ncl = Jb.ncl;
  const int m = prob / ncl, c = prob % ncl;
  const BOp A = Jb.A;
  const T* Ap = optr<T>(A, m, c);
  const int kr = min(p, k);
  T* const Vref = Jb.Vref ? gmem(static_cast<T*>(Jb.Vref)) + (size_t)prob * p * kr : nullptr;
  T* const taus = Jb.tau ? gmem(static_cast<T*>(Jb.tau)) + (size_t)prob * kr : nullptr;
  T* const Rp = gmem(static_cast<T*>(Jb.R)) + (size_t)prob * kr * k;
  const int lane = threadIdx.x % WAVE, rg = lane & 15, cg = lane >> 4;
  T w[RPL][CPL];
#pragma unroll
  for (int i = 0; i < RPL; ++i)
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      const int r = rg + 16 * i, q = cg + 4 * u;
      w[i][u] = (r < p && q < k) ? Ap[r + (long long)q * A.ld] : T(0);
    }
  T tau, diag, v[RPL];
  {
    T x0[RPL];
#pragma unroll
    for (int i = 0; i < RPL; ++i) x0[i] = w[i][0];
    wave_reflector<T, RPL>(x0, 0, p, rg, tau, diag, v);
  }
  for (int j = 0; j < kr; ++j) {
    const int jo = j & 3, jn = j + 1, nn = jn >> 2;
    const T mtau = -tau;
    // column j+1 (slot nn of every lane row) after reflector j, and its reflector
    T xn[RPL];
    {
      T wn[RPL];
#pragma unroll
      for (int i = 0; i < RPL; ++i) wn[i] = T(0);
#pragma unroll
      for (int u = 0; u < CPL; ++u)
        if (u == nn)
#pragma unroll
          for (int i = 0; i < RPL; ++i) wn[i] = w[i][u];
      T d = T(0);
#pragma unroll
      for (int i = 0; i < RPL; ++i) d = fma(v[i], wn[i], d);
      d = group_sum(d, 16);
#pragma unroll
      for (int i = 0; i < RPL; ++i) xn[i] = fma(d * mtau, v[i], wn[i]);
    }
    T tau2, diag2, v2[RPL];
    wave_reflector<T, RPL>(xn, jn, p, rg, tau2, diag2, v2);
    // reflector j on every column q > j (column j+1 again, in its slot)
    T d[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      d[u] = T(0);
#pragma unroll
      for (int i = 0; i < RPL; ++i) d[u] = fma(v[i], w[i][u], d[u]);
    }
#pragma unroll
    for (int u = 0; u < CPL; ++u) d[u] = group_sum(d[u], 16);
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      const int q = cg + 4 * u;
      const T f = (q > j && q < k) ? d[u] * mtau : T(0);
#pragma unroll
      for (int i = 0; i < RPL; ++i) w[i][u] = fma(f, v[i], w[i][u]);
    }
    if (Vref && cg == jo)
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int r = rg + 16 * i;
        if (r < p) Vref[(size_t)j * p + r] = v[i];
      }
    if (lane == 0) {
      if (taus) taus[j] = tau;
      Rp[j + (size_t)j * kr] = diag;
    }
    tau = tau2;
    diag = diag2;
#pragma unroll
    for (int i = 0; i < RPL; ++i) v[i] = v2[i];
  }
  // R: the strict upper part of the first kr rows (diagonal stored above)
#pragma unroll
  for (int i = 0; i < RPL; ++i)
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      const int r = rg + 16 * i, q = cg + 4 * u;
      if (r < kr && q < k && r != q) Rp[r + (size_t)q * kr] = (r < q) ? w[i][u] : T(0);
    }
}

// Shape codes of k_gqr_wave: (rows per lane, column slots) for p <= 16*RPL,
// k <= 4*CPL; FP64 panels use the shapes of at most 32 registers.  Taller
// panels (p > 128) keep the four-wave kernels, which measure faster there.
constexpr int kWaveQrShapes = 8;
__host__ __device__ constexpr int wave_qr_rpl(int code) { return code < 3 ? 2 : code < 6 ? 4 : 8; }
__host__ __device__ constexpr int wave_qr_cpl(int code) { return code < 6 ? 4 << (code % 3) : 4 << (code - 6); }

// One wave (one workgroup) per panel; the job's shape code selects the body.
template <typename T>
__global__ __launch_bounds__(64) void k_gqr_wave(const QJob* __restrict__ jobs, int njobs) {
  const QJob& Jb = jobs[job_of(jobs, njobs, blockIdx.x)];
  const int prob = (int)(blockIdx.x - Jb.block0);
  switch (Jb.pad) {
    case 0: gqr_wave_body<T, 2, 4>(Jb, prob); break;
    case 1: gqr_wave_body<T, 2, 8>(Jb, prob); break;
    case 2: gqr_wave_body<T, 2, 16>(Jb, prob); break;
    case 3: gqr_wave_body<T, 4, 4>(Jb, prob); break;
    case 4: gqr_wave_body<T, 4, 8>(Jb, prob); break;
    case 5: if constexpr (sizeof(T) == 4) gqr_wave_body<T, 4, 16>(Jb, prob); break;
    case 6: gqr_wave_body<T, 8, 4>(Jb, prob); break;
    default: if constexpr (sizeof(T) == 4) gqr_wave_body<T, 8, 8>(Jb, prob); break;
  }
}

// ------------------------------------------------- QR, panel in registers
// Householder QR of a p x k panel (p <= 64*QR_ROWS, k <= 4*QR_SLOTS) with the
// panel in registers: wave w owns the columns q = w + 4u, lane l the rows
// l + 64i.  Step j: the owner of column j forms the reflector (norm by a DPP
// wave sum, v in FP64 as below) and publishes it in LDS (two buffers, so one
// barrier per step suffices); every wave then applies it to its own columns
// q > j.  Same outputs as k_gqr.
template <typename T, int QR_ROWS, int QR_SLOTS>
__device__ __forceinline__ void gqr_reg_body(const QJob& Jb, int prob, T (*vbuf)[WAVE * 8], T* stau) {
  const int p = Jb.p, k = Jb.k, ncl = Jb.ncl;
  const int m = prob / ncl, c = prob % ncl;
  const BOp A = Jb.A;
  const T* Ap = optr<T>(A, m, c);
  const int kr = min(p, k);
  T* const Vref = Jb.Vref ? gmem(static_cast<T*>(Jb.Vref)) + (size_t)prob * p * kr : nullptr;
  T* const taus = Jb.tau ? gmem(static_cast<T*>(Jb.tau)) + (size_t)prob * kr : nullptr;
  const int tid = threadIdx.x, lane = tid % WAVE;
  const int wv = __builtin_amdgcn_readfirstlane(tid / WAVE);
  T w[QR_ROWS][QR_SLOTS];
#pragma unroll
  for (int i = 0; i < QR_ROWS; ++i)
#pragma unroll
    for (int u = 0; u < QR_SLOTS; ++u) {
      const int r = lane + WAVE * i, q = wv + 4 * u;
      w[i][u] = (r < p && q < k) ? Ap[r + (long long)q * A.ld] : T(0);
    }
  for (int j = 0; j < kr; ++j) {
    const int buf = j & 1;
    if (wv == (j & 3)) {
      const int slot = j >> 2;
      T x[QR_ROWS];
#pragma unroll
      for (int i = 0; i < QR_ROWS; ++i) x[i] = T(0);
#pragma unroll
      for (int u = 0; u < QR_SLOTS; ++u)
        if (u == slot)
#pragma unroll
          for (int i = 0; i < QR_ROWS; ++i) x[i] = w[i][u];
      double ss = 0.0, ap = 0.0;
#pragma unroll
      for (int i = 0; i < QR_ROWS; ++i) {
        const int r = lane + WAVE * i;
        const double xv = (double)x[i];
        if (r > j && r < p) ss += xv * xv;
        if (r == j) ap = xv;
      }
      const double tail = wave_sum(ss);
      const double alpha = wave_sum(ap);
      const double nrm = sqrt(alpha * alpha + tail);
      const double beta = alpha >= 0.0 ? -nrm : nrm;
      const bool refl = !(tail == 0.0 || nrm == 0.0);
      const T tau = refl ? (T)((beta - alpha) / beta) : T(0);
      // v = x / v0 formed in FP64: |v_r| <= 1 even for columns far below the
      // FP32 normal range, where an FP32 reciprocal of v0 would overflow
      const double v0 = alpha - beta;
#pragma unroll
      for (int i = 0; i < QR_ROWS; ++i) {
        const int r = lane + WAVE * i;
        T vv = T(0);
        if (refl && r >= j && r < p) vv = (r == j) ? T(1) : (T)((double)x[i] / v0);
        if (r < p) {
          vbuf[buf][r] = vv;
          if (Vref) Vref[(size_t)j * p + r] = vv;
        }
      }
      if (lane == 0) {
        stau[buf] = tau;
        if (taus) taus[j] = tau;
      }
      const T diag = refl ? (T)beta : (T)alpha;
#pragma unroll
      for (int u = 0; u < QR_SLOTS; ++u)
        if (u == slot)
#pragma unroll
          for (int i = 0; i < QR_ROWS; ++i) {
            const int r = lane + WAVE * i;
            if (r == j) w[i][u] = diag;
            else if (r > j) w[i][u] = T(0);
          }
    }
    __syncthreads();
    const T tau = stau[buf];
    if (tau != T(0)) {
      T v[QR_ROWS];
#pragma unroll
      for (int i = 0; i < QR_ROWS; ++i) {
        const int r = lane + WAVE * i;
        v[i] = r < p ? vbuf[buf][r] : T(0);
      }
#pragma unroll
      for (int u = 0; u < QR_SLOTS; ++u) {
        const int q = wv + 4 * u;
        if (q > j && q < k) {
          T d = T(0);
#pragma unroll
          for (int i = 0; i < QR_ROWS; ++i) d = fma(v[i], w[i][u], d);
          d = wave_sum(d) * tau;
#pragma unroll
          for (int i = 0; i < QR_ROWS; ++i) w[i][u] = fma(-d, v[i], w[i][u]);
        }
      }
    }
  }
  // R = upper trapezoid of the first kr rows
  T* Rp = gmem(static_cast<T*>(Jb.R)) + (size_t)prob * kr * k;
#pragma unroll
  for (int i = 0; i < QR_ROWS; ++i)
#pragma unroll
    for (int u = 0; u < QR_SLOTS; ++u) {
      const int r = lane + WAVE * i, q = wv + 4 * u;
      if (r < kr && q < k) Rp[r + (size_t)q * kr] = (r <= q) ? w[i][u] : T(0);
    }
}

template <typename T, int QR_ROWS, int QR_SLOTS>
__global__ __launch_bounds__(256) void k_gqr_reg(const QJob* __restrict__ jobs, int njobs) {
  __shared__ T vbuf[2][WAVE * 8];
  __shared__ T stau[2];
  const QJob& Jb = jobs[job_of(jobs, njobs, blockIdx.x)];
  gqr_reg_body<T, QR_ROWS, QR_SLOTS>(Jb, (int)(blockIdx.x - Jb.block0), vbuf, stau);
}

// All register shapes in one launch (the job's shape code selects the body):
// used when a launch is too small to fill the GPU, where one launch per
// shape would only add their latencies.
template <typename T>
__global__ __launch_bounds__(256) void k_gqr_any(const QJob* __restrict__ jobs, int njobs) {
  __shared__ T vbuf[2][WAVE * 8];
  __shared__ T stau[2];
  const QJob& Jb = jobs[job_of(jobs, njobs, blockIdx.x)];
  const int prob = (int)(blockIdx.x - Jb.block0);
  switch (Jb.pad) {
    case 0: gqr_reg_body<T, 1, 4>(Jb, prob, vbuf, stau); break;
    case 1: gqr_reg_body<T, 1, 8>(Jb, prob, vbuf, stau); break;
    case 2: gqr_reg_body<T, 1, 16>(Jb, prob, vbuf, stau); break;
    case 3: gqr_reg_body<T, 2, 4>(Jb, prob, vbuf, stau); break;
    case 4: gqr_reg_body<T, 2, 8>(Jb, prob, vbuf, stau); break;
    case 5: gqr_reg_body<T, 2, 16>(Jb, prob, vbuf, stau); break;
    case 6: gqr_reg_body<T, 4, 4>(Jb, prob, vbuf, stau); break;
    case 7: gqr_reg_body<T, 4, 8>(Jb, prob, vbuf, stau); break;
    case 8: gqr_reg_body<T, 4, 16>(Jb, prob, vbuf, stau); break;
    case 9: gqr_reg_body<T, 8, 4>(Jb, prob, vbuf, stau); break;
    case 10: gqr_reg_body<T, 8, 8>(Jb, prob, vbuf, stau); break;
    default: gqr_reg_body<T, 8, 16>(Jb, prob, vbuf, stau); break;
  }
}

// ------------------------------------------------------------ QR (R only)
// Householder QR of a p x k panel; one workgroup of 256 threads per problem.
// The panel is copied to LDS (INLDS: every job of the launch) or to a global
// scratch copy.
template <typename T, bool INLDS>
__global__ __launch_bounds__(256) void k_gqr(const QJob* __restrict__ jobs, int njobs) {
  extern __shared__ unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  __shared__ double red[4];
  __shared__ T s_beta, s_tau;
  __shared__ double s_v0;
  const QJob& Jb = jobs[job_of(jobs, njobs, blockIdx.x)];
  const int prob = (int)(blockIdx.x - Jb.block0);
  const int p = Jb.p, k = Jb.k, ncl = Jb.ncl;
  const int m = prob / ncl, c = prob % ncl;
  const BOp A = Jb.A;
  const T* Ap = optr<T>(A, m, c);
  const int krr = min(p, k);
  T* const R = gmem(static_cast<T*>(Jb.R));
  T* const Vref = Jb.Vref ? gmem(static_cast<T*>(Jb.Vref)) + (size_t)prob * p * krr : nullptr;
  T* const taus = Jb.tau ? gmem(static_cast<T*>(Jb.tau)) + (size_t)prob * krr : nullptr;
  T* v = sm;                                  // Householder vector, p entries
  T* W = INLDS ? sm + p : gmem(static_cast<T*>(Jb.ws)) + (size_t)prob * p * k;
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
        T* vo = Vref + (size_t)j * p;
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
      T* vo = Vref + (size_t)j * p;
      for (int r = tid; r < p; r += 256) vo[r] = T(0);
    }
    if (Vref && tid == 0) taus[j] = tau;
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

// Y = Q [Z; 0] with one wave per problem (p <= 16*RPL, t <= 4*CPL), in the
// layout of the one-wave QR: lane l keeps rows rg + 16 i (rg = l mod 16) of
// the output columns cg + 4 u (cg = l / 16), so a reflector step takes RPL
// in-lane products and the in-row group_sum per column slot, and no barrier.
// The reflectors and their taus are staged in LDS (vs); the next reflector is
// read while the current one is applied.
template <typename T, int RPL, int CPL>
__device__ __forceinline__ void gapply_wave_body(const AJob& Jb, int prob, T* vs) {
  const int p = Jb.p, c = Jb.c, t = Jb.t, ncl = Jb.ncl;
  const int m = prob / ncl, cl = prob % ncl;
  const BOp Y = Jb.Y;
  T* y = const_cast<T*>(optr<T>(Y, m, cl));
  const T* z = gmem(static_cast<const T*>(Jb.Z)) + (size_t)(m * ncl + (cl ^ Jb.zxor)) * Jb.sZ;
  const T* vr = gmem(static_cast<const T*>(Jb.Vref)) + (size_t)prob * p * c;
  const T* ta = gmem(static_cast<const T*>(Jb.tau)) + (size_t)prob * c;
  const int lane = threadIdx.x % WAVE, rg = lane & 15, cg = lane >> 4;
  T* ts = vs + (size_t)p * c;
  for (int e = lane; e < p * c; e += WAVE) vs[e] = vr[e];
  for (int e = lane; e < c; e += WAVE) ts[e] = ta[e];
  T yr[RPL][CPL];
#pragma unroll
  for (int i = 0; i < RPL; ++i)
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      const int r = rg + 16 * i, q = cg + 4 * u;
      yr[i][u] = (r < c && q < t) ? z[r + (size_t)q * c] : T(0);
    }
  // wavefront-scope fence: the staged reflectors are visible to every lane
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  T vn[RPL], taun = c > 0 ? ts[c - 1] : T(0);
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int r = rg + 16 * i;
    vn[i] = (c > 0 && r < p) ? vs[(size_t)(c - 1) * p + r] : T(0);
  }
  for (int j = c - 1; j >= 0; --j) {
    T v[RPL];
#pragma unroll
    for (int i = 0; i < RPL; ++i) v[i] = vn[i];
    const T mtau = -taun;
    const int jn = j > 0 ? j - 1 : 0;
    taun = ts[jn];
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int r = rg + 16 * i;
      vn[i] = r < p ? vs[(size_t)jn * p + r] : T(0);
    }
    T d[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      d[u] = T(0);
#pragma unroll
      for (int i = 0; i < RPL; ++i) d[u] = fma(v[i], yr[i][u], d[u]);
    }
#pragma unroll
    for (int u = 0; u < CPL; ++u) d[u] = group_sum(d[u], 16) * mtau;
#pragma unroll
    for (int u = 0; u < CPL; ++u)
#pragma unroll
      for (int i = 0; i < RPL; ++i) yr[i][u] = fma(d[u], v[i], yr[i][u]);
  }
#pragma unroll
  for (int i = 0; i < RPL; ++i)
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      const int r = rg + 16 * i, q = cg + 4 * u;
      if (r < p && q < t) y[r + (long long)q * Y.ld] = yr[i][u];
    }
}

// The job's shape code (RPL index * 3 + CPL index, each over {2, 4, 8})
// selects the one-wave body; FP64 uses the shapes of at most 32 registers.
template <typename T>
__device__ __forceinline__ void gapply_wave(const AJob& Jb, int prob, T* vs) {
  switch (Jb.pad) {
    case 0: gapply_wave_body<T, 2, 2>(Jb, prob, vs); break;
    case 1: gapply_wave_body<T, 2, 4>(Jb, prob, vs); break;
    case 2: gapply_wave_body<T, 2, 8>(Jb, prob, vs); break;
    case 3: gapply_wave_body<T, 4, 2>(Jb, prob, vs); break;
    case 4: gapply_wave_body<T, 4, 4>(Jb, prob, vs); break;
    case 5: gapply_wave_body<T, 4, 8>(Jb, prob, vs); break;
    case 6: gapply_wave_body<T, 8, 2>(Jb, prob, vs); break;
    case 7: gapply_wave_body<T, 8, 4>(Jb, prob, vs); break;
    default: if constexpr (sizeof(T) == 4) gapply_wave_body<T, 8, 8>(Jb, prob, vs); break;
  }
}

// Y = Q [Z; 0] for the Householder Q of a QR with reflectors (v_j, tau_j):
// Y is p x t (column-major, ld = Y.ld, in place), Z is c x t (ld c).  Jobs
// with lds == 2 run four problems per workgroup, one wave each (gapply_wave,
// reflectors in the wave's LDS slot of wslot elements); the others one problem
// per workgroup.
template <typename T>
__global__ __launch_bounds__(256) void k_gapply_q(const AJob* __restrict__ jobs, int njobs) {
  const AJob& Jb = jobs[job_of(jobs, njobs, blockIdx.x)];
  if (Jb.lds == 2) {
    extern __shared__ unsigned char smem_raw[];
    const int wq = threadIdx.x / WAVE;
    const long long pw = (long long)(blockIdx.x - Jb.block0) * 4 + wq;
    if (pw >= (long long)Jb.nmat * Jb.ncl) return;
    gapply_wave<T>(Jb, (int)pw, reinterpret_cast<T*>(smem_raw) + (size_t)wq * Jb.wslot);
    return;
  }
  const int prob = (int)(blockIdx.x - Jb.block0);
  const int p = Jb.p, c = Jb.c, t = Jb.t, ncl = Jb.ncl;
  const int m = prob / ncl, cl = prob % ncl;
  const BOp Y = Jb.Y;
  T* y = const_cast<T*>(optr<T>(Y, m, cl));
  const T* z = gmem(static_cast<const T*>(Jb.Z)) + (size_t)(m * ncl + (cl ^ Jb.zxor)) * Jb.sZ;
  const T* vr = gmem(static_cast<const T*>(Jb.Vref)) + (size_t)prob * p * c;
  const T* ta = gmem(static_cast<const T*>(Jb.tau)) + (size_t)prob * c;
  const int tid = threadIdx.x, wv = tid / WAVE, lane = tid % WAVE;
  if (Jb.lds) {
    // Reflectors (and their taus) in LDS; wave w owns the output columns
    // q = w + 4u and keeps them in registers, lane l the rows l + 64 i, so the
    // reflector steps need no barrier and no LDS stores.
    constexpr int RMAX = kApplyRows, CMAX = kApplyCols;
    extern __shared__ unsigned char smem_raw[];
    T* vs = reinterpret_cast<T*>(smem_raw);
    T* ts = vs + (size_t)p * c;
    for (int e = tid; e < p * c; e += 256) vs[e] = vr[e];
    for (int e = tid; e < c; e += 256) ts[e] = ta[e];
    T yr[RMAX][CMAX];
#pragma unroll
    for (int i = 0; i < RMAX; ++i)
#pragma unroll
      for (int u = 0; u < CMAX; ++u) {
        const int r = lane + WAVE * i, q = wv + 4 * u;
        yr[i][u] = (r < c && q < t) ? z[r + (size_t)q * c] : T(0);
      }
    __syncthreads();
    for (int j = c - 1; j >= 0; --j) {
      const T tau = ts[j];
      if (tau == T(0)) continue;
      T v[RMAX];
#pragma unroll
      for (int i = 0; i < RMAX; ++i) {
        const int r = lane + WAVE * i;
        v[i] = r < p ? vs[(size_t)j * p + r] : T(0);
      }
#pragma unroll
      for (int u = 0; u < CMAX; ++u) {
        if (wv + 4 * u < t) {
          T d = T(0);
#pragma unroll
          for (int i = 0; i < RMAX; ++i) d = fma(v[i], yr[i][u], d);
          d = wave_sum(d) * tau;
#pragma unroll
          for (int i = 0; i < RMAX; ++i) yr[i][u] = fma(-d, v[i], yr[i][u]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < RMAX; ++i)
#pragma unroll
      for (int u = 0; u < CMAX; ++u) {
        const int r = lane + WAVE * i, q = wv + 4 * u;
        if (r < p && q < t) y[r + (long long)q * Y.ld] = yr[i][u];
      }
    return;
  }
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

// Partner of index i in round rnd of the round-robin ordering of cp (even)
// indices (index 0 stays, the others rotate through cp - 1 places); the
// pairs of a round are those of the one-sided Jacobi loop of k_grsvd.
__device__ __forceinline__ int rr_partner(int i, int rnd, int cp) {
  const int m = cp - 1;
  if (i == 0) return 1 + (rnd + m - 1) % m;
  const int a = i - 1, r1 = (rnd + m - 1) % m;
  if (a == r1) return 0;
  return 1 + ((2 * r1 - a) % m + m) % m;
}

// ------------------------------------------------ rank-revealing SVD
// Rank-revealing SVD of a recompression core K (c x c, column-major, used as
// scratch in place), preconditioned one-sided Jacobi:
//  1. column-pivoted Householder QR  K P = Q_K [R_top; R22], stopped once every
//     remaining column norm is <= delta = 0.1 eps nu_1 / sqrt(c) (nu_1 = largest
//     column norm <= s_1), so ||R22||_2 <= 0.1 eps s_1;
//  2. one-sided Jacobi on the thin X = R_top^T (c x t'): X J_X = Usc_X, so
//     R_top = J_X S Utilde^T and the left singular vectors of K are
//     U_K = Q_K [J_X; 0] (J_X is accumulated from plane rotations, hence
//     orthogonal to working precision);
//  3. sort by s, rank_p = #{s_i > eps s_1} (capped by maxrank > 0).
// Outputs per problem: sig[c] (sorted, zero past t'), UK (c x c, column k the
// k-th left singular vector, zero past t').
// NW waves per core, cores of size c <= CMAX (the static arrays' size).  With
// INLDS every job of the launch keeps the core and both work matrices in LDS
// (and the compiler emits LDS instructions for them); without, they work in
// global scratch.
template <typename T, int NW, int CMAX, bool INLDS>
__global__ __launch_bounds__(NW * 64) void k_grsvd_t(const SJob* __restrict__ jobs, int njobs) {
  constexpr int NTH = NW * 64;
  constexpr int GD = NW == 4 ? 16 : 8;   // Gram path: t' <= GD, one thread per entry
  __shared__ double nrm[CMAX];
  __shared__ double taus[CMAX];
  __shared__ T snorm[CMAX];
  __shared__ int spos[CMAX];
  __shared__ double red[NW];
  __shared__ int s_piv, s_stop, nrot, s_rank;
  __shared__ double s_delta2, s_v0;
  __shared__ T s_beta;
  __shared__ double gA[GD * GD], gB[GD * GD], vA[GD * GD], vB[GD * GD];   // FP32 cores, t' <= GD: Gram matrix and rotations
  __shared__ double rc[GD], rs[GD], gdiag[GD];
  __shared__ int rp[GD], gflag;
  const SJob& Jb = jobs[job_of(jobs, njobs, blockIdx.x)];
  const int prob = (int)(blockIdx.x - Jb.block0);
  if (Jb.redo && gmem(Jb.redo)[prob] == 0) return;   // finished by k_grsvd_reg
  const int c = Jb.c, maxrank = Jb.maxrank;
  const double eps = Jb.eps;
  T* const sig = gmem(static_cast<T*>(Jb.sig));
  T* const UK = gmem(static_cast<T*>(Jb.UK));
  int* const rank = gmem(Jb.rank);
  double* const flops = gmem(Jb.flops);
  const int tid = threadIdx.x, wv = tid / WAVE, lane = tid % WAVE;
  extern __shared__ unsigned char smem_raw[];
  T* W;
  T* X;
  T* J;
  if constexpr (INLDS) {   // the core and both work matrices in LDS
    T* sm = reinterpret_cast<T*>(smem_raw);
    const T* src = gmem(static_cast<const T*>(Jb.K)) + (size_t)prob * c * c;
    for (int e = tid; e < c * c; e += NTH) sm[e] = src[e];
    W = sm;
    X = sm + (size_t)c * c;
    J = sm + 2 * (size_t)c * c;
    __syncthreads();
  } else {
    W = gmem(static_cast<T*>(Jb.K)) + (size_t)prob * c * c;
    X = gmem(static_cast<T*>(Jb.X)) + (size_t)prob * c * c;
    J = gmem(static_cast<T*>(Jb.J)) + (size_t)prob * c * c;
  }
  double fl = 0.0;
  int tp = 0;
  // Cores of at most 32: each wave takes 64 / cgl columns at a time, one per
  // group of cgl lanes (lane = row + cgl * column offset), summed by group_sum
  // over cgl lanes; larger cores take one column per wave.
  const int cgl = c <= 16 ? 16 : c <= 32 ? 32 : WAVE, cw = WAVE / cgl;
  const bool grouped = cgl < WAVE;
  for (int j = 0; j < c; ++j) {
    if (grouped) {
      const int r = lane % cgl;
      for (int q0 = j + wv * cw; q0 < c; q0 += NW * cw) {
        const int q = q0 + lane / cgl;
        const double x = (q < c && r >= j && r < c) ? (double)W[r + (size_t)q * c] : 0.0;
        const double ss = group_sum(x * x, cgl);
        if (r == 0 && q < c) nrm[q] = ss;
      }
    } else {
      for (int q = j + wv; q < c; q += NW) {
        const T* col = W + (size_t)q * c;
        double ss = 0.0;
        for (int r = j + lane; r < c; r += WAVE) ss += (double)col[r] * (double)col[r];
        ss = wave_sum(ss);
        if (lane == 0) nrm[q] = ss;
      }
    }
    __syncthreads();
    if (tid < WAVE) {
      double best = -1.0;
      int bi = j;
      for (int q = j + tid; q < c; q += WAVE)
        if (nrm[q] > best) { best = nrm[q]; bi = q; }
      wave_argmax(best, bi);
      if (tid == 0) {
        if (j == 0) {
          // stop once the remaining columns are below 0.1 eps of the largest one
          // (scaled by the core size) or at the rounding floor of the working
          // precision, 4 u ||K||_F, below which they carry no information
          double fro = 0.0;
          for (int q = 0; q < c; ++q) fro += nrm[q];
          const double fl2 = 16.0 * Eps<T>::v * Eps<T>::v * fro;
          s_delta2 = eps > 0.0 ? fmax((0.01 * eps * eps) * best / c, fl2) : 0.0;
        }
        s_piv = bi;
        s_stop = (best <= s_delta2) || !(best > 0.0);
      }
    }
    __syncthreads();
    if (s_stop) break;
    const int pc = s_piv;
    if (pc != j)
      for (int r = tid; r < c; r += NTH) {
        const T a = W[r + (size_t)j * c];
        W[r + (size_t)j * c] = W[r + (size_t)pc * c];
        W[r + (size_t)pc * c] = a;
      }
    __syncthreads();
    double ss = 0.0;
    for (int r = j + 1 + tid; r < c; r += NTH) ss += (double)W[r + (size_t)j * c] * (double)W[r + (size_t)j * c];
    const double tail = block_sum_n<NW>(ss, red);
    if (tid == 0) {
      const double alpha = (double)W[j + (size_t)j * c];
      const double nr = sqrt(alpha * alpha + tail);
      const double beta = alpha >= 0.0 ? -nr : nr;
      if (tail == 0.0 || nr == 0.0) {
        taus[j] = 0.0;
        s_beta = (T)alpha;
      } else {
        taus[j] = (beta - alpha) / beta;
        s_v0 = alpha - beta;
        s_beta = (T)beta;
      }
    }
    __syncthreads();
    const T tau = (T)taus[j];
    if (tau != T(0)) {
      const double v0 = s_v0;
      for (int r = j + 1 + tid; r < c; r += NTH) W[r + (size_t)j * c] = (T)((double)W[r + (size_t)j * c] / v0);
      __syncthreads();
      const T* v = W + (size_t)j * c;
      if (grouped) {
        // v_j = 1 is implicit; rows below j hold v
        const int r = lane % cgl;
        const T vr = r == j ? T(1) : (r > j && r < c) ? v[r] : T(0);
        for (int q0 = j + 1 + wv * cw; q0 < c; q0 += NW * cw) {
          const int q = q0 + lane / cgl;
          const bool ok = q < c && r >= j && r < c;
          const T x = ok ? W[r + (size_t)q * c] : T(0);
          const T d = group_sum(vr * x, cgl) * tau;
          if (ok) W[r + (size_t)q * c] = fma(-d, vr, x);
        }
      } else {
        for (int q = j + 1 + wv; q < c; q += NW) {
          T* col = W + (size_t)q * c;
          T d = lane == 0 ? col[j] : T(0);
          for (int r = j + 1 + lane; r < c; r += WAVE) d = fma(v[r], col[r], d);
          d = wave_sum(d) * tau;
          if (lane == 0) col[j] -= d;
          for (int r = j + 1 + lane; r < c; r += WAVE) col[r] = fma(-d, v[r], col[r]);
        }
      }
    }
    __syncthreads();
    if (tid == 0) W[j + (size_t)j * c] = s_beta;
    __syncthreads();
    tp = j + 1;
    fl += 6.0 * (double)(c - j) * (c - j);
  }
  // X = R_top^T (c x tp), J_X = I (tp x tp), both with leading dimension c
  for (int e = tid; e < c * tp; e += NTH) {
    const int q = e % c, i = e / c;
    X[q + (size_t)i * c] = q >= i ? W[i + (size_t)q * c] : T(0);
  }
  for (int e = tid; e < tp * tp; e += NTH) {
    const int r = e % tp, i = e / tp;
    J[r + (size_t)i * c] = r == i ? T(1) : T(0);
  }
  __syncthreads();
  double ssf = 0.0;   // cores of at most 16: summed by the first wave in both forms
  const int sstride = c <= 16 ? WAVE : NTH;
  for (int e = tid; e < c * tp && tid < sstride; e += sstride) {
    const double x = X[(e % c) + (size_t)(e / c) * c];
    ssf += x * x;
  }
  const double negl2 = block_sum_n<NW>(ssf, red) * Eps<T>::v * Eps<T>::v;
  // a pair counts as orthogonal once |cos| <= sqrt(c) u: rounding the rotated
  // columns to the working precision leaves cosines of that size
  const double tol = fmax(4.0, sqrt((double)c)) * Eps<T>::v;
  const int cp = (tp + 1) & ~1;
  const int npairs = cp / 2;
  // Lanes per column pair: cores of at most 16 (which both the one-wave and
  // the four-wave form take) size the groups for one wave whatever NW is, so
  // that both forms compute every pair's sums alike and give the same bits;
  // larger cores spread over the whole workgroup.
  int g = (c <= 16 ? WAVE : NTH) / max(npairs, 1), gp = 1;
  while (gp * 2 <= g && gp * 2 <= WAVE) gp *= 2;
  g = gp;
  const int slots = NTH / g, gl = tid % g;
  // FP32 cores with t' <= GD: the same rotations applied to the Gram matrix
  // X^T X, formed and rotated in FP64 (one thread per entry), which needs no
  // cross-lane sums.  FP64 keeps the smallest retained s_i^2 ~ (eps s_1)^2
  // to a relative 1e-4 and more, ample for the FP32 truncation.  Cores of at
  // most 16 use it up to t' = 8 in both forms (the one-wave form's limit).
  const bool gram = sizeof(T) == 4 && tp > 1 && tp <= (c <= 16 ? 8 : GD);
  if (gram) {
    const int gi = tid / GD, gk = tid % GD;
    const bool ent = gi < tp && gk < tp;
    if (ent) {
      const T* xi = X + (size_t)gi * c;
      const T* xk = X + (size_t)gk * c;
      double sacc = 0.0;
      for (int q = 0; q < c; ++q) sacc = fma((double)xi[q], (double)xk[q], sacc);
      gA[tid] = sacc;
      vA[tid] = gi == gk ? 1.0 : 0.0;
    }
    __syncthreads();
    double* G = gA;
    double* Gn = gB;
    double* V = vA;
    double* Vn = vB;
    int nsw = 0;
    for (int sweep = 0; sweep < 60; ++sweep) {
      ++nsw;
      if (tid == 0) gflag = 0;
      for (int rnd = 0; rnd < cp - 1; ++rnd) {
        if (tid < GD) {   // one wave: the rotation of every index's pair
          double cv = 1.0, sv = 0.0;
          int px = tid;
          if (tid < tp) {
            const int k = rr_partner(tid, rnd, cp);
            if (k < tp) {
              px = k;
              const int lo = min(tid, k), hi = max(tid, k);
              const double al = G[lo * (GD + 1)], be = G[hi * (GD + 1)], ga = G[lo * GD + hi];
              if (fabs(ga) > tol * sqrt(al * be) && fmax(al, be) > negl2) {
                const double zeta = (be - al) / (2.0 * ga);
                const double az = fabs(zeta);
                double t = (az > 1e15) ? 0.5 / az : 1.0 / (az + sqrt(1.0 + az * az));
                t = copysign(t, zeta);
                const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
                cv = cs;
                sv = tid == lo ? -sn : sn;   // new column x = cv x + sv (partner column)
                gflag = 1;
              }
            }
          }
          rc[tid] = cv;
          rs[tid] = sv;
          rp[tid] = px;
        }
        __syncthreads();
        if (ent) {   // G <- R^T G R, V <- V R
          const int pi = rp[gi], pk = rp[gk];
          const double ai = rc[gi], bi = rs[gi], ak = rc[gk], bk = rs[gk];
          Gn[tid] = ai * (ak * G[gi * GD + gk] + bk * G[gi * GD + pk]) +
                    bi * (ak * G[pi * GD + gk] + bk * G[pi * GD + pk]);
          Vn[tid] = ak * V[gi * GD + gk] + bk * V[gi * GD + pk];
        }
        __syncthreads();
        double* tg = G; G = Gn; Gn = tg;
        double* tv = V; V = Vn; Vn = tv;
      }
      if (!gflag) break;
      __syncthreads();   // every thread has read gflag before it is reset
    }
    if (tid < tp) gdiag[tid] = G[tid * (GD + 1)];
    for (int e = tid; e < tp * tp; e += NTH) {
      const int r = e % tp, i = e / tp;
      J[r + (size_t)i * c] = (T)V[r * GD + i];
    }
    fl += 2.0 * c * tp * tp + nsw * 12.0 * (double)tp * tp * (tp - 1);
    __syncthreads();
  }
  for (int sweep = 0; sweep < 60 && tp > 1 && !gram; ++sweep) {
    if (tid == 0) nrot = 0;
    __syncthreads();
    for (int rnd = 0; rnd < cp - 1; ++rnd) {
      for (int pb = 0; pb < npairs; pb += slots) {
        const int pk = pb + tid / g;
        int i = -1, jj = -1;
        if (pk < npairs) {
          const int a = (pk == 0) ? 0 : ((rnd + pk - 1) % (cp - 1)) + 1;
          const int b = ((rnd + (cp - 1 - pk) - 1) % (cp - 1)) + 1;
          i = min(a, b); jj = max(a, b);
          if (jj >= tp) { i = -1; jj = -1; }
        }
        double al = 0.0, be = 0.0, ga = 0.0;
        if (i >= 0) {
          const T* xi = X + (size_t)i * c;
          const T* xj = X + (size_t)jj * c;
          for (int r = gl; r < c; r += g) {
            const double x = xi[r], y = xj[r];
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
          T* xi = X + (size_t)i * c;
          T* xj = X + (size_t)jj * c;
          for (int r = gl; r < c; r += g) {
            const double x = xi[r], y = xj[r];
            xi[r] = (T)(cs * x - sn * y);
            xj[r] = (T)(sn * x + cs * y);
          }
          T* ji = J + (size_t)i * c;
          T* jjp = J + (size_t)jj * c;
          for (int r = gl; r < tp; r += g) {
            const double x = ji[r], y = jjp[r];
            ji[r] = (T)(cs * x - sn * y);
            jjp[r] = (T)(sn * x + cs * y);
          }
          if (gl == 0) atomicAdd(&nrot, 1);
        }
        __syncthreads();
      }
    }
    __syncthreads();
    const int nr = nrot;
    fl += 3.0 * (double)tp * (tp - 1) * c + (double)nr * (6.0 * c + 6.0 * tp);
    __syncthreads();
    if (nr == 0) break;
  }
  // singular values, sort (descending, ties by index)
  for (int q = tid; q < c; q += NTH) {
    double s2 = 0.0;
    if (q < tp) {
      if (gram) {
        s2 = fmax(gdiag[q], 0.0);
      } else {
        const T* xq = X + (size_t)q * c;
        for (int r = 0; r < c; ++r) s2 += (double)xq[r] * (double)xq[r];
      }
    }
    snorm[q] = (T)sqrt(s2);
  }
  __syncthreads();
  for (int q = tid; q < c; q += NTH) {
    const T v = snorm[q];
    int pos = 0;
    for (int o = 0; o < c; ++o) pos += (snorm[o] > v) || (snorm[o] == v && o < q);
    spos[q] = pos;
  }
  if (tid == 0) {   // numerical rank: keep s_i > eps s_1, capped
    T smax = T(0);
    for (int q = 0; q < c; ++q) smax = snorm[q] > smax ? snorm[q] : smax;
    int t = 0;
    if (smax > T(0)) {
      const double thr = eps * (double)smax;
      for (int q = 0; q < c; ++q) t += ((double)snorm[q] > thr);
    }
    if (maxrank > 0 && t > maxrank) t = maxrank;
    s_rank = t;
  }
  __syncthreads();
  // U_K = Q_K [J_X; 0] with columns in sorted order, built in the work matrix
  // X (free after the sort) when it is in LDS, else directly in UK.  Each wave
  // owns its columns for every reflector, so the loop needs no barriers.
  T* const Yg = UK + (size_t)prob * c * c;
  T* const Y = INLDS ? X : Yg;
  for (int e = tid; e < c * c; e += NTH) {
    const int r = e % c, q = e / c;    // q = source column (unsorted)
    T v = T(0);
    if (q < tp && r < tp) v = J[r + (size_t)q * c];
    if (q < tp) Y[r + (size_t)spos[q] * c] = v;
    else Y[r + (size_t)q * c] = T(0);   // columns past tp stay zero (spos[q] == q there)
  }
  __syncthreads();
  for (int j = tp - 1; j >= 0; --j) {
    const T tau = (T)taus[j];
    if (tau == T(0)) continue;
    const T* v = W + (size_t)j * c;
    if (grouped) {
      const int r = lane % cgl;
      const T vr = r == j ? T(1) : (r > j && r < c) ? v[r] : T(0);
      for (int q0 = wv * cw; q0 < tp; q0 += NW * cw) {
        const int q = q0 + lane / cgl;
        const bool ok = q < tp && r >= j && r < c;
        const T x = ok ? Y[r + (size_t)q * c] : T(0);
        const T d = group_sum(vr * x, cgl) * tau;
        if (ok) Y[r + (size_t)q * c] = fma(-d, vr, x);
      }
    } else {
      for (int q = wv; q < tp; q += NW) {
        T* col = Y + (size_t)q * c;
        const T cj = col[j];
        T d = T(0);
        for (int r = j + 1 + lane; r < c; r += WAVE) d = fma(v[r], col[r], d);
        d = (cj + wave_sum(d)) * tau;
        for (int r = j + 1 + lane; r < c; r += WAVE) col[r] = fma(-d, v[r], col[r]);
        if (lane == 0) col[j] = cj - d;
      }
    }
  }
  // the truncated factor: U_K columns past the rank are zero
  __syncthreads();
  const int t_rank = s_rank;
  if constexpr (INLDS) {
    for (int e = tid; e < c * c; e += NTH) Yg[e] = e / c < t_rank ? Y[e] : T(0);
  } else {
    for (int e = t_rank * c + tid; e < c * c; e += NTH) Yg[e] = T(0);
  }
  T* so = sig + (size_t)prob * c;
  for (int q = tid; q < c; q += NTH) so[spos[q]] = snorm[q];
  if (tid == 0) {
    rank[prob] = t_rank;
    fl += 4.0 * (double)c * tp * tp;
    if (flops) flops[prob] = fl;
  }
}

constexpr int kCopyChunk = 2048;

// A workgroup copies one chunk of kCopyChunk elements of one matrix; every
// thread issues its kCopyChunk / 256 loads before its stores.
template <typename T>
__global__ __launch_bounds__(256) void k_gcopy(const CJob* __restrict__ jobs, int njobs) {
  constexpr int PER = kCopyChunk / 256;
  const CJob& Jb = jobs[job_of(jobs, njobs, blockIdx.x)];
  const long long local = blockIdx.x - Jb.block0;
  const int chunk = (int)(local % Jb.chunks);
  const long long pc = local / Jb.chunks;
  const int m = (int)(pc / Jb.ncl), c = (int)(pc % Jb.ncl);
  const BOp src = Jb.src, dst = Jb.dst;
  const T* sp = optr<T>(src, m, c);
  T* dp = const_cast<T*>(optr<T>(dst, m, c));
  const T* sc = Jb.scale ? gmem(static_cast<const T*>(Jb.scale)) + (long long)(Jb.smul * m + Jb.soff) * Jb.sstride +
                               (long long)c * Jb.scl
                         : nullptr;
  const int rows = Jb.rows, n = rows * Jb.cols, e0 = chunk * kCopyChunk + (int)threadIdx.x;
  const T alpha = (T)Jb.alpha;
  if (Jb.vec) {
    // 16-byte accesses (the launcher checked that rows, leading dimensions
    // and operand offsets are multiples of V elements); the same products
    // element by element
    constexpr int V = 16 / sizeof(T);
    typedef T VT __attribute__((ext_vector_type(V)));
    constexpr int PV = PER / V;
    const int rv = rows / V, nv = n / V, v0 = chunk * (kCopyChunk / V) + (int)threadIdx.x;
    VT w[PV];
    int r4[PV], q4[PV];
#pragma unroll
    for (int u = 0; u < PV; ++u) {
      const int e = v0 + u * 256;
      r4[u] = (e % rv) * V;
      q4[u] = e / rv;
      if (e < nv) w[u] = *reinterpret_cast<const VT*>(sp + r4[u] + (long long)q4[u] * src.ld);
    }
#pragma unroll
    for (int u = 0; u < PV; ++u) {
      if (v0 + u * 256 >= nv) break;
      T* d = dp + r4[u] + (long long)q4[u] * dst.ld;
      VT o;
#pragma unroll
      for (int h = 0; h < V; ++h) {
        T y = alpha * w[u][h];
        if (sc) y *= sc[Jb.sside ? q4[u] : r4[u] + h];
        o[h] = Jb.accumulate ? d[h] + y : y;
      }
      *reinterpret_cast<VT*>(d) = o;
    }
    return;
  }
  T v[PER];
  int rr[PER], qq[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = e0 + u * 256;
    rr[u] = e % rows;
    qq[u] = e / rows;
    v[u] = e < n ? alpha * sp[rr[u] + (long long)qq[u] * src.ld] : T(0);
  }
  if (sc)
#pragma unroll
    for (int u = 0; u < PER; ++u)
      if (e0 + u * 256 < n) v[u] *= sc[Jb.sside ? qq[u] : rr[u]];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    if (e0 + u * 256 >= n) break;
    T* d = dp + rr[u] + (long long)qq[u] * dst.ld;
    *d = Jb.accumulate ? *d + v[u] : v[u];
  }
}

template <typename T>
__global__ void k_fill(T* p, size_t n, T v) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    p[e] = v;
}

// Zero fill of up to kZeroBatch byte ranges (blockIdx.y = range): 16-byte
// stores on the aligned body, single bytes on the unaligned head and tail.
__global__ __launch_bounds__(256) void k_zero_bytes(ZeroArgs z) {
  const int f = blockIdx.y;
  unsigned char* p = z.p[f];
  const unsigned long long bytes = z.n[f];
  const unsigned long long a = reinterpret_cast<uintptr_t>(p);
  unsigned long long head = (16 - (a & 15)) & 15;
  if (head > bytes) head = bytes;
  const unsigned long long nbody = (bytes - head) / 16;
  const unsigned long long tail = bytes - head - 16 * nbody;
  const unsigned long long t = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x;
  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
  uint4* body = reinterpret_cast<uint4*>(p + head);
  for (unsigned long long e = t; e < nbody; e += stride) body[e] = make_uint4(0u, 0u, 0u, 0u);
  if (t < head) p[t] = 0;
  if (t < tail) p[head + 16 * nbody + t] = 0;
}

// Level-0 leaves: the tridiagonal band of each leaf of D_i (`per` workgroups
// per matrix).
template <typename T>
__global__ __launch_bounds__(256) void k_leaves_tridiag(const OpJob* __restrict__ jobs, int njobs) {
  const OpJob& J = jobs[job_of(jobs, njobs, blockIdx.x)];
  const long long local = blockIdx.x - J.block0;
  const int m = (int)(local / J.per), part = (int)(local % J.per);
  const int s = J.s, b = J.b;
  const int blk = J.bmul * m + J.boff;
  const long long n = (long long)s * b;   // 2^L leaves of b x b
  T* lv = gmem(static_cast<T*>(J.out)) + (size_t)m * n;
  const double* dg = gmem(J.diag) + (size_t)blk * s;
  const double* we = gmem(J.west) + (size_t)blk * s;
  const double* ea = gmem(J.east) + (size_t)blk * s;
  for (long long e = (long long)part * 256 + threadIdx.x; e < n; e += (long long)J.per * 256) {
    const int lam = (int)(e / ((long long)b * b));
    const int rem = (int)(e % ((long long)b * b));
    const int r = rem % b, c = rem / b;
    const int gr = lam * b + r;
    const int pnx = J.pnx;
    double v = 0.0;
    if (c == r) v = dg[gr];
    else if (c == r - 1) v = (pnx == 0 || gr % pnx != 0) ? we[gr] : 0.0;
    else if (c == r + 1) v = (pnx == 0 || (gr + 1) % pnx != 0) ? ea[gr] : 0.0;
    else if (pnx > 0 && c == r - pnx) v = gmem(J.south)[(size_t)blk * s + gr];
    else if (pnx > 0 && c == r + pnx) v = gmem(J.north)[(size_t)blk * s + gr];
    lv[e] = (T)v;
  }
}

// Off-diagonal factors of a plane operator (see gplane_factors).  At depth d
// with children of sd unknowns, rank pnx: column q of the first child's U is
// north at its row sd - pnx + q, of the second child's U south at its row q,
// and V holds 1 at the same rows; rank 1: east at the first child's last row,
// west at the second child's first row.  Every entry of U[d] and V[d] is
// written (zeros elsewhere).
template <typename T>
__global__ __launch_bounds__(256) void k_plane_factors(const OpJob* __restrict__ jobs, int njobs) {
  const OpJob& J = jobs[job_of(jobs, njobs, blockIdx.x)];
  const long long local = blockIdx.x - J.block0;
  const int m = (int)(local / J.per), part = (int)(local % J.per);
  const int s = J.s, pnx = J.pnx;
  const int blk = J.bmul * m + J.boff;
  const size_t off = (size_t)blk * s;
  for (int r = part * 256 + threadIdx.x; r < s; r += J.per * 256) {
    for (int d = 1; d <= J.L; ++d) {
      const int sd = s >> d, cl = r / sd, loc = r % sd;
      const int k = sd % pnx == 0 ? pnx : 1;
      int q = -1;
      double u = 0.0;
      if (k == 1) {
        if ((cl & 1) == 0 && loc == sd - 1) { q = 0; u = gmem(J.east)[off + r]; }
        if ((cl & 1) == 1 && loc == 0) { q = 0; u = gmem(J.west)[off + r]; }
      } else {
        if ((cl & 1) == 0 && loc >= sd - pnx) { q = loc - (sd - pnx); u = gmem(J.north)[off + r]; }
        if ((cl & 1) == 1 && loc < pnx) { q = loc; u = gmem(J.south)[off + r]; }
      }
      T* U = gmem(static_cast<T*>(J.U[d])) + (size_t)m * k * s + r;
      T* V = gmem(static_cast<T*>(J.V[d])) + (size_t)m * k * s + r;
      for (int c = 0; c < k; ++c) {
        U[(size_t)c * s] = c == q ? (T)u : T(0);
        V[(size_t)c * s] = c == q ? T(1) : T(0);
      }
    }
  }
}

// Inverse of a tridiagonal block in HODLR form.  With the pivots of the two
// eliminations without pivoting, d_i (top down) and e_i (bottom up), the
// inverse has diagonal g_i = 1 / (d_i + e_i - a_i), and every column z of it
// satisfies z_i = rho_i z_(i+1) above its diagonal (rho_i = -b_i / d_i) and
// z_i = tau_i z_(i-1) below (tau_i = -c_i / e_i).  Hence the leaves follow by
// walking up and down each column from g_j, and the off-diagonal block of
// clusters t (rows) and s (columns) is exactly rank one: for t above s,
// U_t[i] = prod_(k=i..t1-1) rho_k and V_t[j] = g_j prod_(k=t1..j-1) rho_k
// (t1 the first row of s); for t below s, U_t[i] = prod_(k=t0..i) tau_k and
// V_t[j] = g_j prod_(k=j+1..t0-1) tau_k (t0 the first row of t).  All in FP64.
template <typename T>
__global__ __launch_bounds__(256) void k_tridiag_inverse(const OpJob* __restrict__ jobs, int njobs) {
  const OpJob& J = jobs[job_of(jobs, njobs, blockIdx.x)];
  const int s = J.s, b = J.b, L = J.L, bmul = J.bmul, boff = J.boff;
  const double* __restrict__ diag = gmem(J.diag);
  const double* __restrict__ west = gmem(J.west);
  const double* __restrict__ east = gmem(J.east);
  T* __restrict__ lv = gmem(static_cast<T*>(J.out));
  int* const fallback = gmem(J.flag);
  extern __shared__ unsigned char smem_raw[];
  double* A = reinterpret_cast<double*>(smem_raw);   // a_i, then g_i
  double* B = A + s;                                  // b_i, then rho_i
  double* C = B + s;                                  // c_i, then tau_i
  double* Dp = C + s;                                 // d_i
  double* Ep = Dp + s;                                // e_i
  __shared__ int bad;
  const int m = (int)(blockIdx.x - J.block0), tid = threadIdx.x;
  const int blk = bmul * m + boff;
  const double* dg = diag + (size_t)blk * s;
  const double* we = west + (size_t)blk * s;
  const double* ea = east + (size_t)blk * s;
  if (tid == 0) bad = 0;
  for (int i = tid; i < s; i += 256) {
    A[i] = dg[i];
    B[i] = i + 1 < s ? ea[i] : 0.0;
    C[i] = i > 0 ? we[i] : 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    double d = A[0];
    Dp[0] = d;
    bool ok = d != 0.0 && isfinite(d);
    for (int i = 1; i < s; ++i) {
      d = A[i] - C[i] * B[i - 1] / d;
      Dp[i] = d;
      ok = ok && d != 0.0 && isfinite(d);
    }
    if (!ok) bad = 1;
  } else if (tid == WAVE) {
    double e = A[s - 1];
    Ep[s - 1] = e;
    bool ok = e != 0.0 && isfinite(e);
    for (int i = s - 2; i >= 0; --i) {
      e = A[i] - B[i] * C[i + 1] / e;
      Ep[i] = e;
      ok = ok && e != 0.0 && isfinite(e);
    }
    if (!ok) bad = 1;
  }
  __syncthreads();
  if (bad) {
    if (tid == 0) fallback[0] = 1;
    return;
  }
  for (int i = tid; i < s; i += 256) {
    const double gi = 1.0 / (Dp[i] + Ep[i] - A[i]);
    const double ri = i + 1 < s ? -B[i] / Dp[i] : 0.0;
    const double ti = i > 0 ? -C[i] / Ep[i] : 0.0;
    A[i] = gi;
    B[i] = ri;
    C[i] = ti;
  }
  __syncthreads();
  // leaves: column j of leaf l from its diagonal up and down
  const int nleaf = 1 << L;
  T* lvm = lv + (size_t)m * nleaf * b * b;
  for (int j = tid; j < s; j += 256) {
    const int l = j / b, j0 = l * b, jl = j - j0;
    T* col = lvm + (size_t)l * b * b + (size_t)jl * b;
    double v = A[j];
    col[jl] = (T)v;
    for (int i = j - 1; i >= j0; --i) {
      v *= B[i];
      col[i - j0] = (T)v;
    }
    v = A[j];
    for (int i = j + 1; i < j0 + b; ++i) {
      v *= C[i];
      col[i - j0] = (T)v;
    }
  }
  // rank-one factors of every depth: four serial passes per sibling pair
  int ntask = 0;
  for (int d = 1; d <= L; ++d) ntask += 4 << (d - 1);
  for (int task = tid; task < ntask; task += 256) {
    int d = 1, t = task;
    while (t >= (4 << (d - 1))) { t -= 4 << (d - 1); ++d; }
    const int pair = t >> 2, kind = t & 3;
    const int sd = s >> d, t0 = 2 * pair * sd, t1 = t0 + sd;
    T* Ud = gmem(static_cast<T*>(J.U[d])) + (size_t)m * s;
    T* Vd = gmem(static_cast<T*>(J.V[d])) + (size_t)m * s;
    if (kind == 0) {          // U of the upper block, rows of the first cluster
      double u = 1.0;
      for (int i = t1 - 1; i >= t0; --i) { u *= B[i]; Ud[i] = (T)u; }
    } else if (kind == 1) {   // its V, rows of the second cluster
      double q = 1.0;
      for (int j = t1; j < t1 + sd; ++j) { Vd[j] = (T)(A[j] * q); q *= B[j]; }
    } else if (kind == 2) {   // U of the lower block, rows of the second cluster
      double u = 1.0;
      for (int i = t1; i < t1 + sd; ++i) { u *= C[i]; Ud[i] = (T)u; }
    } else {                  // its V, rows of the first cluster
      double q = 1.0;
      for (int j = t1 - 1; j >= t0; --j) { Vd[j] = (T)(A[j] * q); q *= C[j]; }
    }
  }
}

// Level-0 off-diagonal factors of D_i at every depth (rank one, Section 3):
// the upper-right block of a first child couples its last row to the
// sibling's first column (value east), the lower-left block of a second
// child couples its first row to the sibling's last column (value west).
template <typename T>
__global__ __launch_bounds__(256) void k_rank1(const OpJob* __restrict__ jobs, int njobs) {
  const OpJob& J = jobs[job_of(jobs, njobs, blockIdx.x)];
  const long long local = blockIdx.x - J.block0;
  const int m = (int)(local / J.per), part = (int)(local % J.per);
  const int s = J.s;
  const int blk = J.bmul * m + J.boff;
  const double* we = gmem(J.west) + (size_t)blk * s;
  const double* ea = gmem(J.east) + (size_t)blk * s;
  for (int r = part * 256 + threadIdx.x; r < s; r += J.per * 256) {
    for (int d = 1; d <= J.L; ++d) {
      const int sd = s >> d, cl = r / sd, loc = r % sd;
      T u = T(0), v = T(0);
      if ((cl & 1) == 0 && loc == sd - 1) { u = (T)ea[r]; v = T(1); }
      if ((cl & 1) == 1 && loc == 0) { u = (T)we[r]; v = T(1); }
      gmem(static_cast<T*>(J.U[d]))[(size_t)m * s + r] = u;
      gmem(static_cast<T*>(J.V[d]))[(size_t)m * s + r] = v;
    }
  }
}

// Diagonal of a stencil array per block row; block row zblk (if >= 0) gets
// zeros (the coupling that would leave the grid).
template <typename T>
__global__ __launch_bounds__(256) void k_gather_diag(const OpJob* __restrict__ jobs, int njobs) {
  const OpJob& J = jobs[job_of(jobs, njobs, blockIdx.x)];
  const long long local = blockIdx.x - J.block0;
  const int m = (int)(local / J.per), part = (int)(local % J.per);
  const int s = J.s;
  const int blk = J.bmul * m + J.boff;
  const double* src = gmem(J.src) + (size_t)blk * s;
  T* dst = gmem(static_cast<T*>(J.out)) + (size_t)m * s;
  for (int r = part * 256 + threadIdx.x; r < s; r += J.per * 256) dst[r] = blk == J.zblk ? T(0) : (T)src[r];
}

template <typename T>
__global__ __launch_bounds__(256) void k_gto_blocks(const VJob* __restrict__ jobs, int njobs) {
  const VJob& J = jobs[job_of(jobs, njobs, blockIdx.x)];
  const long long part = blockIdx.x - J.block0;
  const int s = J.s, nrhs = J.nrhs;
  const long long n = (long long)s * J.nblk * nrhs, ld = J.ld;
  const double* B = gmem(static_cast<const double*>(J.src));
  T* V = gmem(static_cast<T*>(J.dst));
  for (long long e = part * 256 + threadIdx.x; e < n; e += (long long)J.per * 256) {
    const int j = (int)(e % s);
    const long long t = e / s;
    const int q = (int)(t % nrhs);
    const int i = (int)(t / nrhs);
    V[e] = (T)B[(long long)i * s + j + (long long)q * ld];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_gfrom_blocks(const VJob* __restrict__ jobs, int njobs) {
  const VJob& J = jobs[job_of(jobs, njobs, blockIdx.x)];
  const long long part = blockIdx.x - J.block0;
  const int s = J.s, nrhs = J.nrhs;
  const long long n = (long long)s * J.nblk * nrhs, ld = J.ld;
  const T* V = gmem(static_cast<const T*>(J.src));
  double* B = gmem(static_cast<double*>(J.dst));
  for (long long e = part * 256 + threadIdx.x; e < n; e += (long long)J.per * 256) {
    const int j = (int)(e % s);
    const long long t = e / s;
    const int q = (int)(t % nrhs);
    const int i = (int)(t / nrhs);
    B[(long long)i * s + j + (long long)q * ld] = (double)V[e];
  }
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

__global__ void k_residual3d(int nx, int ny, int nz, const double* diag, const double* west,
                             const double* east, const double* south, const double* north,
                             const double* down, const double* up, const double* X, const double* B,
                             double* R) {
  const long long P = (long long)nx * ny, N = P * nz;
  const int q = blockIdx.y;
  const double* x = X + q * N;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < N;
       e += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(e % nx);
    const int i = (int)((e / nx) % ny);
    const long long k = e / P;
    double ax = diag[e] * x[e];
    if (j > 0) ax += west[e] * x[e - 1];
    if (j + 1 < nx) ax += east[e] * x[e + 1];
    if (i > 0) ax += south[e] * x[e - nx];
    if (i + 1 < ny) ax += north[e] * x[e + nx];
    if (k > 0) ax += down[e] * x[e - P];
    if (k + 1 < nz) ax += up[e] * x[e + P];
    R[e + q * N] = B[e + q * N] - ax;
  }
}

// Full-rank HODLR form of a dense block (see HJob): `per` workgroups per
// matrix walk the s*s entries; entry (r, c) goes to the leaf of r when r and
// c share it, else to U of the depth-d cluster of r (column c - sib start),
// and every depth's V gets the identity on the sibling rows.
template <typename T>
__global__ __launch_bounds__(256) void k_dense_to_hodlr(const HJob* __restrict__ jobs, int njobs) {
  const HJob& J = jobs[job_of(jobs, njobs, blockIdx.x)];
  const long long local = blockIdx.x - J.block0;
  const int m = (int)(local / J.per), part = (int)(local % J.per);
  const int s = J.s, b = J.b, L = J.L;
  const double* A = gmem(J.A) + (size_t)m * s * s;
  const long long n = (long long)s * s;
  for (long long e = (long long)part * 256 + threadIdx.x; e < n; e += (long long)J.per * 256) {
    const int r = (int)(e % s), c = (int)(e / s);
    const double a = m == J.zm ? 0.0 : A[e];
    if (r / b == c / b) {
      const int l = r / b;
      gmem(static_cast<T*>(J.lv))[((size_t)m * (s / b) + l) * b * b + (r - l * b) + (size_t)(c - l * b) * b] = (T)a;
    } else {
      int d = 1;   // first depth at which the clusters of r and c differ
      while (d < L && r / (s >> d) == c / (s >> d)) ++d;
      const int sd = s >> d, q = c % sd;   // column q of U_tau, tau = cluster of r
      gmem(static_cast<T*>(J.U[d]))[(size_t)m * sd * s + (size_t)q * s + r] = (T)a;
    }
    // V_tau = I on the rows of sib(tau): for every depth, V[d] column q at row c is
    // 1 when q == c mod sd (each (c, d, q) written once: by the entry with r == 0)
    if (r == 0) {
      for (int d = 1; d <= L; ++d) {
        const int sd = s >> d;
        T* V = gmem(static_cast<T*>(J.V[d])) + (size_t)m * sd * s;
        for (int q = 0; q < sd; ++q) V[(size_t)q * s + c] = q == c % sd ? T(1) : T(0);
      }
    }
  }
}

// Dense s x s block from a HODLR matrix (or a diagonal): entry (r, c) lies in
// the leaf of r when r and c share it, else in the off-diagonal block of the
// first depth d at which their clusters differ: sum_q U_d[q][r] V_d[q][c].
template <typename T>
__global__ __launch_bounds__(256) void k_dense_blocks(const DenseJob* __restrict__ jobs, int njobs) {
  const DenseJob& J = jobs[job_of(jobs, njobs, blockIdx.x)];
  const long long part = blockIdx.x - J.block0;
  const int s = J.s, b = J.b, L = J.L;
  const long long n = (long long)s * s;
  double* out = gmem(J.out);
  for (long long e = part * 256 + threadIdx.x; e < n; e += (long long)J.per * 256) {
    const int r = (int)(e % s), c = (int)(e / s);
    double v = 0.0;
    if (J.type == 1) {
      if (r == c) v = (double)gmem(static_cast<const T*>(J.lv))[(long long)J.midx * s + r];
    } else if (r / b == c / b) {
      const int l = r / b;
      v = (double)gmem(static_cast<const T*>(J.lv))[((long long)J.midx * (s / b) + l) * b * b + (r - l * b) +
                                                     (long long)(c - l * b) * b];
    } else {
      int d = 1;   // r and c lie in different leaves, so their clusters differ at some d <= L
      while (d < L && r / (s >> d) == c / (s >> d)) ++d;
      const T* U = gmem(static_cast<const T*>(J.U[d])) + (long long)J.midx * J.k[d] * s;
      const T* V = gmem(static_cast<const T*>(J.V[d])) + (long long)J.midx * J.k[d] * s;
      for (int q = 0; q < J.kc[d]; ++q) v += (double)U[r + (long long)q * s] * (double)V[c + (long long)q * s];
    }
    out[r + (long long)c * J.ld] = v;
  }
}

// Grouped refinement vector kernels (several problems per launch).  A job's
// workgroups are (column q, part): q = local / per, part = local % per.
__global__ __launch_bounds__(256) void k_gresidual(const RJob* __restrict__ jobs, int njobs) {
  const RJob& J = jobs[job_of(jobs, njobs, blockIdx.x)];
  const long long local = blockIdx.x - J.block0;
  const int q = (int)(local / J.per), part = (int)(local % J.per);
  const int nx = J.nx, ny = J.ny;
  const long long N = (long long)nx * ny;
  const double* diag = gmem(J.diag);
  const double* west = gmem(J.west);
  const double* east = gmem(J.east);
  const double* south = gmem(J.south);
  const double* north = gmem(J.north);
  const double* x = gmem(J.X) + q * N;
  const double* b = gmem(J.B) + q * N;
  double* r = gmem(J.R) + q * N;
  for (long long e = (long long)part * 256 + threadIdx.x; e < N; e += (long long)J.per * 256) {
    const int j = (int)(e % nx);
    const int i = (int)(e / nx);
    double ax = diag[e] * x[e];
    if (j > 0) ax += west[e] * x[e - 1];
    if (j + 1 < nx) ax += east[e] * x[e + 1];
    if (i > 0) ax += south[e] * x[e - nx];
    if (i + 1 < ny) ax += north[e] * x[e + nx];
    r[e] = b[e] - ax;
  }
}

// Partial sums of squares of column q of job J.R over fixed chunks (the
// chunking depends on N only), then the sum of the parts in order.
__global__ __launch_bounds__(256) void k_gsumsq_part(const RJob* __restrict__ jobs, int njobs) {
  __shared__ double red[4];
  const RJob& J = jobs[job_of(jobs, njobs, blockIdx.x)];
  const long long local = blockIdx.x - J.block0;
  const int q = (int)(local / J.per), part = (int)(local % J.per);
  const long long N = (long long)J.nx * J.ny;
  const long long chunk = (N + J.per - 1) / J.per;
  const long long lo = part * chunk, hi = min(N, lo + chunk);
  const double* a = gmem(J.R) + q * N;
  double s = 0.0;
  for (long long i = lo + threadIdx.x; i < hi; i += 256) s += a[i] * a[i];
  s = block_sum256(s, red);
  if (threadIdx.x == 0) gmem(J.part)[(size_t)q * J.per + part] = s;
}

__global__ __launch_bounds__(256) void k_gsumsq_final(const RJob* __restrict__ jobs, int njobs) {
  __shared__ double red[4];
  const RJob& J = jobs[job_of(jobs, njobs, blockIdx.x)];
  const int q = (int)(blockIdx.x - J.block0);
  double s = 0.0;
  for (int i = threadIdx.x; i < J.per; i += 256) s += gmem(J.part)[(size_t)q * J.per + i];
  s = block_sum256(s, red);
  if (threadIdx.x == 0) gmem(J.out)[q] = s;
}

// X += D (job.B = D, job.R = X).
__global__ __launch_bounds__(256) void k_gaxpy(const RJob* __restrict__ jobs, int njobs) {
  const RJob& J = jobs[job_of(jobs, njobs, blockIdx.x)];
  const long long local = blockIdx.x - J.block0;
  const int q = (int)(local / J.per), part = (int)(local % J.per);
  const long long N = (long long)J.nx * J.ny;
  const double* d = gmem(J.B) + q * N;
  double* x = gmem(J.R) + q * N;
  for (long long e = (long long)part * 256 + threadIdx.x; e < N; e += (long long)J.per * 256) x[e] += d[e];
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

// Krylov vectors (FP64): partial dot products of nvec vectors V_i (stride
// ldv) with w, then a fixed-order sum of the parts (deterministic).
__global__ void k_mdot_part(long long n, long long chunk, const double* __restrict__ V, long long ldv,
                            const double* __restrict__ w, double* __restrict__ part) {
  __shared__ double red[4];
  const int i = blockIdx.y;
  const long long lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
  const double* v = V + (long long)i * ldv;
  double s = 0.0;
  for (long long e = lo + threadIdx.x; e < hi; e += 256) s = fma(v[e], w[e], s);
  s = block_sum256(s, red);
  if (threadIdx.x == 0) part[(size_t)i * gridDim.x + blockIdx.x] = s;
}

// w = a w + sc * sum_i c_i V_i (the nvec coefficients c on the device).
__global__ void k_maxpy(long long n, int nvec, double a, double sc, const double* __restrict__ c,
                        const double* __restrict__ V, long long ldv, double* __restrict__ w) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int i = 0; i < nvec; ++i) acc = fma(c[i], V[(long long)i * ldv + e], acc);
    w[e] = fma(a, w[e], sc * acc);
  }
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

__global__ __launch_bounds__(256) void k_count_nonfinite(const NFJob* __restrict__ jobs, int njobs) {
  const NFJob& J = jobs[job_of(jobs, njobs, blockIdx.x)];
  const long long part = blockIdx.x - J.block0;
  const double* a = gmem(J.a);
  int bad = 0;
  for (long long e = part * 256 + threadIdx.x; e < J.n; e += (long long)J.per * 256) bad |= !isfinite(a[e]);
  if (bad) gmem(J.flag)[0] = 1;
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
namespace {

struct TileCfg { int tm, tn; double eff; };
constexpr TileCfg kTiles[5] = {{64, 64, 1.0}, {64, 16, 0.8}, {16, 64, 0.8}, {32, 32, 0.8}, {16, 16, 0.55}};

int pick_tile(int M, int N) {
  int best = 0;
  double bc = 1e300;
  for (int i = 0; i < 5; ++i) {
    const double pm = (double)((M + kTiles[i].tm - 1) / kTiles[i].tm) * kTiles[i].tm;
    const double pn = (double)((N + kTiles[i].tn - 1) / kTiles[i].tn) * kTiles[i].tn;
    const double cost = pm * pn / kTiles[i].eff;
    if (cost < bc) { bc = cost; best = i; }
  }
  return best;
}

// Let a kernel use more than 64 KB of dynamic LDS (once per kernel).
void allow_large_lds(const void* kern, size_t dyn = kMaxDynLarge) {
  static std::vector<const void*> done;
  if (std::find(done.begin(), done.end(), kern) != done.end()) return;
  ACR_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
  done.push_back(kern);
}

// Kernel names as the profiler reports them ("k_gqr<float>"): the template
// arguments spelled in the source are replaced by the instantiated types.
template <typename X> const char* type_name();
template <> const char* type_name<float>() { return "float"; }
template <> const char* type_name<double>() { return "double"; }

const char* kernel_name(const char* src, const char* t, const char* tin, const char* tout) {
  static std::mutex mu;
  static std::set<std::string> pool;
  std::string out;
  const std::string in(src);
  for (size_t i = 0; i < in.size();) {
    if (std::isalpha((unsigned char)in[i]) || in[i] == '_') {
      size_t j = i;
      while (j < in.size() && (std::isalnum((unsigned char)in[j]) || in[j] == '_')) ++j;
      const std::string w = in.substr(i, j - i);
      out += w == "T" ? t : w == "Tin" ? tin : w == "Tout" ? tout : w;
      i = j;
    } else {
      out += in[i++];
    }
  }
  std::lock_guard<std::mutex> g(mu);
  return pool.insert(out).first->c_str();
}

// Each use site resolves its name once (a static of the instantiation):
// launches no longer build the name string every time.
#define KNAME_T(...) ([]() { static const char* const n_ = kernel_name(#__VA_ARGS__, type_name<T>(), "", ""); return n_; }())
#define KNAME_IO(...) \
  ([]() { static const char* const n_ = kernel_name(#__VA_ARGS__, "", type_name<Tin>(), type_name<Tout>()); return n_; }())
#define KNAME0(...) ([]() { static const char* const n_ = kernel_name(#__VA_ARGS__, "", "", ""); return n_; }())

template <typename J>
const J* upload(const std::vector<J>& v, hipStream_t st) {
  return static_cast<const J*>(desc_put(v.data(), v.size() * sizeof(J), st));
}

}  // namespace

// ------------------------------------------------------------- autotuner
// Choices of kernel variant per shape key, measured on the device (see
// tune_run) and kept in a table that can be saved and loaded as JSON for one
// GPU architecture.  Keys hold shapes only, never anything about the other
// problems of a call, so a problem's result does not depend on what it is
// batched with:
//   "gemm.<f|d>.<M>.<N>.<Kbits>.<Pbits>"  tile shape of the grouped GEMM:
//       kind 0..4 = k_ggemm's five tiles on the vector units, 10..14 (FP32
//       only) = the same tiles on the matrix cores (k_ggemm_mfma).  Within
//       each engine the tiles give the same bits (every output sums its K
//       terms in the same order whatever the tile); the two engines round
//       differently (one FMA per term against four products per MFMA);
//   "qr.<f|d>.<p>.<k>"  Householder QR form of a p x k panel: 4 one wave,
//       2 registers of four waves, 0 LDS (the forms give different bits).
Tuner& Tuner::get() {
  static Tuner t;
  return t;
}

int Tuner::lookup(const std::string& key) {
  if (!active) return -1;
  std::lock_guard<std::mutex> g(mu);
  auto it = table.find(key);
  return it == table.end() ? -1 : it->second;
}

void Tuner::note(const std::string& key, long long nprob) {
  if (!recording) return;
  std::lock_guard<std::mutex> g(mu);
  long long& v = seen[key];
  v = std::max(v, nprob);
}

namespace {
int bits(long long v) {
  int b = 0;
  while (v > 0) { ++b; v >>= 1; }
  return b;
}
template <typename T> char tchar() { return sizeof(T) == 4 ? 'f' : 'd'; }
}  // namespace

// Workgroups of a grouped GEMM job: one per output tile, except for the row
// kernel (kinds 6..8), whose workgroups take four 64-row tiles.
long long gjob_blocks(const GJob& J) {
  const long long t = (long long)J.nmat * J.ncl * J.tilesM * J.tilesN;
  return J.kind >= 6 && J.kind <= 8 ? (t + 3) / 4 : t;
}

// Kernel kinds of the grouped GEMM: 0..4 = tile shapes of k_ggemm,
// 5 = k_gemm_dot (long-K reductions A^T B with small outputs), 6..8 =
// k_gemm_rows with 16 / 32 / 4 columns, 9 = k_gemm_small (short-K reductions),
// 10..14 = the tiles of 0..4 on the matrix cores (FP32, chosen by the tuner
// only: on the shapes of the factorisation the vector tiles are faster).
template <typename T>
void ggemm(hipStream_t st, std::vector<GJob> jobs, const std::vector<GSeg>& segs, int force_tile) {
  constexpr int NK = 15;
  Tuner& tuner = Tuner::get();
  std::vector<GJob> by[NK];
  double fl[NK] = {}, bytes[NK] = {};
  for (auto& J : jobs) {
    if (J.M <= 0 || J.N <= 0 || J.nmat <= 0 || J.ncl <= 0 || J.nseg <= 0) continue;
    double K = 0;
    bool dotok = true, rowok = true;
    for (int sg = 0; sg < J.nseg; ++sg) {
      const GSeg& g = segs[J.seg0 + sg];
      K += g.K;
      if (!(g.A.trans && !g.B.trans)) dotok = false;
      if (g.B.trans) rowok = false;
    }
    int kind;
    if (dotok && J.M <= 64 && J.N <= 64 && K >= 256) {
      kind = 5;
      J.tilesM = (J.M + 7) / 8;
      J.tilesN = (J.N + 7) / 8;
    } else if (dotok && J.M <= 64 && J.N <= 64) {
      kind = 9;
      J.tilesM = (J.M + 15) / 16;
      J.tilesN = (J.N + 15) / 16;
    } else if (rowok && J.M >= 48 && J.N <= (sizeof(T) == 4 ? 32 : 16)) {
      kind = J.N <= 4 ? 8 : J.N <= 16 ? 6 : 7;
      J.tilesM = (J.M + 63) / 64;
      J.tilesN = 1;
    } else {
      kind = pick_tile(J.M, J.N);
      if (force_tile >= 0) {
        kind = force_tile;
      } else if (tuner.active || tuner.recording) {
        const long long npr = (long long)J.nmat * J.ncl;
        char key[96];
        std::snprintf(key, sizeof key, "gemm.%c.%d.%d.%d.%d", tchar<T>(), J.M, J.N, bits((long long)K), bits(npr));
        tuner.note(key, npr);
        const int c = tuner.lookup(key);
        if ((c >= 0 && c <= 4) || (sizeof(T) == 4 && c >= 10 && c <= 14)) kind = c;
      }
      if (kind >= 10 && sizeof(T) != 4) kind -= 10;
      J.tilesM = (J.M + kTiles[kind % 10].tm - 1) / kTiles[kind % 10].tm;
      J.tilesN = (J.N + kTiles[kind % 10].tn - 1) / kTiles[kind % 10].tn;
    }
    const double np = (double)J.nmat * J.ncl;
    fl[kind] += 2.0 * J.M * J.N * K * np;
    bytes[kind] += sizeof(T) * np * ((double)J.M * K + K * J.N + (double)J.M * J.N * (J.beta != 0.0 ? 2 : 1));
    J.kind = kind;
    {
      static const char* names[15][2] = {
          {"gemm.tile64x64", "gemm.tile64x64.M>128"}, {"gemm.tile64x16", "gemm.tile64x16.M>128"},
          {"gemm.tile16x64", "gemm.tile16x64.M>128"}, {"gemm.tile32x32", "gemm.tile32x32.M>128"},
          {"gemm.tile16x16", "gemm.tile16x16.M>128"}, {"gemm.dot", "gemm.dot.K>128"},
          {"gemm.rows16", "gemm.rows16.M>128"}, {"gemm.rows32", "gemm.rows32.M>128"},
          {"gemm.rows4", "gemm.rows4.M>128"}, {"gemm.small", "gemm.small.K>128"},
          {"gemm.mfma64x64", "gemm.mfma64x64.M>128"}, {"gemm.mfma64x16", "gemm.mfma64x16.M>128"},
          {"gemm.mfma16x64", "gemm.mfma16x64.M>128"}, {"gemm.mfma32x32", "gemm.mfma32x32.M>128"},
          {"gemm.mfma16x16", "gemm.mfma16x16.M>128"}};
      const bool big = (kind == 5 || kind == 9) ? K > 128 : J.M > 128;
      Profiler::get().hit(names[kind][big ? 1 : 0], (long long)np);
    }
    by[kind].push_back(J);
  }
  // A small call (few workgroups in all) runs as one launch of k_gemm_any,
  // with the narrow tile shapes widened to 64 x 64.
  {
    int kinds = 0;
    long long total = 0;
    for (int kd = 0; kd < NK; ++kd) {
      if (by[kd].empty()) continue;
      ++kinds;
      for (const auto& J : by[kd]) {
        total += (kd >= 1 && kd <= 4) || kd >= 11
                     ? (long long)J.nmat * J.ncl * ((J.M + 63) / 64) * ((J.N + 63) / 64)
                     : gjob_blocks(J);
      }
    }
    if (kinds > 1 && total <= kSmallLaunch && force_tile < 0) {
      std::vector<char> blob(segs.size() * sizeof(GSeg));
      if (!segs.empty()) std::memcpy(blob.data(), segs.data(), blob.size());
      std::vector<GJob> all;
      double f = 0, by_ = 0;
      long long b0 = 0;
      for (int kd = 0; kd < NK; ++kd) {
        f += fl[kd];
        by_ += bytes[kd];
        for (auto J : by[kd]) {
          if ((kd >= 1 && kd <= 4) || kd >= 11) {   // widened to the 64 x 64 tile of its engine
            J.kind = kd >= 11 ? 10 : 0;
            J.tilesM = (J.M + 63) / 64;
            J.tilesN = (J.N + 63) / 64;
          }
          J.block0 = b0;
          b0 += gjob_blocks(J);
          all.push_back(J);
        }
      }
      const size_t o = (blob.size() + 255) & ~size_t(255);
      blob.resize(o + all.size() * sizeof(GJob));
      std::memcpy(blob.data() + o, all.data(), all.size() * sizeof(GJob));
      char* dev = static_cast<char*>(desc_put(blob.data(), blob.size(), st));
      launch(st, KC_GEMM, f, by_, KNAME_T(k_gemm_any<T>), k_gemm_any<T>, dim3((unsigned)b0), dim3(256), 0,
             reinterpret_cast<const GJob*>(dev + o), (int)all.size(), reinterpret_cast<const GSeg*>(dev));
      return;
    }
  }
  // one upload: segments, then the job lists of every kind
  std::vector<char> blob(segs.size() * sizeof(GSeg));
  if (!segs.empty()) std::memcpy(blob.data(), segs.data(), blob.size());
  size_t off[NK];
  long long nblk[NK] = {};
  for (int kd = 0; kd < NK; ++kd) {
    long long b0 = 0;
    for (auto& J : by[kd]) {
      J.block0 = b0;
      b0 += gjob_blocks(J);
    }
    if (b0 > 0x7fffffffLL) fail(ACR_ERR_INVALID_ARG, "grouped GEMM grid too large");
    nblk[kd] = b0;
    off[kd] = (blob.size() + 255) & ~size_t(255);
    blob.resize(off[kd] + by[kd].size() * sizeof(GJob));
    if (!by[kd].empty()) std::memcpy(blob.data() + off[kd], by[kd].data(), by[kd].size() * sizeof(GJob));
  }
  if (blob.empty()) return;
  char* dev = static_cast<char*>(desc_put(blob.data(), blob.size(), st));
  const GSeg* dsegs = reinterpret_cast<const GSeg*>(dev);
  for (int kd = 0; kd < NK; ++kd) {
    if (by[kd].empty()) continue;
    const GJob* dj = reinterpret_cast<const GJob*>(dev + off[kd]);
    const int nj = (int)by[kd].size();
    const dim3 grid((unsigned)nblk[kd]);
    auto go = [&](const char* name, auto kern, int threads) {
      launch(st, KC_GEMM, fl[kd], bytes[kd], name, kern, grid, dim3(threads), 0, dj, nj, dsegs);
    };
    if (kd >= 10) {   // FP32 tiles on the matrix cores
      switch (kd) {
        case 10: go(KNAME0(k_ggemm_mfma<64, 64, 2, 2, 16>), k_ggemm_mfma<64, 64, 2, 2, 16>, 256); break;
        case 11: go(KNAME0(k_ggemm_mfma<64, 16, 1, 1, 16>), k_ggemm_mfma<64, 16, 1, 1, 16>, 64); break;
        case 12: go(KNAME0(k_ggemm_mfma<16, 64, 1, 1, 16>), k_ggemm_mfma<16, 64, 1, 1, 16>, 64); break;
        case 13: go(KNAME0(k_ggemm_mfma<32, 32, 1, 1, 16>), k_ggemm_mfma<32, 32, 1, 1, 16>, 64); break;
        default: go(KNAME0(k_ggemm_mfma<16, 16, 1, 1, 16>), k_ggemm_mfma<16, 16, 1, 1, 16>, 64); break;
      }
      continue;
    }
    switch (kd) {
      case 0: go(KNAME_T(k_ggemm<T, 64, 64, 16, 4, 4>), k_ggemm<T, 64, 64, 16, 4, 4>, 256); break;
      case 1: go(KNAME_T(k_ggemm<T, 64, 16, 16, 4, 4>), k_ggemm<T, 64, 16, 16, 4, 4>, 64); break;
      case 2: go(KNAME_T(k_ggemm<T, 16, 64, 16, 4, 4>), k_ggemm<T, 16, 64, 16, 4, 4>, 64); break;
      case 3: go(KNAME_T(k_ggemm<T, 32, 32, 16, 4, 4>), k_ggemm<T, 32, 32, 16, 4, 4>, 64); break;
      case 4: go(KNAME_T(k_ggemm<T, 16, 16, 16, 2, 2>), k_ggemm<T, 16, 16, 16, 2, 2>, 64); break;
      case 5: go(KNAME_T(k_gemm_dot<T>), k_gemm_dot<T>, 256); break;
      case 6: go(KNAME_T(k_gemm_rows<T, 16>), k_gemm_rows<T, 16>, 256); break;
      case 7: go(sizeof(T) == 4 ? KNAME_T(k_gemm_rows<T, 32>) : KNAME_T(k_gemm_rows<T, 16>), k_gemm_rows<T, sizeof(T) == 4 ? 32 : 16>, 256); break;
      case 8: go(KNAME_T(k_gemm_rows<T, 4>), k_gemm_rows<T, 4>, 256); break;
      default: go(KNAME_T(k_gemm_small<T>), k_gemm_small<T>, 256); break;
    }
  }
}

template <typename T>
void bgemm(hipStream_t st, int M, int N, int K, int nmat, int ncl, T alpha, const BOp& A,
           const BOp& B, T beta, const BOp& C) {
  if (M <= 0 || N <= 0 || nmat <= 0 || ncl <= 0) return;
  std::vector<GSeg> segs(1);
  segs[0].A = A; segs[0].B = B; segs[0].K = K;
  std::vector<GJob> jobs(1);
  GJob& J = jobs[0];
  J.M = M; J.N = N; J.nmat = nmat; J.ncl = ncl; J.seg0 = 0; J.nseg = 1;
  J.alpha = (double)alpha; J.beta = (double)beta; J.C = C;
  ggemm<T>(st, std::move(jobs), segs);
}

// Small dense inverses, grouped: jobs of one size class share a launch (one
// row per lane and 64/N matrices per wave for n <= 64; one workgroup per
// matrix in LDS for n <= 88; the augmented form, in LDS or global scratch,
// above).  The kernel of a matrix depends on its size n only.
template <typename Tin, typename Tout>
void ginverse(hipStream_t st, std::vector<IJob> jobs) {
  std::vector<IJob> use[6];
  long long b0[6] = {};
  double fl[6] = {}, by[6] = {};
  size_t dyn[6] = {};
  std::vector<DBuf<double>> ws;
  for (auto J : jobs) {
    const int n = J.n;
    if (n <= 0 || J.nprob <= 0) continue;
    int g;
    long long nb = J.nprob;
    if (n <= 64) {
      const int Nt = n <= 8 ? 8 : n <= 16 ? 16 : n <= 32 ? 32 : 64;
      g = Nt == 8 ? 0 : Nt == 16 ? 1 : Nt == 32 ? 2 : 3;
      const long long per = 4LL * (WAVE / Nt);
      nb = (J.nprob + per - 1) / per;
    } else if (n <= 88) {
      g = 4;
      dyn[4] = std::max(dyn[4], (size_t)n * n * sizeof(double));
    } else {
      g = 5;
      const size_t lds = (size_t)n * 2 * n * sizeof(double);
      J.use_lds = lds + 2048 <= kMaxLds ? 1 : 0;
      if (!J.use_lds || n > 128) {
        ws.emplace_back((size_t)J.nprob * n * (2 * n + 1));
        J.ws = ws.back().get();
      }
      if (J.use_lds) dyn[5] = std::max(dyn[5], lds);
    }
    J.block0 = b0[g];
    b0[g] += nb;
    fl[g] += 2.0 * n * n * n * J.nprob;
    by[g] += 2.0 * n * n * J.nprob * sizeof(Tin);
    use[g].push_back(J);
  }
  for (int g = 0; g < 6; ++g) {
    if (use[g].empty()) continue;
    const IJob* dj = upload(use[g], st);
    const int nj = (int)use[g].size();
    const dim3 grid((unsigned)b0[g]);
    switch (g) {
      case 0: launch(st, KC_INVERSE, fl[g], by[g], KNAME_IO(k_inverse_wave<Tin, Tout, 8>), k_inverse_wave<Tin, Tout, 8>, grid, dim3(256), 0, dj, nj); break;
      case 1: launch(st, KC_INVERSE, fl[g], by[g], KNAME_IO(k_inverse_wave<Tin, Tout, 16>), k_inverse_wave<Tin, Tout, 16>, grid, dim3(256), 0, dj, nj); break;
      case 2: launch(st, KC_INVERSE, fl[g], by[g], KNAME_IO(k_inverse_wave<Tin, Tout, 32>), k_inverse_wave<Tin, Tout, 32>, grid, dim3(256), 0, dj, nj); break;
      case 3: launch(st, KC_INVERSE, fl[g], by[g], KNAME_IO(k_inverse_wave<Tin, Tout, 64>), k_inverse_wave<Tin, Tout, 64>, grid, dim3(256), 0, dj, nj); break;
      case 4: launch(st, KC_INVERSE, fl[g], by[g], KNAME_IO(k_inverse_lds<Tin, Tout>), k_inverse_lds<Tin, Tout>, grid, dim3(256), dyn[g], dj, nj); break;
      default: launch(st, KC_INVERSE, fl[g], by[g], KNAME_IO(k_inverse<Tin, Tout>), k_inverse<Tin, Tout>, grid, dim3(256), dyn[g], dj, nj); break;
    }
  }
}

template <typename Tin, typename Tout>
void binverse(hipStream_t st, int n, int nprob, const Tin* A, long long sA, Tout* X, long long sX,
              int* status) {
  std::vector<IJob> jobs(1);
  IJob& J = jobs[0];
  J.n = n; J.nprob = nprob; J.A = A; J.sA = sA; J.X = X; J.sX = sX; J.status = status;
  ginverse<Tin, Tout>(st, std::move(jobs));
}

template <typename T>
void gqr(hipStream_t st, std::vector<QJob> jobs, int force_form) {
  Tuner& tuner = Tuner::get();
  // Panels that fit 64 KB of LDS share one launch; larger ones (up to the
  // 160 KB a gfx950 workgroup may hold) get a launch of their own, so that
  // the many small panels keep their occupancy; the rest work in global memory.
  // Panels of at most 64 register entries per lane go to k_gqr_wave (one wave
  // each, group 4).
  std::vector<DBuf<T>> scratch;
  std::vector<QJob> use[5];
  size_t dyn[5] = {0, 0, 0, 0, 0};
  double fl[5] = {0, 0, 0, 0, 0}, by[5] = {0, 0, 0, 0, 0};
  long long b0[5] = {0, 0, 0, 0, 0};
  auto wave_code = [](int p, int k) {
    int best = -1;
    for (int c = 0; c < kWaveQrShapes; ++c) {
      const int rpl = wave_qr_rpl(c), cpl = wave_qr_cpl(c);
      if (16 * rpl < p || 4 * cpl < k || rpl * cpl * (int)sizeof(T) > 256) continue;
      if (best < 0 || rpl * cpl < wave_qr_rpl(best) * wave_qr_cpl(best)) best = c;
    }
    return best;
  };
  for (auto& J : jobs) {
    if (J.p <= 0 || J.k <= 0 || J.nmat <= 0 || J.ncl <= 0) continue;
    const size_t np = (size_t)J.nmat * J.ncl;
    const size_t panel = (size_t)J.p * J.k * sizeof(T), vb = (size_t)J.p * sizeof(T);
    int g = 0;
    const int rows = (J.p + WAVE - 1) / WAVE, slots = (J.k + 3) / 4;
    int wc = wave_code(J.p, J.k);
    const bool reg_ok = rows <= 8 && slots <= 16 && rows * slots * sizeof(T) <= 64 * 4;
    const bool lds_ok = panel + vb + 1024 <= kMaxLds;
    {   // a tuned (or forced) form: one wave (4), registers (2) or LDS (0)
      int want = force_form;
      if (want < 0 && (tuner.active || tuner.recording) && (int)(wc >= 0) + (int)reg_ok + (int)lds_ok > 1) {
        char key[64];
        std::snprintf(key, sizeof key, "qr.%c.%d.%d", tchar<T>(), J.p, J.k);
        tuner.note(key, (long long)np);
        want = tuner.lookup(key);
      }
      if (want == 2 && reg_ok) wc = -1;
      else if (want == 0 && lds_ok) wc = -2;
    }
    if (wc == -2) {
      J.lds = 1;   // LDS form (g = 0)
    } else if (wc >= 0) {
      g = 4;
      J.lds = 0;
      J.pad = wc;
    } else if (reg_ok) {   // panel in registers
      g = 2;
      J.lds = 0;
      J.pad = (rows <= 1 ? 0 : rows <= 2 ? 1 : rows <= 4 ? 2 : 3) * 3 + (slots <= 4 ? 0 : slots <= 8 ? 1 : 2);
    } else if (panel + vb + 1024 <= kMaxLds) {
      J.lds = 1;
    } else if (panel + vb <= kMaxDynLarge) {
      J.lds = 1;
      g = 1;
    } else {
      J.lds = 0;
      g = 3;
      scratch.emplace_back(np * J.p * J.k);
      J.ws = scratch.back().get();
    }
    if (g == 0 || g == 1 || g == 3) dyn[g] = std::max(dyn[g], J.lds ? panel + vb : vb);
    {
      static const char* names[5][2] = {{"qr.lds", "qr.lds.p>128"}, {"qr.lds_large", "qr.lds_large.p>128"},
                                        {"qr.reg", "qr.reg.p>128"}, {"qr.global", "qr.global.p>128"},
                                        {"qr.wave", "qr.wave.p>128"}};
      Profiler::get().hit(names[g][J.p > 128 ? 1 : 0], (long long)np);
    }
    J.block0 = b0[g];
    b0[g] += (long long)np;
    const double p = J.p, k = J.k, kr = std::min(J.p, J.k);
    fl[g] += np * (p >= k ? 2.0 * k * k * (p - k / 3.0) : 2.0 * p * p * (k - p / 3.0));
    by[g] += (double)sizeof(T) * np * (p * k + kr * k + (J.Vref ? p * kr : 0.0));
    use[g].push_back(J);
  }
  if (!use[4].empty()) {
    const QJob* dj = upload(use[4], st);
    launch(st, KC_QR, fl[4], by[4], KNAME_T(k_gqr_wave<T>), k_gqr_wave<T>, dim3((unsigned)b0[4]), dim3(WAVE), 0, dj,
           (int)use[4].size());
  }
  if (!use[2].empty() && b0[2] <= kSmallLaunch) {
    const QJob* dj = upload(use[2], st);
    launch(st, KC_QR, fl[2], by[2], KNAME_T(k_gqr_any<T>), k_gqr_any<T>, dim3((unsigned)b0[2]), dim3(256), 0, dj,
           (int)use[2].size());
  } else if (!use[2].empty()) {
    // one launch per register shape (rows per lane, columns per wave / 4)
    std::vector<QJob> by_shape[12];
    for (auto& J : use[2]) by_shape[J.pad].push_back(J);
    for (int sh = 0; sh < 12; ++sh) {
      auto& v = by_shape[sh];
      if (v.empty()) continue;
      long long nb = 0;
      double f = 0, b = 0;
      for (auto& J : v) {
        J.block0 = nb;
        const double np = (double)J.nmat * J.ncl, p = J.p, k = J.k;
        nb += (long long)np;
        f += np * (p >= k ? 2.0 * k * k * (p - k / 3.0) : 2.0 * p * p * (k - p / 3.0));
        b += (double)sizeof(T) * np * (p * k + std::min(p, k) * k + (J.Vref ? p * std::min(p, k) : 0.0));
      }
      const QJob* dj = upload(v, st);
      const int nj = (int)v.size();
      auto go = [&](const char* name, auto kern) {
        launch(st, KC_QR, f, b, name, kern, dim3((unsigned)nb), dim3(256), 0, dj, nj);
      };
      switch (sh) {
        case 0: go(KNAME_T(k_gqr_reg<T, 1, 4>), k_gqr_reg<T, 1, 4>); break;
        case 1: go(KNAME_T(k_gqr_reg<T, 1, 8>), k_gqr_reg<T, 1, 8>); break;
        case 2: go(KNAME_T(k_gqr_reg<T, 1, 16>), k_gqr_reg<T, 1, 16>); break;
        case 3: go(KNAME_T(k_gqr_reg<T, 2, 4>), k_gqr_reg<T, 2, 4>); break;
        case 4: go(KNAME_T(k_gqr_reg<T, 2, 8>), k_gqr_reg<T, 2, 8>); break;
        case 5: go(KNAME_T(k_gqr_reg<T, 2, 16>), k_gqr_reg<T, 2, 16>); break;
        case 6: go(KNAME_T(k_gqr_reg<T, 4, 4>), k_gqr_reg<T, 4, 4>); break;
        case 7: go(KNAME_T(k_gqr_reg<T, 4, 8>), k_gqr_reg<T, 4, 8>); break;
        case 8: go(KNAME_T(k_gqr_reg<T, 4, 16>), k_gqr_reg<T, 4, 16>); break;
        case 9: go(KNAME_T(k_gqr_reg<T, 8, 4>), k_gqr_reg<T, 8, 4>); break;
        case 10: go(KNAME_T(k_gqr_reg<T, 8, 8>), k_gqr_reg<T, 8, 8>); break;
        default: go(KNAME_T(k_gqr_reg<T, 8, 16>), k_gqr_reg<T, 8, 16>); break;
      }
    }
  }
  for (int g : {0, 1, 3}) {   // panels in LDS (64 KB, the full workgroup LDS), then in global scratch
    if (use[g].empty()) continue;
    const QJob* dj = upload(use[g], st);
    const int nj = (int)use[g].size();
    if (g == 3) {
      launch(st, KC_QR, fl[g], by[g], KNAME_T(k_gqr<T, false>), k_gqr<T, false>, dim3((unsigned)b0[g]), dim3(256),
             dyn[g], dj, nj);
      continue;
    }
    if (g == 1) allow_large_lds(reinterpret_cast<const void*>(k_gqr<T, true>));
    launch(st, KC_QR, fl[g], by[g], KNAME_T(k_gqr<T, true>), k_gqr<T, true>, dim3((unsigned)b0[g]), dim3(256),
           dyn[g], dj, nj);
  }
}

// --------------------------------------------------------- tuning runs
namespace {

// Average time of fn() (which enqueues on st) over `reps` runs after one warm-up.
template <typename F>
double time_on_device(hipStream_t st, int reps, F&& fn) {
  fn();
  queue_flush();
  hipEvent_t a, b;
  ACR_HIP(hipEventCreate(&a));
  ACR_HIP(hipEventCreate(&b));
  ACR_HIP(hipEventRecord(a, st));
  for (int r = 0; r < reps; ++r) {
    fn();
    queue_flush();
  }
  ACR_HIP(hipEventRecord(b, st));
  ACR_HIP(hipEventSynchronize(b));
  float ms = 0.0f;
  ACR_HIP(hipEventElapsedTime(&ms, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms / reps;
}

template <typename T>
__global__ void k_tune_fill(T* p, size_t n, unsigned seed) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    unsigned h = (unsigned)e * 2654435761u ^ seed;
    h ^= h >> 13; h *= 0x5bd1e995u; h ^= h >> 15;
    p[e] = (T)((double)(h & 0xffffff) / 16777216.0 - 0.5);
  }
}

template <typename T>
void tune_fill(hipStream_t st, T* p, size_t n, unsigned seed) {
  launch(st, KC_OTHER, 0.0, 0.0, "k_tune_fill", k_tune_fill<T>, dim3(grid1((long long)n, 256, 4096)), dim3(256), 0,
         p, n, seed);
}

// Fastest tile of a recorded GEMM key: M x N x K products of the key's size
// classes on synthetic operands.
template <typename T>
int tune_gemm(hipStream_t st, int M, int N, int kbits, int pbits) {
  const int K = kbits <= 1 ? 1 : (1 << (kbits - 1)) + (1 << (kbits - 1)) / 2;
  const long long np = std::min<long long>(pbits <= 1 ? 1 : (1LL << (pbits - 1)) + (1LL << (pbits - 1)) / 2, 16384);
  DBuf<T> A((size_t)np * M * K), B((size_t)np * K * N), C((size_t)np * M * N);
  tune_fill<T>(st, A.get(), A.size(), 1u);
  tune_fill<T>(st, B.get(), B.size(), 2u);
  GSeg g;
  g.A = bop(A.get(), M, (long long)M * K);
  g.B = bop(B.get(), K, (long long)K * N);
  g.K = K;
  GJob J;
  J.M = M; J.N = N; J.nmat = (int)np; J.ncl = 1; J.C = bop(C.get(), M, (long long)M * N); J.seg0 = 0; J.nseg = 1;
  int best = -1;
  double bt = 1e300;
  for (int kind : {0, 1, 2, 3, 4, 10, 11, 12, 13, 14}) {
    if (kind >= 10 && sizeof(T) != 4) break;
    const double t = time_on_device(st, 5, [&] { ggemm<T>(st, {J}, {g}, kind); });
    if (t < bt) { bt = t; best = kind; }
  }
  return best;
}

// Fastest QR form of a recorded panel key among the forms it allows.
template <typename T>
int tune_qr(hipStream_t st, int p, int k, long long nprob) {
  const long long np = std::max<long long>(1, std::min<long long>(nprob, 8192));
  const int c = std::min(p, k);
  DBuf<T> A((size_t)np * p * k), R((size_t)np * c * k), V((size_t)np * p * c), tau((size_t)np * c);
  tune_fill<T>(st, A.get(), A.size(), 3u);
  QJob J;
  J.p = p; J.k = k; J.nmat = (int)np; J.ncl = 1; J.A = bop(A.get(), p, (long long)p * k);
  J.R = R.get(); J.Vref = V.get(); J.tau = tau.get();
  int best = -1;
  double bt = 1e300;
  for (int form : {4, 2, 0}) {
    const double t = time_on_device(st, 5, [&] { gqr<T>(st, {J}, form); });
    if (t < bt) { bt = t; best = form; }
  }
  return best;
}

}  // namespace

int tune_run(hipStream_t st) {
  Tuner& tu = Tuner::get();
  std::map<std::string, long long> keys;
  {
    std::lock_guard<std::mutex> g(tu.mu);
    keys = tu.seen;
  }
  const bool was = tu.active;
  tu.active = false;   // measure the forms themselves
  int n = 0;
  try {
    for (auto& kv : keys) {
      {
        std::lock_guard<std::mutex> g(tu.mu);
        if (tu.table.count(kv.first)) continue;
      }
      char t = 0;
      int a = 0, b = 0, c = 0, d = 0;
      int choice = -1;
      if (std::sscanf(kv.first.c_str(), "gemm.%c.%d.%d.%d.%d", &t, &a, &b, &c, &d) == 5) {
        choice = t == 'f' ? tune_gemm<float>(st, a, b, c, d) : tune_gemm<double>(st, a, b, c, d);
      } else if (std::sscanf(kv.first.c_str(), "qr.%c.%d.%d", &t, &a, &b) == 3) {
        choice = t == 'f' ? tune_qr<float>(st, a, b, kv.second) : tune_qr<double>(st, a, b, kv.second);
      }
      if (choice < 0) continue;
      std::lock_guard<std::mutex> g(tu.mu);
      tu.table[kv.first] = choice;
      ++n;
    }
  } catch (...) {
    tu.active = was;
    throw;
  }
  tu.active = was;
  return n;
}

template <typename T>
void bqr_r(hipStream_t st, int p, int k, int nmat, int ncl, const BOp& A, T* R, T* Vref, T* tau) {
  std::vector<QJob> jobs(1);
  QJob& J = jobs[0];
  J.p = p; J.k = k; J.nmat = nmat; J.ncl = ncl; J.A = A; J.R = R; J.Vref = Vref; J.tau = tau;
  gqr<T>(st, std::move(jobs));
}

template <typename T>
void gapply_q(hipStream_t st, std::vector<AJob> jobs) {
  // reflectors + output tile in LDS: up to 64 KB in one launch, up to the
  // full gfx950 workgroup LDS in a second one, otherwise in global memory.
  // Problems of at most 128 rows and 32 output columns whose reflectors take
  // at most 16 KB run one wave each, four to a workgroup of launch 0.
  std::vector<AJob> use[2];
  size_t dyn[2] = {0, 0};
  double fl[2] = {0, 0}, by[2] = {0, 0};
  long long b0[2] = {0, 0};
  auto ix = [](int n, int unit) { return n <= 2 * unit ? 0 : n <= 4 * unit ? 1 : 2; };
  auto wave_ok = [&](const AJob& J, size_t need) {
    const int code = ix(J.p, 16) * 3 + ix(J.t, 4);
    return J.p <= 128 && J.t <= 32 && need <= 16384 && (sizeof(T) == 4 || code != 8);
  };
  size_t wneed = 0;
  for (auto& J : jobs) {
    if (J.p <= 0 || J.t <= 0 || J.nmat <= 0 || J.ncl <= 0) continue;
    const size_t need = ((size_t)J.p * J.c + J.c) * sizeof(T);
    if (wave_ok(J, need)) wneed = std::max(wneed, need);
  }
  dyn[0] = 4 * wneed;
  for (auto& J : jobs) {
    if (J.p <= 0 || J.t <= 0 || J.nmat <= 0 || J.ncl <= 0) continue;
    const size_t need = ((size_t)J.p * J.c + J.c) * sizeof(T);
    int g = 0;
    const double np = (double)J.nmat * J.ncl;
    long long nb = (long long)np;
    J.lds = J.p <= WAVE * kApplyRows && J.t <= 4 * kApplyCols;
    if (wave_ok(J, need)) {
      J.lds = 2;
      J.pad = ix(J.p, 16) * 3 + ix(J.t, 4);
      J.wslot = (int)(wneed / sizeof(T));
      nb = (nb + 3) / 4;
    } else if (J.lds && need + 2048 > kMaxLds) {
      if (need <= kMaxDynLarge) g = 1;
      else J.lds = 0;
    }
    if (J.lds == 1) dyn[g] = std::max(dyn[g], need);
    {
      const int v = J.lds == 2 ? 0 : J.lds == 0 ? 1 : g == 0 ? 2 : 3;
      static const char* names[4][2] = {{"applyq.wave", "applyq.wave.p>128"}, {"applyq.global", "applyq.global.p>128"},
                                        {"applyq.lds", "applyq.lds.p>128"}, {"applyq.lds_large", "applyq.lds_large.p>128"}};
      Profiler::get().hit(names[v][J.p > 128 ? 1 : 0], (long long)np);
    }
    J.block0 = b0[g];
    b0[g] += nb;
    fl[g] += 4.0 * np * J.t * ((double)J.p * J.c - 0.5 * J.c * J.c);
    by[g] += (double)sizeof(T) * np * ((double)J.p * J.c + (double)J.c * J.t + (double)J.p * J.t);
    use[g].push_back(J);
  }
  for (int g = 0; g < 2; ++g) {
    if (use[g].empty()) continue;
    if (g == 1) allow_large_lds(reinterpret_cast<const void*>(k_gapply_q<T>));
    const AJob* dj = upload(use[g], st);
    launch(st, KC_APPLYQ, fl[g], by[g], KNAME_T(k_gapply_q<T>), k_gapply_q<T>, dim3((unsigned)b0[g]), dim3(256),
           dyn[g], dj, (int)use[g].size());
  }
}

template <typename T>
void bapply_q(hipStream_t st, int p, int c, int t, int nmat, int ncl, const T* Vref, const T* tau,
              const T* Z, long long sZ, int zxor, const BOp& Y) {
  std::vector<AJob> jobs(1);
  AJob& J = jobs[0];
  J.p = p; J.c = c; J.t = t; J.nmat = nmat; J.ncl = ncl; J.zxor = zxor;
  J.Vref = Vref; J.tau = tau; J.Z = Z; J.sZ = sZ; J.Y = Y;
  gapply_q<T>(st, std::move(jobs));
}

constexpr int kSvdMaxCore = 1024;

template <typename T>
void grsvd(hipStream_t st, std::vector<SJob> jobs) {
  // Cores of size 48..64 go to k_grsvd_reg first; the few whose numerical rank
  // exceeds its register budget are flagged and redone by k_grsvd, which
  // returns at once for every other problem.  k_grsvd keeps the core and its
  // two work matrices in LDS: launch 0 holds the jobs that fit next to the
  // kernel's static arrays in 64 KB, launch 1 those that fit the full gfx950
  // workgroup LDS; larger cores work in global scratch.  When a call holds
  // many cores of size <= 16 (most of the recompressions of a factorisation),
  // those run one wave each (launch 2), so that many more fit on a CU.
  constexpr size_t kStatic = 21504;   // static LDS of k_grsvd_t<T, 4, 512> (21000 bytes in FP32)
  std::vector<DBuf<T>> scratch;
  std::vector<SJob> use[5], reg;
  Profiler& P = Profiler::get();
  const bool prof = P.on(KC_SVD);
  double* fl = nullptr;
  long long b0[5] = {0, 0, 0, 0, 0}, total = 0, nreg = 0, nsmall = 0;
  size_t dyn[5] = {0, 0, 0, 0, 0};
  double by[5] = {0, 0, 0, 0, 0};
  for (auto& J : jobs) {
    if (J.c <= 0 || J.nprob <= 0) continue;
    if (J.c > kSvdMaxCore) fail(ACR_ERR_INVALID_ARG, "rank-revealing SVD core larger than 1024");
    total += J.nprob;
    if (J.c <= 16) nsmall += J.nprob;
  }
  // A core's result never depends on the other problems of the call: cores of
  // at most 16 give the same bits in the one-wave and the four-wave form, so
  // a call with few of them keeps them in the four-wave launch (one launch
  // instead of two at the small levels); cores of 48..64 always take the
  // register form (whose results differ from the LDS form's).
  const bool use_small = nsmall > kSmallLaunch;
  const bool use_reg = true;
  for (auto& J : jobs)
    if (use_reg && J.c >= 48 && J.c <= 64 && J.nprob > 0) nreg += J.nprob;
  if (total == 0) return;
  if (prof) {
    std::lock_guard<std::mutex> g(P.mu());
    P.owned_d().emplace_back((size_t)total);
    fl = P.owned_d().back().get();
  }
  DBuf<int> redo((size_t)nreg);
  if (nreg) memset_async(redo.get(), 0, (size_t)nreg * sizeof(int), st);
  long long done = 0, rdone = 0, rb0 = 0;
  double rby = 0;
  for (auto& J : jobs) {
    if (J.c <= 0 || J.nprob <= 0) continue;
    J.flops = fl ? fl + done : nullptr;
    done += J.nprob;
    J.redo = nullptr;
    if (use_reg && J.c >= 48 && J.c <= 64) {
      J.redo = redo.get() + rdone;
      rdone += J.nprob;
      SJob R = J;
      R.block0 = rb0;
      rb0 += J.nprob;
      rby += 4.0 * (double)J.c * J.c * J.nprob * sizeof(T);
      reg.push_back(R);
    }
    const size_t need = 3 * (size_t)J.c * J.c * sizeof(T);
    int g = use_small && J.c <= 16 ? 2 : 0;
    J.lds = 1;
    if (g == 0 && need + kStatic > kMaxLds) {
      if (need + kStatic <= kMaxLdsLarge) g = 1;
      else { J.lds = 0; g = J.c > 512 ? 4 : 3; }
    }
    {
      static const char* names[5] = {"svd.lds", "svd.lds_large", "svd.wave16", "svd.global", "svd.global1024"};
      Profiler::get().hit(J.redo ? "svd.reg" : names[g], J.nprob);
      Profiler::get().hit(J.c <= 16 ? "svd.c<=16" : J.c <= 32 ? "svd.c17-32" : J.c < 48 ? "svd.c33-47"
                          : J.c <= 64 ? "svd.c48-64" : "svd.c>64", J.nprob);
    }
    if (J.lds) {
      dyn[g] = std::max(dyn[g], need);
    } else {
      scratch.emplace_back((size_t)J.nprob * J.c * J.c);
      J.X = scratch.back().get();
      scratch.emplace_back((size_t)J.nprob * J.c * J.c);
      J.J = scratch.back().get();
    }
    J.block0 = b0[g];
    b0[g] += J.nprob;
    if (!J.redo) by[g] += 4.0 * (double)J.c * J.c * J.nprob * sizeof(T);
    use[g].push_back(J);
  }
  if (!reg.empty()) {
    const SJob* dj = upload(reg, st);
    launch(st, KC_SVD, 0.0, rby, KNAME_T(k_grsvd_reg<T>), k_grsvd_reg<T>, dim3((unsigned)rb0), dim3(256), 0, dj,
           (int)reg.size());
  }
  // launches: 0 and 1 in LDS (64 KB / the full workgroup LDS), 2 the small
  // one-wave cores, 3 the cores that work in global scratch, 4 those of more
  // than 512 columns
  for (int g = 0; g < 5; ++g) {
    if (use[g].empty()) continue;
    const SJob* dj = upload(use[g], st);
    const int nj = (int)use[g].size();
    const dim3 grid((unsigned)b0[g]);
    if (g == 2) {
      launch(st, KC_SVD, 0.0, by[g], KNAME_T(k_grsvd_t<T, 1, 16, true>), k_grsvd_t<T, 1, 16, true>, grid,
             dim3(WAVE), dyn[g], dj, nj);
    } else if (g == 3) {
      launch(st, KC_SVD, 0.0, by[g], KNAME_T(k_grsvd_t<T, 4, 512, false>), k_grsvd_t<T, 4, 512, false>, grid,
             dim3(256), 0, dj, nj);
    } else if (g == 4) {
      launch(st, KC_SVD, 0.0, by[g], KNAME_T(k_grsvd_t<T, 4, kSvdMaxCore, false>),
             k_grsvd_t<T, 4, kSvdMaxCore, false>, grid, dim3(256), 0, dj, nj);
    } else {
      if (g == 1) allow_large_lds(reinterpret_cast<const void*>(k_grsvd_t<T, 4, 512, true>), kMaxLdsLarge - kStatic);
      launch(st, KC_SVD, 0.0, by[g], KNAME_T(k_grsvd_t<T, 4, 512, true>), k_grsvd_t<T, 4, 512, true>, grid,
             dim3(256), dyn[g], dj, nj);
    }
  }
  if (fl) {   // device-counted flops of every problem, credited to the last launch
    const int n = (int)total;
    Queue::get().op(st, [=]() {
      std::lock_guard<std::mutex> g(Profiler::get().mu());
      auto& recs = Profiler::get().recs();
      if (!recs.empty() && recs.back().cls == KC_SVD) { recs.back().dev_flops = fl; recs.back().nprob = n; }
    });
  }
}

template <typename T>
void brsvd(hipStream_t st, int c, int nprob, T* K, T* sig, T* UK, int* rank, double eps, int maxrank) {
  std::vector<SJob> jobs(1);
  SJob& J = jobs[0];
  J.c = c; J.nprob = nprob; J.K = K; J.sig = sig; J.UK = UK; J.rank = rank; J.eps = eps; J.maxrank = maxrank;
  grsvd<T>(st, std::move(jobs));
}


template <typename T>
void gcopy(hipStream_t st, std::vector<CJob> jobs) {
  std::vector<CJob> use;
  long long b0 = 0;
  double by = 0;
  for (auto& J : jobs) {
    if (J.rows <= 0 || J.cols <= 0 || J.nmat <= 0 || J.ncl <= 0) continue;
    const long long n = (long long)J.rows * J.cols;
    if (n > 0x7fffffffLL - kCopyChunk) fail(ACR_ERR_INVALID_ARG, "grouped copy: matrix too large");
    J.chunks = (int)((n + kCopyChunk - 1) / kCopyChunk);
    J.block0 = b0;
    b0 += (long long)J.nmat * J.ncl * J.chunks;
    {   // 16-byte accesses when every operand start and column is 16-byte aligned
      const long long V = 16 / (long long)sizeof(T);
      auto al = [&](const BOp& o) {
        return reinterpret_cast<uintptr_t>(o.p) % 16 == 0 && o.ld % V == 0 && o.sm % V == 0 && o.sc_pair % V == 0 &&
               o.sc_odd % V == 0;
      };
      J.vec = J.rows % V == 0 && al(J.src) && al(J.dst);
    }
    by += (2.0 + J.accumulate) * n * J.nmat * J.ncl * sizeof(T);
    use.push_back(J);
  }
  if (use.empty()) return;
  if (b0 > 0x7fffffffLL) fail(ACR_ERR_INVALID_ARG, "grouped copy grid too large");
  const CJob* dj = upload(use, st);
  launch(st, KC_COPY, 0.0, by, KNAME_T(k_gcopy<T>), k_gcopy<T>, dim3((unsigned)b0), dim3(256), 0, dj, (int)use.size());
}

template <typename T>
HmvStep hmv_plan(std::vector<MVJob> jobs, const std::vector<MVTerm>& terms) {
  constexpr int CH = 16;
  // every job gets its own copies of its terms, with the places of their
  // projections in the buffer
  HmvStep h;
  std::vector<MVJob>& use = h.jobs;
  std::vector<MVTerm>& tm = h.terms;
  std::vector<MVRed>& reds = h.reds;
  long long rows = 0, units = 0, tsize = 0;
  double flr = 0, byr = 0, fla = 0, bya = 0;
  int maxnr = 1;
  bool w64 = true;   // then every s = b 2^L and every row count are multiples of 64
  for (auto J : jobs) {
    if (J.nmat <= 0) continue;
    const int s = J.s, b = J.b, L = J.L, nrhs = J.nrhs;
    if (nrhs < 1 || nrhs > 8) fail(ACR_ERR_INTERNAL, "matvec takes 1..8 right-hand sides");
    if (b < 1 || b > 256 || L > kMvMaxDepth || (b << L) != s) fail(ACR_ERR_INTERNAL, "matvec shape");
    maxnr = std::max(maxnr, nrhs);
    if (b % WAVE != 0) w64 = false;
    const int t0 = (int)tm.size();
    for (int t = 0; t < J.nterm; ++t) {
      MVTerm M = terms[J.term0 + t];
      M.s = s;
      M.nrhs = nrhs;
      double e = s;
      if (M.type == 0) {
        int upm = 0;
        for (int d = 1; d <= kMvMaxDepth; ++d)
          if (d > L) M.kc[d] = 0;
        for (int d = 1; d <= L; ++d) {
          if (M.kc[d] < 0 || M.kc[d] > M.k[d]) fail(ACR_ERR_INTERNAL, "matvec: rank above the allocation");
          upm += (1 << d) * ((M.kc[d] + CH - 1) / CH);
          const double ka = M.kmean[d] > 0.0f ? std::min<double>(M.kmean[d], M.kc[d]) : M.kc[d];
          flr += 2.0 * J.nmat * s * ka * nrhs;
          byr += (double)J.nmat * s * (ka + (M.kc[d] ? nrhs : 0)) * sizeof(T);
          e += (double)s * ka;
        }
        e += (double)s * (b - 1);
        if (upm > 0) {
          MVRed R;
          R.block0 = units;
          R.term = (int)tm.size();
          R.upm = upm;
          reds.push_back(R);
          units += (long long)J.nmat * upm;
        }
      }
      fla += 2.0 * J.nmat * e * nrhs;
      bya += (double)J.nmat * (e + (double)s * nrhs) * sizeof(T);
      tm.push_back(M);
    }
    J.term0 = t0;
    J.block0 = rows;
    rows += (long long)J.nmat * s;
    bya += (double)J.nmat * s * nrhs * sizeof(T) * (J.C0 ? 2 : 1);
    use.push_back(J);
  }
  if (use.empty()) return h;
  const int NR = maxnr <= 1 ? 1 : maxnr <= 2 ? 2 : maxnr <= 4 ? 4 : 8;
  // projection slots: NR per column (the kernels index with the launch's NR)
  for (auto& M : tm) {
    if (M.type != 0) continue;
    int off = 0;
    for (int d = 1; d <= kMvMaxDepth; ++d) {
      M.toff[d] = off;
      off += (1 << d) * M.kc[d] * NR;
    }
    M.tstride = off;
  }
  {   // place each term's projections: terms of job j follow in order
    long long base = 0;
    for (auto& J : use)
      for (int t = 0; t < J.nterm; ++t) {
        MVTerm& M = tm[J.term0 + t];
        if (M.type != 0) continue;
        M.tbase = base;
        base += (long long)J.nmat * M.tstride;
      }
    tsize = base;
  }
  if ((rows + WAVE - 1) / WAVE > 0x7fffffffLL || (units + 3) / 4 > 0x7fffffffLL)
    fail(ACR_ERR_INVALID_ARG, "matvec grid too large");
  h.rows = rows; h.units = units; h.tsize = tsize; h.NR = NR; h.w64 = w64;
  h.flr = flr; h.byr = byr; h.fla = fla; h.bya = bya;
  return h;
}

template <typename T>
void hmv_launch(hipStream_t st, const HmvStep& h, const MVRed* dr, const MVTerm* dt, const MVJob* dj, T* tbuf) {
  if (h.rows <= 0) return;
  if (h.units > 0) {
    const dim3 grid((unsigned)((h.units + 3) / 4));
    const int nr = (int)h.reds.size();
    auto go = [&](const char* name, auto kern) {
      launch(st, KC_MATVEC, h.flr, h.byr, name, kern, grid, dim3(256), 0, dr, nr, dt, h.units, tbuf);
    };
    switch (h.NR) {
      case 1: go(KNAME_T(k_hmv_reduce<T, 1>), k_hmv_reduce<T, 1>); break;
      case 2: go(KNAME_T(k_hmv_reduce<T, 2>), k_hmv_reduce<T, 2>); break;
      case 4: go(KNAME_T(k_hmv_reduce<T, 4>), k_hmv_reduce<T, 4>); break;
      default: go(KNAME_T(k_hmv_reduce<T, 8>), k_hmv_reduce<T, 8>); break;
    }
  }
  const dim3 grid((unsigned)((h.rows + WAVE - 1) / WAVE));
  const int nj = (int)h.jobs.size();
  auto go = [&](const char* name, auto kern) {
    launch(st, KC_MATVEC, h.fla, h.bya, name, kern, grid, dim3(WAVE), 0, dj, nj, dt, h.rows, (const T*)tbuf);
  };
#define ACR_HMV_APPLY(NRV)                                                                   \
  if (h.w64) go(KNAME_T(k_hmv_apply<T, NRV, true>), k_hmv_apply<T, NRV, true>);            \
  else go(KNAME_T(k_hmv_apply<T, NRV, false>), k_hmv_apply<T, NRV, false>);
  switch (h.NR) {
    case 1: ACR_HMV_APPLY(1) break;
    case 2: ACR_HMV_APPLY(2) break;
    case 4: ACR_HMV_APPLY(4) break;
    default: ACR_HMV_APPLY(8) break;
  }
#undef ACR_HMV_APPLY
}

template <typename T>
void ghmv(hipStream_t st, std::vector<MVJob> jobs, const std::vector<MVTerm>& terms) {
  const HmvStep h = hmv_plan<T>(std::move(jobs), terms);
  if (h.rows <= 0) return;
  DBuf<T> tbuf((size_t)std::max<long long>(h.tsize, 1));
  const MVTerm* dt = h.terms.empty() ? nullptr : upload(h.terms, st);
  const MVRed* dr = h.units > 0 ? upload(h.reds, st) : nullptr;
  const MVJob* dj = upload(h.jobs, st);
  hmv_launch<T>(st, h, dr, dt, dj, tbuf.get());
}

template <typename T>
void PBuilder::step(std::vector<MVJob> js, const std::vector<MVTerm>& tms) {
  constexpr int CH = 16;
  auto producer = [&](const void* base, long long blk, long long vs, int* dep, int* need, int& nd) {
    auto it = prod_.find(reinterpret_cast<long long>(base) + blk * vs);
    if (it == prod_.end()) return;   // written before the pass
    for (int e = 0; e < nd; ++e)
      if (dep[e] == it->second.first) return;
    if (nd >= kPMaxDep) fail(ACR_ERR_INTERNAL, "persistent solve: too many dependencies");
    dep[nd] = it->second.first;
    need[nd] = it->second.second;
    ++nd;
  };
  for (auto J : js) {
    if (J.nmat <= 0) continue;
    const int s = J.s, b = J.b, L = J.L, nrhs = J.nrhs;
    if (nrhs < 1 || nrhs > NR) fail(ACR_ERR_INTERNAL, "persistent solve: right-hand sides above the plan's slots");
    if (b < 1 || b > 256 || L > kMvMaxDepth || (b << L) != s) fail(ACR_ERR_INTERNAL, "matvec shape");
    if (b % WAVE != 0) w64 = false;
    const long long vs = (long long)s * nrhs * (long long)sizeof(T);
    const int t0 = (int)terms.size();
    std::vector<int> upm(J.nterm, 0);
    for (int t = 0; t < J.nterm; ++t) {
      MVTerm M = tms[J.term0 + t];
      M.s = s;
      M.nrhs = nrhs;
      double e = s;
      if (M.type == 0) {
        for (int d = L + 1; d <= kMvMaxDepth; ++d) M.kc[d] = 0;
        int off = 0;
        for (int d = 1; d <= L; ++d) {
          if (M.kc[d] < 0 || M.kc[d] > M.k[d]) fail(ACR_ERR_INTERNAL, "matvec: rank above the allocation");
          upm[t] += (1 << d) * ((M.kc[d] + CH - 1) / CH);
          M.toff[d] = off;
          off += (1 << d) * M.kc[d] * NR;
          const double ka = M.kmean[d] > 0.0f ? std::min<double>(M.kmean[d], M.kc[d]) : M.kc[d];
          flops += 2.0 * J.nmat * s * ka * nrhs;
          bytes += (double)J.nmat * s * (ka + (M.kc[d] ? nrhs : 0)) * sizeof(T);
          e += (double)s * ka;
        }
        for (int d = L + 1; d <= kMvMaxDepth; ++d) M.toff[d] = off;
        e += (double)s * (b - 1);
        M.tstride = off;
        M.tbase = tsize;
        tsize += (long long)J.nmat * off;
      }
      flops += 2.0 * J.nmat * e * nrhs;
      bytes += (double)J.nmat * (e + (double)s * nrhs) * sizeof(T);
      terms.push_back(M);
    }
    bytes += (double)J.nmat * s * nrhs * sizeof(T) * (J.C0 ? 2 : 1);
    J.term0 = t0;
    J.block0 = 0;
    const int ji = (int)jobs.size();
    jobs.push_back(J);
    for (int m = 0; m < J.nmat; ++m) {
      PTask ap;
      ap.kind = 1;
      ap.idx = ji;
      ap.m = m;
      for (int t = 0; t < J.nterm; ++t) {
        const MVTerm& M = terms[t0 + t];
        const long long yb = (long long)M.ymul * m + M.yoff;
        if (M.type == 0 && upm[t] > 0) {   // projection tasks of this (term, matrix)
          const int rc = nctr++;
          int nrt = 0;
          for (int u = 0; u < upm[t]; u += kPUnits, ++nrt) {
            PTask rp;
            rp.kind = 0;
            rp.idx = t0 + t;
            rp.m = m;
            rp.u0 = u;
            rp.u1 = std::min(upm[t], u + kPUnits);
            rp.done = rc;
            producer(M.y, yb, vs, rp.dep, rp.need, rp.ndep);
            tasks.push_back(rp);
          }
          ap.dep[ap.ndep] = rc;
          ap.need[ap.ndep] = nrt;
          ++ap.ndep;
        }
        producer(M.y, yb, vs, ap.dep, ap.need, ap.ndep);
      }
      if (J.C0) producer(J.C0, (long long)J.cmul * m + J.coff, vs, ap.dep, ap.need, ap.ndep);
      const int oc = nctr++;
      int nat = 0;
      ap.done = oc;
      for (int r = 0; r < s; r += kPRows, ++nat) {
        PTask t = ap;
        t.u0 = r;
        t.u1 = std::min(s, r + kPRows);
        tasks.push_back(t);
      }
      prod_[reinterpret_cast<long long>(J.out) + ((long long)J.omul * m + J.ooff) * vs] = {oc, nat};
    }
  }
}

void PBuilder::check() const {
  std::vector<long long> total((size_t)nctr, 0), seen((size_t)nctr, 0);
  for (const PTask& t : tasks) {
    if (t.done < 0 || t.done >= nctr) fail(ACR_ERR_INTERNAL, "persistent solve: counter out of range");
    ++total[(size_t)t.done];
  }
  for (const PTask& t : tasks) {
    if (t.ndep < 0 || t.ndep > kPMaxDep || t.u0 < 0 || t.u1 <= t.u0)
      fail(ACR_ERR_INTERNAL, "persistent solve: malformed task");
    for (int e = 0; e < t.ndep; ++e) {
      const int c = t.dep[e];
      if (c < 0 || c >= nctr || c == t.done || t.need[e] <= 0 || seen[(size_t)c] != t.need[e] ||
          total[(size_t)c] != t.need[e])
        fail(ACR_ERR_INTERNAL, "persistent solve: a task waits for work listed after it");
    }
    ++seen[(size_t)t.done];
  }
}

template <typename T>
void psolve_run(hipStream_t st, std::vector<PInst> insts, int NR, bool w64, int* ctl, const std::vector<VJob>& fin,
                double flops, double bytes) {
  long long nt = 0;
  for (auto& I : insts) {
    I.task0 = nt;
    nt += I.ntasks;
  }
  if (nt <= 0) return;
  if (nt > 0x7fffffffLL) fail(ACR_ERR_INVALID_ARG, "persistent solve: too many tasks");
  const PInst* di = upload(insts, st);
  // one workgroup per CU: the deep levels hold a few hundred tasks at a time
  const unsigned grid = (unsigned)std::min<long long>(nt, 256);
  const long long limit = SolveMode::get().limit.load();
  const int ni = (int)insts.size();
  auto go = [&](const char* name, auto kern) {
    launch(st, KC_MATVEC, flops, bytes, name, kern, dim3(grid), dim3(256), 0, di, ni, nt, ctl, ctl + 1, limit);
  };
#define ACR_PSOLVE(NRV)                                                         \
  if (w64) go(KNAME_T(k_psolve<T, NRV, true>), k_psolve<T, NRV, true>);      \
  else go(KNAME_T(k_psolve<T, NRV, false>), k_psolve<T, NRV, false>);
  switch (NR) {
    case 1: ACR_PSOLVE(1) break;
    case 2: ACR_PSOLVE(2) break;
    case 4: ACR_PSOLVE(4) break;
    default: ACR_PSOLVE(8) break;
  }
#undef ACR_PSOLVE
  // NaN for the final unknowns if a wait gave up (nothing happens otherwise)
  long long b0 = 0;
  std::vector<VJob> use;
  for (auto J : fin) {
    const long long n = (long long)J.s * J.nblk * J.nrhs;
    if (n <= 0) continue;
    J.per = (int)std::min<long long>((n + 255) / 256, 1024);
    J.block0 = b0;
    b0 += J.per;
    use.push_back(J);
  }
  if (use.empty()) return;
  const VJob* dj = upload(use, st);
  launch(st, KC_OTHER, 0.0, 0.0, KNAME_T(k_pcheck<T>), k_pcheck<T>, dim3((unsigned)b0), dim3(256), 0, dj,
         (int)use.size(), (const int*)(ctl + 1));
}

template <typename T>
void ghmv(hipStream_t st, int s, int b, int L, int nrhs, std::vector<MVJob> jobs,
          const std::vector<MVTerm>& terms) {
  for (auto& J : jobs) { J.s = s; J.b = b; J.L = L; J.nrhs = nrhs; }
  ghmv<T>(st, std::move(jobs), terms);
}

template <typename T>
void gto_blocks(hipStream_t st, std::vector<VJob> jobs) {
  long long b0 = 0;
  double by = 0;
  std::vector<VJob> use;
  for (auto J : jobs) {
    const long long n = (long long)J.s * J.nblk * J.nrhs;
    if (n <= 0) continue;
    J.per = (int)std::min<long long>((n + 255) / 256, 4096);
    J.block0 = b0;
    b0 += J.per;
    by += (double)n * (8 + sizeof(T));
    use.push_back(J);
  }
  if (use.empty()) return;
  const VJob* dj = upload(use, st);
  launch(st, KC_OTHER, 0.0, by, KNAME_T(k_gto_blocks<T>), k_gto_blocks<T>, dim3((unsigned)b0), dim3(256), 0, dj,
         (int)use.size());
}

template <typename T>
void gfrom_blocks(hipStream_t st, std::vector<VJob> jobs) {
  long long b0 = 0;
  double by = 0;
  std::vector<VJob> use;
  for (auto J : jobs) {
    const long long n = (long long)J.s * J.nblk * J.nrhs;
    if (n <= 0) continue;
    J.per = (int)std::min<long long>((n + 255) / 256, 4096);
    J.block0 = b0;
    b0 += J.per;
    by += (double)n * (8 + sizeof(T));
    use.push_back(J);
  }
  if (use.empty()) return;
  const VJob* dj = upload(use, st);
  launch(st, KC_OTHER, 0.0, by, KNAME_T(k_gfrom_blocks<T>), k_gfrom_blocks<T>, dim3((unsigned)b0), dim3(256), 0, dj,
         (int)use.size());
}

template <typename T>
void bcopy(hipStream_t st, int rows, int cols, int nmat, T alpha, const BOp& src, const BOp& dst) {
  std::vector<CJob> jobs(1);
  CJob& J = jobs[0];
  J.rows = rows; J.cols = cols; J.nmat = nmat; J.ncl = 1; J.alpha = (double)alpha; J.src = src; J.dst = dst;
  gcopy<T>(st, std::move(jobs));
}

template <typename T>
void badd(hipStream_t st, int rows, int cols, int nmat, T alpha, const BOp& src, const BOp& dst) {
  std::vector<CJob> jobs(1);
  CJob& J = jobs[0];
  J.rows = rows; J.cols = cols; J.nmat = nmat; J.ncl = 1; J.alpha = (double)alpha; J.src = src; J.dst = dst;
  J.accumulate = 1;
  gcopy<T>(st, std::move(jobs));
}

void zero_bytes_now(const ZeroArgs& z, hipStream_t st) {
  if (z.count <= 0) return;
  unsigned long long most = 0, total = 0;
  for (int i = 0; i < z.count; ++i) {
    most = std::max(most, z.n[i]);
    total += z.n[i];
  }
  ProfScope ps(KC_OTHER, st, 0.0, (double)total, Phase::cur(), "k_zero_bytes");
  const long long work = std::max<long long>((long long)(most / 16), 16);
  hipLaunchKernelGGL(k_zero_bytes, dim3(grid1(work, 256, 4096), z.count), dim3(256), 0, st, z);
  ACR_HIP(hipGetLastError());
}

template <typename T>
void fill(hipStream_t st, T* p, size_t n, T v) {
  if (!n) return;
  launch(st, KC_OTHER, 0.0, (double)n * sizeof(T), KNAME_T(k_fill<T>), k_fill<T>, dim3(grid1((long long)n, 256, 16384)),
         dim3(256), 0, p, n, v);
}

template <typename T>
void bscale(hipStream_t st, int rows, int cols, int nmat, int ncl, const BOp& X, const T* vec,
            int vmul, int voff, long long vstride, long long vcl, int side, T alpha) {
  std::vector<CJob> jobs(1);
  CJob& J = jobs[0];
  J.rows = rows; J.cols = cols; J.nmat = nmat; J.ncl = ncl; J.alpha = (double)alpha; J.src = X; J.dst = X;
  J.scale = vec; J.smul = vmul; J.soff = voff; J.sstride = vstride; J.scl = vcl; J.sside = side;
  gcopy<T>(st, std::move(jobs));
}

namespace {
// Workgroups per matrix of an ingest job covering `work` elements per matrix.
int ingest_per(long long work, int cap) { return (int)std::max(1LL, std::min<long long>((work + 255) / 256, cap)); }

template <typename T, typename K>
void launch_opjobs(hipStream_t st, std::vector<OpJob> jobs, long long (*work)(const OpJob&), int cap, int cls,
                   const char* name, K kern, size_t dyn = 0, bool one_per_matrix = false) {
  long long b0 = 0;
  std::vector<OpJob> use;
  double by = 0;
  for (auto J : jobs) {
    if (J.nmat <= 0 || J.s <= 0) continue;
    J.per = one_per_matrix ? 1 : ingest_per(work(J), cap);
    J.block0 = b0;
    b0 += (long long)J.nmat * J.per;
    by += (double)J.nmat * work(J) * sizeof(T);
    use.push_back(J);
  }
  if (use.empty()) return;
  if (b0 > 0x7fffffffLL) fail(ACR_ERR_INVALID_ARG, "ingest grid too large");
  const OpJob* dj = upload(use, st);
  launch(st, cls, 0.0, by, name, kern, dim3((unsigned)b0), dim3(256), dyn, dj, (int)use.size());
}
}  // namespace

template <typename T>
void gleaves_tridiag(hipStream_t st, std::vector<OpJob> jobs) {
  launch_opjobs<T>(st, std::move(jobs), [](const OpJob& J) { return (long long)J.s * J.b; }, 64, KC_OTHER,
                   KNAME_T(k_leaves_tridiag<T>), k_leaves_tridiag<T>);
}

template <typename T>
void grank1_factors(hipStream_t st, std::vector<OpJob> jobs) {
  for (const auto& J : jobs)
    if (J.L > kMvMaxDepth) fail(ACR_ERR_INTERNAL, "rank-one factors: HODLR too deep");
  launch_opjobs<T>(st, std::move(jobs), [](const OpJob& J) { return (long long)J.s * std::max(J.L, 1); }, 16,
                   KC_OTHER, KNAME_T(k_rank1<T>), k_rank1<T>);
}

int plane_rank(int s, int d, int pnx) { return (s >> d) % pnx == 0 ? pnx : 1; }

template <typename T>
void gplane_factors(hipStream_t st, std::vector<OpJob> jobs) {
  for (const auto& J : jobs)
    if (J.L > kMvMaxDepth || J.pnx <= 0) fail(ACR_ERR_INTERNAL, "plane factors: bad job");
  launch_opjobs<T>(st, std::move(jobs),
                   [](const OpJob& J) {
                     long long w = 0;
                     for (int d = 1; d <= J.L; ++d) w += (long long)J.s * plane_rank(J.s, d, J.pnx);
                     return std::max(w, (long long)J.s);
                   },
                   16, KC_OTHER, KNAME_T(k_plane_factors<T>), k_plane_factors<T>);
}

template <typename T>
void ggather_diag(hipStream_t st, std::vector<OpJob> jobs) {
  launch_opjobs<T>(st, std::move(jobs), [](const OpJob& J) { return (long long)J.s; }, 16, KC_OTHER,
                   KNAME_T(k_gather_diag<T>), k_gather_diag<T>);
}

template <typename T>
void gtridiag_inverse(hipStream_t st, std::vector<OpJob> jobs) {
  int smax = 0;
  for (const auto& J : jobs) {
    if (J.nmat <= 0) continue;
    if (J.s > 3072 || J.L > kMvMaxDepth) fail(ACR_ERR_INTERNAL, "tridiagonal inverse: block too large");
    smax = std::max(smax, J.s);
  }
  if (smax == 0) return;
  const size_t dyn = 5 * (size_t)smax * sizeof(double);
  if (dyn > kMaxLds - 1024) allow_large_lds(reinterpret_cast<const void*>(k_tridiag_inverse<T>));
  launch_opjobs<T>(st, std::move(jobs), [](const OpJob& J) { return (long long)J.s * J.b + 2LL * J.s * J.L; }, 1,
                   KC_INVERSE, KNAME_T(k_tridiag_inverse<T>), k_tridiag_inverse<T>, dyn, true);
}

template <typename T>
void to_blocks(hipStream_t st, int s, int nblk, int nrhs, const double* B, long long ld, T* V) {
  const long long n = (long long)s * nblk * nrhs;
  if (n <= 0) return;
  launch(st, KC_OTHER, 0.0, (double)n * (8 + sizeof(T)), KNAME_T(k_to_blocks<T>), k_to_blocks<T>, dim3(grid1(n, 256, 16384)),
         dim3(256), 0, s, nblk, nrhs, B, ld, V);
}

template <typename T>
void from_blocks(hipStream_t st, int s, int nblk, int nrhs, const T* V, double* B, long long ld) {
  const long long n = (long long)s * nblk * nrhs;
  if (n <= 0) return;
  launch(st, KC_OTHER, 0.0, (double)n * (8 + sizeof(T)), KNAME_T(k_from_blocks<T>), k_from_blocks<T>, dim3(grid1(n, 256, 16384)),
         dim3(256), 0, s, nblk, nrhs, V, B, ld);
}

template <typename T>
void bdiag_axpy(hipStream_t st, int s, int nrhs, int nmat, T alpha, const T* d, int dmul, int doff,
                const T* x, int xmul, int xoff, T* y, int ymul, int yoff) {
  if (nmat <= 0) return;
  dim3 g(grid1((long long)s * nrhs, 256, 256), nmat);
  launch(st, KC_MATVEC, 2.0 * s * nrhs * nmat, (double)sizeof(T) * nmat * (3.0 * s * nrhs + s),
KNAME_T(k_bdiag_axpy<T>),          k_bdiag_axpy<T>, g, dim3(256), 0, s, nrhs, alpha, d, dmul, doff, x, xmul, xoff, y, ymul, yoff);
}

void stencil_residual(hipStream_t st, int nx, int ny, int nrhs, const double* diag,
                      const double* west, const double* east, const double* south,
                      const double* north, const double* X, const double* B, double* R) {
  const long long N = (long long)nx * ny;
  dim3 g(grid1(N, 256, 8192), nrhs);
  launch(st, KC_OTHER, 10.0 * N * nrhs, 8.0 * N * (5.0 + 3.0 * nrhs), KNAME0(k_residual), k_residual, g, dim3(256), 0, nx, ny,
         diag, west, east, south, north, X, B, R);
}

void stencil_residual3d(hipStream_t st, int nx, int ny, int nz, int nrhs, const double* const* a7,
                        const double* X, const double* B, double* R) {
  const long long N = (long long)nx * ny * nz;
  dim3 g(grid1(N, 256, 8192), nrhs);
  launch(st, KC_OTHER, 14.0 * N * nrhs, 8.0 * N * (7.0 + 3.0 * nrhs), KNAME0(k_residual3d), k_residual3d, g,
         dim3(256), 0, nx, ny, nz, a7[0], a7[1], a7[2], a7[3], a7[4], a7[5], a7[6], X, B, R);
}

namespace {
// Workgroups per column of a grouped vector job of N values.
int vec_per(long long N) { return (int)std::min<long long>(std::max<long long>(1, (N + 2047) / 2048), 512); }

void launch_rjobs(hipStream_t st, std::vector<RJob> jobs, int (*per)(const RJob&), bool per_column_only,
                  const char* name, void (*kern)(const RJob*, int), double bytes_per_value) {
  long long b0 = 0;
  double by = 0;
  std::vector<RJob> use;
  for (auto J : jobs) {
    const long long N = (long long)J.nx * J.ny;
    if (N <= 0 || J.nrhs <= 0) continue;
    J.per = per(J);
    J.block0 = b0;
    b0 += per_column_only ? J.nrhs : (long long)J.nrhs * J.per;
    by += bytes_per_value * N * J.nrhs;
    use.push_back(J);
  }
  if (use.empty()) return;
  const RJob* dj = upload(use, st);
  launch(st, KC_OTHER, 0.0, by, name, kern, dim3((unsigned)b0), dim3(256), 0, dj, (int)use.size());
}
}  // namespace

template <typename T>
void gdense_to_hodlr(hipStream_t st, std::vector<HJob> jobs) {
  long long b0 = 0;
  std::vector<HJob> use;
  for (auto J : jobs) {
    if (J.nmat <= 0 || J.s <= 0) continue;
    if (J.L > kMvMaxDepth) fail(ACR_ERR_INTERNAL, "dense ingest: HODLR too deep");
    J.per = (int)std::min<long long>(((long long)J.s * J.s + 1023) / 1024, 256);
    J.block0 = b0;
    b0 += (long long)J.nmat * J.per;
    use.push_back(J);
  }
  if (use.empty()) return;
  const HJob* dj = upload(use, st);
  launch(st, KC_COPY, 0.0, 0.0, KNAME_T(k_dense_to_hodlr<T>), k_dense_to_hodlr<T>, dim3((unsigned)b0), dim3(256), 0,
         dj, (int)use.size());
}

template <typename T>
void gdense_blocks(hipStream_t st, std::vector<DenseJob> jobs) {
  long long b0 = 0;
  std::vector<DenseJob> use;
  for (auto J : jobs) {
    if (J.s <= 0) continue;
    J.per = (int)std::min<long long>(((long long)J.s * J.s + 1023) / 1024, 256);
    J.block0 = b0;
    b0 += J.per;
    use.push_back(J);
  }
  if (use.empty()) return;
  const DenseJob* dj = upload(use, st);
  launch(st, KC_COPY, 0.0, 0.0, KNAME_T(k_dense_blocks<T>), k_dense_blocks<T>, dim3((unsigned)b0), dim3(256), 0, dj,
         (int)use.size());
}

void gresidual(hipStream_t st, std::vector<RJob> jobs) {
  launch_rjobs(st, std::move(jobs), [](const RJob& J) { return vec_per((long long)J.nx * J.ny); }, false,
               KNAME0(k_gresidual), k_gresidual, 64.0);
}

void gcol_sumsq(hipStream_t st, std::vector<RJob> jobs) {
  // the parts buffer of every job, then the two passes
  size_t tot = 0;
  for (auto& J : jobs) tot += (size_t)J.nrhs * vec_per((long long)J.nx * J.ny);
  DBuf<double> part(std::max<size_t>(tot, 1));
  size_t off = 0;
  for (auto& J : jobs) {
    J.part = part.get() + off;
    off += (size_t)J.nrhs * vec_per((long long)J.nx * J.ny);
  }
  auto per = [](const RJob& J) { return vec_per((long long)J.nx * J.ny); };
  launch_rjobs(st, jobs, per, false, KNAME0(k_gsumsq_part), k_gsumsq_part, 8.0);
  launch_rjobs(st, jobs, per, true, KNAME0(k_gsumsq_final), k_gsumsq_final, 0.0);
}

void gaxpy(hipStream_t st, std::vector<RJob> jobs) {
  launch_rjobs(st, std::move(jobs), [](const RJob& J) { return vec_per((long long)J.nx * J.ny); }, false,
               KNAME0(k_gaxpy), k_gaxpy, 24.0);
}

void col_sumsq(hipStream_t st, long long n, int ncol, const double* A, double* out) {
  const int nparts = (int)std::min<long long>(512, std::max<long long>(1, (n + 4095) / 4096));
  const long long chunk = (n + nparts - 1) / nparts;
  DBuf<double> part((size_t)nparts * ncol);
  launch(st, KC_OTHER, 0.0, 8.0 * n * ncol, KNAME0(k_col_sumsq_part), k_col_sumsq_part, dim3(nparts, ncol), dim3(256), 0, n, chunk, A,
         part.get());
  launch(st, KC_OTHER, 0.0, 0.0, KNAME0(k_col_sumsq_final), k_col_sumsq_final, dim3(ncol), dim3(256), 0, nparts, (const double*)part.get(),
         out);
}

void mdot(hipStream_t st, long long n, int nvec, const double* V, long long ldv, const double* w, double* out) {
  if (nvec <= 0) return;
  const int nparts = (int)std::min<long long>(512, std::max<long long>(1, (n + 4095) / 4096));
  const long long chunk = (n + nparts - 1) / nparts;
  DBuf<double> part((size_t)nparts * nvec);
  launch(st, KC_OTHER, 2.0 * n * nvec, 8.0 * n * (nvec + 1), KNAME0(k_mdot_part), k_mdot_part, dim3(nparts, nvec),
         dim3(256), 0, n, chunk, V, ldv, w, part.get());
  launch(st, KC_OTHER, 0.0, 0.0, KNAME0(k_col_sumsq_final), k_col_sumsq_final, dim3(nvec), dim3(256), 0, nparts,
         (const double*)part.get(), out);
}

void maxpy(hipStream_t st, long long n, int nvec, double a, double sc, const double* c, const double* V,
           long long ldv, double* w) {
  launch(st, KC_OTHER, 2.0 * n * nvec, 8.0 * n * (nvec + 2), KNAME0(k_maxpy), k_maxpy, dim3(grid1(n, 256, 16384)),
         dim3(256), 0, n, nvec, a, sc, c, V, ldv, w);
}

void gflag_nonfinite(hipStream_t st, std::vector<NFJob> jobs) {
  long long b0 = 0;
  double by = 0;
  std::vector<NFJob> use;
  for (auto J : jobs) {
    if (J.n <= 0) continue;
    J.per = (int)std::min<long long>((J.n + 255) / 256, 1024);
    J.block0 = b0;
    b0 += J.per;
    by += 8.0 * J.n;
    use.push_back(J);
  }
  if (use.empty()) return;
  const NFJob* dj = upload(use, st);
  launch(st, KC_OTHER, 0.0, by, KNAME0(k_count_nonfinite), k_count_nonfinite, dim3((unsigned)b0), dim3(256), 0, dj,
         (int)use.size());
}

template <typename T>
void scan_values(hipStream_t st, long long n, const T* a, bool* bad, double* amax) {
  *bad = false;
  *amax = 0.0;
  if (n <= 0) return;
  const unsigned g = grid1(n, 256, 1024);
  DBuf<int> flag(1);
  DBuf<double> mx(g);
  memset_async(flag.get(), 0, sizeof(int), st);
  launch(st, KC_OTHER, 0.0, (double)n * sizeof(T), KNAME_T(k_scan_values<T>), k_scan_values<T>, dim3(g), dim3(256), 0, n, a, flag.get(),
         mx.get());
  int hb = 0;
  std::vector<double> hm(g);
  Queue::get().flush();
  ACR_HIP(hipMemcpyAsync(&hb, flag.get(), sizeof(int), hipMemcpyDeviceToHost, st));
  ACR_HIP(hipMemcpyAsync(hm.data(), mx.get(), g * sizeof(double), hipMemcpyDeviceToHost, st));
  ACR_HIP(hipStreamSynchronize(st));
  *bad = hb != 0;
  for (double v : hm) *amax = std::max(*amax, v);
}
template void scan_values<float>(hipStream_t, long long, const float*, bool*, double*);
template void scan_values<double>(hipStream_t, long long, const double*, bool*, double*);

void axpy_d(hipStream_t st, long long n, const double* D, double* X) {
  launch(st, KC_OTHER, 0.0, 24.0 * n, KNAME0(k_axpy_d), k_axpy_d, dim3(grid1(n, 256, 16384)), dim3(256), 0, n, D, X);
}

#define INST(T)                                                                                   \
  template void gtridiag_inverse<T>(hipStream_t, std::vector<OpJob>);                              \
  template void gleaves_tridiag<T>(hipStream_t, std::vector<OpJob>);                               \
  template void grank1_factors<T>(hipStream_t, std::vector<OpJob>);                                \
  template void gplane_factors<T>(hipStream_t, std::vector<OpJob>);                                \
  template void ggather_diag<T>(hipStream_t, std::vector<OpJob>);                                  \
  template void ggemm<T>(hipStream_t, std::vector<GJob>, const std::vector<GSeg>&, int);          \
  template void ghmv<T>(hipStream_t, int, int, int, int, std::vector<MVJob>, const std::vector<MVTerm>&); \
  template void ghmv<T>(hipStream_t, std::vector<MVJob>, const std::vector<MVTerm>&);              \
  template HmvStep hmv_plan<T>(std::vector<MVJob>, const std::vector<MVTerm>&);                    \
  template void hmv_launch<T>(hipStream_t, const HmvStep&, const MVRed*, const MVTerm*, const MVJob*, T*); \
  template void gto_blocks<T>(hipStream_t, std::vector<VJob>);                                     \
  template void PBuilder::step<T>(std::vector<MVJob>, const std::vector<MVTerm>&);                \
  template void psolve_run<T>(hipStream_t, std::vector<PInst>, int, bool, int*, const std::vector<VJob>&, \
                              double, double);                                                     \
  template void gdense_blocks<T>(hipStream_t, std::vector<DenseJob>);                              \
  template void gdense_to_hodlr<T>(hipStream_t, std::vector<HJob>);                                \
  template void gfrom_blocks<T>(hipStream_t, std::vector<VJob>);                                   \
  template void gqr<T>(hipStream_t, std::vector<QJob>, int);                                      \
  template void grsvd<T>(hipStream_t, std::vector<SJob>);                                         \
  template void gapply_q<T>(hipStream_t, std::vector<AJob>);                                      \
  template void gcopy<T>(hipStream_t, std::vector<CJob>);                                         \
  template void bgemm<T>(hipStream_t, int, int, int, int, int, T, const BOp&, const BOp&, T,      \
                         const BOp&);                                                             \
  template void bqr_r<T>(hipStream_t, int, int, int, int, const BOp&, T*, T*, T*);                \
  template void bapply_q<T>(hipStream_t, int, int, int, int, int, const T*, const T*, const T*,   \
                            long long, int, const BOp&);                                          \
  template void brsvd<T>(hipStream_t, int, int, T*, T*, T*, int*, double, int);                   \
  template void bcopy<T>(hipStream_t, int, int, int, T, const BOp&, const BOp&);                  \
  template void badd<T>(hipStream_t, int, int, int, T, const BOp&, const BOp&);                   \
  template void fill<T>(hipStream_t, T*, size_t, T);                                              \
  template void bscale<T>(hipStream_t, int, int, int, int, const BOp&, const T*, int, int,        \
                          long long, long long, int, T);                                          \
  template void to_blocks<T>(hipStream_t, int, int, int, const double*, long long, T*);           \
  template void from_blocks<T>(hipStream_t, int, int, int, const T*, double*, long long);         \
  template void bdiag_axpy<T>(hipStream_t, int, int, int, T, const T*, int, int, const T*, int,   \
                              int, T*, int, int);

INST(float)
INST(double)
#undef INST

template void binverse<double, double>(hipStream_t, int, int, const double*, long long, double*,
                                       long long, int*);
template void ginverse<double, double>(hipStream_t, std::vector<IJob>);
template void ginverse<double, float>(hipStream_t, std::vector<IJob>);
template void ginverse<float, float>(hipStream_t, std::vector<IJob>);
template void binverse<float, float>(hipStream_t, int, int, const float*, long long, float*,
                                     long long, int*);

}  // namespace acr
