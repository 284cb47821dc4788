// Grouped GEMM on MFMA for the block-pair products of a fermionic
// contraction (Eq. standardcontract after the signed permutes): one launch
// covers every charge group. Each group g computes
//   C_g = alpha * op(A_g) op(B_g) (+ beta C_g)
// and either writes a plain row-major matrix or scatters straight into the
// block layout of the output tensor (row combos x column combos -> block).
//
// Arithmetic: FP64 (v_mfma_f64_16x16x4f64), FP32 (v_mfma_f32_16x16x4f32), or
// split BF16 (x = hi + lo, both BF16 rounded to nearest even; hi*hi + hi*lo +
// lo*hi on v_mfma_f32_16x16x32_bf16 with FP32 accumulation).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>

#include "common.h"

namespace ftn {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int GT = 256;  // threads per workgroup: 4 waves in a 2 x 2 grid

struct GemmLaunch {
  const GemmGroup* groups;
  int ngroups;
  int64_t ntiles;
  GemmScatter sc;
  double alpha, beta;
};

// tiles of one group are consecutive; consecutive tiles land on one XCD
__device__ inline int64_t xcd_tile(int64_t bid, int64_t nt) {
  if (nt < 8) return bid;
  int64_t x = bid & 7, i = bid >> 3;
  int64_t base = nt >> 3, rem = nt & 7;
  return x * base + (x < rem ? x : rem) + i;
}

// tile (tm, tn), tm <= tn, of index lt in the row-major upper triangle of an
// nt x nt tile grid
__device__ inline void tri_tile(int64_t lt, int64_t nt, int64_t& tm, int64_t& tn) {
  int64_t r = 0;
  while (lt >= nt - r) {
    lt -= nt - r;
    ++r;
  }
  tm = r;
  tn = r + lt;
}

__device__ inline int find_group(const GemmGroup* g, int ng, int64_t tile) {
  int lo = 0, hi = ng - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (g[mid].tile0 <= tile)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// largest i in [0, n) with v[i] <= x
__device__ inline int upper_index(const int64_t* v, int n, int64_t x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (v[mid] <= x)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <int BM, int BN>
struct EpiTab {
  int32_t rfi[BM];
  int64_t rlr[BM];
  int32_t cgj[BN];
  int64_t clc[BN];
  int64_t cnd[BN];
};

template <int BM, int BN>
__device__ inline void build_epi(EpiTab<BM, BN>& e, const GemmGroup& G, const GemmScatter& sc,
                                 int64_t m0, int64_t n0) {
  for (int r = threadIdx.x; r < BM; r += blockDim.x) {
    int64_t m = m0 + r;
    if (m < G.M) {
      int fi = upper_index(sc.rc_start + G.rc_base, G.nrc, m);
      e.rfi[r] = fi;
      e.rlr[r] = m - sc.rc_start[G.rc_base + fi];
    }
  }
  for (int c = threadIdx.x; c < BN; c += blockDim.x) {
    int64_t n = n0 + c;
    if (n < G.N) {
      int gj = upper_index(sc.cc_start + G.cc_base, G.ncc, n);
      e.cgj[c] = gj;
      e.clc[c] = n - sc.cc_start[G.cc_base + gj];
      e.cnd[c] = sc.cc_dim[G.cc_base + gj];
    }
  }
}

// ---------------------------------------------------------------------------
// FP64 / FP32 MFMA kernel: BM x BN tile per workgroup, 4 waves in a
// WGM x WGN grid, BK = 16. The next K slice is fetched into registers while
// the MFMAs consume the current one, and LDS is double-buffered, so each K
// step costs one barrier. LDS holds A as [k][m] and B as [k][n] (one padding
// column) so that the 16 lanes reading an MFMA operand column touch
// consecutive addresses and the global-to-LDS stores do not collide.
// Output modes per group: plain (alpha / beta), block scatter, or raw
// partial sums of a K slice into the split-K workspace; a group marked `neg`
// writes its product negated in each of them.
constexpr int GBK = 16;

template <typename T>
struct MfmaOp;
// Operand layout (both types): A[lane % 16][lane / 16], B[lane / 16][lane % 16].
// Accumulator item r of lane l holds column l % 16 and row
//   FP64: l / 16 + 4 r        FP32: 4 (l / 16) + r
// (measured with an in-bounds probe of the builtins on gfx950).
template <>
struct MfmaOp<double> {
  typedef d4 acc_t;
  __device__ static inline d4 run(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct MfmaOp<float> {
  typedef f4 acc_t;
  __device__ static inline f4 run(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};


template <typename T, int BM, int BN, int WGM, int WGN>
__global__ void __launch_bounds__(64 * WGM * WGN) k_gemm(GemmLaunch L, const T* __restrict__ A, const T* __restrict__ B,
                                             T* __restrict__ C, T* __restrict__ Wk) {
  constexpr int NT = 64 * WGM * WGN;  // threads
  typedef typename MfmaOp<T>::acc_t acc_t;
  constexpr int WM = BM / WGM, WN = BN / WGN;  // per-wave tile
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int NA = BM * GBK / NT, NB = BN * GBK / NT;
  static_assert(TM >= 1 && TN >= 1 && NA >= 1 && NB >= 1, "tile shape");
  __shared__ T As[2][GBK][BM + 1];
  __shared__ T Bs[2][GBK][BN + 1];
  __shared__ EpiTab<BM, BN> epi;
  __shared__ int s_g;

  const int64_t tile = xcd_tile(blockIdx.x, L.ntiles);
  if (threadIdx.x == 0) s_g = find_group(L.groups, L.ngroups, tile);
  __syncthreads();
  const GemmGroup G = L.groups[s_g];
  const int64_t lt = tile - G.tile0;
  int64_t tm = lt / G.ntn, tn = lt % G.ntn;
  if (G.sym) tri_tile(lt, G.ntn, tm, tn);
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const bool mirror = G.sym && G.scatter == 0 && tm != tn;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  const T* Ag = A + G.a_off;
  const T* Bg = B + G.b_off;

  // Operand loaders. A thread's share of the A slice is NA entries e = tid +
  // NT u: either 16 consecutive k of rows tid / 16 + 16 u (A row-major along k)
  // or consecutive m of k-rows tid / BM + (NT / BM) u (A stored transposed);
  // B likewise. Each entry is base + u su + kt sk; the masks for the fixed
  // dimension are computed once, and out-of-range entries load a valid
  // address and are zeroed (no branches in the K loop).
  const int t = threadIdx.x;
  int64_t a_base, a_su, a_sk, b_base, b_su, b_sk;
  int a_k0, a_ku, a_l0, a_lu, b_k0, b_ku, b_l0, b_lu;  // k of entry u, LDS column of entry u
  uint32_t a_ok = 0, b_ok = 0;
  if (!G.transA) {
    a_base = (m0 + t / GBK) * G.lda + t % GBK;
    a_su = (int64_t)(NT / GBK) * G.lda;
    a_sk = GBK;
    a_k0 = t % GBK;
    a_ku = 0;
    a_l0 = t / GBK;
    a_lu = NT / GBK;
#pragma unroll
    for (int u = 0; u < NA; ++u)
      if (m0 + a_l0 + a_lu * u < G.M) a_ok |= 1u << u;
  } else {
    a_base = (int64_t)(t / BM) * G.lda + m0 + t % BM;
    a_su = (int64_t)(NT / BM) * G.lda;
    a_sk = (int64_t)GBK * G.lda;
    a_k0 = t / BM;
    a_ku = NT / BM;
    a_l0 = t % BM;
    a_lu = 0;
    if (m0 + a_l0 < G.M) a_ok = ~0u;
  }
  if (!G.transB) {
    b_base = (int64_t)(t / BN) * G.ldb + n0 + t % BN;
    b_su = (int64_t)(NT / BN) * G.ldb;
    b_sk = (int64_t)GBK * G.ldb;
    b_k0 = t / BN;
    b_ku = NT / BN;
    b_l0 = t % BN;
    b_lu = 0;
    if (n0 + b_l0 < G.N) b_ok = ~0u;
  } else {
    b_base = (n0 + t / GBK) * G.ldb + t % GBK;
    b_su = (int64_t)(NT / GBK) * G.ldb;
    b_sk = GBK;
    b_k0 = t % GBK;
    b_ku = 0;
    b_l0 = t / GBK;
    b_lu = NT / GBK;
#pragma unroll
    for (int u = 0; u < NB; ++u)
      if (n0 + b_l0 + b_lu * u < G.N) b_ok |= 1u << u;
  }
  T ra[NA], rb[NB];
  auto fetch = [&](int64_t kt) {
    const int64_t k0 = kt * GBK;
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const bool ok = ((a_ok >> u) & 1u) && (k0 + a_k0 + a_ku * u < G.K);
      const int64_t off = a_base + u * a_su + kt * a_sk;
      const T v = Ag[ok ? off : 0];
      ra[u] = ok ? v : T(0);
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const bool ok = ((b_ok >> u) & 1u) && (k0 + b_k0 + b_ku * u < G.K);
      const int64_t off = b_base + u * b_su + kt * b_sk;
      const T v = Bg[ok ? off : 0];
      rb[u] = ok ? v : T(0);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int u = 0; u < NA; ++u) As[buf][a_k0 + a_ku * u][a_l0 + a_lu * u] = ra[u];
#pragma unroll
    for (int u = 0; u < NB; ++u) Bs[buf][b_k0 + b_ku * u][b_l0 + b_lu * u] = rb[u];
  };

  acc_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;

  const int64_t nk = (G.K + GBK - 1) / GBK;
  if (nk > 0) {
    fetch(0);
    stash(0);
  }
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = (int)(kt & 1);
    if (kt + 1 < nk) fetch(kt + 1);
#pragma unroll
    for (int kk = 0; kk < GBK; kk += 4) {
      T a[TM], b[TN];
      const int kr = kk + (lane >> 4), c = lane & 15;
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = As[cur][kr][wm * WM + 16 * i + c];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = Bs[cur][kr][wn * WN + 16 * j + c];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = MfmaOp<T>::run(a[i], b[j], acc[i][j]);
    }
    if (kt + 1 < nk) stash(cur ^ 1);
    __syncthreads();
  }

  if (G.scatter == 1) {
    build_epi<BM, BN>(epi, G, L.sc, m0, n0);
    __syncthreads();
  }
  const T alpha = (T)(G.neg ? -L.alpha : L.alpha), beta = (T)L.beta;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = wm * WM + 16 * i + MfmaOp<T>::row(lane, r);
        const int cc = wn * WN + 16 * j + (lane & 15);
        const int64_t m = m0 + rr, n = n0 + cc;
        if (m >= G.M || n >= G.N) continue;
        if (G.scatter == 1) {
          const int64_t bo = L.sc.boff[G.boff_base + (int64_t)epi.rfi[rr] * G.ncc + epi.cgj[cc]];
          if (bo >= 0) C[bo + epi.rlr[rr] * epi.cnd[cc] + epi.clc[cc]] = alpha * acc[i][j][r];
        } else if (G.scatter == 2) {
          Wk[G.c_off + m * G.ldc + n] = G.neg ? -acc[i][j][r] : acc[i][j][r];
        } else {
          const T v = alpha * acc[i][j][r];
          T* p = C + G.c_off + m * G.ldc + n;
          *p = beta != (T)0 ? v + beta * *p : v;
          if (mirror) {
            T* pt = C + G.c_off + n * G.ldc + m;
            *pt = beta != (T)0 ? v + beta * *pt : v;
          }
        }
      }
}

// split-K finish: C = alpha * (sum of the K-slice partials) (+ beta C)
template <typename T>
__global__ void k_splitk_reduce(const SplitRed* __restrict__ R, int nr, int64_t total, const T* __restrict__ Wk,
                                T* __restrict__ C, double alpha, double beta) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= total) return;
  int lo = 0, hi = nr - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (R[mid].e0 <= e)
      lo = mid;
    else
      hi = mid - 1;
  }
  const SplitRed r = R[lo];
  const int64_t loc = e - r.e0, mn = r.M * r.N;
  const int64_t m = loc / r.N, n = loc % r.N;
  const int64_t src = (r.sym && m > n) ? n * r.N + m : loc;
  T sum = T(0);
  for (int q = 0; q < r.S; ++q) sum += Wk[r.w_off + q * mn + src];
  T* p = C + r.c_off + m * r.ldc + n;
  const T v = (T)alpha * sum;
  *p = beta != 0.0 ? v + (T)beta * *p : v;
}

// ---------------------------------------------------------------------------
// split-BF16 x3 kernel (FP32 in and out). LDS holds hi/lo halves as [m][k]
// and [n][k] so that one lane's 8 consecutive k values are one 16-byte read.
template <int BM, int BN, int BK>
__global__ void __launch_bounds__(GT) k_gemm_bf16x3(GemmLaunch L, const float* __restrict__ A,
                                                    const float* __restrict__ B, float* __restrict__ C) {
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int KP = BK + 8;  // padded row (keeps 16-byte alignment)
  __shared__ __attribute__((aligned(16))) __bf16 Ah[BM][KP];
  __shared__ __attribute__((aligned(16))) __bf16 Al[BM][KP];
  __shared__ __attribute__((aligned(16))) __bf16 Bh[BN][KP];
  __shared__ __attribute__((aligned(16))) __bf16 Bl[BN][KP];
  __shared__ EpiTab<BM, BN> epi;
  __shared__ int s_g;

  const int64_t tile = xcd_tile(blockIdx.x, L.ntiles);
  if (threadIdx.x == 0) s_g = find_group(L.groups, L.ngroups, tile);
  __syncthreads();
  const GemmGroup G = L.groups[s_g];
  const int64_t lt = tile - G.tile0;
  const int64_t m0 = (lt / G.ntn) * BM, n0 = (lt % G.ntn) * BN;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  f4 acc[TM][TN];
  for (int i = 0; i < TM; ++i)
    for (int j = 0; j < TN; ++j)
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.f;

  const float* Ag = A + G.a_off;
  const float* Bg = B + G.b_off;
  for (int64_t k0 = 0; k0 < G.K; k0 += BK) {
    for (int e = threadIdx.x; e < BM * BK; e += GT) {
      int mm, kk;
      if (G.transA) {
        kk = e / BM;
        mm = e % BM;
      } else {
        mm = e / BK;
        kk = e % BK;
      }
      int64_t m = m0 + mm, k = k0 + kk;
      float v = 0.f;
      if (m < G.M && k < G.K) v = G.transA ? Ag[k * G.lda + m] : Ag[m * G.lda + k];
      __bf16 h = (__bf16)v;
      Ah[mm][kk] = h;
      Al[mm][kk] = (__bf16)(v - (float)h);
    }
    for (int e = threadIdx.x; e < BK * BN; e += GT) {
      int kk, nn;
      if (G.transB) {
        nn = e / BK;
        kk = e % BK;
      } else {
        kk = e / BN;
        nn = e % BN;
      }
      int64_t k = k0 + kk, n = n0 + nn;
      float v = 0.f;
      if (k < G.K && n < G.N) v = G.transB ? Bg[n * G.ldb + k] : Bg[k * G.ldb + n];
      __bf16 h = (__bf16)v;
      Bh[nn][kk] = h;
      Bl[nn][kk] = (__bf16)(v - (float)h);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {
      const int ko = kk + 8 * (lane >> 4), c = lane & 15;
      bf8 ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        ah[i] = *(const bf8*)&Ah[wm * WM + 16 * i + c][ko];
        al[i] = *(const bf8*)&Al[wm * WM + 16 * i + c][ko];
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        bh[j] = *(const bf8*)&Bh[wn * WN + 16 * j + c][ko];
        bl[j] = *(const bf8*)&Bl[wn * WN + 16 * j + c][ko];
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
  }

  if (G.scatter) {
    build_epi<BM, BN>(epi, G, L.sc, m0, n0);
    __syncthreads();
  }
  const float alpha = (float)(G.neg ? -L.alpha : L.alpha), beta = (float)L.beta;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = wm * WM + 16 * i + 4 * (lane >> 4) + r;
        const int cc = wn * WN + 16 * j + (lane & 15);
        const int64_t m = m0 + rr, n = n0 + cc;
        if (m >= G.M || n >= G.N) continue;
        float v = alpha * acc[i][j][r];
        if (G.scatter) {
          const int64_t bo = L.sc.boff[G.boff_base + (int64_t)epi.rfi[rr] * G.ncc + epi.cgj[cc]];
          if (bo >= 0) C[bo + epi.rlr[rr] * epi.cnd[cc] + epi.clc[cc]] = v;
        } else {
          float* p = C + G.c_off + m * G.ldc + n;
          *p = beta != 0.f ? v + beta * *p : v;
        }
      }
}

// ---------------------------------------------------------------------------
double gemm_flops(const std::vector<GemmGroup>& groups) {
  double f = 0;
  // a symmetric product is priced as its triangle: M (M + 1) K
  for (auto& g : groups)
    f += (g.sym ? (double)(g.M + 1) : 2.0 * (double)g.N) * (double)g.M * (double)g.K;
  return f;
}

constexpr int TBM = 64, TBN = 64;  // split-BF16 tile

// tile configurations of the FP64 / FP32 kernel
// ---------------------------------------------------------------------------
// Tall FP64 products C = alpha A B (+ beta C, or a block scatter) with A
// (M x K) and B (K x N) row-major, N <= 16, K <= 256 and M large: a tall
// factor times a small matrix, bound by streaming A once. The MFMA tiles
// above stage A through LDS, whose 64 KB per workgroup leave too few
// resident workgroups to keep HBM busy here. Instead B (at most 256 x 16)
// is the only LDS operand; each wave takes four 16-row tiles and feeds A to
// v_mfma_f64_16x16x4f64 straight from its registers: lane (r, g) = (lane %
// 16, lane / 16) loads the four consecutive entries k0 + 4g .. k0 + 4g + 3 of
// row r (two 16-byte loads, a 128-byte line per row across the four lane
// groups), and the four MFMAs of a 16-wide K step take them as their K slot
// g (the B operand is read from LDS in the same order). The loads of the
// next K step are issued before the MFMAs of the current one.
constexpr int TL_T = 256, TL_RT = 4, TL_BM = 16 * TL_RT * (TL_T / 64), TL_KMAX = 256, TL_N = 16;

template <bool VEC>
__global__ void __launch_bounds__(TL_T) k_gemm_tall(GemmLaunch L, const double* __restrict__ A,
                                                    const double* __restrict__ B, double* __restrict__ C) {
  __shared__ double Bs[TL_KMAX][TL_N];
  __shared__ EpiTab<TL_BM, TL_N> epi;
  __shared__ int s_g;
  const int64_t tile = xcd_tile(blockIdx.x, L.ntiles);
  if (threadIdx.x == 0) s_g = find_group(L.groups, L.ngroups, tile);
  __syncthreads();
  const GemmGroup G = L.groups[s_g];
  const int64_t mb = (tile - G.tile0) * TL_BM;
  const int K = (int)G.K, N = (int)G.N, kp = (K + 15) & ~15;
  for (int e = threadIdx.x; e < kp * TL_N; e += TL_T) {
    const int k = e / TL_N, n = e % TL_N;
    Bs[k][n] = k < K && n < N ? B[G.b_off + (int64_t)k * G.ldb + n] : 0.0;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, r = lane & 15, g = lane >> 4;
  const int64_t m0 = mb + 64 * w;
  const double* ap[TL_RT];
  bool rok[TL_RT];
#pragma unroll
  for (int t = 0; t < TL_RT; ++t) {
    const int64_t m = m0 + 16 * t + r;
    rok[t] = m < G.M;
    ap[t] = A + G.a_off + (rok[t] ? m : 0) * G.lda + 4 * g;
  }
  // entries k0 + 4g .. k0 + 4g + 3 of each of the lane's rows (zero past M or K)
  auto load = [&](double2 (&buf)[TL_RT][2], int k0) {
    const int k = k0 + 4 * g;
#pragma unroll
    for (int t = 0; t < TL_RT; ++t) {
      const double* q = ap[t] + k0;
      if constexpr (VEC) {  // K % 4 == 0 and every row start on a pair boundary
        if (rok[t] && k < K) {
          buf[t][0] = *(const double2*)q;
          buf[t][1] = *(const double2*)(q + 2);
        } else {
          buf[t][0] = buf[t][1] = double2{0.0, 0.0};
        }
      } else {
        buf[t][0].x = rok[t] && k < K ? q[0] : 0.0;
        buf[t][0].y = rok[t] && k + 1 < K ? q[1] : 0.0;
        buf[t][1].x = rok[t] && k + 2 < K ? q[2] : 0.0;
        buf[t][1].y = rok[t] && k + 3 < K ? q[3] : 0.0;
      }
    }
  };
  d4 acc[TL_RT];
#pragma unroll
  for (int t = 0; t < TL_RT; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
  double2 cur[TL_RT][2], nxt[TL_RT][2];
  load(cur, 0);
  __syncthreads();  // B in LDS
  const int nks = kp / 16;
  for (int ks = 0; ks < nks; ++ks) {
    if (ks + 1 < nks) load(nxt, 16 * (ks + 1));
    const int kb = 16 * ks + 4 * g;
    const double b0 = Bs[kb][r], b1 = Bs[kb + 1][r], b2 = Bs[kb + 2][r], b3 = Bs[kb + 3][r];
#pragma unroll
    for (int t = 0; t < TL_RT; ++t) {
      acc[t] = MfmaOp<double>::run(cur[t][0].x, b0, acc[t]);
      acc[t] = MfmaOp<double>::run(cur[t][0].y, b1, acc[t]);
      acc[t] = MfmaOp<double>::run(cur[t][1].x, b2, acc[t]);
      acc[t] = MfmaOp<double>::run(cur[t][1].y, b3, acc[t]);
    }
#pragma unroll
    for (int t = 0; t < TL_RT; ++t) {
      cur[t][0] = nxt[t][0];
      cur[t][1] = nxt[t][1];
    }
  }
  if (G.scatter == 1) {
    build_epi<TL_BM, TL_N>(epi, G, L.sc, mb, 0);
    __syncthreads();
  }
  const double alpha = G.neg ? -L.alpha : L.alpha, beta = L.beta;
  if (r >= N) return;
#pragma unroll
  for (int t = 0; t < TL_RT; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int rr = 64 * w + 16 * t + MfmaOp<double>::row(lane, i);
      const int64_t m = mb + rr;
      if (m >= G.M) continue;
      const double v = alpha * acc[t][i];
      if (G.scatter == 1) {
        const int64_t bo = L.sc.boff[G.boff_base + (int64_t)epi.rfi[rr] * G.ncc + epi.cgj[r]];
        if (bo >= 0) C[bo + epi.rlr[rr] * epi.cnd[r] + epi.clc[r]] = v;
      } else {
        double* p = C + G.c_off + m * G.ldc + r;
        *p = beta != 0.0 ? v + beta * *p : v;
      }
    }
}

// the tall kernel takes FP64 groups of plain or block-scatter output with
// A and B untransposed, N <= 16, K <= 256 and at least one tall A
static bool tall_form(const std::vector<GemmGroup>& gs, int kind) {
  if (kind != FTN_GEMM_F64) return false;
  bool tall = false;
  for (auto& g : gs) {
    if (g.M <= 0 || g.N <= 0) continue;
    if (g.transA || g.transB || g.sym || g.scatter == 2 || g.N > TL_N || g.K > TL_KMAX || g.K < 1) return false;
    if (g.M >= 4096) tall = true;
  }
  return tall;
}

enum { CFG_64 = 0, CFG_128 = 1, CFG_256x16 = 2, CFG_256x32 = 3, CFG_16x256 = 4, CFG_32x256 = 5, CFG_TALL = 6 };
static const int CFG_BM[] = {64, 128, 256, 256, 16, 32, TL_BM};
static const int CFG_BN[] = {64, 128, 16, 32, 256, 256, TL_N};
constexpr int NCU = 256;  // compute units to fill

static int choose_cfg(const std::vector<GemmGroup>& gs) {
  int64_t maxM = 0, maxN = 0, t128 = 0;
  for (auto& g : gs) {
    maxM = std::max(maxM, g.M);
    maxN = std::max(maxN, g.N);
    const int64_t a = cdiv(g.M, 128);
    t128 += (g.sym && g.M == g.N) ? a * (a + 1) / 2 : a * cdiv(g.N, 128);
  }
  if (maxN <= 16 && maxM >= 256) return CFG_256x16;
  if (maxN <= 32 && maxM >= 256) return CFG_256x32;
  if (maxM <= 16 && maxN >= 256) return CFG_16x256;
  if (maxM <= 32 && maxN >= 256) return CFG_32x256;
  if (t128 >= NCU && std::min(maxM, maxN) >= 128) return CFG_128;
  return CFG_64;
}

int gemm_ncfg() { return 6; }

void gemm_plan(GemmPlan& p, const std::vector<GemmGroup>& groups, int kind, hipStream_t s, bool persistent) {
  std::vector<GemmGroup> gs;
  for (auto& g : groups)
    if (g.M > 0 && g.N > 0) gs.push_back(g);
  int cfg = -1, split = -1;
  if (tall_form(gs, kind))
    cfg = CFG_TALL;  // not a tuning choice: the tall kernel is the streaming bound
  else if (kind != FTN_GEMM_BF16X3 && !gs.empty())
    tune_choice(gs, kind, s, &cfg, &split);
  gemm_plan_with(p, gs, kind, s, persistent, cfg, split);
}

void gemm_plan_with(GemmPlan& p, const std::vector<GemmGroup>& groups, int kind, hipStream_t s,
                    bool persistent, int cfg_override, int split_override) {
  p.host.clear();
  p.red_host.clear();
  p.kind = kind;
  p.ws_elems = 0;
  p.flops = 0;
  std::vector<GemmGroup> gs;
  for (auto& g : groups)
    if (g.M > 0 && g.N > 0) gs.push_back(g);
  p.flops = gemm_flops(gs);
  p.abytes = 0;
  for (auto& g : gs) p.abytes += (double)(g.M * g.K + g.K * g.N + g.M * g.N);
  p.cfg = kind == FTN_GEMM_BF16X3 ? CFG_64 : (cfg_override >= 0 ? cfg_override : choose_cfg(gs));
  const int bm = kind == FTN_GEMM_BF16X3 ? TBM : CFG_BM[p.cfg], bn = kind == FTN_GEMM_BF16X3 ? TBN : CFG_BN[p.cfg];
  // the triangle of tiles needs square tiles, a square product and a plain
  // output (the split-BF16 kernel multiplies the full grid)
  for (auto& g : gs)
    if (g.sym && (kind == FTN_GEMM_BF16X3 || bm != bn || g.M != g.N || g.scatter == 1)) g.sym = 0;
  auto ntiles_of = [&](const GemmGroup& g) {
    const int64_t a = cdiv(g.M, bm), b = cdiv(g.N, bn);
    return g.sym ? a * (a + 1) / 2 : a * b;
  };
  int64_t tiles = 0;
  for (auto& g : gs) tiles += ntiles_of(g);
  // split-K for plain outputs when the tiles alone give fewer than four
  // workgroups per compute unit: more resident workgroups hide the latency
  // of the K loop, and the partial sums cost one extra pass over C
  int64_t split = 1;
  if (kind != FTN_GEMM_BF16X3 && tiles > 0 && tiles < 4 * NCU) split = std::max<int64_t>(1, cdiv(8 * NCU, tiles));
  if (kind != FTN_GEMM_BF16X3 && split_override >= 1) split = split_override;
  if (p.cfg == CFG_TALL) {
    if (!tall_form(gs, kind)) fail(FTN_EINVAL, "tall GEMM configuration for groups it does not take");
    split = 1;  // K <= 256: one pass
  }
  p.split = split;
  int64_t t = 0;
  for (auto g : gs) {
    const int64_t S = g.scatter ? 1 : std::min<int64_t>(split, std::min<int64_t>(256, g.K / 128));
    g.ntm = cdiv(g.M, bm);
    g.ntn = cdiv(g.N, bn);
    if (S <= 1) {
      g.tile0 = t;
      t += ntiles_of(g);
      p.host.push_back(g);
      continue;
    }
    const int64_t kc = cdiv(cdiv(g.K, S), GBK) * GBK;
    const int64_t ns = cdiv(g.K, kc);
    SplitRed r;
    std::memset(&r, 0, sizeof(r));
    r.M = g.M;
    r.N = g.N;
    r.c_off = g.c_off;
    r.ldc = g.ldc;
    r.w_off = p.ws_elems;
    r.S = (int)ns;
    r.sym = g.sym;
    p.red_host.push_back(r);
    for (int64_t q = 0; q < ns; ++q) {
      GemmGroup h = g;
      const int64_t k0 = q * kc;
      h.K = std::min(kc, g.K - k0);
      h.a_off = g.a_off + (g.transA ? k0 * g.lda : k0);
      h.b_off = g.b_off + (g.transB ? k0 : k0 * g.ldb);
      h.scatter = 2;
      h.c_off = p.ws_elems + q * g.M * g.N;
      h.ldc = g.N;
      h.tile0 = t;
      t += ntiles_of(h);
      p.host.push_back(h);
    }
    p.ws_elems += ns * g.M * g.N;
  }
  int64_t e0 = 0;
  for (auto& r : p.red_host) {
    r.e0 = e0;
    e0 += r.M * r.N;
  }
  p.red_elems = e0;
  if (t > 0x7fffffffLL) fail(FTN_EINVAL, "GEMM too large");
  p.ntiles = t;
  p.groups = persistent ? persist<GemmGroup>(p.host.size()) : DBuf<GemmGroup>(p.host.size(), s);
  if (!p.host.empty())
    h2d(p.groups.p, p.host.data(), p.host.size() * sizeof(GemmGroup), s);
  p.red = persistent ? persist<SplitRed>(p.red_host.size()) : DBuf<SplitRed>(p.red_host.size(), s);
  if (!p.red_host.empty())
    h2d(p.red.p, p.red_host.data(), p.red_host.size() * sizeof(SplitRed), s);
}

template <typename T>
static void launch_cfg(int cfg, dim3 grid, hipStream_t s, const GemmLaunch& L, const T* A, const T* B, T* C, T* W,
                       hipEvent_t e0, hipEvent_t e1) {
  switch (cfg) {
    case CFG_128:
      ELAUNCH((k_gemm<T, 128, 128, 2, 4>), grid, dim3(512), 0, s, e0, e1, L, A, B, C, W);
      break;
    case CFG_256x16:
      ELAUNCH((k_gemm<T, 256, 16, 4, 1>), grid, dim3(GT), 0, s, e0, e1, L, A, B, C, W);
      break;
    case CFG_256x32:
      ELAUNCH((k_gemm<T, 256, 32, 4, 1>), grid, dim3(GT), 0, s, e0, e1, L, A, B, C, W);
      break;
    case CFG_16x256:
      ELAUNCH((k_gemm<T, 16, 256, 1, 4>), grid, dim3(GT), 0, s, e0, e1, L, A, B, C, W);
      break;
    case CFG_32x256:
      ELAUNCH((k_gemm<T, 32, 256, 1, 4>), grid, dim3(GT), 0, s, e0, e1, L, A, B, C, W);
      break;
    default:
      ELAUNCH((k_gemm<T, 64, 64, 2, 2>), grid, dim3(GT), 0, s, e0, e1, L, A, B, C, W);
      break;
  }
}

void run_gemm(const GemmPlan& p, int dtype, const void* A, const void* B, void* C,
              const GemmScatter* sc, hipStream_t s, double alpha, double beta, void* ws_ext) {
  if (p.ntiles == 0) return;
  GemmLaunch L;
  L.groups = p.groups.p;
  L.ngroups = (int)p.host.size();
  L.ntiles = p.ntiles;
  L.alpha = alpha;
  L.beta = beta;
  std::memset(&L.sc, 0, sizeof(L.sc));
  if (sc) L.sc = *sc;
  dim3 grid((unsigned)p.ntiles);
  // FTN_TRACE_GEMM: one line per launch; FTN_TRACE_GEMM=2 also times it
  // (synchronising the stream around the launch)
  static const char* trace_env = std::getenv("FTN_TRACE_GEMM");
  static const bool trace = trace_env != nullptr;
  static const bool trace_time = trace && trace_env[0] == '2';
  hipEvent_t te0 = nullptr, te1 = nullptr;
  if (trace_time) {
    HIPC(hipEventCreate(&te0));
    HIPC(hipEventCreate(&te1));
    HIPC(hipEventRecord(te0, s));
  }
  if (trace && !trace_time) {
    int64_t mm = 0, mn = 0, mk = 0;
    for (auto& g : p.host) {
      mm = std::max(mm, g.M);
      mn = std::max(mn, g.N);
      mk = std::max(mk, g.K);
    }
    std::fprintf(stderr, "[gemm] tiles %lld groups %zu flops %.4g bytes %.4g maxM %lld maxN %lld maxK %lld ta %d tb %d sc %d cfg %d split %zu\n",
                 (long long)p.ntiles, p.host.size(), p.flops, p.abytes * (dtype == FTN_F64 ? 8.0 : 4.0), (long long)mm,
                 (long long)mn, (long long)mk,
                 p.host[0].transA, p.host[0].transB, p.host[0].scatter, p.cfg, p.red_host.size());
  }
  const size_t es = dtype == FTN_F64 ? 8 : 4;
  DBuf<char> ws_own(ws_ext ? 0 : p.ws_elems * es, s);
  char* wsp = ws_ext ? (char*)ws_ext : ws_own.p;
  void* tok = prof_begin(s);
  if (p.kind == FTN_GEMM_F64 && p.cfg == CFG_TALL) {
    if (dtype != FTN_F64) fail(FTN_ENOTSUP, "FP64 GEMM needs FP64 tensors");
    // pair loads of A: K a multiple of 4 and every row start 16-byte aligned
    bool vec = ((uintptr_t)A & 15) == 0;
    for (auto& g : p.host) vec = vec && g.K % 4 == 0 && g.lda % 2 == 0 && g.a_off % 2 == 0;
    if (vec)
      ELAUNCH((k_gemm_tall<true>), grid, dim3(TL_T), 0, s, prof_ev(tok, 0), prof_ev(tok, 1), L, (const double*)A,
              (const double*)B, (double*)C);
    else
      ELAUNCH((k_gemm_tall<false>), grid, dim3(TL_T), 0, s, prof_ev(tok, 0), prof_ev(tok, 1), L, (const double*)A,
              (const double*)B, (double*)C);
    HIPC(hipGetLastError());
    prof_end(tok, s, FTN_PROF_K_GEMM_F64_TALL, p.flops, p.abytes * (double)es);
    tok = nullptr;
  } else if (p.kind == FTN_GEMM_F64) {
    if (dtype != FTN_F64) fail(FTN_ENOTSUP, "FP64 GEMM needs FP64 tensors");
    launch_cfg<double>(p.cfg, grid, s, L, (const double*)A, (const double*)B, (double*)C, (double*)wsp,
                       prof_ev(tok, 0), prof_ev(tok, 1));
    HIPC(hipGetLastError());
    // the GEMM kernel and the reduction are timed apart (per-kernel classes)
    prof_end(tok, s, FTN_PROF_K_GEMM_F64_64x64 + p.cfg, p.flops, p.abytes * (double)es);
    tok = nullptr;
    if (p.red_elems) {
      double rb = 0;  // partials read, output written (and read when accumulating)
      for (auto& r : p.red_host) rb += (double)r.M * r.N * (r.S + 1 + (beta != 0.0 ? 1 : 0)) * es;
      void* tr = prof_begin(s);
      ELAUNCH((k_splitk_reduce<double>), dim3((unsigned)cdiv(p.red_elems, 256)), dim3(256), 0, s, prof_ev(tr, 0),
              prof_ev(tr, 1), p.red.p, (int)p.red_host.size(), p.red_elems, (const double*)wsp, (double*)C, alpha,
              beta);
      prof_end(tr, s, FTN_PROF_K_SPLITK_F64, rb, rb);
    }
  } else if (p.kind == FTN_GEMM_F32) {
    if (dtype != FTN_F32) fail(FTN_ENOTSUP, "FP32 GEMM needs FP32 tensors");
    // one timed call: the GEMM kernel's start to the reduction's end
    launch_cfg<float>(p.cfg, grid, s, L, (const float*)A, (const float*)B, (float*)C, (float*)wsp, prof_ev(tok, 0),
                      p.red_elems ? nullptr : prof_ev(tok, 1));
    if (p.red_elems)
      ELAUNCH((k_splitk_reduce<float>), dim3((unsigned)cdiv(p.red_elems, 256)), dim3(256), 0, s, nullptr,
              prof_ev(tok, 1), p.red.p, (int)p.red_host.size(), p.red_elems, (const float*)wsp, (float*)C, alpha,
              beta);
  } else if (p.kind == FTN_GEMM_BF16X3) {
    if (dtype != FTN_F32) fail(FTN_ENOTSUP, "split-BF16 GEMM needs FP32 tensors");
    ELAUNCH((k_gemm_bf16x3<TBM, TBN, 32>), grid, dim3(GT), 0, s, prof_ev(tok, 0), prof_ev(tok, 1), L,
            (const float*)A, (const float*)B, (float*)C);
  } else {
    fail(FTN_EINVAL, "unknown GEMM kind");
  }
  HIPC(hipGetLastError());
  if (tok) prof_end(tok, s, p.kind == FTN_GEMM_F32 ? FTN_PROF_GEMM_F32 : FTN_PROF_GEMM_BF16X3, p.flops,
                    p.abytes * (double)es);
  if (trace_time) {
    HIPC(hipEventRecord(te1, s));
    HIPC(hipEventSynchronize(te1));
    float ms = 0;
    HIPC(hipEventElapsedTime(&ms, te0, te1));
    int64_t mm = 0, mn = 0, mk = 0;
    for (auto& g : p.host) {
      mm = std::max(mm, g.M);
      mn = std::max(mn, g.N);
      mk = std::max(mk, g.K);
    }
    std::fprintf(stderr, "[gemm] us %.1f tflops %.2f tiles %lld groups %zu flops %.4g bytes %.4g maxM %lld maxN %lld maxK %lld ta %d tb %d sym %d sc %d cfg %d split %lld\n",
                 1000.0 * ms, ms > 0 ? p.flops / (ms * 1e-3) / 1e12 : 0.0, (long long)p.ntiles, p.host.size(), p.flops,
                 p.abytes * (double)es, (long long)mm, (long long)mn, (long long)mk, p.host[0].transA, p.host[0].transB, p.host[0].sym,
                 p.host[0].scatter, p.cfg, (long long)p.split);
    (void)hipEventDestroy(te0);
    (void)hipEventDestroy(te1);
  }
}

// ---------------------------------------------------------------------------
// Tall-skinny products C = alpha op(A)^T B (+ beta C), A (K x M) and B (K x N)
// row-major with M, N <= 32 and a long K: the Gram matrices of tall thin
// factors. They are bound by reading A and B once; MFMA tiles of 64 x 64
// would leave nearly all of their work and loads idle. C is cut into 8 x 8
// parts; each thread owns one part (64 accumulators in registers) and a
// stride of rows of its workgroup's chunk of K, reading its eight entries of
// A and of B per row straight from memory. The threads of one part are
// summed by a fixed butterfly across the wavefront and then across the
// workgroup's waves in LDS; the chunks' partial C go to a workspace that a
// second kernel sums in a fixed order into C, so results are deterministic.
constexpr int SK_T = 256, SK_MAX = 32, SK_P = 8;

struct SkinnyGroup {
  int64_t M, N, K, a_off, lda, b_off, ldb, c_off, ldc, w_off, kc;
  int chunks, pp;  // chunks of K; parts of C rounded up to a power of two
  int same, pad;   // B is A (same matrix, offsets and strides): diagonal parts load one row
};

template <typename T>
struct Pair2;
template <>
struct Pair2<double> {
  using type = double2;
};
template <>
struct Pair2<float> {
  using type = float2;
};

// eight entries of a row; VEC: as four aligned pairs (the host checked the
// alignment of every row start), else one by one with entries past `lim`
// read as zero
template <typename T, bool VEC>
__device__ __forceinline__ void skinny_row(T (&x)[SK_P], const T* p, int lim) {
  if constexpr (VEC) {
    using P2 = typename Pair2<T>::type;
#pragma unroll
    for (int a = 0; a < SK_P / 2; ++a) {
      const P2 v = reinterpret_cast<const P2*>(p)[a];
      x[2 * a] = v.x;
      x[2 * a + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int a = 0; a < SK_P; ++a) x[a] = a < lim ? p[a] : T(0);
  }
}

template <typename T, bool VEC>
__global__ void __launch_bounds__(SK_T) k_skinny_atb(const SkinnyGroup* gs, const T* __restrict__ A,
                                                     const T* __restrict__ B, T* __restrict__ W) {
  const SkinnyGroup G = gs[blockIdx.y];
  const int ch = blockIdx.x;
  if (ch >= G.chunks) return;
  __shared__ T red[SK_T / 64][(SK_MAX / SK_P) * (SK_MAX / SK_P)][SK_P * SK_P];
  const int m = (int)G.M, n = (int)G.N, t = threadIdx.x, pp = G.pp;
  const int pn = (n + SK_P - 1) / SK_P, np = ((m + SK_P - 1) / SK_P) * pn;
  const int part = t % pp, lane_rows = SK_T / pp, rl = t / pp;
  const int i0 = (part / pn) * SK_P, j0 = (part % pn) * SK_P;
  const bool act = part < np;
  T acc[SK_P][SK_P];
#pragma unroll
  for (int a = 0; a < SK_P; ++a)
#pragma unroll
    for (int b = 0; b < SK_P; ++b) acc[a][b] = T(0);
  const int64_t k0 = (int64_t)ch * G.kc, k1 = k0 + G.kc < G.K ? k0 + G.kc : G.K;
  if (act) {
    const T* pa = A + G.a_off + i0;
    const T* pb = B + G.b_off + j0;
    const bool diag = G.same && i0 == j0;
#pragma unroll 2
    for (int64_t r = k0 + rl; r < k1; r += lane_rows) {
      T xa[SK_P], xb[SK_P];
      skinny_row<T, VEC>(xa, pa + r * G.lda, m - i0);
      if (diag) {
#pragma unroll
        for (int b = 0; b < SK_P; ++b) xb[b] = xa[b];
      } else {
        skinny_row<T, VEC>(xb, pb + r * G.ldb, n - j0);
      }
#pragma unroll
      for (int a = 0; a < SK_P; ++a)
#pragma unroll
        for (int b = 0; b < SK_P; ++b) acc[a][b] += xa[a] * xb[b];
    }
  }
  // lanes of one part sit pp apart within a wavefront (pp divides 64)
  for (int off = pp; off < 64; off <<= 1)
#pragma unroll
    for (int a = 0; a < SK_P; ++a)
#pragma unroll
      for (int b = 0; b < SK_P; ++b) acc[a][b] += __shfl_xor(acc[a][b], off, 64);
  const int wv = t / 64, ln = t % 64;
  if (ln < pp && act) {
#pragma unroll
    for (int a = 0; a < SK_P; ++a)
#pragma unroll
      for (int b = 0; b < SK_P; ++b) red[wv][part][a * SK_P + b] = acc[a][b];
  }
  __syncthreads();
  const int mn = m * n;
  T* w = W + G.w_off + (int64_t)ch * mn;
  for (int e = t; e < mn; e += SK_T) {
    const int i = e / n, j = e - i * n;
    const int pt = (i / SK_P) * pn + j / SK_P, sl = (i % SK_P) * SK_P + j % SK_P;
    T s = red[0][pt][sl];
    for (int u = 1; u < SK_T / 64; ++u) s += red[u][pt][sl];
    w[e] = s;
  }
}

// one wavefront per entry of C: lane l sums the chunks l, l + 64, ... (four
// loads in flight), then a fixed butterfly across the wavefront
template <typename T>
__global__ void __launch_bounds__(256) k_skinny_reduce(const SkinnyGroup* gs, const T* __restrict__ W,
                                                       T* __restrict__ C, double alpha, double beta) {
  const SkinnyGroup G = gs[blockIdx.y];
  const int mn = (int)(G.M * G.N), ln = threadIdx.x % 64;
  const int e = blockIdx.x * 4 + threadIdx.x / 64;
  if (e >= mn) return;  // whole wavefronts leave together
  const T* w = W + G.w_off + e;
  T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
  int c = ln;
  for (; c + 192 < G.chunks; c += 256) {
    s0 += w[(int64_t)c * mn];
    s1 += w[(int64_t)(c + 64) * mn];
    s2 += w[(int64_t)(c + 128) * mn];
    s3 += w[(int64_t)(c + 192) * mn];
  }
  for (; c < G.chunks; c += 64) s0 += w[(int64_t)c * mn];
  T s = (s0 + s1) + (s2 + s3);
  for (int off = 1; off < 64; off <<= 1) s += __shfl_xor(s, off, 64);
  if (ln == 0) {
    const int i = e / (int)G.N, j = e - i * (int)G.N;
    T* p = C + G.c_off + i * G.ldc + j;
    *p = beta != 0.0 ? (T)alpha * s + (T)beta * *p : (T)alpha * s;
  }
}

// groups all of the tall-skinny A^T B form (plain outputs), at least one of
// them with a long K
static bool skinny_form(const std::vector<GemmGroup>& gs) {
  bool any = false;
  for (auto& g : gs) {
    if (g.M <= 0 || g.N <= 0) continue;
    if (!g.transA || g.transB || g.scatter || g.neg || g.M > SK_MAX || g.N > SK_MAX) return false;
    if (g.K >= 1024) any = true;
  }
  return any;
}

template <typename T>
static void run_skinny(const std::vector<GemmGroup>& gs, const T* A, const T* B, T* C, hipStream_t s,
                       double alpha, double beta, int cls, double flops) {
  std::vector<SkinnyGroup> sg;
  int64_t ws = 0, tot_k = 0;
  int maxch = 1;
  bool vec = ((uintptr_t)A % (2 * sizeof(T))) == 0 && ((uintptr_t)B % (2 * sizeof(T))) == 0;
  for (auto& g : gs)
    if (g.M > 0 && g.N > 0) tot_k += g.K;
  for (auto& g : gs) {
    if (g.M <= 0 || g.N <= 0) continue;
    SkinnyGroup x;
    x.M = g.M;
    x.N = g.N;
    x.K = g.K;
    x.a_off = g.a_off;
    x.lda = g.lda;
    x.b_off = g.b_off;
    x.ldb = g.ldb;
    x.c_off = g.c_off;
    x.ldc = g.ldc;
    // about 2048 workgroups over all groups, chunks of at least 1024 rows
    const int64_t want = std::max<int64_t>(1, (int64_t)(2048.0 * (double)g.K / (double)std::max<int64_t>(tot_k, 1)));
    x.chunks = (int)std::min<int64_t>(want, std::max<int64_t>(1, g.K / 1024));
    x.kc = std::max<int64_t>(1, cdiv(g.K, x.chunks));
    x.chunks = g.K > 0 ? (int)cdiv(g.K, x.kc) : 1;
    x.w_off = ws;
    ws += (int64_t)x.chunks * g.M * g.N;
    const int np = (int)(cdiv(g.M, SK_P) * cdiv(g.N, SK_P));
    x.pp = 1;
    while (x.pp < np) x.pp <<= 1;
    x.same = (const void*)A == (const void*)B && g.a_off == g.b_off && g.lda == g.ldb ? 1 : 0;
    x.pad = 0;
    // pair loads: whole parts of 8 and every row start on a pair boundary
    vec = vec && g.M % SK_P == 0 && g.N % SK_P == 0 && g.lda % 2 == 0 && g.ldb % 2 == 0 && g.a_off % 2 == 0 &&
          g.b_off % 2 == 0;
    maxch = std::max(maxch, x.chunks);
    sg.push_back(x);
  }
  if (sg.empty()) return;
  DBuf<SkinnyGroup> d = to_device(sg, s);
  DBuf<T> W(ws, s);
  // FTN_TRACE_GEMM=2: one timed line per launch (synchronising the stream)
  static const char* trace_env = std::getenv("FTN_TRACE_GEMM");
  static const bool trace_time = trace_env && trace_env[0] == '2';
  hipEvent_t te0 = nullptr, te1 = nullptr;
  if (trace_time) {
    HIPC(hipEventCreate(&te0));
    HIPC(hipEventCreate(&te1));
    HIPC(hipEventRecord(te0, s));
  }
  void* tok = prof_begin(s);
  if (vec)
    ELAUNCH((k_skinny_atb<T, true>), dim3((unsigned)maxch, (unsigned)sg.size()), dim3(SK_T), 0, s, prof_ev(tok, 0),
            nullptr, d.p, A, B, W.p);
  else
    ELAUNCH((k_skinny_atb<T, false>), dim3((unsigned)maxch, (unsigned)sg.size()), dim3(SK_T), 0, s, prof_ev(tok, 0),
            nullptr, d.p, A, B, W.p);
  int64_t max_mn = 1;
  for (auto& g : sg) max_mn = std::max(max_mn, g.M * g.N);
  ELAUNCH((k_skinny_reduce<T>), dim3((unsigned)cdiv(max_mn, 4), (unsigned)sg.size()), dim3(256), 0, s, nullptr,
          prof_ev(tok, 1), d.p, W.p, C, alpha, beta);
  // algorithmic bytes: A and B read once (once in all when they are the same
  // matrix, as for a Gram matrix), C written
  double ab = 0;
  for (auto& g : sg) {
    ab += (double)(g.K * (g.same && g.M == g.N ? g.M : g.M + g.N) + g.M * g.N);
  }
  prof_end(tok, s, cls, flops, ab * sizeof(T));
  if (trace_time) {
    HIPC(hipEventRecord(te1, s));
    HIPC(hipEventSynchronize(te1));
    float ms = 0;
    HIPC(hipEventElapsedTime(&ms, te0, te1));
    int64_t mm = 0, mn = 0, mk = 0;
    for (auto& g : sg) {
      mm = std::max(mm, g.M);
      mn = std::max(mn, g.N);
      mk = std::max(mk, g.K);
    }
    std::fprintf(stderr, "[skinny] us %.1f GB/s %.1f groups %zu blocks %d bytes %.4g maxM %lld maxN %lld maxK %lld\n",
                 1000.0 * ms, ms > 0 ? ab * sizeof(T) / (ms * 1e-3) / 1e9 : 0.0, sg.size(), maxch, ab * sizeof(T),
                 (long long)mm, (long long)mn, (long long)mk);
    HIPC(hipEventDestroy(te0));
    HIPC(hipEventDestroy(te1));
  }
}

// Plans of the grouped products issued by the factorisations are cached by
// the groups' shapes and offsets (which are relative to the operand base
// pointers, so a repeated step meets the same keys): a hit costs no host
// planning and no upload of the group tables. Cached plans keep their tables
// in device memory of their own; a plan is complete on the device before it
// is cached, since another stream may use it next.
namespace {
std::mutex g_gp_mu;
auto& g_gp = *new std::unordered_map<std::string, std::shared_ptr<const GemmPlan>>();
constexpr size_t GP_CACHE_MAX = 8192;

std::string groups_key(const std::vector<GemmGroup>& gs, int kind) {
  std::string k;
  k.reserve(8 + gs.size() * 18 * 8);
  auto put = [&](int64_t v) { k.append(reinterpret_cast<const char*>(&v), sizeof(v)); };
  put(kind);
  for (const GemmGroup& g : gs) {
    put(g.M);
    put(g.N);
    put(g.K);
    put(g.a_off);
    put(g.b_off);
    put(g.lda);
    put(g.ldb);
    put(g.transA);
    put(g.transB);
    put(g.c_off);
    put(g.ldc);
    put(g.scatter);
    put(g.sym);
    put(g.neg);
    if (g.scatter == 1) {
      put(g.nrc);
      put(g.ncc);
      put(g.rc_base);
      put(g.cc_base);
      put(g.boff_base);
    }
  }
  return k;
}
}  // namespace

std::shared_ptr<const GemmPlan> gemm_plan_cached(const std::vector<GemmGroup>& groups, int kind, hipStream_t s) {
  const std::string key = groups_key(groups, kind);
  {
    std::lock_guard<std::mutex> g(g_gp_mu);
    auto it = g_gp.find(key);
    if (it != g_gp.end()) return it->second;
  }
  auto P = std::make_shared<GemmPlan>();
  gemm_plan(*P, groups, kind, s, true);
  HIPC(hipStreamSynchronize(s));
  std::lock_guard<std::mutex> g(g_gp_mu);
  if (g_gp.size() >= GP_CACHE_MAX) g_gp.clear();
  return g_gp.try_emplace(key, std::move(P)).first->second;
}

void run_grouped_gemm(int gemm, int dtype, const std::vector<GemmGroup>& groups, const void* A,
                      const void* B, void* C, const GemmScatter* sc, hipStream_t s, double alpha,
                      double beta) {
  if (!sc && gemm != FTN_GEMM_BF16X3 && skinny_form(groups)) {
    double fl = 0;
    for (auto& g : groups)
      if (g.M > 0 && g.N > 0) fl += 2.0 * (double)g.M * g.N * g.K;
    if (gemm == FTN_GEMM_F64) {
      if (dtype != FTN_F64) fail(FTN_ENOTSUP, "FP64 GEMM needs FP64 tensors");
      run_skinny<double>(groups, (const double*)A, (const double*)B, (double*)C, s, alpha, beta,
                         FTN_PROF_K_SKINNY_F64, fl);
    } else {
      if (dtype != FTN_F32) fail(FTN_ENOTSUP, "FP32 GEMM needs FP32 tensors");
      run_skinny<float>(groups, (const float*)A, (const float*)B, (float*)C, s, alpha, beta, FTN_PROF_GEMM_F32,
                        fl);
    }
    return;
  }
  const std::shared_ptr<const GemmPlan> p = gemm_plan_cached(groups, gemm, s);
  run_gemm(*p, dtype, A, B, C, sc, s, alpha, beta);
}

}  // namespace ftn
