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
  for (int r = threadIdx.x; r < BM; r += GT) {
    int64_t m = m0 + r;
    if (m < G.M) {
      int fi = upper_index(sc.rc_start + G.rc_base, G.nrc, m);
      e.rfi[r] = fi;
      e.rlr[r] = m - sc.rc_start[G.rc_base + fi];
    }
  }
  for (int c = threadIdx.x; c < BN; c += GT) {
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
// FP64 / FP32 MFMA kernel. LDS holds A as [k][m] and B as [k][n] so that the
// 16 lanes reading one MFMA operand column touch consecutive addresses.
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

template <typename T, int BM, int BN, int BK>
__global__ void __launch_bounds__(GT) k_gemm(GemmLaunch L, const T* __restrict__ A, const T* __restrict__ B,
                                             T* __restrict__ C) {
  typedef typename MfmaOp<T>::acc_t acc_t;
  constexpr int WM = BM / 2, WN = BN / 2;  // per-wave tile
  constexpr int TM = WM / 16, TN = WN / 16;
  __shared__ T As[BK][BM + 1];
  __shared__ T Bs[BK][BN + 1];
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

  acc_t acc[TM][TN];
  for (int i = 0; i < TM; ++i)
    for (int j = 0; j < TN; ++j)
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;

  const T* Ag = A + G.a_off;
  const T* Bg = B + G.b_off;
  for (int64_t k0 = 0; k0 < G.K; k0 += BK) {
    // A tile: element (m, k)
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
      T v = 0;
      if (m < G.M && k < G.K) v = G.transA ? Ag[k * G.lda + m] : Ag[m * G.lda + k];
      As[kk][mm] = v;
    }
    // B tile: element (k, n)
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
      T v = 0;
      if (k < G.K && n < G.N) v = G.transB ? Bg[n * G.ldb + k] : Bg[k * G.ldb + n];
      Bs[kk][nn] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T a[TM], b[TN];
      const int kr = kk + (lane >> 4), c = lane & 15;
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = As[kr][wm * WM + 16 * i + c];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = Bs[kr][wn * WN + 16 * j + c];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = MfmaOp<T>::run(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }

  if (G.scatter) {
    build_epi<BM, BN>(epi, G, L.sc, m0, n0);
    __syncthreads();
  }
  const T alpha = (T)L.alpha, beta = (T)L.beta;
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
        T v = alpha * acc[i][j][r];
        if (G.scatter) {
          const int64_t bo = L.sc.boff[G.boff_base + (int64_t)epi.rfi[rr] * G.ncc + epi.cgj[cc]];
          if (bo >= 0) C[bo + epi.rlr[rr] * epi.cnd[cc] + epi.clc[cc]] = v;
        } else {
          T* p = C + G.c_off + m * G.ldc + n;
          *p = beta != (T)0 ? v + beta * *p : v;
        }
      }
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
  const float alpha = (float)L.alpha, beta = (float)L.beta;
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
  for (auto& g : groups) f += 2.0 * (double)g.M * (double)g.N * (double)g.K;
  return f;
}

constexpr int TBM = 64, TBN = 64;

void gemm_plan(GemmPlan& p, const std::vector<GemmGroup>& groups, int kind, hipStream_t s, bool persistent) {
  p.host.clear();
  p.kind = kind;
  int64_t t = 0;
  for (auto g : groups) {
    if (g.M <= 0 || g.N <= 0) continue;
    g.ntm = cdiv(g.M, TBM);
    g.ntn = cdiv(g.N, TBN);
    g.tile0 = t;
    t += g.ntm * g.ntn;
    p.host.push_back(g);
  }
  if (t > 0x7fffffffLL) fail(FTN_EINVAL, "GEMM too large");
  p.ntiles = t;
  p.groups = persistent ? persist<GemmGroup>(p.host.size()) : DBuf<GemmGroup>(p.host.size(), s);
  if (!p.host.empty())
    HIPC(hipMemcpyAsync(p.groups.p, p.host.data(), p.host.size() * sizeof(GemmGroup), hipMemcpyHostToDevice, s));
}

void run_gemm(const GemmPlan& p, int dtype, const void* A, const void* B, void* C,
              const GemmScatter* sc, hipStream_t s, double alpha, double beta) {
  if (p.ntiles == 0) return;
  GemmLaunch L;
  L.groups = p.groups.p;
  L.ngroups = (int)p.host.size();
  L.ntiles = p.ntiles;
  L.alpha = alpha;
  L.beta = beta;
  std::memset(&L.sc, 0, sizeof(L.sc));
  if (sc) L.sc = *sc;
  dim3 grid((unsigned)p.ntiles), block(GT);
  void* tok = prof_begin(s);
  if (p.kind == FTN_GEMM_F64) {
    if (dtype != FTN_F64) fail(FTN_ENOTSUP, "FP64 GEMM needs FP64 tensors");
    LAUNCH((k_gemm<double, TBM, TBN, 16>), grid, block, 0, s, L, (const double*)A,
                       (const double*)B, (double*)C);
  } else if (p.kind == FTN_GEMM_F32) {
    if (dtype != FTN_F32) fail(FTN_ENOTSUP, "FP32 GEMM needs FP32 tensors");
    LAUNCH((k_gemm<float, TBM, TBN, 16>), grid, block, 0, s, L, (const float*)A,
                       (const float*)B, (float*)C);
  } else if (p.kind == FTN_GEMM_BF16X3) {
    if (dtype != FTN_F32) fail(FTN_ENOTSUP, "split-BF16 GEMM needs FP32 tensors");
    LAUNCH((k_gemm_bf16x3<TBM, TBN, 32>), grid, block, 0, s, L, (const float*)A,
                       (const float*)B, (float*)C);
  } else {
    fail(FTN_EINVAL, "unknown GEMM kind");
  }
  HIPC(hipGetLastError());
  prof_end(tok, s, p.kind == FTN_GEMM_F64 ? FTN_PROF_GEMM_F64 : (p.kind == FTN_GEMM_F32 ? FTN_PROF_GEMM_F32 : FTN_PROF_GEMM_BF16X3),
           gemm_flops(p.host));
}

void run_grouped_gemm(int gemm, int dtype, const std::vector<GemmGroup>& groups, const void* A,
                      const void* B, void* C, const GemmScatter* sc, hipStream_t s, double alpha,
                      double beta) {
  GemmPlan p;
  gemm_plan(p, groups, gemm, s);
  run_gemm(p, dtype, A, B, C, sc, s, alpha, beta);
}

}  // namespace ftn
