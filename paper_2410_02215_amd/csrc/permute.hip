// Signed permutes: fermionic transposition (Eq. transposition), arrow
// reversal (Sec. II.E), fusion (Sec. IV.A) and the block <-> fused-matrix
// copies around the grouped GEMM. The sign of every block is computed on the
// device from the parity bits of its sectors (integer, bit-exact).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <numeric>

#include "common.h"

namespace ftn {

SignOp make_signop(int ndim, const int* perm, int nA, int nG) {
  SignOp op;
  std::memset(&op, 0, sizeof(op));
  op.ndim = ndim;
  op.nA = nA;
  op.nG = nG;
  for (int p = 0; p < ndim; ++p) op.perm[p] = perm[p];
  // inverted pairs (p < u, perm[p] > perm[u]) contribute p_{perm[p]} p_{perm[u]}
  for (int p = 0; p < ndim; ++p) {
    uint32_t m = 0;
    for (int u = p + 1; u < ndim; ++u)
      if (perm[u] < perm[p]) m |= 1u << perm[u];
    op.kmask[p] = m;
  }
  return op;
}

__device__ inline int sign_bit(const SignOp& op, uint32_t P, int extra) {
  int e = op.phase ^ extra;
  for (int p = 0; p < op.ndim; ++p)
    if ((P >> op.perm[p]) & 1u) e ^= __popc(P & op.kmask[p]) & 1;
  int n = __popc(P & op.rev_mask);
  e ^= ((n * (n - 1)) >> 1) & 1;
  e ^= __popc(P & op.flip_mask) & 1;
  return e & 1;
}

constexpr int PM_THREADS = 256;
constexpr int PM_TILE = 2048;  // entries of one sub-tile
constexpr int PM_SUB = 4;      // consecutive sub-tiles of one block per workgroup (at most)

__host__ __device__ inline int pow2ceil(int64_t v) {
  int p = 1;
  while (p < v && p < (1 << 30)) p <<= 1;
  return p;
}

// one thread per task: strides of both sides, leg merging, tiling, sign
__global__ void k_perm_desc(SignOp op, const PermTask* __restrict__ tasks, int64_t ntasks,
                            const int32_t* __restrict__ shapes, const int64_t* __restrict__ offsets,
                            const uint32_t* __restrict__ parmask, PermDesc* __restrict__ desc,
                            int64_t* __restrict__ tiles) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= ntasks) return;
  const PermTask tk = tasks[t];
  PermDesc D;
  D.boff = 0;
  D.moff = 0;
  D.m = 0;
  D.y = -1;
  D.mode = 3;
  D.ta = D.tr = 1;
  D.neg = 0;
  D.sub = PM_SUB;
  D.nx = D.nr = D.rows = D.nel = D.nsub = 0;
  for (int j = 0; j < MAXD; ++j) {
    D.sb[j] = D.ts[j] = 0;
    D.dim[j] = 1;
  }
  int64_t ntile = 0;
  if (!tk.skip) {
    const int64_t b = tk.block;
    const int n = op.ndim;
    int32_t d[MAXD];
    int64_t str[MAXD];
    for (int j = 0; j < n; ++j) d[j] = shapes[b * n + j];
    // strided side: segments A | G | B of the destination order (Eq. transposition
    // order, then the fused-matrix layout of the GEMM operands)
    const int nA = op.nA, nAG = op.nA + op.nG;
    int64_t st = 1;
    for (int p = n - 1; p >= nAG; --p) {
      str[op.perm[p]] = st;
      st *= d[op.perm[p]];
    }
    int64_t g = 1;
    for (int p = nAG - 1; p >= nA; --p) {
      str[op.perm[p]] = tk.bext * g;
      g *= d[op.perm[p]];
    }
    const int64_t gx = tk.gext ? tk.gext : g;
    st = tk.bext * gx;
    for (int p = nA - 1; p >= 0; --p) {
      str[op.perm[p]] = st;
      st *= d[op.perm[p]];
    }
    D.boff = offsets[b];
    D.moff = tk.moff;
    D.nel = offsets[b + 1] - offsets[b];
    D.neg = sign_bit(op, parmask[b], tk.extra);
    // merge from the innermost block leg outwards; size-1 legs carry nothing
    int m = 0;
    int64_t bst = 1;
    for (int j = n - 1; j >= 0; --j) {
      if (d[j] == 1) continue;
      if (m > 0 && str[j] == D.ts[m - 1] * D.dim[m - 1]) {
        D.dim[m - 1] *= d[j];
      } else {
        D.dim[m] = d[j];
        D.sb[m] = bst;
        D.ts[m] = str[j];
        ++m;
      }
      bst *= d[j];
    }
    if (m == 0) {  // a single entry
      D.dim[0] = 1;
      D.sb[0] = 1;
      D.ts[0] = 1;
      m = 1;
    }
    D.m = m;
    for (int k = 0; k < m; ++k)
      if (D.ts[k] == 1) D.y = k;
    const int64_t dx = D.dim[0];
    if (D.nel == 0) {
      D.mode = 3;
    } else if (D.ts[0] == 1) {  // rows of leg 0 are contiguous on both sides
      D.mode = 0;
      D.rows = D.nel / dx;
      D.ta = max(2, min(pow2ceil(dx), 256));
      // few rows: longer row pieces, so that the tile's rows are all used
      if (D.rows * D.ta < PM_TILE) D.ta = max(2, min(pow2ceil(dx), PM_TILE / pow2ceil(D.rows)));
      D.tr = PM_TILE / D.ta;
      D.nx = (dx + D.ta - 1) / D.ta;
      D.nr = (D.rows + D.tr - 1) / D.tr;
      ntile = D.nx * D.nr;
    } else if (D.y > 0) {  // transpose leg 0 against leg y through LDS
      D.mode = 1;
      const int64_t dy = D.dim[D.y];
      D.rows = dy;
      // both walks should cover whole 256-byte runs: at most 64 along leg 0
      // unless leg y is too short to fill the tile
      D.ta = min(pow2ceil(dx), 64);
      D.tr = min(pow2ceil(dy), PM_TILE / D.ta);
      if (D.ta * D.tr < PM_TILE) D.ta = min(pow2ceil(dx), PM_TILE / D.tr);
      D.nx = (dx + D.ta - 1) / D.ta;
      D.nr = (dy + D.tr - 1) / D.tr;
      ntile = (D.nel / (dx * dy)) * D.nx * D.nr;
      // whole-size tiles: one per workgroup (no serial round trips); smaller
      // ones are grouped so that a workgroup still moves a full tile's worth
      D.sub = D.ta * D.tr >= PM_TILE ? 1 : PM_SUB;
    } else {
      D.mode = 2;
      ntile = (D.nel + PM_TILE - 1) / PM_TILE;
    }
  }
  D.nsub = ntile;
  desc[t] = D;
  tiles[t] = (ntile + D.sub - 1) / D.sub;
}

// task of every tile (once per plan)
__global__ void k_tile_task(const int64_t* __restrict__ tile_start, int64_t ntasks, int64_t ntiles,
                            int32_t* __restrict__ tile_task) {
  const int64_t tl = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (tl >= ntiles) return;
  int64_t lo = 0, hi = ntasks - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (tile_start[mid] <= tl)
      lo = mid;
    else
      hi = mid - 1;
  }
  tile_task[tl] = (int32_t)lo;
}

template <typename T>
struct Pair;
template <>
struct Pair<double> {
  typedef double2 type;
};
template <>
struct Pair<float> {
  typedef float2 type;
};

// One LDS-staged transpose tile of NU * 2 * PM_THREADS entries with every
// access in bounds and pair-aligned: pair u of a thread is entry
// e = 2 threadIdx.x + 2 PM_THREADS u of the tile, so along the block-side
// walk (leg 0 fastest) it advances by whole rows and along the strided-side
// walk (leg y fastest) by whole columns. One pointer per walk, stepped by a
// uniform stride; all loads of a thread leave before the first wait.
struct TileWalk {
  void *bq, *sq;           // first pair of this thread on the block / strided side
  int64_t bstep, sstep;    // advance per pair (elements)
  int tb0, tbstep;         // staging index of the block-side walk and its step
  int ts0, tsstep, ld;     // staging index of the strided-side walk, its step, row length
};

template <typename T, int DIR, int NU>
__device__ __forceinline__ void perm_tile_t(T* tile, const TileWalk& w, T v) {
  typedef typename Pair<T>::type T2;
  T* bq = (T*)w.bq;
  T* sq = (T*)w.sq;
  T2 buf[NU];
  if (DIR == 0) {
#pragma unroll
    for (int u = 0; u < NU; ++u) buf[u] = *(const T2*)(bq + u * w.bstep);
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      T* t = tile + w.tb0 + u * w.tbstep;
      t[0] = v * buf[u].x;
      t[1] = v * buf[u].y;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const T* t = tile + w.ts0 + u * w.tsstep;
      T2 o;
      o.x = t[0];
      o.y = t[w.ld];
      *(T2*)(sq + u * w.sstep) = o;
    }
  } else {
#pragma unroll
    for (int u = 0; u < NU; ++u) buf[u] = *(const T2*)(sq + u * w.sstep);
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      T* t = tile + w.ts0 + u * w.tsstep;
      t[0] = v * buf[u].x;
      t[w.ld] = v * buf[u].y;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const T* t = tile + w.tb0 + u * w.tbstep;
      T2 o;
      o.x = t[0];
      o.y = t[1];
      *(T2*)(bq + u * w.bstep) = o;
    }
  }
}

template <typename T, int DIR>
__global__ void __launch_bounds__(PM_THREADS)
    k_block_perm(const PermDesc* __restrict__ desc, const int64_t* __restrict__ tile_start,
                 const int32_t* __restrict__ tile_task, const T* __restrict__ src, T* __restrict__ dst,
                 T alpha) {
  // transpose staging (tr x (ta + 1) entries, tr <= PM_TILE / 2) or row bases
  __shared__ double smem[PM_TILE + PM_TILE / 2];
  T* tile = (T*)smem;
  int64_t* rbase = (int64_t*)smem;
  const int64_t tl = blockIdx.x;
  // the task and its descriptor are the same for the whole workgroup: read
  // through the scalar cache, with no staging or barrier before the loads
  const int task = __builtin_amdgcn_readfirstlane(tile_task[tl]);
  const PermDesc& D = desc[task];
  const int64_t first = (tl - tile_start[task]) * D.sub;
  const T v = D.neg ? -alpha : alpha;
  const int ta = D.ta, tr = D.tr;
  const int lta = __ffs(ta) - 1, ltr = __ffs(tr) - 1;  // ta, tr are powers of two
  for (int k = 0; k < D.sub; ++k) {
    const int64_t lt = first + k;
    if (lt >= D.nsub) break;
    if (D.mode == 0) {
      const int64_t ix = lt % D.nx, ir = lt / D.nx;
      const int64_t x0 = ix * ta, r0 = ir * tr, dx = D.dim[0];
      // strided-side base of each row of the sub-tile (rows enumerate legs 1..m-1)
      for (int r = threadIdx.x; r < tr; r += PM_THREADS) {
        int64_t q = r0 + r, a = 0;
        for (int j = 1; j < D.m; ++j) {
          const int64_t dj = D.dim[j];
          a += (q % dj) * D.ts[j];
          q /= dj;
        }
        rbase[r] = a;
      }
      __syncthreads();
      typedef typename Pair<T>::type T2;
      constexpr int PPT = PM_TILE / (2 * PM_THREADS);
      // whole tile with every pair aligned on both sides and rows of at most
      // 2 * PM_THREADS entries: pair u of a thread sits u * (2 PM_THREADS / ta)
      // rows below its first, at the same column; unchecked 2-wide accesses
      // with no branch around them, so that all loads leave before the first
      // wait
      {
        constexpr int STEP = 2 * PM_THREADS;
        bool even = ((D.boff | dx | D.moff) & 1) == 0 &&
                    ((((uintptr_t)src) | ((uintptr_t)dst)) & (sizeof(T2) - 1)) == 0;
        for (int j = 1; j < D.m; ++j) even = even && (D.ts[j] & 1) == 0;
        if (even && ta <= STEP && r0 + tr <= D.rows && x0 + ta <= dx) {
          const int e0 = 2 * threadIdx.x, ra = STEP >> lta, rb0 = e0 >> lta, ib0 = e0 & (ta - 1);
          T* bq = (DIR == 0 ? const_cast<T*>(src) : dst) + D.boff + (r0 + rb0) * dx + x0 + ib0;
          T* sq = (DIR == 0 ? dst : const_cast<T*>(src)) + D.moff + x0 + ib0;
          const int64_t bstep = (int64_t)ra * dx;
          T2 buf[PPT];
#pragma unroll
          for (int u = 0; u < PPT; ++u)
            buf[u] = DIR == 0 ? *(const T2*)(bq + u * bstep) : *(const T2*)(sq + rbase[rb0 + u * ra]);
#pragma unroll
          for (int u = 0; u < PPT; ++u) {
            T2 w;
            w.x = v * buf[u].x;
            w.y = v * buf[u].y;
            *(T2*)(DIR == 0 ? sq + rbase[rb0 + u * ra] : bq + u * bstep) = w;
          }
          __syncthreads();  // rbase is rewritten by the next sub-tile
          continue;
        }
      }
      // two neighbouring entries of a row per thread (ta is an even power of
      // two, so a pair never straddles rows): one 2-wide load and store when
      // both addresses are aligned to the pair, else two single entries. The
      // PPT pairs of a thread are all loaded before any is stored, so that
      // each thread keeps several loads in flight.
      T2 buf[PPT];
      unsigned okm = 0, twom = 0, vecm = 0;
      // block-side and strided-side index of pair u of this thread (the
      // stores recompute them rather than keep them in registers)
      auto idx = [&](int u, int64_t& bi, int64_t& si) {
        const int e = 2 * threadIdx.x + u * 2 * PM_THREADS;
        const int r = e >> lta, i = e & (ta - 1);
        const int64_t row = r0 + r, x = x0 + i;
        const bool ok = row < D.rows && x < dx;
        bi = D.boff + row * dx + x;
        si = D.moff + (ok ? rbase[r] : 0) + x;
        return ok;
      };
#pragma unroll
      for (int u = 0; u < PPT; ++u) {
        int64_t bi, si;
        const bool ok = idx(u, bi, si);
        const int64_t x = x0 + ((2 * threadIdx.x + u * 2 * PM_THREADS) & (ta - 1));
        const T* sp = DIR == 0 ? src + bi : src + si;
        T* dp = DIR == 0 ? dst + si : dst + bi;
        const bool two = x + 1 < dx;
        const bool vec = two && ((((uintptr_t)sp) | ((uintptr_t)dp)) & (sizeof(T2) - 1)) == 0;
        okm |= ok ? 1u << u : 0u;
        twom |= two ? 1u << u : 0u;
        vecm |= vec ? 1u << u : 0u;
        if (ok) {
          if (vec) {
            buf[u] = *(const T2*)sp;
          } else {
            buf[u].x = sp[0];
            buf[u].y = two ? sp[1] : T(0);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < PPT; ++u) {
        if (!((okm >> u) & 1u)) continue;
        int64_t bi, si;
        idx(u, bi, si);
        T* dp = DIR == 0 ? dst + si : dst + bi;
        T2 b;
        b.x = v * buf[u].x;
        b.y = v * buf[u].y;
        if ((vecm >> u) & 1u) {
          *(T2*)dp = b;
        } else {
          dp[0] = b.x;
          if ((twom >> u) & 1u) dp[1] = b.y;
        }
      }
    } else if (D.mode == 1) {
      const int y = D.y;
      const int64_t per = D.nx * D.nr;
      const int64_t bt = lt / per, rem = lt % per;
      const int64_t ix = rem % D.nx, ir = rem / D.nx;
      const int64_t x0 = ix * ta, y0 = ir * tr, dx = D.dim[0], dy = D.dim[y];
      // batch position over the legs other than 0 and y (every thread, no
      // barrier before the loads)
      int64_t bbase = D.boff, sbase = D.moff;
      {
        int64_t q = bt;
        for (int j = 1; j < D.m && q; ++j) {
          if (j == y) continue;
          const int64_t dj = D.dim[j];
          const int64_t ij = q % dj;
          q /= dj;
          bbase += ij * D.sb[j];
          sbase += ij * D.ts[j];
        }
      }
      const int64_t sby = D.sb[y], tsx = D.ts[0];
      const int ld = ta + 1, n = ta * tr;
      typedef typename Pair<T>::type T2;
      constexpr int PPT = PM_TILE / (2 * PM_THREADS);
      // whole tile of at least 2 * PM_THREADS entries (n = NU 2 PM_THREADS,
      // NU = 1, 2 or 4), every pair aligned on both sides, ta and tr at most
      // 2 * PM_THREADS: unchecked 2-wide accesses with no branch around them
      // (perm_tile_t)
      constexpr int STEP = 2 * PM_THREADS;
      if (n >= STEP && ta <= STEP && tr <= STEP && x0 + ta <= dx && y0 + tr <= dy &&
          ((bbase | sby | sbase | tsx) & 1) == 0 && ((((uintptr_t)src) | ((uintptr_t)dst)) & (sizeof(T2) - 1)) == 0) {
        const int e0 = 2 * threadIdx.x;
        const int ra = STEP >> lta, rb0 = e0 >> lta, ib0 = e0 & (ta - 1);  // block-side walk
        const int ia = STEP >> ltr, rs0 = e0 & (tr - 1), is0 = e0 >> ltr;  // strided-side walk
        T* bq = (DIR == 0 ? const_cast<T*>(src) : dst) + bbase + (y0 + rb0) * sby + x0 + ib0;
        T* sq = (DIR == 0 ? dst : const_cast<T*>(src)) + sbase + y0 + rs0 + (x0 + is0) * tsx;
        const int64_t bstep = (int64_t)ra * sby, sstep = (int64_t)ia * tsx;
        const TileWalk w{bq, sq, bstep, sstep, (rb0 * ld + ib0), ra * ld, (rs0 * ld + is0), ia, ld};
        if (n == PM_TILE)
          perm_tile_t<T, DIR, PM_TILE / STEP>(tile, w, v);
        else if (n == 2 * STEP)
          perm_tile_t<T, DIR, 2>(tile, w, v);
        else
          perm_tile_t<T, DIR, 1>(tile, w, v);
        __syncthreads();  // the staging buffer is reused by the next sub-tile
        continue;
      }
      // the block side is walked with leg 0 fastest, the strided side with leg y;
      // each thread moves two neighbours along the contiguous direction of the
      // side it touches (ta and tr are powers of two >= 2), with one 2-wide
      // access when the pair is aligned
      auto ld2 = [](const T* p, bool two, T& a0, T& a1) {
        if (two && (((uintptr_t)p) & (sizeof(T2) - 1)) == 0) {
          const T2 t = *(const T2*)p;
          a0 = t.x;
          a1 = t.y;
        } else {
          a0 = p[0];
          a1 = two ? p[1] : T(0);
        }
      };
      auto st2 = [](T* p, bool two, T b0, T b1) {
        if (two && (((uintptr_t)p) & (sizeof(T2) - 1)) == 0) {
          T2 t;
          t.x = b0;
          t.y = b1;
          *(T2*)p = t;
        } else {
          p[0] = b0;
          if (two) p[1] = b1;
        }
      };
      // the loads of a thread are issued together (PPT pairs at most) before
      // the staging writes, so that several are in flight
      if (DIR == 0) {
        T la0[PPT], la1[PPT];
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
          const int e = 2 * threadIdx.x + u * 2 * PM_THREADS;
          const int r = e >> lta, i = e & (ta - 1);
          const int64_t yy = y0 + r, x = x0 + i;
          la0[u] = la1[u] = T(0);
          if (e < n && yy < dy && x < dx) ld2(src + bbase + yy * sby + x, x + 1 < dx, la0[u], la1[u]);
        }
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
          const int e = 2 * threadIdx.x + u * 2 * PM_THREADS;
          const int r = e >> lta, i = e & (ta - 1);
          const int64_t yy = y0 + r, x = x0 + i;
          if (e < n && yy < dy && x < dx) {
            tile[r * ld + i] = v * la0[u];
            tile[r * ld + i + 1] = v * la1[u];
          }
        }
        __syncthreads();
        for (int e = 2 * threadIdx.x; e < n; e += 2 * PM_THREADS) {
          const int r = e & (tr - 1), i = e >> ltr;
          const int64_t yy = y0 + r, x = x0 + i;
          if (yy < dy && x < dx)
            st2(dst + sbase + yy + x * tsx, yy + 1 < dy, tile[r * ld + i], tile[(r + 1) * ld + i]);
        }
      } else {
        T la0[PPT], la1[PPT];
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
          const int e = 2 * threadIdx.x + u * 2 * PM_THREADS;
          const int r = e & (tr - 1), i = e >> ltr;
          const int64_t yy = y0 + r, x = x0 + i;
          la0[u] = la1[u] = T(0);
          if (e < n && yy < dy && x < dx) ld2(src + sbase + yy + x * tsx, yy + 1 < dy, la0[u], la1[u]);
        }
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
          const int e = 2 * threadIdx.x + u * 2 * PM_THREADS;
          const int r = e & (tr - 1), i = e >> ltr;
          const int64_t yy = y0 + r, x = x0 + i;
          if (e < n && yy < dy && x < dx) {
            tile[r * ld + i] = v * la0[u];
            tile[(r + 1) * ld + i] = v * la1[u];
          }
        }
        __syncthreads();
        for (int e = 2 * threadIdx.x; e < n; e += 2 * PM_THREADS) {
          const int r = e >> lta, i = e & (ta - 1);
          const int64_t yy = y0 + r, x = x0 + i;
          if (yy < dy && x < dx) st2(dst + bbase + yy * sby + x, x + 1 < dx, tile[r * ld + i], tile[r * ld + i + 1]);
        }
      }
    } else if (D.mode == 2) {
      const int64_t e0 = lt * PM_TILE;
      for (int j = threadIdx.x; j < PM_TILE; j += PM_THREADS) {
        const int64_t e = e0 + j;
        if (e >= D.nel) break;
        int64_t q = e, a = 0;
        for (int i = 0; i < D.m; ++i) {
          const int64_t di = D.dim[i];
          a += (q % di) * D.ts[i];
          q /= di;
        }
        if (DIR == 0)
          dst[D.moff + a] = v * src[D.boff + e];
        else
          dst[D.boff + e] = v * src[D.moff + a];
      }
    }
    __syncthreads();  // the staging buffer is reused by the next sub-tile
  }
}

void perm_plan_build(PermPlan& p, const Structure& S, hipStream_t s) {
  p.ntasks = S.nblocks;
  p.nelem = S.size;
  p.ntiles = 0;
  if (!p.ntasks) return;
  p.desc = persist<PermDesc>(p.ntasks);
  p.tile_start = persist<int64_t>(p.ntasks);
  DBuf<int64_t> total(1, s);
  LAUNCH(k_perm_desc, dim3((unsigned)cdiv(p.ntasks, 128)), dim3(128), 0, s, p.op, p.tasks.p, p.ntasks,
         S.d_shapes.p, S.d_offsets.p, S.d_parmask.p, p.desc.p, p.tile_start.p);
  scan_exclusive(p.tile_start.p, p.ntasks, total.p, s);
  int64_t tot = 0;
  HIPC(hipMemcpyAsync(&tot, total.p, 8, hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  if (tot > 0x7fffffffLL) fail(FTN_EINVAL, "permute too large");
  p.ntiles = tot;
  if (tot > 0) {
    p.tile_task = persist<int32_t>(tot);
    LAUNCH(k_tile_task, dim3((unsigned)cdiv(tot, 256)), dim3(256), 0, s, p.tile_start.p, p.ntasks, tot,
           p.tile_task.p);
  }
}

void run_perm(int dir, const Structure& S, int dtype, const PermPlan& p, const void* src, void* dst,
              hipStream_t s, double alpha) {
  if (p.ntiles == 0) return;
  // FTN_TRACE_PERM: one line per launch; FTN_TRACE_PERM=2 also times it
  // (synchronising the stream around the launch)
  static const char* trace_env = std::getenv("FTN_TRACE_PERM");
  static const bool trace = trace_env != nullptr;
  static const bool trace_time = trace && trace_env[0] == '2';
  hipEvent_t te0 = nullptr, te1 = nullptr;
  if (trace) {
    int64_t big = 0;
    for (int64_t b = 1; b < S.nblocks; ++b)
      if (S.offsets[b + 1] - S.offsets[b] > S.offsets[big + 1] - S.offsets[big]) big = b;
    std::string sh, pm;
    for (int j = 0; j < S.ndim; ++j) sh += std::to_string(S.shapes[big * S.ndim + j]) + " ";
    for (int j = 0; j < p.op.ndim; ++j) pm += std::to_string(p.op.perm[j]) + " ";
    // entries moved per copy mode (descriptors read back: trace runs only)
    std::vector<PermDesc> hd(p.ntasks);
    HIPC(hipMemcpyAsync(hd.data(), p.desc.p, p.ntasks * sizeof(PermDesc), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    int64_t em[4] = {0, 0, 0, 0}, dxs = 0;
    for (auto& d : hd) {
      em[d.mode & 3] += d.nel;
      if (d.mode == 0) dxs += d.nel * d.dim[0];
    }
    std::fprintf(stderr, "[perm] dir %d nel %lld bytes %lld nblocks %lld nA %d nG %d perm [%s] biggest [%s] modes %lld "
                 "%lld %lld row0 %.1f\n", dir, (long long)p.nelem,
                 (long long)(2 * p.nelem * (dtype == FTN_F64 ? 8 : 4)), (long long)S.nblocks, p.op.nA, p.op.nG,
                 pm.c_str(), sh.c_str(),
                 (long long)em[0], (long long)em[1], (long long)em[2], em[0] ? (double)dxs / em[0] : 0.0);
  }
  if (trace_time) {
    HIPC(hipEventCreate(&te0));
    HIPC(hipEventCreate(&te1));
    HIPC(hipEventRecord(te0, s));
  }
  void* tok = prof_begin(s);
  const dim3 grid((unsigned)p.ntiles), block(PM_THREADS);
  if (dtype == FTN_F64) {
    auto k = dir == 0 ? k_block_perm<double, 0> : k_block_perm<double, 1>;
    ELAUNCH(k, grid, block, 0, s, prof_ev(tok, 0), prof_ev(tok, 1), p.desc.p, p.tile_start.p, p.tile_task.p,
            (const double*)src, (double*)dst, alpha);
  } else {
    auto k = dir == 0 ? k_block_perm<float, 0> : k_block_perm<float, 1>;
    ELAUNCH(k, grid, block, 0, s, prof_ev(tok, 0), prof_ev(tok, 1), p.desc.p, p.tile_start.p, p.tile_task.p,
            (const float*)src, (float*)dst, (float)alpha);
  }
  HIPC(hipGetLastError());
  const double pb = 2.0 * (double)p.nelem * (dtype == FTN_F64 ? 8 : 4);
  prof_end(tok, s, FTN_PROF_PERMUTE, pb, pb);
  if (trace_time) {
    HIPC(hipEventRecord(te1, s));
    HIPC(hipEventSynchronize(te1));
    float ms = 0;
    HIPC(hipEventElapsedTime(&ms, te0, te1));
    std::fprintf(stderr, "[perm-time] us %.1f GB/s %.0f\n", 1000.0 * ms, ms > 0 ? pb / (ms * 1e-3) / 1e9 : 0.0);
    (void)hipEventDestroy(te0);
    (void)hipEventDestroy(te1);
  }
}

// ---------------------------------------------------------------------------
// unary key matching on the device
__global__ void k_unary_tasks(int n, SignOp op, const int32_t* __restrict__ skeys, int64_t snb,
                              const int32_t* __restrict__ dkeys, const int64_t* __restrict__ doff,
                              int64_t dnb, const int32_t* __restrict__ remap,
                              const int32_t* __restrict__ rbase, PermTask* tasks) {
  int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= snb) return;
  int32_t nk[MAXD];
  for (int p = 0; p < n; ++p) {
    int leg = op.perm[p];
    nk[p] = remap[rbase[leg] + skeys[b * n + leg]];
  }
  int64_t lo = 0, hi = dnb;
  int64_t found = -1;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    int c = 0;
    for (int i = 0; i < n && !c; ++i) {
      int32_t x = dkeys[mid * n + i];
      c = x < nk[i] ? -1 : (x > nk[i] ? 1 : 0);
    }
    if (c == 0) {
      found = mid;
      break;
    }
    if (c < 0)
      lo = mid + 1;
    else
      hi = mid;
  }
  PermTask t;
  t.block = b;
  t.moff = found >= 0 ? doff[found] : 0;
  t.gext = 0;
  t.bext = 1;
  t.skip = found < 0;
  t.extra = 0;
  tasks[b] = t;
}

void unary_tasks(const Structure& src, const Structure& dst, const SignOp& op,
                 const std::vector<int32_t>& remap, const std::vector<int>& remap_base,
                 DBuf<PermTask>& tasks, hipStream_t s) {
  tasks = persist<PermTask>(src.nblocks);
  if (!src.nblocks) return;
  std::vector<int32_t> rb(remap_base.begin(), remap_base.end());
  DBuf<int32_t> drm = to_device(remap, s);
  DBuf<int32_t> drb = to_device(rb, s);
  LAUNCH(k_unary_tasks, dim3((unsigned)cdiv(src.nblocks, 128)), dim3(128), 0, s, src.ndim,
                     op, src.d_keys.p, src.nblocks, dst.d_keys.p, dst.d_offsets.p, dst.nblocks, drm.p,
                     drb.p, tasks.p);
}

// cache of unary permutes: output structure + ready plan per (input
// structure, operation)
namespace {
struct UnaryPlan {
  std::shared_ptr<const Structure> out;
  PermPlan pp;
};
std::mutex g_unary_mu;
auto* g_unary = new std::unordered_map<std::string, std::shared_ptr<UnaryPlan>>();
}  // namespace

std::vector<int64_t> block_sizes(const Structure& s) {
  std::vector<int64_t> v(s.nblocks);
  for (int64_t b = 0; b < s.nblocks; ++b) v[b] = s.offsets[b + 1] - s.offsets[b];
  return v;
}

// shared driver of the unary signed permutes
static std::unique_ptr<Tensor> unary_signed(const Tensor& a, const std::vector<Leg>& out_legs,
                                            const SignOp& op, const std::vector<int32_t>& remap,
                                            const std::vector<int>& rbase, hipStream_t s,
                                            const Q* total = nullptr) {
  if (a.ndim() == 0) {
    auto out = make_tensor(a.sym(), a.dtype, out_legs, total ? *total : a.total(), s, false);
    if (a.size()) {
      HIPC(hipMemcpyAsync(out->data, a.data, a.esize(), hipMemcpyDeviceToDevice, s));
      if (op.phase) {
        auto neg = op_scale(*out, -1.0, s);
        return neg;
      }
    }
    return out;
  }
  std::string key = a.st->skey + "|u|";
  key.append((const char*)&op, sizeof(op));
  key.append((const char*)remap.data(), remap.size() * sizeof(int32_t));
  key += structure_key(a.sym(), out_legs, total ? *total : a.total());
  std::shared_ptr<UnaryPlan> U;
  {
    std::lock_guard<std::mutex> g(g_unary_mu);
    auto it = g_unary->find(key);
    if (it != g_unary->end()) U = it->second;
  }
  if (!U) {
    U = std::make_shared<UnaryPlan>();
    U->out = get_structure(a.sym(), out_legs, total ? *total : a.total(), s);
    U->pp.op = op;
    unary_tasks(a.S(), *U->out, op, remap, rbase, U->pp.tasks, s);
    if (U->out->size != a.size()) fail(FTN_EINVAL, "internal: unary permute changed the size");
    perm_plan_build(U->pp, a.S(), s);
    HIPC(hipStreamSynchronize(s));  // cached plans may be used on other streams
    std::lock_guard<std::mutex> g(g_unary_mu);
    if (g_unary->size() > 8192) g_unary->clear();
    g_unary->emplace(key, U);
  }
  auto out = make_tensor(U->out, a.dtype, s, false);
  run_perm(0, a.S(), a.dtype, U->pp, a.data, out->data, s);
  return out;
}

static void identity_remap(const Structure& a, std::vector<int32_t>& remap, std::vector<int>& rbase) {
  for (int i = 0; i < a.ndim; ++i) {
    rbase.push_back((int)remap.size());
    for (int k = 0; k < a.legs[i].nsect(); ++k) remap.push_back(k);
  }
}

std::unique_ptr<Tensor> op_ftranspose(const Tensor& a, const std::vector<int>& perm, hipStream_t s) {
  const int n = a.ndim();
  if ((int)perm.size() != n) fail(FTN_EINVAL, "permutation length differs from ndim");
  std::vector<int> chk(perm);
  std::sort(chk.begin(), chk.end());
  for (int i = 0; i < n; ++i)
    if (chk[i] != i) fail(FTN_EINVAL, "not a permutation");
  std::vector<Leg> legs(n);
  for (int p = 0; p < n; ++p) legs[p] = a.legs()[perm[p]];
  SignOp op = make_signop(n, perm.data(), n, 0);
  std::vector<int32_t> remap;
  std::vector<int> rbase;
  identity_remap(a.S(), remap, rbase);
  return unary_signed(a, legs, op, remap, rbase, s);
}

// conjugated leg: charges negated and re-sorted; remap old sector -> new
static Leg conj_leg(int sym, const Leg& l, std::vector<int32_t>& remap) {
  std::vector<std::pair<Q, int>> v;
  for (int k = 0; k < l.nsect(); ++k) v.push_back({q_neg(sym, l.q[k]), k});
  std::sort(v.begin(), v.end(), [](const std::pair<Q, int>& x, const std::pair<Q, int>& y) {
    return q_lt(x.first, y.first);
  });
  Leg o;
  o.dual = 1 - l.dual;
  remap.assign(l.nsect(), 0);
  for (int i = 0; i < (int)v.size(); ++i) {
    o.q.push_back(v[i].first);
    o.d.push_back(l.d[v[i].second]);
    remap[v[i].second] = i;
  }
  return o;
}

std::unique_ptr<Tensor> op_flip_dual(const Tensor& a, int leg, int with_sign, hipStream_t s) {
  const int n = a.ndim();
  if (leg < 0 || leg >= n) fail(FTN_EINVAL, "leg out of range");
  std::vector<Leg> legs = a.legs();
  std::vector<int32_t> lr;
  legs[leg] = conj_leg(a.sym(), a.legs()[leg], lr);
  std::vector<int32_t> remap;
  std::vector<int> rbase;
  for (int i = 0; i < n; ++i) {
    rbase.push_back((int)remap.size());
    if (i == leg)
      remap.insert(remap.end(), lr.begin(), lr.end());
    else
      for (int k = 0; k < a.legs()[i].nsect(); ++k) remap.push_back(k);
  }
  std::vector<int> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  SignOp op = make_signop(n, perm.data(), n, 0);
  bool sign = with_sign < 0 ? a.legs()[leg].dual == 1 : with_sign != 0;
  if (sign) op.flip_mask = 1u << leg;
  return unary_signed(a, legs, op, remap, rbase, s);
}

std::unique_ptr<Tensor> op_dagger(const Tensor& a, hipStream_t s) {
  const int n = a.ndim();
  std::vector<int> perm(n);
  std::vector<Leg> legs(n);
  for (int p = 0; p < n; ++p) {
    perm[p] = n - 1 - p;
    legs[p] = a.legs()[n - 1 - p];
    legs[p].dual = 1 - legs[p].dual;
  }
  SignOp op = make_signop(n, perm.data(), n, 0);
  // the Koszul sign of the full reversal equals the pairwise-product sign
  // over all legs; adding the latter cancels it (a plain relabelling)
  op.rev_mask = n ? (uint32_t)((1ull << n) - 1) : 0u;
  std::vector<int32_t> remap;
  std::vector<int> rbase;
  identity_remap(a.S(), remap, rbase);
  Q tot = q_neg(a.sym(), a.total());
  return unary_signed(a, legs, op, remap, rbase, s, &tot);
}

std::unique_ptr<Tensor> op_leg_sign(const Tensor& a, int leg, hipStream_t s) {
  const int n = a.ndim();
  std::vector<int> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  SignOp op = make_signop(n, perm.data(), n, 0);
  op.flip_mask = 1u << leg;
  std::vector<int32_t> remap;
  std::vector<int> rbase;
  identity_remap(a.S(), remap, rbase);
  return unary_signed(a, a.legs(), op, remap, rbase, s);
}

// ---------------------------------------------------------------------------
// fusion (Sec. IV.A)
std::unique_ptr<Tensor> op_fuse(const Tensor& a, const std::vector<int>& glegs, int conv, int rev,
                                hipStream_t s) {
  const int n = a.ndim();
  const int m = (int)glegs.size();
  const int sym = a.sym();
  if (m < 1) fail(FTN_EINVAL, "fuse needs at least one leg");
  std::string key = a.st->skey + "|f|" + std::to_string(conv) + "," + std::to_string(rev) + "|";
  for (int l : glegs) key += std::to_string(l) + ",";
  {
    std::lock_guard<std::mutex> g(g_unary_mu);
    auto it = g_unary->find(key);
    if (it != g_unary->end()) {
      auto U = it->second;
      auto out = make_tensor(U->out, a.dtype, s, false);
      run_perm(0, a.S(), a.dtype, U->pp, a.data, out->data, s);
      return out;
    }
  }
  std::vector<int> isg(n, 0);
  for (int l : glegs) {
    if (l < 0 || l >= n || isg[l]) fail(FTN_EINVAL, "bad fuse legs");
    isg[l] = 1;
  }
  std::vector<int> rest;
  for (int i = 0; i < n; ++i)
    if (!isg[i]) rest.push_back(i);
  int pos = 0;
  for (int i : rest)
    if (i < glegs[0]) ++pos;
  std::vector<int> order(rest.begin(), rest.begin() + pos);
  order.insert(order.end(), glegs.begin(), glegs.end());
  order.insert(order.end(), rest.begin() + pos, rest.end());
  // components after dual alignment
  const int d0 = a.legs()[glegs[0]].dual;
  std::vector<Leg> comp(m);
  std::vector<std::vector<int32_t>> cremap(m);
  uint32_t flip = 0;
  for (int j = 0; j < m; ++j) {
    const Leg& l = a.legs()[glegs[j]];
    if (l.dual != d0) {
      comp[j] = conj_leg(sym, l, cremap[j]);
      if (conv == FTN_LOCAL && l.dual == 1) flip |= 1u << glegs[j];
    } else {
      comp[j] = l;
      cremap[j].resize(l.nsect());
      std::iota(cremap[j].begin(), cremap[j].end(), 0);
    }
  }
  bool do_rev = conv == FTN_LOCAL ? d0 == 1 : rev != 0;
  // fused leg: combos in lexicographic order grouped by total charge
  std::map<std::pair<int, int>, std::vector<std::pair<std::vector<int>, int64_t>>> groups;
  std::vector<int> idx(m, 0);
  int64_t ncomb = 1;
  for (auto& c : comp) ncomb *= c.nsect();
  for (int64_t c = 0; c < ncomb; ++c) {
    int64_t r = c;
    for (int j = m - 1; j >= 0; --j) {
      idx[j] = (int)(r % comp[j].nsect());
      r /= comp[j].nsect();
    }
    Q qq{0, 0};
    int64_t d = 1;
    for (int j = 0; j < m; ++j) {
      qq = q_add(sym, qq, comp[j].q[idx[j]]);
      d *= comp[j].d[idx[j]];
    }
    groups[{qq.a, qq.b}].push_back({idx, d});
  }
  Leg fl;
  fl.dual = d0;
  std::map<std::vector<int>, std::pair<int, int64_t>> table;
  int si = 0;
  for (auto& g : groups) {
    int64_t off = 0;
    for (auto& e : g.second) {
      table[e.first] = {si, off};
      off += e.second;
    }
    fl.q.push_back(Q{g.first.first, g.first.second});
    fl.d.push_back(off);
    ++si;
  }
  std::vector<Leg> out_legs;
  for (int i = 0; i < pos; ++i) out_legs.push_back(a.legs()[rest[i]]);
  out_legs.push_back(fl);
  for (size_t i = pos; i < rest.size(); ++i) out_legs.push_back(a.legs()[rest[i]]);
  // every output entry is written by exactly one source block
  auto out = make_tensor(sym, a.dtype, out_legs, a.total(), s, false);
  const Structure& A = a.S();
  const Structure& O = out->S();
  SignOp op = make_signop(n, order.data(), pos, m);
  op.flip_mask = flip;
  if (do_rev)
    for (int l : glegs) op.rev_mask |= 1u << l;
  // tasks (host): each source block writes a slab of one output block
  std::vector<PermTask> tasks(A.nblocks);
  std::vector<int32_t> okey(O.ndim);
  std::vector<int> ck(m);
  for (int64_t b = 0; b < A.nblocks; ++b) {
    const int32_t* k = &A.keys[b * n];
    for (int j = 0; j < m; ++j) ck[j] = cremap[j][k[glegs[j]]];
    auto te = table.at(ck);
    int t = 0;
    for (int i = 0; i < pos; ++i) okey[t++] = k[rest[i]];
    okey[t++] = te.first;
    for (size_t i = pos; i < rest.size(); ++i) okey[t++] = k[rest[i]];
    int64_t ob = block_index(O, okey.data());
    if (ob < 0) fail(FTN_EINVAL, "internal: fused block missing");
    int64_t bext = 1;
    for (size_t i = pos; i < rest.size(); ++i) bext *= A.shapes[b * n + rest[i]];
    PermTask tk;
    tk.block = b;
    tk.bext = bext;
    tk.gext = fl.d[te.first];
    tk.moff = O.offsets[ob] + te.second * bext;
    tk.skip = 0;
    tk.extra = 0;
    tasks[b] = tk;
  }
  auto U = std::make_shared<UnaryPlan>();
  U->out = out->st;
  U->pp.op = op;
  U->pp.tasks = persist_upload(tasks, s);
  perm_plan_build(U->pp, A, s);
  HIPC(hipStreamSynchronize(s));  // cached plans may be used on other streams
  run_perm(0, A, a.dtype, U->pp, a.data, out->data, s);
  std::lock_guard<std::mutex> g(g_unary_mu);
  if (g_unary->size() > 8192) g_unary->clear();
  g_unary->emplace(key, U);
  return out;
}

// Adjoint of fusion: every entry of the fused tensor is one entry of a with
// a sign, so the cotangent of a is the same signed map read backwards
std::unique_ptr<Tensor> op_fuse_backward(const Tensor& a, const std::vector<int>& glegs, int conv, int rev,
                                         const Tensor& dout, hipStream_t s) {
  std::string key = a.st->skey + "|f|" + std::to_string(conv) + "," + std::to_string(rev) + "|";
  for (int l : glegs) key += std::to_string(l) + ",";
  std::shared_ptr<UnaryPlan> U;
  for (int attempt = 0; attempt < 2 && !U; ++attempt) {
    {
      std::lock_guard<std::mutex> g(g_unary_mu);
      auto it = g_unary->find(key);
      if (it != g_unary->end()) U = it->second;
    }
    if (!U) (void)op_fuse(a, glegs, conv, rev, s);  // builds and caches the plan
  }
  if (!U) fail(FTN_EINVAL, "internal: fusion plan not available");
  if (dout.st->skey != U->out->skey) fail(FTN_EINVAL, "cotangent does not have the structure of the fused tensor");
  if (dout.dtype != a.dtype) fail(FTN_ENOTSUP, "cotangent dtype differs");
  auto da = make_tensor(a.st, a.dtype, s, false);  // every entry is read back from one fused entry
  if (a.size()) run_perm(1, a.S(), a.dtype, U->pp, dout.data, da->data, s);
  return da;
}

}  // namespace ftn
