// Bond compression (Sec. II.A truncated SVD over all symmetry blocks; used
// by approximate contraction, Fig. 1b and Sec. III), FP64 throughout.
//
// For the bond between A (leg la) and B (leg lb), per bond charge q:
//   A~_q (M x d) and B~_q (d x N) are the fused matrices of the contraction
//   plan (signed permutes). G_A = A~^T A~ and G_B = B~ B~^T (split-K MFMA
//   GEMMs) are factored by pivoted Cholesky, G_A = R_A^T R_A, G_B = R_B^T
//   R_B, so A~ = Q_A R_A and B~ = R_B^T Q_B with orthonormal Q's. The SVD of
//   X = R_A R_B^T = U S V^T gives the best rank-chi approximation of A~ B~,
//   with the chi largest values kept over all charges. The projectors
//   P_A = R_B^T V S^-1/2 and P_B = S^-1/2 U^T R_A give A' = A~ P_A and
//   B' = P_B B~, computed as ordinary fermionic contractions of A and B with
//   2-leg block-diagonal tensors followed by transpositions that put the new
//   bond back in place. A per-sector sign (the bond parity of the local
//   convention) commutes with the block-diagonal projectors, so the same
//   A', B' serve both conventions.
// The SVD of X: the smaller Gram matrix H of X is diagonalised with a cyclic
// Jacobi method in LDS when its order is <= 128, otherwise its leading
// eigenspace is found by subspace iteration (Cholesky-QR orthonormalisation)
// followed by a Rayleigh-Ritz step on a 128-dimensional subspace.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace ftn {

constexpr int LT = 1024;     // threads of the factorisation kernels
constexpr int JMAX = 128;    // largest order diagonalised in LDS
constexpr int CHOL_MAX = 4096;

typedef double d4 __attribute__((ext_vector_type(4)));
static_assert(LT == 1024 && JMAX == 128, "register staging assumes 1024 threads and order 128");

__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// ---------------------------------------------------------------------------
// Blocked pivoted Cholesky (Gram matrices up to 4096): a panel kernel factors
// up to 64 pivoted columns per launch (one workgroup per matrix), followed by
// an MFMA GEMM that removes the panel from the Schur complement,
// G <- G - R_p^T R_p. R is kept in original column order (R[l][c]), so the
// update needs no gather. Stops at the numerical rank (largest remaining
// pivot not above tol * largest diagonal of G).
struct CholState {
  double* G;    // d x d, overwritten by the Schur complement
  double* R;    // d x d, zeroed on entry
  double* dp;   // d: remaining pivots by position
  int* piv;     // d: original index at each position
  double* thr;  // 1: absolute pivot threshold
  int* rank;    // 1: -1 while running, then the rank
  int d;
  int pad;
};

__global__ void __launch_bounds__(LT) k_chol_init(const CholState* st, double tol) {
  const CholState S = st[blockIdx.x];
  const int d = S.d, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  __shared__ double red[LT / 64];
  double m = 0.0;
  for (int i = tid; i < d; i += LT) {
    double v = S.G[(int64_t)i * d + i];
    S.dp[i] = v;
    S.piv[i] = i;
    m = fmax(m, v);
  }
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if (lane == 0) red[w] = m;
  __syncthreads();
  if (tid == 0) {
    double mm = 0.0;
    for (int i = 0; i < LT / 64; ++i) mm = fmax(mm, red[i]);
    S.thr[0] = tol * mm;
    S.rank[0] = (mm > 0.0 && d > 0) ? -1 : 0;
  }
}

__global__ void __launch_bounds__(LT) k_chol_panel(const CholState* st, int j0, int nb) {
  const CholState S = st[blockIdx.x];
  const int d = S.d, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (j0 >= d || S.rank[0] >= 0) return;
  __shared__ double dp[CHOL_MAX];
  __shared__ int piv[CHOL_MAX];
  __shared__ double red_v[LT / 64];
  __shared__ int red_i[LT / 64];
  __shared__ int s_stop;
  for (int i = tid; i < d; i += LT) {
    dp[i] = S.dp[i];
    piv[i] = S.piv[i];
  }
  if (tid == 0) s_stop = -1;
  __syncthreads();
  const double thr = S.thr[0];
  const int jend = min(j0 + nb, d);
  for (int j = j0; j < jend; ++j) {
    double bv = -1.0;
    int bi = d;
    for (int i = j + tid; i < d; i += LT)
      if (dp[i] > bv) {
        bv = dp[i];
        bi = i;
      }
    for (int o = 32; o > 0; o >>= 1) {
      double ov = __shfl_xor(bv, o);
      int oi = __shfl_xor(bi, o);
      if (ov > bv || (ov == bv && oi < bi)) {
        bv = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      red_v[w] = bv;
      red_i[w] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double v = -1.0;
      int p = d;
      for (int i = 0; i < LT / 64; ++i)
        if (red_v[i] > v || (red_v[i] == v && red_i[i] < p)) {
          v = red_v[i];
          p = red_i[i];
        }
      if (!(v > thr)) {
        s_stop = j;
      } else if (p != j) {
        double t = dp[j];
        dp[j] = dp[p];
        dp[p] = t;
        int ti = piv[j];
        piv[j] = piv[p];
        piv[p] = ti;
      }
    }
    __syncthreads();
    if (s_stop >= 0) break;
    const int cj = piv[j];
    const double rjj = sqrt(dp[j]);
    if (tid == 0) S.R[(int64_t)j * d + cj] = rjj;
    for (int i = j + 1 + tid; i < d; i += LT) {
      const int ci = piv[i];
      double sacc = S.G[(int64_t)cj * d + ci];
      for (int l = j0; l < j; ++l) sacc -= S.R[(int64_t)l * d + cj] * S.R[(int64_t)l * d + ci];
      const double r = sacc / rjj;
      S.R[(int64_t)j * d + ci] = r;
      dp[i] = fmax(dp[i] - r * r, 0.0);
    }
    __syncthreads();
  }
  for (int i = tid; i < d; i += LT) {
    S.dp[i] = dp[i];
    S.piv[i] = piv[i];
  }
  if (tid == 0) {
    if (s_stop >= 0)
      S.rank[0] = s_stop;
    else if (jend == d)
      S.rank[0] = d;
  }
}

// ---------------------------------------------------------------------------
// Cyclic Jacobi eigensolver for a symmetric n x n matrix (n <= 128), one
// workgroup per matrix, in two phases.
// Phase 1 keeps the upper triangle in LDS and sweeps it in round-robin
// order: per round, n/2 disjoint rotations are chosen, then every 2 x 2
// block (pair k1, pair k2) is updated as J_k1^T A J_k2 by one thread, which
// needs one barrier per round and no eigenvector traffic. The rotations are
// logged to global memory. Phase 2 reuses the LDS for V = I and replays the
// log: each wave owns a set of rows of V and applies every round to them
// (lane k = rotation k), so rounds need no workgroup barrier. Sweeps stop
// when the off-diagonal norm^2 is <= 1e-30 of the diagonal norm^2.
// Outputs: eigenvalues descending (ties: lower index first) and the matching
// eigenvector columns (row-major n x n).
constexpr int JAC_SWEEPS = 30;

struct EigJob {
  const double* H;  // n x n input
  double* V;        // n x n eigenvectors (columns), output
  double* W;        // n eigenvalues, output (descending)
  double2* rot;     // rotation log: (c, s) per rotation
  int* rpq;         // rotation log: p | q << 16
  int n;
  int pad;
};

__host__ __device__ inline int64_t jacobi_log_len(int n) {
  const int n2 = n + (n & 1);
  return (int64_t)JAC_SWEEPS * (n2 - 1) * (n2 / 2);
}

__device__ inline void rr_pair(int n2, int r, int i, int& p, int& q) {
  // round-robin tournament on n2 (even) players: fixed player n2-1
  if (i == 0) {
    p = r;
    q = n2 - 1;
  } else {
    p = (r + i) % (n2 - 1);
    q = (r - i + (n2 - 1)) % (n2 - 1);
  }
  if (p > q) {
    int t = p;
    p = q;
    q = t;
  }
}

__global__ void __launch_bounds__(LT) k_jacobi_eig(const EigJob* jobs) {
  const EigJob J = jobs[blockIdx.x];
  const int n = J.n;
  if (n <= 0) return;
  __shared__ double A[JMAX][JMAX + 1];
  __shared__ double2 cs[JMAX / 2];
  __shared__ int pq[JMAX / 2];
  __shared__ double ev[JMAX];
  __shared__ int rk[JMAX];
  __shared__ double red[2][LT / 64];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int n2 = n + (n & 1);  // an odd order gets a zero row / column
  const int np = n2 / 2;
  for (int e = tid; e < n2 * n2; e += LT) {
    const int i = e / n2, j = e % n2;
    if (i <= j) A[i][j] = (j < n) ? J.H[(int64_t)i * n + j] : 0.0;
  }
  __syncthreads();
  int nr = 0;  // rounds done (the same in every thread)
  for (int sweep = 0; sweep < JAC_SWEEPS; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < n2 * n2; e += LT) {
      const int i = e / n2, j = e % n2;
      if (i < j)
        off += A[i][j] * A[i][j];
      else if (i == j)
        tot += A[i][i] * A[i][i];
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o);
      tot += __shfl_xor(tot, o);
    }
    if (lane == 0) {
      red[0][w] = off;
      red[1][w] = tot;
    }
    __syncthreads();
    off = 0.0;
    tot = 0.0;
    for (int i = 0; i < LT / 64; ++i) {
      off += red[0][i];
      tot += red[1][i];
    }
    __syncthreads();
    if (off == 0.0 || 2.0 * off <= 1e-30 * tot) break;
    for (int r = 0; r < n2 - 1; ++r, ++nr) {
      if (tid < np) {
        int p, q;
        rr_pair(n2, r, tid, p, q);
        double c = 1.0, s = 0.0;
        const double apq = A[p][q];
        if (apq != 0.0) {
          const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
          const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
        }
        cs[tid] = make_double2(c, s);
        pq[tid] = p | (q << 16);
        J.rot[(int64_t)nr * np + tid] = make_double2(c, s);
        J.rpq[(int64_t)nr * np + tid] = p | (q << 16);
      }
      __syncthreads();
      for (int e = tid; e < np * np; e += LT) {
        const int k1 = e / np, k2 = e % np;
        if (k1 > k2) continue;
        const int v1 = pq[k1];
        const int p1 = v1 & 0xffff, q1 = v1 >> 16;
        const double2 r1 = cs[k1];
        if (k1 == k2) {
          const double apq = A[p1][q1], t = r1.y / r1.x;
          A[p1][p1] -= t * apq;
          A[q1][q1] += t * apq;
          A[p1][q1] = 0.0;
        } else {
          const int v2 = pq[k2];
          const int p2 = v2 & 0xffff, q2 = v2 >> 16;
          const double2 r2 = cs[k2];
          double* a00 = &A[min(p1, p2)][max(p1, p2)];
          double* a01 = &A[min(p1, q2)][max(p1, q2)];
          double* a10 = &A[min(q1, p2)][max(q1, p2)];
          double* a11 = &A[min(q1, q2)][max(q1, q2)];
          const double b00 = *a00, b01 = *a01, b10 = *a10, b11 = *a11;
          const double r00 = r1.x * b00 - r1.y * b10, r01 = r1.x * b01 - r1.y * b11;
          const double r10 = r1.y * b00 + r1.x * b10, r11 = r1.y * b01 + r1.x * b11;
          *a00 = r2.x * r00 - r2.y * r01;
          *a01 = r2.y * r00 + r2.x * r01;
          *a10 = r2.x * r10 - r2.y * r11;
          *a11 = r2.y * r10 + r2.x * r11;
        }
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < n; i += LT) ev[i] = A[i][i];
  __syncthreads();
  for (int e = tid; e < n2 * n2; e += LT) {
    const int i = e / n2, j = e % n2;
    A[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (lane < np) {
    for (int t = 0; t < nr; ++t) {
      const double2 r = J.rot[(int64_t)t * np + lane];
      const int v = J.rpq[(int64_t)t * np + lane];
      const int p = v & 0xffff, q = v >> 16;
      for (int i = w; i < n2; i += LT / 64) {
        const double vp = A[i][p], vq = A[i][q];
        A[i][p] = r.x * vp - r.y * vq;
        A[i][q] = r.y * vp + r.x * vq;
      }
    }
  }
  __syncthreads();
  for (int i = tid; i < n; i += LT) {
    const double v = ev[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double u = ev[j];
      rank += (u > v) || (u == v && j < i);
    }
    rk[i] = rank;
    J.W[rank] = v;
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += LT) {
    const int r = e / n, i = e % n;
    J.V[(int64_t)r * n + rk[i]] = A[r][i];
  }
}

// ---------------------------------------------------------------------------
// Rank-revealing orthonormalisation factor (one workgroup per matrix): for
// the Gram matrix G = Y^T Y (p x p, p <= 128), symmetric-pivoted Cholesky
// G = P^T R^T R P stops at the numerical rank r (largest remaining pivot not
// above tol * largest diagonal). The output M (p x p) has
// M[piv[i]][c] = R11^-1[i][c] for i <= c < r and zeros elsewhere, so Y M has
// r orthonormal columns followed by zero columns: dependent directions are
// dropped instead of amplified.
// The factorisation is left-looking in LDS: row j of R is written over the
// (no longer needed) row of G of the j-th pivot, eight threads per column
// share each dot product, and every wave chooses the pivot itself from a
// double-buffered diagonal, so a step costs one barrier. R is then
// gathered into pivot order, padded with the identity to order 128, and
// inverted in place: 16 x 16 diagonal blocks by back substitution, then
// three doubling levels [U11 U12; 0 U22]^-1 = [U11^-1, -U11^-1 U12 U22^-1;
// 0, U22^-1] with FP64 MFMA tiles (the product U11^-1 U12 is staged in the
// free lower triangle).
struct OrthJob {
  const double* G;
  double* M;  // p x p output
  int p;
  int pad;
};

__global__ void __launch_bounds__(LT) k_orth_factor(const OrthJob* jobs, double tol) {
  const OrthJob J = jobs[blockIdx.x];
  const int p = J.p;
  __shared__ double A[JMAX][JMAX + 1];
  __shared__ double dpb[2][JMAX];
  __shared__ int sel[JMAX], pos[JMAX];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int e = tid; e < p * p; e += LT) A[e / p][e % p] = J.G[e];
  for (int i = tid; i < JMAX; i += LT) {
    pos[i] = -1;
    dpb[0][i] = (i < p) ? J.G[(int64_t)i * p + i] : -1.0;
  }
  __syncthreads();
  double mx = 0.0;
  for (int i = lane; i < p; i += 64) mx = fmax(mx, dpb[0][i]);
  mx = wave_max(mx);
  const double thr = tol * mx;
  int r = (mx > 0.0) ? p : 0;
  int cur = 0;
  for (int j = 0; j < r; ++j) {
    const double* dpc = dpb[cur];
    double* dpn = dpb[cur ^ 1];
    double bv = -1.0;
    int bi = JMAX;
    for (int i = lane; i < p; i += 64) {
      const double v = dpc[i];
      if (v > bv) {
        bv = v;
        bi = i;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(bv, o);
      const int oi = __shfl_xor(bi, o);
      if (ov > bv || (ov == bv && oi < bi)) {
        bv = ov;
        bi = oi;
      }
    }
    if (!(bv > thr)) {
      r = j;
      break;
    }
    const int cj = bi;
    const double rjj = sqrt(bv), inv = 1.0 / rjj;
    const int c = tid >> 3, sub = tid & 7;
    const bool act = c < p && c != cj && dpc[c] >= 0.0;
    double sacc = 0.0;
    if (act)
      for (int l = sub; l < j; l += 8) {
        const int o = sel[l];
        sacc += A[o][cj] * A[o][c];
      }
    sacc += __shfl_xor(sacc, 1);
    sacc += __shfl_xor(sacc, 2);
    sacc += __shfl_xor(sacc, 4);
    if (sub == 0 && c < p) {
      if (act) {
        const double v = (A[cj][c] - sacc) * inv;
        A[cj][c] = v;
        dpn[c] = fmax(dpc[c] - v * v, 0.0);
      } else {
        dpn[c] = -1.0;
      }
    }
    if (tid == 0) {
      A[cj][cj] = rjj;
      sel[j] = cj;
      pos[cj] = j;
    }
    cur ^= 1;
    __syncthreads();
  }
  // R in pivot order, identity beyond the rank (through registers)
  double v[JMAX * JMAX / LT];
#pragma unroll
  for (int u = 0; u < JMAX * JMAX / LT; ++u) {
    const int e = tid + u * LT, l = e >> 7, i = e & 127;
    double x = 0.0;
    if (l <= i) x = (i < r) ? A[sel[l]][sel[i]] : (l == i ? 1.0 : 0.0);
    v[u] = x;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < JMAX * JMAX / LT; ++u) {
    const int e = tid + u * LT;
    A[e >> 7][e & 127] = v[u];
  }
  __syncthreads();
  // 16 x 16 diagonal blocks: lane c of wave w solves column c of block w
  if (w < JMAX / 16 && lane < 16) {
    const int o = 16 * w, c = lane;
    double x[16];
#pragma unroll
    for (int i = 15; i >= 0; --i) {
      double s = (i == c) ? 1.0 : 0.0;
#pragma unroll
      for (int q = i + 1; q < 16; ++q) s -= A[o + i][o + q] * x[q];
      x[i] = (i <= c) ? s / A[o + i][o + i] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (i <= c) A[o + i][o + c] = x[i];
  }
  __syncthreads();
  const int li = lane & 15, lk = lane >> 4;
  for (int h = 16; h < JMAX; h *= 2) {
    const int m = 2 * h, nt = h / 16, tiles = (JMAX / m) * nt * nt;
    const int pr = w / (nt * nt), t = w % (nt * nt);
    const int b = pr * m, i0 = 16 * (t / nt), j0 = 16 * (t % nt);
    if (w < tiles) {  // T = U11^-1 U12 into the lower-left block
      d4 acc = {0.0, 0.0, 0.0, 0.0};
      for (int k0 = i0; k0 < h; k0 += 4) {
        const int k = k0 + lk;
        const double a = (k >= i0 + li) ? A[b + i0 + li][b + k] : 0.0;
        const double bb = A[b + k][b + h + j0 + li];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc, 0, 0, 0);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) A[b + h + i0 + lk + 4 * q][b + j0 + li] = acc[q];
    }
    __syncthreads();
    if (w < tiles) {  // U12 <- -T U22^-1
      d4 acc = {0.0, 0.0, 0.0, 0.0};
      for (int k0 = 0; k0 < j0 + 16; k0 += 4) {
        const int k = k0 + lk;
        const double a = A[b + h + i0 + li][b + k];
        const double bb = (k <= j0 + li) ? A[b + h + k][b + h + j0 + li] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc, 0, 0, 0);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) A[b + i0 + lk + 4 * q][b + h + j0 + li] = -acc[q];
    }
    __syncthreads();
  }
  for (int e = tid; e < p * p; e += LT) {
    const int o = e / p, c = e % p, i = pos[o];
    J.M[e] = (i >= 0 && c < r && i <= c) ? A[i][c] : 0.0;
  }
}

// ---------------------------------------------------------------------------
// global top-chi selection over all groups (one workgroup). Order: larger
// value, then lower charge rank of the group, then lower index.
__global__ void __launch_bounds__(LT) k_select(const double* vals, const int* grp, const int* idx,
                                               const int* crank, int n, int ngroups, int64_t chi,
                                               double cutoff, int* kept, double* stats) {
  __shared__ int cnt[1024];
  __shared__ double red[LT / 64];
  __shared__ double s_max;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int g = tid; g < ngroups; g += LT) cnt[g] = 0;
  double m = 0;
  for (int i = tid; i < n; i += LT) m = fmax(m, vals[i]);
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if (lane == 0) red[w] = m;
  __syncthreads();
  if (tid == 0) {
    double mm = 0;
    for (int i = 0; i < LT / 64; ++i) mm = fmax(mm, red[i]);
    s_max = mm;
  }
  __syncthreads();
  double disc = 0;
  for (int i = tid; i < n; i += LT) {
    const double v = vals[i];
    const int cg = crank[grp[i]];
    int64_t rank = 0;
    for (int j = 0; j < n; ++j) {
      const double u = vals[j];
      const int cu = crank[grp[j]];
      rank += (u > v) || (u == v && (cu < cg || (cu == cg && idx[j] < idx[i])));
    }
    bool keep = rank < chi && v > cutoff * s_max && v > 0.0;
    if (keep)
      atomicAdd(&cnt[grp[i]], 1);
    else
      disc += v * v;
    if (rank == chi - 1) stats[1] = v;  // chi-th value
    if (rank == chi) stats[2] = v;      // (chi+1)-th value
  }
  for (int o = 32; o > 0; o >>= 1) disc += __shfl_xor(disc, o);
  if (lane == 0) red[w] = disc;
  __syncthreads();
  if (tid == 0) {
    double s = 0;
    for (int i = 0; i < LT / 64; ++i) s += red[i];
    stats[0] = s;
  }
  for (int g = tid; g < ngroups; g += LT) kept[g] = cnt[g];
}

// ---------------------------------------------------------------------------
// small elementwise helpers
__global__ void k_sum_partials(const double* P, int64_t n, int nparts, double* out) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0;
  for (int k = 0; k < nparts; ++k) s += P[(int64_t)k * n + i];
  out[i] = s;
}

// deterministic pseudo-random start block (splitmix64 of the index)
__global__ void k_fill_random(double* X, int64_t n, uint64_t seed) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  X[i] = (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

// column scaling: X[:, j] *= f(w[j]) for j < k (row-major rows x ld)
// mode 0: 1/sqrt(w); mode 1: sqrt(w); mode 2: 1/w
__global__ void k_scale_cols(double* X, int64_t rows, int64_t ld, int k, const double* w, int mode) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= rows * k) return;
  int64_t r = e / k;
  int j = (int)(e % k);
  double v = w[j];
  double f = mode == 0 ? 1.0 / sqrt(v) : (mode == 1 ? sqrt(v) : 1.0 / v);
  X[r * ld + j] *= f;
}

__global__ void k_sqrt_inplace(double* w, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[i] = sqrt(fmax(w[i], 0.0));
}

template <typename S, typename D>
__global__ void k_convert(const S* x, D* y, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = (D)x[i];
}

static void launch_1d(int64_t n, hipStream_t s, void (*k)(double*, int), double* a, int b) {
  if (n <= 0) return;
  LAUNCH(k, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, a, b);
  HIPC(hipGetLastError());
}

// ---------------------------------------------------------------------------
static GemmGroup plain_group(int64_t M, int64_t N, int64_t K, int64_t a_off, int64_t lda, int ta,
                             int64_t b_off, int64_t ldb, int tb, int64_t c_off, int64_t ldc) {
  GemmGroup g;
  std::memset(&g, 0, sizeof(g));
  g.M = M;
  g.N = N;
  g.K = K;
  g.a_off = a_off;
  g.lda = lda;
  g.transA = ta;
  g.b_off = b_off;
  g.ldb = ldb;
  g.transB = tb;
  g.c_off = c_off;
  g.ldc = ldc;
  return g;
}

// per bond sector q
struct Sect {
  int64_t M, N, d;       // rows of A~, cols of B~, bond dim
  int64_t a_off, b_off;  // into A~ / B~
  int rA = 0, rB = 0;    // Cholesky ranks
  int ns = 0;            // order of H
  int p = 0;             // subspace size (<= JMAX) or ns
  bool iterate = false;
  int kept = 0;
  Q charge;
  int crank = 0;
};

// Leading spectral data of X (rA x rB) per sector. Output: eigenvalues of the
// smaller Gram matrix H (= s^2, descending) in W and its eigenvectors in V
// (ns x p, ld p), ns = min(rA, rB). Orders <= JMAX: Jacobi on H directly.
// Larger orders: block power iteration with X and X^T alternately (the Gram
// matrices of the iterates then span s^2, not s^4), each iterate
// orthonormalised twice by the rank-revealing factor, and a Rayleigh-Ritz
// step T = (X Q)^T (X Q) every 8 iterations until the leading Ritz values are
// stable (relative change <= 1e-14 of the largest) or 96 iterations.
static void eig_top(std::vector<Sect>& S, int64_t chi, const double* H, const std::vector<int64_t>& hoff,
                    const double* X, const std::vector<int64_t>& xoff, double* V, const std::vector<int64_t>& voff,
                    double* W, const std::vector<int64_t>& woff, hipStream_t s) {
  const int ng = (int)S.size();
  std::vector<EigJob> ej;
  std::vector<int64_t> log_off;
  int64_t log_n = 0;
  for (int g = 0; g < ng; ++g)
    if (!S[g].iterate && S[g].ns > 0) {
      log_off.push_back(log_n);
      log_n += jacobi_log_len(S[g].ns);
    }
  DBuf<double2> lrot(std::max<int64_t>(log_n, 1), s);
  DBuf<int> lpq(std::max<int64_t>(log_n, 1), s);
  {
    int t = 0;
    for (int g = 0; g < ng; ++g)
      if (!S[g].iterate && S[g].ns > 0) {
        EigJob j;
        j.H = H + hoff[g];
        j.V = V + voff[g];
        j.W = W + woff[g];
        j.rot = lrot.p + log_off[t];
        j.rpq = lpq.p + log_off[t++];
        j.n = S[g].ns;
        j.pad = 0;
        ej.push_back(j);
      }
  }
  if (!ej.empty()) {
    DBuf<EigJob> dj = to_device(ej, s);
    LAUNCH(k_jacobi_eig, dim3((unsigned)ej.size()), dim3(LT), 0, s, dj.p);
    HIPC(hipStreamSynchronize(s));
  }
  std::vector<int> it;
  for (int g = 0; g < ng; ++g)
    if (S[g].iterate) it.push_back(g);
  if (it.empty()) return;
  const int ni = (int)it.size();
  // per iterated sector: eigen side e (dim ne), other side o (dim no)
  std::vector<int64_t> ne(ni), no(ni), qoff(ni), zoff(ni), goff(ni);
  int64_t qn = 0, zn = 0, gn = 0;
  for (int t = 0; t < ni; ++t) {
    const Sect& x = S[it[t]];
    const bool eR = x.rB <= x.rA;  // eigenvectors live in the rB space
    ne[t] = eR ? x.rB : x.rA;
    no[t] = eR ? x.rA : x.rB;
    qoff[t] = qn;
    qn += ne[t] * x.p;
    zoff[t] = zn;
    zn += no[t] * x.p;
    goff[t] = gn;
    gn += (int64_t)x.p * x.p;
  }
  DBuf<double> Qa(qn, s), Qb(qn, s), Za(zn, s), Zb(zn, s), Gm(gn, s), Mm(gn, s), Tm(gn, s), Wv(gn, s),
      Wt(std::max<int64_t>(ni * (int64_t)JMAX, 1), s);
  DBuf<double2> rrot(ni * jacobi_log_len(JMAX), s);
  DBuf<int> rrpq(ni * jacobi_log_len(JMAX), s);
  // GEMM plans (reused every iteration)
  std::vector<GemmGroup> gxq, gxz, gq_gram, gz_gram, gq_app, gz_app, gt;
  for (int t = 0; t < ni; ++t) {
    const Sect& x = S[it[t]];
    const int64_t p = x.p;
    const bool eR = x.rB <= x.rA;
    // Z = op(X) Q : eR -> X (rA x rB) * Q (rB x p); else X^T (rB x rA) * Q (rA x p)
    gxq.push_back(plain_group(no[t], p, ne[t], xoff[it[t]], x.rB, eR ? 0 : 1, qoff[t], p, 0, zoff[t], p));
    // Q = op(X)^T Z : eR -> X^T * Z; else X * Z
    gxz.push_back(plain_group(ne[t], p, no[t], xoff[it[t]], x.rB, eR ? 1 : 0, zoff[t], p, 0, qoff[t], p));
    gq_gram.push_back(plain_group(p, p, ne[t], qoff[t], p, 1, qoff[t], p, 0, goff[t], p));
    gz_gram.push_back(plain_group(p, p, no[t], zoff[t], p, 1, zoff[t], p, 0, goff[t], p));
    gq_app.push_back(plain_group(ne[t], p, p, qoff[t], p, 0, goff[t], p, 0, qoff[t], p));
    gz_app.push_back(plain_group(no[t], p, p, zoff[t], p, 0, goff[t], p, 0, zoff[t], p));
    gt.push_back(plain_group(ne[t], p, p, qoff[t], p, 0, goff[t], p, 0, voff[it[t]], p));
  }
  GemmPlan Pxq, Pxz, Pqg, Pzg, Pqa, Pza, Pv;
  gemm_plan(Pxq, gxq, FTN_GEMM_F64, s);
  gemm_plan(Pxz, gxz, FTN_GEMM_F64, s);
  gemm_plan(Pqg, gq_gram, FTN_GEMM_F64, s);
  gemm_plan(Pzg, gz_gram, FTN_GEMM_F64, s);
  gemm_plan(Pqa, gq_app, FTN_GEMM_F64, s);
  gemm_plan(Pza, gz_app, FTN_GEMM_F64, s);
  gemm_plan(Pv, gt, FTN_GEMM_F64, s);
  std::vector<OrthJob> oj;
  std::vector<EigJob> ejr;
  for (int t = 0; t < ni; ++t) {
    OrthJob o;
    o.G = Gm.p + goff[t];
    o.M = Mm.p + goff[t];
    o.p = S[it[t]].p;
    o.pad = 0;
    oj.push_back(o);
    EigJob e;
    e.H = Tm.p + goff[t];
    e.V = Wv.p + goff[t];
    e.W = Wt.p + (int64_t)t * JMAX;
    e.rot = rrot.p + t * jacobi_log_len(JMAX);
    e.rpq = rrpq.p + t * jacobi_log_len(JMAX);
    e.n = S[it[t]].p;
    e.pad = 0;
    ejr.push_back(e);
  }
  DBuf<OrthJob> doj = to_device(oj, s);
  DBuf<EigJob> dej = to_device(ejr, s);
  HIPC(hipStreamSynchronize(s));
  const double tol = 1e-13;
  // Y (buffer y) <- orthonormal basis of its columns, through scratch o
  auto orth = [&](const GemmPlan& gram, const GemmPlan& app, double* y, double* o) {
    run_gemm(gram, FTN_F64, y, y, Gm.p, nullptr, s);
    LAUNCH(k_orth_factor, dim3((unsigned)ni), dim3(LT), 0, s, doj.p, tol);
    run_gemm(app, FTN_F64, y, Mm.p, o, nullptr, s);
  };
  LAUNCH(k_fill_random, dim3((unsigned)cdiv(qn, 256)), dim3(256), 0, s, Qa.p, qn, (uint64_t)0x5eedf00dull);
  orth(Pqg, Pqa, Qa.p, Qb.p);
  orth(Pqg, Pqa, Qb.p, Qa.p);  // Q in Qa
  std::vector<double> prev, cur(ni * (int64_t)JMAX);
  const int max_iter = 96, check = 8;
  for (int k = 1; k <= max_iter; ++k) {
    run_gemm(Pxq, FTN_F64, X, Qa.p, Za.p, nullptr, s);
    orth(Pzg, Pza, Za.p, Zb.p);
    orth(Pzg, Pza, Zb.p, Za.p);
    run_gemm(Pxz, FTN_F64, X, Za.p, Qa.p, nullptr, s);
    orth(Pqg, Pqa, Qa.p, Qb.p);
    orth(Pqg, Pqa, Qb.p, Qa.p);
    if (k % check == 0 || k == max_iter) {
      // Rayleigh-Ritz: Z = op(X) Q; T = Z^T Z
      run_gemm(Pxq, FTN_F64, X, Qa.p, Za.p, nullptr, s);
      run_gemm(Pzg, FTN_F64, Za.p, Za.p, Tm.p, nullptr, s);
      LAUNCH(k_jacobi_eig, dim3((unsigned)ni), dim3(LT), 0, s, dej.p);
      HIPC(hipMemcpyAsync(cur.data(), Wt.p, cur.size() * 8, hipMemcpyDeviceToHost, s));
      HIPC(hipStreamSynchronize(s));
      bool done = !prev.empty();
      for (int t = 0; t < ni && done; ++t) {
        const int kk = (int)std::min<int64_t>(chi, S[it[t]].p);
        const double top = std::max(cur[(int64_t)t * JMAX], 1e-300);
        for (int q = 0; q < kk; ++q)
          if (std::fabs(cur[(int64_t)t * JMAX + q] - prev[(int64_t)t * JMAX + q]) > 1e-14 * top) done = false;
      }
      prev = cur;
      if (done) break;
    }
  }
  // outputs: eigenvalues, eigenvectors V = Q Wv
  for (int t = 0; t < ni; ++t)
    HIPC(hipMemcpyAsync(W + woff[it[t]], Wt.p + (int64_t)t * JMAX, S[it[t]].p * 8, hipMemcpyDeviceToDevice, s));
  run_gemm(Pv, FTN_F64, Qa.p, Wv.p, V, nullptr, s);
  HIPC(hipStreamSynchronize(s));
}

CompressResult op_compress_bond(const Tensor& a, const Tensor& b, int la, int lb, int64_t chi, double cutoff,
                                int conv, hipStream_t s) {
  CompressResult res;
  if (a.sym() != b.sym()) fail(FTN_EINVAL, "symmetry mismatch");
  if (a.dtype != b.dtype) fail(FTN_ENOTSUP, "operands must have the same dtype");
  if (conv != FTN_LOCAL && conv != FTN_GLOBAL) fail(FTN_EINVAL, "unknown convention");
  const Leg& LA = a.legs()[la];
  const Leg& LB = b.legs()[lb];
  if (LA.dual == LB.dual) fail(FTN_ECHARGE, "bond legs must have opposite duals");
  const int sym = a.sym();
  if (a.size() == 0 || b.size() == 0) fail(FTN_EINVAL, "compress_bond: empty tensor");
  const int gk = a.dtype == FTN_F64 ? FTN_GEMM_F64 : FTN_GEMM_F32;
  auto P = dot_plan(a, b, {la}, {lb}, FTN_GLOBAL, gk, s);
  DotPlanView pv = dot_plan_view(*P);
  // fused matrices (FP64)
  DBuf<double> At(pv.asz, s), Bt(pv.bsz, s);
  if (a.dtype == FTN_F64) {
    run_perm(0, a.S(), a.dtype, *pv.pa, a.data, At.p, s);
    run_perm(0, b.S(), b.dtype, *pv.pb, b.data, Bt.p, s);
  } else {
    DBuf<float> a32(pv.asz, s), b32(pv.bsz, s);
    run_perm(0, a.S(), a.dtype, *pv.pa, a.data, a32.p, s);
    run_perm(0, b.S(), b.dtype, *pv.pb, b.data, b32.p, s);
    if (pv.asz)
      LAUNCH((k_convert<float, double>), dim3((unsigned)cdiv(pv.asz, 256)), dim3(256), 0, s, a32.p,
                         At.p, pv.asz);
    if (pv.bsz)
      LAUNCH((k_convert<float, double>), dim3((unsigned)cdiv(pv.bsz, 256)), dim3(256), 0, s, b32.p,
                         Bt.p, pv.bsz);
    HIPC(hipGetLastError());
    HIPC(hipStreamSynchronize(s));
  }
  // sectors: one GEMM group per bond charge present on both legs
  std::vector<Sect> S;
  for (size_t gi = 0; gi < pv.groups.size(); ++gi) {
    const GemmGroup& g = pv.groups[gi];
    if (g.K == 0) continue;  // charge absent on one side: contributes nothing
    Sect x;
    x.M = g.M;
    x.N = g.N;
    x.d = g.K;
    x.a_off = g.a_off;
    x.b_off = g.b_off;
    x.charge = q_signed(sym, LA.dual, pv.gq[gi]);  // Q = sigma(la) q
    S.push_back(x);
  }
  const int ng = (int)S.size();
  if (ng == 0) {
    auto leg_str = [](const Leg& l) {
      std::string r = "dual " + std::to_string(l.dual) + " [";
      for (int k = 0; k < l.nsect(); ++k)
        r += "(" + std::to_string(l.q[k].a) + "," + std::to_string(l.q[k].b) + "):" + std::to_string(l.d[k]) + " ";
      return r + "]";
    };
    std::string g;
    for (size_t gi = 0; gi < pv.groups.size(); ++gi)
      g += " {M " + std::to_string(pv.groups[gi].M) + " N " + std::to_string(pv.groups[gi].N) + " K " +
           std::to_string(pv.groups[gi].K) + "}";
    fail(FTN_EINVAL, "compress_bond: no charge sector common to both bond legs: A leg " + std::to_string(la) +
                         " of " + std::to_string(a.ndim()) + " " + leg_str(LA) + ", B leg " + std::to_string(lb) +
                         " of " + std::to_string(b.ndim()) + " " + leg_str(LB) + ", sizes " +
                         std::to_string(a.size()) + " / " + std::to_string(b.size()) + ", groups" + g);
  }
  {
    std::vector<int> order(ng);
    for (int g = 0; g < ng; ++g) order[g] = g;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return q_lt(S[x].charge, S[y].charge); });
    for (int r = 0; r < ng; ++r) S[order[r]].crank = r;
  }
  // Gram matrices with split-K
  std::vector<int64_t> goffA(ng), goffB(ng);
  int64_t gsz = 0;
  for (int g = 0; g < ng; ++g) {
    goffA[g] = gsz;
    gsz += S[g].d * S[g].d;
    goffB[g] = gsz;
    gsz += S[g].d * S[g].d;
  }
  DBuf<double> Gm(std::max<int64_t>(gsz, 1), s);
  {
    int64_t tiles = 0;
    for (auto& x : S) tiles += 2 * cdiv(x.d, 64) * cdiv(x.d, 64);
    int64_t maxk = 1;
    for (auto& x : S) maxk = std::max(maxk, std::max(x.M, x.N));
    int nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(2048, std::max<int64_t>(tiles, 1)), cdiv(maxk, 256)));
    DBuf<double> part((int64_t)nsplit * std::max<int64_t>(gsz, 1), s);
    std::vector<GemmGroup> gA, gB;
    for (int k = 0; k < nsplit; ++k)
      for (int g = 0; g < ng; ++g) {
        const Sect& x = S[g];
        int64_t ca = cdiv(x.M, nsplit), k0 = std::min<int64_t>(k * ca, x.M), k1 = std::min<int64_t>(k0 + ca, x.M);
        // G_A = A~^T A~ : op(A) = A~^T (transA, lda = d), op(B) = A~ (ldb = d)
        gA.push_back(plain_group(x.d, x.d, k1 - k0, x.a_off + k0 * x.d, x.d, 1, x.a_off + k0 * x.d, x.d, 0,
                                 (int64_t)k * gsz + goffA[g], x.d));
        int64_t cb = cdiv(x.N, nsplit), j0 = std::min<int64_t>(k * cb, x.N), j1 = std::min<int64_t>(j0 + cb, x.N);
        // G_B = B~ B~^T : op(A) = B~ (lda = N), op(B) = B~^T (transB, ldb = N)
        gB.push_back(plain_group(x.d, x.d, j1 - j0, x.b_off + j0, x.N, 0, x.b_off + j0, x.N, 1,
                                 (int64_t)k * gsz + goffB[g], x.d));
      }
    run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gA, At.p, At.p, part.p, nullptr, s);
    run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gB, Bt.p, Bt.p, part.p, nullptr, s);
    LAUNCH(k_sum_partials, dim3((unsigned)cdiv(gsz, 256)), dim3(256), 0, s, part.p, gsz, nsplit, Gm.p);
    HIPC(hipGetLastError());
  }
  // pivoted Cholesky of both Gram matrices (blocked: panel + MFMA update)
  DBuf<double> Rm(std::max<int64_t>(gsz, 1), s);
  HIPC(hipMemsetAsync(Rm.p, 0, std::max<int64_t>(gsz, 1) * 8, s));
  {
    const int nm = 2 * ng;
    std::vector<int64_t> moff(nm), md(nm);
    int64_t dsum = 0, dmax = 0;
    for (int g = 0; g < ng; ++g) {
      if (S[g].d > CHOL_MAX) fail(FTN_ENOTSUP, "bond sector larger than 4096");
      moff[2 * g] = goffA[g];
      moff[2 * g + 1] = goffB[g];
      md[2 * g] = md[2 * g + 1] = S[g].d;
      dsum += 2 * S[g].d;
      dmax = std::max(dmax, S[g].d);
    }
    DBuf<double> dpv(std::max<int64_t>(dsum, 1), s), thr(nm, s);
    DBuf<int> pv(std::max<int64_t>(dsum, 1), s), rk(nm, s);
    std::vector<CholState> cs(nm);
    int64_t o = 0;
    for (int m = 0; m < nm; ++m) {
      cs[m] = CholState{Gm.p + moff[m], Rm.p + moff[m], dpv.p + o, pv.p + o, thr.p + m, rk.p + m, (int)md[m], 0};
      o += md[m];
    }
    DBuf<CholState> dcs = to_device(cs, s);
    const int nb = 64;
    LAUNCH(k_chol_init, dim3(nm), dim3(LT), 0, s, dcs.p, 1e-13);
    std::vector<GemmPlan> upd;
    for (int j0 = 0; j0 < dmax; j0 += nb) {
      LAUNCH(k_chol_panel, dim3(nm), dim3(LT), 0, s, dcs.p, j0, nb);
      std::vector<GemmGroup> gs;
      for (int m = 0; m < nm; ++m) {
        const int64_t d = md[m];
        if (j0 + nb >= d) continue;  // no later panel reads this matrix
        const int64_t kk = std::min<int64_t>(nb, d - j0);
        gs.push_back(plain_group(d, d, kk, moff[m] + j0 * d, d, 1, moff[m] + j0 * d, d, 0, moff[m], d));
      }
      if (!gs.empty()) {
        upd.emplace_back();
        gemm_plan(upd.back(), gs, FTN_GEMM_F64, s);
        run_gemm(upd.back(), FTN_F64, Rm.p, Rm.p, Gm.p, nullptr, s, -1.0, 1.0);
      }
    }
    std::vector<int> rks(nm);
    HIPC(hipMemcpyAsync(rks.data(), rk.p, nm * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    for (int g = 0; g < ng; ++g) {
      S[g].rA = rks[2 * g];
      S[g].rB = rks[2 * g + 1];
      if (S[g].rA < 0 || S[g].rB < 0) fail(FTN_EINVAL, "internal: Cholesky did not finish");
    }
  }
  // X = R_A R_B^T (rA x rB); H = X^T X (rB <= rA) or X X^T
  std::vector<int64_t> xoff(ng), hoff(ng), voff(ng), woff(ng), uoff(ng);
  int64_t xs = 0, hs = 0, vs = 0, ws = 0, us = 0;
  for (int g = 0; g < ng; ++g) {
    Sect& x = S[g];
    x.ns = std::min(x.rA, x.rB);
    x.iterate = x.ns > JMAX;
    x.p = x.iterate ? JMAX : x.ns;
    xoff[g] = xs;
    xs += (int64_t)x.rA * x.rB;
    hoff[g] = hs;
    hs += (int64_t)x.ns * x.ns;
    voff[g] = vs;
    vs += (int64_t)x.ns * x.p;
    woff[g] = ws;
    ws += std::max(x.p, 1);
    uoff[g] = us;
    us += (int64_t)std::max(x.rA, x.rB) * std::max(x.p, 1);
  }
  DBuf<double> Xm(std::max<int64_t>(xs, 1), s), Hm(std::max<int64_t>(hs, 1), s), Vm(std::max<int64_t>(vs, 1), s),
      Wm(std::max<int64_t>(ws, 1), s), Um(std::max<int64_t>(us, 1), s);
  {
    std::vector<GemmGroup> gx, gh;
    for (int g = 0; g < ng; ++g) {
      const Sect& x = S[g];
      // R_A rows are rA x d (row-major, ld d); X = R_A R_B^T
      gx.push_back(plain_group(x.rA, x.rB, x.d, goffA[g], x.d, 0, goffB[g], x.d, 1, xoff[g], x.rB));
      if (x.rB <= x.rA)  // H = X^T X (rB x rB)
        gh.push_back(plain_group(x.rB, x.rB, x.rA, xoff[g], x.rB, 1, xoff[g], x.rB, 0, hoff[g], x.rB));
      else  // H = X X^T (rA x rA)
        gh.push_back(plain_group(x.rA, x.rA, x.rB, xoff[g], x.rB, 0, xoff[g], x.rB, 1, hoff[g], x.rA));
    }
    run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gx, Rm.p, Rm.p, Xm.p, nullptr, s);
    run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gh, Xm.p, Xm.p, Hm.p, nullptr, s);
  }
  eig_top(S, chi, Hm.p, hoff, Xm.p, xoff, Vm.p, voff, Wm.p, woff, s);
  // singular values = sqrt(eigenvalues); selection
  launch_1d(std::max<int64_t>(ws, 1), s, k_sqrt_inplace, Wm.p, (int)std::max<int64_t>(ws, 1));
  {
    std::vector<int> grp, idx, crank(ng);
    std::vector<int64_t> pos;
    for (int g = 0; g < ng; ++g) {
      crank[g] = S[g].crank;
      for (int i = 0; i < S[g].p; ++i) {
        grp.push_back(g);
        idx.push_back(i);
        pos.push_back(woff[g] + i);
      }
    }
    const int n = (int)grp.size();
    std::vector<double> hw(std::max<int64_t>(ws, 1));
    HIPC(hipMemcpyAsync(hw.data(), Wm.p, hw.size() * 8, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    std::vector<double> vals(n);
    for (int i = 0; i < n; ++i) {
      vals[i] = hw[pos[i]];
      if (!std::isfinite(vals[i])) fail(FTN_ENOCONV, "compress_bond: non-finite singular value");
    }
    DBuf<double> dv = to_device(vals, s);
    DBuf<int> dg = to_device(grp, s), di = to_device(idx, s), dc = to_device(crank, s);
    DBuf<int> dk(std::max(ng, 1), s);
    DBuf<double> dst(4, s);
    std::vector<double> st(4, 0.0);
    HIPC(hipMemsetAsync(dst.p, 0, 32, s));
    if (ng > 1024) fail(FTN_ENOTSUP, "more than 1024 bond sectors");
    // the Gram route resolves singular values to ~1e-8 of the largest, so a
    // relative cutoff below 1e-6 is raised to 1e-6 (values under it are zero)
    const double eff_cut = std::max(cutoff, 1e-6);
    if (n)
      LAUNCH(k_select, dim3(1), dim3(LT), 0, s, dv.p, dg.p, di.p, dc.p, n, ng, chi, eff_cut, dk.p, dst.p);
    HIPC(hipGetLastError());
    std::vector<int> kept(std::max(ng, 1), 0);
    if (n) HIPC(hipMemcpyAsync(kept.data(), dk.p, ng * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(st.data(), dst.p, 32, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    res.discarded = st[0];
    // values dropped because a side's Gram rank was below the sector dim are
    // exactly zero and add nothing
    double a1 = st[1], a2 = st[2];
    res.near_tie = (a2 > 0 && std::fabs(a1 - a2) <= 1e3 * 2.220446049250313e-16 * std::fabs(a1));
    for (int g = 0; g < ng; ++g) S[g].kept = kept[g];
    for (int g = 0; g < ng; ++g)
      for (int i = 0; i < S[g].kept; ++i) res.svals.push_back(hw[woff[g] + i]);
    std::sort(res.svals.begin(), res.svals.end(), std::greater<double>());
  }
  // projectors. With H = X^T X: V (rB x k) from H, U = X V S^-1.
  // With H = X X^T: U (rA x k) from H, V = X^T U S^-1.
  // P_A = R_B^T V S^-1/2 (d x k); P_B = S^-1/2 U^T R_A (k x d)
  std::vector<int64_t> pa_off(ng), pb_off(ng);
  int64_t pas = 0;
  for (int g = 0; g < ng; ++g) {
    pa_off[g] = pas;
    pas += S[g].d * S[g].kept;
    pb_off[g] = pas;
    pas += S[g].kept * S[g].d;
  }
  DBuf<double> PAB(std::max<int64_t>(pas, 1), s);
  {
    // the other singular vectors: O = X V or X^T U (then scaled by 1/s)
    std::vector<GemmGroup> go;
    for (int g = 0; g < ng; ++g) {
      const Sect& x = S[g];
      if (!x.kept) continue;
      if (x.rB <= x.rA)  // U = X V : (rA x rB)(rB x k)
        go.push_back(plain_group(x.rA, x.kept, x.rB, xoff[g], x.rB, 0, voff[g], x.p, 0, uoff[g], x.kept));
      else  // V = X^T U : (rB x rA)(rA x k)
        go.push_back(plain_group(x.rB, x.kept, x.rA, xoff[g], x.rB, 1, voff[g], x.p, 0, uoff[g], x.kept));
    }
    run_grouped_gemm(FTN_GEMM_F64, FTN_F64, go, Xm.p, Vm.p, Um.p, nullptr, s);
    for (int g = 0; g < ng; ++g) {
      const Sect& x = S[g];
      if (!x.kept) continue;
      // O = X V (rows rA) or X^T U (rows rB); O / s are the other singular
      // vectors, and both sides are then scaled by s^-1/2
      const int64_t rows = x.rB <= x.rA ? x.rA : x.rB;
      LAUNCH(k_scale_cols, dim3((unsigned)cdiv(rows * x.kept, 256)), dim3(256), 0, s, Um.p + uoff[g],
                         rows, (int64_t)x.kept, x.kept, Wm.p + woff[g], 2);
      LAUNCH(k_scale_cols, dim3((unsigned)cdiv((int64_t)x.ns * x.kept, 256)), dim3(256), 0, s,
                         Vm.p + voff[g], (int64_t)x.ns, (int64_t)x.p, x.kept, Wm.p + woff[g], 0);
      LAUNCH(k_scale_cols, dim3((unsigned)cdiv(rows * x.kept, 256)), dim3(256), 0, s, Um.p + uoff[g],
                         rows, (int64_t)x.kept, x.kept, Wm.p + woff[g], 0);
      HIPC(hipGetLastError());
    }
    // now: Vs = V S^-1/2 and Us = U S^-1/2 (for whichever side)
    std::vector<GemmGroup> gpa, gpb;
    for (int g = 0; g < ng; ++g) {
      const Sect& x = S[g];
      if (!x.kept) continue;
      if (x.rB <= x.rA) {
        // eigen side = V (rB x k, ld p) in Vm; other = U (rA x k, ld k) in Um
        // P_A = R_B^T V : (d x rB)(rB x k)
        gpa.push_back(plain_group(x.d, x.kept, x.rB, goffB[g], x.d, 1, voff[g], x.p, 0, pa_off[g], x.kept));
        // P_B = U^T R_A : (k x rA)(rA x d)
        gpb.push_back(plain_group(x.kept, x.d, x.rA, uoff[g], x.kept, 1, goffA[g], x.d, 0, pb_off[g], x.d));
      } else {
        // eigen side = U (rA x k, ld p) in Vm; other = V (rB x k, ld k) in Um
        gpa.push_back(plain_group(x.d, x.kept, x.rB, goffB[g], x.d, 1, uoff[g], x.kept, 0, pa_off[g], x.kept));
        gpb.push_back(plain_group(x.kept, x.d, x.rA, voff[g], x.p, 1, goffA[g], x.d, 0, pb_off[g], x.d));
      }
    }
    // operand buffers differ per case; run each case separately
    std::vector<GemmGroup> pa1, pa2, pb1, pb2;
    {
      int t = 0;
      for (int g = 0; g < ng; ++g) {
        const Sect& x = S[g];
        if (!x.kept) continue;
        if (x.rB <= x.rA) {
          pa1.push_back(gpa[t]);
          pb1.push_back(gpb[t]);
        } else {
          pa2.push_back(gpa[t]);
          pb2.push_back(gpb[t]);
        }
        ++t;
      }
    }
    if (!pa1.empty()) {
      run_grouped_gemm(FTN_GEMM_F64, FTN_F64, pa1, Rm.p, Vm.p, PAB.p, nullptr, s);
      run_grouped_gemm(FTN_GEMM_F64, FTN_F64, pb1, Um.p, Rm.p, PAB.p, nullptr, s);
    }
    if (!pa2.empty()) {
      run_grouped_gemm(FTN_GEMM_F64, FTN_F64, pa2, Rm.p, Um.p, PAB.p, nullptr, s);
      run_grouped_gemm(FTN_GEMM_F64, FTN_F64, pb2, Vm.p, Rm.p, PAB.p, nullptr, s);
    }
  }
  // projector tensors: P_A legs (conj of la, new) and P_B legs (new', conj of lb)
  std::vector<int> order(ng);
  for (int g = 0; g < ng; ++g) order[g] = g;
  std::sort(order.begin(), order.end(), [&](int x, int y) { return q_lt(S[x].charge, S[y].charge); });
  Leg nla, nlb;  // new bond legs
  nla.dual = LA.dual;
  nlb.dual = LB.dual;
  for (int g : order)
    if (S[g].kept) {
      nla.q.push_back(S[g].charge);
      nla.d.push_back(S[g].kept);
      nlb.q.push_back(S[g].charge);
      nlb.d.push_back(S[g].kept);
    }
  Leg cla = LA, clb = LB;  // partners of la / lb
  cla.dual = 1 - LA.dual;
  clb.dual = 1 - LB.dual;
  Q zero{0, 0};
  auto PA = make_tensor(sym, FTN_F64, {cla, nla}, zero, s, true);
  auto PB = make_tensor(sym, FTN_F64, {nlb, clb}, zero, s, true);
  {
    // block (q, q) of P_A has shape d_q x k_q; of P_B k_q x d_q
    for (int g = 0; g < ng; ++g) {
      const Sect& x = S[g];
      if (!x.kept) continue;
      int32_t ka[2] = {LA.find(x.charge), nla.find(x.charge)};
      int32_t kb[2] = {nlb.find(x.charge), LB.find(x.charge)};
      int64_t ba = block_index(PA->S(), ka), bb = block_index(PB->S(), kb);
      if (ba < 0 || bb < 0) fail(FTN_EINVAL, "internal: projector block missing");
      HIPC(hipMemcpyAsync((double*)PA->data + PA->S().offsets[ba], PAB.p + pa_off[g], x.d * x.kept * 8,
                          hipMemcpyDeviceToDevice, s));
      HIPC(hipMemcpyAsync((double*)PB->data + PB->S().offsets[bb], PAB.p + pb_off[g], x.kept * x.d * 8,
                          hipMemcpyDeviceToDevice, s));
    }
  }
  std::unique_ptr<Tensor> PAc, PBc;
  const Tensor* pa_t = PA.get();
  const Tensor* pb_t = PB.get();
  if (a.dtype != FTN_F64) {
    PAc = op_cast(*PA, a.dtype, s);
    PBc = op_cast(*PB, a.dtype, s);
    pa_t = PAc.get();
    pb_t = PBc.get();
  }
  // A' = F(A P_A) with the new leg moved back to la; B' = F(P_B B) likewise
  auto A1 = op_ftensordot(a, *pa_t, {la}, {0}, FTN_GLOBAL, gk, s);
  auto B1 = op_ftensordot(*pb_t, b, {1}, {lb}, FTN_GLOBAL, gk, s);
  const int na = a.ndim(), nb = b.ndim();
  std::vector<int> perm_a(na), perm_b(nb);
  {
    // A1 legs: rest(A) ++ [new]; want new at position la
    int t = 0;
    for (int i = 0; i < na; ++i) perm_a[i] = (i == la) ? (na - 1) : t++;
    // B1 legs: [new] ++ rest(B); want new at position lb
    t = 1;
    for (int i = 0; i < nb; ++i) perm_b[i] = (i == lb) ? 0 : t++;
  }
  res.a = op_ftranspose(*A1, perm_a, s);
  res.b = op_ftranspose(*B1, perm_b, s);
  (void)conv;
  return res;
}

}  // namespace ftn
