// Bond compression (Sec. II.A truncated SVD over all symmetry blocks; used
// by approximate contraction, Fig. 1b and Sec. III), FP64 throughout.
//
// For the bond between A (leg la) and B (leg lb), per bond charge q:
//   A~_q (M x d) and B~_q (d x N) are the fused matrices of the contraction
//   plan (signed permutes), and G_A = A~^T A~, G_B = B~ B~^T their Gram
//   matrices (split-K MFMA GEMMs). With A~ = Q_A R_A (G_A = R_A^T R_A) and
//   B~ = R_B^T Q_B, the best rank-chi approximation of A~ B~ comes from the
//   SVD X = R_A R_B^T = U S V^T, the chi largest values kept over all
//   charges, through the projectors P_A = R_B^T V S^-1/2 and
//   P_B = S^-1/2 U^T R_A. Only R_A is formed: the eigenvectors U of
//   T = X X^T = R_A G_B R_A^T (eigenvalues S^2) give V S = X^T U, hence
//   P_A = G_B R_A^T U S^-3/2 and P_B = S^-1/2 (R_A^T U)^T, with no inverse
//   of an ill-conditioned factor. A' = A~ P_A and B' = P_B B~ are ordinary
//   fermionic contractions of A and B with 2-leg block-diagonal tensors
//   followed by transpositions that put the new bond back in place. A
//   per-sector sign (the bond parity of the local convention) commutes with
//   the block-diagonal projectors, so the same A', B' serve both
//   conventions.
// R_A (and R_B for large sectors) come from a blocked right-looking Cholesky
// that drops dependent columns (pivot below 1e-13 of the largest diagonal).
// T is diagonalised by a cyclic Jacobi method in LDS when d <= 128; larger
// sectors find the leading left singular subspace of X = R_A R_B^T by block
// power iteration with X^T and X alternately on a 128-column basis.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>

#include "common.h"

namespace ftn {

constexpr int LT = 1024;     // threads of the factorisation kernels
constexpr int JMAX = 128;    // largest order diagonalised in LDS

typedef double d4 __attribute__((ext_vector_type(4)));
static_assert(LT == 1024 && JMAX == 128, "register staging assumes 1024 threads and order 128");

__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// ---------------------------------------------------------------------------
// Cyclic Jacobi eigensolver for a symmetric n x n matrix (n <= 128), in two
// kernels.
// k_jacobi_sweep (one workgroup per matrix) keeps the upper triangle in LDS
// and sweeps it in round-robin order. Per round, wave 0 computes the n/2
// disjoint rotations (lane k: pair k) and publishes them in LDS; after one
// barrier every thread updates its 2 x 2 blocks (pair k1, pair k2) as
// J_k1^T A J_k2 in place (a fixed list of at most three blocks per thread;
// every element belongs to exactly one block of a round, so reads and
// writes of a round need no barrier between them); a second barrier ends
// the round. The rotations are logged to global memory. Sweeps stop when the
// off-diagonal norm^2 is <= max(1e-30, (4 n u)^2) of the diagonal norm^2
// (jacobi_stop). The eigenvalues
// are written sorted, with the rank of each diagonal position.
// k_jacobi_vectors replays the log onto V = I: rows of V are independent, so
// each wave owns one row, the log is read ahead in blocks of rounds, and no
// barrier is needed; the columns are scattered to their eigenvalue ranks.
// Outputs: eigenvalues descending (ties: lower index first) and the matching
// eigenvector columns (row-major n x n).
constexpr int JAC_SWEEPS = 30;
constexpr int NPAIR = 3;  // block pairs per thread: 64 * 65 / 2 <= 3 * 1024
constexpr int JV_WAVES = 4;  // rows of V per workgroup of k_jacobi_vectors

struct EigJob {
  const double* H;  // n x n input
  double* V;        // n x n eigenvectors (columns), output
  double* W;        // n eigenvalues, output (descending)
  double2* rot;     // rotation log: (c, s) per rotation
  int* rpq;         // rotation log: p | q << 16
  int* rounds;      // number of rounds done (written by the sweeps)
  int* rk;          // n: rank of each diagonal position (written by the sweeps)
  int n;
  int pad;
};

__host__ __device__ inline int64_t jacobi_log_len(int n) {
  const int n2 = n + (n & 1);
  return (int64_t)JAC_SWEEPS * (n2 - 1) * (n2 / 2);
}

__device__ inline void rr_pair(int n2, int r, int i, int& p, int& q) {
  // round-robin tournament on n2 (even) players: fixed player n2-1
  const int m = n2 - 1;
  if (i == 0) {
    p = r;
    q = m;
  } else {
    p = r + i;
    if (p >= m) p -= m;
    q = r - i;
    if (q < 0) q += m;
  }
  if (p > q) {
    const int t = p;
    p = q;
    q = t;
  }
}

// workgroup barrier that orders LDS only (the rotation log stores to global
// memory stay in flight)
__device__ inline void sync_lds() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Rotation annihilating a_pq: t = tan(theta) = sign(tau) / (|tau| + sqrt(1 +
// tau^2)) with tau = (a_qq - a_pp) / (2 a_pq) (|t| <= 1; a huge tau gives
// t = 0), c = 1 / sqrt(1 + t^2) by the hardware reciprocal square root and
// two Newton steps, s = t c.
__device__ inline void jac_rotation(double app, double aqq, double apq, double& c, double& sn, double& t) {
  c = 1.0;
  sn = 0.0;
  t = 0.0;
  if (apq != 0.0) {
    const double tau = (aqq - app) / (2.0 * apq);
    t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
    const double q = 1.0 + t * t, h = 0.5 * q;
    double y = __builtin_amdgcn_rsq(q);
    y = y * (1.5 - h * y * y);
    y = y * (1.5 - h * y * y);
    c = y;
    sn = t * y;
  }
}

// Sweeps stop when the off-diagonal sum of squares is at most this fraction
// of the diagonal's: 1e-30, or (4 n u)^2 when that is larger, since every
// rotation rounds the entries it touches by about u times the largest ones
// and the off-diagonal part settles near (n u)^2 of the diagonal's.
__host__ __device__ inline double jacobi_stop(int n) {
  const double f = 4.0 * n * 0x1p-53;
  return fmax(1e-30, f * f);
}

__global__ void __launch_bounds__(LT) k_jacobi_sweep(const JobTable<EigJob> jobs) {
  const EigJob J = jobs[blockIdx.x];
  const int n = J.n;
  if (n <= 0) return;
  __shared__ double A[JMAX][JMAX + 1];
  __shared__ double ev[JMAX];
  __shared__ double red[2][LT / 64];
  __shared__ double2 rcs[JMAX / 2];  // the round's rotations (c, s)
  __shared__ double rt[JMAX / 2];    // and t = s / c
  __shared__ int rpq_s[JMAX / 2];    // and p | q << 16
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int n2 = n + (n & 1);  // an odd order gets a zero row / column
  const int np = n2 / 2;
  for (int e = tid; e < n2 * n2; e += LT) {
    const int i = e / n2, j = e % n2;
    if (i <= j) A[i][j] = (j < n) ? J.H[(int64_t)i * n + j] : 0.0;
  }
  __syncthreads();
  // the block pairs (k1 <= k2) this thread updates every round
  int pk1[NPAIR], pk2[NPAIR];
  bool pact[NPAIR];
  {
    const int npairs = np * (np + 1) / 2;
#pragma unroll
    for (int u = 0; u < NPAIR; ++u) {
      const int e = tid + u * LT;
      pact[u] = e < npairs;
      int k1 = 0, rem = pact[u] ? e : 0;
      while (rem >= np - k1) {
        rem -= np - k1;
        ++k1;
      }
      pk1[u] = k1;
      pk2[u] = k1 + rem;
    }
  }
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
    if (off == 0.0 || 2.0 * off <= jacobi_stop(n) * tot) break;
    for (int r = 0; r < n2 - 1; ++r, ++nr) {
      if (w == 0 && lane < np) {
        int p, q;
        rr_pair(n2, r, lane, p, q);
        double c, sn, t;
        jac_rotation(A[p][p], A[q][q], A[p][q], c, sn, t);
        rcs[lane] = make_double2(c, sn);
        rt[lane] = t;
        rpq_s[lane] = p | (q << 16);
        J.rot[(int64_t)nr * np + lane] = make_double2(c, sn);
        J.rpq[(int64_t)nr * np + lane] = p | (q << 16);
      }
      sync_lds();
      double* Af = &A[0][0];
#pragma unroll
      for (int u = 0; u < NPAIR; ++u) {
        if (!pact[u]) continue;
        const int v1 = rpq_s[pk1[u]], v2 = rpq_s[pk2[u]];
        const int p1 = v1 & 0xffff, q1 = v1 >> 16, p2 = v2 & 0xffff, q2 = v2 >> 16;
        if (pk1[u] == pk2[u]) {
          // diagonal block: a_pq is annihilated
          const int a0 = p1 * (JMAX + 1) + p1, a1 = p1 * (JMAX + 1) + q1, a2 = q1 * (JMAX + 1) + q1;
          const double b0 = Af[a0], b1 = Af[a1], b2 = Af[a2], t = rt[pk1[u]];
          Af[a0] = b0 - t * b1;
          Af[a2] = b2 + t * b1;
          Af[a1] = 0.0;
        } else {
          const double2 ra = rcs[pk1[u]], rb = rcs[pk2[u]];
          const int a0 = min(p1, p2) * (JMAX + 1) + max(p1, p2);
          const int a1 = min(p1, q2) * (JMAX + 1) + max(p1, q2);
          const int a2 = min(q1, p2) * (JMAX + 1) + max(q1, p2);
          const int a3 = min(q1, q2) * (JMAX + 1) + max(q1, q2);
          const double b0 = Af[a0], b1 = Af[a1], b2 = Af[a2], b3 = Af[a3];
          const double r00 = ra.x * b0 - ra.y * b2, r01 = ra.x * b1 - ra.y * b3;
          const double r10 = ra.y * b0 + ra.x * b2, r11 = ra.y * b1 + ra.x * b3;
          Af[a0] = rb.x * r00 - rb.y * r01;
          Af[a1] = rb.y * r00 + rb.x * r01;
          Af[a2] = rb.x * r10 - rb.y * r11;
          Af[a3] = rb.y * r10 + rb.x * r11;
        }
      }
      sync_lds();
    }
  }
  for (int i = tid; i < n; i += LT) ev[i] = A[i][i];
  if (tid == 0) J.rounds[0] = nr;
  __syncthreads();
  for (int i = tid; i < n; i += LT) {
    const double v = ev[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double u = ev[j];
      rank += (u > v) || (u == v && j < i);
    }
    J.rk[i] = rank;
    J.W[rank] = v;
  }
}

constexpr int NPAIR_LA = 3;  // off-diagonal blocks per thread of waves 1..15: 64 * 63 / 2 <= 3 * 960

// partner of index x in round r (round-robin on n2 players, fixed player n2-1)
__device__ inline int rr_partner(int n2, int r, int x) {
  const int m = n2 - 1;
  if (x == m) return r;
  int y = 2 * r - x;
  if (y < 0) y += m;
  if (y >= m) y -= m;
  return y == x ? m : y;
}
// index of the pair that holds x in round r
__device__ inline int rr_slot(int n2, int r, int x) {
  const int m = n2 - 1, np = n2 / 2;
  if (x == m || x == r) return 0;
  int d = x - r;
  if (d < 0) d += m;
  return d <= np - 1 ? d : m - d;
}


// The same sweeps with one barrier per round (for n2 >= 6, where no 2 x 2
// block of a round holds two pivots of the next round, and no pivot of the
// next round lies in a diagonal block of this one): wave 0 updates the
// diagonal blocks and, for every pair of the next round, the block that
// holds its pivot, and computes the next round's rotations from those fresh
// values (cross-lane reads for the new diagonal entries) into the other LDS
// buffer; waves 1..15 update the remaining blocks meanwhile. Every entry gets
// the same operations in the same order as in k_jacobi_sweep, so the results
// are bitwise the same.
__global__ void __launch_bounds__(LT) k_jacobi_sweep_la(const JobTable<EigJob> jobs) {
  const EigJob J = jobs[blockIdx.x];
  const int n = J.n;
  if (n <= 0) return;
  __shared__ double A[JMAX][JMAX + 1];
  __shared__ double ev[JMAX];
  __shared__ double red[2][LT / 64];
  __shared__ double2 rcs[2][JMAX / 2];
  __shared__ double rt[2][JMAX / 2];
  __shared__ int rpq_s[2][JMAX / 2];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int n2 = n + (n & 1), np = n2 / 2, m = n2 - 1;
  for (int e = tid; e < n2 * n2; e += LT) {
    const int i = e / n2, j = e % n2;
    if (i <= j) A[i][j] = (j < n) ? J.H[(int64_t)i * n + j] : 0.0;
  }
  __syncthreads();
  // the off-diagonal blocks (k1 < k2) of this thread; a block that holds a
  // pivot of the next round is wave 0's. Which blocks those are does not
  // depend on the round (partners in round r + 1 of the pair in slot k of
  // round r sit in fixed slots), so they are found once, from round 0.
  int pk1[NPAIR_LA], pk2[NPAIR_LA];
  bool pact[NPAIR_LA];
  {
    const int nb = np * (np - 1) / 2;
#pragma unroll
    for (int u = 0; u < NPAIR_LA; ++u) {
      const int e = (tid - 64) + u * (LT - 64);
      pact[u] = w > 0 && e < nb;
      int k1 = 0, rem = pact[u] ? e : 0;
      while (rem >= np - 1 - k1) {
        rem -= np - 1 - k1;
        ++k1;
      }
      pk1[u] = k1;
      pk2[u] = k1 + 1 + rem;
      if (pact[u]) {
        int p1, q1, p2, q2;
        rr_pair(n2, 0, pk1[u], p1, q1);
        rr_pair(n2, 0, pk2[u], p2, q2);
        const int r1 = m > 1 ? 1 : 0;
        const int x1 = rr_partner(n2, r1, p1), y1 = rr_partner(n2, r1, q1);
        if (x1 == p2 || x1 == q2 || y1 == p2 || y1 == q2) pact[u] = false;
      }
    }
  }
  int cur = 0;
  if (w == 0 && lane < np) {  // rotations of round 0
    int p, q;
    rr_pair(n2, 0, lane, p, q);
    double c, sn, t;
    jac_rotation(A[p][p], A[q][q], A[p][q], c, sn, t);
    rcs[0][lane] = make_double2(c, sn);
    rt[0][lane] = t;
    rpq_s[0][lane] = p | (q << 16);
  }
  __syncthreads();
  int nr = 0;
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
    if (off == 0.0 || 2.0 * off <= jacobi_stop(n) * tot) break;
    for (int r = 0; r < m; ++r, ++nr) {
      const int r2 = r + 1 == m ? 0 : r + 1;
      double* Af = &A[0][0];
      if (w > 0) {
#pragma unroll
        for (int u = 0; u < NPAIR_LA; ++u) {
          if (!pact[u]) continue;
          const int v1 = rpq_s[cur][pk1[u]], v2 = rpq_s[cur][pk2[u]];
          const int p1 = v1 & 0xffff, q1 = v1 >> 16, p2 = v2 & 0xffff, q2 = v2 >> 16;
          const double2 ra = rcs[cur][pk1[u]], rb = rcs[cur][pk2[u]];
          const int a0 = min(p1, p2) * (JMAX + 1) + max(p1, p2);
          const int a1 = min(p1, q2) * (JMAX + 1) + max(p1, q2);
          const int a2 = min(q1, p2) * (JMAX + 1) + max(q1, p2);
          const int a3 = min(q1, q2) * (JMAX + 1) + max(q1, q2);
          const double b0 = Af[a0], b1 = Af[a1], b2 = Af[a2], b3 = Af[a3];
          const double r00 = ra.x * b0 - ra.y * b2, r01 = ra.x * b1 - ra.y * b3;
          const double r10 = ra.y * b0 + ra.x * b2, r11 = ra.y * b1 + ra.x * b3;
          Af[a0] = rb.x * r00 - rb.y * r01;
          Af[a1] = rb.y * r00 + rb.x * r01;
          Af[a2] = rb.x * r10 - rb.y * r11;
          Af[a3] = rb.y * r10 + rb.x * r11;
        }
      } else {
        // the round being applied goes to the log
        int pl = 0, ql = 0;
        double dpp = 0.0, dqq = 0.0;
        if (lane < np) {
          const int v = rpq_s[cur][lane];
          pl = v & 0xffff;
          ql = v >> 16;
          J.rot[(int64_t)nr * np + lane] = rcs[cur][lane];
          J.rpq[(int64_t)nr * np + lane] = v;
          // diagonal block of pair lane: a_pq is annihilated
          const double b0 = A[pl][pl], b1 = A[pl][ql], b2 = A[ql][ql], t = rt[cur][lane];
          dpp = b0 - t * b1;
          dqq = b2 + t * b1;
          A[pl][pl] = dpp;
          A[ql][ql] = dqq;
          A[pl][ql] = 0.0;
        }
        // next round's pair `lane`: its pivot block in this round
        int pn = 0, qn = 0, ka = 0, kb = 0;
        double apq_n = 0.0;
        if (lane < np) {
          rr_pair(n2, r2, lane, pn, qn);
          const int sa = rr_slot(n2, r, pn), sb = rr_slot(n2, r, qn);
          ka = sa;
          kb = sb;
          const int k1 = min(sa, sb), k2 = max(sa, sb);
          const int v1 = rpq_s[cur][k1], v2 = rpq_s[cur][k2];
          const int p1 = v1 & 0xffff, q1 = v1 >> 16, p2 = v2 & 0xffff, q2 = v2 >> 16;
          const double2 ra = rcs[cur][k1], rb = rcs[cur][k2];
          const int a0 = min(p1, p2) * (JMAX + 1) + max(p1, p2);
          const int a1 = min(p1, q2) * (JMAX + 1) + max(p1, q2);
          const int a2 = min(q1, p2) * (JMAX + 1) + max(q1, p2);
          const int a3 = min(q1, q2) * (JMAX + 1) + max(q1, q2);
          const double b0 = Af[a0], b1 = Af[a1], b2 = Af[a2], b3 = Af[a3];
          const double r00 = ra.x * b0 - ra.y * b2, r01 = ra.x * b1 - ra.y * b3;
          const double r10 = ra.y * b0 + ra.x * b2, r11 = ra.y * b1 + ra.x * b3;
          const double n0 = rb.x * r00 - rb.y * r01, n1 = rb.y * r00 + rb.x * r01;
          const double n2v = rb.x * r10 - rb.y * r11, n3 = rb.y * r10 + rb.x * r11;
          Af[a0] = n0;
          Af[a1] = n1;
          Af[a2] = n2v;
          Af[a3] = n3;
          const int at = pn * (JMAX + 1) + qn;  // pn < qn
          apq_n = at == a0 ? n0 : at == a1 ? n1 : at == a2 ? n2v : n3;
        }
        // the new diagonal entries of pn and qn, from the lanes that own them
        const double dpa = __shfl(dpp, ka), dqa = __shfl(dqq, ka), dpb = __shfl(dpp, kb), dqb = __shfl(dqq, kb);
        const int pa = __shfl(pl, ka), pb = __shfl(pl, kb);
        if (lane < np) {
          const double app = pn == pa ? dpa : dqa;
          const double aqq = qn == pb ? dpb : dqb;
          double c, sn, t;
          jac_rotation(app, aqq, apq_n, c, sn, t);
          rcs[cur ^ 1][lane] = make_double2(c, sn);
          rt[cur ^ 1][lane] = t;
          rpq_s[cur ^ 1][lane] = pn | (qn << 16);
        }
      }
      sync_lds();
      cur ^= 1;
    }
  }
  for (int i = tid; i < n; i += LT) ev[i] = A[i][i];
  if (tid == 0) J.rounds[0] = nr;
  __syncthreads();
  for (int i = tid; i < n; i += LT) {
    const double v = ev[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double u = ev[j];
      rank += (u > v) || (u == v && j < i);
    }
    J.rk[i] = rank;
    J.W[rank] = v;
  }
}
// grid (jobs, ceil(n / JV_WAVES)), JV_WAVES waves: wave w owns row
// blockIdx.y * JV_WAVES + w of V and lane k applies rotation k of every
// round; the log is read PF rounds ahead, double-buffered in registers.
__global__ void __launch_bounds__(64 * JV_WAVES) k_jacobi_vectors(const JobTable<EigJob> jobs) {
  constexpr int PF = 8;
  const EigJob J = jobs[blockIdx.x];
  const int n = J.n;
  const int n2 = n + (n & 1), np = n2 / 2;
  __shared__ double Vs[JV_WAVES][JMAX + 2];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int row = blockIdx.y * JV_WAVES + w;
  if (row >= n) return;
  double* V = Vs[w];
  for (int j = lane; j < n2; j += 64) V[j] = (row == j) ? 1.0 : 0.0;
  const int nr = *J.rounds;
  if (lane < np && nr > 0) {
    auto load = [&](int t, double2& r, int& v) {
      const int tt = min(t, nr - 1);  // reads past the last round are clamped (and unused)
      r = J.rot[(int64_t)tt * np + lane];
      v = J.rpq[(int64_t)tt * np + lane];
    };
    auto apply = [&](const double2 r, const int v) {
      const int p = v & 0xffff, q = v >> 16;
      const double vp = V[p], vq = V[q];
      V[p] = r.x * vp - r.y * vq;
      V[q] = r.y * vp + r.x * vq;
    };
    double2 ra[PF], rb[PF];
    int va[PF], vb[PF];
#pragma unroll
    for (int k = 0; k < PF; ++k) load(k, ra[k], va[k]);
    const int nfull = nr / PF;
    int b = 0;
    for (; b + 2 <= nfull; b += 2) {
#pragma unroll
      for (int k = 0; k < PF; ++k) load((b + 1) * PF + k, rb[k], vb[k]);
#pragma unroll
      for (int k = 0; k < PF; ++k) apply(ra[k], va[k]);
#pragma unroll
      for (int k = 0; k < PF; ++k) load((b + 2) * PF + k, ra[k], va[k]);
#pragma unroll
      for (int k = 0; k < PF; ++k) apply(rb[k], vb[k]);
    }
    for (int t = b * PF; t < nr; ++t) {
      double2 r;
      int v;
      load(t, r, v);
      apply(r, v);
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  for (int c = lane; c < n; c += 64) J.V[(int64_t)row * n + J.rk[c]] = V[c];
}

// value of v in lane l (l the same for the whole wavefront), read through
// the scalar unit rather than a cross-lane permute
__device__ __forceinline__ double readlane_d(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// ---------------------------------------------------------------------------
// Rank-revealing orthonormalisation factor (one workgroup per matrix): for
// the Gram matrix G = Y^T Y (p x p, p <= 128), Cholesky G = R^T R in which a
// column whose pivot (its squared distance from the span of the previous
// columns) is not above tol * (largest diagonal of G) is dropped: its row of
// R is zero and its column of the output is zero. The output M (p x p) is
// R^-1 with the dropped columns cleared, so Y M has orthonormal columns (up
// to the conditioning of the kept ones) and zero columns: dependent
// directions are dropped instead of amplified. R itself (rows of dropped
// columns zero) can be written as well or instead.
// Blocked in LDS, upper triangle only, panels of 16: one wave factors the
// 16 x 16 diagonal block in registers (four entries per lane, rows
// broadcast by cross-lane reads; pivots by a reciprocal square root with
// two Newton steps), the panel row R12 = R11^-T A12 is solved one column per
// thread with the stored reciprocals of the pivots, and the trailing update
// A22 -= R12^T R12 runs on FP64 MFMA tiles. The work is done at the order
// p padded with the identity to the next power of two (16 .. 128). R is
// inverted in place: 16 x 16 diagonal blocks by back substitution, then up
// to three doubling levels
// [U11 U12; 0 U22]^-1 = [U11^-1, -U11^-1 U12 U22^-1; 0, U22^-1] on MFMA
// tiles (U11^-1 U12 is staged in the free lower triangle).
struct OrthJob {
  const double* G;    // p x p input, leading dimension ldg
  double* R;          // optional: R (upper, dropped rows and lower part zero), ld ldr
  double* M;          // optional: R^-1 with dropped columns zero, ld ldm
  const double* thr;  // optional absolute pivot threshold (else tol * max diag)
  int p, ldg, ldr, ldm;
};

__global__ void __launch_bounds__(LT) k_orth_factor(const JobTable<OrthJob> jobs, double tol) {
  const OrthJob J = jobs[blockIdx.x];
  const int p = J.p;
  __shared__ double A[JMAX][JMAX + 1];
  __shared__ int dr[JMAX];
  __shared__ double rinv[JMAX];  // 1 / R_jj, 0 for a dropped column
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  // working order: p padded with the identity to a power of two >= 16
  int pn = 16;
  while (pn < p) pn *= 2;
  const int lpn = __ffs(pn) - 1;
  for (int e = tid; e < pn * pn; e += LT) {
    const int i = e >> lpn, c = e & (pn - 1);
    A[i][c] = (i < p && c < p) ? J.G[(int64_t)i * J.ldg + c] : (i == c ? 1.0 : 0.0);
  }
  __syncthreads();
  double mx = 0.0;
  for (int i = lane; i < p; i += 64) mx = fmax(mx, A[i][i]);
  mx = wave_max(mx);
  const double thr = J.thr ? *J.thr : tol * mx;
  for (int j0 = 0; j0 < pn; j0 += 16) {
    if (w == 0) {  // 16 x 16 diagonal block in registers of wave 0
      // lane: column b = lane & 15, rows a0 + t (t < 4), a0 = 4 (lane >> 4)
      const int b = lane & 15, a0 = 4 * (lane >> 4);
      double x[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) x[t] = A[j0 + a0 + t][j0 + b];
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        const int j = j0 + jj, tj = jj & 3, lb = 16 * (jj >> 2);
        const double d = readlane_d(x[tj], lb + jj);  // the pivot: one lane, known at compile time
        const bool drop = (j < p) && !(d > thr);
        // 1 / sqrt(d): hardware estimate and two Newton steps
        double y = __builtin_amdgcn_rsq(d);
        const double h = 0.5 * d;
        y = y * (1.5 - h * y * y);
        y = y * (1.5 - h * y * y);
        const double r = drop ? 1.0 : d * y, inv = drop ? 1.0 : y;
        if (lane >= lb && lane < lb + 16) {  // these lanes hold row jj in x[tj]
          if (b > jj) x[tj] = drop ? 0.0 : x[tj] * inv;
          else if (b == jj) x[tj] = r;
        }
        const double rbv = __shfl(x[tj], lb + b);
        double ra[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) ra[t] = __shfl(x[tj], lb + a0 + t);
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (a0 + t > jj && b >= a0 + t) x[t] -= ra[t] * rbv;
        if (lane == 0) {
          dr[j] = drop ? 1 : 0;
          rinv[j] = drop ? 0.0 : inv;
        }
      }
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (a0 + t <= b) A[j0 + a0 + t][j0 + b] = x[t];
    }
    __syncthreads();
    const int rest = pn - j0 - 16;
    if (tid < rest) {  // R12 = R11^-T A12, column c (right-looking: independent updates per step)
      const int c = j0 + 16 + tid;
      double x[16];
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) x[jj] = A[j0 + jj][c];
#pragma unroll
      for (int l = 0; l < 16; ++l) {
        x[l] *= rinv[j0 + l];
#pragma unroll
        for (int jj = l + 1; jj < 16; ++jj) x[jj] -= A[j0 + l][j0 + jj] * x[l];
      }
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) A[j0 + jj][c] = x[jj];
    }
    __syncthreads();
    if (rest > 0) {  // A22 -= R12^T R12 on the upper-triangle tiles
      const int nt = rest / 16, ntile = nt * (nt + 1) / 2, base = j0 + 16;
      for (int t = w; t < ntile; t += LT / 64) {
        int ti = 0, u = t;
        while (u >= nt - ti) {
          u -= nt - ti;
          ++ti;
        }
        const int tj = ti + u;
        d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k0 = 0; k0 < 16; k0 += 4) {
          const double a = A[j0 + k0 + lk][base + 16 * ti + li];
          const double bb = A[j0 + k0 + lk][base + 16 * tj + li];
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc, 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) A[base + 16 * ti + lk + 4 * q][base + 16 * tj + li] -= acc[q];
      }
    }
    __syncthreads();
  }
  if (J.R) {
    for (int e = tid; e < p * p; e += LT) {
      const int i = e / p, c = e % p;
      J.R[(int64_t)i * J.ldr + c] = (i <= c && !dr[i]) ? A[i][c] : 0.0;
    }
  }
  if (!J.M) return;
  // every wave has read R before the inversion below overwrites it in place
  __syncthreads();
  // 16 x 16 diagonal blocks: lane c of wave w solves column c of block w
  if (w < pn / 16 && lane < 16) {
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
  for (int h = 16; h < pn; h *= 2) {
    const int m = 2 * h, nt = h / 16, tiles = (pn / m) * nt * nt;
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
    const int i = e / p, c = e % p;
    J.M[(int64_t)i * J.ldm + c] = (i <= c && !dr[c]) ? A[i][c] : 0.0;
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

// projector blocks from F, GF (d x k) and the singular values:
//   side A: Pa = GF S^-3/2, Pb = S^-1/2 F^T;  side B: Pa = F S^-1/2, Pb = S^-3/2 GF^T
__global__ void k_proj_out(const double* F, const double* GF, int64_t d, int k, const double* sv, int sideA,
                           double* Pa, double* Pb) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= d * k) return;
  const int64_t r = e / k;
  const int c = (int)(e % k);
  const double h = 1.0 / sqrt(sv[c]), h3 = h * h * h;
  Pa[e] = sideA ? GF[e] * h3 : F[e] * h;
  Pb[(int64_t)c * d + r] = sideA ? F[e] * h : GF[e] * h3;
}

// W[i, j] = V[i, j] * sv[j] for j < cols (V row-major with ld ldv, W ld cols)
struct ScaleColsJob {
  const double* V;
  const double* sv;
  double* W;
  int64_t rows, cols, ldv;
};
__global__ void k_scale_cols(const JobTable<ScaleColsJob> jobs) {
  const ScaleColsJob J = jobs[blockIdx.y];
  const int64_t n = J.rows * J.cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / J.cols, j = e % J.cols;
    J.W[e] = J.V[i * J.ldv + j] * J.sv[j];
  }
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

// a product known to be symmetric (op(B) = op(A)^T): only its upper tiles
// are multiplied, the output is still written in full
static GemmGroup sym_group(GemmGroup g) {
  g.sym = 1;
  return g;
}

// launches timed under the factorisation class of the opt-in profiler; the
// work figure is the textbook flop count of what the launch computes:
// Cholesky of a p x p matrix p^3/3, a triangular inverse p^3/3, and a
// symmetric eigendecomposition with eigenvectors 9 n^3 (tridiagonal
// reduction plus implicit QR), whatever the algorithm actually runs
#define FACTOR_LAUNCH(cls, work, kern, grid, block, shm, stream, ...)                          \
  do {                                                                                       \
    void* tok_ = prof_begin(s);                                                              \
    ELAUNCH(kern, grid, block, shm, stream, prof_ev(tok_, 0), prof_ev(tok_, 1), __VA_ARGS__); \
    prof_end(tok_, s, (cls), (work));                                                        \
  } while (0)

static double orth_flops(const std::vector<OrthJob>& oj) {
  double f = 0;
  for (const OrthJob& o : oj) {
    const double p3 = (double)o.p * o.p * o.p;
    f += p3 / 3.0 + (o.M ? p3 / 3.0 : 0.0);
  }
  return f;
}

static double eig_flops(const std::vector<EigJob>& ej) {
  double f = 0;
  for (const EigJob& e : ej) f += 9.0 * (double)e.n * e.n * e.n;
  return f;
}

// Eigendecompositions of the jobs' matrices (H, V, W and n set by the
// caller): the sweeps, then the replay of their rotation logs onto V, timed
// as one factorisation launch. The logs and per-job counters are allocated
// here. With `rounds`, the rounds each job took are copied back (the stream
// is synchronised).
static void jacobi_eig(std::vector<EigJob>& ej, hipStream_t s, std::vector<int>* rounds = nullptr) {
  const int nj = (int)ej.size();
  if (nj == 0) return;
  int64_t log_n = 0;
  int nmax = 0;
  for (const EigJob& e : ej) {
    log_n += jacobi_log_len(e.n);
    nmax = std::max(nmax, e.n);
  }
  DBuf<double2> lrot(std::max<int64_t>(log_n, 1), s);
  DBuf<int> lpq(std::max<int64_t>(log_n, 1), s), aux((int64_t)nj * (JMAX + 1), s);
  int64_t o = 0;
  for (int t = 0; t < nj; ++t) {
    EigJob& e = ej[t];
    if (e.n > JMAX) fail(FTN_ENOTSUP, "eigensolver order above 128");
    e.rot = lrot.p + o;
    e.rpq = lpq.p + o;
    o += jacobi_log_len(e.n);
    e.rounds = aux.p + (int64_t)t * (JMAX + 1);
    e.rk = e.rounds + 1;
    e.pad = 0;
  }
  // orders of 63 and up take the sweep with one barrier per round (faster
  // there); the jobs are ordered so that each kernel gets a contiguous range
  std::vector<EigJob> ord(ej);
  std::stable_partition(ord.begin(), ord.end(), [](const EigJob& e) { return e.n < 63; });
  int nsmall = 0;
  while (nsmall < nj && ord[nsmall].n < 63) ++nsmall;
  const Jobs<EigJob> dj(ord, s);
  if (nsmall > 0) {
    const std::vector<EigJob> part(ord.begin(), ord.begin() + nsmall);
    const Jobs<EigJob> dp(part, s);
    FACTOR_LAUNCH(FTN_PROF_K_JACOBI, eig_flops(part), k_jacobi_sweep, dim3((unsigned)nsmall), dim3(LT), 0, s, dp.t);
  }
  if (nsmall < nj) {
    const std::vector<EigJob> part(ord.begin() + nsmall, ord.end());
    const Jobs<EigJob> dp(part, s);
    FACTOR_LAUNCH(FTN_PROF_K_JACOBI_LA, eig_flops(part), k_jacobi_sweep_la, dim3((unsigned)(nj - nsmall)), dim3(LT), 0,
                  s, dp.t);
  }
  if (nmax > 0)
    FACTOR_LAUNCH(FTN_PROF_K_JACOBI_VEC, 0.0, k_jacobi_vectors, dim3((unsigned)nj, (unsigned)cdiv(nmax, JV_WAVES)),
                  dim3(64 * JV_WAVES), 0, s, dj.t);
  if (rounds) {
    rounds->assign(nj, 0);
    for (int t = 0; t < nj; ++t)
      HIPC(hipMemcpyAsync(rounds->data() + t, aux.p + (int64_t)t * (JMAX + 1), sizeof(int), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
  }
}

// ---------------------------------------------------------------------------
// Symmetric eigendecomposition of orders 129 to 1024 by block Jacobi. The
// indices are cut into nb = 2 ceil(n / 128) contiguous blocks of near-equal
// size (at most 64 each), and a sweep meets every two blocks once (a
// round-robin tournament over the blocks: nb / 2 disjoint pairs per round).
// In a round the principal submatrix of every pair (order at most 128) is
// diagonalised completely by the LDS eigensolver above; the pairs'
// eigenvector matrices, embedded in one orthogonal Q, then rotate the whole
// matrix, H <- Q^T H Q, and the accumulated vectors, V <- V Q (dense FP64
// GEMMs). Sweeps repeat until the off-diagonal Frobenius norm is at most
// 8 n u of the matrix's (each rotation of the whole matrix rounds every entry
// by about u |H|, so smaller targets are out of reach), at most 40 sweeps.
// Outputs as jacobi_eig's: values descending (ties: lower index first) and
// the matching eigenvectors as columns.
constexpr int EIG_BIG_MAX = 1024;
constexpr int BLK_SWEEPS = 40;

struct BlkPair {
  const double* H;  // n x n matrix being diagonalised
  double* sub;      // ns x ns principal submatrix of the pair (rows of block i, then block j)
  const double* vs; // ns x ns eigenvectors of sub (columns)
  double* Q;        // n x n rotation of this round
  int n, i0, i1, j0, j1;
};

__device__ inline int blk_index(const BlkPair& P, int a) {
  const int ni = P.i1 - P.i0;
  return a < ni ? P.i0 + a : P.j0 + a - ni;
}

// grid (chunks, pairs)
__global__ void k_blk_gather(const BlkPair* pairs) {
  const BlkPair P = pairs[blockIdx.y];
  const int ns = (P.i1 - P.i0) + (P.j1 - P.j0);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ns * ns; e += gridDim.x * blockDim.x) {
    const int a = e / ns, b = e % ns;
    P.sub[e] = P.H[(int64_t)blk_index(P, a) * P.n + blk_index(P, b)];
  }
}

// rows of Q that belong to the pair, written in full (zero outside the
// pair's columns), so that the pairs of a round cover all of Q
__global__ void k_blk_scatter(const BlkPair* pairs) {
  const BlkPair P = pairs[blockIdx.y];
  const int ni = P.i1 - P.i0, ns = ni + (P.j1 - P.j0), n = P.n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)ns * n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(e / n), c = (int)(e % n);
    int b = -1;
    if (c >= P.i0 && c < P.i1) b = c - P.i0;
    else if (c >= P.j0 && c < P.j1) b = ni + c - P.j0;
    P.Q[(int64_t)blk_index(P, a) * n + c] = b >= 0 ? P.vs[(int64_t)a * ns + b] : 0.0;
  }
}

struct BlkMat {
  const double* H;  // n x n
  const double* V;  // n x n accumulated vectors
  double* Vout;     // n x n eigenvectors by rank (EigJob.V)
  double* W;        // n values by rank (EigJob.W)
  double* norms;    // 2: off-diagonal and total sums of squares
  int n;
};

// one workgroup per matrix: sums of squares off the diagonal and in total
__global__ void __launch_bounds__(1024) k_blk_offnorm(const BlkMat* mats) {
  const BlkMat M = mats[blockIdx.x];
  __shared__ double red[2][16];
  double off = 0.0, tot = 0.0;
  const int64_t nn = (int64_t)M.n * M.n;
  for (int64_t e = threadIdx.x; e < nn; e += blockDim.x) {
    const double v = M.H[e];
    tot += v * v;
    if (e / M.n != e % M.n) off += v * v;
  }
  for (int o = 32; o > 0; o >>= 1) {
    off += __shfl_xor(off, o);
    tot += __shfl_xor(tot, o);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = off;
    red[1][w] = tot;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int i = 0; i < 16; ++i) {
      a += red[0][i];
      b += red[1][i];
    }
    M.norms[0] = a;
    M.norms[1] = b;
  }
}

// one workgroup per matrix: values by rank and the vectors' columns moved to
// their ranks
__global__ void __launch_bounds__(1024) k_blk_finish(const BlkMat* mats) {
  const BlkMat M = mats[blockIdx.x];
  const int n = M.n;
  __shared__ double dg[EIG_BIG_MAX];
  __shared__ int rk[EIG_BIG_MAX];
  for (int i = threadIdx.x; i < n; i += blockDim.x) dg[i] = M.H[(int64_t)i * n + i];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double v = dg[i];
    int r = 0;
    for (int j = 0; j < n; ++j) r += (dg[j] > v) || (dg[j] == v && j < i);
    rk[i] = r;
    M.W[r] = v;
  }
  __syncthreads();
  for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += blockDim.x) {
    const int64_t row = e / n;
    const int c = (int)(e % n);
    M.Vout[row * n + rk[c]] = M.V[e];
  }
}

__global__ void k_set_identity(double* X, const int64_t* off, const int* dim) {
  const int m = blockIdx.y, n = dim[m];
  double* Y = X + off[m];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)n * n;
       e += (int64_t)gridDim.x * blockDim.x)
    Y[e] = (e / n == e % n) ? 1.0 : 0.0;
}

// round-robin tournament on nb (even) players: pair i of round r
static void rr_pair_host(int nb, int r, int i, int& p, int& q) {
  const int m = nb - 1;
  if (i == 0) {
    p = r;
    q = m;
  } else {
    p = (r + i) % m;
    q = ((r - i) % m + m) % m;
  }
  if (p > q) std::swap(p, q);
}

static void block_jacobi_eig(std::vector<EigJob>& ej, hipStream_t s) {
  const int nj = (int)ej.size();
  if (!nj) return;
  std::vector<int64_t> off(nj);
  std::vector<int> dim(nj), nb(nj);
  int64_t tot = 0;
  int nbmax = 0;
  for (int j = 0; j < nj; ++j) {
    const int n = ej[j].n;
    if (n <= JMAX || n > EIG_BIG_MAX) fail(FTN_EINVAL, "internal: block Jacobi order out of range");
    off[j] = tot;
    tot += (int64_t)n * n;
    dim[j] = n;
    nb[j] = 2 * (int)cdiv(n, JMAX);
    nbmax = std::max(nbmax, nb[j]);
  }
  // H (working copy) | V0 | V1 | Q | T, each `tot`
  DBuf<double> Wk(5 * tot, s), nrm(2 * nj, s), sub((int64_t)nbmax / 2 * nj * JMAX * JMAX, s),
      vs((int64_t)nbmax / 2 * nj * JMAX * JMAX, s), wv((int64_t)nbmax / 2 * nj * JMAX, s);
  double *Hw = Wk.p, *Qw = Wk.p + 3 * tot;
  for (int j = 0; j < nj; ++j)
    HIPC(hipMemcpyAsync(Hw + off[j], ej[j].H, (size_t)dim[j] * dim[j] * 8, hipMemcpyDeviceToDevice, s));
  DBuf<int64_t> doff = to_device(std::vector<int64_t>(off), s);
  DBuf<int> ddim = to_device(dim, s);
  LAUNCH(k_set_identity, dim3(64, (unsigned)nj), dim3(256), 0, s, Wk.p + tot, doff.p, ddim.p);
  std::vector<int> vcur(nj, 1);  // which V slot (1 or 2) holds the accumulated vectors
  std::vector<char> done(nj, 0);
  std::vector<double> hn(2 * nj);
  for (int sweep = 0; sweep < BLK_SWEEPS; ++sweep) {
    for (int r = 0; r < nbmax - 1; ++r) {
      std::vector<BlkPair> pr;
      std::vector<EigJob> inner;
      std::vector<int> owner;
      for (int j = 0; j < nj; ++j) {
        if (done[j] || r >= nb[j] - 1) continue;
        const int n = dim[j];
        for (int i = 0; i < nb[j] / 2; ++i) {
          int p, q;
          rr_pair_host(nb[j], r, i, p, q);
          BlkPair P;
          P.H = Hw + off[j];
          P.n = n;
          P.i0 = (int)((int64_t)p * n / nb[j]);
          P.i1 = (int)((int64_t)(p + 1) * n / nb[j]);
          P.j0 = (int)((int64_t)q * n / nb[j]);
          P.j1 = (int)((int64_t)(q + 1) * n / nb[j]);
          const int64_t slot = (int64_t)pr.size();
          P.sub = sub.p + slot * JMAX * JMAX;
          P.vs = vs.p + slot * JMAX * JMAX;
          P.Q = Qw + off[j];
          EigJob e{};
          e.H = P.sub;
          e.V = vs.p + slot * JMAX * JMAX;
          e.W = wv.p + slot * JMAX;
          e.n = (P.i1 - P.i0) + (P.j1 - P.j0);
          pr.push_back(P);
          inner.push_back(e);
        }
        owner.push_back(j);
      }
      if (owner.empty()) continue;
      DBuf<BlkPair> dp = to_device(pr, s);
      LAUNCH(k_blk_gather, dim3(16, (unsigned)pr.size()), dim3(256), 0, s, dp.p);
      jacobi_eig(inner, s);
      LAUNCH(k_blk_scatter, dim3(32, (unsigned)pr.size()), dim3(256), 0, s, dp.p);
      // T = H Q, H = Q^T T, V' = V Q
      std::vector<GemmGroup> g1, g2, g3;
      for (int j : owner) {
        const int64_t n = dim[j];
        g1.push_back(plain_group(n, n, n, off[j], n, 0, 3 * tot + off[j], n, 0, 4 * tot + off[j], n));
        g2.push_back(plain_group(n, n, n, 3 * tot + off[j], n, 1, 4 * tot + off[j], n, 0, off[j], n));
        g3.push_back(plain_group(n, n, n, vcur[j] * tot + off[j], n, 0, 3 * tot + off[j], n, 0,
                                 (3 - vcur[j]) * tot + off[j], n));
      }
      run_grouped_gemm(FTN_GEMM_F64, FTN_F64, g1, Wk.p, Wk.p, Wk.p, nullptr, s);
      run_grouped_gemm(FTN_GEMM_F64, FTN_F64, g2, Wk.p, Wk.p, Wk.p, nullptr, s);
      run_grouped_gemm(FTN_GEMM_F64, FTN_F64, g3, Wk.p, Wk.p, Wk.p, nullptr, s);
      for (int j : owner) vcur[j] = 3 - vcur[j];
    }
    // convergence of every matrix still running
    std::vector<BlkMat> bm;
    std::vector<int> idx;
    for (int j = 0; j < nj; ++j) {
      if (done[j]) continue;
      BlkMat b{};
      b.H = Hw + off[j];
      b.norms = nrm.p + 2 * j;
      b.n = dim[j];
      bm.push_back(b);
      idx.push_back(j);
    }
    if (bm.empty()) break;
    DBuf<BlkMat> db = to_device(bm, s);
    LAUNCH(k_blk_offnorm, dim3((unsigned)bm.size()), dim3(1024), 0, s, db.p);
    HIPC(hipMemcpyAsync(hn.data(), nrm.p, 2 * nj * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    bool all = true;
    for (int j : idx) {
      const double lim = 8.0 * dim[j] * 0x1p-53;
      if (hn[2 * j] <= lim * lim * hn[2 * j + 1]) done[j] = 1;
      all = all && done[j];
    }
    if (all) break;
  }
  std::vector<BlkMat> fin(nj);
  for (int j = 0; j < nj; ++j) {
    fin[j] = BlkMat{};
    fin[j].H = Hw + off[j];
    fin[j].V = Wk.p + vcur[j] * tot + off[j];
    fin[j].Vout = ej[j].V;
    fin[j].W = ej[j].W;
    fin[j].n = dim[j];
  }
  DBuf<BlkMat> df = to_device(fin, s);
  LAUNCH(k_blk_finish, dim3((unsigned)nj), dim3(1024), 0, s, df.p);
}

// eigendecompositions of any order up to 1024: LDS sweeps up to 128, block
// Jacobi above
static void sym_eig(const std::vector<EigJob>& ej, hipStream_t s) {
  std::vector<EigJob> small, big;
  for (const EigJob& e : ej) (e.n <= JMAX ? small : big).push_back(e);
  if (!small.empty()) jacobi_eig(small, s);
  if (!big.empty()) block_jacobi_eig(big, s);
}

// ---------------------------------------------------------------------------
// One-sided (Hestenes) Jacobi SVD of a small matrix X (r x c, r, c <= 128),
// one workgroup per matrix. The columns of X are rotated in pairs until they
// are mutually orthogonal: X V = W, W = U S with S the column norms. The
// singular values come from the columns themselves, not from a Gram matrix,
// so they are accurate to about eps * |X| (a Gram matrix X X^T holds s^2
// only to eps * |X|^2, which loses every s below ~1e-8 |X|).
// The c columns live in LDS (column-major, padded); a round applies the c/2
// disjoint rotations of a round-robin tournament, one column pair per wave
// at a time (the three inner products are wave reductions); a pair is
// rotated when |x_p . x_q| > tol sqrt(|x_p|^2 |x_q|^2). Sweeps stop after one
// without rotation (at most JAC_SWEEPS). Outputs: the m = min(r, c) largest
// s^2 in descending order (ties: lower column first) and U (r x m, ld ldu),
// column k = the k-th column of W divided by its norm (zero if the norm is);
// every rotation (c, s) with its column pair is logged per round in the
// format of the two-sided sweeps, with the rank of every column, so that
// k_jacobi_vectors replays them onto the identity and returns V (c x c,
// columns in rank order) as the product of the rotations: V is orthogonal
// to working precision however small a singular value is, which X^T U / s
// is not (its error grows like eps |X| / s).
struct SvdJob {
  const double* X;  // r x c row-major, leading dimension ldx
  double* U;        // r x m, leading dimension ldu
  double* W;        // m values s^2, descending
  double2* rot;     // rotation log (c, s), np per round
  int* rpq;         // rotation log: p | q << 16
  int* rounds;      // rounds done
  int* rk;          // c: rank of every column by its final norm
  int r, c, ldx, ldu;
};

__global__ void __launch_bounds__(LT) k_svd_cols(const JobTable<SvdJob> jobs, double tol) {
  const SvdJob J = jobs[blockIdx.x];
  const int r = J.r, c = J.c;
  if (r <= 0 || c <= 0) return;
  __shared__ double Xc[JMAX][JMAX + 1];
  __shared__ double nrm[JMAX + 1];
  __shared__ int rot_any;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nw = LT / 64;
  for (int e = tid; e < r * c; e += LT) {
    const int i = e / c, j = e % c;
    Xc[j][i] = J.X[(int64_t)i * J.ldx + j];
  }
  const int n2 = c + (c & 1);  // an odd count gets a zero column
  if (c & 1)
    for (int i = tid; i < r; i += LT) Xc[c][i] = 0.0;
  const int np = n2 / 2;
  const bool l0 = lane < r, l1 = lane + 64 < r;
  // |X|_F^2 for the absolute noise floor of a pair's inner product
  __shared__ double fro_part[LT / 64];
  __syncthreads();
  {
    double t = 0.0;
    for (int e = tid; e < r * c; e += LT) {
      const double x = Xc[e % c][e / c];
      t += x * x;
    }
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
    if (lane == 0) fro_part[w] = t;
  }
  __syncthreads();
  double fro2 = 0.0;
  for (int k = 0; k < nw; ++k) fro2 += fro_part[k];
  // a pair is rotated when its inner product is above tol * sqrt(a b) (tol =
  // rows * eps, the rounding level of a length-r inner product) and above the
  // rounding level of the whole matrix, 4 r eps^2 |X|_F^2: below it the two
  // columns are round-off of zero directions and rotating them changes
  // nothing but would keep the sweeps from ending
  const double rtol = fmax(tol, (double)r * 2.220446049250313e-16);
  const double floor_g = 4.0 * (double)r * 4.930380657631324e-32 * fro2;
  // Each half-wave (32 lanes, four entries of a column each) takes one
  // pair at a time, so a wave rotates two pairs at once. Only the cross
  // product x_p . x_q needs a reduction: the squared column norms are exact
  // at the start of a sweep and carried through its rotations by
  // |x_p'|^2 = |x_p|^2 - t g, |x_q'|^2 = |x_q|^2 + t g.
  const int hl = lane & 31, hw = lane >> 5;
  const int nh = 2 * nw;  // half-waves
  int nr = 0;
  for (int sweep = 0; sweep < JAC_SWEEPS; ++sweep) {
    if (tid == 0) rot_any = 0;
    __syncthreads();
    for (int j = w; j < n2; j += nw) {
      double t = 0.0;
      if (j < c) {
        const double v0 = l0 ? Xc[j][lane] : 0.0, v1 = l1 ? Xc[j][lane + 64] : 0.0;
        t = v0 * v0 + v1 * v1;
      }
      for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
      if (lane == 0) nrm[j] = t;
    }
    __syncthreads();
    for (int rd = 0; rd < n2 - 1; ++rd, ++nr) {
      for (int k = 2 * w + hw; k < np; k += nh) {
        int p, q;
        rr_pair(n2, rd, k, p, q);
        double lc = 1.0, ls = 0.0;
        double xp[4], xq[4];
        double g = 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = hl + 32 * u;
          xp[u] = i < r ? Xc[p][i] : 0.0;
          xq[u] = i < r ? Xc[q][i] : 0.0;
          g += xp[u] * xq[u];
        }
        for (int o = 16; o > 0; o >>= 1) g += __shfl_xor(g, o);
        const double a = fmax(nrm[p], 0.0), b = fmax(nrm[q], 0.0);
        if (fabs(g) > floor_g && fabs(g) > rtol * sqrt(a * b)) {
          const double zeta = (b - a) / (2.0 * g);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int i = hl + 32 * u;
            if (i < r) {
              Xc[p][i] = cs * xp[u] - sn * xq[u];
              Xc[q][i] = sn * xp[u] + cs * xq[u];
            }
          }
          if (hl == 0) {
            nrm[p] = a - t * g;
            nrm[q] = b + t * g;
            rot_any = 1;
          }
          lc = cs;
          ls = sn;
        }
        if (hl == 0) {
          J.rot[(int64_t)nr * np + k] = make_double2(lc, ls);
          J.rpq[(int64_t)nr * np + k] = p | (q << 16);
        }
      }
      __syncthreads();
    }
    if (!rot_any) break;
    __syncthreads();
  }
  if (tid == 0) J.rounds[0] = nr;
  // column norms, ranks by (larger norm, lower index), sorted outputs
  for (int j = w; j < c; j += nw) {
    const double v0 = l0 ? Xc[j][lane] : 0.0, v1 = l1 ? Xc[j][lane + 64] : 0.0;
    double t = v0 * v0 + v1 * v1;
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
    if (lane == 0) nrm[j] = t;
  }
  __syncthreads();
  const int m = r < c ? r : c;
  for (int j = w; j < c; j += nw) {
    const double sj = nrm[j];
    int rank = 0;
    for (int k = 0; k < c; ++k) rank += (nrm[k] > sj || (nrm[k] == sj && k < j)) ? 1 : 0;
    if (lane == 0) J.rk[j] = rank;
    if (rank >= m) continue;
    const double inv = sj > 0.0 ? 1.0 / sqrt(sj) : 0.0;
    if (l0) J.U[(int64_t)lane * J.ldu + rank] = Xc[j][lane] * inv;
    if (l1) J.U[(int64_t)(lane + 64) * J.ldu + rank] = Xc[j][lane + 64] * inv;
    if (lane == 0) J.W[rank] = sj;
  }
}

// thin SVD of every listed X (textbook thin-SVD flops 14 m n^2 + 8 n^3, m >= n):
// U, s^2 and V[t] (c x c, columns in rank order, ld c) of job t
static void svd_cols(std::vector<SvdJob>& sj, const std::vector<double*>& V, hipStream_t s) {
  if (sj.empty()) return;
  const int nj = (int)sj.size();
  double f = 0;
  int64_t log_n = 0;
  int cmax = 0;
  for (const SvdJob& j : sj) {
    if (j.r > JMAX || j.c > JMAX) fail(FTN_ENOTSUP, "one-sided Jacobi order above 128");
    const double m = std::max(j.r, j.c), n = std::min(j.r, j.c);
    f += 14.0 * m * n * n + 8.0 * n * n * n;
    log_n += jacobi_log_len(j.c);
    cmax = std::max(cmax, j.c);
  }
  DBuf<double2> lrot(std::max<int64_t>(log_n, 1), s);
  DBuf<int> lpq(std::max<int64_t>(log_n, 1), s), aux((int64_t)nj * (JMAX + 1), s);
  std::vector<EigJob> ej(nj);
  int64_t o = 0;
  for (int t = 0; t < nj; ++t) {
    SvdJob& j = sj[t];
    j.rot = lrot.p + o;
    j.rpq = lpq.p + o;
    o += jacobi_log_len(j.c);
    j.rounds = aux.p + (int64_t)t * (JMAX + 1);
    j.rk = j.rounds + 1;
    EigJob& e = ej[t];
    e = EigJob{};
    e.V = V[t];
    e.rot = j.rot;
    e.rpq = j.rpq;
    e.rounds = j.rounds;
    e.rk = j.rk;
    e.n = j.c;
  }
  const Jobs<SvdJob> d(sj, s);
  const Jobs<EigJob> de(ej, s);
  FACTOR_LAUNCH(FTN_PROF_K_SVD_COLS, f, k_svd_cols, dim3((unsigned)nj), dim3(LT), 0, s, d.t, 1e-15);
  FACTOR_LAUNCH(FTN_PROF_K_JACOBI_VEC, 0.0, k_jacobi_vectors, dim3((unsigned)nj, (unsigned)cdiv(cmax, JV_WAVES)),
                dim3(64 * JV_WAVES), 0, s, de.t);
}

// per bond sector q
struct Sect {
  int64_t M, N, d;       // rows of A~, cols of B~, bond dim
  int64_t a_off, b_off;  // into A~ / B~
  int rA = 0, rB = 0;    // ranks of the dropping Cholesky factors
  int ns = 0;            // min(rA, rB)
  int p = 0;             // number of singular values computed: ns or JMAX
  bool iterate = false;
  bool sideA = true;     // eigenvectors live on the A side (U) or the B side (V)
  bool acc = false;      // d <= 128: accurate factors, X formed explicitly
  bool svd = false;      // spectrum redone by the one-sided Jacobi SVD of X (V available)
  bool thin = false;     // N <= d < M: spectrum from Y = A~ B~ (M x N), no factor of A~
  int kept = 0;
  Q charge;
  int crank = 0;
};

// tol * (largest diagonal) per matrix
struct DiagJob {
  const double* G;
  double* thr;
  int d;
  int pad;
};
__global__ void __launch_bounds__(256) k_diag_thr(const JobTable<DiagJob> jobs, double tol) {
  const DiagJob J = jobs[blockIdx.x];
  __shared__ double red[4];
  double m = 0.0;
  for (int i = threadIdx.x; i < J.d; i += 256) m = fmax(m, J.G[(int64_t)i * J.d + i]);
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) J.thr[0] = tol * fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// strict lower triangle of each d x d matrix <- 0
__global__ void k_zero_lower(double* G, const int64_t* off, const int64_t* dim, int nm) {
  const int m = blockIdx.y;
  if (m >= nm) return;
  const int64_t d = dim[m];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < d * d; e += (int64_t)gridDim.x * blockDim.x)
    if (e / d > e % d) G[off[m] + e] = 0.0;
}

// Rows of R with a non-zero diagonal (the kept columns) packed to the top of
// the matrix at the same offset of Rc; rank[m] = their number. One
// workgroup per matrix.
__global__ void __launch_bounds__(1024) k_pack_rows(const double* G, const int64_t* off, const int64_t* dim,
                                                    double* Rc, int* rank) {
  const int m = blockIdx.x;
  const int64_t d = dim[m];
  const double* R = G + off[m];
  double* O = Rc + off[m];
  __shared__ int cnt[1024];
  __shared__ int base;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (int64_t j0 = 0; j0 < d; j0 += 1024) {
    const int64_t j = j0 + threadIdx.x;
    const int kept = (j < d && R[j * d + j] != 0.0) ? 1 : 0;
    cnt[threadIdx.x] = kept;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {  // inclusive scan
      const int v = threadIdx.x >= o ? cnt[threadIdx.x - o] : 0;
      __syncthreads();
      cnt[threadIdx.x] += v;
      __syncthreads();
    }
    const int pos = base + cnt[threadIdx.x] - kept;
    const int tot = cnt[1023];
    __syncthreads();
    cnt[threadIdx.x] = kept ? -1 - pos : 0;  // destination row of each kept row
    __syncthreads();
    // copy this chunk's kept rows (one wave per row, round robin)
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int r = w; r < 1024 && j0 + r < d; r += 16) {
      const int c = cnt[r];
      if (c >= 0) continue;
      const int64_t dst = -1 - c, src = j0 + r;
      for (int64_t col = lane; col < d; col += 64) O[dst * d + col] = R[src * d + col];
    }
    __syncthreads();
    if (threadIdx.x == 0) base += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) rank[m] = base;
}

// In-place dropping Cholesky of the Gram matrices at offsets off[m] (d_m x
// d_m) of Gm: on return each holds R (upper triangular, rows of dropped
// columns zero, strict lower triangle zero) with R^T R = G on the kept
// columns. Right-looking in panels of 128: the diagonal block is factored in
// LDS (k_orth_factor, which also returns its inverse), the panel row is
// R12 = R11^-T A12 (a GEMM with the inverse), and the trailing matrix is
// updated by G22 -= R12^T R12 (GEMM). A column is dropped when its pivot is
// not above tol * (largest diagonal of G). With Mout, also the inverse in the
// convention of k_orth_factor (R with ones on the dropped diagonal, inverted,
// dropped columns cleared) at the same offsets of Mout: the diagonal blocks
// come from the LDS factorisations and block column j above them is
// -M[0:j, 0:j] R[0:j, j] M_jj (two GEMMs per panel, left to right).
static void chol_drop(double* Gm, const std::vector<int64_t>& off, const std::vector<int64_t>& dim, double tol,
                      hipStream_t s, double* Mout = nullptr) {
  const int nm = (int)off.size();
  if (!nm) return;
  const int64_t NB = JMAX;
  DBuf<double> thr(nm, s);
  {
    std::vector<DiagJob> dj(nm);
    for (int m = 0; m < nm; ++m) dj[m] = DiagJob{Gm + off[m], thr.p + m, (int)dim[m], 0};
    const Jobs<DiagJob> d(dj, s);
    LAUNCH(k_diag_thr, dim3(nm), dim3(256), 0, s, d.t, tol);
  }
  int64_t dmax = 0, r12n = 0;
  std::vector<int64_t> r12off(nm);
  for (int m = 0; m < nm; ++m) {
    dmax = std::max(dmax, dim[m]);
    r12off[m] = r12n;
    r12n += NB * std::max<int64_t>(dim[m] - NB, 0);
  }
  DBuf<double> Minv(Mout ? 1 : nm * NB * NB, s), R12(std::max<int64_t>(r12n, 1), s);
  if (Mout)
    for (int m = 0; m < nm; ++m) HIPC(hipMemsetAsync(Mout + off[m], 0, (size_t)dim[m] * dim[m] * 8, s));
  for (int64_t j0 = 0; j0 < dmax; j0 += NB) {
    std::vector<OrthJob> oj;
    std::vector<GemmGroup> gt, gs;
    for (int m = 0; m < nm; ++m) {
      const int64_t d = dim[m];
      if (d <= j0) continue;
      const int64_t nb = std::min(NB, d - j0), rest = d - j0 - nb;
      double* blk = Gm + off[m] + j0 * d + j0;
      OrthJob o;
      o.G = blk;
      o.R = blk;
      o.M = Mout ? Mout + off[m] + j0 * d + j0 : rest > 0 ? Minv.p + m * NB * NB : nullptr;
      o.thr = thr.p + m;
      o.p = (int)nb;
      o.ldg = o.ldr = (int)d;
      o.ldm = Mout ? (int)d : (int)NB;
      oj.push_back(o);
      if (rest > 0) {
        if (Mout)
          gt.push_back(plain_group(nb, rest, nb, off[m] + j0 * d + j0, d, 1, off[m] + j0 * d + j0 + nb, d, 0,
                                   r12off[m], rest));
        else
          gt.push_back(
              plain_group(nb, rest, nb, m * NB * NB, NB, 1, off[m] + j0 * d + j0 + nb, d, 0, r12off[m], rest));
        gs.push_back(sym_group(plain_group(rest, rest, nb, r12off[m], rest, 1, r12off[m], rest, 0,
                                           off[m] + (j0 + nb) * d + j0 + nb, d)));
      }
    }
    const Jobs<OrthJob> doj(oj, s);
    FACTOR_LAUNCH(FTN_PROF_K_ORTH, orth_flops(oj), k_orth_factor, dim3((unsigned)oj.size()), dim3(LT), 0, s, doj.t, tol);
    if (!gt.empty()) {
      run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gt, Mout ? Mout : Minv.p, Gm, R12.p, nullptr, s);
      run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gs, R12.p, R12.p, Gm, nullptr, s, -1.0, 1.0);
      for (int m = 0; m < nm; ++m) {
        const int64_t d = dim[m];
        if (d <= j0 + NB) continue;
        const int64_t rest = d - j0 - NB;
        HIPC(hipMemcpy2DAsync(Gm + off[m] + j0 * d + j0 + NB, d * 8, R12.p + r12off[m], rest * 8, rest * 8, NB,
                              hipMemcpyDeviceToDevice, s));
      }
    }
  }
  DBuf<int64_t> doff = to_device(off, s), ddim = to_device(dim, s);
  LAUNCH(k_zero_lower, dim3((unsigned)std::min<int64_t>(cdiv(dmax * dmax, 256), 4096), nm), dim3(256), 0, s, Gm,
         doff.p, ddim.p, nm);
  if (!Mout || dmax <= NB) return;
  DBuf<double> T((int64_t)nm * dmax * NB, s);
  for (int64_t j0 = NB; j0 < dmax; j0 += NB) {
    std::vector<GemmGroup> g1, g2;
    for (int m = 0; m < nm; ++m) {
      const int64_t d = dim[m];
      if (d <= j0) continue;
      const int64_t nb = std::min(NB, d - j0), to = (int64_t)m * dmax * NB;
      g1.push_back(plain_group(j0, nb, j0, off[m], d, 0, off[m] + j0, d, 0, to, nb));  // M[0:j,0:j] R[0:j,j]
      g2.push_back(plain_group(j0, nb, nb, to, nb, 0, off[m] + j0 * d + j0, d, 0, off[m] + j0, d));  // (..) M_jj
    }
    run_grouped_gemm(FTN_GEMM_F64, FTN_F64, g1, Mout, Gm, T.p, nullptr, s);
    run_grouped_gemm(FTN_GEMM_F64, FTN_F64, g2, T.p, Mout, Mout, nullptr, s, -1.0, 0.0);
  }
}

// ---------------------------------------------------------------------------
// Accurate triangular factors of sectors up to order 1024. The Gram matrix
// G = A^T A of a factor A (m x d) holds a direction of A with singular value
// s only to about eps * |A|^2 / s^2, so directions below ~1e-8 of |A| are
// lost, although the product X = R_A R_B^T can need them when the leading
// directions of the two sides are nearly orthogonal. The factor is therefore
// taken as A itself when m <= d (R = A, rank m), and otherwise
// by shifted Cholesky QR applied three times: R1 = chol(G + sigma I) with
// sigma = 11 (m d + d (d + 1)) u |A|_F^2 (u = 2^-53), Q1 = A R1^-1, then two
// dropping Cholesky QR passes on Q1, R = R3 R2 R1. The shift keeps the
// first factorisation defined for any conditioning and the later passes
// recover the small directions from A itself; rows whose pivot is not above
// 1e-13 of the largest in a later pass (exact dependencies) are dropped.
// Each Cholesky factorisation runs in LDS (k_orth_factor) for d <= 128 and
// as the blocked chol_drop with its inverse above.

struct ShiftJob {
  const double* G;  // d x d Gram matrix (ld d)
  double* W;        // output G + sigma I (ld d)
  int d;
  int pad;
  int64_t m;        // rows of the factor
};

__global__ void __launch_bounds__(256) k_shift_diag(const JobTable<ShiftJob> jobs) {
  const ShiftJob J = jobs[blockIdx.x];
  const int d = J.d;
  __shared__ double red[4];
  double t = 0;
  for (int i = threadIdx.x; i < d; i += 256) t += J.G[(int64_t)i * d + i];
  for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  const double tr = red[0] + red[1] + red[2] + red[3];
  const double sigma = 11.0 * ((double)J.m * d + (double)d * (d + 1)) * 0x1p-53 * tr;
  for (int64_t e = threadIdx.x; e < (int64_t)d * d; e += 256) {
    const int64_t i = e / d, c = e % d;
    J.W[e] = J.G[e] + (i == c ? sigma : 0.0);
  }
}

struct RowsJob {
  const double* src;  // A (m x d, ld) or, transposed, B (d x m, ld)
  double* dst;        // m x d (ld d)
  int64_t ld, m;
  int d, trans;
};

__global__ void k_copy_rows(const JobTable<RowsJob> jobs) {
  const RowsJob J = jobs[blockIdx.y];
  const int64_t n = J.m * J.d;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / J.d, c = e % J.d;
    J.dst[e] = J.trans ? J.src[c * J.ld + i] : J.src[i * J.ld + c];
  }
}

// one factor to refine: the source matrix is A (rows x d, ld) or B^T
// (B is d x rows with ld, trans = 1), side 0 = A~ buffer, 1 = B~ buffer
struct AccSrc {
  int side;
  int trans;
  int64_t off, ld, m;
  int64_t goff;  // Gram matrix and output R (d x d) offset
  int d;
  int64_t qoff = 0;  // optional output Q (m x d) offset
  int64_t moff = 0;  // optional output R^-1 (d x d, dropped columns zero) offset
};

// R (d x d, zero rows for dropped directions) of every listed factor into
// Rout at goff, from the Gram matrices Gm at goff and the sources; with Qout,
// also Q (m x d, orthonormal kept columns, zero dropped ones) at qoff, so
// that the source equals Q R; with Minv as well, the inverse used for Q
// (source x Minv = Q, the product of the three passes' inverses with
// dropped columns zero) at moff
static void acc_factor(const std::vector<AccSrc>& J, const double* At, const double* Bt, const double* Gm,
                       double* Rout, hipStream_t s, double* Qout = nullptr, double* Minv = nullptr) {
  const int nj = (int)J.size();
  if (!nj) return;
  std::vector<int64_t> wo(nj), qo(nj);
  int64_t ws = 0, qs = 0;
  for (int j = 0; j < nj; ++j) {
    wo[j] = ws;
    ws += (int64_t)J[j].d * J[j].d;
    qo[j] = qs;
    qs += J[j].m * J[j].d;
  }
  // W: R1 | R2 | R3 | M1 | M2 | T | M3 (each ws); Q: Q1 | Q2 (each qs)
  DBuf<double> W(7 * ws, s), Q(2 * qs, s);
  double *R1 = W.p, *R2 = W.p + ws, *R3 = W.p + 2 * ws, *M1 = W.p + 3 * ws, *M2 = W.p + 4 * ws,
         *M3 = W.p + 6 * ws;
  {
    std::vector<ShiftJob> sj(nj);
    for (int j = 0; j < nj; ++j) sj[j] = ShiftJob{Gm + J[j].goff, R1 + wo[j], J[j].d, 0, J[j].m};
    const Jobs<ShiftJob> d(sj, s);
    LAUNCH(k_shift_diag, dim3(nj), dim3(256), 0, s, d.t);
  }
  auto factor = [&](double* R, double* M, double tol) {
    std::vector<OrthJob> oj;
    std::vector<int64_t> boff, bdim;
    for (int j = 0; j < nj; ++j) {
      if (J[j].d > JMAX) {
        boff.push_back(wo[j]);
        bdim.push_back(J[j].d);
        continue;
      }
      OrthJob o;
      o.G = R + wo[j];
      o.R = R + wo[j];
      o.M = M ? M + wo[j] : nullptr;
      o.thr = nullptr;
      o.p = o.ldg = o.ldr = o.ldm = J[j].d;
      oj.push_back(o);
    }
    if (!oj.empty()) {
      const Jobs<OrthJob> d(oj, s);
      FACTOR_LAUNCH(FTN_PROF_K_ORTH, orth_flops(oj), k_orth_factor, dim3((unsigned)oj.size()), dim3(LT), 0, s, d.t, tol);
    }
    if (!boff.empty()) chol_drop(R, boff, bdim, tol, s, M);
  };
  // pass 1: no column is dropped (G + sigma I is positive definite)
  factor(R1, M1, 0.0);
  {
    // Q1 = source * R1^-1, per side (the sources live in two buffers)
    for (int side = 0; side < 2; ++side) {
      std::vector<GemmGroup> g;
      for (int j = 0; j < nj; ++j)
        if (J[j].side == side)
          g.push_back(plain_group(J[j].m, J[j].d, J[j].d, J[j].off, J[j].ld, J[j].trans, 3 * ws + wo[j], J[j].d, 0,
                                  qo[j], J[j].d));
      if (!g.empty()) run_grouped_gemm(FTN_GEMM_F64, FTN_F64, g, side ? Bt : At, W.p, Q.p, nullptr, s);
    }
  }
  std::vector<GemmGroup> gg2, gq2, gg3, gt, gr;
  for (int j = 0; j < nj; ++j) {
    const int64_t d = J[j].d, m = J[j].m;
    gg2.push_back(sym_group(plain_group(d, d, m, qo[j], d, 1, qo[j], d, 0, ws + wo[j], d)));    // G2 = Q1^T Q1
    gq2.push_back(plain_group(m, d, d, qo[j], d, 0, 4 * ws + wo[j], d, 0, qs + qo[j], d));      // Q2 = Q1 M2
    gg3.push_back(sym_group(plain_group(d, d, m, qs + qo[j], d, 1, qs + qo[j], d, 0, 2 * ws + wo[j], d)));  // G3
    gt.push_back(plain_group(d, d, d, 2 * ws + wo[j], d, 0, ws + wo[j], d, 0, 5 * ws + wo[j], d));  // T = R3 R2
    gr.push_back(plain_group(d, d, d, 5 * ws + wo[j], d, 0, wo[j], d, 0, J[j].goff, d));         // R = T R1
  }
  run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gg2, Q.p, Q.p, W.p, nullptr, s);
  factor(R2, M2, 1e-13);
  run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gq2, Q.p, W.p, Q.p, nullptr, s);
  run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gg3, Q.p, Q.p, W.p, nullptr, s);
  factor(R3, Qout ? M3 : nullptr, 1e-13);
  run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gt, W.p, W.p, W.p, nullptr, s);
  run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gr, W.p, W.p, Rout, nullptr, s);
  if (Qout) {
    std::vector<GemmGroup> gq3;  // Q = Q2 M3
    for (int j = 0; j < nj; ++j)
      gq3.push_back(plain_group(J[j].m, J[j].d, J[j].d, qs + qo[j], J[j].d, 0, 6 * ws + wo[j], J[j].d, 0, J[j].qoff,
                                J[j].d));
    run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gq3, Q.p, W.p, Qout, nullptr, s);
    if (Minv) {
      // M1 M2 into the free T slot, then (M1 M2) M3
      std::vector<GemmGroup> g12, g123;
      for (int j = 0; j < nj; ++j) {
        const int64_t d = J[j].d;
        g12.push_back(plain_group(d, d, d, 3 * ws + wo[j], d, 0, 4 * ws + wo[j], d, 0, 5 * ws + wo[j], d));
        g123.push_back(plain_group(d, d, d, 5 * ws + wo[j], d, 0, 6 * ws + wo[j], d, 0, J[j].moff, d));
      }
      run_grouped_gemm(FTN_GEMM_F64, FTN_F64, g12, W.p, W.p, W.p, nullptr, s);
      run_grouped_gemm(FTN_GEMM_F64, FTN_F64, g123, W.p, W.p, Minv, nullptr, s);
    }
  }
}

// Leading singular triplets of X = R_A R_B^T (rA x rB) per sector.
// Outputs: lam (p) = s^2 descending, and in E:
//   ns = min(rA, rB) <= JMAX: the eigenvectors (ns x ns) of H (given in
//   Hm: X X^T when rA <= rB, else X^T X), by cyclic Jacobi;
//   larger: the left singular vectors U (rA x JMAX) from block power
//   iteration applying X^T and X alternately to a JMAX-column basis (each
//   product scales the columns by s, not s^2), with one dropping
//   Cholesky-QR after each product (two before each Rayleigh-Ritz step,
//   every 4 iterations) until the Ritz values that can be kept (those among
//   the chi + 8 largest over all sectors) are stable (change
//   <= 1e-14 of the largest) or 96 iterations.
static void x_spectrum(std::vector<Sect>& S, int64_t chi, const double* Hm, const std::vector<int64_t>& hoff,
                       const double* Xm, const std::vector<int64_t>& xoff, double* Em, const std::vector<int64_t>& eoff,
                       double* Lm, const std::vector<int64_t>& loff, hipStream_t s) {
  const int ng = (int)S.size();
  const double tol = 1e-13;
  std::vector<int> dir, it;
  for (int g = 0; g < ng; ++g)
    if (S[g].ns > 0) (S[g].iterate ? it : dir).push_back(g);
  static const bool trace = std::getenv("FTN_TRACE") != nullptr;
  if (!dir.empty()) {
    const int nd = (int)dir.size();
    std::vector<EigJob> ej;
    for (int t = 0; t < nd; ++t) {
      const int g = dir[t];
      EigJob j{};
      j.H = Hm + hoff[g];
      j.V = Em + eoff[g];
      j.W = Lm + loff[g];
      j.n = S[g].ns;
      ej.push_back(j);
    }
    std::vector<int> r;
    jacobi_eig(ej, s, trace ? &r : nullptr);
    if (trace) {
      std::string t;
      for (int i = 0; i < nd; ++i) t += std::to_string(S[dir[i]].ns) + ":" + std::to_string(r[i]) + " ";
      std::fprintf(stderr, "[ftn] jacobi order:rounds %s\n", t.c_str());
    }
  }
  if (it.empty()) return;
  const int ni = (int)it.size();
  const int64_t p = JMAX;
  std::vector<int64_t> qo(ni), zo(ni);
  int64_t qn = 0, zn = 0;
  for (int t = 0; t < ni; ++t) {
    qo[t] = qn;
    qn += (int64_t)S[it[t]].rA * p;
    zo[t] = zn;
    zn += (int64_t)S[it[t]].rB * p;
  }
  DBuf<double> Q0(qn, s), Q1(qn, s), Z0(zn, s), Z1(zn, s), Z2(zn, s), Gy(ni * p * p, s), Mm(ni * p * p, s),
      Tr(ni * p * p, s), Zs(ni * p * p, s);
  std::string rr_trace;
  std::vector<GemmGroup> gxt, gx, ggq, ggz, gaq, gaz, ge;
  for (int t = 0; t < ni; ++t) {
    const int g = it[t];
    const int64_t rA = S[g].rA, rB = S[g].rB, go = (int64_t)t * p * p;
    gxt.push_back(plain_group(rB, p, rA, xoff[g], rB, 1, qo[t], p, 0, zo[t], p));  // Z = X^T Q
    gx.push_back(plain_group(rA, p, rB, xoff[g], rB, 0, zo[t], p, 0, qo[t], p));   // Q = X Z
    ggq.push_back(sym_group(plain_group(p, p, rA, qo[t], p, 1, qo[t], p, 0, go, p)));  // Q^T Q
    ggz.push_back(sym_group(plain_group(p, p, rB, zo[t], p, 1, zo[t], p, 0, go, p)));  // Z^T Z
    gaq.push_back(plain_group(rA, p, p, qo[t], p, 0, go, p, 0, qo[t], p));         // Q M
    gaz.push_back(plain_group(rB, p, p, zo[t], p, 0, go, p, 0, zo[t], p));         // Z M
    ge.push_back(plain_group(rA, p, p, qo[t], p, 0, go, p, 0, eoff[g], p));        // E = Q Zs
  }
  const auto cpx = gemm_plan_cached(gxt, FTN_GEMM_F64, s), cx = gemm_plan_cached(gx, FTN_GEMM_F64, s),
             cgq = gemm_plan_cached(ggq, FTN_GEMM_F64, s), cgz = gemm_plan_cached(ggz, FTN_GEMM_F64, s),
             caq = gemm_plan_cached(gaq, FTN_GEMM_F64, s), caz = gemm_plan_cached(gaz, FTN_GEMM_F64, s),
             ce = gemm_plan_cached(ge, FTN_GEMM_F64, s);
  const GemmPlan &Pxt = *cpx, &Px = *cx, &Pgq = *cgq, &Pgz = *cgz, &Paq = *caq, &Paz = *caz, &Pe = *ce;
  std::vector<OrthJob> oj;
  std::vector<EigJob> ej;
  for (int t = 0; t < ni; ++t) {
    const int g = it[t];
    const int64_t go = (int64_t)t * p * p;
    OrthJob o;
    o.G = Gy.p + go;
    o.R = nullptr;
    o.M = Mm.p + go;
    o.thr = nullptr;
    o.p = o.ldg = o.ldr = o.ldm = (int)p;
    oj.push_back(o);
    EigJob e{};
    e.H = Tr.p + go;
    e.V = Zs.p + go;
    e.W = Lm + loff[g];
    e.n = (int)p;
    ej.push_back(e);
  }
  const Jobs<OrthJob> doj(oj, s);
  const double of_it = orth_flops(oj);
  double *q = Q0.p, *qt = Q1.p, *z = Z0.p, *zt = Z1.p, *zu = Z2.p;
  // y <- orthonormal basis of span(y), dependent columns zeroed
  auto orth = [&](const GemmPlan& gram, const GemmPlan& app, double*& y, double*& yt) {
    run_gemm(gram, FTN_F64, y, y, Gy.p, nullptr, s);
    FACTOR_LAUNCH(FTN_PROF_K_ORTH, of_it, k_orth_factor, dim3((unsigned)ni), dim3(LT), 0, s, doj.t, tol);
    run_gemm(app, FTN_F64, y, Mm.p, yt, nullptr, s);
    std::swap(y, yt);
  };
  LAUNCH(k_fill_random, dim3((unsigned)cdiv(qn, 256)), dim3(256), 0, s, q, qn, (uint64_t)0x5eedf00dull);
  orth(Pgq, Paq, q, qt);
  orth(Pgq, Paq, q, qt);
  std::vector<double> prev, cur(ni * p);
  // values of the directly solved sectors (final): with the current Ritz
  // values they decide which values can be kept, and only those (plus a
  // margin of 8) have to converge
  std::vector<double> dvals;
  {
    std::vector<double> hw;
    for (int g : dir) {
      hw.resize(S[g].p);
      HIPC(hipMemcpyAsync(hw.data(), Lm + loff[g], S[g].p * 8, hipMemcpyDeviceToHost, s));
      HIPC(hipStreamSynchronize(s));
      dvals.insert(dvals.end(), hw.begin(), hw.end());
    }
  }
  auto needed = [&](const std::vector<double>& rv) {
    // rv: Ritz values of the iterated sectors (p each, descending); returns
    // per iterated sector how many of its leading values are within the
    // chi + 8 largest of all sectors
    std::vector<std::pair<double, int>> all;
    for (double v : dvals) all.push_back({v, -1});
    for (int t = 0; t < ni; ++t)
      for (int j = 0; j < p; ++j) all.push_back({rv[t * p + j], t});
    const size_t top = std::min<size_t>(all.size(), (size_t)std::max<int64_t>(chi, 0) + 8);
    std::partial_sort(all.begin(), all.begin() + top, all.end(),
                      [](const std::pair<double, int>& a, const std::pair<double, int>& b) { return a.first > b.first; });
    std::vector<int> kk(ni, 0);
    for (size_t i = 0; i < top; ++i)
      if (all[i].second >= 0) ++kk[all[i].second];
    return kk;
  };
  const int max_iter = 96, check = 4;
  int iters = 0;
  bool have_next = false;  // z already holds X^T q (computed for the last check)
  for (int k = 1; k <= max_iter; ++k) {
    iters = k;
    if (!have_next) run_gemm(Pxt, FTN_F64, Xm, q, z, nullptr, s);
    have_next = false;
    orth(Pgz, Paz, z, zt);
    run_gemm(Px, FTN_F64, Xm, z, q, nullptr, s);
    orth(Pgq, Paq, q, qt);
    if (k % check == 0 || k == max_iter) {
      orth(Pgq, Paq, q, qt);
      // Rayleigh-Ritz: W = X^T Q, Tr = W^T W = Q^T X X^T Q
      run_gemm(Pxt, FTN_F64, Xm, q, zu, nullptr, s);
      run_gemm(Pgz, FTN_F64, zu, zu, Tr.p, nullptr, s);
      std::vector<int> rr;
      jacobi_eig(ej, s, trace ? &rr : nullptr);
      for (int t = 0; t < ni; ++t)
        HIPC(hipMemcpyAsync(cur.data() + t * p, Lm + loff[it[t]], p * 8, hipMemcpyDeviceToHost, s));
      HIPC(hipStreamSynchronize(s));
      if (trace) rr_trace += " " + std::to_string(rr[0]);
      bool done = !prev.empty();
      const std::vector<int> kks = needed(cur);
      for (int t = 0; t < ni && done; ++t) {
        const int kk = std::min(kks[t], (int)p);
        const double top = std::max(cur[t * p], 1e-300);
        for (int j = 0; j < kk; ++j)
          if (std::fabs(cur[t * p + j] - prev[t * p + j]) > 1e-14 * top) done = false;
      }
      prev = cur;
      if (done) break;
      // continue from the Ritz vectors: the next T is then nearly diagonal
      // and its Jacobi solve converges in a few sweeps
      run_gemm(Paq, FTN_F64, q, Zs.p, qt, nullptr, s);
      std::swap(q, qt);
      run_gemm(Paz, FTN_F64, zu, Zs.p, zt, nullptr, s);
      std::swap(zu, zt);
      std::swap(z, zu);  // the next half step X^T q is ready
      have_next = true;
    }
  }
  if (trace) {
    std::string dd;
    for (int t = 0; t < ni; ++t) dd += std::to_string(S[it[t]].rA) + "x" + std::to_string(S[it[t]].rB) + " ";
    std::fprintf(stderr, "[ftn] subspace iteration: %d iterations, sectors %s, Rayleigh-Ritz rounds%s\n", iters,
                 dd.c_str(), rr_trace.c_str());
  }
  run_gemm(Pe, FTN_F64, q, Zs.p, Em, nullptr, s);
}

// number of K slices of the Gram products G_A = A~^T A~ (one launch over
// all sectors and slices; G_B likewise): each slice multiplies the upper
// triangle of tiles (128 x 128 when every sector has d >= 128, else 64 x 64)
// over K / slices, so the launch takes ceil(slices * tiles / CUs) waves of
// tiles of duration ~ 1 / slices. The count with the fewest waves per slice
// is taken (the smallest one within 3% of the best, since every slice adds
// a partial matrix to sum).
static int gram_split(const std::vector<Sect>& S, int64_t maxk) {
  int64_t dmin = INT64_MAX, tri = 0;
  for (auto& x : S) dmin = std::min(dmin, x.d);
  const int64_t bt = dmin >= 128 ? 128 : 64;
  for (auto& x : S) {
    const int64_t t = cdiv(x.d, bt);
    tri += t * (t + 1) / 2;
  }
  const int cap = (int)std::max<int64_t>(1, std::min<int64_t>(64, cdiv(maxk, 256)));
  if (tri == 0) return 1;
  const int ncu = 256;
  auto cost = [&](int k) { return (double)cdiv((int64_t)k * tri, ncu) / k; };
  double best = 1e300;
  for (int k = 1; k <= cap; ++k) best = std::min(best, cost(k));
  for (int k = 1; k <= cap; ++k)
    if (cost(k) <= 1.03 * best) return k;
  return 1;
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
    // no bond charge carries blocks on both sides: F(AB) is exactly zero
    // across this bond, no singular value is kept and the bond leg is left
    // with no sector on both tensors (which then hold no block)
    std::vector<Leg> la_legs = a.legs(), lb_legs = b.legs();
    la_legs[la].q.clear();
    la_legs[la].d.clear();
    lb_legs[lb].q.clear();
    lb_legs[lb].d.clear();
    res.a = make_tensor(sym, a.dtype, la_legs, a.total(), s, true);
    res.b = make_tensor(sym, b.dtype, lb_legs, b.total(), s, true);
    return res;
  }
  {
    std::vector<int> order(ng);
    for (int g = 0; g < ng; ++g) order[g] = g;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return q_lt(S[x].charge, S[y].charge); });
    for (int r = 0; r < ng; ++r) S[order[r]].crank = r;
  }
  // Sectors with d <= 128 whose B side is thin (N <= d) while A~ is tall
  // (M > d): the product C = A~ B~ has rank <= N, and its singular values and
  // right singular vectors are those of R_Y from a QR of Y = A~ B~ (M x N,
  // shifted Cholesky QR three times), so the tall A~ is never factored (its
  // Gram matrix and Cholesky-QR passes cost M d^2 each, Y's M N^2). (For
  // d > 128 the same route measured slower on the 40-site workload: those
  // sectors' A sides are not tall enough to pay for its extra small
  // factorisations, and their spectra send them to the one-sided SVD.) The
  // route adds about ten launches per compression, so it is taken only when
  // A~ holds at least 2^22 entries: below that, its passes over A~ cost less
  // than the launches (small networks, e.g. sampled amplitudes, stay on the
  // Gram route).
  constexpr int64_t THIN_MIN_ENTRIES = int64_t(1) << 22;
  for (auto& x : S)
    x.thin = x.d <= JMAX && x.N >= 1 && x.N <= x.d && x.M > x.d && x.M * x.d >= THIN_MIN_ENTRIES;
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
    int64_t maxk = 1;
    for (auto& x : S) maxk = std::max(maxk, std::max(x.M, x.N));
    const int nsplit = gram_split(S, maxk);
    DBuf<double> part((int64_t)nsplit * std::max<int64_t>(gsz, 1), s);
    std::vector<GemmGroup> gA, gB;
    for (int k = 0; k < nsplit; ++k)
      for (int g = 0; g < ng; ++g) {
        const Sect& x = S[g];
        if (x.thin) continue;  // neither Gram matrix is used
        int64_t ca = cdiv(x.M, nsplit), k0 = std::min<int64_t>(k * ca, x.M), k1 = std::min<int64_t>(k0 + ca, x.M);
        // G_A = A~^T A~ : op(A) = A~^T (transA, lda = d), op(B) = A~ (ldb = d)
        gA.push_back(sym_group(plain_group(x.d, x.d, k1 - k0, x.a_off + k0 * x.d, x.d, 1, x.a_off + k0 * x.d, x.d,
                                           0, (int64_t)k * gsz + goffA[g], x.d)));
        int64_t cb = cdiv(x.N, nsplit), j0 = std::min<int64_t>(k * cb, x.N), j1 = std::min<int64_t>(j0 + cb, x.N);
        // G_B = B~ B~^T : op(A) = B~ (lda = N), op(B) = B~^T (transB, ldb = N)
        gB.push_back(sym_group(plain_group(x.d, x.d, j1 - j0, x.b_off + j0, x.N, 0, x.b_off + j0, x.N, 1,
                                           (int64_t)k * gsz + goffB[g], x.d)));
      }
    if (!gA.empty()) {
      run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gA, At.p, At.p, part.p, nullptr, s);
      run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gB, Bt.p, Bt.p, part.p, nullptr, s);
    }
    LAUNCH(k_sum_partials, dim3((unsigned)cdiv(gsz, 256)), dim3(256), 0, s, part.p, gsz, nsplit, Gm.p);
    HIPC(hipGetLastError());
  }
  // G_A = R_A^T R_A and G_B = R_B^T R_B. Sectors with d <= 128 take the
  // accurate factors (the factor itself when it has at most d rows, else
  // shifted Cholesky QR three times); larger ones a dropping Cholesky of a
  // copy of the Gram matrix (the Gram matrices are needed again). The kept
  // rows are packed into Rc (rank x d at the Gram offsets).
  std::vector<int> ranks(2 * ng, -1);
  DBuf<double> Rc(std::max<int64_t>(gsz, 1), s);
  {
    DBuf<double> Fm(std::max<int64_t>(gsz, 1), s);
    std::vector<int64_t> coffs, cdims, poffs, pdims;
    std::vector<int> pidx;
    std::vector<AccSrc> acc;
    std::vector<RowsJob> rows;
    int64_t maxrows = 0;
    for (int g = 0; g < ng; ++g) {
      const Sect& x = S[g];
      for (int side = 0; side < 2; ++side) {
        const int64_t off = side ? goffB[g] : goffA[g];
        const int64_t m = side ? x.N : x.M;
        if (x.thin && side == 0) {  // R_Y stands in for R_A R_B^T (below)
          ranks[2 * g] = (int)x.N;
          continue;
        }
        if (x.d > JMAX && !x.thin) {
          HIPC(hipMemcpyAsync(Fm.p + off, Gm.p + off, x.d * x.d * 8, hipMemcpyDeviceToDevice, s));
          coffs.push_back(off);
          cdims.push_back(x.d);
        } else if (m <= x.d) {
          RowsJob r;
          r.src = side ? Bt.p + x.b_off : At.p + x.a_off;
          r.dst = Rc.p + off;
          r.ld = side ? x.N : x.d;
          r.m = m;
          r.d = (int)x.d;
          r.trans = side;
          rows.push_back(r);
          maxrows = std::max(maxrows, m * x.d);
          ranks[2 * g + side] = (int)m;
          continue;
        } else {
          AccSrc a;
          a.side = side;
          a.trans = side;
          a.off = side ? x.b_off : x.a_off;
          a.ld = side ? x.N : x.d;
          a.m = m;
          a.goff = off;
          a.d = (int)x.d;
          acc.push_back(a);
        }
        poffs.push_back(off);
        pdims.push_back(x.d);
        pidx.push_back(2 * g + side);
      }
    }
    if (!coffs.empty()) chol_drop(Fm.p, coffs, cdims, 1e-13, s);
    acc_factor(acc, At.p, Bt.p, Gm.p, Fm.p, s);
    if (!rows.empty()) {
      const Jobs<RowsJob> dr(rows, s);
      LAUNCH(k_copy_rows, dim3((unsigned)std::min<int64_t>(cdiv(maxrows, 256), 1024), (unsigned)rows.size()),
             dim3(256), 0, s, dr.t);
    }
    const int np = (int)poffs.size();
    std::vector<int> prk(std::max(np, 1));
    if (np) {
      DBuf<int64_t> doff = to_device(poffs, s), ddim = to_device(pdims, s);
      DBuf<int> drk(np, s);
      LAUNCH(k_pack_rows, dim3(np), dim3(1024), 0, s, Fm.p, doff.p, ddim.p, Rc.p, drk.p);
      HIPC(hipMemcpyAsync(prk.data(), drk.p, np * sizeof(int), hipMemcpyDeviceToHost, s));
    }
    HIPC(hipStreamSynchronize(s));
    for (int i = 0; i < np; ++i) ranks[pidx[i]] = prk[i];
  }
  // thin sectors: Y = A~ B~ (M x N) and R_Y (N x N) from its QR; a left
  // inverse E of B~ (d x N) for the B-side projector P_B = S^1/2 V_k^T E (so
  // that P_B B~ = S^1/2 V_k^T): E0 = R_t^-1 Q_t^T from the QR of B~, then one
  // Newton step E = 2 E0 - (E0 B~) E0, which squares the residual I - E B~
  // (E0 alone leaves it at about u cond(B~)^2)
  std::vector<int64_t> tyo(ng, 0), tno(ng, 0), tqo(ng, 0);
  int64_t tys = 0, tns = 0, tqs = 0;
  for (int g = 0; g < ng; ++g) {
    const Sect& x = S[g];
    if (!x.thin) continue;
    tyo[g] = tys;
    tys += x.M * x.N;
    tno[g] = tns;
    tns += x.N * x.N;
    tqo[g] = tqs;
    tqs += x.d * x.N;
  }
  DBuf<double> RY(std::max<int64_t>(tns, 1), s), Rti(std::max<int64_t>(tns, 1), s), Qt(std::max<int64_t>(tqs, 1), s),
      El(std::max<int64_t>(tqs, 1), s);
  if (tns) {
    DBuf<double> Yb(tys, s), GY(tns, s), Gt(tns, s), Rt(tns, s);
    std::vector<GemmGroup> gy, ggy, ggt;
    std::vector<AccSrc> jy, jt;
    for (int g = 0; g < ng; ++g) {
      const Sect& x = S[g];
      if (!x.thin) continue;
      gy.push_back(plain_group(x.M, x.N, x.d, x.a_off, x.d, 0, x.b_off, x.N, 0, tyo[g], x.N));
      ggy.push_back(sym_group(plain_group(x.N, x.N, x.M, tyo[g], x.N, 1, tyo[g], x.N, 0, tno[g], x.N)));
      ggt.push_back(sym_group(plain_group(x.N, x.N, x.d, x.b_off, x.N, 1, x.b_off, x.N, 0, tno[g], x.N)));
      AccSrc u;
      u.side = 0;
      u.trans = 0;
      u.off = tyo[g];
      u.ld = x.N;
      u.m = x.M;
      u.goff = tno[g];
      u.d = (int)x.N;
      jy.push_back(u);
      AccSrc t;
      t.side = 1;
      t.trans = 0;
      t.off = x.b_off;
      t.ld = x.N;
      t.m = x.d;
      t.goff = tno[g];
      t.d = (int)x.N;
      t.qoff = tqo[g];
      t.moff = tno[g];
      jt.push_back(t);
    }
    run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gy, At.p, Bt.p, Yb.p, nullptr, s);
    run_grouped_gemm(FTN_GEMM_F64, FTN_F64, ggy, Yb.p, Yb.p, GY.p, nullptr, s);
    run_grouped_gemm(FTN_GEMM_F64, FTN_F64, ggt, Bt.p, Bt.p, Gt.p, nullptr, s);
    acc_factor(jy, Yb.p, Bt.p, GY.p, RY.p, s);
    acc_factor(jt, Yb.p, Bt.p, Gt.p, Rt.p, s, Qt.p, Rti.p);
    std::vector<GemmGroup> ge0, gz, ge1;
    for (int g = 0; g < ng; ++g) {
      const Sect& x = S[g];
      if (!x.thin) continue;
      ge0.push_back(plain_group(x.N, x.d, x.N, tno[g], x.N, 0, tqo[g], x.N, 1, tqo[g], x.d));  // E0 = R_t^-1 Q_t^T
      gz.push_back(plain_group(x.N, x.N, x.d, tqo[g], x.d, 0, x.b_off, x.N, 0, tno[g], x.N));    // Z = E0 B~
      ge1.push_back(plain_group(x.N, x.d, x.N, tno[g], x.N, 0, tqo[g], x.d, 0, tqo[g], x.d));   // E = 2 E0 - Z E0
    }
    DBuf<double> E0(tqs, s), Zt(tns, s);
    run_grouped_gemm(FTN_GEMM_F64, FTN_F64, ge0, Rti.p, Qt.p, E0.p, nullptr, s);
    run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gz, E0.p, Bt.p, Zt.p, nullptr, s);
    HIPC(hipMemcpyAsync(El.p, E0.p, tqs * 8, hipMemcpyDeviceToDevice, s));
    run_grouped_gemm(FTN_GEMM_F64, FTN_F64, ge1, Zt.p, E0.p, El.p, nullptr, s, -1.0, 2.0);
  }
  // per sector: the side with the smaller rank (A when rA <= rB, and always
  // for iterated sectors) gives R = R_side, G_o = the other Gram matrix;
  // direct sectors diagonalise H = R G_o R^T (r x r, = X X^T or X^T X),
  // iterated ones use X = R_A R_B^T (rA x rB)
  std::vector<int64_t> xoff(ng), hoff(ng), eoff(ng), loff(ng), u1off(ng);
  int64_t xs = 0, hs = 0, es = 0, ls = 0, u1s = 0;
  for (int g = 0; g < ng; ++g) {
    Sect& x = S[g];
    x.rA = ranks[2 * g];
    x.rB = ranks[2 * g + 1];
    x.ns = std::min(x.rA, x.rB);
    x.iterate = x.ns > JMAX;
    x.p = x.iterate ? JMAX : x.ns;
    x.sideA = x.iterate || x.rA <= x.rB;
    x.acc = x.d <= JMAX || x.thin;
    xoff[g] = xs;
    xs += (x.iterate || x.acc) ? (int64_t)x.rA * x.rB : 0;
    hoff[g] = hs;
    hs += x.iterate ? 0 : (int64_t)x.ns * x.ns;
    u1off[g] = u1s;
    u1s += x.iterate ? 0 : x.d * x.ns;
    eoff[g] = es;
    es += (int64_t)(x.iterate ? x.rA : x.ns) * x.p;
    loff[g] = ls;
    ls += std::max(x.p, 1);
  }
  // right singular vectors (r_o x r_o) of the sectors with exact factors
  std::vector<int64_t> voff(ng, 0);
  int64_t vs = 0;
  for (int g = 0; g < ng; ++g) {
    const Sect& x = S[g];
    voff[g] = vs;
    if (x.acc && x.ns && !x.iterate) {
      const int64_t r_o = x.sideA ? x.rB : x.rA;
      vs += r_o * r_o;
    }
  }
  DBuf<double> Xm(std::max<int64_t>(xs, 1), s), Hm(std::max<int64_t>(hs, 1), s), Em(std::max<int64_t>(es, 1), s),
      Lm(std::max<int64_t>(ls, 1), s), Vm(std::max<int64_t>(vs, 1), s);
  HIPC(hipMemsetAsync(Lm.p, 0, std::max<int64_t>(ls, 1) * 8, s));
  {
    DBuf<double> U1(std::max<int64_t>(u1s, 1), s);
    std::vector<GemmGroup> gx, gu, gh, gxs, gxh;
    for (int g = 0; g < ng; ++g) {
      const Sect& x = S[g];
      if (!x.ns) continue;
      if (x.iterate) {
        gx.push_back(plain_group(x.rA, x.rB, x.d, goffA[g], x.d, 0, goffB[g], x.d, 1, xoff[g], x.rB));
        continue;
      }
      const int64_t ro = x.sideA ? goffA[g] : goffB[g], go = x.sideA ? goffB[g] : goffA[g];
      if (x.acc) {
        // accurate factors: X = R R_o^T (r x r_o), H = X X^T; a thin sector
        // takes X = R_Y (N x N: the same singular values and right vectors)
        const int64_t r = x.ns, r_o = x.sideA ? x.rB : x.rA;
        if (x.thin)
          HIPC(hipMemcpyAsync(Xm.p + xoff[g], RY.p + tno[g], x.N * x.N * 8, hipMemcpyDeviceToDevice, s));
        else
          gxs.push_back(plain_group(r, r_o, x.d, ro, x.d, 0, go, x.d, 1, xoff[g], r_o));
        gxh.push_back(sym_group(plain_group(r, r, r_o, xoff[g], r_o, 0, xoff[g], r_o, 1, hoff[g], r)));
        continue;
      }
      // U1 = G_o R^T (d x r), H = R U1 (r x r)
      gu.push_back(plain_group(x.d, x.ns, x.d, go, x.d, 0, ro, x.d, 1, u1off[g], x.ns));
      gh.push_back(plain_group(x.ns, x.ns, x.d, ro, x.d, 0, u1off[g], x.ns, 0, hoff[g], x.ns));
    }
    if (!gx.empty()) run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gx, Rc.p, Rc.p, Xm.p, nullptr, s);
    if (!gxs.empty()) run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gxs, Rc.p, Rc.p, Xm.p, nullptr, s);
    if (!gxh.empty()) run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gxh, Xm.p, Xm.p, Hm.p, nullptr, s);
    if (!gu.empty()) {
      run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gu, Gm.p, Rc.p, U1.p, nullptr, s);
      run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gh, Rc.p, U1.p, Hm.p, nullptr, s);
    }
  }
  x_spectrum(S, chi, Hm.p, hoff, Xm.p, xoff, Em.p, eoff, Lm.p, loff, s);
  // singular values = sqrt(eigenvalues); selection
  launch_1d(std::max<int64_t>(ls, 1), s, k_sqrt_inplace, Lm.p, (int)std::max<int64_t>(ls, 1));
  {
    std::vector<int> grp, idx, crank(ng);
    std::vector<int64_t> pos;
    for (int g = 0; g < ng; ++g) {
      crank[g] = S[g].crank;
      for (int i = 0; i < S[g].p; ++i) {
        grp.push_back(g);
        idx.push_back(i);
        pos.push_back(loff[g] + i);
      }
    }
    const int n = (int)grp.size();
    std::vector<double> hw(std::max<int64_t>(ls, 1));
    HIPC(hipMemcpyAsync(hw.data(), Lm.p, hw.size() * 8, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    // The eigenvalues of H = X X^T hold a singular value s only to about
    // eps s_max^2 / s. A sector with exact factors whose values that matter
    // (kept, or among the chi + 1 largest overall that decide the cut) reach
    // below 1e-4 of its largest is redone by the one-sided Jacobi SVD of X
    // itself, which resolves s to ~eps s_max; its projectors then use the V
    // of that SVD.
    {
      std::vector<std::pair<double, int>> cand;
      for (int i = 0; i < n; ++i) cand.push_back({hw[pos[i]], grp[i]});
      const size_t top = std::min<size_t>(cand.size(), (size_t)std::max<int64_t>(chi, 0) + 1);
      std::partial_sort(cand.begin(), cand.begin() + top, cand.end(),
                        [](const std::pair<double, int>& a, const std::pair<double, int>& b) { return a.first > b.first; });
      std::vector<double> smax(ng, 0.0);
      for (int i = 0; i < n; ++i) smax[grp[i]] = std::max(smax[grp[i]], hw[pos[i]]);
      std::vector<int> redo(ng, 0);
      for (size_t t = 0; t < top; ++t) {
        const int g = cand[t].second;
        if (S[g].acc && !S[g].iterate && cand[t].first < 1e-4 * smax[g]) redo[g] = 1;
      }
      std::vector<SvdJob> sj;
      std::vector<double*> vv;
      for (int g = 0; g < ng; ++g) {
        if (!redo[g]) continue;
        S[g].svd = true;
        const int r = S[g].ns, c = S[g].sideA ? S[g].rB : S[g].rA;
        SvdJob j{};
        j.X = Xm.p + xoff[g];
        j.U = Em.p + eoff[g];
        j.W = Lm.p + loff[g];
        j.r = r;
        j.c = c;
        j.ldx = c;
        j.ldu = S[g].p;
        sj.push_back(j);
        vv.push_back(Vm.p + voff[g]);
      }
      if (!sj.empty()) {
        svd_cols(sj, vv, s);
        for (int g = 0; g < ng; ++g)
          if (redo[g]) launch_1d(S[g].p, s, k_sqrt_inplace, Lm.p + loff[g], S[g].p);
        HIPC(hipMemcpyAsync(hw.data(), Lm.p, hw.size() * 8, hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
      }
    }
    std::vector<double> vals(n);
    for (int i = 0; i < n; ++i) {
      vals[i] = hw[pos[i]];
      if (!std::isfinite(vals[i])) fail(FTN_ENOCONV, "compress_bond: non-finite singular value");
    }
    // sectors without exact factors (bond sector above 128) reach their
    // values through Gram matrices, which resolve a singular value only down
    // to ~1e-7 of the sector's largest: values below 1e-6 of it are zero
    {
      std::vector<double> smax(ng, 0.0);
      for (int i = 0; i < n; ++i) smax[grp[i]] = std::max(smax[grp[i]], vals[i]);
      for (int i = 0; i < n; ++i)
        if (!S[grp[i]].acc && vals[i] < 1e-6 * smax[grp[i]]) vals[i] = 0.0;
    }
    if (ng > 1024) fail(FTN_ENOTSUP, "more than 1024 bond sectors");
    if (cutoff < 0 || !std::isfinite(cutoff)) fail(FTN_EINVAL, "cutoff must be finite and >= 0");
    const double eff_cut = cutoff;
    // inputs of the selection in one upload (values | group | index | charge
    // rank), its outputs in one read-back (4 statistics | kept per group)
    const int64_t ni8 = cdiv(n, 2), nc8 = cdiv(ng, 2);
    std::vector<double> pin(std::max<int64_t>(n + 2 * ni8 + nc8, 1), 0.0);
    std::copy(vals.begin(), vals.end(), pin.begin());
    std::memcpy(pin.data() + n, grp.data(), n * sizeof(int));
    std::memcpy(pin.data() + n + ni8, idx.data(), n * sizeof(int));
    std::memcpy(pin.data() + n + 2 * ni8, crank.data(), ng * sizeof(int));
    DBuf<double> dpin = to_device(pin, s);
    const double* dv = dpin.p;
    const int *dg = (const int*)(dpin.p + n), *di = (const int*)(dpin.p + n + ni8),
              *dc = (const int*)(dpin.p + n + 2 * ni8);
    DBuf<double> dout(4 + std::max<int64_t>(nc8, 1), s);
    int* dk = (int*)(dout.p + 4);
    HIPC(hipMemsetAsync(dout.p, 0, 32, s));
    if (n) LAUNCH(k_select, dim3(1), dim3(LT), 0, s, dv, dg, di, dc, n, ng, chi, eff_cut, dk, dout.p);
    HIPC(hipGetLastError());
    std::vector<double> hout(4 + std::max<int64_t>(nc8, 1), 0.0);
    HIPC(hipMemcpyAsync(hout.data(), dout.p, (4 + (n ? nc8 : 0)) * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    std::vector<double> st(hout.begin(), hout.begin() + 4);
    std::vector<int> kept(std::max(ng, 1), 0);
    if (n) std::memcpy(kept.data(), hout.data() + 4, ng * sizeof(int));
    res.discarded = st[0];
    double a1 = st[1], a2 = st[2];
    res.near_tie = (a2 > 0 && std::fabs(a1 - a2) <= 1e3 * 2.220446049250313e-16 * std::fabs(a1));
    static const bool trace = std::getenv("FTN_TRACE") != nullptr;
    if (trace) {
      double smax = 0;
      for (double v : vals) smax = std::max(smax, v);
      std::string d;
      for (int g = 0; g < ng; ++g)
        d += std::to_string(S[g].d) + ":" + std::to_string(kept[g]) + "(" + std::to_string(S[g].M) + "x" +
             std::to_string(S[g].N) + " r" + std::to_string(S[g].rA) + "/" + std::to_string(S[g].rB) + ") ";
      std::fprintf(stderr, "[ftn] compress: sectors %s chi-th %.17g next %.17g max %.17g\n", d.c_str(), a1, a2, smax);
    }
    for (int g = 0; g < ng; ++g) S[g].kept = kept[g];
    {
      auto qr = [](double m, double n) {
        const double a = std::max(m, n), b = std::min(m, n);
        return 4.0 * a * b * b - 4.0 * b * b * b / 3.0;
      };
      for (int g = 0; g < ng; ++g) {
        const double M = (double)S[g].M, N = (double)S[g].N, d = (double)S[g].d;
        const double ra = std::min(M, d), rb = std::min(N, d);
        const double hi = std::max(ra, rb), lo = std::min(ra, rb);
        res.textbook_flops += qr(M, d) + qr(N, d) + 14.0 * hi * lo * lo + 8.0 * lo * lo * lo +
                              2.0 * (M * ra + N * rb) * S[g].kept;
      }
    }
    for (int g = 0; g < ng; ++g)
      for (int i = 0; i < S[g].kept; ++i) res.svals.push_back(hw[loff[g] + i]);
    std::sort(res.svals.begin(), res.svals.end(), std::greater<double>());
  }
  // projectors. E_k (r x k): the leading eigenvectors of H (direct) or the
  // left singular vectors of X (iterated). With F = R^T E_k and GF = G_o F
  // (both d x k):
  //   side A: P_A = GF S^-3/2, P_B = S^-1/2 F^T   (E_k = U)
  //   side B: P_A = F S^-1/2,  P_B = S^-3/2 GF^T  (E_k = V)
  // (from P_A = R_B^T V S^-1/2, P_B = S^-1/2 U^T R_A and X^T U = V S).
  std::vector<int64_t> pa_off(ng), pb_off(ng), fo(ng);
  int64_t pas = 0, fs = 0;
  for (int g = 0; g < ng; ++g) {
    const Sect& x = S[g];
    pa_off[g] = pas;
    pas += x.d * x.kept;
    pb_off[g] = pas;
    pas += x.kept * x.d;
    fo[g] = fs;
    fs += x.d * x.kept;
  }
  DBuf<double> PAB(std::max<int64_t>(pas, 1), s), Fk(std::max<int64_t>(fs, 1), s), GF(std::max<int64_t>(fs, 1), s);
  {
    // with accurate factors GF = R_o^T (X^T E_k) replaces G_o F
    std::vector<GemmGroup> gf, ggf, gw, gwf;
    std::vector<ScaleColsJob> scols;
    std::vector<int64_t> wo(ng);
    int64_t wsz = 0;
    for (int g = 0; g < ng; ++g) {
      const Sect& x = S[g];
      wo[g] = wsz;
      if (x.kept && x.acc) wsz += (int64_t)(x.sideA ? x.rB : x.rA) * x.kept;
    }
    DBuf<double> Wk(std::max<int64_t>(wsz, 1), s);
    for (int g = 0; g < ng; ++g) {
      const Sect& x = S[g];
      if (!x.kept) continue;
      const int64_t r = x.sideA ? x.rA : x.rB;
      const int64_t ro = x.sideA ? goffA[g] : goffB[g], go = x.sideA ? goffB[g] : goffA[g];
      if (!x.thin) gf.push_back(plain_group(x.d, x.kept, r, ro, x.d, 1, eoff[g], x.p, 0, fo[g], x.kept));
      if (x.acc) {
        // W_k = V_k S_k: from the accumulated rotations of the one-sided SVD,
        // else X^T E_k (accurate while the kept values stay above 1e-4 s_max)
        const int64_t r_o = x.sideA ? x.rB : x.rA;
        if (x.svd)
          scols.push_back(ScaleColsJob{Vm.p + voff[g], Lm.p + loff[g], Wk.p + wo[g], r_o, x.kept, r_o});
        else
          gw.push_back(plain_group(r_o, x.kept, r, xoff[g], r_o, 1, eoff[g], x.p, 0, wo[g], x.kept));
        gwf.push_back(plain_group(x.d, x.kept, r_o, go, x.d, 1, wo[g], x.kept, 0, fo[g], x.kept));
      } else {
        ggf.push_back(plain_group(x.d, x.kept, x.d, go, x.d, 0, fo[g], x.kept, 0, fo[g], x.kept));
      }
    }
    bool anykept = false;
    for (int g = 0; g < ng; ++g) anykept = anykept || S[g].kept > 0;
    if (anykept) {
      if (!gf.empty()) run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gf, Rc.p, Em.p, Fk.p, nullptr, s);
      if (!ggf.empty()) run_grouped_gemm(FTN_GEMM_F64, FTN_F64, ggf, Gm.p, Fk.p, GF.p, nullptr, s);
      if (!scols.empty()) {
        int64_t mx = 1;
        for (auto& j : scols) mx = std::max<int64_t>(mx, j.rows * j.cols);
        const Jobs<ScaleColsJob> dj(scols, s);
        LAUNCH(k_scale_cols, dim3((unsigned)std::min<int64_t>(cdiv(mx, 256), 1024), (unsigned)scols.size()), dim3(256),
               0, s, dj.t);
      }
      if (!gw.empty()) run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gw, Xm.p, Em.p, Wk.p, nullptr, s);
      if (!gwf.empty()) run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gwf, Rc.p, Wk.p, GF.p, nullptr, s);
      {
        // thin sectors: F = E^T W_k (W_k = V_k S_k), so that
        // P_B = S^-1/2 F^T = S^1/2 V_k^T E
        std::vector<GemmGroup> gt1;
        for (int g = 0; g < ng; ++g) {
          const Sect& x = S[g];
          if (!x.kept || !x.thin) continue;
          gt1.push_back(plain_group(x.d, x.kept, x.N, tqo[g], x.d, 1, wo[g], x.kept, 0, fo[g], x.kept));
        }
        if (!gt1.empty()) run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gt1, El.p, Wk.p, Fk.p, nullptr, s);
      }
      for (int g = 0; g < ng; ++g) {
        const Sect& x = S[g];
        if (!x.kept) continue;
        const int64_t n = x.d * x.kept;
        LAUNCH(k_proj_out, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, Fk.p + fo[g], GF.p + fo[g], x.d, x.kept,
               Lm.p + loff[g], (int)x.sideA, PAB.p + pa_off[g], PAB.p + pb_off[g]);
      }
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

// ---------------------------------------------------------------------------
// Adjoint of bond compression (derivative of the truncated SVD, the kept
// count per sector held fixed). Per bond charge, with the fused matrices
// A~ (M x d) and B~ (d x N) of the forward contraction, the product
// C = A~ B~ = U S V^T and the outputs A' = U_k S_k^1/2, B' = S_k^1/2 V_k^T.
// Exact factors A~ = Q_A R_A, B~^T = Q_B R_B (shifted Cholesky QR three
// times, Q explicit) give X = R_A R_B^T = U_X S V_X^T with U = Q_A U_X and
// V = Q_B V_X. For cotangents dA', dB' the cotangent of C is
//   dC = U Y V^T + (I - U U^T) Gu S_k^-1 V_k^T + U_k S_k^-1 Gv^T (I - V V^T)
// with Gu = dA' S_k^1/2, Gv = dB'^T S_k^1/2, a = U^T Gu, b = V^T Gv and
//   Y_xy = [y < k, x != y] (a_xy s_y + b_xy s_x) / (s_y^2 - s_x^2)
//        + [x < k, x != y] (a_yx s_y + b_yx s_x) / (s_x^2 - s_y^2)
//        + [x = y < k] (a_xx + b_xx) / (2 s_x)
// (U and V over the nonzero singular values; the projections onto their
// complements carry the directions outside the column and row spaces). Then
// dA~ = dC B~^T = dA' P_A^T + Q_A W_A and dB~ = A~^T dC = P_B^T dB' + W_B Q_B^T
// with the projectors P_A = R_B^T V_k S_k^-1/2, P_B = S_k^-1/2 U_k^T R_A and
//   W_A = U_X [Y G1 - a S_k^-1 G1_k + E_k (S_k^-1/2 qb^T R_B - S_k^-1 b^T G1)],
//   W_B = R_A^T [U_X (Y V_X^T - a S_k^-1 V_Xk^T) - U_Xk S_k^-1 b^T V_X^T
//                + qa S_k^-1/2 V_Xk^T],
// where G1 = V_X^T R_B, qa = Q_A^T dA' and qb = Q_B^T dB'^T (so that
// a = U_X^T qa S_k^1/2 and b = V_X^T qb S_k^1/2). Only these products touch
// the tall dimensions. The signs of the kept singular vectors follow the
// forward outputs (the derivative of a loss that is invariant under
// A' -> A' D, B' -> D B' for diagonal D = +-1 does not depend on them).
// Couplings between singular values closer than 1e-13 of s_max^2 are dropped.

struct AdjJob {
  const double *U, *lam, *X, *RA, *RB;  // d x d (U columns = eigenvectors of X X^T, descending)
  const double *qa, *qb, *qf;           // d x k: Q_A^T dA', Q_B^T dB'^T, Q_A^T A'
  double *WA, *WB, *PAt, *PB;           // d x d, d x d, k x d, k x d
  double* ws;                           // scratch: 7 d x d
  int d, k;
};

__device__ inline void adj_sync() { __syncthreads(); }

__global__ void __launch_bounds__(1024) k_svd_adjoint(const AdjJob* jobs) {
  const AdjJob J = jobs[blockIdx.x];
  const int d = J.d, k = J.k, tid = threadIdx.x;
  __shared__ double sv[EIG_BIG_MAX], sg[EIG_BIG_MAX];
  __shared__ int rho_s;
  const int64_t dd = (int64_t)d * d;
  double *Us = J.ws, *V = J.ws + dd, *al = J.ws + 2 * dd, *be = J.ws + 3 * dd, *Y = J.ws + 4 * dd,
         *G1 = J.ws + 5 * dd, *Z = J.ws + 6 * dd;
  for (int j = tid; j < d; j += blockDim.x) sv[j] = sqrt(fmax(J.lam[j], 0.0));
  adj_sync();
  if (tid == 0) {
    int r = 0;
    while (r < d && sv[r] > 1e-12 * sv[0]) ++r;
    rho_s = r;
  }
  // signs of the kept vectors from the forward outputs
  for (int i = tid; i < k; i += blockDim.x) {
    double t = 0;
    for (int l = 0; l < d; ++l) t += J.qf[(int64_t)l * k + i] * J.U[(int64_t)l * d + i];
    sg[i] = t < 0 ? -1.0 : 1.0;
  }
  adj_sync();
  const int rho = rho_s;
  const double s0 = sv[0], tie = 1e-13 * s0 * s0;
  for (int64_t e = tid; e < dd; e += blockDim.x) {
    const int j = (int)(e % d);
    Us[e] = J.U[e] * (j < k ? sg[j] : 1.0);
  }
  adj_sync();
  // V (d x rho) = X^T U S^-1
  for (int64_t e = tid; e < (int64_t)d * rho; e += blockDim.x) {
    const int r = (int)(e / rho), j = (int)(e % rho);
    double t = 0;
    for (int l = 0; l < d; ++l) t += J.X[(int64_t)l * d + r] * Us[(int64_t)l * d + j];
    V[(int64_t)r * d + j] = t / sv[j];
  }
  adj_sync();
  // a, b (rho x k)
  for (int64_t e = tid; e < (int64_t)rho * k; e += blockDim.x) {
    const int j = (int)(e / k), i = (int)(e % k);
    double ta = 0, tb = 0;
    for (int l = 0; l < d; ++l) {
      ta += Us[(int64_t)l * d + j] * J.qa[(int64_t)l * k + i];
      tb += V[(int64_t)l * d + j] * J.qb[(int64_t)l * k + i];
    }
    const double r = sqrt(sv[i]);
    al[(int64_t)j * d + i] = ta * r;
    be[(int64_t)j * d + i] = tb * r;
  }
  adj_sync();
  // Y (rho x rho)
  for (int64_t e = tid; e < (int64_t)rho * rho; e += blockDim.x) {
    const int x = (int)(e / rho), y = (int)(e % rho);
    double t = 0;
    if (x == y) {
      if (x < k) t = (al[(int64_t)x * d + x] + be[(int64_t)x * d + x]) / (2.0 * sv[x]);
    } else {
      const double sx = sv[x], sy = sv[y];
      const double del = sy * sy - sx * sx;  // s_y^2 - s_x^2
      if (fabs(del) > tie) {
        if (y < k) t += (al[(int64_t)x * d + y] * sy + be[(int64_t)x * d + y] * sx) / del;
        if (x < k) t -= (al[(int64_t)y * d + x] * sy + be[(int64_t)y * d + x] * sx) / del;
      }
    }
    Y[(int64_t)x * d + y] = t;
  }
  adj_sync();
  // G1 = V^T R_B (rho x d)
  for (int64_t e = tid; e < (int64_t)rho * d; e += blockDim.x) {
    const int j = (int)(e / d), c = (int)(e % d);
    double t = 0;
    for (int l = 0; l < d; ++l) t += V[(int64_t)l * d + j] * J.RB[(int64_t)l * d + c];
    G1[(int64_t)j * d + c] = t;
  }
  adj_sync();
  // Z = Y G1 - a S^-1 G1_k + E_k (S^-1/2 qb^T R_B - S^-1 b^T G1)   (rho x d)
  for (int64_t e = tid; e < (int64_t)rho * d; e += blockDim.x) {
    const int x = (int)(e / d), c = (int)(e % d);
    double t = 0;
    for (int y = 0; y < rho; ++y) t += Y[(int64_t)x * d + y] * G1[(int64_t)y * d + c];
    for (int i = 0; i < k; ++i) t -= al[(int64_t)x * d + i] / sv[i] * G1[(int64_t)i * d + c];
    if (x < k) {
      double u = 0, w = 0;
      for (int l = 0; l < d; ++l) u += J.qb[(int64_t)l * k + x] * J.RB[(int64_t)l * d + c];
      for (int j = 0; j < rho; ++j) w += be[(int64_t)j * d + x] * G1[(int64_t)j * d + c];
      t += u / sqrt(sv[x]) - w / sv[x];
    }
    Z[(int64_t)x * d + c] = t;
  }
  adj_sync();
  // W_A = U_rho Z (d x d); P_A^T = S^-1/2 G1_k; P_B = S^-1/2 U_k^T R_A
  for (int64_t e = tid; e < dd; e += blockDim.x) {
    const int r = (int)(e / d), c = (int)(e % d);
    double t = 0;
    for (int x = 0; x < rho; ++x) t += Us[(int64_t)r * d + x] * Z[(int64_t)x * d + c];
    J.WA[e] = t;
  }
  for (int64_t e = tid; e < (int64_t)k * d; e += blockDim.x) {
    const int i = (int)(e / d), c = (int)(e % d);
    J.PAt[e] = G1[(int64_t)i * d + c] / sqrt(sv[i]);
    double t = 0;
    for (int l = 0; l < d; ++l) t += Us[(int64_t)l * d + i] * J.RA[(int64_t)l * d + c];
    J.PB[e] = t / sqrt(sv[i]);
  }
  adj_sync();
  // Z <- Y V^T - a S^-1 V_k^T - E_k S^-1 b^T V^T   (rho x d, columns = rows of V)
  for (int64_t e = tid; e < (int64_t)rho * d; e += blockDim.x) {
    const int x = (int)(e / d), c = (int)(e % d);
    double t = 0;
    for (int y = 0; y < rho; ++y) t += Y[(int64_t)x * d + y] * V[(int64_t)c * d + y];
    for (int i = 0; i < k; ++i) t -= al[(int64_t)x * d + i] / sv[i] * V[(int64_t)c * d + i];
    if (x < k) {
      double w = 0;
      for (int j = 0; j < rho; ++j) w += be[(int64_t)j * d + x] * V[(int64_t)c * d + j];
      t -= w / sv[x];
    }
    Z[(int64_t)x * d + c] = t;
  }
  adj_sync();
  // inner (d x d) = U_rho Z + qa S^-1/2 V_k^T, kept in G1's place
  double* In = G1;
  for (int64_t e = tid; e < dd; e += blockDim.x) {
    const int r = (int)(e / d), c = (int)(e % d);
    double t = 0;
    for (int x = 0; x < rho; ++x) t += Us[(int64_t)r * d + x] * Z[(int64_t)x * d + c];
    for (int i = 0; i < k; ++i) t += J.qa[(int64_t)r * k + i] / sqrt(sv[i]) * V[(int64_t)c * d + i];
    In[e] = t;
  }
  adj_sync();
  // W_B = R_A^T inner
  for (int64_t e = tid; e < dd; e += blockDim.x) {
    const int r = (int)(e / d), c = (int)(e % d);
    double t = 0;
    for (int l = 0; l < d; ++l) t += J.RA[(int64_t)l * d + r] * In[(int64_t)l * d + c];
    J.WB[e] = t;
  }
}

void op_compress_bond_backward(const Tensor& a, const Tensor& b, int la, int lb, int64_t chi, double cutoff, int conv,
                               const Tensor& dao, const Tensor& dbo, hipStream_t s, std::unique_ptr<Tensor>& da,
                               std::unique_ptr<Tensor>& db) {
  if (a.dtype != FTN_F64 || b.dtype != FTN_F64 || dao.dtype != FTN_F64 || dbo.dtype != FTN_F64)
    fail(FTN_ENOTSUP, "compress_bond_backward: FP64 only");
  // the forward outputs (the same deterministic computation)
  CompressResult fw = op_compress_bond(a, b, la, lb, chi, cutoff, conv, s);
  if (dao.st->skey != fw.a->st->skey || dbo.st->skey != fw.b->st->skey)
    fail(FTN_EINVAL, "compress_bond_backward: cotangents must have the structures of the compressed tensors");
  const int sym = a.sym();
  const Leg& LA = a.legs()[la];
  const Leg& LB = b.legs()[lb];
  const Leg& nla = fw.a->legs()[la];
  const Leg& nlb = fw.b->legs()[lb];
  Leg cla = LA, clb = LB;
  cla.dual = 1 - LA.dual;
  clb.dual = 1 - LB.dual;
  Q zero{0, 0};
  da = make_tensor(a.st, FTN_F64, s, true);
  db = make_tensor(b.st, FTN_F64, s, true);
  if (nla.nsect() == 0) return;  // nothing kept: the outputs do not depend on a, b
  // plans of the forward's absorptions A1 = F(a P_A), B1 = F(P_B b)
  auto PA0 = make_tensor(sym, FTN_F64, {cla, nla}, zero, s, true);
  auto PB0 = make_tensor(sym, FTN_F64, {nlb, clb}, zero, s, true);
  auto PlA = dot_plan(a, *PA0, {la}, {0}, FTN_GLOBAL, FTN_GEMM_F64, s);
  auto PlB = dot_plan(*PB0, b, {1}, {lb}, FTN_GLOBAL, FTN_GEMM_F64, s);
  const DotPlanView va = dot_plan_view(*PlA), vb = dot_plan_view(*PlB);
  // A1 / B1 layouts of the outputs and cotangents (bond leg moved back)
  const int na = a.ndim(), nb = b.ndim();
  std::vector<int> inv_a(na), inv_b(nb);
  {
    int t = 0;
    for (int i = 0; i < na; ++i)
      if (i != la) inv_a[t++] = i;
    inv_a[na - 1] = la;
    inv_b[0] = lb;
    t = 1;
    for (int i = 0; i < nb; ++i)
      if (i != lb) inv_b[t++] = i;
  }
  auto A1 = op_ftranspose(*fw.a, inv_a, s), dA1 = op_ftranspose(dao, inv_a, s);
  auto dB1 = op_ftranspose(dbo, inv_b, s);
  std::vector<int64_t> fa_off, fb_off;
  const int64_t fa_n = dot_gather_output(*PlA, *A1, nullptr, fa_off, s);
  const int64_t fb_n = dot_gather_output(*PlB, *dB1, nullptr, fb_off, s);
  DBuf<double> Af(std::max<int64_t>(fa_n, 1), s), dAf(std::max<int64_t>(fa_n, 1), s), dBf(std::max<int64_t>(fb_n, 1), s);
  dot_gather_output(*PlA, *A1, Af.p, fa_off, s);
  dot_gather_output(*PlA, *dA1, dAf.p, fa_off, s);
  dot_gather_output(*PlB, *dB1, dBf.p, fb_off, s);
  // fused inputs
  DBuf<double> At(std::max<int64_t>(va.asz, 1), s), Bt(std::max<int64_t>(vb.bsz, 1), s);
  run_perm(0, a.S(), FTN_F64, *va.pa, a.data, At.p, s);
  run_perm(0, b.S(), FTN_F64, *vb.pb, b.data, Bt.p, s);
  // sectors: groups of the A plan matched to groups of the B plan by charge
  struct BS {
    int ga, gb;
    int64_t M, N, d, k;
    int64_t a_off, b_off, fa, fb;
  };
  std::vector<BS> S;
  for (size_t g = 0; g < va.groups.size(); ++g) {
    const GemmGroup& G = va.groups[g];
    if (G.K == 0 || G.N == 0) continue;
    int h = -1;
    for (size_t j = 0; j < vb.groups.size(); ++j)
      if (q_eq(vb.gq[j], va.gq[g])) h = (int)j;
    if (h < 0) fail(FTN_EINVAL, "internal: compress backward sector without a partner");
    const GemmGroup& H = vb.groups[h];
    if (H.K != G.K || H.M != G.N) fail(FTN_EINVAL, "internal: compress backward sector mismatch");
    if (G.K > EIG_BIG_MAX)
      fail(FTN_ENOTSUP, "compress_bond_backward: bond sectors larger than 1024 are not supported");
    BS x;
    x.ga = (int)g;
    x.gb = h;
    x.M = G.M;
    x.N = H.N;
    x.d = G.K;
    x.k = G.N;
    x.a_off = G.a_off;
    x.b_off = H.b_off;
    x.fa = fa_off[g];
    x.fb = fb_off[h];
    S.push_back(x);
  }
  const int ns = (int)S.size();
  if (!ns) return;
  // per-sector buffers
  std::vector<int64_t> go(ns), qao(ns), qbo(ns), ko(ns);
  int64_t gs = 0, qas = 0, qbs = 0, ks = 0;
  for (int i = 0; i < ns; ++i) {
    go[i] = gs;
    gs += S[i].d * S[i].d;
    qao[i] = qas;
    qas += S[i].M * S[i].d;
    qbo[i] = qbs;
    qbs += S[i].N * S[i].d;
    ko[i] = ks;
    ks += S[i].d * S[i].k;
  }
  DBuf<double> GA(gs, s), GB(gs, s), RA(gs, s), RB(gs, s), QA(std::max<int64_t>(qas, 1), s),
      QB(std::max<int64_t>(qbs, 1), s), X(gs, s), Hm(gs, s), U(gs, s), lam(std::max<int64_t>(gs, 1), s);
  {
    std::vector<GemmGroup> ga, gb;
    for (int i = 0; i < ns; ++i) {
      const BS& x = S[i];
      ga.push_back(sym_group(plain_group(x.d, x.d, x.M, x.a_off, x.d, 1, x.a_off, x.d, 0, go[i], x.d)));
      gb.push_back(sym_group(plain_group(x.d, x.d, x.N, x.b_off, x.N, 0, x.b_off, x.N, 1, go[i], x.d)));
    }
    run_grouped_gemm(FTN_GEMM_F64, FTN_F64, ga, At.p, At.p, GA.p, nullptr, s);
    run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gb, Bt.p, Bt.p, GB.p, nullptr, s);
  }
  {
    std::vector<AccSrc> ja, jb;
    for (int i = 0; i < ns; ++i) {
      const BS& x = S[i];
      AccSrc u;
      u.side = 0;
      u.trans = 0;
      u.off = x.a_off;
      u.ld = x.d;
      u.m = x.M;
      u.goff = go[i];
      u.d = (int)x.d;
      u.qoff = qao[i];
      ja.push_back(u);
      u.side = 1;
      u.trans = 1;
      u.off = x.b_off;
      u.ld = x.N;
      u.m = x.N;
      u.qoff = qbo[i];
      jb.push_back(u);
    }
    acc_factor(ja, At.p, Bt.p, GA.p, RA.p, s, QA.p);
    acc_factor(jb, At.p, Bt.p, GB.p, RB.p, s, QB.p);
  }
  {
    // X = R_A R_B^T, H = X X^T, all eigenpairs of H
    std::vector<GemmGroup> gx, gh;
    for (int i = 0; i < ns; ++i) {
      const int64_t d = S[i].d;
      gx.push_back(plain_group(d, d, d, go[i], d, 0, go[i], d, 1, go[i], d));
      gh.push_back(sym_group(plain_group(d, d, d, go[i], d, 0, go[i], d, 1, go[i], d)));
    }
    run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gx, RA.p, RB.p, X.p, nullptr, s);
    run_grouped_gemm(FTN_GEMM_F64, FTN_F64, gh, X.p, X.p, Hm.p, nullptr, s);
    std::vector<EigJob> ej(ns);
    for (int i = 0; i < ns; ++i) {
      EigJob& j = ej[i];
      j = EigJob{};
      j.H = Hm.p + go[i];
      j.V = U.p + go[i];
      j.W = lam.p + go[i];
      j.n = (int)S[i].d;
    }
    sym_eig(ej, s);
  }
  // qa = Q_A^T dA', qb = Q_B^T dB'^T, qf = Q_A^T A'   (d x k)
  DBuf<double> qa(std::max<int64_t>(ks, 1), s), qb(std::max<int64_t>(ks, 1), s), qf(std::max<int64_t>(ks, 1), s);
  {
    std::vector<GemmGroup> g1, g2;
    for (int i = 0; i < ns; ++i) {
      const BS& x = S[i];
      g1.push_back(plain_group(x.d, x.k, x.M, qao[i], x.d, 1, x.fa, x.k, 0, ko[i], x.k));
      g2.push_back(plain_group(x.d, x.k, x.N, qbo[i], x.d, 1, x.fb, x.N, 1, ko[i], x.k));
    }
    run_grouped_gemm(FTN_GEMM_F64, FTN_F64, g1, QA.p, dAf.p, qa.p, nullptr, s);
    run_grouped_gemm(FTN_GEMM_F64, FTN_F64, g1, QA.p, Af.p, qf.p, nullptr, s);
    run_grouped_gemm(FTN_GEMM_F64, FTN_F64, g2, QB.p, dBf.p, qb.p, nullptr, s);
  }
  // the small adjoint algebra, one workgroup per sector
  DBuf<double> WA(gs, s), WB(gs, s), PAt(std::max<int64_t>(ks, 1), s), PB(std::max<int64_t>(ks, 1), s),
      scratch(7 * gs, s);
  {
    std::vector<AdjJob> jobs(ns);
    for (int i = 0; i < ns; ++i) {
      AdjJob& j = jobs[i];
      j.U = U.p + go[i];
      j.lam = lam.p + go[i];
      j.X = X.p + go[i];
      j.RA = RA.p + go[i];
      j.RB = RB.p + go[i];
      j.qa = qa.p + ko[i];
      j.qb = qb.p + ko[i];
      j.qf = qf.p + ko[i];
      j.WA = WA.p + go[i];
      j.WB = WB.p + go[i];
      j.PAt = PAt.p + ko[i];
      j.PB = PB.p + ko[i];
      j.ws = scratch.p + 7 * go[i];
      j.d = (int)S[i].d;
      j.k = (int)S[i].k;
    }
    DBuf<AdjJob> dj = to_device(jobs, s);
    LAUNCH(k_svd_adjoint, dim3((unsigned)ns), dim3(1024), 0, s, dj.p);
  }
  // dA~ = dA' P_A^T + Q_A W_A ; dB~ = P_B^T dB' + W_B Q_B^T (in the A / B plan layouts)
  DBuf<double> dAt(std::max<int64_t>(va.asz, 1), s), dBt(std::max<int64_t>(vb.bsz, 1), s);
  if (va.asz) HIPC(hipMemsetAsync(dAt.p, 0, va.asz * 8, s));
  if (vb.bsz) HIPC(hipMemsetAsync(dBt.p, 0, vb.bsz * 8, s));
  {
    std::vector<GemmGroup> a1, a2, b1, b2;
    for (int i = 0; i < ns; ++i) {
      const BS& x = S[i];
      a1.push_back(plain_group(x.M, x.d, x.k, x.fa, x.k, 0, ko[i], x.d, 0, x.a_off, x.d));
      a2.push_back(plain_group(x.M, x.d, x.d, qao[i], x.d, 0, go[i], x.d, 0, x.a_off, x.d));
      b1.push_back(plain_group(x.d, x.N, x.k, ko[i], x.d, 1, x.fb, x.N, 0, x.b_off, x.N));
      b2.push_back(plain_group(x.d, x.N, x.d, go[i], x.d, 0, qbo[i], x.d, 1, x.b_off, x.N));
    }
    run_grouped_gemm(FTN_GEMM_F64, FTN_F64, a1, dAf.p, PAt.p, dAt.p, nullptr, s);
    run_grouped_gemm(FTN_GEMM_F64, FTN_F64, a2, QA.p, WA.p, dAt.p, nullptr, s, 1.0, 1.0);
    run_grouped_gemm(FTN_GEMM_F64, FTN_F64, b1, PB.p, dBf.p, dBt.p, nullptr, s);
    run_grouped_gemm(FTN_GEMM_F64, FTN_F64, b2, WB.p, QB.p, dBt.p, nullptr, s, 1.0, 1.0);
  }
  run_perm(1, a.S(), FTN_F64, *va.pa, dAt.p, da->data, s);
  run_perm(1, b.S(), FTN_F64, *vb.pb, dBt.p, db->data, s);
  HIPC(hipStreamSynchronize(s));
}

}  // namespace ftn
