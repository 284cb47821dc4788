// Fermionic pairwise contraction, Eq. (standardcontract), as signed permutes
// into per-charge fused matrices plus one grouped MFMA GEMM.
//
// For contracted charge Q (the sigma-weighted charge of the contracted legs
// seen from A), every free-A sector combination f with charge s(A) - Q pairs
// with every common contracted combination k of charge Q, and every free-B
// combination g with charge s(B) + Q; so A~_Q (rows f, cols k), B~_Q (rows
// k, cols g) and C_Q = A~_Q B~_Q are dense, and each output block (f, g)
// belongs to exactly one Q. Signs (per block, on the device):
//   A: Koszul sign of A -> free(A) ++ axes_a;
//   B: Koszul sign of B -> axes_b ++ free(B), the pairing reversal
//      sum_{s<t} p_s p_t, and (local convention, Eq. fermionictn2) the bond
//      parity of every bond whose end on A is '+'.
// Host code only builds leg-level combination tables; per-block matching,
// signs and the output block table are computed by device kernels, and the
// resulting plan is cached per (structures, axes, convention, dtype, gemm).
#include <algorithm>
#include <map>
#include <mutex>

#include "common.h"

namespace ftn {

struct DotSide {
  int n;       // legs of the tensor
  int nf, nc;  // free / contracted legs
  int fpos[MAXD];
  int64_t fmul[MAXD];
  int cpos[MAXD];
  int64_t cmul[MAXD];
  int kbase[MAXD];
};

// per block of one operand: free combo r, contracted combo kk ->
// moff = base[r] + kpos[kk] * kmul[r], gext = ext[r]
__global__ void k_dot_tasks(DotSide d, const int32_t* __restrict__ keys, int64_t nb,
                            const int32_t* __restrict__ kmap, const int64_t* __restrict__ base,
                            const int64_t* __restrict__ kmul, const int64_t* __restrict__ ext,
                            const int64_t* __restrict__ kpos, PermTask* tasks) {
  int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int32_t* k = keys + b * d.n;
  int64_t r = 0;
  for (int i = 0; i < d.nf; ++i) r += (int64_t)k[d.fpos[i]] * d.fmul[i];
  int64_t kk = 0;
  bool ok = true;
  for (int t = 0; t < d.nc; ++t) {
    int32_t c = kmap[d.kbase[t] + k[d.cpos[t]]];
    if (c < 0) ok = false;
    kk += (int64_t)(c < 0 ? 0 : c) * d.cmul[t];
  }
  PermTask tk;
  tk.block = b;
  tk.bext = 1;
  tk.extra = 0;
  ok = ok && base[r] >= 0;
  tk.skip = ok ? 0 : 1;
  tk.moff = ok ? base[r] + kpos[kk] * kmul[r] : 0;
  tk.gext = ok ? ext[r] : 1;
  tasks[b] = tk;
}

// per output block: (row combo, col combo) -> block offset table
struct BoffArgs {
  int n, nfa, nfb;
  int64_t fmul[MAXD];
  int64_t gmul[MAXD];
};
__global__ void k_dot_boff(BoffArgs a, const int32_t* __restrict__ keys, const int64_t* __restrict__ off,
                           int64_t nb, const int32_t* __restrict__ rgroup, const int32_t* __restrict__ rlocal,
                           const int32_t* __restrict__ clocal, const int64_t* __restrict__ gbase,
                           const int32_t* __restrict__ gncc, int64_t* boff) {
  int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= nb) return;
  int64_t r = 0, c = 0;
  for (int i = 0; i < a.nfa; ++i) r += (int64_t)keys[b * a.n + i] * a.fmul[i];
  for (int i = 0; i < a.nfb; ++i) c += (int64_t)keys[b * a.n + a.nfa + i] * a.gmul[i];
  int g = rgroup[r];
  if (g < 0 || clocal[c] < 0) return;
  boff[gbase[g] + (int64_t)rlocal[r] * gncc[g] + clocal[c]] = off[b];
}

struct Combos {
  std::vector<Q> q;
  std::vector<int64_t> d;
};

// all combinations (lexicographic, last leg fastest) of the given per-leg
// sector lists; charge = sum of sigma(dual) * q
static Combos combos(int sym, const std::vector<std::vector<Q>>& qs, const std::vector<std::vector<int64_t>>& ds,
                     const std::vector<int>& duals) {
  Combos c;
  const int n = (int)qs.size();
  int64_t tot = 1;
  for (auto& v : qs) tot *= (int64_t)v.size();
  c.q.resize(tot);
  c.d.resize(tot);
  std::vector<int> idx(n, 0);
  for (int64_t t = 0; t < tot; ++t) {
    int64_t r = t;
    for (int i = n - 1; i >= 0; --i) {
      idx[i] = (int)(r % (int64_t)qs[i].size());
      r /= (int64_t)qs[i].size();
    }
    Q acc{0, 0};
    int64_t dd = 1;
    for (int i = 0; i < n; ++i) {
      acc = q_add(sym, acc, q_signed(sym, duals[i], qs[i][idx[i]]));
      dd *= ds[i][idx[i]];
    }
    c.q[t] = acc;
    c.d[t] = dd;
  }
  return c;
}

struct DotPlan {
  std::shared_ptr<const Structure> cst;
  PermPlan pa, pb;
  GemmPlan gp;
  DBuf<int64_t> rc_start, cc_start, cc_dim, boff;
  GemmScatter sc;
  // forward product reading A's blocks where they lie (set when A needs no
  // fused copy); gp above keeps the fused-operand form for the adjoint
  bool direct_a = false;
  GemmPlan gpd;
  int64_t asz = 0, bsz = 0;
  double flops = 0;
  std::vector<Q> gq;  // contracted charge Q of each GEMM group
};

static std::mutex g_plan_mu;
static auto& g_plans = *new std::unordered_map<std::string, std::shared_ptr<DotPlan>>();

// the sign bit a signed permute with descriptor op gives a block of parity
// mask P (the device's sign_bit, for plans built on the host)
static int host_sign_bit(const SignOp& op, uint32_t P) {
  int e = op.phase;
  for (int p = 0; p < op.ndim; ++p)
    if ((P >> op.perm[p]) & 1u) e ^= __builtin_popcount(P & op.kmask[p]) & 1;
  const int n = __builtin_popcount(P & op.rev_mask);
  e ^= ((n * (n - 1)) >> 1) & 1;
  e ^= __builtin_popcount(P & op.flip_mask) & 1;
  return e & 1;
}

static std::shared_ptr<DotPlan> build_plan(const Tensor& A, const Tensor& B, const std::vector<int>& axa,
                                           const std::vector<int>& axb, int conv, int gemm, hipStream_t s) {
  const int sym = A.sym();
  const int na = A.ndim(), nb = B.ndim(), k = (int)axa.size();
  std::vector<int> isa(na, 0), isb(nb, 0);
  for (int t = 0; t < k; ++t) {
    if (axa[t] < 0 || axa[t] >= na || axb[t] < 0 || axb[t] >= nb) fail(FTN_EINVAL, "axis out of range");
    if (isa[axa[t]] || isb[axb[t]]) fail(FTN_EINVAL, "repeated axis");
    isa[axa[t]] = isb[axb[t]] = 1;
  }
  std::vector<int> fa, fb;
  for (int i = 0; i < na; ++i)
    if (!isa[i]) fa.push_back(i);
  for (int i = 0; i < nb; ++i)
    if (!isb[i]) fb.push_back(i);
  if ((int)fa.size() + (int)fb.size() > MAXD) fail(FTN_EINVAL, "result would have more than 16 legs");
  // common sectors of each contracted pair
  std::vector<std::vector<Q>> kq(k);
  std::vector<std::vector<int64_t>> kd(k);
  std::vector<std::vector<int32_t>> kmapA(k), kmapB(k);
  std::vector<int> kdual(k);
  for (int t = 0; t < k; ++t) {
    const Leg& la = A.legs()[axa[t]];
    const Leg& lb = B.legs()[axb[t]];
    if (la.dual == lb.dual) fail(FTN_ECHARGE, "contracted legs must have opposite duals");
    kmapA[t].assign(la.nsect(), -1);
    kmapB[t].assign(lb.nsect(), -1);
    for (int sa = 0; sa < la.nsect(); ++sa) {
      int sb = lb.find(la.q[sa]);
      if (sb < 0) continue;
      if (lb.d[sb] != la.d[sa]) fail(FTN_ECHARGE, "sector dimension mismatch on a contracted bond");
      kmapA[t][sa] = kmapB[t][sb] = (int32_t)kq[t].size();
      kq[t].push_back(la.q[sa]);
      kd[t].push_back(la.d[sa]);
    }
    kdual[t] = la.dual;
  }
  auto leg_tabs = [&](const Tensor& T, const std::vector<int>& legs, std::vector<std::vector<Q>>& qs,
                      std::vector<std::vector<int64_t>>& ds, std::vector<int>& du) {
    for (int l : legs) {
      qs.push_back(T.legs()[l].q);
      ds.push_back(T.legs()[l].d);
      du.push_back(T.legs()[l].dual);
    }
  };
  std::vector<std::vector<Q>> rq, cq;
  std::vector<std::vector<int64_t>> rd, cd;
  std::vector<int> rdu, cdu;
  leg_tabs(A, fa, rq, rd, rdu);
  leg_tabs(B, fb, cq, cd, cdu);
  Combos R = combos(sym, rq, rd, rdu);
  Combos Cc = combos(sym, cq, cd, cdu);
  Combos K = combos(sym, kq, kd, kdual);
  const Q sA = A.total(), sB = B.total();
  // groups by row charge, in order of first appearance
  std::vector<Q> gQ;
  std::vector<int32_t> rgroup(R.q.size(), -1);
  for (size_t r = 0; r < R.q.size(); ++r) {
    Q Qg = q_add(sym, sA, q_neg(sym, R.q[r]));
    int g = -1;
    for (size_t i = 0; i < gQ.size(); ++i)
      if (q_eq(gQ[i], Qg)) g = (int)i;
    if (g < 0) {
      g = (int)gQ.size();
      gQ.push_back(Qg);
    }
    rgroup[r] = g;
  }
  const int G = (int)gQ.size();
  std::vector<int64_t> M(G, 0), Kg(G, 0), N(G, 0);
  std::vector<int32_t> rlocal(R.q.size()), clocal(Cc.q.size(), -1), cgroup(Cc.q.size(), -1);
  std::vector<int32_t> nrc(G, 0), ncc(G, 0);
  std::vector<int64_t> roff(R.q.size()), coff(Cc.q.size(), 0), kpos(K.q.size(), 0);
  for (size_t r = 0; r < R.q.size(); ++r) {
    int g = rgroup[r];
    roff[r] = M[g];
    M[g] += R.d[r];
    rlocal[r] = nrc[g]++;
  }
  for (size_t c = 0; c < Cc.q.size(); ++c) {
    for (int g = 0; g < G; ++g) {
      if (q_eq(Cc.q[c], q_add(sym, sB, gQ[g]))) {
        cgroup[c] = g;
        coff[c] = N[g];
        N[g] += Cc.d[c];
        clocal[c] = ncc[g]++;
        break;
      }
    }
  }
  for (size_t kk = 0; kk < K.q.size(); ++kk) {
    for (int g = 0; g < G; ++g) {
      if (q_eq(K.q[kk], gQ[g])) {
        kpos[kk] = Kg[g];
        Kg[g] += K.d[kk];
        break;
      }
    }
  }
  // A in place. Let A's contracted legs be one run c0 .. c0+k-1 in their
  // original order, and let every charge group hold a single contracted sector
  // combination. A block of row combination r, with P entries over the free legs
  // before the run, Kd over the run and S over the free legs after it, is stored
  // as [P][Kd][S]. Its rows of the group's fused matrix (row p S + s, column k)
  // are then, for each p, the transpose of the Kd x S row-major matrix at
  // p Kd S; without free legs after the run (S = 1) the block is itself the
  // P x Kd row-major slab. Moving the run behind the S legs is the only
  // exchange of legs in A's permute, so its sign (Eq. standardcontract gives A
  // no other) is one per block: (-1)^(parity of the run x parity of the S legs).
  // The product then reads A in place, as one GEMM group per row combination
  // (per p when S > 1, transposed, its sign carried by the group), and A's
  // permute and temporary are skipped. Groups shorter than a tile pad the
  // product, so the fused copy stays when the split adds more than 1/8 of
  // padded rows (or more than 2^16 groups).
  const int nf = (int)fa.size();
  const int c0 = k > 0 ? axa[0] : 0;
  bool direct = k > 0;
  for (int t = 0; direct && t < k; ++t) direct = axa[t] == c0 + t;
  const bool trail = c0 + k < na;  // free legs after the run: transposed groups
  std::vector<int64_t> kofg(G, -1), ablk(R.q.size(), -1), apre(R.q.size(), 1), asuf(R.q.size(), 1);
  std::vector<int32_t> aneg(R.q.size(), 0);
  if (direct) {
    std::vector<int> nkg(G, 0);
    for (size_t kk = 0; kk < K.q.size(); ++kk)
      for (int g = 0; g < G; ++g)
        if (q_eq(K.q[kk], gQ[g])) {
          ++nkg[g];
          kofg[g] = (int64_t)kk;
          break;
        }
    for (int g = 0; direct && g < G; ++g) direct = N[g] == 0 || M[g] == 0 || nkg[g] <= 1;
  }
  if (direct) {
    const Structure& AS = A.S();
    std::vector<int> order(fa);
    order.insert(order.end(), axa.begin(), axa.end());
    const SignOp aop = make_signop(na, order.data(), nf, k);
    for (int64_t b = 0; b < AS.nblocks; ++b) {
      const int32_t* key = &AS.keys[b * na];
      int64_t r = 0, kk = 0;
      bool ok = true;
      for (int i = 0; i < nf; ++i) r = r * A.legs()[fa[i]].nsect() + key[fa[i]];
      for (int t = 0; t < k; ++t) {
        const int32_t c = kmapA[t][key[c0 + t]];
        ok = ok && c >= 0;
        kk = kk * (int64_t)kq[t].size() + (c < 0 ? 0 : c);
      }
      if (!ok || kk != kofg[rgroup[r]]) continue;
      ablk[r] = b;
      for (int i = 0; i < c0; ++i) apre[r] *= AS.shapes[b * na + i];
      for (int i = c0 + k; i < na; ++i) asuf[r] *= AS.shapes[b * na + i];
      aneg[r] = host_sign_bit(aop, AS.parmask[b]);
    }
    // (a group without contracted combinations, K = 0, stays whole: its
    // product writes zeros and reads no A)
    int64_t rows_f = 0, rows_d = 0, nsub = 0;
    for (int g = 0; g < G; ++g)
      if (N[g] > 0 && M[g] > 0) {
        rows_f += cdiv(M[g], 128) * 128;
        if (Kg[g] == 0) rows_d += cdiv(M[g], 128) * 128;
      }
    for (size_t r = 0; direct && r < R.q.size(); ++r) {
      const int g = rgroup[r];
      if (N[g] == 0 || M[g] == 0 || Kg[g] == 0) continue;
      direct = ablk[r] >= 0;
      if (trail) {
        rows_d += apre[r] * (cdiv(asuf[r], 128) * 128);
        nsub += apre[r];
      } else {
        rows_d += cdiv(R.d[r], 128) * 128;
        nsub += 1;
      }
    }
    direct = direct && 8 * rows_d <= 9 * rows_f && nsub <= (1 << 16);
  }
  // buffers: A~ groups, B~ groups; groups without columns are dropped
  auto P = std::make_shared<DotPlan>();
  std::vector<int64_t> abase(G, -1), bbase(G, -1);
  for (int g = 0; g < G; ++g) {
    if (N[g] == 0) continue;
    abase[g] = P->asz;
    P->asz += M[g] * Kg[g];
    bbase[g] = P->bsz;
    P->bsz += Kg[g] * N[g];
  }
  // output structure
  std::vector<Leg> clegs;
  for (int l : fa) clegs.push_back(A.legs()[l]);
  for (int l : fb) clegs.push_back(B.legs()[l]);
  P->cst = get_structure(sym, clegs, q_add(sym, sA, sB), s);
  // per free combo tables
  std::vector<int64_t> abase_r(R.q.size()), amul_r(R.q.size(), 1), aext_r(R.q.size());
  for (size_t r = 0; r < R.q.size(); ++r) {
    int g = rgroup[r];
    abase_r[r] = abase[g] < 0 ? -1 : abase[g] + roff[r] * Kg[g];
    aext_r[r] = Kg[g];
  }
  std::vector<int64_t> bbase_c(Cc.q.size()), bmul_c(Cc.q.size()), bext_c(Cc.q.size());
  for (size_t c = 0; c < Cc.q.size(); ++c) {
    int g = cgroup[c];
    bbase_c[c] = (g < 0 || bbase[g] < 0) ? -1 : bbase[g] + coff[c];
    bmul_c[c] = g < 0 ? 0 : N[g];
    bext_c[c] = g < 0 ? 1 : N[g];
  }
  // side descriptors (mixed radix over sector indices)
  auto side = [&](const Tensor& T, const std::vector<int>& f, const std::vector<int>& ax,
                  const std::vector<std::vector<int32_t>>& kmap, std::vector<int32_t>& kflat) {
    DotSide d;
    std::memset(&d, 0, sizeof(d));
    d.n = T.ndim();
    d.nf = (int)f.size();
    d.nc = (int)ax.size();
    int64_t m = 1;
    for (int i = d.nf - 1; i >= 0; --i) {
      d.fpos[i] = f[i];
      d.fmul[i] = m;
      m *= T.legs()[f[i]].nsect();
    }
    m = 1;
    for (int t = d.nc - 1; t >= 0; --t) {
      d.cpos[t] = ax[t];
      d.cmul[t] = m;
      m *= (int64_t)kq[t].size();
    }
    for (int t = 0; t < d.nc; ++t) {
      d.kbase[t] = (int)kflat.size();
      kflat.insert(kflat.end(), kmap[t].begin(), kmap[t].end());
    }
    return d;
  };
  std::vector<int32_t> kfa, kfb;
  DotSide da = side(A, fa, axa, kmapA, kfa);
  DotSide db = side(B, fb, axb, kmapB, kfb);
  if (kfa.empty()) kfa.push_back(0);
  if (kfb.empty()) kfb.push_back(0);
  if (kpos.empty()) kpos.push_back(0);
  // device tasks for A and B
  {
    DBuf<int32_t> dkm = to_device(kfa, s);
    DBuf<int64_t> d1 = to_device(abase_r, s), d2 = to_device(amul_r, s), d3 = to_device(aext_r, s);
    DBuf<int64_t> dk = to_device(kpos, s);
    std::vector<int> order(fa);
    order.insert(order.end(), axa.begin(), axa.end());
    P->pa.op = make_signop(na, order.data(), (int)fa.size(), k);
    P->pa.tasks = persist<PermTask>(A.nblocks());
    if (A.nblocks())
      LAUNCH(k_dot_tasks, dim3((unsigned)cdiv(A.nblocks(), 128)), dim3(128), 0, s, da,
                         A.S().d_keys.p, A.nblocks(), dkm.p, d1.p, d2.p, d3.p, dk.p, P->pa.tasks.p);
    HIPC(hipGetLastError());
    perm_plan_build(P->pa, A.S(), s);
  }
  {
    DBuf<int32_t> dkm = to_device(kfb, s);
    DBuf<int64_t> d1 = to_device(bbase_c, s), d2 = to_device(bmul_c, s), d3 = to_device(bext_c, s);
    DBuf<int64_t> dk = to_device(kpos, s);
    std::vector<int> order(axb);
    order.insert(order.end(), fb.begin(), fb.end());
    SignOp op = make_signop(nb, order.data(), k, (int)fb.size());
    for (int t = 0; t < k; ++t) op.rev_mask |= 1u << axb[t];
    if (conv == FTN_LOCAL)
      for (int t = 0; t < k; ++t)
        if (A.legs()[axa[t]].dual == 0) op.flip_mask |= 1u << axb[t];
    P->pb.op = op;
    P->pb.tasks = persist<PermTask>(B.nblocks());
    if (B.nblocks())
      LAUNCH(k_dot_tasks, dim3((unsigned)cdiv(B.nblocks(), 128)), dim3(128), 0, s, db,
                         B.S().d_keys.p, B.nblocks(), dkm.p, d1.p, d2.p, d3.p, dk.p, P->pb.tasks.p);
    HIPC(hipGetLastError());
    perm_plan_build(P->pb, B.S(), s);
  }
  // scatter tables + GEMM groups
  std::vector<int64_t> rcs, ccs, ccd, gboff(G, 0);
  std::vector<int32_t> gncc(G, 0);
  std::vector<GemmGroup> groups, dgroups;
  std::vector<int64_t> drow;  // per in-place group: its row table entry
  int64_t boff_n = 0;
  for (int g = 0; g < G; ++g) {
    // a group without rows or columns writes nothing (and the GEMM plan
    // drops it, so the charge list must skip it too)
    if (N[g] == 0 || M[g] == 0) continue;
    GemmGroup gg;
    std::memset(&gg, 0, sizeof(gg));
    gg.M = M[g];
    gg.N = N[g];
    gg.K = Kg[g];
    gg.a_off = abase[g];
    gg.b_off = bbase[g];
    gg.lda = std::max<int64_t>(Kg[g], 1);
    gg.ldb = N[g];
    gg.scatter = 1;
    gg.rc_base = (int64_t)rcs.size();
    gg.cc_base = (int64_t)ccs.size();
    for (size_t r = 0; r < R.q.size(); ++r)
      if (rgroup[r] == g) rcs.push_back(roff[r]);
    for (size_t c = 0; c < Cc.q.size(); ++c)
      if (cgroup[c] == g) {
        ccs.push_back(coff[c]);
        ccd.push_back(Cc.d[c]);
      }
    gg.nrc = nrc[g];
    gg.ncc = ncc[g];
    gg.boff_base = boff_n;
    P->gq.push_back(gQ[g]);
    gboff[g] = boff_n;
    gncc[g] = ncc[g];
    if (direct && Kg[g] == 0) {
      GemmGroup d = gg;
      d.a_off = 0;
      d.lda = 1;
      dgroups.push_back(d);
      drow.push_back(INT64_MIN);  // keeps the group's own row table
    } else if (direct)
      for (size_t r = 0; r < R.q.size(); ++r) {
        if (rgroup[r] != g) continue;
        const int64_t ps = trail ? apre[r] : 1;
        for (int64_t q = 0; q < ps; ++q) {
          GemmGroup d = gg;
          d.M = trail ? asuf[r] : R.d[r];
          d.a_off = A.S().offsets[ablk[r]] + q * Kg[g] * asuf[r];
          d.transA = trail ? 1 : 0;
          d.lda = trail ? asuf[r] : Kg[g];
          d.neg = aneg[r];
          d.nrc = 1;  // one row table entry: row m of the group is row m + q S of block r
          d.boff_base = boff_n + (int64_t)rlocal[r] * ncc[g];
          dgroups.push_back(d);
          drow.push_back(-q * asuf[r]);
        }
      }
    boff_n += (int64_t)nrc[g] * ncc[g];
    groups.push_back(gg);
  }
  for (size_t i = 0; i < dgroups.size(); ++i)
    if (drow[i] != INT64_MIN) {
      dgroups[i].rc_base = (int64_t)rcs.size();
      rcs.push_back(drow[i]);
    }
  P->rc_start = persist_upload(rcs, s);
  P->cc_start = persist_upload(ccs, s);
  P->cc_dim = persist_upload(ccd, s);
  P->boff = persist<int64_t>(std::max<int64_t>(boff_n, 1));
  HIPC(hipMemsetAsync(P->boff.p, 0xff, std::max<int64_t>(boff_n, 1) * sizeof(int64_t), s));  // -1
  {
    const Structure& CS = *P->cst;
    BoffArgs ba;
    std::memset(&ba, 0, sizeof(ba));
    ba.n = CS.ndim;
    ba.nfa = (int)fa.size();
    ba.nfb = (int)fb.size();
    int64_t m = 1;
    for (int i = ba.nfa - 1; i >= 0; --i) {
      ba.fmul[i] = m;
      m *= A.legs()[fa[i]].nsect();
    }
    m = 1;
    for (int i = ba.nfb - 1; i >= 0; --i) {
      ba.gmul[i] = m;
      m *= B.legs()[fb[i]].nsect();
    }
    DBuf<int32_t> drg = to_device(rgroup, s), drl = to_device(rlocal, s), dcl = to_device(clocal, s);
    DBuf<int64_t> dgb = to_device(gboff, s);
    DBuf<int32_t> dgn = to_device(gncc, s);
    if (CS.nblocks) {
      if (CS.ndim == 0) {
        // scalar output: one block at offset 0
        std::vector<int64_t> z(1, 0);
        h2d(P->boff.p, z.data(), 8, s);
      } else {
        LAUNCH(k_dot_boff, dim3((unsigned)cdiv(CS.nblocks, 128)), dim3(128), 0, s, ba,
                           CS.d_keys.p, CS.d_offsets.p, CS.nblocks, drg.p, drl.p, dcl.p, dgb.p, dgn.p,
                           P->boff.p);
        HIPC(hipGetLastError());
      }
    }
  }
  P->sc.rc_start = P->rc_start.p;
  P->sc.cc_start = P->cc_start.p;
  P->sc.cc_dim = P->cc_dim.p;
  P->sc.boff = P->boff.p;
  gemm_plan(P->gp, groups, gemm, s, true);
  P->direct_a = direct && !dgroups.empty();
  if (P->direct_a) gemm_plan(P->gpd, dgroups, gemm, s, true);
  P->flops = gemm_flops(groups);
  // cached plans may be used on other streams: finish building them here
  HIPC(hipStreamSynchronize(s));
  return P;
}

static std::string plan_key(const Tensor& a, const Tensor& b, const std::vector<int>& axa,
                            const std::vector<int>& axb, int conv, int gemm) {
  std::string key = a.st->skey + "|" + b.st->skey + "|";
  for (int x : axa) key += std::to_string(x) + ",";
  key += "|";
  for (int x : axb) key += std::to_string(x) + ",";
  key += "|" + std::to_string(conv) + "|" + std::to_string(gemm);
  return key;
}

std::shared_ptr<DotPlan> dot_plan_lookup(const Tensor& a, const Tensor& b, const std::vector<int>& axa,
                                         const std::vector<int>& axb, int conv, int gemm) {
  const std::string key = plan_key(a, b, axa, axb, conv, gemm);
  std::lock_guard<std::mutex> g(g_plan_mu);
  auto it = g_plans.find(key);
  return it == g_plans.end() ? nullptr : it->second;
}

std::shared_ptr<DotPlan> dot_plan(const Tensor& a, const Tensor& b, const std::vector<int>& axa,
                                  const std::vector<int>& axb, int conv, int gemm, hipStream_t s) {
  const std::string key = plan_key(a, b, axa, axb, conv, gemm);
  {
    std::lock_guard<std::mutex> g(g_plan_mu);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) return it->second;
  }
  auto P = build_plan(a, b, axa, axb, conv, gemm, s);
  std::lock_guard<std::mutex> g(g_plan_mu);
  if (g_plans.size() > 4096) g_plans.clear();
  g_plans.emplace(key, P);
  return P;
}

DotPlanView dot_plan_view(const DotPlan& p) {
  DotPlanView v;
  v.groups = p.gp.host;
  v.gq = p.gq;
  v.pa = &p.pa;
  v.pb = &p.pb;
  v.asz = p.asz;
  v.bsz = p.bsz;
  return v;
}

std::unique_ptr<Tensor> op_ftensordot(const Tensor& a, const Tensor& b, const std::vector<int>& axa,
                                      const std::vector<int>& axb, int conv, int gemm, hipStream_t s,
                                      double* flops) {
  if (a.sym() != b.sym()) fail(FTN_EINVAL, "symmetry mismatch");
  if (a.dtype != b.dtype) fail(FTN_ENOTSUP, "operands must have the same dtype");
  if (axa.size() != axb.size()) fail(FTN_EINVAL, "axes length mismatch");
  if (conv != FTN_LOCAL && conv != FTN_GLOBAL) fail(FTN_EINVAL, "unknown convention");
  if (gemm == FTN_GEMM_F64 && a.dtype != FTN_F64) fail(FTN_ENOTSUP, "FP64 GEMM needs FP64 tensors");
  if (gemm != FTN_GEMM_F64 && a.dtype != FTN_F32) fail(FTN_ENOTSUP, "FP32 / split-BF16 GEMM needs FP32 tensors");
  std::shared_ptr<DotPlan> P = dot_plan(a, b, axa, axb, conv, gemm, s);
  auto out = make_tensor(P->cst, a.dtype, s, false);
  if (flops) *flops = P->flops;
  if (out->size() == 0) return out;
  const size_t es = a.esize();
  void* At = (P->asz && !P->direct_a) ? dmalloc(P->asz * es, s) : nullptr;
  void* Bt = P->bsz ? dmalloc(P->bsz * es, s) : nullptr;
  try {
    if (!P->direct_a) run_perm(0, a.S(), a.dtype, P->pa, a.data, At, s);
    run_perm(0, b.S(), b.dtype, P->pb, b.data, Bt, s);
    if (P->direct_a)
      run_gemm(P->gpd, a.dtype, a.data, Bt, out->data, &P->sc, s);
    else
      run_gemm(P->gp, a.dtype, At, Bt, out->data, &P->sc, s);
  } catch (...) {
    dfree(At, s);
    dfree(Bt, s);
    throw;
  }
  dfree(At, s);
  dfree(Bt, s);
  return out;
}

void op_ftensordot_into(const Tensor& a, const Tensor& b, const std::vector<int>& axa,
                        const std::vector<int>& axb, int conv, int gemm, hipStream_t s, void* out,
                        int64_t out_elems, char* scratch, size_t scratch_bytes) {
  if (a.sym() != b.sym()) fail(FTN_EINVAL, "symmetry mismatch");
  if (a.dtype != b.dtype) fail(FTN_ENOTSUP, "operands must have the same dtype");
  if (axa.size() != axb.size()) fail(FTN_EINVAL, "axes length mismatch");
  if (conv != FTN_LOCAL && conv != FTN_GLOBAL) fail(FTN_EINVAL, "unknown convention");
  if (gemm == FTN_GEMM_F64 && a.dtype != FTN_F64) fail(FTN_ENOTSUP, "FP64 GEMM needs FP64 tensors");
  if (gemm != FTN_GEMM_F64 && a.dtype != FTN_F32) fail(FTN_ENOTSUP, "FP32 / split-BF16 GEMM needs FP32 tensors");
  std::shared_ptr<DotPlan> P = dot_plan_lookup(a, b, axa, axb, conv, gemm);
  if (!P)
    fail(FTN_ENOTSUP,
         "no cached plan for this contraction: call ftn_ftensordot once with operands of the same structures, "
         "axes, convention and GEMM form");
  if (out_elems != P->cst->size)
    fail(FTN_EINVAL, "output buffer holds " + std::to_string(out_elems) + " entries, the contraction gives " +
                         std::to_string(P->cst->size));
  if (P->cst->size == 0) return;
  if (!out) fail(FTN_EINVAL, "null output buffer");
  const size_t es = a.esize();
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  const GemmPlan& gp = P->direct_a ? P->gpd : P->gp;
  const size_t ba = P->direct_a ? 0 : up(P->asz * es), bb = up(P->bsz * es), bw = up(gp.ws_elems * es);
  if (ba + bb + bw > scratch_bytes)
    fail(FTN_EINVAL, "contraction needs " + std::to_string(ba + bb + bw) + " bytes of temporaries, the scratch buffer holds " +
                         std::to_string(scratch_bytes));
  char* At = scratch;
  char* Bt = scratch + ba;
  char* W = scratch + ba + bb;
  if (!P->direct_a) run_perm(0, a.S(), a.dtype, P->pa, a.data, At, s);
  run_perm(0, b.S(), b.dtype, P->pb, b.data, Bt, s);
  run_gemm(gp, a.dtype, P->direct_a ? a.data : At, Bt, out, &P->sc, s, 1.0, 0.0, W);
}

// ---------------------------------------------------------------------------
// Adjoint of the contraction (the map is bilinear, Eq. standardcontract):
// with the signed fused matrices A~_Q, B~_Q and C_Q = A~_Q B~_Q,
//   dA~_Q = dC_Q B~_Q^T,  dB~_Q = A~_Q^T dC_Q,
// and dA, dB are the signed permutes run backwards (a signed permutation is
// inverted by its transpose, which carries the same signs).

// largest i in [0, n) with v[i] <= x
__device__ inline int upper_idx(const int64_t* v, int n, int64_t x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (v[mid] <= x)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// dC (block layout of C) -> fused matrices F_g (M_g x N_g at f_off[g])
template <typename T>
__global__ void k_gather_fused(const GemmGroup* __restrict__ groups, int ng, const int64_t* __restrict__ f_off,
                               int64_t total, GemmScatter sc, const T* __restrict__ dC, T* __restrict__ F) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int g = upper_idx(f_off, ng, e);
  const GemmGroup G = groups[g];
  const int64_t loc = e - f_off[g];
  const int64_t m = loc / G.N, n = loc % G.N;
  const int rfi = upper_idx(sc.rc_start + G.rc_base, G.nrc, m);
  const int cgj = upper_idx(sc.cc_start + G.cc_base, G.ncc, n);
  const int64_t rlr = m - sc.rc_start[G.rc_base + rfi];
  const int64_t clc = n - sc.cc_start[G.cc_base + cgj];
  const int64_t cnd = sc.cc_dim[G.cc_base + cgj];
  const int64_t bo = sc.boff[G.boff_base + (int64_t)rfi * G.ncc + cgj];
  F[e] = bo >= 0 ? dC[bo + rlr * cnd + clc] : T(0);
}

int64_t dot_gather_output(const DotPlan& P, const Tensor& c, double* F, std::vector<int64_t>& f_off,
                          hipStream_t s) {
  if (c.st->skey != P.cst->skey) fail(FTN_EINVAL, "tensor does not have the structure of the contraction's output");
  if (c.dtype != FTN_F64) fail(FTN_ENOTSUP, "FP64 only");
  const std::vector<GemmGroup>& groups = P.gp.host;
  f_off.assign(groups.size(), 0);
  int64_t ftot = 0;
  for (size_t g = 0; g < groups.size(); ++g) {
    f_off[g] = ftot;
    ftot += groups[g].M * groups[g].N;
  }
  if (!F || ftot == 0) return ftot;
  if (c.size() == 0) {
    HIPC(hipMemsetAsync(F, 0, ftot * 8, s));
    return ftot;
  }
  DBuf<int64_t> dfo = to_device(f_off, s);
  LAUNCH(k_gather_fused<double>, dim3((unsigned)cdiv(ftot, 256)), dim3(256), 0, s, P.gp.groups.p, (int)groups.size(),
         dfo.p, ftot, P.sc, (const double*)c.data, F);
  return ftot;
}

void op_ftensordot_backward(const Tensor& a, const Tensor& b, const Tensor& dc, const std::vector<int>& axa,
                            const std::vector<int>& axb, int conv, int gemm, hipStream_t s,
                            std::unique_ptr<Tensor>& da, std::unique_ptr<Tensor>& db) {
  if (a.sym() != b.sym() || dc.sym() != a.sym()) fail(FTN_EINVAL, "symmetry mismatch");
  if (a.dtype != b.dtype || dc.dtype != a.dtype) fail(FTN_ENOTSUP, "operands must have the same dtype");
  if (axa.size() != axb.size()) fail(FTN_EINVAL, "axes length mismatch");
  if (conv != FTN_LOCAL && conv != FTN_GLOBAL) fail(FTN_EINVAL, "unknown convention");
  if (gemm == FTN_GEMM_F64 && a.dtype != FTN_F64) fail(FTN_ENOTSUP, "FP64 GEMM needs FP64 tensors");
  if (gemm != FTN_GEMM_F64 && a.dtype != FTN_F32) fail(FTN_ENOTSUP, "FP32 / split-BF16 GEMM needs FP32 tensors");
  std::shared_ptr<DotPlan> P = dot_plan(a, b, axa, axb, conv, gemm, s);
  if (dc.st->skey != P->cst->skey) fail(FTN_EINVAL, "dC does not have the structure of the contraction's output");
  da = make_tensor(a.st, a.dtype, s, true);
  db = make_tensor(b.st, b.dtype, s, true);
  const std::vector<GemmGroup>& groups = P->gp.host;
  if (groups.empty() || dc.size() == 0) return;
  const size_t es = a.esize();
  std::vector<int64_t> f_off(groups.size());
  int64_t ftot = 0;
  for (size_t g = 0; g < groups.size(); ++g) {
    f_off[g] = ftot;
    ftot += groups[g].M * groups[g].N;
  }
  DBuf<char> At(P->asz * es, s), Bt(P->bsz * es, s), dAt(P->asz * es, s), dBt(P->bsz * es, s), F(ftot * es, s);
  if (P->asz) HIPC(hipMemsetAsync(dAt.p, 0, P->asz * es, s));
  if (P->bsz) HIPC(hipMemsetAsync(dBt.p, 0, P->bsz * es, s));
  run_perm(0, a.S(), a.dtype, P->pa, a.data, At.p, s);
  run_perm(0, b.S(), b.dtype, P->pb, b.data, Bt.p, s);
  {
    DBuf<int64_t> dfo = to_device(f_off, s);
    const dim3 grid((unsigned)cdiv(ftot, 256)), block(256);
    if (a.dtype == FTN_F64)
      LAUNCH(k_gather_fused<double>, grid, block, 0, s, P->gp.groups.p, (int)groups.size(), dfo.p, ftot, P->sc,
             (const double*)dc.data, (double*)F.p);
    else
      LAUNCH(k_gather_fused<float>, grid, block, 0, s, P->gp.groups.p, (int)groups.size(), dfo.p, ftot, P->sc,
             (const float*)dc.data, (float*)F.p);
  }
  std::vector<GemmGroup> ga, gb;
  for (size_t g = 0; g < groups.size(); ++g) {
    const GemmGroup& G = groups[g];
    GemmGroup x;
    std::memset(&x, 0, sizeof(x));
    if (G.K > 0) {  // dA~ = F B~^T (M x K)
      x.M = G.M;
      x.N = G.K;
      x.K = G.N;
      x.a_off = f_off[g];
      x.lda = G.N;
      x.b_off = G.b_off;
      x.ldb = G.ldb;
      x.transB = 1;
      x.c_off = G.a_off;
      x.ldc = G.lda;
      ga.push_back(x);
      std::memset(&x, 0, sizeof(x));  // dB~ = A~^T F (K x N)
      x.M = G.K;
      x.N = G.N;
      x.K = G.M;
      x.a_off = G.a_off;
      x.lda = G.lda;
      x.transA = 1;
      x.b_off = f_off[g];
      x.ldb = G.N;
      x.c_off = G.b_off;
      x.ldc = G.ldb;
      gb.push_back(x);
    }
  }
  if (!ga.empty()) {
    run_grouped_gemm(gemm, a.dtype, ga, F.p, Bt.p, dAt.p, nullptr, s);
    run_grouped_gemm(gemm, a.dtype, gb, At.p, F.p, dBt.p, nullptr, s);
  }
  run_perm(1, a.S(), a.dtype, P->pa, dAt.p, da->data, s);
  run_perm(1, b.S(), b.dtype, P->pb, dBt.p, db->data, s);
}

}  // namespace ftn
