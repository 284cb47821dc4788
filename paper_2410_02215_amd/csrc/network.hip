// Network contraction along an SSA path (Fig. 1; Secs. II.C-II.E, III).
//
// Networks are contracted in the locally ordered form (Sec. II.E): every
// step is a pairwise ftensordot with the local convention. A network given
// with global positions (Sec. II.D, Eq. fermionictn) is translated once: the
// positions define a DAG whose arrows run from later to earlier tensors, so
// the duals of every bond whose '-' end (arrow head) sits on the later tensor
// are relabelled (a change of charge labels only; in the global convention
// duals carry no sign), and odd tensors receive a size-1 odd dummy leg in
// front. At the end the dummy legs are sorted by position and the phase
// (-1)^{m(m-1)/2} of having prepended them is removed.
//
// Approximate contraction compresses as early as possible (Sec. III): after
// each step the bonds the new tensor shares with one neighbour are fused
// (Sec. IV.A) and each such bond larger than chi is compressed. Every
// intermediate is rescaled by a power of two (exact), kept in an exponent.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "common.h"

namespace ftn {
Tensor* handle_tensor(ftn_tensor_t h);
ftn_tensor_t make_handle(std::unique_ptr<Tensor> t);
}  // namespace ftn

using namespace ftn;

namespace {
struct Label {
  int kind;  // 0 bond (a = bond id), 1 open (a = tensor, b = leg), 2 dummy (a = tensor)
  int a, b;
  bool operator==(const Label& o) const { return kind == o.kind && a == o.a && b == o.b; }
};
}  // namespace

struct ftn_net {
  int n = 0;
  int nbonds = 0;
  std::vector<std::unique_ptr<Tensor>> T;  // local form, dummies prepended
  std::vector<std::vector<Label>> lab;
  std::vector<int> dummy_rank;  // -1 for even tensors
};

template <typename F>
static int guarded_net(F&& f) {
  try {
    f();
    return FTN_OK;
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return FTN_EINVAL;
  } catch (...) {
    set_last_error("unknown internal error");
    return FTN_EINVAL;
  }
}

static std::unique_ptr<Tensor> with_dummy(const Tensor& t, hipStream_t s) {
  const int sym = t.sym();
  Leg d;
  d.dual = 0;
  d.q.push_back(q_neg(sym, t.total()));
  d.d.push_back(1);
  std::vector<Leg> legs;
  legs.push_back(d);
  for (auto& l : t.legs()) legs.push_back(l);
  if (legs.size() > (size_t)MAXD) fail(FTN_EINVAL, "odd tensor with 16 legs cannot take a dummy leg");
  auto st = get_structure(sym, legs, Q{0, 0}, s);
  return share_tensor(t, st);
}

extern "C" int ftn_net_create(int ntensors, const ftn_tensor_t* tensors, int nbonds, const int32_t* bond_ends,
                              ftn_conv conv, const int32_t* positions, ftn_net_t* out) {
  return guarded_net([&] {
    if (!out || ntensors < 1 || !tensors || nbonds < 0 || (nbonds && !bond_ends))
      fail(FTN_EINVAL, "bad network arguments");
    if (conv != FTN_LOCAL && conv != FTN_GLOBAL) fail(FTN_EINVAL, "unknown convention");
    if (conv == FTN_GLOBAL && !positions) fail(FTN_EINVAL, "the global convention needs positions");
    hipStream_t s = nullptr;
    auto net = std::make_unique<ftn_net>();
    net->n = ntensors;
    net->nbonds = nbonds;
    int sym = -1;
    for (int t = 0; t < ntensors; ++t) {
      Tensor* x = handle_tensor(tensors[t]);
      if (!x) fail(FTN_EINVAL, "null tensor in network");
      if (sym < 0) sym = x->sym();
      if (x->sym() != sym) fail(FTN_EINVAL, "mixed symmetries in one network");
      net->T.push_back(share_tensor(*x, x->st));
      std::vector<Label> L;
      for (int l = 0; l < x->ndim(); ++l) L.push_back(Label{1, t, l});
      net->lab.push_back(L);
    }
    if (positions) {
      std::vector<int> chk(positions, positions + ntensors);
      std::sort(chk.begin(), chk.end());
      for (int i = 1; i < ntensors; ++i)
        if (chk[i] == chk[i - 1]) fail(FTN_EINVAL, "positions must be distinct");
    }
    for (int b = 0; b < nbonds; ++b) {
      int t1 = bond_ends[4 * b], l1 = bond_ends[4 * b + 1], t2 = bond_ends[4 * b + 2], l2 = bond_ends[4 * b + 3];
      if (t1 < 0 || t1 >= ntensors || t2 < 0 || t2 >= ntensors || t1 == t2) fail(FTN_EINVAL, "bad bond tensor");
      if (l1 < 0 || l1 >= net->T[t1]->ndim() || l2 < 0 || l2 >= net->T[t2]->ndim()) fail(FTN_EINVAL, "bad bond leg");
      if (net->lab[t1][l1].kind != 1 || net->lab[t2][l2].kind != 1) fail(FTN_EINVAL, "leg used by two bonds");
      const Leg& A = net->T[t1]->legs()[l1];
      const Leg& B = net->T[t2]->legs()[l2];
      if (A.dual == B.dual) fail(FTN_ECHARGE, "bonded legs must have opposite duals");
      net->lab[t1][l1] = Label{0, b, 0};
      net->lab[t2][l2] = Label{0, b, 0};
      if (conv == FTN_GLOBAL) {
        int head = A.dual == 1 ? t1 : t2;
        int other = head == t1 ? t2 : t1;
        if (positions[head] > positions[other]) {
          net->T[t1] = op_flip_dual(*net->T[t1], l1, 0, s);
          net->T[t2] = op_flip_dual(*net->T[t2], l2, 0, s);
        }
      }
    }
    // dummy legs of odd tensors, ranked by position (or index)
    std::vector<int> odd;
    for (int t = 0; t < ntensors; ++t)
      if (net->T[t]->parity()) odd.push_back(t);
    std::sort(odd.begin(), odd.end(), [&](int x, int y) {
      return positions ? positions[x] < positions[y] : x < y;
    });
    net->dummy_rank.assign(ntensors, -1);
    for (size_t r = 0; r < odd.size(); ++r) {
      int t = odd[r];
      net->dummy_rank[t] = (int)r;
      net->T[t] = with_dummy(*net->T[t], s);
      net->lab[t].insert(net->lab[t].begin(), Label{2, t, 0});
    }
    HIPC(hipStreamSynchronize(s));
    *out = net.release();
  });
}

extern "C" int ftn_net_free(ftn_net_t net) {
  return guarded_net([&] { delete net; });
}

static std::vector<int> shared_legs(const std::vector<Label>& a, const std::vector<Label>& b, std::vector<int>& lb) {
  std::vector<std::pair<int, std::pair<int, int>>> v;
  for (int i = 0; i < (int)a.size(); ++i) {
    if (a[i].kind != 0) continue;
    for (int j = 0; j < (int)b.size(); ++j)
      if (b[j] == a[i]) v.push_back({a[i].a, {i, j}});
  }
  std::sort(v.begin(), v.end());
  std::vector<int> la;
  lb.clear();
  for (auto& x : v) {
    la.push_back(x.second.first);
    lb.push_back(x.second.second);
  }
  return la;
}

extern "C" int ftn_contract_network(ftn_net_t net, int nsteps, const int32_t* ssa_path, int64_t chi,
                                    ftn_gemm gemm, ftn_stream_t stream, double* mantissa, int64_t* exp2,
                                    ftn_tensor_t* open_out, int32_t* leg_src, double* stats) {
  return guarded_net([&] {
    if (!net || (nsteps && !ssa_path)) fail(FTN_EINVAL, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    const int n = net->n;
    if (nsteps != n - 1) fail(FTN_EINVAL, "a path over n tensors has n-1 steps");
    std::vector<std::unique_ptr<Tensor>> T;
    std::vector<std::vector<Label>> L;
    for (int t = 0; t < n; ++t) {
      T.push_back(share_tensor(*net->T[t], net->T[t]->st));
      L.push_back(net->lab[t]);
    }
    std::vector<int> alive(n, 1);
    std::vector<int> ssa(n);
    for (int t = 0; t < n; ++t) ssa[t] = t;
    int next_bond = net->nbonds;
    int64_t e2 = 0;
    const bool trace = std::getenv("FTN_TRACE") != nullptr;
    double st[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = 0; k < nsteps; ++k) {
      int i = ssa_path[2 * k], j = ssa_path[2 * k + 1];
      if (i < 0 || j < 0 || i >= (int)ssa.size() || j >= (int)ssa.size() || i == j)
        fail(FTN_EINVAL, "bad SSA id in path step " + std::to_string(k));
      int x = ssa[i], y = ssa[j];
      if (x < 0 || y < 0 || !alive[x] || !alive[y]) fail(FTN_EINVAL, "path uses a consumed tensor");
      std::vector<int> ly;
      std::vector<int> lx = shared_legs(L[x], L[y], ly);
      double fl = 0;
      auto Z = op_ftensordot(*T[x], *T[y], lx, ly, FTN_LOCAL, gemm, s, &fl);
      st[0] += fl;
      std::vector<Label> lz;
      for (int q = 0; q < (int)L[x].size(); ++q)
        if (std::find(lx.begin(), lx.end(), q) == lx.end()) lz.push_back(L[x][q]);
      for (int q = 0; q < (int)L[y].size(); ++q)
        if (std::find(ly.begin(), ly.end(), q) == ly.end()) lz.push_back(L[y][q]);
      int z = (int)T.size();
      T.push_back(std::move(Z));
      L.push_back(lz);
      alive.push_back(1);
      alive[x] = alive[y] = 0;
      T[x].reset();
      T[y].reset();
      ssa[i] = ssa[j] = -1;
      ssa.push_back(z);
      if (chi > 0) {
        // neighbours of z in increasing id order
        std::vector<int> nbs;
        for (int w = 0; w < (int)T.size(); ++w) {
          if (w == z || !alive[w]) continue;
          std::vector<int> tmp;
          if (!shared_legs(L[z], L[w], tmp).empty()) nbs.push_back(w);
        }
        for (int w : nbs) {
          std::vector<int> lw;
          std::vector<int> lzs = shared_legs(L[z], L[w], lw);
          if (lzs.size() > 1) {
            auto Zf = op_fuse(*T[z], lzs, FTN_LOCAL, 0, s);
            auto Wf = op_fuse(*T[w], lw, FTN_LOCAL, 0, s);
            Label nb{0, next_bond++, 0};
            auto relabel = [&](std::vector<Label>& lab, const std::vector<int>& legs) {
              std::vector<Label> rest;
              int pos = 0;
              for (int q = 0; q < (int)lab.size(); ++q) {
                if (std::find(legs.begin(), legs.end(), q) != legs.end()) continue;
                if (q < legs[0]) ++pos;
                rest.push_back(lab[q]);
              }
              rest.insert(rest.begin() + pos, nb);
              lab = rest;
            };
            relabel(L[z], lzs);
            relabel(L[w], lw);
            T[z] = std::move(Zf);
            T[w] = std::move(Wf);
            lzs = shared_legs(L[z], L[w], lw);
          }
          const int64_t dim = T[z]->legs()[lzs[0]].size();
          // a tensor with no allowed block is exactly zero: nothing to truncate
          if (dim > chi && T[z]->size() > 0 && T[w]->size() > 0) {
            CompressResult r = op_compress_bond(*T[z], *T[w], lzs[0], lw[0], chi, 1e-6, FTN_LOCAL, s);
            T[z] = std::move(r.a);
            T[w] = std::move(r.b);
            st[1] += 1;
            st[2] += r.discarded;
            st[3] += r.near_tie ? 1 : 0;
          }
        }
      }
      st[4] = std::max(st[4], (double)T[z]->size());
      if (trace) {
        std::string d;
        for (auto& l : T[z]->legs()) d += std::to_string(l.size()) + (l.dual ? "-" : "+") + " ";
        std::fprintf(stderr, "[ftn] step %d: (%d,%d) -> %d legs [%s] size %lld\n", k, i, j, T[z]->ndim(),
                     d.c_str(), (long long)T[z]->size());
      }
      double m = op_max_abs(*T[z], s);
      if (m > 0 && std::isfinite(m)) {
        int e;
        std::frexp(m, &e);
        scale_inplace(*T[z], std::ldexp(1.0, -e), s);
        e2 += e;
      }
    }
    int fin = -1;
    for (int t = 0; t < (int)T.size(); ++t)
      if (alive[t]) {
        if (fin >= 0) fail(FTN_EINVAL, "path does not contract the network to one tensor");
        fin = t;
      }
    std::unique_ptr<Tensor> F = std::move(T[fin]);
    std::vector<Label> lf = L[fin];
    // dummy legs: sort by rank, drop, remove the prepending phase
    std::vector<int> dpos, others;
    for (int q = 0; q < (int)lf.size(); ++q) (lf[q].kind == 2 ? dpos : others).push_back(q);
    const int m = (int)dpos.size();
    if (m) {
      std::sort(dpos.begin(), dpos.end(),
                [&](int a, int b) { return net->dummy_rank[lf[a].a] < net->dummy_rank[lf[b].a]; });
      std::vector<int> perm(dpos);
      perm.insert(perm.end(), others.begin(), others.end());
      F = op_ftranspose(*F, perm, s);
      const int sym = F->sym();
      Q tot = F->total();
      for (int q = 0; q < m; ++q) {
        const Leg& l = F->legs()[q];
        tot = q_add(sym, tot, q_neg(sym, q_signed(sym, l.dual, l.q[0])));
      }
      std::vector<Leg> rest(F->legs().begin() + m, F->legs().end());
      auto stq = get_structure(sym, rest, tot, s);
      if (stq->size != F->size()) fail(FTN_EINVAL, "internal: dummy legs with several blocks");
      F = share_tensor(*F, stq);
      if ((m * (m - 1) / 2) % 2) F = op_scale(*F, -1.0, s);
      std::vector<Label> nl;
      for (int q : others) nl.push_back(lf[q]);
      lf = nl;
    }
    if (stats)
      for (int q = 0; q < 8; ++q) stats[q] = st[q];
    if (exp2) *exp2 = e2;
    if (F->ndim() == 0) {
      double v = 0.0;
      if (F->size()) {
        if (F->dtype == FTN_F64) {
          HIPC(hipMemcpyAsync(&v, F->data, 8, hipMemcpyDeviceToHost, s));
        } else {
          float f = 0;
          HIPC(hipMemcpyAsync(&f, F->data, 4, hipMemcpyDeviceToHost, s));
          HIPC(hipStreamSynchronize(s));
          v = f;
        }
      }
      HIPC(hipStreamSynchronize(s));
      if (mantissa) *mantissa = v;
      if (open_out) *open_out = nullptr;
    } else {
      if (mantissa) *mantissa = 1.0;
      if (!open_out) fail(FTN_EINVAL, "network has open legs: pass open_out");
      if (leg_src)
        for (int q = 0; q < (int)lf.size(); ++q) {
          leg_src[2 * q] = lf[q].a;
          leg_src[2 * q + 1] = lf[q].b;
        }
      *open_out = make_handle(std::move(F));
    }
  });
}
