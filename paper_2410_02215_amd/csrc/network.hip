// Network contraction along an SSA path (Fig. 1; Secs. II.C-II.E, III).
//
// Networks are contracted in the locally ordered form (Sec. II.E): every
// step is a pairwise ftensordot with the local convention. A network given
// with global positions (Sec. II.D, Eq. fermionictn) is translated once: the
// positions define a DAG whose arrows run from later to earlier tensors, so
// the duals of every bond whose '-' end (arrow head) sits on the later tensor
// are relabelled (a change of charge labels only; in the global convention
// duals carry no sign).
//
// Odd tensors. Sec. II.E gives each odd tensor a size-1 odd dummy leg in
// front, sorts the dummies by the global order at the end and removes the
// phase (-1)^{m(m-1)/2} of having prepended m of them. The dummy legs are not
// materialised here (a boundary of many odd tensors would collect more legs
// than a block key holds); their effect is a sign tracked per tensor. Write
// an intermediate as D_X X, with D_X the product of its dummies in rank order
// and X its body, whose parity is |D_X| mod 2. Contracting D_X X with D_Y Y
// moves D_Y past X, (-1)^{|D_X||D_Y|}, and sorting the merged dummies costs
// the parity of the rank inversions between D_X and D_Y; the body is the
// plain contraction of X and Y. Fusion and compression act on bond legs,
// which never cross a leading dummy, so they are unchanged.
//
// Approximate contraction compresses as early as possible (Sec. III): after
// each step the bonds the new tensor shares with one neighbour are fused
// (Sec. IV.A) and each such bond larger than chi is compressed. Every
// intermediate is rescaled by a power of two (exact), kept in an exponent.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <unordered_map>
#include <mutex>
#include <thread>

#include "common.h"

namespace ftn {
Tensor* handle_tensor(ftn_tensor_t h);
ftn_tensor_t make_handle(std::unique_ptr<Tensor> t);
}  // namespace ftn

using namespace ftn;

// relative singular-value cutoff of the compressions of a network: values
// not above 1e-12 of the largest are numerically zero (FP64 round-off of the
// decomposition is ~1e-15 of the largest)
constexpr double NET_CUTOFF = 1e-12;

namespace {
struct Label {
  int kind;  // 0 bond (a = bond id), 1 open (a = tensor, b = leg)
  int a, b;
  bool operator==(const Label& o) const { return kind == o.kind && a == o.a && b == o.b; }
};
}  // namespace

struct ftn_net {
  int n = 0;
  int nbonds = 0;
  std::vector<std::unique_ptr<Tensor>> T;  // local form
  std::vector<std::vector<Label>> lab;
  std::vector<int> dummy_rank;  // rank of the dummy of an odd tensor by position; -1 if even
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

// the local form of a network: bonds labelled, global arrows translated,
// the dummy rank of every odd tensor (by position, else by index)
static std::unique_ptr<ftn_net> build_net(const std::vector<const Tensor*>& tensors, int nbonds,
                                          const int32_t* bond_ends, int conv, const int32_t* positions,
                                          hipStream_t s) {
  const int ntensors = (int)tensors.size();
  if (ntensors < 1 || nbonds < 0 || (nbonds && !bond_ends)) fail(FTN_EINVAL, "bad network arguments");
  if (conv != FTN_LOCAL && conv != FTN_GLOBAL) fail(FTN_EINVAL, "unknown convention");
  if (conv == FTN_GLOBAL && !positions) fail(FTN_EINVAL, "the global convention needs positions");
  auto net = std::make_unique<ftn_net>();
  net->n = ntensors;
  net->nbonds = nbonds;
  int sym = -1;
  for (int t = 0; t < ntensors; ++t) {
    const Tensor* x = tensors[t];
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
  // dummies of odd tensors, ranked by position (or index)
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
  }
  HIPC(hipStreamSynchronize(s));
  return net;
}

extern "C" int ftn_net_create(int ntensors, const ftn_tensor_t* tensors, int nbonds, const int32_t* bond_ends,
                              ftn_conv conv, const int32_t* positions, ftn_net_t* out) {
  return guarded_net([&] {
    if (!out || ntensors < 1 || !tensors) fail(FTN_EINVAL, "bad network arguments");
    std::vector<const Tensor*> ts(ntensors);
    for (int t = 0; t < ntensors; ++t) ts[t] = handle_tensor(tensors[t]);
    *out = build_net(ts, nbonds, bond_ends, conv, positions, nullptr).release();
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

// contracts a network along an SSA path (see ftn_contract_network)
static void contract_net(const ftn_net* net, int nsteps, const int32_t* ssa_path, int64_t chi, int gemm,
                         hipStream_t s, double* mantissa, int64_t* exp2, ftn_tensor_t* open_out,
                         int32_t* leg_src, double* stats) {
  if (!net || (nsteps && !ssa_path)) fail(FTN_EINVAL, "bad arguments");
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
  // dummy ranks carried by every live tensor (ascending), and the sign
  // exponent accumulated by moving and sorting them
  std::vector<std::vector<int>> D(n);
  for (int t = 0; t < n; ++t)
    if (net->dummy_rank[t] >= 0) D[t].push_back(net->dummy_rank[t]);
  int sgn = 0;
  int next_bond = net->nbonds;
  int64_t e2 = 0;
  // binary exponents taken out of the intermediates, summed on the device
  DBuf<int64_t> de2(1, s);
  HIPC(hipMemsetAsync(de2.p, 0, sizeof(int64_t), s));
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
    {
      const std::vector<int>&dx = D[x], &dy = D[y];
      int e = (int)((dx.size() & 1) & (dy.size() & 1));
      for (int a : dx)
        for (int b : dy) e ^= a > b ? 1 : 0;
      sgn ^= e;
      std::vector<int> dz(dx.size() + dy.size());
      std::merge(dx.begin(), dx.end(), dy.begin(), dy.end(), dz.begin());
      D.push_back(dz);
      D[x].clear();
      D[y].clear();
    }
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
          CompressResult r = op_compress_bond(*T[z], *T[w], lzs[0], lw[0], chi, NET_CUTOFF, FTN_LOCAL, s);
          T[z] = std::move(r.a);
          T[w] = std::move(r.b);
          st[1] += 1;
          st[2] += r.discarded;
          st[3] += r.near_tie ? 1 : 0;
          st[5] += r.textbook_flops;
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
    normalise_pow2(*T[z], de2.p, s);
  }
  int fin = -1;
  for (int t = 0; t < (int)T.size(); ++t)
    if (alive[t]) {
      if (fin >= 0) fail(FTN_EINVAL, "path does not contract the network to one tensor");
      fin = t;
    }
  std::unique_ptr<Tensor> F = std::move(T[fin]);
  std::vector<Label> lf = L[fin];
  // the dummies of the final tensor are all m of them, in rank order:
  // removing them costs the phase (-1)^{m(m-1)/2}
  const int64_t m = (int64_t)D[fin].size();
  if (((m * (m - 1) / 2) & 1) ^ sgn) F = op_scale(*F, -1.0, s);
  if (stats)
    for (int q = 0; q < 8; ++q) stats[q] = st[q];
  {
    int64_t de = 0;
    HIPC(hipMemcpyAsync(&de, de2.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    e2 += de;
  }
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
}

// ---------------------------------------------------------------------------
// Reverse-mode derivative of a closed network's value (local convention).
// The forward pass is the driver above, step for step, on reference-counted
// tensors; with a tape it records every operation with its inputs: the
// contraction, each fusion, each compression and the power-of-two rescaling
// of the new tensor (its exponent kept on the device). The backward pass
// walks the tape in reverse and maps cotangents through the adjoints of the
// library: ftn_ftensordot_backward, ftn_fuse_backward,
// ftn_compress_bond_backward (kept counts fixed), and the rescaling itself.
// The signs of the dummy legs of odd tensors are a constant factor of the
// value, applied to the seed. With recomputation checkpoints every
// `checkpoint` path steps, the first pass keeps only the tensors alive at the
// start of each segment (the environments at its boundary); the backward pass
// recomputes one segment at a time with the tape on and passes the
// cotangents of its boundary tensors to the segment before it. The kernels are
// deterministic, so a recomputed segment reproduces the first pass.

namespace {
struct GState {
  std::vector<std::shared_ptr<Tensor>> T;
  std::vector<std::vector<Label>> L;
  std::vector<std::vector<int>> D;
  std::vector<int> alive, ssa;
  int sgn = 0;
  int next_bond = 0;
};
struct GOp {
  int kind = 0;  // 0 contraction, 1 fusion, 2 compression, 3 rescaling
  std::shared_ptr<Tensor> a, b, c, d;
  std::vector<int> xa, xb;     // contracted axes (xa also: fused legs)
  int la = 0, lb = 0;          // compressed bond legs
  const int64_t* e = nullptr;  // rescaling: device exponent
};

template <typename T>
__global__ void k_axpy_inplace(T* __restrict__ y, const T* __restrict__ x, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] += x[i];
}
__global__ void k_scale_pow2_by(double* __restrict__ x, int64_t n, const int64_t* __restrict__ e) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] = ldexp(x[i], (int)-*e);
}
}  // namespace

static void gstep(GState& G, int k, int i, int j, int64_t chi, int gemm, hipStream_t s, int64_t* edev,
                  std::vector<GOp>* tape) {
  if (i < 0 || j < 0 || i >= (int)G.ssa.size() || j >= (int)G.ssa.size() || i == j)
    fail(FTN_EINVAL, "bad SSA id in path step " + std::to_string(k));
  const int x = G.ssa[i], y = G.ssa[j];
  if (x < 0 || y < 0 || !G.alive[x] || !G.alive[y]) fail(FTN_EINVAL, "path uses a consumed tensor");
  std::vector<int> ly;
  std::vector<int> lx = shared_legs(G.L[x], G.L[y], ly);
  std::shared_ptr<Tensor> Z(op_ftensordot(*G.T[x], *G.T[y], lx, ly, FTN_LOCAL, gemm, s, nullptr).release());
  if (tape) {
    GOp o;
    o.kind = 0;
    o.a = G.T[x];
    o.b = G.T[y];
    o.c = Z;
    o.xa = lx;
    o.xb = ly;
    tape->push_back(o);
  }
  {
    const std::vector<int>&dx = G.D[x], &dy = G.D[y];
    int e = (int)((dx.size() & 1) & (dy.size() & 1));
    for (int a : dx)
      for (int b : dy) e ^= a > b ? 1 : 0;
    G.sgn ^= e;
    std::vector<int> dz(dx.size() + dy.size());
    std::merge(dx.begin(), dx.end(), dy.begin(), dy.end(), dz.begin());
    G.D.push_back(dz);
    G.D[x].clear();
    G.D[y].clear();
  }
  std::vector<Label> lz;
  for (int q = 0; q < (int)G.L[x].size(); ++q)
    if (std::find(lx.begin(), lx.end(), q) == lx.end()) lz.push_back(G.L[x][q]);
  for (int q = 0; q < (int)G.L[y].size(); ++q)
    if (std::find(ly.begin(), ly.end(), q) == ly.end()) lz.push_back(G.L[y][q]);
  const int z = (int)G.T.size();
  G.T.push_back(Z);
  G.L.push_back(lz);
  G.alive.push_back(1);
  G.alive[x] = G.alive[y] = 0;
  G.T[x].reset();
  G.T[y].reset();
  G.ssa[i] = G.ssa[j] = -1;
  G.ssa.push_back(z);
  if (chi > 0) {
    std::vector<int> nbs;
    for (int w = 0; w < (int)G.T.size(); ++w) {
      if (w == z || !G.alive[w]) continue;
      std::vector<int> tmp;
      if (!shared_legs(G.L[z], G.L[w], tmp).empty()) nbs.push_back(w);
    }
    for (int w : nbs) {
      std::vector<int> lw;
      std::vector<int> lzs = shared_legs(G.L[z], G.L[w], lw);
      if (lzs.size() > 1) {
        std::shared_ptr<Tensor> Zf(op_fuse(*G.T[z], lzs, FTN_LOCAL, 0, s).release());
        std::shared_ptr<Tensor> Wf(op_fuse(*G.T[w], lw, FTN_LOCAL, 0, s).release());
        if (tape) {
          GOp o;
          o.kind = 1;
          o.a = G.T[z];
          o.c = Zf;
          o.xa = lzs;
          tape->push_back(o);
          o.a = G.T[w];
          o.c = Wf;
          o.xa = lw;
          tape->push_back(o);
        }
        Label nb{0, G.next_bond++, 0};
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
        relabel(G.L[z], lzs);
        relabel(G.L[w], lw);
        G.T[z] = Zf;
        G.T[w] = Wf;
        lzs = shared_legs(G.L[z], G.L[w], lw);
      }
      const int64_t dim = G.T[z]->legs()[lzs[0]].size();
      if (dim > chi && G.T[z]->size() > 0 && G.T[w]->size() > 0) {
        CompressResult r = op_compress_bond(*G.T[z], *G.T[w], lzs[0], lw[0], chi, NET_CUTOFF, FTN_LOCAL, s);
        std::shared_ptr<Tensor> Zc(r.a.release()), Wc(r.b.release());
        if (tape) {
          GOp o;
          o.kind = 2;
          o.a = G.T[z];
          o.b = G.T[w];
          o.c = Zc;
          o.d = Wc;
          o.la = lzs[0];
          o.lb = lw[0];
          tape->push_back(o);
        }
        G.T[z] = Zc;
        G.T[w] = Wc;
      }
    }
  }
  normalise_pow2(*G.T[z], edev, s);
  if (tape) {
    GOp o;
    o.kind = 3;
    o.a = G.T[z];
    o.e = edev;
    tape->push_back(o);
  }
}

static void add_into(std::unordered_map<const Tensor*, std::shared_ptr<Tensor>>& cot, const Tensor* key,
                     std::unique_ptr<Tensor> v, hipStream_t s) {
  auto it = cot.find(key);
  if (it == cot.end()) {
    cot.emplace(key, std::shared_ptr<Tensor>(v.release()));
    return;
  }
  Tensor& y = *it->second;
  if (y.st->skey != v->st->skey) fail(FTN_EINVAL, "internal: cotangent structures differ");
  const int64_t n = y.size();
  if (n)
    LAUNCH(k_axpy_inplace<double>, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, (double*)y.data,
           (const double*)v->data, n);
  HIPC(hipGetLastError());
}

// cotangents of the tape's inputs from those of its outputs (in cot)
static void backprop(const std::vector<GOp>& tape, std::unordered_map<const Tensor*, std::shared_ptr<Tensor>>& cot,
                     int64_t chi, int gemm, hipStream_t s) {
  for (auto it = tape.rbegin(); it != tape.rend(); ++it) {
    const GOp& o = *it;
    if (o.kind == 3) {
      auto f = cot.find(o.a.get());
      if (f != cot.end() && f->second->size())
        LAUNCH(k_scale_pow2_by, dim3((unsigned)cdiv(f->second->size(), 256)), dim3(256), 0, s,
               (double*)f->second->data, f->second->size(), o.e);
      HIPC(hipGetLastError());
      continue;
    }
    auto fc = cot.find(o.c.get());
    std::shared_ptr<Tensor> dc = fc == cot.end() ? nullptr : fc->second;
    std::shared_ptr<Tensor> dd;
    if (o.kind == 2) {
      auto fd = cot.find(o.d.get());
      if (fd != cot.end()) dd = fd->second;
    }
    if (!dc && !dd) continue;
    if (o.kind == 0) {
      std::unique_ptr<Tensor> da, db;
      op_ftensordot_backward(*o.a, *o.b, *dc, o.xa, o.xb, FTN_LOCAL, gemm, s, da, db);
      add_into(cot, o.a.get(), std::move(da), s);
      add_into(cot, o.b.get(), std::move(db), s);
    } else if (o.kind == 1) {
      add_into(cot, o.a.get(), op_fuse_backward(*o.a, o.xa, FTN_LOCAL, 0, *dc, s), s);
    } else {
      if (!dc) dc.reset(make_tensor(o.c->st, FTN_F64, s, true).release());
      if (!dd) dd.reset(make_tensor(o.d->st, FTN_F64, s, true).release());
      std::unique_ptr<Tensor> da, db;
      op_compress_bond_backward(*o.a, *o.b, o.la, o.lb, chi, NET_CUTOFF, FTN_LOCAL, *dc, *dd, s, da, db);
      add_into(cot, o.a.get(), std::move(da), s);
      add_into(cot, o.b.get(), std::move(db), s);
      cot.erase(o.d.get());
    }
    cot.erase(o.c.get());
  }
}

static void net_grad(const ftn_net* net, int nsteps, const int32_t* ssa_path, int64_t chi, int gemm, int checkpoint,
                     hipStream_t s, double* mantissa, int64_t* exp2, std::vector<std::unique_ptr<Tensor>>& grads) {
  if (!net || (nsteps && !ssa_path)) fail(FTN_EINVAL, "bad arguments");
  const int n = net->n;
  if (nsteps != n - 1) fail(FTN_EINVAL, "a path over n tensors has n-1 steps");
  if (gemm != FTN_GEMM_F64) fail(FTN_ENOTSUP, "network gradients need the FP64 GEMM form");
  if (checkpoint < 0) fail(FTN_EINVAL, "checkpoint must be >= 0");
  GState G;
  for (int t = 0; t < n; ++t) {
    if (net->T[t]->dtype != FTN_F64) fail(FTN_ENOTSUP, "network gradients need FP64 tensors");
    G.T.push_back(std::shared_ptr<Tensor>(share_tensor(*net->T[t], net->T[t]->st).release()));
    G.L.push_back(net->lab[t]);
    G.D.push_back(net->dummy_rank[t] >= 0 ? std::vector<int>{net->dummy_rank[t]} : std::vector<int>{});
    G.alive.push_back(1);
    G.ssa.push_back(t);
  }
  G.next_bond = net->nbonds;
  const int seg = (checkpoint > 0 && checkpoint < nsteps) ? checkpoint : std::max(nsteps, 1);
  const bool recompute = seg < nsteps;
  DBuf<int64_t> edev(std::max(nsteps, 1), s);
  HIPC(hipMemsetAsync(edev.p, 0, std::max(nsteps, 1) * sizeof(int64_t), s));
  std::vector<GState> starts;
  std::vector<GOp> tape;
  for (int k = 0; k < nsteps; ++k) {
    if (k % seg == 0) starts.push_back(G);
    gstep(G, k, ssa_path[2 * k], ssa_path[2 * k + 1], chi, gemm, s, edev.p + k, recompute ? nullptr : &tape);
  }
  if (nsteps == 0) starts.push_back(G);
  int fin = -1;
  for (int t = 0; t < (int)G.T.size(); ++t)
    if (G.alive[t]) {
      if (fin >= 0) fail(FTN_EINVAL, "path does not contract the network to one tensor");
      fin = t;
    }
  const Tensor& F = *G.T[fin];
  if (F.ndim() != 0) fail(FTN_ENOTSUP, "network gradients need a closed network (a scalar value)");
  const int64_t m = (int64_t)G.D[fin].size();
  const double sign = (((m * (m - 1) / 2) & 1) ^ G.sgn) ? -1.0 : 1.0;
  std::vector<int64_t> eh(std::max(nsteps, 1), 0);
  double v = 0.0;
  HIPC(hipMemcpyAsync(eh.data(), edev.p, eh.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  if (F.size()) HIPC(hipMemcpyAsync(&v, F.data, 8, hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  int64_t e2 = 0;
  for (int k = 0; k < nsteps; ++k) e2 += eh[k];
  if (mantissa) *mantissa = sign * v;
  if (exp2) *exp2 = e2;
  // cotangents of the tensors alive at a segment boundary, by slot
  std::map<int, std::shared_ptr<Tensor>> bcot;
  if (F.size()) {
    std::shared_ptr<Tensor> seed(make_tensor(F.st, FTN_F64, s, false).release());
    h2d(seed->data, &sign, 8, s);
    bcot[fin] = seed;
  }
  const int nseg = (int)starts.size();
  DBuf<int64_t> edev2(recompute ? std::max(nsteps, 1) : 1, s);
  for (int g = nseg - 1; g >= 0 && !bcot.empty(); --g) {
    const int k0 = g * seg, k1 = std::min(nsteps, k0 + seg);
    const GState* end = &G;
    GState G2;
    if (recompute) {
      G2 = starts[g];
      tape.clear();
      HIPC(hipMemsetAsync(edev2.p + k0, 0, (k1 - k0) * sizeof(int64_t), s));
      for (int k = k0; k < k1; ++k)
        gstep(G2, k, ssa_path[2 * k], ssa_path[2 * k + 1], chi, gemm, s, edev2.p + k, &tape);
      end = &G2;
    }
    std::unordered_map<const Tensor*, std::shared_ptr<Tensor>> cot;
    for (auto& kv : bcot) cot[end->T[kv.first].get()] = kv.second;
    bcot.clear();
    backprop(tape, cot, chi, gemm, s);
    tape.clear();
    const GState& S0 = starts[g];
    for (int t = 0; t < (int)S0.T.size(); ++t) {
      if (!S0.alive[t] || !S0.T[t]) continue;
      auto f = cot.find(S0.T[t].get());
      if (f != cot.end()) bcot[t] = f->second;
    }
  }
  grads.clear();
  for (int t = 0; t < n; ++t) {
    auto f = bcot.find(t);
    if (f != bcot.end() && f->second->st->skey == net->T[t]->st->skey) {
      grads.push_back(share_tensor(*f->second, f->second->st));
    } else {
      grads.push_back(make_tensor(net->T[t]->st, FTN_F64, s, true));
    }
  }
}

extern "C" int ftn_contract_network_grad(ftn_net_t net, int nsteps, const int32_t* ssa_path, int64_t chi,
                                         ftn_gemm gemm, int checkpoint, ftn_stream_t stream, double* mantissa,
                                         int64_t* exp2, ftn_tensor_t* grads) {
  return guarded_net([&] {
    if (!net || !grads) fail(FTN_EINVAL, "null argument");
    std::vector<std::unique_ptr<Tensor>> g;
    net_grad(net, nsteps, ssa_path, chi, gemm, checkpoint, (hipStream_t)stream, mantissa, exp2, g);
    for (size_t t = 0; t < g.size(); ++t) grads[t] = make_handle(std::move(g[t]));
  });
}

extern "C" int ftn_contract_network(ftn_net_t net, int nsteps, const int32_t* ssa_path, int64_t chi,
                                    ftn_gemm gemm, ftn_stream_t stream, double* mantissa, int64_t* exp2,
                                    ftn_tensor_t* open_out, int32_t* leg_src, double* stats) {
  return guarded_net([&] {
    contract_net(net, nsteps, ssa_path, chi, gemm, (hipStream_t)stream, mantissa, exp2, open_out, leg_src, stats);
  });
}

// ---------------------------------------------------------------------------
// Amplitudes <n|psi> (see ftn_amplitudes in ftn.h). The projection of a site
// tensor on physical index v is the contraction e_v . T over leg 0, with e_v
// the one-hot vector on the partner leg; with e_v on the left and its leg the
// arrow head this contraction carries no sign, so it is exactly T[v, ...].
// Every projection needed is made once; samples then run as independent
// closed networks, pulled from a shared counter by worker threads that each
// own a HIP stream. The worker streams are created once per device and kept
// for the life of the process.

static std::mutex g_ws_mu;
static std::map<int, std::vector<hipStream_t>> g_ws;

static std::vector<hipStream_t> worker_streams(int dev, int n) {
  std::lock_guard<std::mutex> g(g_ws_mu);
  std::vector<hipStream_t>& v = g_ws[dev];
  while ((int)v.size() < n) {
    hipStream_t st = nullptr;
    HIPC(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));  // default priority
    v.push_back(st);
  }
  return std::vector<hipStream_t>(v.begin(), v.begin() + n);
}

static std::unique_ptr<Tensor> one_hot_partner(const Tensor& t, int64_t v, hipStream_t s) {
  const int sym = t.sym();
  const Leg& p = t.legs()[0];
  int k = 0;
  int64_t off = 0;
  while (k < p.nsect() && v >= off + p.d[k]) off += p.d[k++];
  if (k == p.nsect()) fail(FTN_EINVAL, "physical index out of range");
  Leg e = p;
  e.dual = 1 - p.dual;
  auto out = make_tensor(sym, t.dtype, std::vector<Leg>{e}, q_signed(sym, e.dual, p.q[k]), s, true);
  if (out->size() != p.d[k]) fail(FTN_EINVAL, "internal: one-hot vector with several blocks");
  if (t.dtype == FTN_F64) {
    const double one = 1.0;
    h2d((char*)out->data + (v - off) * 8, &one, 8, s);
  } else {
    const float one = 1.0f;
    h2d((char*)out->data + (v - off) * 4, &one, 4, s);
  }
  return out;
}

extern "C" int ftn_amplitudes(int nsites, const ftn_tensor_t* sites, int nbonds, const int32_t* bond_ends,
                              int nsteps, const int32_t* ssa_path, int64_t chi, ftn_gemm gemm, int64_t nsamples,
                              const int32_t* configs, int nworkers, ftn_stream_t stream, double* mantissa,
                              int64_t* exp2) {
  return guarded_net([&] {
    if (nsites < 1 || !sites || nbonds < 0 || (nbonds && !bond_ends) || nsamples < 0 ||
        (nsamples && (!configs || !mantissa || !exp2)))
      fail(FTN_EINVAL, "bad amplitude arguments");
    if (nsteps != nsites - 1 || (nsteps && !ssa_path)) fail(FTN_EINVAL, "a path over n tensors has n-1 steps");
    hipStream_t s = (hipStream_t)stream;
    std::vector<const Tensor*> T(nsites);
    for (int i = 0; i < nsites; ++i) {
      T[i] = handle_tensor(sites[i]);
      if (!T[i]) fail(FTN_EINVAL, "null site tensor");
      if (T[i]->ndim() < 1) fail(FTN_EINVAL, "a site tensor needs a physical leg (leg 0)");
      if (T[i]->sym() != T[0]->sym() || T[i]->dtype != T[0]->dtype)
        fail(FTN_ENOTSUP, "site tensors must share symmetry and dtype");
    }
    std::vector<int32_t> be(4 * (size_t)nbonds);
    for (int b = 0; b < nbonds; ++b) {
      for (int e = 0; e < 2; ++e) {
        const int t = bond_ends[4 * b + 2 * e], l = bond_ends[4 * b + 2 * e + 1];
        if (t < 0 || t >= nsites || l < 1 || l >= T[t]->ndim()) fail(FTN_EINVAL, "bad bond end (legs >= 1)");
        be[4 * b + 2 * e] = t;
        be[4 * b + 2 * e + 1] = l - 1;
      }
    }
    // projections used by any sample, and the parity of every physical index
    std::vector<std::vector<std::unique_ptr<Tensor>>> proj(nsites);
    std::vector<std::vector<int>> ppar(nsites);
    for (int i = 0; i < nsites; ++i) {
      const Leg& p = T[i]->legs()[0];
      proj[i].resize(p.size());
      for (int k = 0; k < p.nsect(); ++k)
        for (int64_t j = 0; j < p.d[k]; ++j) ppar[i].push_back(q_par(p.q[k]));
    }
    for (int64_t k = 0; k < nsamples; ++k)
      for (int i = 0; i < nsites; ++i) {
        const int v = configs[k * nsites + i];
        if (v < 0 || v >= (int)proj[i].size()) fail(FTN_EINVAL, "configuration index out of range");
        if (!proj[i][v]) {
          auto e = one_hot_partner(*T[i], v, s);
          const int pg = T[i]->dtype == FTN_F64 ? FTN_GEMM_F64 : FTN_GEMM_F32;
          proj[i][v] = op_ftensordot(*e, *T[i], {0}, {0}, FTN_LOCAL, pg, s, nullptr);
        }
      }
    HIPC(hipStreamSynchronize(s));
    if (nsamples == 0) return;
    int dev = 0;
    HIPC(hipGetDevice(&dev));
    const int nw = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)std::max(nworkers, 1), 64, nsamples}));
    std::atomic<int64_t> next{0};
    std::atomic<bool> stop{false};
    std::mutex mu;
    int err_code = 0;
    std::string err_msg;
    const std::vector<hipStream_t> wss = worker_streams(dev, nw);
    auto work = [&](int w) {
      hipStream_t ws = wss[w];
      // the calling thread keeps its instrumentation when it works alone
      prof_quiet(nw > 1);
      try {
        HIPC(hipSetDevice(dev));
        std::vector<const Tensor*> P(nsites);
        for (;;) {
          const int64_t k = next.fetch_add(1);
          if (k >= nsamples || stop.load()) break;
          const int32_t* c = configs + k * nsites;
          // (-1)^E: the physical leg of site i passes the bond legs of the
          // sites before it, of parity p(T_j) + p(n_j)
          int e = 0, acc = 0;
          for (int i = 0; i < nsites; ++i) {
            P[i] = proj[i][c[i]].get();
            const int pn = ppar[i][c[i]];
            e ^= pn & acc;
            acc ^= T[i]->parity() ^ pn;
          }
          auto net = build_net(P, nbonds, be.data(), FTN_LOCAL, nullptr, ws);
          double m = 0;
          int64_t x = 0;
          contract_net(net.get(), nsteps, ssa_path, chi, gemm, ws, &m, &x, nullptr, nullptr, nullptr);
          mantissa[k] = e ? -m : m;
          exp2[k] = x;
        }
      } catch (const Error& ex) {
        std::lock_guard<std::mutex> g(mu);
        if (!err_code) {
          err_code = ex.code;
          err_msg = ex.msg;
        }
        stop = true;
      } catch (const std::exception& ex) {
        std::lock_guard<std::mutex> g(mu);
        if (!err_code) {
          err_code = FTN_EINVAL;
          err_msg = ex.what();
        }
        stop = true;
      }
      (void)hipStreamSynchronize(ws);
      prof_quiet(false);
    };
    std::vector<std::thread> th;
    for (int w = 1; w < nw; ++w) th.emplace_back(work, w);
    work(0);
    for (auto& t : th) t.join();
    if (err_code) fail(err_code, err_msg);
  });
}
