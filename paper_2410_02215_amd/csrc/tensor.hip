// Symmetric block-sparse tensors on the device: allocation, block
// enumeration (Eq. symmetryrule), dense <-> block conversion, elementwise ops.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace ftn {

// ---------------------------------------------------------------------------
// errors
static thread_local std::string g_last_error;
void set_last_error(const std::string& msg) { g_last_error = msg; }
const char* last_error_cstr() { return g_last_error.c_str(); }

void fail(int code, const std::string& msg) { throw Error{code, msg}; }

void check_launch(const char* name, dim3 grid, dim3 block) {
  const uint64_t threads = (uint64_t)grid.x * grid.y * grid.z * block.x * block.y * block.z;
  if (grid.x == 0 || grid.y == 0 || grid.z == 0 || block.x == 0)
    fail(FTN_EINVAL, std::string("internal: empty launch of ") + name);
  if ((uint64_t)grid.x * block.x >= (1ull << 32) || threads >= (1ull << 32))
    fail(FTN_EINVAL, std::string("internal: launch of ") + name + " exceeds 2^32 work-items (grid " +
                         std::to_string(grid.x) + ")");
}

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (e == hipErrorOutOfMemory) fail(FTN_ENOMEM, m);
    fail(FTN_EHIP, m);
  }
}

// ---------------------------------------------------------------------------
// allocator: stream-ordered pool by default, or an external callback pair
static void* (*g_alloc)(size_t, ftn_stream_t, void*) = nullptr;
static void (*g_free)(void*, ftn_stream_t, void*) = nullptr;
static void* g_alloc_ctx = nullptr;

void set_allocator(void* (*a)(size_t, ftn_stream_t, void*), void (*f)(void*, ftn_stream_t, void*),
                   void* ctx) {
  g_alloc = a;
  g_free = f;
  g_alloc_ctx = ctx;
}

// Caching allocator for temporaries. Freed blocks are kept per device in a
// size-ordered pool tagged with the stream that freed them; a request on the
// same stream may reuse a block at once (stream order makes it safe), and a
// block freed on another stream is reused only once the event recorded at
// its release has completed. Sizes are rounded to 512 B (small) or 2 MiB
// (large) and a block is reused for requests down to half its size. On
// out-of-memory every cached block is released and the allocation retried.
namespace {
struct Block {
  void* p;
  size_t size;
  hipStream_t s;
  hipEvent_t ev;  // recorded at release (for reuse on another stream)
};
struct DevCache {
  std::multimap<size_t, Block> free_;      // by size
  std::unordered_map<void*, size_t> live;  // pointer -> rounded size
  std::vector<hipEvent_t> events;          // idle events for reuse
  // bytes handed out (rounded sizes), their high-water mark, and bytes held
  // from hipMalloc (handed out + cached)
  size_t in_use = 0, peak = 0, reserved = 0;
  void take(void* p, size_t sz) {
    live[p] = sz;
    in_use += sz;
    peak = std::max(peak, in_use);
  }
};
std::mutex g_cache_mu;
std::unordered_map<int, DevCache>* g_cache = new std::unordered_map<int, DevCache>();
// blocks of external allocators, with the free function that owns each
struct ExtOwner {
  void (*free_fn)(void*, ftn_stream_t, void*);
  void* ctx;
};
std::unordered_map<void*, ExtOwner>* g_ext = new std::unordered_map<void*, ExtOwner>();

size_t round_size(size_t b) {
  const size_t big = 2u << 20;
  return b < big ? (b + 511) & ~(size_t)511 : (b + big - 1) & ~(big - 1);
}

void release_cached(DevCache& c) {
  if (c.free_.empty()) return;
  (void)hipDeviceSynchronize();
  for (auto& kv : c.free_) {
    (void)hipFree(kv.second.p);
    c.reserved -= kv.first;
    if (kv.second.ev) c.events.push_back(kv.second.ev);
  }
  c.free_.clear();
}
}  // namespace

void* dmalloc(size_t bytes, hipStream_t s, bool persistent) {
  if (bytes == 0) return nullptr;
  void* p = nullptr;
  if (g_alloc && !persistent) {
    auto fr = g_free;
    void* ctx = g_alloc_ctx;
    p = g_alloc(bytes, (ftn_stream_t)s, ctx);
    if (!p) fail(FTN_ENOMEM, "external allocator returned NULL for " + std::to_string(bytes) + " bytes");
    // remembered with the allocator that made it: a block is always returned
    // to its own allocator, even after another one has been registered
    std::lock_guard<std::mutex> g(g_cache_mu);
    (*g_ext)[p] = ExtOwner{fr, ctx};
    return p;
  }
  if (persistent) {
    HIPC(hipMalloc(&p, bytes));
    return p;
  }
  int dev = 0;
  HIPC(hipGetDevice(&dev));
  const size_t sz = round_size(bytes);
  std::lock_guard<std::mutex> g(g_cache_mu);
  DevCache& c = (*g_cache)[dev];
  for (auto it = c.free_.lower_bound(sz); it != c.free_.end() && it->first <= 2 * sz; ++it) {
    Block& b = it->second;
    if (b.s != s && (!b.ev || hipEventQuery(b.ev) != hipSuccess)) {
      (void)hipGetLastError();
      continue;
    }
    p = b.p;
    c.take(p, it->first);
    if (b.ev) c.events.push_back(b.ev);
    c.free_.erase(it);
    return p;
  }
  hipError_t e = hipMalloc(&p, sz);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    release_cached(c);
    e = hipMalloc(&p, sz);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(e == hipErrorOutOfMemory ? FTN_ENOMEM : FTN_EHIP,
         "hipMalloc(" + std::to_string(sz) + "): " + hipGetErrorString(e));
  }
  c.reserved += sz;
  c.take(p, sz);
  return p;
}

void dfree(void* p, hipStream_t s, bool persistent) {
  if (!p) return;
  if (persistent) {
    (void)hipFree(p);
    return;
  }
  {
    ExtOwner o{nullptr, nullptr};
    {
      std::lock_guard<std::mutex> g(g_cache_mu);
      auto it = g_ext->find(p);
      if (it != g_ext->end()) {
        o = it->second;
        g_ext->erase(it);
      }
    }
    if (o.free_fn) {
      o.free_fn(p, (ftn_stream_t)s, o.ctx);
      return;
    }
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  // the block leaves the live set under the lock, its release event is
  // recorded outside it (the block is nobody else's until it is listed as
  // free again), so threads on other streams do not wait behind the call
  Block b{p, 0, s, nullptr};
  {
    std::lock_guard<std::mutex> g(g_cache_mu);
    DevCache& c = (*g_cache)[dev];
    auto it = c.live.find(p);
    if (it == c.live.end()) return;  // not from this cache
    b.size = it->second;
    c.in_use -= it->second;
    c.live.erase(it);
    if (!c.events.empty()) {
      b.ev = c.events.back();
      c.events.pop_back();
    }
  }
  if (!b.ev && hipEventCreateWithFlags(&b.ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    b.ev = nullptr;
  }
  bool idle_ev = false;
  if (b.ev && hipEventRecord(b.ev, s) != hipSuccess) {
    (void)hipGetLastError();
    idle_ev = true;
  }
  std::lock_guard<std::mutex> g(g_cache_mu);
  DevCache& c = (*g_cache)[dev];
  if (idle_ev) {
    c.events.push_back(b.ev);
    b.ev = nullptr;
  }
  c.free_.emplace(b.size, b);
}

void memory_stats(int dev, int64_t* in_use, int64_t* peak, int64_t* reserved, bool reset_peak) {
  std::lock_guard<std::mutex> g(g_cache_mu);
  DevCache& c = (*g_cache)[dev];
  if (in_use) *in_use = (int64_t)c.in_use;
  if (peak) *peak = (int64_t)c.peak;
  if (reserved) *reserved = (int64_t)c.reserved;
  if (reset_peak) c.peak = c.in_use;
}

// ---------------------------------------------------------------------------
// pinned staging rings for small host-to-device copies, one per stream, so
// that threads driving different streams never wait for one another (a
// shared ring serialised every upload of every worker thread behind one
// lock): 4 chunks of 2 MiB per stream; a copy never spans chunks; when the
// ring moves on from a chunk an event is recorded behind the copies
// enqueued so far, and a chunk is written again only after its event has
// completed. Rings live as long as the process (one per stream handle seen).
namespace {
constexpr size_t RING_CH = 2u << 20, RING_N = 4;
struct Ring {
  std::mutex mu;
  char* buf = nullptr;
  bool failed = false;
  size_t cur = 0, off = 0;
  hipEvent_t ev[RING_N] = {};
  bool pending[RING_N] = {};
};
std::mutex g_rings_mu;
std::unordered_map<hipStream_t, Ring*>* g_rings = new std::unordered_map<hipStream_t, Ring*>();

Ring* ring_of(hipStream_t s) {
  std::lock_guard<std::mutex> g(g_rings_mu);
  Ring*& r = (*g_rings)[s];
  if (!r) r = new Ring();
  return r;
}
}  // namespace

void h2d(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (!bytes) return;
  Ring* r = ring_of(s);
  std::lock_guard<std::mutex> g(r->mu);
  if (!r->buf && !r->failed) {
    if (hipHostMalloc((void**)&r->buf, RING_CH * RING_N, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      r->buf = nullptr;
      r->failed = true;
    }
  }
  if (!r->buf || bytes > RING_CH) {
    HIPC(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
    return;
  }
  if (r->off + bytes > RING_CH) {
    if (!r->ev[r->cur]) HIPC(hipEventCreateWithFlags(&r->ev[r->cur], hipEventDisableTiming));
    HIPC(hipEventRecord(r->ev[r->cur], s));
    r->pending[r->cur] = true;
    r->cur = (r->cur + 1) % RING_N;
    r->off = 0;
    if (r->pending[r->cur]) {
      HIPC(hipEventSynchronize(r->ev[r->cur]));
      r->pending[r->cur] = false;
    }
  }
  char* stage = r->buf + r->cur * RING_CH + r->off;
  std::memcpy(stage, src, bytes);
  HIPC(hipMemcpyAsync(dst, stage, bytes, hipMemcpyHostToDevice, s));
  r->off = (r->off + bytes + 255) & ~(size_t)255;
}

// ---------------------------------------------------------------------------
// single-workgroup exclusive scan of int64 values (block counts, sizes)
constexpr int SCAN_T = 1024;

__global__ void __launch_bounds__(SCAN_T) k_scan_exclusive(int64_t* v, int64_t n, int64_t* total) {
  __shared__ int64_t sh[SCAN_T];
  int64_t carry = 0;
  const int tid = threadIdx.x;
  for (int64_t base = 0; base < n; base += (int64_t)SCAN_T * 4) {
    int64_t loc[4];
    int64_t s = 0;
    for (int j = 0; j < 4; ++j) {
      int64_t i = base + (int64_t)tid * 4 + j;
      loc[j] = i < n ? v[i] : 0;
      s += loc[j];
    }
    sh[tid] = s;
    __syncthreads();
    for (int off = 1; off < SCAN_T; off <<= 1) {
      int64_t x = tid >= off ? sh[tid - off] : 0;
      __syncthreads();
      sh[tid] += x;
      __syncthreads();
    }
    int64_t excl = carry + sh[tid] - s;
    for (int j = 0; j < 4; ++j) {
      int64_t i = base + (int64_t)tid * 4 + j;
      if (i < n) v[i] = excl;
      excl += loc[j];
    }
    carry += sh[SCAN_T - 1];
    __syncthreads();
  }
  if (tid == 0 && total) *total = carry;
}

void scan_exclusive(int64_t* v, int64_t n, int64_t* total_out, hipStream_t s) {
  LAUNCH(k_scan_exclusive, dim3(1), dim3(SCAN_T), 0, s, v, n, total_out);
  HIPC(hipGetLastError());
}

// ---------------------------------------------------------------------------
// leg tables
void make_devlegs(const std::vector<Leg>& legs, int sym, Q total, hipStream_t s, DevLegs& out) {
  LegTab& t = out.tab;
  std::memset(&t, 0, sizeof(t));
  t.ndim = (int)legs.size();
  t.sym = sym;
  t.total = q_canon(sym, total);
  std::vector<Q> q;
  std::vector<int64_t> d;
  for (int i = 0; i < t.ndim; ++i) {
    t.nsect[i] = legs[i].nsect();
    t.base[i] = (int)q.size();
    t.dual[i] = legs[i].dual;
    for (int k = 0; k < legs[i].nsect(); ++k) {
      q.push_back(legs[i].q[k]);
      d.push_back(legs[i].d[k]);
    }
  }
  out.q = DBuf<Q>(q.size(), s);
  out.d = DBuf<int64_t>(d.size(), s);
  out.q.upload(q.data(), q.size());
  out.d.upload(d.data(), d.size());
  HIPC(hipStreamSynchronize(s));  // host vectors go out of scope
}

// ---------------------------------------------------------------------------
// K1: block enumeration. Thread t decodes the key prefix over legs 0..n-2
// (mixed radix, last leg fastest = lexicographic); the symmetry rule fixes the
// charge of the last leg, which has at most one matching sector.
__global__ void k_enum_flags(LegTab lt, const Q* __restrict__ q, int64_t P, int32_t* last,
                             int64_t* flag) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= P) return;
  const int n = lt.ndim, sym = lt.sym;
  Q acc{0, 0};
  int64_t rem = t;
  for (int i = n - 2; i >= 0; --i) {
    int ns = lt.nsect[i];
    int k = (int)(rem % ns);
    rem /= ns;
    acc = q_add(sym, acc, q_signed(sym, lt.dual[i], q[lt.base[i] + k]));
  }
  Q need = q_signed(sym, lt.dual[n - 1], q_add(sym, lt.total, q_neg(sym, acc)));
  int found = -1;
  for (int k = 0; k < lt.nsect[n - 1]; ++k) {
    if (q_eq(q[lt.base[n - 1] + k], need)) {
      found = k;
      break;
    }
  }
  last[t] = found;
  flag[t] = found >= 0 ? 1 : 0;
}

__global__ void k_enum_write(LegTab lt, const Q* __restrict__ q, const int64_t* __restrict__ dims,
                             int64_t P, const int32_t* last, const int64_t* pos, int32_t* keys,
                             int64_t* sizes, int32_t* shapes, uint32_t* parmask) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= P || last[t] < 0) return;
  const int n = lt.ndim;
  const int64_t b = pos[t];
  int64_t rem = t;
  int64_t sz = 1;
  uint32_t pm = 0;
  int k = last[t];
  keys[b * n + n - 1] = k;
  int64_t d = dims[lt.base[n - 1] + k];
  shapes[b * n + n - 1] = (int32_t)d;
  sz *= d;
  pm |= (uint32_t)q_par(q[lt.base[n - 1] + k]) << (n - 1);
  for (int i = n - 2; i >= 0; --i) {
    int ns = lt.nsect[i];
    int ki = (int)(rem % ns);
    rem /= ns;
    keys[b * n + i] = ki;
    int64_t di = dims[lt.base[i] + ki];
    shapes[b * n + i] = (int32_t)di;
    sz *= di;
    pm |= (uint32_t)q_par(q[lt.base[i] + ki]) << i;
  }
  sizes[b] = sz;
  parmask[b] = pm;
}

std::string structure_key(int sym, const std::vector<Leg>& legs, Q total) {
  std::string k;
  auto put = [&](const void* p, size_t n) { k.append((const char*)p, n); };
  int32_t hdr[4] = {sym, (int32_t)legs.size(), total.a, total.b};
  put(hdr, sizeof(hdr));
  for (auto& l : legs) {
    int32_t h[2] = {l.dual, l.nsect()};
    put(h, sizeof(h));
    put(l.q.data(), l.q.size() * sizeof(Q));
    put(l.d.data(), l.d.size() * sizeof(int64_t));
  }
  return k;
}

static std::mutex g_struct_mu;
static auto& g_structs = *new std::unordered_map<std::string, std::shared_ptr<const Structure>>();

static void validate_legs(int sym, const std::vector<Leg>& legs) {
  if (legs.size() > (size_t)MAXD) fail(FTN_EINVAL, "too many legs (max 16)");
  for (size_t i = 0; i < legs.size(); ++i) {
    const Leg& l = legs[i];
    if (l.dual != 0 && l.dual != 1) fail(FTN_EINVAL, "dual flag must be 0 or 1");
    for (int k = 0; k < l.nsect(); ++k) {
      if (l.d[k] <= 0) fail(FTN_EINVAL, "sector dims must be positive");
      Q c = q_canon(sym, l.q[k]);
      if (!q_eq(c, l.q[k])) fail(FTN_EINVAL, "charge out of range for the symmetry");
      if (k && !q_lt(l.q[k - 1], l.q[k])) fail(FTN_EINVAL, "sector charges must be strictly ascending");
    }
  }
}

std::shared_ptr<const Structure> get_structure(int sym, const std::vector<Leg>& legs, Q total,
                                               hipStream_t s) {
  if (sym < 0 || sym > 2) fail(FTN_EINVAL, "unknown symmetry");
  validate_legs(sym, legs);
  total = q_canon(sym, total);
  std::string key = structure_key(sym, legs, total);
  {
    std::lock_guard<std::mutex> g(g_struct_mu);
    auto it = g_structs.find(key);
    if (it != g_structs.end()) return it->second;
  }
  auto st = std::make_shared<Structure>();
  st->sym = sym;
  st->ndim = (int)legs.size();
  st->legs = legs;
  st->total = total;
  st->skey = key;
  const int n = st->ndim;
  bool empty_leg = false;
  for (auto& l : legs) empty_leg |= (l.nsect() == 0);
  if (n == 0) {
    st->nblocks = (total.a == 0 && total.b == 0) ? 1 : 0;
    st->offsets = {0, st->nblocks};
    st->parmask.assign(st->nblocks, 0);
    st->size = st->nblocks;
  } else if (empty_leg) {
    st->nblocks = 0;
    st->offsets = {0};
    st->size = 0;
  } else {
    DevLegs dl;
    make_devlegs(legs, sym, total, s, dl);
    int64_t P = 1;
    for (int i = 0; i < n - 1; ++i) P *= legs[i].nsect();
    DBuf<int32_t> last(P, s);
    DBuf<int64_t> flag(P + 1, s);
    const int T = 256;
    LAUNCH(k_enum_flags, dim3((unsigned)cdiv(P, T)), dim3(T), 0, s, dl.tab, dl.q.p, P,
                       last.p, flag.p);
    HIPC(hipGetLastError());
    scan_exclusive(flag.p, P, flag.p + P, s);
    int64_t nb = 0;
    HIPC(hipMemcpyAsync(&nb, flag.p + P, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    st->nblocks = nb;
    Structure* w = st.get();
    // a cached structure's tables are read by kernels of every stream; they
    // are released (on eviction) by hipFree, which waits for all streams,
    // never through the stream-ordered cache
    w->d_keys = DBuf<int32_t>(nb * n, nullptr, true);
    w->d_offsets = DBuf<int64_t>(nb + 1, nullptr, true);
    w->d_shapes = DBuf<int32_t>(nb * n, nullptr, true);
    w->d_parmask = DBuf<uint32_t>(nb, nullptr, true);
    if (nb) {
      LAUNCH(k_enum_write, dim3((unsigned)cdiv(P, T)), dim3(T), 0, s, dl.tab, dl.q.p,
                         dl.d.p, P, last.p, flag.p, w->d_keys.p, w->d_offsets.p, w->d_shapes.p,
                         w->d_parmask.p);
      HIPC(hipGetLastError());
    }
    scan_exclusive(w->d_offsets.p, nb, w->d_offsets.p + nb, s);
    w->keys.resize(nb * n);
    w->offsets.resize(nb + 1);
    w->parmask.resize(nb);
    std::vector<int32_t> sh(nb * n);
    if (nb) {
      HIPC(hipMemcpyAsync(w->keys.data(), w->d_keys.p, nb * n * 4, hipMemcpyDeviceToHost, s));
      HIPC(hipMemcpyAsync(w->parmask.data(), w->d_parmask.p, nb * 4, hipMemcpyDeviceToHost, s));
      HIPC(hipMemcpyAsync(sh.data(), w->d_shapes.p, nb * n * 4, hipMemcpyDeviceToHost, s));
    }
    HIPC(hipMemcpyAsync(w->offsets.data(), w->d_offsets.p, (nb + 1) * 8, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    w->shapes.assign(sh.begin(), sh.end());
    w->size = w->offsets[nb];
  }
  if (st->d_offsets.p == nullptr) {  // scalar / empty structures: small uploads
    Structure* w = st.get();
    w->d_offsets = DBuf<int64_t>(w->offsets.size(), nullptr, true);
    HIPC(hipMemcpy(w->d_offsets.p, w->offsets.data(), w->offsets.size() * 8, hipMemcpyHostToDevice));
    if (w->nblocks) {
      w->d_parmask = DBuf<uint32_t>(w->nblocks, nullptr, true);
      HIPC(hipMemcpy(w->d_parmask.p, w->parmask.data(), w->nblocks * 4, hipMemcpyHostToDevice));
    }
  }
  std::lock_guard<std::mutex> g(g_struct_mu);
  if (g_structs.size() > 8192) {
    for (auto it = g_structs.begin(); it != g_structs.end();) {
      if (it->second.use_count() == 1)
        it = g_structs.erase(it);
      else
        ++it;
    }
  }
  auto ins = g_structs.emplace(key, st);
  return ins.first->second;
}

std::unique_ptr<Tensor> make_tensor(std::shared_ptr<const Structure> st, int dtype, hipStream_t s,
                                    bool zero) {
  if (dtype != FTN_F64 && dtype != FTN_F32) fail(FTN_EINVAL, "unknown dtype");
  auto t = std::make_unique<Tensor>();
  t->st = std::move(st);
  t->dtype = dtype;
  size_t bytes = (size_t)t->size() * t->esize();
  void* p = dmalloc(bytes, s);
  t->buf = std::shared_ptr<void>(p, [s](void* q) { dfree(q, s); });
  t->data = p;
  if (zero && bytes) HIPC(hipMemsetAsync(t->data, 0, bytes, s));
  return t;
}

std::unique_ptr<Tensor> make_tensor(int sym, int dtype, const std::vector<Leg>& legs, Q total,
                                    hipStream_t s, bool zero) {
  return make_tensor(get_structure(sym, legs, total, s), dtype, s, zero);
}

std::unique_ptr<Tensor> share_tensor(const Tensor& t, std::shared_ptr<const Structure> st) {
  if (st->size != t.size()) fail(FTN_EINVAL, "internal: shared view with a different size");
  auto o = std::make_unique<Tensor>();
  o->st = std::move(st);
  o->dtype = t.dtype;
  o->buf = t.buf;
  o->data = t.data;
  return o;
}

int64_t block_index(const Structure& t, const int32_t* key) {
  int64_t lo = 0, hi = t.nblocks;
  const int n = t.ndim;
  while (lo < hi) {
    int64_t mid = (lo + hi) / 2;
    const int32_t* k = &t.keys[mid * n];
    int c = 0;
    for (int i = 0; i < n && !c; ++i) c = (k[i] < key[i]) ? -1 : (k[i] > key[i] ? 1 : 0);
    if (c == 0) return mid;
    if (c < 0)
      lo = mid + 1;
    else
      hi = mid;
  }
  return -1;
}

// ---------------------------------------------------------------------------
// dense <-> blocks: one thread per stored entry; the block is found by binary
// search over the block offsets.
struct DenseMap {
  int ndim;
  int64_t dstride[MAXD];  // dense strides
  int sbase[MAXD];        // base into the sector offset table per leg
};

__device__ inline int64_t find_block(const int64_t* off, int64_t nb, int64_t e) {
  int64_t lo = 0, hi = nb - 1;
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) / 2;
    if (off[mid] <= e)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <typename T, int DIR>
__global__ void k_dense_blocks(DenseMap m, const int32_t* __restrict__ keys,
                               const int32_t* __restrict__ shapes, const int64_t* __restrict__ off,
                               int64_t nb, int64_t size, const int64_t* __restrict__ soff,
                               T* blk, T* dense) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= size) return;
  int64_t b = find_block(off, nb, e);
  int64_t r = e - off[b];
  int64_t di = 0;
  for (int i = m.ndim - 1; i >= 0; --i) {
    int64_t d = shapes[b * m.ndim + i];
    int64_t li = r % d;
    r /= d;
    int64_t gi = soff[m.sbase[i] + keys[b * m.ndim + i]] + li;
    di += gi * m.dstride[i];
  }
  if (DIR == 0)
    blk[e] = dense[di];
  else
    dense[di] = blk[e];
}

static void dense_map(const Structure& st, DenseMap& m, std::vector<int64_t>& soff) {
  m.ndim = st.ndim;
  int64_t stride = 1;
  for (int i = st.ndim - 1; i >= 0; --i) {
    m.dstride[i] = stride;
    stride *= st.legs[i].size();
  }
  for (int i = 0; i < st.ndim; ++i) {
    m.sbase[i] = (int)soff.size();
    int64_t o = 0;
    for (int k = 0; k < st.legs[i].nsect(); ++k) {
      soff.push_back(o);
      o += st.legs[i].d[k];
    }
  }
}

template <int DIR>
static void dense_io(const Tensor& t, void* dense, hipStream_t s) {
  const Structure& st = t.S();
  if (st.size == 0) return;
  if (st.ndim == 0) {
    if (DIR == 0)
      HIPC(hipMemcpyAsync(t.data, dense, t.esize(), hipMemcpyDeviceToDevice, s));
    else
      HIPC(hipMemcpyAsync(dense, t.data, t.esize(), hipMemcpyDeviceToDevice, s));
    return;
  }
  DenseMap m;
  std::vector<int64_t> soff;
  dense_map(st, m, soff);
  DBuf<int64_t> dso = to_device(soff, s);
  const int T = 256;
  dim3 g((unsigned)cdiv(st.size, T));
  if (t.dtype == FTN_F64)
    LAUNCH((k_dense_blocks<double, DIR>), g, dim3(T), 0, s, m, st.d_keys.p, st.d_shapes.p,
                       st.d_offsets.p, st.nblocks, st.size, dso.p, (double*)t.data, (double*)dense);
  else
    LAUNCH((k_dense_blocks<float, DIR>), g, dim3(T), 0, s, m, st.d_keys.p, st.d_shapes.p,
                       st.d_offsets.p, st.nblocks, st.size, dso.p, (float*)t.data, (float*)dense);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(s));  // soff / dso lifetime
}

void gather_dense(Tensor& t, const void* dense, hipStream_t s) { dense_io<0>(t, const_cast<void*>(dense), s); }

void scatter_dense(const Tensor& t, void* dense, hipStream_t s) {
  size_t n = 1;
  for (auto& l : t.legs()) n *= (size_t)l.size();
  HIPC(hipMemsetAsync(dense, 0, n * t.esize(), s));
  dense_io<1>(t, dense, s);
}

// ---------------------------------------------------------------------------
// elementwise
template <typename T>
__global__ void k_scale(const T* __restrict__ x, T* __restrict__ y, int64_t n, T a) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}

template <typename S, typename D>
__global__ void k_cast(const S* __restrict__ x, D* __restrict__ y, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = (D)x[i];
}

std::unique_ptr<Tensor> op_scale(const Tensor& a, double alpha, hipStream_t s) {
  auto out = make_tensor(a.st, a.dtype, s, false);
  int64_t n = a.size();
  if (n) {
    dim3 g((unsigned)cdiv(n, 256));
    if (a.dtype == FTN_F64)
      LAUNCH(k_scale<double>, g, dim3(256), 0, s, (const double*)a.data, (double*)out->data, n, alpha);
    else
      LAUNCH(k_scale<float>, g, dim3(256), 0, s, (const float*)a.data, (float*)out->data, n,
                         (float)alpha);
    HIPC(hipGetLastError());
  }
  return out;
}

std::unique_ptr<Tensor> op_cast(const Tensor& a, int dtype, hipStream_t s) {
  auto out = make_tensor(a.st, dtype, s, false);
  int64_t n = a.size();
  if (!n) return out;
  dim3 g((unsigned)cdiv(n, 256));
  if (a.dtype == dtype) {
    HIPC(hipMemcpyAsync(out->data, a.data, n * a.esize(), hipMemcpyDeviceToDevice, s));
  } else if (a.dtype == FTN_F64) {
    LAUNCH((k_cast<double, float>), g, dim3(256), 0, s, (const double*)a.data, (float*)out->data, n);
  } else {
    LAUNCH((k_cast<float, double>), g, dim3(256), 0, s, (const float*)a.data, (double*)out->data, n);
  }
  HIPC(hipGetLastError());
  return out;
}

// max |x| over the data (two-pass: per-workgroup maxima, then one workgroup)
template <typename T>
__global__ void k_absmax(const T* __restrict__ x, int64_t n, double* part) {
  __shared__ double sh[256];
  double m = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double v = fabs((double)x[i]);
    m = v > m ? v : m;
  }
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_max_reduce(const double* part, int n, double* out) {
  __shared__ double sh[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, part[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

double op_max_abs(const Tensor& a, hipStream_t s) {
  int64_t n = a.size();
  if (!n) return 0.0;
  int nb = (int)std::min<int64_t>(1024, cdiv(n, 256));
  DBuf<double> part(nb + 1, s);
  if (a.dtype == FTN_F64)
    LAUNCH(k_absmax<double>, dim3(nb), dim3(256), 0, s, (const double*)a.data, n, part.p);
  else
    LAUNCH(k_absmax<float>, dim3(nb), dim3(256), 0, s, (const float*)a.data, n, part.p);
  LAUNCH(k_max_reduce, dim3(1), dim3(256), 0, s, part.p, nb, part.p + nb);
  HIPC(hipGetLastError());
  double m = 0.0;
  HIPC(hipMemcpyAsync(&m, part.p + nb, 8, hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  return m;
}

// t <- 2^-e t with e the binary exponent of m = *mx (m = f 2^e, f in
// [1/2, 1)) when m is positive and finite; e is added to *e2
template <typename T>
__global__ void k_scale_pow2(T* __restrict__ x, int64_t n, const double* __restrict__ mx, int64_t* e2) {
  const double m = *mx;
  if (!(m > 0.0) || !isfinite(m)) return;
  int e;
  (void)frexp(m, &e);
  const T a = (T)ldexp(1.0, -e);
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i == 0) *e2 += e;
  if (i < n) x[i] = a * x[i];
}

void normalise_pow2(Tensor& t, int64_t* e2, hipStream_t s) {
  const int64_t n = t.size();
  if (!n) return;
  const int nb = (int)std::min<int64_t>(1024, cdiv(n, 256));
  DBuf<double> part(nb + 1, s);
  if (t.dtype == FTN_F64)
    LAUNCH(k_absmax<double>, dim3(nb), dim3(256), 0, s, (const double*)t.data, n, part.p);
  else
    LAUNCH(k_absmax<float>, dim3(nb), dim3(256), 0, s, (const float*)t.data, n, part.p);
  LAUNCH(k_max_reduce, dim3(1), dim3(256), 0, s, part.p, nb, part.p + nb);
  const dim3 g((unsigned)cdiv(n, 256));
  if (t.dtype == FTN_F64)
    LAUNCH(k_scale_pow2<double>, g, dim3(256), 0, s, (double*)t.data, n, part.p + nb, e2);
  else
    LAUNCH(k_scale_pow2<float>, g, dim3(256), 0, s, (float*)t.data, n, part.p + nb, e2);
  HIPC(hipGetLastError());
}

template <typename T>
__global__ void k_axpy(T* __restrict__ y, const T* __restrict__ x, int64_t n, T alpha) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] += alpha * x[i];
}

std::unique_ptr<Tensor> op_axpy(double alpha, const Tensor& x, const Tensor& y, hipStream_t s) {
  if (x.st->skey != y.st->skey) fail(FTN_EINVAL, "axpy: the tensors must have the same structure");
  if (x.dtype != y.dtype) fail(FTN_ENOTSUP, "axpy: the tensors must have the same dtype");
  auto out = make_tensor(y.st, y.dtype, s, false);
  const int64_t n = y.size();
  if (!n) return out;
  HIPC(hipMemcpyAsync(out->data, y.data, n * y.esize(), hipMemcpyDeviceToDevice, s));
  const dim3 g((unsigned)cdiv(n, 256));
  if (y.dtype == FTN_F64)
    LAUNCH(k_axpy<double>, g, dim3(256), 0, s, (double*)out->data, (const double*)x.data, n, alpha);
  else
    LAUNCH(k_axpy<float>, g, dim3(256), 0, s, (float*)out->data, (const float*)x.data, n, (float)alpha);
  HIPC(hipGetLastError());
  return out;
}

void scale_inplace(Tensor& t, double alpha, hipStream_t s) {
  int64_t n = t.size();
  if (!n) return;
  dim3 g((unsigned)cdiv(n, 256));
  if (t.dtype == FTN_F64)
    LAUNCH(k_scale<double>, g, dim3(256), 0, s, (const double*)t.data, (double*)t.data, n, alpha);
  else
    LAUNCH(k_scale<float>, g, dim3(256), 0, s, (const float*)t.data, (float*)t.data, n, (float)alpha);
  HIPC(hipGetLastError());
}

}  // namespace ftn
