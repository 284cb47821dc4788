// Internal declarations of the fermionic tensor library (not part of the ABI).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/ftn.h"

namespace ftn {

constexpr int MAXD = 16;  // maximum number of legs of one tensor

// ---------------------------------------------------------------------------
// errors: internal code throws Error; the C ABI catches it and returns code.
struct Error {
  int code;
  std::string msg;
};
[[noreturn]] void fail(int code, const std::string& msg);
void hip_check(hipError_t e, const char* what);
#define HIPC(x) ::ftn::hip_check((x), #x)
// host-side check of a launch configuration (names the kernel on failure)
void check_launch(const char* name, dim3 grid, dim3 block);
#define LAUNCH(kern, grid, block, shm, stream, ...)                                   \
  do {                                                                                \
    ::ftn::check_launch(#kern, (grid), (block));                                      \
    hipLaunchKernelGGL(kern, (grid), (block), (shm), (stream), __VA_ARGS__);          \
    ::ftn::hip_check(hipGetLastError(), #kern);                                       \
  } while (0)
// the same with HIP events attached to the dispatch itself (either may be
// null): the start event takes the time the kernel starts, the stop event
// the time it ends, so an event pair times exactly one kernel
#define ELAUNCH(kern, grid, block, shm, stream, ev0, ev1, ...)                               \
  do {                                                                                       \
    ::ftn::check_launch(#kern, (grid), (block));                                             \
    hipExtLaunchKernelGGL(kern, (grid), (block), (shm), (stream), (ev0), (ev1), 0, __VA_ARGS__); \
    ::ftn::hip_check(hipGetLastError(), #kern);                                              \
  } while (0)
void set_last_error(const std::string& msg);

// ---------------------------------------------------------------------------
// charges: (q0, q1); Z2 keeps q0 in {0,1}, q1 = 0.
struct Q {
  int32_t a, b;
};
__host__ __device__ inline Q q_canon(int sym, Q q) {
  if (sym == FTN_Z2) return Q{q.a & 1, 0};
  if (sym == FTN_U1) return Q{q.a, 0};
  return q;
}
__host__ __device__ inline Q q_add(int sym, Q x, Q y) { return q_canon(sym, Q{x.a + y.a, x.b + y.b}); }
__host__ __device__ inline Q q_neg(int sym, Q x) { return q_canon(sym, Q{-x.a, -x.b}); }
__host__ __device__ inline Q q_signed(int sym, int dual, Q x) { return dual ? q_neg(sym, x) : q_canon(sym, x); }
__host__ __device__ inline bool q_eq(Q x, Q y) { return x.a == y.a && x.b == y.b; }
__host__ __device__ inline bool q_lt(Q x, Q y) { return x.a < y.a || (x.a == y.a && x.b < y.b); }
__host__ __device__ inline int q_par(Q x) { return (x.a + x.b) & 1; }

// ---------------------------------------------------------------------------
struct Leg {
  std::vector<Q> q;        // sector charges, strictly ascending
  std::vector<int64_t> d;  // sector dims (> 0)
  int dual = 0;            // 0 '+', 1 '-'
  int nsect() const { return (int)q.size(); }
  int64_t size() const {
    int64_t s = 0;
    for (auto x : d) s += x;
    return s;
  }
  int find(Q c) const {
    for (int i = 0; i < nsect(); ++i)
      if (q_eq(q[i], c)) return i;
    return -1;
  }
  bool operator==(const Leg& o) const {
    if (dual != o.dual || q.size() != o.q.size()) return false;
    for (size_t i = 0; i < q.size(); ++i)
      if (!q_eq(q[i], o.q[i]) || d[i] != o.d[i]) return false;
    return true;
  }
};

// ---------------------------------------------------------------------------
// device memory
// stream-ordered device memory from the pool (any stream, the null stream
// included); persistent buffers of cached plans use hipMalloc / hipFree
void* dmalloc(size_t bytes, hipStream_t s, bool persistent = false);
void dfree(void* p, hipStream_t s, bool persistent = false);
// host-to-device copy ordered on s; small copies go through a pinned staging
// ring so that they are asynchronous, and src may be reused on return
void h2d(void* dst, const void* src, size_t bytes, hipStream_t s);

template <typename T>
struct DBuf {  // owning device buffer, released stream-ordered
  T* p = nullptr;
  size_t n = 0;
  hipStream_t s = nullptr;
  bool pers = false;
  DBuf() = default;
  DBuf(size_t n_, hipStream_t s_, bool persistent = false) : n(n_), s(s_), pers(persistent) {
    p = n ? (T*)dmalloc(n * sizeof(T), s, pers) : nullptr;
  }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept { *this = std::move(o); }
  DBuf& operator=(DBuf&& o) noexcept {
    reset();
    p = o.p; n = o.n; s = o.s; pers = o.pers;
    o.p = nullptr; o.n = 0;
    return *this;
  }
  ~DBuf() { reset(); }
  void reset() {
    if (p) dfree(p, s, pers);
    p = nullptr;
    n = 0;
  }
  void upload(const T* h, size_t cnt) {
    if (cnt) h2d(p, h, cnt * sizeof(T), s);
  }
};

// upload a host vector into a new device buffer, ordered on s (the vector
// may be released right after the call)
template <typename T>
DBuf<T> to_device(const std::vector<T>& v, hipStream_t s) {
  DBuf<T> b(v.size(), s);
  b.upload(v.data(), v.size());
  return b;
}

// Job table of a kernel that runs one workgroup (or one grid row) per job.
// Up to JT_INLINE jobs travel by value in the kernel arguments, so that the
// common case of a few sectors needs no upload; longer tables are uploaded.
constexpr int JT_INLINE = 8;
template <typename J>
struct JobTable {
  const J* p;  // uploaded table, or null: the jobs are in v
  J v[JT_INLINE];
  __device__ __forceinline__ J operator[](int64_t i) const { return p ? p[i] : v[i]; }
};
template <typename J>
struct Jobs {  // host side: the table and, for long ones, its device copy
  JobTable<J> t;
  DBuf<J> buf;
  Jobs(const J* jobs, size_t n, hipStream_t s) {
    static_assert(sizeof(JobTable<J>) <= 2048, "job table too large for the kernel arguments");
    std::memset(&t, 0, sizeof(t));
    if (n <= (size_t)JT_INLINE) {
      for (size_t i = 0; i < n; ++i) t.v[i] = jobs[i];
    } else {
      buf = DBuf<J>(n, s);
      buf.upload(jobs, n);
      t.p = buf.p;
    }
  }
  Jobs(const std::vector<J>& jobs, hipStream_t s) : Jobs(jobs.data(), jobs.size(), s) {}
};

// buffers of cached plans live for the whole process: allocated with
// hipMalloc (no stream), filled on the stream that builds the plan
template <typename T>
DBuf<T> persist(size_t n) {
  return DBuf<T>(n, nullptr, true);
}
template <typename T>
DBuf<T> persist_upload(const std::vector<T>& v, hipStream_t s) {
  DBuf<T> b(v.size(), nullptr, true);
  if (v.size()) h2d(b.p, v.data(), v.size() * sizeof(T), s);
  return b;
}

// ---------------------------------------------------------------------------
// tensors: immutable block structure (shared, cached) + data
struct Structure {
  int sym = FTN_Z2;
  int ndim = 0;
  std::vector<Leg> legs;
  Q total{0, 0};
  int64_t nblocks = 0;
  int64_t size = 0;
  std::vector<int32_t> keys;     // nblocks * ndim sector indices, lexicographic
  std::vector<int64_t> offsets;  // nblocks + 1
  std::vector<int64_t> shapes;   // nblocks * ndim
  std::vector<uint32_t> parmask; // nblocks, bit i = parity of leg i's sector
  DBuf<int32_t> d_keys;
  DBuf<int64_t> d_offsets;
  DBuf<int32_t> d_shapes;
  DBuf<uint32_t> d_parmask;
  std::string skey;
};

// structure of (sym, legs, total): enumerated on the device the first time,
// then served from a process-wide cache
std::shared_ptr<const Structure> get_structure(int sym, const std::vector<Leg>& legs, Q total,
                                               hipStream_t s);
std::string structure_key(int sym, const std::vector<Leg>& legs, Q total);

struct Tensor {
  std::shared_ptr<const Structure> st;
  int dtype = FTN_F64;
  std::shared_ptr<void> buf;  // owns the device data (shared by views)
  void* data = nullptr;
  const Structure& S() const { return *st; }
  int sym() const { return st->sym; }
  int ndim() const { return st->ndim; }
  const std::vector<Leg>& legs() const { return st->legs; }
  Q total() const { return st->total; }
  int64_t size() const { return st->size; }
  int64_t nblocks() const { return st->nblocks; }
  size_t esize() const { return dtype == FTN_F64 ? 8 : 4; }
  int parity() const { return q_par(st->total); }
};

// new tensor with the given structure; data zeroed if zero = true
std::unique_ptr<Tensor> make_tensor(int sym, int dtype, const std::vector<Leg>& legs, Q total,
                                    hipStream_t s, bool zero = true);
std::unique_ptr<Tensor> make_tensor(std::shared_ptr<const Structure> st, int dtype, hipStream_t s,
                                    bool zero = true);
int64_t block_index(const Structure& t, const int32_t* key);  // -1 if absent (host)
// a tensor sharing t's data under another structure of the same layout
std::unique_ptr<Tensor> share_tensor(const Tensor& t, std::shared_ptr<const Structure> st);
void scale_inplace(Tensor& t, double alpha, hipStream_t s);
// t <- 2^-e t, e the binary exponent of max |t| (when positive and finite),
// e added to the device counter *e2; no host synchronisation
void normalise_pow2(Tensor& t, int64_t* e2, hipStream_t s);

// leg tables passed by value to kernels
struct LegTab {
  int ndim;
  int sym;
  int nsect[MAXD];
  int base[MAXD];
  int dual[MAXD];
  Q total;
};

// flattened sector arrays of a tensor's legs, resident on the device
struct DevLegs {
  LegTab tab;
  DBuf<Q> q;
  DBuf<int64_t> d;
};
void make_devlegs(const std::vector<Leg>& legs, int sym, Q total, hipStream_t s, DevLegs& out);

// exclusive scan of n int64 values in place on the device; writes the total
// to total_out (device pointer, may be null)
void scan_exclusive(int64_t* v, int64_t n, int64_t* total_out, hipStream_t s);

// ---------------------------------------------------------------------------
// signed block <-> matrix permute (sign computation fused into the copy)
//
// A block of tensor t (legs in t's order, row-major) is mapped to a strided
// region: the destination order is perm (position p holds leg perm[p]) and is
// cut into three segments A = [0, nA), G = [nA, nA+nG), B = [nA+nG, ndim).
// Address = moff + idx_B + bext * (idx_G + gext * idx_A) where idx_X is the
// row-major index inside segment X (gext = 0 means the natural size of G).
struct SignOp {
  uint32_t kmask[MAXD];  // Koszul mask per destination position
  int perm[MAXD];
  int ndim;
  int nA, nG;
  uint32_t rev_mask;     // legs whose pairwise parity products add to the sign
  uint32_t flip_mask;    // legs whose parities add to the sign
  int phase;             // constant sign bit
};
SignOp make_signop(int ndim, const int* perm, int nA, int nG);

struct PermTask {
  int64_t block;  // block index in the tensor whose structure is given
  int64_t moff;   // strided-side element offset
  int64_t gext;   // extent of segment G when forming segment A's strides
  int64_t bext;   // extent of segment B (row length of the strided side)
  int32_t skip;   // 1: nothing to do
  int32_t extra;  // extra sign bit of this task
};

std::vector<int64_t> block_sizes(const Structure& s);

// Per-block copy descriptor, built on the device from a task: the block's
// legs with size 1 removed and neighbours that are contiguous on both sides
// merged (index 0 = innermost on the block side, block stride 1), and the
// tiling chosen for it.
struct PermDesc {
  int64_t boff;        // block offset on the block side
  int64_t moff;        // offset on the strided side
  int64_t sb[MAXD];    // merged legs: block-side strides
  int64_t ts[MAXD];    // merged legs: strided-side strides
  int32_t dim[MAXD];   // merged legs: extents
  int32_t m;           // number of merged legs
  int32_t y;           // merged leg with strided-side stride 1, or -1
  int32_t mode;        // 0 rows contiguous on both sides, 1 LDS transpose, 2 per element, 3 nothing
  int32_t ta, tr;      // tile: extent along leg 0, rows per tile (powers of two)
  int32_t neg;         // sign bit of the block
  int32_t sub;         // sub-tiles per workgroup (1 in mode 1, else up to PM_SUB)
  int64_t nx, nr;      // tiles along leg 0 and along the rows
  int64_t rows;        // rows: mode 0 all outer positions, mode 1 the extent of leg y
  int64_t nel;         // entries of the block
  int64_t nsub;        // sub-tiles of the block
};
// a ready-to-launch permute: tasks, descriptors and tile map on the device
struct PermPlan {
  SignOp op;
  DBuf<PermTask> tasks;
  DBuf<PermDesc> desc;
  DBuf<int64_t> tile_start;
  DBuf<int32_t> tile_task;  // task of each tile
  int64_t ntasks = 0, ntiles = 0;
  int64_t nelem = 0;  // elements moved per run (for the profile)
};
// builds descriptors and the tile map for the tasks of the blocks of `st`
// (synchronises s once, for the tile count)
void perm_plan_build(PermPlan& p, const Structure& st, hipStream_t s);
// dir = 0: block -> strided region; dir = 1: strided region -> block.
// `st` gives the block structure, dtype the element type. No host sync.
void run_perm(int dir, const Structure& st, int dtype, const PermPlan& p, const void* src, void* dst,
              hipStream_t s, double alpha = 1.0);

// device key matching for unary ops: source block b maps to the output block
// whose key is (remap[leg][key[perm[p]]])_p; fills tasks (moff = offset of the
// output block, single segment)
void unary_tasks(const Structure& src, const Structure& dst, const SignOp& op,
                 const std::vector<int32_t>& remap, const std::vector<int>& remap_base,
                 DBuf<PermTask>& tasks, hipStream_t s);

// ---------------------------------------------------------------------------
// grouped GEMM
struct GemmGroup {
  int64_t M, N, K;
  int64_t a_off, b_off;  // element offsets into the A / B matrix buffers
  int64_t lda, ldb;
  int32_t transA, transB;
  // output: a plain matrix (c_off, ldc), a block scatter (scatter == 1) or a
  // split-K partial into the plan's workspace (scatter == 2, at c_off, ldc)
  int64_t c_off, ldc;
  // scatter tables (when scatter == 1): row combos / col combos of the group
  int32_t scatter;
  // sym: op(A) op(B) is symmetric (M == N, B the transpose of A); only the
  // tiles on and above the diagonal are multiplied and the result is
  // mirrored, so C is still written in full
  int32_t sym;
  int32_t nrc, ncc;         // number of row / col combos
  // neg: the group's product enters its output negated (the sign of an
  // operand block that is read in place instead of through a signed permute)
  int32_t neg, pad;
  int64_t rc_base, cc_base; // offsets into the combo start arrays
  int64_t boff_base;        // offset into block offset table (nrc * ncc)
  int64_t tile0;            // first tile index of this group
  int64_t ntm, ntn;         // tiles along M and N
};
struct GemmScatter {
  const int64_t* rc_start;  // per row combo: first row; terminated per group by M
  const int64_t* cc_start;  // per col combo: first col
  const int64_t* cc_dim;    // per col combo: its dim (row length in the block)
  const int64_t* boff;      // block offsets into C
};
// split-K reduction of one plain output: C = alpha * sum_q W[w_off + q M N]
// (+ beta C); e0 = first element of this output in the reduction grid
struct SplitRed {
  int64_t M, N, c_off, ldc, w_off, e0;
  int S;
  int sym;  // element (m, n) with m > n is taken from the partials at (n, m)
};
// a ready-to-launch grouped GEMM (group table resident on the device). Groups
// whose tiles alone cannot fill the chip are cut into K slices that write
// partial sums (GemmGroup::scatter == 2) reduced by a second kernel.
struct GemmPlan {
  std::vector<GemmGroup> host;
  DBuf<GemmGroup> groups;
  std::vector<SplitRed> red_host;
  DBuf<SplitRed> red;
  int64_t ntiles = 0;
  int64_t ws_elems = 0, red_elems = 0;
  double flops = 0;
  int kind = FTN_GEMM_F64;
  int cfg = 0;
  int64_t split = 1;
  double abytes = 0;  // algorithmic bytes per run: entries of A, B and C once (FP64 count)
};
void gemm_plan(GemmPlan& p, const std::vector<GemmGroup>& groups, int kind, hipStream_t s,
               bool persistent = false);
// the same with the tile configuration (0 .. gemm_ncfg()-1) and the split-K
// factor given (-1: the built-in heuristic)
void gemm_plan_with(GemmPlan& p, const std::vector<GemmGroup>& groups, int kind, hipStream_t s,
                    bool persistent, int cfg, int split);
int gemm_ncfg();
// a plan for these groups from the process-wide cache of grouped-product
// plans (built, uploaded and completed on s on a miss)
std::shared_ptr<const GemmPlan> gemm_plan_cached(const std::vector<GemmGroup>& groups, int kind, hipStream_t s);
// tile autotuner: the (cfg, split) for these groups from the tuning cache, or
// tuned now (tuning mode), or -1 / -1 (the built-in heuristic)
void tune_choice(const std::vector<GemmGroup>& gs, int kind, hipStream_t s, int* cfg, int* split);
// C[g] = alpha * op(A[g]) op(B[g]) (+ beta C for plain outputs). No host sync.
// ws (may be null): caller-owned split-K workspace of p.ws_elems entries;
// without it the workspace is taken from the caching allocator
void run_gemm(const GemmPlan& p, int dtype, const void* A, const void* B, void* C,
              const GemmScatter* sc, hipStream_t s, double alpha = 1.0, double beta = 0.0,
              void* ws = nullptr);
// one-off convenience: plan + run (the plan's table is freed stream-ordered)
void run_grouped_gemm(int gemm, int dtype, const std::vector<GemmGroup>& groups, const void* A,
                      const void* B, void* C, const GemmScatter* sc, hipStream_t s,
                      double alpha = 1.0, double beta = 0.0);
double gemm_flops(const std::vector<GemmGroup>& groups);

// ---------------------------------------------------------------------------
// operations
std::unique_ptr<Tensor> op_ftranspose(const Tensor& a, const std::vector<int>& perm, hipStream_t s);
std::unique_ptr<Tensor> op_flip_dual(const Tensor& a, int leg, int with_sign, hipStream_t s);
std::unique_ptr<Tensor> op_dagger(const Tensor& a, hipStream_t s);
std::unique_ptr<Tensor> op_fuse(const Tensor& a, const std::vector<int>& legs, int conv, int rev,
                                hipStream_t s);
std::unique_ptr<Tensor> op_fuse_backward(const Tensor& a, const std::vector<int>& glegs, int conv, int rev,
                                         const Tensor& dout, hipStream_t s);
std::unique_ptr<Tensor> op_scale(const Tensor& a, double alpha, hipStream_t s);
// alpha * x + y (same structure and dtype) as a new tensor
std::unique_ptr<Tensor> op_axpy(double alpha, const Tensor& x, const Tensor& y, hipStream_t s);
std::unique_ptr<Tensor> op_cast(const Tensor& a, int dtype, hipStream_t s);
std::unique_ptr<Tensor> op_leg_sign(const Tensor& a, int leg, hipStream_t s);
std::unique_ptr<Tensor> op_ftensordot(const Tensor& a, const Tensor& b, const std::vector<int>& axa,
                                      const std::vector<int>& axb, int conv, int gemm, hipStream_t s,
                                      double* flops = nullptr);
struct CompressResult {
  std::unique_ptr<Tensor> a, b;
  double discarded = 0.0;
  std::vector<double> svals;
  bool near_tie = false;
  // textbook flops of the decomposition per bond sector (m >= n): QR of A~
  // and LQ of B~ with thin Q, 4 m n^2 - 4 n^3 / 3 each; thin SVD of the
  // r_A x r_B core, 14 m n^2 + 8 n^3; absorbing the kept k vectors into both
  // tall factors, 2 M r_A k + 2 N r_B k
  double textbook_flops = 0.0;
};
CompressResult op_compress_bond(const Tensor& a, const Tensor& b, int la, int lb, int64_t chi,
                                double cutoff, int conv, hipStream_t s);
// cotangents (da, db) of compress_bond for cotangents (dao, dbo) of its
// outputs (kept counts fixed; FP64; bond sectors up to 128)
void op_compress_bond_backward(const Tensor& a, const Tensor& b, int la, int lb, int64_t chi, double cutoff,
                               int conv, const Tensor& dao, const Tensor& dbo, hipStream_t s,
                               std::unique_ptr<Tensor>& da, std::unique_ptr<Tensor>& db);
double op_max_abs(const Tensor& a, hipStream_t s);  // synchronises

// contraction plans (shared with the compression code)
struct DotPlan;
struct DotPlanView {
  std::vector<GemmGroup> groups;
  std::vector<Q> gq;  // contracted charge of each group
  const PermPlan* pa;
  const PermPlan* pb;
  int64_t asz, bsz;
};
std::shared_ptr<DotPlan> dot_plan(const Tensor& a, const Tensor& b, const std::vector<int>& axa,
                                  const std::vector<int>& axb, int conv, int gemm, hipStream_t s);
DotPlanView dot_plan_view(const DotPlan& p);
// the cached plan of a contraction, or null if none was built (no allocation)
std::shared_ptr<DotPlan> dot_plan_lookup(const Tensor& a, const Tensor& b, const std::vector<int>& axa,
                                         const std::vector<int>& axb, int conv, int gemm);
// op_ftensordot with a cached plan, every temporary in `scratch` (device,
// `scratch_bytes`) and the output blocks written to `out` (device, out_elems
// entries in the output structure's block layout); allocates nothing
void op_ftensordot_into(const Tensor& a, const Tensor& b, const std::vector<int>& axa,
                        const std::vector<int>& axb, int conv, int gemm, hipStream_t s, void* out,
                        int64_t out_elems, char* scratch, size_t scratch_bytes);
// the fused per-group matrices (group g: M_g x N_g row-major at f_off[g], the
// GEMM output layout before the block scatter) of a tensor c that has the
// plan's output structure; F may be null to get only the size
int64_t dot_gather_output(const DotPlan& P, const Tensor& c, double* F, std::vector<int64_t>& f_off,
                          hipStream_t s);
// adjoint of op_ftensordot: da, db (structures of a, b) from dc
void op_ftensordot_backward(const Tensor& a, const Tensor& b, const Tensor& dc, const std::vector<int>& axa,
                            const std::vector<int>& axb, int conv, int gemm, hipStream_t s,
                            std::unique_ptr<Tensor>& da, std::unique_ptr<Tensor>& db);

// block copies between dense and block layouts
void gather_dense(Tensor& t, const void* dense, hipStream_t s);
void scatter_dense(const Tensor& t, void* dense, hipStream_t s);

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// event timing of instrumented launches (profile.hip)
bool prof_on();
void* prof_begin(hipStream_t s);
// the start (which = 0) or stop (1) event of a timing token, null without one;
// the launch being timed takes them (ELAUNCH)
hipEvent_t prof_ev(void* tok, int which);
// bytes: algorithmic bytes of the launch (operands read once, results written once)
void prof_end(void* tok, hipStream_t s, int cls, double work, double bytes = 0.0);
// suppress instrumentation on the calling thread (library worker threads)
void prof_quiet(bool on);

}  // namespace ftn
