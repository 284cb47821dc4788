// C ABI entry points: argument validation, handle management and error
// translation. Every call returns FTN_OK or a negative code; exceptions never
// cross this boundary.
#include <cstdio>

#include "common.h"

namespace ftn {
const char* last_error_cstr();
void set_allocator(void* (*a)(size_t, ftn_stream_t, void*), void (*f)(void*, ftn_stream_t, void*), void* ctx);
void memory_stats(int dev, int64_t* in_use, int64_t* peak, int64_t* reserved, bool reset_peak);
}  // namespace ftn

struct ftn_tensor {
  std::unique_ptr<ftn::Tensor> t;
};

using namespace ftn;

template <typename F>
static int guarded(F&& f) {
  try {
    f();
    return FTN_OK;
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return FTN_ENOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return FTN_EINVAL;
  } catch (...) {
    set_last_error("unknown internal error");
    return FTN_EINVAL;
  }
}

static ftn_tensor_t wrap(std::unique_ptr<Tensor> t) {
  auto* h = new ftn_tensor;
  h->t = std::move(t);
  return h;
}

static const Tensor& T(ftn_tensor_t h) {
  if (!h || !h->t) fail(FTN_EINVAL, "null tensor handle");
  return *h->t;
}

static std::vector<Leg> parse_legs(int sym, int ndim, const int32_t* nsect, const int32_t* charges,
                                   const int64_t* dims, const uint8_t* dual) {
  if (ndim < 0 || ndim > MAXD) fail(FTN_EINVAL, "ndim must be in [0, 16]");
  if (ndim && (!nsect || !dual)) fail(FTN_EINVAL, "null leg description");
  std::vector<Leg> legs(ndim);
  int64_t pos = 0;
  for (int i = 0; i < ndim; ++i) {
    if (nsect[i] < 0) fail(FTN_EINVAL, "negative sector count");
    if (nsect[i] && (!charges || !dims)) fail(FTN_EINVAL, "null sector arrays");
    legs[i].dual = dual[i];
    for (int k = 0; k < nsect[i]; ++k, ++pos) {
      legs[i].q.push_back(Q{charges[2 * pos], charges[2 * pos + 1]});
      legs[i].d.push_back(dims[pos]);
    }
    (void)sym;
  }
  return legs;
}

extern "C" {

const char* ftn_last_error(void) { return last_error_cstr(); }

const char* ftn_version(void) { return "ftn 0.1 gfx950"; }

int ftn_set_allocator(void* (*alloc_fn)(size_t, ftn_stream_t, void*), void (*free_fn)(void*, ftn_stream_t, void*),
                      void* ctx) {
  return guarded([&] {
    if ((alloc_fn == nullptr) != (free_fn == nullptr)) fail(FTN_EINVAL, "give both allocator functions or neither");
    set_allocator(alloc_fn, free_fn, ctx);
  });
}

int ftn_memory_stats(int device, int64_t* in_use, int64_t* peak, int64_t* reserved, int reset_peak) {
  return guarded([&] {
    int n = 0;
    HIPC(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) fail(FTN_EINVAL, "no such device");
    memory_stats(device, in_use, peak, reserved, reset_peak != 0);
  });
}

int ftn_tensor_create(ftn_sym sym, ftn_dtype dtype, int ndim, const int32_t* nsect, const int32_t* charges,
                      const int64_t* sect_dims, const uint8_t* dual, const int32_t* total_charge,
                      const void* src, ftn_stream_t stream, ftn_tensor_t* out) {
  return guarded([&] {
    if (!out || !total_charge) fail(FTN_EINVAL, "null argument");
    auto legs = parse_legs(sym, ndim, nsect, charges, sect_dims, dual);
    hipStream_t s = (hipStream_t)stream;
    auto t = make_tensor(sym, dtype, legs, Q{total_charge[0], total_charge[1]}, s, src == nullptr);
    if (src && t->size())
      HIPC(hipMemcpyAsync(t->data, src, t->size() * t->esize(), hipMemcpyDeviceToDevice, s));
    *out = wrap(std::move(t));
  });
}

int ftn_tensor_wrap(ftn_sym sym, ftn_dtype dtype, int ndim, const int32_t* nsect, const int32_t* charges,
                    const int64_t* sect_dims, const uint8_t* dual, const int32_t* total_charge, void* dev_data,
                    ftn_stream_t stream, ftn_tensor_t* out) {
  return guarded([&] {
    if (!out || !total_charge) fail(FTN_EINVAL, "null argument");
    auto legs = parse_legs(sym, ndim, nsect, charges, sect_dims, dual);
    hipStream_t s = (hipStream_t)stream;
    auto st = get_structure(sym, legs, Q{total_charge[0], total_charge[1]}, s);
    if (st->size && !dev_data) fail(FTN_EINVAL, "null data for a tensor with entries");
    if (dtype != FTN_F64 && dtype != FTN_F32) fail(FTN_EINVAL, "unknown dtype");
    auto t = std::make_unique<Tensor>();
    t->st = st;
    t->dtype = dtype;
    t->buf = std::shared_ptr<void>(dev_data, [](void*) {});  // borrowed: the caller keeps it alive
    t->data = dev_data;
    *out = wrap(std::move(t));
  });
}

int ftn_tensor_from_dense(ftn_sym sym, ftn_dtype dtype, int ndim, const int32_t* nsect, const int32_t* charges,
                          const int64_t* sect_dims, const uint8_t* dual, const int32_t* total_charge,
                          const void* dense, ftn_stream_t stream, ftn_tensor_t* out) {
  return guarded([&] {
    if (!out || !total_charge || !dense) fail(FTN_EINVAL, "null argument");
    auto legs = parse_legs(sym, ndim, nsect, charges, sect_dims, dual);
    hipStream_t s = (hipStream_t)stream;
    auto t = make_tensor(sym, dtype, legs, Q{total_charge[0], total_charge[1]}, s, false);
    gather_dense(*t, dense, s);
    *out = wrap(std::move(t));
  });
}

int ftn_tensor_to_dense(ftn_tensor_t t, void* dense, ftn_stream_t stream) {
  return guarded([&] {
    if (!dense) fail(FTN_EINVAL, "null dense pointer");
    scatter_dense(T(t), dense, (hipStream_t)stream);
  });
}

int ftn_tensor_info(ftn_tensor_t t, int* sym, int* dtype, int* ndim, int64_t* nblocks, int64_t* size,
                    int32_t total_charge[2]) {
  return guarded([&] {
    const Tensor& x = T(t);
    if (sym) *sym = x.sym();
    if (dtype) *dtype = x.dtype;
    if (ndim) *ndim = x.ndim();
    if (nblocks) *nblocks = x.nblocks();
    if (size) *size = x.size();
    if (total_charge) {
      total_charge[0] = x.total().a;
      total_charge[1] = x.total().b;
    }
  });
}

int ftn_tensor_blocks(ftn_tensor_t t, const int32_t** keys, const int64_t** offsets, const int64_t** shapes) {
  return guarded([&] {
    const Structure& s = T(t).S();
    if (keys) *keys = s.keys.data();
    if (offsets) *offsets = s.offsets.data();
    if (shapes) *shapes = s.shapes.data();
  });
}

int ftn_tensor_leg(ftn_tensor_t t, int leg, int32_t* nsect, const int32_t** charges, const int64_t** dims,
                   uint8_t* dual) {
  return guarded([&] {
    const Tensor& x = T(t);
    if (leg < 0 || leg >= x.ndim()) fail(FTN_EINVAL, "leg out of range");
    const Leg& l = x.legs()[leg];
    if (nsect) *nsect = l.nsect();
    if (charges) *charges = (const int32_t*)l.q.data();
    if (dims) *dims = l.d.data();
    if (dual) *dual = (uint8_t)l.dual;
  });
}

int ftn_tensor_data(ftn_tensor_t t, void** dev_ptr) {
  return guarded([&] {
    if (!dev_ptr) fail(FTN_EINVAL, "null pointer");
    *dev_ptr = T(t).data;
  });
}

int ftn_tensor_copy_data(ftn_tensor_t t, void* dst, ftn_stream_t stream) {
  return guarded([&] {
    const Tensor& x = T(t);
    if (!dst && x.size()) fail(FTN_EINVAL, "null destination");
    if (x.size())
      HIPC(hipMemcpyAsync(dst, x.data, x.size() * x.esize(), hipMemcpyDeviceToDevice, (hipStream_t)stream));
  });
}

int ftn_tensor_cast(ftn_tensor_t t, ftn_dtype dtype, ftn_stream_t stream, ftn_tensor_t* out) {
  return guarded([&] {
    if (!out) fail(FTN_EINVAL, "null out");
    *out = wrap(op_cast(T(t), dtype, (hipStream_t)stream));
  });
}

int ftn_tensor_scale(ftn_tensor_t t, double alpha, ftn_stream_t stream, ftn_tensor_t* out) {
  return guarded([&] {
    if (!out) fail(FTN_EINVAL, "null out");
    *out = wrap(op_scale(T(t), alpha, (hipStream_t)stream));
  });
}

int ftn_tensor_axpy(double alpha, ftn_tensor_t x, ftn_tensor_t y, ftn_stream_t stream, ftn_tensor_t* out) {
  return guarded([&] {
    if (!out) fail(FTN_EINVAL, "null out");
    *out = wrap(op_axpy(alpha, T(x), T(y), (hipStream_t)stream));
  });
}

int ftn_tensor_free(ftn_tensor_t t) {
  return guarded([&] { delete t; });
}

int ftn_ftranspose(ftn_tensor_t a, const int32_t* perm, ftn_stream_t stream, ftn_tensor_t* out) {
  return guarded([&] {
    if (!out) fail(FTN_EINVAL, "null out");
    const Tensor& x = T(a);
    if (x.ndim() && !perm) fail(FTN_EINVAL, "null permutation");
    std::vector<int> p(perm, perm + x.ndim());
    *out = wrap(op_ftranspose(x, p, (hipStream_t)stream));
  });
}

int ftn_flip_dual(ftn_tensor_t a, int leg, int with_sign, ftn_stream_t stream, ftn_tensor_t* out) {
  return guarded([&] {
    if (!out) fail(FTN_EINVAL, "null out");
    *out = wrap(op_flip_dual(T(a), leg, with_sign, (hipStream_t)stream));
  });
}

int ftn_dagger(ftn_tensor_t a, ftn_stream_t stream, ftn_tensor_t* out) {
  return guarded([&] {
    if (!out) fail(FTN_EINVAL, "null out");
    *out = wrap(op_dagger(T(a), (hipStream_t)stream));
  });
}

int ftn_fuse(ftn_tensor_t a, int nlegs, const int32_t* legs, ftn_conv conv, int rev, ftn_stream_t stream,
             ftn_tensor_t* out) {
  return guarded([&] {
    if (!out || !legs || nlegs < 1) fail(FTN_EINVAL, "bad arguments");
    std::vector<int> l(legs, legs + nlegs);
    *out = wrap(op_fuse(T(a), l, conv, rev, (hipStream_t)stream));
  });
}

int ftn_fuse_backward(ftn_tensor_t a, int nlegs, const int32_t* legs, ftn_conv conv, int rev, ftn_tensor_t dout,
                      ftn_stream_t stream, ftn_tensor_t* da) {
  return guarded([&] {
    if (!da || !legs || nlegs < 1) fail(FTN_EINVAL, "bad arguments");
    std::vector<int> l(legs, legs + nlegs);
    *da = wrap(op_fuse_backward(T(a), l, conv, rev, T(dout), (hipStream_t)stream));
  });
}

int ftn_ftensordot(ftn_tensor_t a, ftn_tensor_t b, int naxes, const int32_t* axes_a, const int32_t* axes_b,
                   ftn_conv conv, ftn_gemm gemm, ftn_stream_t stream, ftn_tensor_t* out) {
  return guarded([&] {
    if (!out || naxes < 0 || (naxes && (!axes_a || !axes_b))) fail(FTN_EINVAL, "bad arguments");
    std::vector<int> xa(axes_a, axes_a + naxes), xb(axes_b, axes_b + naxes);
    *out = wrap(op_ftensordot(T(a), T(b), xa, xb, conv, gemm, (hipStream_t)stream));
  });
}

int ftn_ftensordot_backward(ftn_tensor_t a, ftn_tensor_t b, ftn_tensor_t dc, int naxes, const int32_t* axes_a,
                            const int32_t* axes_b, ftn_conv conv, ftn_gemm gemm, ftn_stream_t stream,
                            ftn_tensor_t* da, ftn_tensor_t* db) {
  return guarded([&] {
    if (!da || !db || naxes < 0 || (naxes && (!axes_a || !axes_b))) fail(FTN_EINVAL, "bad arguments");
    std::vector<int> xa(axes_a, axes_a + naxes), xb(axes_b, axes_b + naxes);
    std::unique_ptr<Tensor> ga, gb;
    op_ftensordot_backward(T(a), T(b), T(dc), xa, xb, conv, gemm, (hipStream_t)stream, ga, gb);
    *da = wrap(std::move(ga));
    *db = wrap(std::move(gb));
  });
}

int ftn_compress_bond(ftn_tensor_t a, ftn_tensor_t b, int leg_a, int leg_b, int64_t chi, double cutoff,
                      ftn_conv conv, ftn_stream_t stream, ftn_tensor_t* a_out, ftn_tensor_t* b_out,
                      double* discarded_weight, double* svals, int64_t* nkept) {
  return guarded([&] {
    if (!a_out || !b_out) fail(FTN_EINVAL, "null out");
    if (chi < 1) fail(FTN_EINVAL, "chi must be >= 1");
    const Tensor& x = T(a);
    const Tensor& y = T(b);
    if (leg_a < 0 || leg_a >= x.ndim() || leg_b < 0 || leg_b >= y.ndim()) fail(FTN_EINVAL, "leg out of range");
    CompressResult r = op_compress_bond(x, y, leg_a, leg_b, chi, cutoff, conv, (hipStream_t)stream);
    if (discarded_weight) *discarded_weight = r.discarded;
    if (svals)
      for (size_t i = 0; i < r.svals.size(); ++i) svals[i] = r.svals[i];
    if (nkept) *nkept = (int64_t)r.svals.size();
    *a_out = wrap(std::move(r.a));
    *b_out = wrap(std::move(r.b));
  });
}

int ftn_compress_bond_backward(ftn_tensor_t a, ftn_tensor_t b, int leg_a, int leg_b, int64_t chi, double cutoff,
                               ftn_conv conv, ftn_tensor_t da_out, ftn_tensor_t db_out, ftn_stream_t stream,
                               ftn_tensor_t* da, ftn_tensor_t* db) {
  return guarded([&] {
    if (!da || !db) fail(FTN_EINVAL, "null out");
    if (chi < 1) fail(FTN_EINVAL, "chi must be >= 1");
    const Tensor& x = T(a);
    const Tensor& y = T(b);
    if (leg_a < 0 || leg_a >= x.ndim() || leg_b < 0 || leg_b >= y.ndim()) fail(FTN_EINVAL, "leg out of range");
    std::unique_ptr<Tensor> ga, gb;
    op_compress_bond_backward(x, y, leg_a, leg_b, chi, cutoff, conv, T(da_out), T(db_out), (hipStream_t)stream, ga,
                              gb);
    *da = wrap(std::move(ga));
    *db = wrap(std::move(gb));
  });
}

}  // extern "C"

// helpers for the network driver (same translation unit family)
namespace ftn {
Tensor* handle_tensor(ftn_tensor_t h) { return h ? h->t.get() : nullptr; }
ftn_tensor_t make_handle(std::unique_ptr<Tensor> t) { return wrap(std::move(t)); }
}  // namespace ftn
