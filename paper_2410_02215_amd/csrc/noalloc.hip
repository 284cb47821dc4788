// Allocation-free contraction (ftn_ftensordot_noalloc): the fused-matrix
// temporaries and the split-K workspace of a contraction live in one
// statically sized device array per GPU instead of the caching allocator, and
// the output blocks go to a caller-provided buffer.
//
// `scratch` below is a device symbol. In host code its name is not a device
// address, so host code only ever uses the address hipGetSymbolAddress
// returns for it on each device (taken once per device, with that device
// current, on the first call there) and passes that pointer to the kernels.
#include <mutex>

#include "common.h"

namespace ftn {

Tensor* handle_tensor(ftn_tensor_t h);

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;  // 64 MiB per GPU
constexpr int NOALLOC_MAX_DEVICES = 64;

static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static char* g_scratch_ptr[NOALLOC_MAX_DEVICES];

static char* scratch_on_current_device() {
  int dev = 0;
  HIPC(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) fail(FTN_ENOTSUP, "device index beyond the scratch table");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      fail(FTN_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = (char*)p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace ftn

using namespace ftn;

extern "C" int ftn_ftensordot_noalloc(ftn_tensor_t a, ftn_tensor_t b, int naxes, const int32_t* axes_a,
                                      const int32_t* axes_b, ftn_conv conv, ftn_gemm gemm,
                                      ftn_stream_t stream, void* out_data, int64_t out_size) {
  try {
    const Tensor* x = handle_tensor(a);
    const Tensor* y = handle_tensor(b);
    if (!x || !y) fail(FTN_EINVAL, "null tensor handle");
    if (naxes < 0 || naxes > MAXD || (naxes && (!axes_a || !axes_b))) fail(FTN_EINVAL, "bad axes");
    if (out_size < 0) fail(FTN_EINVAL, "negative output size");
    std::vector<int> xa(axes_a, axes_a + naxes), xb(axes_b, axes_b + naxes);
    char* ws = scratch_on_current_device();
    op_ftensordot_into(*x, *y, xa, xb, conv, gemm, (hipStream_t)stream, out_data, out_size, ws,
                       NOALLOC_SCRATCH_BYTES);
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
