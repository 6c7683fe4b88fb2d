// cprand_mttkrp_sampled_noalloc: the sampled MTTKRP of cprand_mttkrp_sampled
// for callers that cannot allocate device memory.  Its scratch (the partial
// products and Gram partials of the gather) lives in one fixed device array
// per GPU, declared here, instead of a caller workspace.
//
// Host code never passes `scratch` itself to a kernel: in host code that
// name is a host-side stand-in, not a device address.  The device address is
// looked up once per device (hipGetSymbolAddress, with that device current)
// and every launch receives that address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "api_internal.hpp"

namespace cprand {
namespace {

static __device__ __align__(256) unsigned char scratch[CPRAND_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch`, looked up on the first
// call made with that device current.
int scratch_address(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return set_error(CPRAND_EUNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return set_error(CPRAND_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return CPRAND_OK;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace
}  // namespace cprand

using namespace cprand;

extern "C" int cprand_mttkrp_sampled_noalloc(const cprand_tensor *X, int32_t n, const void *const *A, int32_t R,
                                             int32_t S, const int32_t *idx, const double *w, void *W, double *V,
                                             void *stream) {
    g_last_error.clear();
    int rc = check_tensor(X, "X");
    if (rc) return rc;
    const int kind = kind_of(X->dtype);
    if (kind != K_F64 && kind != K_F32 && kind != K_BF16)
        return set_error(CPRAND_EUNSUPPORTED, "cprand_mttkrp_sampled_noalloc takes F64, F32 or BF16 tensors");
    rc = check_mttkrp_args(X, n, A, R, S, idx, w, nullptr, W, V);
    if (rc) return rc;
    size_t wbytes = 0, vbytes = 0;
    mttkrp_scratch_bytes(X, n, R, S, &wbytes, &vbytes);
    const size_t need = align256(wbytes) + vbytes;
    if (need > (size_t)CPRAND_NOALLOC_SCRATCH_BYTES)
        return set_error(CPRAND_EINVAL, "this shape needs %zu bytes of scratch, more than the %zu of the fixed array",
                         need, (size_t)CPRAND_NOALLOC_SCRATCH_BYTES);
    void *base = nullptr;
    rc = scratch_address(&base);
    if (rc) return rc;
    char *b = (char *)base;
    return mttkrp_sampled_run(X, n, A, R, S, idx, w, nullptr, W, V, b, (double *)(b + align256(wbytes)), nullptr,
                              (hipStream_t)stream);
}
