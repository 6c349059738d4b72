// noalloc.hip -- the fixed scratch area behind lsp_periodogram_noalloc.
//
// The array lives in device memory for as long as the library stays loaded:
// each GPU the library runs on holds its own copy at its own address.  In
// host code `scratch` names a host-side stand-in, not device memory, so host
// code never passes it to a kernel or a copy: it asks noalloc_scratch() for
// the device address, which is looked up once per device (with that device
// current) and kept.
#include <mutex>

#include "internal.h"

namespace lsp {

static __device__ __align__(256) unsigned char scratch[LSP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

hipError_t noalloc_scratch(int dev, void **ptr, size_t *bytes)
{
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *bytes = sizeof(scratch);
    return hipSuccess;
}

}  // namespace lsp
