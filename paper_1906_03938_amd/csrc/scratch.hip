// The library's static device scratch array: the workspace of contour_moments_noalloc, the
// entry point for callers that cannot allocate device memory.  Every GPU the library runs on
// holds its own copy (kScratchBytes) from the code object's load until the process ends;
// every allocation-free call on a GPU shares that GPU's copy, so such calls must not overlap
// in time on one device, and each call writes every byte it later reads.
#include <mutex>

#include "internal.h"

namespace bemrat {

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void *g_addr[kMaxDevices] = {};

}  // namespace

// Device address of the current device's scratch array.  In host code `scratch` names a
// host-side stand-in, not device memory, so the address is taken once per device (with that
// device current) from the runtime and cached; kernels receive it as an argument.
hipError_t scratch_region(void **ptr, size_t *bytes) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_addr[dev] = p;
    }
    *ptr = g_addr[dev];
    *bytes = kScratchBytes;
    return hipSuccess;
}

}  // namespace bemrat
