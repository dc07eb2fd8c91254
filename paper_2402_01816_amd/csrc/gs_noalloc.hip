// The plain float64 sort without any allocation: its workspace (half buffer
// and control area) is a static device array, `scratch`, that every device
// the library runs on holds from the moment the library's code is loaded
// there until the process ends.
//
// Host code never passes `scratch` itself to a kernel or a copy: in host code
// the name stands for a host-side shadow, not a device address.  The device
// address is looked up once per device, with that device current, and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "gs_internal.h"

// workspace of gs_sort_f64 at buffer fraction 0.5 for every n up to
// kNoAllocMaxKeys: a half buffer of 2^21 doubles (16 MiB) plus the control
// area (under 100 KiB at 2^22 keys), rounded up to 17 MiB
static __device__ __align__(256) char scratch[gs::kNoAllocScratchBytes];

namespace gs {

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char *g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch(char **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = (char *)p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace gs
