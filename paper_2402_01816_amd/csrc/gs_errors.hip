// Device-side failures of asynchronous calls: the error words of a call's
// control areas, the per-device sticky flags they are collected into, and the
// test setting of the bounded waits.
//
// A kernel that meets a failure it cannot return (a bounded wait that gave up,
// a work capacity exceeded, segment offsets that are not monotone) sets a word
// in the call's workspace.  A call made with a report reads those words after
// synchronising; every call, with or without a report, also ORs them into
// flags that live in device memory for the life of the process (one set per
// device), so a caller that never asks for a report can still find out.
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>

#include "gs_internal.h"

namespace gs {

// the sticky flags: word 0 holds the DEVERR_* bits of every call so far
__device__ __align__(256) unsigned sticky_flags[64];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_sticky_mu;
unsigned *g_sticky_ptr[kMaxDevices] = {};
std::atomic<unsigned> g_test_wait{0};

// Address of the current device's copy of sticky_flags, looked up once per
// device (each device holds its own copy at its own address).
hipError_t sticky_ptr(unsigned **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_sticky_mu);
    if (!g_sticky_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(sticky_flags));
        if (e != hipSuccess) return e;
        g_sticky_ptr[dev] = (unsigned *)p;
    }
    *out = g_sticky_ptr[dev];
    return hipSuccess;
}

}  // namespace

unsigned test_wait_word() { return g_test_wait.load(std::memory_order_relaxed); }
void set_test_wait_word(unsigned w) { g_test_wait.store(w, std::memory_order_relaxed); }

__global__ void fill_ctrl_kernel(unsigned *p, int64_t count, unsigned test)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) {
        if (i == kErrWord || i == kMovedWord || i == kMovedWord + 1) continue;
        p[i] = i == kTestWord ? test : 0u;
    }
}

void launch_fill_ctrl(unsigned *ctrl, int64_t count, hipStream_t st)
{
    if (count <= 0) return;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_ctrl_kernel, dim3((unsigned)blocks), dim3(256), 0, st, ctrl, count, test_wait_word());
}

__global__ void err_begin_kernel(ErrWords e)
{
    const int i = threadIdx.x;
    if (i < e.count) e.w[i][0] = 0u;
}

__global__ void err_end_kernel(ErrWords e, unsigned *sticky)
{
    if (threadIdx.x != 0) return;
    unsigned f = 0;
    for (int i = 0; i < e.count; ++i)
        if (__hip_atomic_load(e.w[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) f |= e.bit[i];
    if (f) __hip_atomic_fetch_or(sticky, f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

hipError_t err_words_begin(const ErrWords &e, hipStream_t st)
{
    if (e.count <= 0) return hipSuccess;
    hipLaunchKernelGGL(err_begin_kernel, dim3(1), dim3(64), 0, st, e);
    return hipGetLastError();
}

hipError_t err_words_end(const ErrWords &e, hipStream_t st)
{
    if (e.count <= 0) return hipSuccess;
    unsigned *sticky = nullptr;
    hipError_t r = sticky_ptr(&sticky);
    if (r != hipSuccess) return r;
    hipLaunchKernelGGL(err_end_kernel, dim3(1), dim3(64), 0, st, e, sticky);
    return hipGetLastError();
}

hipError_t sticky_errors_read(unsigned *flags, bool clear)
{
    unsigned *sticky = nullptr;
    hipError_t e = sticky_ptr(&sticky);
    if (e != hipSuccess) return e;
    e = hipMemcpy(flags, sticky, 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && clear) {
        const unsigned zero = 0;
        e = hipMemcpy(sticky, &zero, 4, hipMemcpyHostToDevice);
    }
    return e;
}

}  // namespace gs
