// A streaming copy of float64 arrays: the empirical bandwidth ceiling a
// sorting pass is compared with (a pass reads and writes every key once, as a
// copy does), and the learned path's move of its sorted first half into the
// half buffer (skipped on the device when that path was rejected).
#include <hip/hip_runtime.h>

#include "gs_internal.h"

namespace gs {

namespace {

typedef double f64x2 __attribute__((ext_vector_type(2)));

constexpr int kCopyThreads = 256;
constexpr int kCopyUnroll = 4;
constexpr unsigned kCopyGroups = 16384;     // the fastest of 1024 .. 16384 work-groups measured

// 16-byte non-temporal loads and stores, four per thread in flight, over a
// grid-stride loop (both pointers 16-byte aligned)
__global__ __launch_bounds__(kCopyThreads) void copy_pairs_kernel(const f64x2 *__restrict__ src,
                                                                  f64x2 *__restrict__ dst, int64_t pairs,
                                                                  const unsigned *skip_if)
{
    if (skip_if && *skip_if) return;
    const int64_t stride = (int64_t)gridDim.x * kCopyThreads * kCopyUnroll;
    for (int64_t base = (int64_t)blockIdx.x * kCopyThreads * kCopyUnroll + threadIdx.x; base < pairs;
         base += stride) {
        f64x2 v[kCopyUnroll];
#pragma unroll
        for (int r = 0; r < kCopyUnroll; ++r) {
            const int64_t i = base + r * kCopyThreads;
            if (i < pairs) v[r] = __builtin_nontemporal_load(src + i);
        }
#pragma unroll
        for (int r = 0; r < kCopyUnroll; ++r) {
            const int64_t i = base + r * kCopyThreads;
            if (i < pairs) __builtin_nontemporal_store(v[r], dst + i);
        }
    }
}

// 8-byte elements (unaligned pairs, and the odd last element)
__global__ __launch_bounds__(kCopyThreads) void copy_single_kernel(const double *__restrict__ src,
                                                                   double *__restrict__ dst, int64_t n,
                                                                   const unsigned *skip_if)
{
    if (skip_if && *skip_if) return;
    const int64_t stride = (int64_t)gridDim.x * kCopyThreads;
    for (int64_t i = (int64_t)blockIdx.x * kCopyThreads + threadIdx.x; i < n; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

unsigned copy_grid(int64_t items, int64_t per_group)
{
    const int64_t g = (items + per_group - 1) / per_group;
    return (unsigned)(g < 1 ? 1 : g > kCopyGroups ? kCopyGroups : g);
}

}  // namespace

hipError_t copy_f64_async(const double *src, double *dst, int64_t n, hipStream_t st, const unsigned *skip_if)
{
    if (n <= 0) return hipSuccess;
    const bool aligned = ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15) == 0;
    if (aligned) {
        const int64_t pairs = n / 2;
        if (pairs > 0)
            hipLaunchKernelGGL(copy_pairs_kernel, dim3(copy_grid(pairs, kCopyThreads * kCopyUnroll)),
                               dim3(kCopyThreads), 0, st, reinterpret_cast<const f64x2 *>(src),
                               reinterpret_cast<f64x2 *>(dst), pairs, skip_if);
        if (n & 1)
            hipLaunchKernelGGL(copy_single_kernel, dim3(1), dim3(kCopyThreads), 0, st, src + (n - 1),
                               dst + (n - 1), (int64_t)1, skip_if);
    } else {
        hipLaunchKernelGGL(copy_single_kernel, dim3(copy_grid(n, kCopyThreads)), dim3(kCopyThreads), 0, st, src,
                           dst, n, skip_if);
    }
    return hipGetLastError();
}

}  // namespace gs
