// Device-side building blocks shared by the sorting kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "frog_geometry.h"

namespace gs {

// ---------------------------------------------------------------------------
// key types
// ---------------------------------------------------------------------------
// float64: IEEE `<`, NaN greater than everything and tied with every NaN,
// -0.0 tied with +0.0.  less(a,b) = a is not NaN and not (a >= b).
struct KeyF64 {
    using T = double;
    static __device__ __forceinline__ bool less(double a, double b) { return (a == a) && !(a >= b); }
    static __device__ __forceinline__ double pad() { return __builtin_nan(""); }
};

// float64 keys of a block known to hold no NaN: plain IEEE `<` (still ties
// -0.0 with +0.0).  Used where a block checked its keys first.
struct KeyF64NoNaN {
    using T = double;
    static __device__ __forceinline__ bool less(double a, double b) { return a < b; }
    static __device__ __forceinline__ double pad() { return __builtin_inf(); }
};

struct KeyU64 {
    using T = uint64_t;
    static __device__ __forceinline__ bool less(uint64_t a, uint64_t b) { return a < b; }
    static __device__ __forceinline__ uint64_t pad() { return ~(uint64_t)0; }
};

struct NoVal {};

// ---------------------------------------------------------------------------
// the logical frog space: slots [0, n) live in the caller's array, slots
// [n, n + n/2) in the half buffer
// ---------------------------------------------------------------------------
template <class T>
struct Space {
    T *D;
    T *H;
    int64_t n;
    __device__ __forceinline__ T *at(int64_t p) const { return p < n ? D + p : H + (p - n); }
};

// ---------------------------------------------------------------------------
// device-side gate: a launch whose gate word differs from `run_if` exits at
// once, so a call can enqueue alternative paths and let a device flag decide
// ---------------------------------------------------------------------------
struct Gate {
    const unsigned *p;
    unsigned run_if;
    __device__ __forceinline__ bool closed() const { return p != nullptr && *p != run_if; }
};

// ---------------------------------------------------------------------------
// merges of one launch: every node of one frog-tree level, or one explicit node
// ---------------------------------------------------------------------------
struct MergeGeo {
    int64_t n_total;
    int depth;
    int single;       // 1: the launch merges exactly the node m1
    FrogMerge m1;
    __device__ __forceinline__ FrogMerge node(int64_t idx) const
    {
        return single ? m1 : frog_merge_of(frog_node(n_total, depth, idx));
    }
};

// ---------------------------------------------------------------------------
// ordered-store protocol
// ---------------------------------------------------------------------------
// A frog merge writes into slots that still hold unread elements of its outer
// run (the leaf launch likewise writes over input chunks of other leaves).
// Every work item publishes a status word once its inputs sit in LDS, and
// before storing it waits for exactly the work items that read the slots it is
// about to overwrite (its dependency window, a range of tickets).  Those always
// hold smaller tickets, so they are already running and publish without
// waiting on anything: the waits cannot deadlock.
// Status words: (epoch << 2) | 1; epochs differ between launches of one call
// and the words are cleared at the start of every call.
enum : unsigned { ST_LOADED = 1u };

__device__ __forceinline__ unsigned ld_status(const unsigned *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_status(unsigned *p, unsigned v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Every wait is bounded: a wait that exceeds kSpinLimit polls sets *err (the
// call then reports a device error) and gives up, so no wave spins forever.
constexpr unsigned kSpinLimit = 1u << 22;

// Called by one full wavefront: returns once every ticket in [lo, hi] other
// than `self` has published its loaded status for `epoch`.
__device__ __forceinline__ void wait_window(const unsigned *status, int64_t lo, int64_t hi,
                                            int64_t self, unsigned epoch, unsigned *err)
{
    const int lane = threadIdx.x & 63;
    const unsigned want = epoch << 2;
    for (int64_t base = lo; base <= hi; base += 64) {
        const int64_t idx = base + lane;
        if (idx <= hi && idx != self) {
            unsigned spins = 0;
            unsigned st = ld_status(status + idx);
            while ((st & ~3u) != want && spins < kSpinLimit) {
                __builtin_amdgcn_s_sleep(1);
                st = ld_status(status + idx);
                ++spins;
            }
            if (spins >= kSpinLimit)
                __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ---------------------------------------------------------------------------
// merge path
// ---------------------------------------------------------------------------
// Stable merge of runs A (first in input order) and B: on a tie the A element
// comes first.  For an output prefix of length k, the number of A elements in
// it is the first a in [max(0,k-nb), min(k,na)] with less(B[k-1-a], A[a]).
template <class KT, class GetA, class GetB>
__device__ __forceinline__ int merge_path_lds(int k, int na, int nb, GetA A, GetB B)
{
    int lo = k > nb ? k - nb : 0;
    int hi = k < na ? k : na;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (KT::less(B(k - 1 - mid), A(mid))) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

}  // namespace gs
