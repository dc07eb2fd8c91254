// Work-group building blocks shared by the sorting kernels: the LDS layout,
// the branch-free serial merge and the stable block sort.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "gs_device.h"

namespace gs {

template <class V>
struct ValOps {
    static constexpr bool has = true;
};
template <>
struct ValOps<NoVal> {
    static constexpr bool has = false;
};

// LDS index with one pad slot per 16 elements: a thread's IPT consecutive
// outputs, and merge heads spaced about 8 apart, land in distinct banks.
__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }
// slots for TILE elements plus one readable slot past the end
template <int TILE>
constexpr int lds_slots() { return TILE + TILE / 16 + 2; }

// Serial stable merge of IPT outputs from LDS runs A = [a_base, a_base+na) and
// B = [b_base, b_base+nb) (logical LDS indices) starting at A index ai and B
// index bi; on a tie the A element goes first.  Branch free: the heads of both
// runs stay in registers, every step costs one comparison and one LDS read,
// and reads past a run's end (clamped to `limit`, a readable slot) are never
// selected.  Outputs beyond the runs' total are garbage and must be ignored.
template <class KT, int IPT, bool WANT_SRC>
__device__ __forceinline__ void serial_merge(const typename KT::T *sk, int a_base, int na, int b_base,
                                             int nb, int ai, int bi, int limit,
                                             typename KT::T (&k)[IPT], int (&src)[IPT])
{
    using K = typename KT::T;
    K va = sk[lpad(min(a_base + ai, limit))];
    K vb = sk[lpad(min(b_base + bi, limit))];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const bool takeB = (bi < nb) & ((ai >= na) | KT::less(vb, va));
        k[i] = takeB ? vb : va;
        if constexpr (WANT_SRC) src[i] = takeB ? b_base + bi : a_base + ai;
        bi += takeB ? 1 : 0;
        ai += takeB ? 0 : 1;
        const int nidx = min(takeB ? b_base + bi : a_base + ai, limit);
        const K nv = sk[lpad(nidx)];
        va = takeB ? va : nv;
        vb = takeB ? nv : vb;
    }
}

// ---------------------------------------------------------------------------
// block sort in LDS
// ---------------------------------------------------------------------------
// Sorts the TILE keys (and values) held in sk/sv (lpad layout) stably: a
// per-thread odd-even transposition sort of IPT consecutive keys (only
// adjacent strict inversions are exchanged, so equal keys keep their order),
// then merge rounds that double the sorted run length up to `maxw` (a power of
// two in [IPT, TILE]): each aligned block of maxw keys ends up sorted on its
// own, which lets one work-group sort several short arrays at once.  With
// PARTIAL, the caller guarantees that slots at or past `active` hold only
// padding, which sorts after every real key.  Then within every merge pair the
// real keys stay at the front, so slots at or past `active` hold padding after
// every round too, and a thread whose keys or outputs all lie there skips its
// work.
template <class KT, class VS, bool HV, int NT, int IPT, bool PARTIAL = false>
__device__ __forceinline__ void block_sort_lds(typename KT::T *sk, VS *sv, int maxw = NT * IPT,
                                               int active = NT * IPT)
{
    using K = typename KT::T;
    constexpr int TILE = NT * IPT;
    const int tid = threadIdx.x;
    K k[IPT];
    VS v[IPT];
    int srcix[IPT];
    const int base = tid * IPT;
    const bool work = !PARTIAL || base < active;
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        k[i] = sk[lpad(base + i)];
        if constexpr (HV) v[i] = sv[lpad(base + i)];
    }
    if (work) {
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
#pragma unroll
            for (int i = (r & 1); i + 1 < IPT; i += 2) {
                const bool sw = KT::less(k[i + 1], k[i]);
                const K lo = sw ? k[i + 1] : k[i];
                const K hi = sw ? k[i] : k[i + 1];
                k[i] = lo;
                k[i + 1] = hi;
                if constexpr (HV) {
                    const VS vlo = sw ? v[i + 1] : v[i];
                    const VS vhi = sw ? v[i] : v[i + 1];
                    v[i] = vlo;
                    v[i + 1] = vhi;
                }
            }
        }
    }
    __syncthreads();
    if (work) {
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            sk[lpad(base + i)] = k[i];
            if constexpr (HV) sv[lpad(base + i)] = v[i];
        }
    }
    __syncthreads();

    for (int w = IPT; w < maxw; w *= 2) {
        if (work) {
            const int a0 = (base / (2 * w)) * 2 * w;
            const int b0 = a0 + w;
            const int kd = base - a0;
            const int ai = merge_path_lds<KT>(kd, w, w, [&](int i) { return sk[lpad(a0 + i)]; },
                                              [&](int i) { return sk[lpad(b0 + i)]; });
            serial_merge<KT, IPT, HV>(sk, a0, w, b0, w, ai, kd - ai, TILE, k, srcix);
            if constexpr (HV) {
#pragma unroll
                for (int i = 0; i < IPT; ++i) v[i] = sv[lpad(srcix[i])];
            }
        }
        __syncthreads();
        if (work) {
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                sk[lpad(base + i)] = k[i];
                if constexpr (HV) sv[lpad(base + i)] = v[i];
            }
        }
        __syncthreads();
    }
}

// f64 blocks without NaN sort with one comparison instead of two; the choice
// is uniform per work-group.
template <class KT>
struct FastKey {
    using type = KT;
};
template <>
struct FastKey<KeyF64> {
    using type = KeyF64NoNaN;
};
template <>
struct FastKey<KeyF64Desc> {
    using type = KeyF64DescNoNaN;
};

template <class K>
__device__ __forceinline__ bool is_nan_key(K x)
{
    if constexpr (std::is_same<K, double>::value) return x != x;
    else return false;
}

}  // namespace gs
