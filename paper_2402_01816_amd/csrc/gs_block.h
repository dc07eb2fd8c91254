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
// and a lookahead past a run's end is never selected.  Positions are tracked
// absolutely; a lookahead never passes its run's end and every run ends at or
// before `limit` (the tile's end, a readable slot), so only the first two
// reads need clamping.  Outputs beyond the runs' total are garbage and must be
// ignored.
template <class KT, int IPT, bool WANT_SRC>
__device__ __forceinline__ void serial_merge(const typename KT::T *sk, int a_base, int na, int b_base,
                                             int nb, int ai, int bi, int limit,
                                             typename KT::T (&k)[IPT], int (&src)[IPT])
{
    using K = typename KT::T;
    int pa = a_base + ai, pb = b_base + bi;
    const int ea = a_base + na, eb = b_base + nb;
    K va = sk[lpad(min(pa, limit))];
    K vb = sk[lpad(min(pb, limit))];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const bool takeB = (pb < eb) & ((pa >= ea) | KT::less(vb, va));
        k[i] = takeB ? vb : va;
        if constexpr (WANT_SRC) src[i] = takeB ? pb : pa;
        pb += takeB ? 1 : 0;
        pa += takeB ? 0 : 1;
        const K nv = sk[lpad(takeB ? pb : pa)];
        va = takeB ? va : nv;
        vb = takeB ? nv : vb;
    }
}

// Batcher's odd-even merge sort network on N = 2^k registers (Knuth, TAOCP
// vol. 3, 5.3.4, Algorithm M): compare-exchange (lo[c], hi[c]) in order c.
template <int N>
struct SortNet {
    int lo[N * N], hi[N * N];
    int count;
};

template <int N>
constexpr SortNet<N> batcher_net()
{
    SortNet<N> s{};
    s.count = 0;
    for (int p = 1; p < N; p *= 2)
        for (int k = p; k >= 1; k /= 2)
            for (int j = k % p; j < N - k; j += 2 * k)
                for (int i = 0; i < (k < N - j - k ? k : N - j - k); ++i)
                    if ((i + j) / (2 * p) == (i + j + k) / (2 * p)) {
                        s.lo[s.count] = i + j;
                        s.hi[s.count] = i + j + k;
                        ++s.count;
                    }
    return s;
}

// Key orders whose compare-exchange may be a min and a max: float64 blocks
// with no NaN and no signed zero, where the min and the max of two keys are
// the two keys themselves, bit for bit (equal keys are identical there).
// dir 1: ascending, -1: descending, 0: compare and select only.
template <class KT>
struct NetMinMax {
    static constexpr int dir = 0;
};
template <>
struct NetMinMax<KeyF64NoNaN> {
    static constexpr int dir = 1;
};
template <>
struct NetMinMax<KeyF64DescNoNaN> {
    static constexpr int dir = -1;
};

// A neighbour lane's key, moved with DPP (no LDS traffic): QP is the DPP
// control -- a quad permutation (0x00-0xff) or 0x141, the mirror of each
// group of eight lanes.
template <int QP>
__device__ __forceinline__ double quad_swap(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), QP, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), QP, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// One compare-exchange kept on one side: the earlier position of the pair
// keeps the key that comes first in the order, the later one the other.
template <int DIR>
__device__ __forceinline__ double keep_side(double mine, double other, bool earlier)
{
    const double mn = __builtin_fmin(mine, other), mx = __builtin_fmax(mine, other);
    return (earlier == (DIR > 0)) ? mn : mx;
}

// Sorts the IPT keys of a bitonic sequence held in registers (half-cleaners
// of strides IPT/2 .. 1, each compare-exchange one min and one max).
template <int DIR, int IPT>
__device__ __forceinline__ void bitonic_clean_regs(double (&k)[IPT])
{
#pragma unroll
    for (int s = IPT / 2; s >= 1; s /= 2) {
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            if ((i & s) == 0) {
                const double a = k[i], b = k[i + s];
                const double mn = __builtin_fmin(a, b), mx = __builtin_fmax(a, b);
                k[i] = DIR > 0 ? mn : mx;
                k[i + s] = DIR > 0 ? mx : mn;
            }
        }
    }
}

// The first merge rounds of the block sort across neighbouring lanes, for
// blocks whose equal keys are bit for bit identical: every lane holds IPT
// sorted keys (positions IPT*lane ..), and a bitonic merger (a flip stage
// pairing position p with the mirror position of the merged run, then
// half-cleaners) turns runs of IPT into runs of 2*IPT (lanes t, t^1), with
// rounds >= 2 into runs of 4*IPT (lanes of a quad) and with rounds >= 3 into
// runs of 8*IPT (eight lanes).  Any order among
// identical keys is the stable one, so the unstable merger gives the stable
// result.  Every lane of the wave must execute this (DPP reads neighbours).
template <int DIR, int IPT>
__device__ __forceinline__ void lane_merge_rounds(double (&k)[IPT], int rounds)
{
    const int lane = threadIdx.x & 63;
    if (rounds >= 1) {                   // lanes t, t^1: flip, then in-register cleaners
        double o[IPT];
#pragma unroll
        for (int r = 0; r < IPT; ++r) o[r] = quad_swap<0xB1>(k[IPT - 1 - r]);
        const bool earlier = (lane & 1) == 0;
#pragma unroll
        for (int r = 0; r < IPT; ++r) k[r] = keep_side<DIR>(k[r], o[r], earlier);
        bitonic_clean_regs<DIR, IPT>(k);
    }
    if (rounds >= 2) {                   // a quad: flip (t, 3-t), cleaner (t, t^1), in-register cleaners
        double o[IPT];
#pragma unroll
        for (int r = 0; r < IPT; ++r) o[r] = quad_swap<0x1B>(k[IPT - 1 - r]);
        const bool earlier = (lane & 2) == 0;
#pragma unroll
        for (int r = 0; r < IPT; ++r) k[r] = keep_side<DIR>(k[r], o[r], earlier);
#pragma unroll
        for (int r = 0; r < IPT; ++r) o[r] = quad_swap<0xB1>(k[r]);
        const bool earlier1 = (lane & 1) == 0;
#pragma unroll
        for (int r = 0; r < IPT; ++r) k[r] = keep_side<DIR>(k[r], o[r], earlier1);
        bitonic_clean_regs<DIR, IPT>(k);
    }
    if (rounds >= 3) {                   // eight lanes: flip (t, 7-t), cleaners (t, t^2), (t, t^1), in-register
        double o[IPT];
#pragma unroll
        for (int r = 0; r < IPT; ++r) o[r] = quad_swap<0x141>(k[IPT - 1 - r]);   // mirror within 8 lanes
        const bool earlier = (lane & 4) == 0;
#pragma unroll
        for (int r = 0; r < IPT; ++r) k[r] = keep_side<DIR>(k[r], o[r], earlier);
#pragma unroll
        for (int r = 0; r < IPT; ++r) o[r] = quad_swap<0x4E>(k[r]);
        const bool earlier2 = (lane & 2) == 0;
#pragma unroll
        for (int r = 0; r < IPT; ++r) k[r] = keep_side<DIR>(k[r], o[r], earlier2);
#pragma unroll
        for (int r = 0; r < IPT; ++r) o[r] = quad_swap<0xB1>(k[r]);
        const bool earlier1 = (lane & 1) == 0;
#pragma unroll
        for (int r = 0; r < IPT; ++r) k[r] = keep_side<DIR>(k[r], o[r], earlier1);
        bitonic_clean_regs<DIR, IPT>(k);
    }
}

// The first / second of two keys in the order DIR (1 ascending, -1
// descending), as one min and one max: exact for keys whose equal values are
// bit for bit identical (no NaN, no signed zero).
template <int DIR>
__device__ __forceinline__ double first_of(double a, double b)
{
    return DIR > 0 ? __builtin_fmin(a, b) : __builtin_fmax(a, b);
}
template <int DIR>
__device__ __forceinline__ double second_of(double a, double b)
{
    return DIR > 0 ? __builtin_fmax(a, b) : __builtin_fmin(a, b);
}

// The LDS merge rounds of the block sort for blocks whose equal keys are bit
// for bit identical, on runs stored alternately in order and reversed (run r
// of a round reversed when r is odd): the first run of a pair is read from
// its start, the second from its end, so the two heads a thread merges never
// leave the pair -- a run that runs out continues into the other run's
// largest keys, which come out no earlier than the keys still needed (equal
// ones are identical) -- and the serial merge needs no bounds checks.  Each
// step keeps the two heads as (kept, new): the output is the first of them,
// the kept one the second, and the run the next head comes from follows from
// the comparison and the previous step's run.  Every thread holds IPT sorted
// keys of runs of w0 (positions IPT*thread ..); on return sk holds every
// aligned block of maxw keys sorted in order.
template <class KT, int DIR, int NT, int IPT>
__device__ __forceinline__ void block_merge_rounds_identical(typename KT::T *sk, typename KT::T (&k)[IPT], int w0,
                                                             int maxw)
{
    using K = typename KT::T;
    const int base = threadIdx.x * IPT;
    {
        const int r0 = base / w0, off = base - r0 * w0;
        const bool rev = (r0 & 1) && w0 < maxw;
#pragma unroll
        for (int i = 0; i < IPT; ++i) sk[lpad(rev ? r0 * w0 + w0 - 1 - off - i : base + i)] = k[i];
    }
    __syncthreads();
    for (int w = w0; w < maxw; w *= 2) {
        const int a0 = (base / (2 * w)) * 2 * w, kd = base - a0, top = a0 + 2 * w - 1;
        // merge-path split: view a = sk[a0 + i], view b = sk[top - j]
        int lo = kd > w ? kd - w : 0, hi = kd < w ? kd : w;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (KT::less(sk[lpad(top - (kd - 1 - mid))], sk[lpad(a0 + mid)])) hi = mid;
            else lo = mid + 1;
        }
        int sa = a0 + lo, sb = top - (kd - lo);
        K keep = sk[lpad(sa)], nv = sk[lpad(sb)];
        bool tb = true;                  // the run of nv: true = the second run
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            const bool lt = KT::less(nv, keep);
            tb = lt == tb;               // the run the output comes from
            k[i] = first_of<DIR>(keep, nv);
            keep = second_of<DIR>(keep, nv);
            if (i + 1 < IPT) {
                sb -= tb ? 1 : 0;
                sa += tb ? 0 : 1;
                nv = sk[lpad(tb ? sb : sa)];
            }
        }
        __syncthreads();
        const bool rev = ((base / (2 * w)) & 1) && 2 * w < maxw;
#pragma unroll
        for (int i = 0; i < IPT; ++i) sk[lpad(rev ? top - kd - i : base + i)] = k[i];
        __syncthreads();
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
// work.  With `ties_identical` (keys only; the caller has checked that equal
// keys are bit for bit equal, so no order among them can be seen) the
// per-thread sort is Batcher's network, half the compare-exchanges of the
// transposition sort, and for float64 orders the first (up to three) merge
// rounds run across lanes in registers (lane_merge_rounds) instead of
// through LDS.
template <class KT, class VS, bool HV, int NT, int IPT, bool PARTIAL = false>
__device__ __forceinline__ void block_sort_lds(typename KT::T *sk, VS *sv, int maxw = NT * IPT,
                                               int active = NT * IPT, bool ties_identical = false)
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
    bool network = false;
    if constexpr (!HV) network = ties_identical;
    if (work && network) {
        constexpr SortNet<IPT> net = batcher_net<IPT>();
#pragma unroll
        for (int c = 0; c < net.count; ++c) {
            const K a = k[net.lo[c]], b = k[net.hi[c]];
            const bool sw = KT::less(b, a);
            k[net.lo[c]] = sw ? b : a;
            k[net.hi[c]] = sw ? a : b;
        }
    } else if (work) {
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
    // identical ties: the first rounds across lanes, in registers (every lane
    // of the wave joins; lanes past `active` hold padding, which stays behind)
    int w0 = IPT;
    if constexpr (!HV && NetMinMax<KT>::dir != 0) {
        if (network) {
            const int rounds = maxw >= 8 * IPT ? 3 : maxw >= 4 * IPT ? 2 : maxw >= 2 * IPT ? 1 : 0;
            lane_merge_rounds<NetMinMax<KT>::dir, IPT>(k, rounds);
            w0 = IPT << rounds;
            // a whole block: the remaining rounds on alternately reversed runs
            if constexpr (!PARTIAL) {
                __syncthreads();
                block_merge_rounds_identical<KT, NetMinMax<KT>::dir, NT, IPT>(sk, k, w0, maxw);
                return;
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

    for (int w = w0; w < maxw; w *= 2) {
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

// Keys whose ties may differ in their bits: NaN payloads and the two zeros.
// Without them, equal keys are identical.
template <class K>
__device__ __forceinline__ bool tie_bits_may_differ(K x)
{
    if constexpr (std::is_same<K, double>::value) return x != x || x == 0.0;
    else return true;
}

// Order properties of one neighbour pair (a, b) under the key order KT, as
// bits that stay set only while every pair has them: bit 0 in order
// (b not before a), bit 1 strictly decreasing, bit 2 non-increasing, bit 3
// neither key one whose ties could differ in their bits.  A run whose pairs
// all keep bit 0 is already sorted; one whose pairs all keep bit 1 -- or,
// keys without values, bits 2 and 3 -- is sorted by one reversal.
template <class KT>
__device__ __forceinline__ unsigned order_bits(typename KT::T a, typename KT::T b)
{
    return (!KT::less(b, a) ? 1u : 0u) | (KT::less(b, a) ? 2u : 0u) | (!KT::less(a, b) ? 4u : 0u) |
           (!tie_bits_may_differ(a) && !tie_bits_may_differ(b) ? 8u : 0u);
}

// Whether the properties still possible can decide anything (otherwise the
// run must be sorted and checking further pairs is pointless).
template <class KT>
__device__ __forceinline__ bool order_decisive(unsigned bits, bool keys_only)
{
    const bool rev_ties = keys_only && (bits & 4u) && (bits & 8u);
    return (bits & 1u) || (bits & 2u) || rev_ties;
}

}  // namespace gs
