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
__device__ __forceinline__ constexpr int lpad(int i) { return i + (i >> 4); }
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

// The register phase of the block sort for float64 blocks whose equal keys are
// bit for bit identical, 16 keys per thread: Batcher's network on each
// thread's keys, then up to four bitonic merge levels across 2, 4, 8 and 16
// lanes, so that runs of w = min(maxw, 256) keys end up sorted -- in the
// order DIR where w == maxw, else alternately in order and reversed (run r
// reversed when r is odd), the layout the LDS rounds take.
//
// Every compare-exchange is one instruction per key by a sign convention: a
// lane whose keys must come out in descending value order (a block sorted in
// reverse, or the lane that keeps the larger keys of a cross-lane pair) holds
// its keys negated, so that sorting ascending in storage sorts it the way it
// needs.  A cross-lane pair always has one plain and one negated lane, and
// both keep min(own, -partner): the plain one the smaller key, the negated one
// the negated larger key.  Between stages the lanes whose role changes negate
// their keys (a multiply by -1, exact for the finite and infinite keys these
// blocks hold).  The merge levels: 2 lanes (half-cleaner on lane bit 0, then
// in-register half-cleaners), 4 lanes (half-cleaners on lane bits 1 and 0; its
// runs all ascend, which the next level needs), 8 lanes (a flip that pairs
// lane t with 7 - t and register r with 15 - r, then half-cleaners on lane
// bits 1 and 0) and 16 lanes (half-cleaners on lane bits 3 to 0; lane t ^ 8
// is a rotation of the 16-lane row by 8, lane t ^ 4 the quad reversal of the
// 8-lane mirror).  Position bit 4 + j is lane bit j.  Every lane of the wave
// must execute this (DPP reads neighbours).
template <int DIR, int IPT>
__device__ __forceinline__ void register_sort_identical(double (&k)[IPT], int maxw)
{
    static_assert(IPT == 16, "lane bit j is position bit 4 + j");
    // (the lane is made opaque: inside a loop over leaves the values derived
    // from it would otherwise be hoisted out of the loop and spilled)
    unsigned lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));
    const bool b0 = lane & 1, b1 = (lane >> 1) & 1, b2 = (lane >> 2) & 1, b3 = (lane >> 3) & 1,
               b4 = (lane >> 4) & 1;
    const bool neg = DIR < 0;
    bool cur = false;
    auto set_mode = [&](bool m) {
        // kept a multiply (an empty asm hides that s is +-1): its result is a
        // canonical float, so the min and max that follow need no extra
        // canonicalising instruction, as a sign flip on the bits would
        double s = m != cur ? -1.0 : 1.0;
        asm volatile("" : "+v"(s));
#pragma unroll
        for (int r = 0; r < IPT; ++r) k[r] *= s;
        cur = m;
    };
    // keep min(own, -partner): partner register r (MIRROR: 15 - r) of the lane QP reads
    auto cross = [&](auto qp, auto mirror) {
        constexpr int QP = decltype(qp)::value;
        constexpr bool MIRROR = decltype(mirror)::value;
        double o[IPT];
#pragma unroll
        for (int r = 0; r < IPT; ++r) o[r] = quad_swap<QP>(k[MIRROR ? IPT - 1 - r : r]);
#pragma unroll
        for (int r = 0; r < IPT; ++r) k[r] = __builtin_fmin(k[r], -o[r]);
    };
    // keep min(own, -partner) with the partner two DPP moves away (register r)
    auto cross2 = [&](auto qp1, auto qp2) {
        constexpr int QP1 = decltype(qp1)::value, QP2 = decltype(qp2)::value;
        double o[IPT];
#pragma unroll
        for (int r = 0; r < IPT; ++r) o[r] = quad_swap<QP2>(quad_swap<QP1>(k[r]));
#pragma unroll
        for (int r = 0; r < IPT; ++r) k[r] = __builtin_fmin(k[r], -o[r]);
    };
    using X1 = std::integral_constant<int, 0xB1>;    // lane t ^ 1
    using X2 = std::integral_constant<int, 0x4E>;    // lane t ^ 2
    using QR = std::integral_constant<int, 0x1B>;    // lane reversal within a quad
    using M8 = std::integral_constant<int, 0x141>;   // lane 7 - t within eight
    using R8 = std::integral_constant<int, 0x128>;   // lane t ^ 8 (a row of 16 rotated by 8)
    using Same = std::false_type;
    using Mirror = std::true_type;

    // levels 0-3 in registers; their runs alternate with position bit 4
    set_mode(neg ^ (maxw > 16 && b0));
    {
        constexpr SortNet<IPT> net = batcher_net<IPT>();
#pragma unroll
        for (int c = 0; c < net.count; ++c) {
            const double a = k[net.lo[c]], b = k[net.hi[c]];
            k[net.lo[c]] = __builtin_fmin(a, b);
            k[net.hi[c]] = __builtin_fmax(a, b);
        }
    }
    if (maxw >= 32) {                    // level 4: runs alternate with bit 5 unless last
        const bool d = maxw > 32 && b1;
        set_mode(neg ^ b0 ^ d);
        cross(X1{}, Same{});
        set_mode(neg ^ d);
        bitonic_clean_regs<1, IPT>(k);
    }
    if (maxw >= 64) {                    // level 5: every run ascends
        set_mode(neg ^ b1);
        cross(X2{}, Same{});
        set_mode(neg ^ b0);
        cross(X1{}, Same{});
        set_mode(neg);
        bitonic_clean_regs<1, IPT>(k);
    }
    if (maxw >= 128) {                   // level 6: runs alternate with bit 7 unless last
        const bool d = maxw > 128 && b3;
        set_mode(neg ^ b2 ^ d);
        cross(M8{}, Mirror{});
        set_mode(neg ^ b1 ^ d);
        cross(X2{}, Same{});
        set_mode(neg ^ b0 ^ d);
        cross(X1{}, Same{});
        set_mode(neg ^ d);
        bitonic_clean_regs<1, IPT>(k);
    }
    if (maxw >= 256) {                   // level 7: runs alternate with bit 8 unless last
        const bool d = maxw > 256 && b4;
        set_mode(neg ^ b3 ^ d);
        cross(R8{}, Same{});
        set_mode(neg ^ b2 ^ d);
        cross2(M8{}, QR{});
        set_mode(neg ^ b1 ^ d);
        cross(X2{}, Same{});
        set_mode(neg ^ b0 ^ d);
        cross(X1{}, Same{});
        set_mode(neg ^ d);
        bitonic_clean_regs<1, IPT>(k);
    }
    set_mode(false);
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

// Byte offset of logical LDS index i in the lpad layout.  For a base b that is
// a multiple of 16, lpad8(b + x) == lpad8(b) + lpad8(x).
__device__ __forceinline__ unsigned lpad8(unsigned i) { return (i + (i >> 4)) << 3; }

// The LDS merge rounds of the block sort for blocks whose equal keys are bit
// for bit identical, on runs stored alternately in order and reversed (run r
// of a round reversed when r is odd): the first run of a pair is read from
// its start, the second from its end, so the two heads a thread merges never
// leave the pair -- a run that runs out continues into the other run's
// largest keys, which come out no earlier than the keys still needed (equal
// ones are identical) -- and the serial merge needs no bounds checks.  Each
// step keeps the two heads as (kept, new): the output is the first of them,
// the kept one the second, and the run the next head comes from follows from
// the comparison and the previous step's run.  Merge
// pairs, thread positions and the reversed second views all start at
// multiples of 16, where the pad layout is linear, so every probe address is
// a per-pair base plus lpad8 of a small index.  Every thread holds IPT sorted
// keys of runs of w0 (positions IPT*thread ..), the runs already alternately
// in order and reversed when w0 < maxw; on return sk holds every aligned block
// of maxw keys sorted in order.  Threads whose maxw block starts at or past
// `active` hold only padding and skip the work.
template <class KT, int DIR, int NT, int IPT>
__device__ __forceinline__ void block_merge_rounds_identical(typename KT::T *sk, typename KT::T (&k)[IPT], int w0,
                                                             int maxw, int active)
{
    static_assert(IPT == 16, "the address arithmetic assumes 16 keys per thread, the pad period");
    using K = typename KT::T;
    char *lb = reinterpret_cast<char *>(sk);
    unsigned tix = threadIdx.x;
    asm volatile("" : "+v"(tix));                   // (not hoisted out of a loop over leaves)
    const unsigned base = tix * IPT;
    const bool work = base < (((unsigned)active + maxw - 1) & ~(unsigned)(maxw - 1));
    if (work) {
        const unsigned b8 = lpad8(base);
#pragma unroll
        for (int i = 0; i < IPT; ++i) *reinterpret_cast<K *>(lb + b8 + 8u * i) = k[i];
    }
    __syncthreads();
    for (unsigned w = w0; w < (unsigned)maxw; w *= 2) {
        const unsigned a0 = base & ~(2 * w - 1), kd = base - a0;
        if (work) {
            // merge-path split over views a[i] = sk[a0 + i], b[j] = sk[a0 + 2w - 1 - j]:
            // the probe pair (a[mid], b[kd - 1 - mid]) sits at a0 + mid and c0 + mid
            const unsigned c0 = a0 + 2 * w - kd;
            const unsigned pa = lpad8(a0), pc = lpad8(c0);
            unsigned lo = kd > w ? kd - w : 0, hi = kd < w ? kd : w;
            while (lo < hi) {
                const unsigned mid = (lo + hi) >> 1, pm = lpad8(mid);
                if (KT::less(*reinterpret_cast<const K *>(lb + pc + pm), *reinterpret_cast<const K *>(lb + pa + pm)))
                    hi = mid;
                else
                    lo = mid + 1;
            }
            unsigned sa = a0 + lo, sb = sa + 2 * w - 1 - kd;   // the heads of both views
            K keep = *reinterpret_cast<const K *>(lb + lpad8(sa));
            K nv = *reinterpret_cast<const K *>(lb + lpad8(sb));
            bool tb = true;                          // the run of nv: true = the second run
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                const bool lt = KT::less(nv, keep);
                tb = lt == tb;                       // the run the next head comes from
                k[i] = first_of<DIR>(keep, nv);
                keep = second_of<DIR>(keep, nv);
                if (i + 1 < IPT) {
                    const unsigned inc = tb ? 0u : 1u;
                    sa += inc;
                    sb += inc - 1u;
                    nv = *reinterpret_cast<const K *>(lb + lpad8(tb ? sb : sa));
                }
            }
        }
        __syncthreads();
        // the pair's output is run (a0 / 2w); odd ones are stored reversed
        // unless this was the last round
        const bool rev = ((base / (2 * w)) & 1) && 2 * w < (unsigned)maxw;
        if (work) {
            // two straight-line stores of the 16 keys, from one base each
            if (rev) {
                const unsigned b8 = lpad8(a0 + 2 * w - IPT - kd);
#pragma unroll
                for (int i = 0; i < IPT; ++i) *reinterpret_cast<K *>(lb + b8 + 8u * (IPT - 1 - i)) = k[i];
            } else {
                const unsigned b8 = lpad8(base);
#pragma unroll
                for (int i = 0; i < IPT; ++i) *reinterpret_cast<K *>(lb + b8 + 8u * i) = k[i];
            }
        }
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
    if constexpr (!HV && NetMinMax<KT>::dir != 0 && IPT == 16) {
        // every thread joins (padding keys are all equal, so sorting them
        // changes nothing)
        if (network) {
            register_sort_identical<NetMinMax<KT>::dir, IPT>(k, maxw);
            __syncthreads();
            block_merge_rounds_identical<KT, NetMinMax<KT>::dir, NT, IPT>(sk, k, maxw < 256 ? maxw : 256, maxw,
                                                                           active);
            return;
        }
    }
    if (work && network) {
        constexpr SortNet<IPT> net = batcher_net<IPT>();
#pragma unroll
        for (int c = 0; c < net.count; ++c) {
            const K a = k[net.lo[c]], b = k[net.hi[c]];
            if constexpr (NetMinMax<KT>::dir != 0) {
                // a compare-exchange as one min and one max
                k[net.lo[c]] = first_of<NetMinMax<KT>::dir>(a, b);
                k[net.hi[c]] = second_of<NetMinMax<KT>::dir>(a, b);
            } else {
                const bool sw = KT::less(b, a);
                k[net.lo[c]] = sw ? b : a;
                k[net.hi[c]] = sw ? a : b;
            }
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

// float64 class masks of __builtin_amdgcn_class: signalling and quiet NaN,
// negative and positive zero
constexpr int kClassNaN = 0x3, kClassNaNOrZero = 0x63;

template <class K>
__device__ __forceinline__ bool is_nan_key(K x)
{
    if constexpr (std::is_same<K, double>::value) return __builtin_amdgcn_class(x, kClassNaN);
    else return false;
}

// Keys whose ties may differ in their bits: NaN payloads and the two zeros.
// Without them, equal keys are identical.
template <class K>
__device__ __forceinline__ bool tie_bits_may_differ(K x)
{
    if constexpr (std::is_same<K, double>::value) return __builtin_amdgcn_class(x, kClassNaNOrZero);
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
