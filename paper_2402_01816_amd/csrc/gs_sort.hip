// Plain frog mergesort for one array: leaf block sort fused with the setup
// placement, merge-path partition, dependency windows, and the in-place frog
// merge per level.
//
// Paper: "Symmetric merging" (mirrored child placement, merge from the inner
// ends outward), "Frogsort1" (rule 1: surplus to the outer side; rule 2:
// buffer floor(n/2); the setup recursion that places elements before merging).
#include <hip/hip_runtime.h>

#include <string.h>

#include <type_traits>

#include "gs_block.h"
#include "gs_device.h"
#include "gs_internal.h"

namespace gs {

// ---------------------------------------------------------------------------
// small utilities
// ---------------------------------------------------------------------------
__global__ void fill_u32_kernel(unsigned *p, int64_t count, unsigned v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = v;
}

void launch_fill_u32(unsigned *p, int64_t count, unsigned v, hipStream_t st)
{
    if (count <= 0) return;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, count, v);
}

// Every key is read once and written once per level: the leaf and merge
// accesses can bypass the caches' normal retention.
#ifndef GS_MERGE_NT
#define GS_MERGE_NT 1
#endif
#if GS_MERGE_NT
#define GS_MERGE_LOAD(ptr) __builtin_nontemporal_load(ptr)
#define GS_MERGE_STORE(v, ptr) __builtin_nontemporal_store((v), (ptr))
#else
#define GS_MERGE_LOAD(ptr) (*(ptr))
#define GS_MERGE_STORE(v, ptr) (*(ptr) = (v))
#endif

// ---------------------------------------------------------------------------
// leaf kernel: sort each leaf's input chunk and place it at its frog slot
// ---------------------------------------------------------------------------
// Leaf i of a problem takes the i-th contiguous chunk of its input (the order
// the setup recursion visits elements) and leaves it sorted at its data start,
// which is never before its input offset.  A leaf's output can therefore only
// cover input chunks of leaves with a larger index: leaves take tickets in
// descending index order, and each waits for the leaves whose chunks its
// output covers.  One leaf per work-group, or with PERSIST (a problem table,
// whose leaf count is on the device) work-groups take tickets until none is
// left (a leaf waits only on smaller tickets, held by work-groups already
// running), so the grid need not exceed the resident work-groups.  (The
// loop's register pressure costs the one-leaf form spills, so it stays a
// separate instance.)
// The value held by the next lane of the 16-lane row (DPP row shift; the
// last lane of a row gets its own value back).
template <class K>
__device__ __forceinline__ K lane_next(K x)
{
    static_assert(sizeof(K) == 8, "64-bit keys");
    const long long b = (long long)__builtin_bit_cast(unsigned long long, x);
    const int lo = __builtin_amdgcn_update_dpp((int)(b & 0xffffffffll), (int)(b & 0xffffffffll), 0x101, 0xF, 0xF,
                                               false);
    const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), 0x101, 0xF, 0xF, false);
    return __builtin_bit_cast(K, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Order of the chunk in sk[0, len) (lpad layout), the same answer in every
// thread: 1 if no neighbour pair is out of order, 2 if every pair strictly
// decreases, else 0.  Each thread checks the pairs that start among its IPT
// consecutive slots.
template <class KT, class VS, int NT, int IPT>
__device__ __forceinline__ int chunk_order(const typename KT::T *sk, int len)
{
    using K = typename KT::T;
    const int base = threadIdx.x * IPT;
    bool up = true, down = true;
    if (base < len - 1) {
        K prev = sk[lpad(base)];
#pragma unroll
        for (int i = 1; i <= IPT; ++i) {
            if (base + i < len) {
                const K x = sk[lpad(base + i)];
                up &= !KT::less(x, prev);
                down &= KT::less(x, prev);
                prev = x;
            }
        }
    }
    const bool not_up = __syncthreads_or(!up) != 0;
    const bool not_down = __syncthreads_or(!down) != 0;
    return !not_up ? 1 : !not_down ? 2 : 0;
}

template <class KT, class V, int NT, int IPT, int WAVES, bool F2, bool PERSIST>
__global__ __launch_bounds__(NT, WAVES) void leaf_kernel(typename KT::T *Dk, typename KT::T *Hk, V *Dv, V *Hv,
                                                  Forest F, unsigned *ticket_ctr, unsigned *status,
                                                  unsigned epoch, unsigned *err, uint64_t *moved, Gate gate)
{
    using K = typename KT::T;
    using KF = typename FastKey<KT>::type;
    constexpr bool HV = ValOps<V>::has;
    using VS = typename std::conditional<HV, V, char>::type;
    constexpr int TILE = NT * IPT;
    constexpr int SLOTS = lds_slots<TILE>();
    static_assert(NT % 16 == 0, "slot tid + r * NT pads as lpad(tid) + r * lpad(NT)");
    __shared__ K sk[SLOTS];
    __shared__ VS sv[HV ? SLOTS : 1];
    __shared__ unsigned s_ticket, s_order;
    if (gate.closed()) return;

    const int64_t L = F.probs ? (int64_t)*F.nprob : 1;
    const int64_t total = F2 ? F.f2.nleaves : F.probs ? (int64_t)F.tbase[L] : ((int64_t)1 << F.p0.depth);
    for (;;) {
        // (with PERSIST the thread index is made opaque on every pass, so that
        // values derived from it are not hoisted out of the loop, where they
        // would stay live through the whole sort and spill)
        int tid = threadIdx.x;
        if constexpr (PERSIST) asm volatile("" : "+v"(tid));
        if (tid == 0) s_ticket = atomicAdd(ticket_ctr, 1u);
        __syncthreads();
        const int64_t t = __builtin_amdgcn_readfirstlane(s_ticket);
        if (tid == 0) s_order = 0;
        __syncthreads();
        if (t >= total) break;
        Prob P = F.p0;
        int64_t base = 0;
        if (F.probs) {
            const int64_t s = forest_locate_wave(F.tbase, L, t);
            P = F.probs[s];
            base = F.tbase[s];
        }
        const int64_t nleaves = F2 ? F.f2.nleaves : ((int64_t)1 << P.depth);
        const int64_t leaf = nleaves - 1 - (t - base);
        int64_t src, dst;
        int len;
        int64_t wlo = 1, whi = 0;        // Frogsort2: dependency window, found up front
        if constexpr (F2) {
            src = F.f2.leaf_c[leaf];
            len = (int)(F.f2.leaf_c[leaf + 1] - src);
            dst = F.f2.leaf_d[leaf];
            if (dst < P.n) {
                const int64_t end = (dst + len < P.n ? dst + len : P.n) - 1;
                wlo = nleaves - 1 - locate_i64(F.f2.leaf_c, nleaves, end);
                whi = nleaves - 1 - locate_i64(F.f2.leaf_c, nleaves, dst);
            }
        } else {
            const FrogNode f = frog_node(P.n, P.depth, leaf);
            src = f.in_off;
            len = (int)f.n;
            dst = frog_data_start(f);
        }
        const Space<K> keys{Dk + P.doff, Hk + P.hoff, P.n};
        const Space<V> vals{HV ? Dv + P.doff : nullptr, HV ? Hv + P.hoff : nullptr, P.n};

        // load the chunk (input elements all live in the caller's array), all
        // loads issued before the first LDS write: a whole tile straight, a
        // short chunk from clamped indices
        bool nan_here = false, ties_identical = false;
        {
            K lk[IPT];
            VS lv[IPT];
            const K *ks = keys.D + src;
            if (len == TILE) {
                // a uniform base plus a 32-bit offset per load
                const char *kb = reinterpret_cast<const char *>(ks);
#pragma unroll
                for (int r = 0; r < IPT; ++r) {
                    lk[r] = GS_MERGE_LOAD(reinterpret_cast<const K *>(kb + (unsigned)(tid + r * NT) * sizeof(K)));
                    if constexpr (HV) lv[r] = vals.D[src + tid + r * NT];
                }
            } else {
#pragma unroll
                for (int r = 0; r < IPT; ++r) {
                    const int ic = min(tid + r * NT, len - 1);
                    lk[r] = GS_MERGE_LOAD(ks + ic);
                    if constexpr (HV) lv[r] = vals.D[src + ic];
                }
            }
            // NaN keys and zeros (the keys whose ties may differ in their
            // bits) are rare: one class test per key finds whether any is
            // here, and only then the NaNs are looked for
            bool differ = false;
#pragma unroll
            for (int r = 0; r < IPT; ++r) differ |= tie_bits_may_differ(lk[r]);
            // Squidsort: a first look at the chunk's order from the pairs
            // (i, i+1) with i = tid, the neighbour taken from the next lane
            // of the row; s_order bit 0: some pair falls, bit 1: some pair
            // does not fall (both: the chunk is neither in order nor
            // strictly decreasing)
            if (F.dirs) {
                const K nb = lane_next(lk[0]);
                const bool ok = (tid & 15) != 15 && tid + 1 < len;
                const bool falls = ok && KT::less(nb, lk[0]), rises = ok && !KT::less(nb, lk[0]);
                const unsigned bits = (__ballot(falls) ? 1u : 0u) | (__ballot(rises) ? 2u : 0u);
                if ((tid & 63) == 0 && bits) atomicOr(&s_order, bits);
            }
            const bool any_differ = __syncthreads_or(differ) != 0;
            bool any_nan = false;
            if (any_differ) {
#pragma unroll
                for (int r = 0; r < IPT; ++r) nan_here |= is_nan_key(lk[r]);
                any_nan = __syncthreads_or(nan_here) != 0;
            }
            ties_identical = !HV && !any_differ;
            // tid + r * NT with NT a multiple of 16: lpad of it is lpad(tid) + r * lpad(NT)
            const int lt = lpad(tid);
            if (len == TILE) {
#pragma unroll
                for (int r = 0; r < IPT; ++r) {
                    sk[lt + r * lpad(NT)] = lk[r];
                    if constexpr (HV) sv[lt + r * lpad(NT)] = lv[r];
                }
            } else {
                // slots past the chunk get a padding key that sorts after
                // every real key (ties with it stay behind the real keys)
                const K pad = any_nan ? KT::pad() : KF::pad();
#pragma unroll
                for (int r = 0; r < IPT; ++r) {
                    const int i = tid + r * NT;
                    sk[lt + r * lpad(NT)] = i < len ? lk[r] : pad;
                    if constexpr (HV) sv[lt + r * lpad(NT)] = i < len ? lv[r] : VS();
                }
            }
            nan_here = any_nan;
        }
        __syncthreads();
        if (tid == 0) st_status(status + t, (epoch << 2) | ST_LOADED);

        // Squidsort: a chunk already in order stays as it is (ascending run),
        // a strictly decreasing one too (descending run: reversed, it is the
        // stable result); only the others are sorted
        int ord = 0;                     // 0: to be sorted, 1: in order, 2: strictly decreasing
        if (F.dirs) {
            ord = len <= 1 ? 1 : s_order == 3u ? 0 : chunk_order<KT, VS, NT, IPT>(sk, len);
            if (tid == 0)
                F.dirs[((int64_t)1 << P.depth) - 1 + leaf] =
                    (uint8_t)(len <= 1 ? DIR_NONE : ord == 2 ? DIR_DESC : DIR_ASC);
        }
        if (tid == 0 && moved) atomicAdd((unsigned long long *)moved, (unsigned long long)len);

        // a short leaf (keys-only sorts: the forest's segments and buckets
        // have them) is sorted in the smallest power-of-two prefix holding
        // it, skipping the work on the padding past it
        if (ord != 0) {
            // nothing to sort
        } else if (HV || len == TILE) {
            if (nan_here) block_sort_lds<KT, VS, HV, NT, IPT>(sk, sv);
            else block_sort_lds<KF, VS, HV, NT, IPT>(sk, sv, TILE, TILE, ties_identical);
        } else if constexpr (!HV) {
            int maxw = IPT;
            while (maxw < len) maxw *= 2;
            if (nan_here) block_sort_lds<KT, VS, HV, NT, IPT, true>(sk, sv, maxw, len);
            else block_sort_lds<KF, VS, HV, NT, IPT, true>(sk, sv, maxw, len, ties_identical);
        }

        // wait for the leaves whose input chunks the destination covers
        if constexpr (F2) {
            if (tid < 64 && wlo <= whi) wait_window(status, wlo, whi, t, epoch, err);
        } else if (tid < 64) {
            int64_t wl, wh;
            leaf_window(P.n, P.depth, leaf, &wl, &wh);
            if (wl <= wh) wait_window(status, base + wl, base + wh, t, epoch, err);
        }
        __syncthreads();

        // run samples of the leaf's run: per stretch of samp_tile ranks its
        // first key (a left child) or its last (a right child)
        if constexpr (!F2) {
            if (F.samp && !F.probs) {
                const int nst = (len + F.samp_tile - 1) / F.samp_tile;
                if (tid < nst) {
                    const int f = tid * F.samp_tile, l = min(f + F.samp_tile, len) - 1;
                    reinterpret_cast<K *>(F.samp)[leaf * F.samp_leaf_tiles + tid] = sk[lpad(leaf & 1 ? l : f)];
                }
            }
        }

        // the destination lies in one space unless it straddles the end of
        // the caller's array
        const bool in_d = dst + len <= P.n, in_h = dst >= P.n;
        if (in_d || in_h) {
            K *ko = in_d ? keys.D + dst : keys.H + (dst - P.n);
            V *vo = nullptr;
            if constexpr (HV) vo = in_d ? vals.D + dst : vals.H + (dst - P.n);
            const int lt = lpad(tid);
            char *kb = reinterpret_cast<char *>(ko);
            if (len == TILE) {
#pragma unroll
                for (int r = 0; r < IPT; ++r) {
                    GS_MERGE_STORE(sk[lt + r * lpad(NT)], reinterpret_cast<K *>(kb + (unsigned)(tid + r * NT) * sizeof(K)));
                    if constexpr (HV) vo[tid + r * NT] = sv[lt + r * lpad(NT)];
                }
            } else {
#pragma unroll
                for (int r = 0; r < IPT; ++r) {
                    const int i = tid + r * NT;
                    if (i < len) {
                        GS_MERGE_STORE(sk[lt + r * lpad(NT)], reinterpret_cast<K *>(kb + (unsigned)i * sizeof(K)));
                        if constexpr (HV) vo[i] = sv[lt + r * lpad(NT)];
                    }
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < IPT; ++r) {
                const int i = tid + r * NT;
                if (i < len) {
                    GS_MERGE_STORE(sk[lpad(i)], keys.at(dst + i));
                    if constexpr (HV) *vals.at(dst + i) = sv[lpad(i)];
                }
            }
        }
        if constexpr (!PERSIST) break;
    }
}

// ---------------------------------------------------------------------------
// forest prefix sums: tickets and splits of every round over the problems
// ---------------------------------------------------------------------------
// One work-group per round (round 0: leaves).  A round whose totals would pass
// the capacity of the workspace arrays is cut to zero work and flags *err (the
// call then fails instead of writing out of bounds).
template <int TILE>
__global__ __launch_bounds__(1024) void forest_scan_kernel(Forest F, unsigned *tbase, unsigned *sbase,
                                                           int64_t cap_leaves, int64_t cap_tickets,
                                                           int64_t cap_splits, unsigned *err, Gate gate)
{
    constexpr int NT = 1024, PER = 4;
    __shared__ unsigned s_t[NT], s_s[NT];
    __shared__ int64_t s_carry_t, s_carry_s;
    if (gate.closed()) return;
    const int round = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t L = *F.nprob;
    unsigned *trow = tbase + (int64_t)round * F.stride;
    unsigned *srow = sbase + (int64_t)round * F.stride;
    if (tid == 0) {
        s_carry_t = 0;
        s_carry_s = 0;
    }
    __syncthreads();
    for (int64_t c0 = 0; c0 < L; c0 += NT * PER) {
        unsigned tc[PER], sc[PER], tsum = 0, ssum = 0;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int64_t s = c0 + (int64_t)tid * PER + k;
            tc[k] = sc[k] = 0;
            if (s < L) {
                const Prob P = F.probs[s];
                tc[k] = (unsigned)forest_tickets<TILE>(F, P, round);
                sc[k] = (unsigned)forest_splits<TILE>(F, P, round);
            }
            tsum += tc[k];
            ssum += sc[k];
        }
        s_t[tid] = tsum;
        s_s[tid] = ssum;
        __syncthreads();
        for (int d = 1; d < NT; d *= 2) {            // inclusive scan
            const unsigned at = tid >= d ? s_t[tid - d] : 0u;
            const unsigned as = tid >= d ? s_s[tid - d] : 0u;
            __syncthreads();
            s_t[tid] += at;
            s_s[tid] += as;
            __syncthreads();
        }
        int64_t rt = s_carry_t + s_t[tid] - tsum, rs = s_carry_s + s_s[tid] - ssum;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int64_t s = c0 + (int64_t)tid * PER + k;
            if (s < L) {
                trow[s] = (unsigned)rt;
                srow[s] = (unsigned)rs;
            }
            rt += tc[k];
            rs += sc[k];
        }
        __syncthreads();
        if (tid == NT - 1) {
            s_carry_t = rt;
            s_carry_s = rs;
        }
        __syncthreads();
    }
    if (tid == 0) {
        int64_t tt = s_carry_t, ts = s_carry_s;
        if (tt > (round == 0 ? cap_leaves : cap_tickets) || ts > cap_splits) {
            __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            tt = 0;
            ts = 0;
            for (int64_t s = 0; s < L; ++s) trow[s] = srow[s] = 0;
        }
        trow[L] = (unsigned)tt;
        srow[L] = (unsigned)ts;
    }
}

// ---------------------------------------------------------------------------
// partition kernel: merge-path splits at every tile boundary of every node
// ---------------------------------------------------------------------------
// How a node of the single Frogsort1 tree forms its run from its children's
// runs (directions dL, dR): the concatenation when both come back ascending
// and the first run's last key is not above the second run's first, or both
// descending and every key of the second run is below every key of the first
// ("Full adaptivity": the non-overlap test; "Squidsort"); otherwise an
// ascending merge, after turning a descending outer run around.  *dir
// receives the node's direction.
template <class KT>
__device__ __forceinline__ int node_kind(const Space<typename KT::T> &keys, const FrogMerge &m, int dL, int dR,
                                         unsigned *dir)
{
    if (m.nl > 0 && m.nr > 0) {
        const RunView L = view_of(m.l0, m.nl, dL == DIR_DESC), R = view_of(m.r0, m.nr, dR == DIR_DESC);
        if (dL != DIR_DESC && dR != DIR_DESC &&
            !KT::less(*keys.at(view_slot(R, 0)), *keys.at(view_slot(L, m.nl - 1)))) {
            *dir = DIR_ASC;
            return NODE_CONCAT;
        }
        if (dL != DIR_ASC && dR != DIR_ASC &&
            KT::less(*keys.at(view_slot(R, m.nr - 1)), *keys.at(view_slot(L, 0)))) {
            *dir = DIR_DESC;
            return NODE_CONCAT;
        }
    }
    const int douter = m.outer != 1 ? dL : dR;
    *dir = DIR_ASC;
    return douter == DIR_DESC ? NODE_MERGE_REV : NODE_MERGE;
}

// Merge-path split of the views' stable merge: the number of view-a
// elements among the first kk outputs.  (The searches are bound by the rate
// of random reads: one probe per step beats several probes per step.)
template <class KT>
__device__ __forceinline__ int64_t view_split(const Space<typename KT::T> &keys, const NodeViews &v, int64_t kk)
{
    int64_t lo = kk > v.b.n ? kk - v.b.n : 0;
    int64_t hi = kk < v.a.n ? kk : v.a.n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (KT::less(*keys.at(view_slot(v.b, kk - 1 - mid)), *keys.at(view_slot(v.a, mid)))) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// The same split for a plain merge of two ascending runs whose run samples
// the previous round left (sa: the first keys of the first run's stretches of
// T ranks, sb: the last keys of the second run's) and kk a multiple of T below the node's
// size.  The merge-path predicate (the first run's element i comes before the
// output's element kk - 1 - i of the second run) is monotone in i, and at
// i = c T it compares the first key of the first run's stretch c with the last
// key of the second run's stretch j - c - 1 (kk = j T): both are samples.  A
// search over the samples brackets the split within T + 1 positions, and a
// search over the keys finishes it.
template <class KT>
__device__ __forceinline__ int64_t sampled_split(const Space<typename KT::T> &keys, const NodeViews &v, int64_t kk,
                                                 const typename KT::T *sa, const typename KT::T *sb, int64_t T)
{
    const int64_t lo = kk > v.b.n ? kk - v.b.n : 0, hi = kk < v.a.n ? kk : v.a.n;
    if (lo >= hi) return lo;
    const int64_t j = kk / T;
    const int64_t clo = (lo + T - 1) / T, chi = (hi + T - 1) / T;   // c T in [lo, hi)
    int64_t a = clo, b = chi;
    while (a < b) {
        const int64_t mid = (a + b) >> 1;
        if (KT::less(sb[j - mid - 1], sa[mid])) b = mid;
        else a = mid + 1;
    }
    int64_t flo = a > clo ? (a - 1) * T + 1 : lo;
    int64_t fhi = a < chi ? a * T : hi;
    while (flo < fhi) {
        const int64_t mid = (flo + fhi) >> 1;
        if (KT::less(*keys.at(view_slot(v.b, kk - 1 - mid)), *keys.at(view_slot(v.a, mid)))) fhi = mid;
        else flo = mid + 1;
    }
    return flo;
}

// One thread per (node, boundary j): the number of view-a elements among the
// first j*TILE outputs of the node's merge (no search for a concatenation).
// For the single Frogsort1 tree the node's mode is decided here from its
// children's directions (every thread of the node decides alike; the one
// with j = 0 records the mode and the node's direction, and flags the round
// if the node's outer run has to be turned around before the merge).  The
// splits read a descending run from its end, the sequence it holds once
// turned.
template <class KT, int TILE>
__global__ __launch_bounds__(256) void partition_kernel(typename KT::T *Dk, typename KT::T *Hk, Forest F,
                                                        int round, int64_t *splits, unsigned *turn_flag, Gate gate)
{
    using K = typename KT::T;
    if (gate.closed()) return;
    const int64_t L = F.probs ? (int64_t)*F.nprob : 1;
    const unsigned *srow = F.probs ? F.sbase + (int64_t)round * F.stride : nullptr;
    const int64_t total = F.use_f2  ? (int64_t)F.f2.rs[round]
                          : F.probs ? (int64_t)srow[L] : forest_splits<TILE>(F, F.p0, round);
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < total;
         w += (int64_t)gridDim.x * blockDim.x) {
        Prob P = F.p0;
        FrogMerge m;
        int64_t j, node = 0;
        if (F.use_f2) {
            const unsigned b0 = F.f2.rb[round], b1 = F.f2.rb[round + 1];
            const int64_t k = b0 + forest_locate(F.f2.node_sb + b0, b1 - b0, w);
            j = w - F.f2.node_sb[k];
            m = f2_merge(F.f2.node_s[k], F.f2.node_n[k], F.f2.q);
        } else {
            int64_t base = 0;
            if (F.probs) {
                const int64_t s = forest_locate(srow, L, w);
                P = F.probs[s];
                base = srow[s];
            }
            const int64_t tpn = forest_tpn<TILE>(F, P, round);
            const int64_t lw = w - base;
            node = lw / (tpn + 1);
            j = lw - node * (tpn + 1);
            m = forest_merge(F, P, round, node);
        }
        const Space<K> keys{Dk + P.doff, Hk + P.hoff, P.n};
        int kind = NODE_MERGE, dL = DIR_ASC, dR = DIR_ASC;
        if (F.dirs) {
            const int dep = P.depth - round;
            const uint8_t *cd = F.dirs + ((int64_t)2 << dep) - 1 + 2 * node;
            dL = (int)cd[0];
            dR = (int)cd[1];
            unsigned ndir = DIR_ASC;
            kind = node_kind<KT>(keys, m, dL, dR, &ndir);
            if (j == 0) {
                F.dirs[((int64_t)1 << dep) - 1 + node] = (uint8_t)ndir;
                F.modes[node] = (uint8_t)node_mode_pack(kind, dL, dR);
                if (kind == NODE_MERGE_REV) atomicOr(turn_flag, 1u);
            }
        }
        const NodeViews v = node_views(m, kind, dL, dR, false);
        const int64_t nn = m.nl + m.nr;
        int64_t kk = j * TILE;
        if (kk > nn) kk = nn;
        // two ascending children of the single tree: their run samples
        // (written by the previous round, node 2 node and 2 node + 1 at the
        // depth below) bracket the split
        const bool sampled = F.samp && !F.probs && !F.use_f2 && kind == NODE_MERGE && dL == DIR_ASC &&
                             dR == DIR_ASC && kk < nn && F.samp_tile * kSampPerTile == TILE;
        if (v.copy) {
            splits[w] = kk < v.a.n ? kk : v.a.n;
        } else if (sampled) {
            const int64_t ct = round == 1 ? F.samp_leaf_tiles : forest_tpn<TILE>(F, P, round - 1) * kSampPerTile;
            const K *sb0 = reinterpret_cast<const K *>(F.samp);
            splits[w] = sampled_split<KT>(keys, v, kk, sb0 + (2 * node) * ct, sb0 + (2 * node + 1) * ct,
                                          (int64_t)(TILE / kSampPerTile));
        } else {
            splits[w] = view_split<KT>(keys, v, kk);
        }
    }
}

// ---------------------------------------------------------------------------
// turning descending outer runs around (Squidsort, single Frogsort1 tree)
// ---------------------------------------------------------------------------
// Done by the tile-descriptor launch of a round (between the partition and
// the merge launches; the descriptors do not read keys): every node marked
// NODE_MERGE_REV gets its outer run reversed in place, so the merge reads it
// ascending.  Work-groups take chunks of kTurnChunk element pairs.
constexpr int64_t kTurnChunk = 4096;
template <class K, class V>
__device__ __forceinline__ void turn_outer_runs(K *Dk, K *Hk, V *Dv, V *Hv, const Forest &F, int round,
                                                uint64_t *moved)
{
    const int dep = F.p0.depth - round;
    const int64_t nodes = (int64_t)1 << dep;
    const int64_t chunks = (frog_max_node(F.p0.n, dep) / 2 + 1 + kTurnChunk - 1) / kTurnChunk;
    const Space<K> ks{Dk + F.p0.doff, Hk + F.p0.hoff, F.p0.n};
    const Space<V> vs{ValOps<V>::has ? Dv + F.p0.doff : nullptr, ValOps<V>::has ? Hv + F.p0.hoff : nullptr, F.p0.n};
    for (int64_t w = blockIdx.x; w < nodes * chunks; w += gridDim.x) {
        const int64_t node = w / chunks, c = w - node * chunks;
        if (node_mode_kind(F.modes[node]) != NODE_MERGE_REV) continue;
        const FrogMerge m = frog_merge_of(frog_node(F.p0.n, dep, node));
        const int64_t x0 = m.outer != 1 ? m.l0 : m.r0, nx = m.outer != 1 ? m.nl : m.nr;
        const int64_t pairs = nx / 2, e = (c + 1) * kTurnChunk < pairs ? (c + 1) * kTurnChunk : pairs;
        if (c == 0 && threadIdx.x == 0) atomicAdd((unsigned long long *)moved, (unsigned long long)(2 * pairs));
        for (int64_t i = c * kTurnChunk + threadIdx.x; i < e; i += blockDim.x) {
            K *a = ks.at(x0 + i), *b = ks.at(x0 + nx - 1 - i);
            const K ka = *a, kb = *b;
            *a = kb;
            *b = ka;
            if constexpr (ValOps<V>::has) {
                V *va = vs.at(x0 + i), *vb = vs.at(x0 + nx - 1 - i);
                const V xa = *va, xb = *vb;
                *va = xb;
                *vb = xa;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// tile descriptors with their dependency windows
// ---------------------------------------------------------------------------
// A tile overwrites the slots [o, o + cnt); the elements of the outer run in
// those slots are read by the tiles whose inputs include them, which the
// splits give (tile_window in frog_geometry.h); their tickets form one
// contiguous range that never passes the tile's own.
template <class K, class V, int TILE>
__global__ __launch_bounds__(256) void tiles_kernel(K *Dk, K *Hk, V *Dv, V *Hv, Forest F, int round,
                                                    const int64_t *splits, TileDesc *desc, const unsigned *turn_flag,
                                                    uint64_t *moved, Gate gate)
{
    if (gate.closed()) return;
    if (F.dirs && *turn_flag) turn_outer_runs<K, V>(Dk, Hk, Dv, Hv, F, round, moved);
    const int64_t L = F.probs ? (int64_t)*F.nprob : 1;
    const unsigned *trow = F.probs ? F.tbase + (int64_t)round * F.stride : nullptr;
    const unsigned *srow = F.probs ? F.sbase + (int64_t)round * F.stride : nullptr;
    const int64_t total = F.use_f2  ? (int64_t)F.f2.rt[round]
                          : F.probs ? (int64_t)trow[L] : forest_tickets<TILE>(F, F.p0, round);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        int64_t s = 0, tpn, q, first, node = 0;
        const int64_t *sp;
        FrogMerge m;
        if (F.use_f2) {
            // a node has ceil(n / TILE) tiles and one split more
            const unsigned b0 = F.f2.rb[round], b1 = F.f2.rb[round + 1];
            const int64_t k = b0 + forest_locate(F.f2.node_tb + b0, b1 - b0, t);
            m = f2_merge(F.f2.node_s[k], F.f2.node_n[k], F.f2.q);
            tpn = (m.nl + m.nr + TILE - 1) / TILE;
            first = F.f2.node_tb[k];
            q = t - first;
            sp = splits + F.f2.node_sb[k];
        } else {
            Prob P = F.p0;
            int64_t tb = 0, sb = 0;
            if (F.probs) {
                s = forest_locate(trow, L, t);
                P = F.probs[s];
                tb = trow[s];
                sb = srow[s];
            }
            tpn = forest_tpn<TILE>(F, P, round);
            const int64_t lt = t - tb;
            node = lt / tpn;
            q = lt - node * tpn;
            first = tb + node * tpn;
            sp = splits + sb + node * (tpn + 1);
            m = forest_merge(F, P, round, node);
        }
        int kind = NODE_MERGE, dL = DIR_ASC, dR = DIR_ASC;
        if (F.dirs) {
            const unsigned w = F.modes[node];     // written by the partition launch
            kind = node_mode_kind(w);
            dL = node_mode_dl(w);
            dR = node_mode_dr(w);
        }
        // the outer run of a NODE_MERGE_REV node has been turned around by now
        const NodeViews v = node_views(m, kind, dL, dR, true);
        const int64_t nn = m.nl + m.nr;
        const int64_t j = m.left ? (tpn - 1 - q) : q;
        int64_t k0 = j * TILE;
        const int samp = F.samp && !F.probs && !F.use_f2 ? (int)(2 * (node * tpn + j) + (node & 1)) : -1;
        if (k0 > nn) k0 = nn;
        int64_t k1 = k0 + TILE;
        if (k1 > nn) k1 = nn;
        TileDesc T;
        T.prob = F.probs ? (int)s : samp;
        T.cnt = (int)(k1 - k0);
        T.la = 0;
        T.pa = T.pb = T.o = 0;
        T.flags = (v.copy ? TF_COPY : 0) | (v.a.step < 0 ? TF_AREV : 0) | (v.b.step < 0 ? TF_BREV : 0);
        int64_t lo = 1, hi = 0;          // empty window
        if (k0 < k1) {
            // Splits of sorted runs are monotone and every tile takes between
            // 0 and cnt elements from each view; the clamp keeps the
            // descriptor within the views whatever the runs hold (it changes
            // nothing for sorted runs).
            const int64_t a0 = sp[j];
            int64_t a1 = sp[j + 1];
            const int64_t a1lo = a0 > k1 - v.b.n ? a0 : k1 - v.b.n;
            const int64_t a1hi = a0 + (k1 - k0) < v.a.n ? a0 + (k1 - k0) : v.a.n;
            a1 = a1 < a1lo ? a1lo : a1 > a1hi ? a1hi : a1;
            T.la = (int)(a1 - a0);
            // lowest slot of each view's range: view indices [a0, a1) of a,
            // [k0 - a0, k1 - a1) of b
            T.pa = v.a.step > 0 ? view_slot(v.a, a0) : view_slot(v.a, a1 - 1);
            T.pb = v.b.step > 0 ? view_slot(v.b, k0 - a0) : view_slot(v.b, k1 - a1 - 1);
            T.o = m.out0 + k0;
            tile_window(v, m.out0, m.left, sp, tpn, TILE, j, first, &lo, &hi);
            // the window lies within the node's tickets and never passes the
            // tile's own (again a no-op for sorted runs)
            if (lo <= hi) {
                lo = lo < first ? first : lo;
                hi = hi > t ? t : hi;
            }
        }
        T.dlo = (unsigned)lo;
        T.dhi = (unsigned)hi;
        // A tile that takes all its inputs from one run, stepping upwards, at
        // the very slots it writes (the outer run's elements that stay in
        // place: half of every merge on presorted input, "Symmetric merging",
        // and the outer half of a concatenation) moves nothing; nobody else
        // writes into its range, so it needs no wait.
        const bool in_place = T.cnt == 0 || (T.la == T.cnt && v.a.step > 0 && T.pa == T.o) ||
                              (T.la == 0 && v.b.step > 0 && T.pb == T.o);
        if (in_place) T.flags |= TF_SKIP;
        desc[t] = T;
    }
}

// ---------------------------------------------------------------------------
// merge kernel: persistent work-groups, one output tile per iteration
// ---------------------------------------------------------------------------
// A left node writes its output top-down (its outer run is the left child's
// data, which only moves right); a right node bottom-up (its outer run is the
// right child's data, which only moves left).  Inner runs lie outside the
// output.  Tickets are handed out in each node's write order, in chunks of
// GS_MERGE_CLAIM consecutive tickets; chunk j belongs to counter group
// j % kMergeGroups, and work-group b claims from group b % kMergeGroups, each
// counter on its own cache line (a single device-wide counter limits the rate
// at which tiles can start).  A work-group takes the next ticket and issues
// that tile's loads while it merges and stores the current one.  It processes
// its tickets in increasing order and waits only on smaller tickets; the
// smallest ticket not yet loaded is always claimed (every group's earlier
// tickets have loaded, so its work-groups finish them and claim on), so the
// waits cannot deadlock.
#ifndef GS_MERGE_CLAIM
#define GS_MERGE_CLAIM 1
#endif
// Reverses the staged elements at LDS positions [first, first + len).
template <class K, class VS, bool HV, int NT>
__device__ __forceinline__ void reverse_lds(K *sk, VS *sv, int first, int len)
{
    for (int i = threadIdx.x; i < len / 2; i += NT) {
        const int a = lpad(first + i), b = lpad(first + len - 1 - i);
        const K ka = sk[a], kb = sk[b];
        sk[a] = kb;
        sk[b] = ka;
        if constexpr (HV) {
            const VS va = sv[a], vb = sv[b];
            sv[a] = vb;
            sv[b] = va;
        }
    }
}

// The thread's IPT outputs of a tile staged in LDS (view-a inputs at
// [0, la), view-b inputs at [la, cnt)), merged under order KO.
template <class KO, class VS, bool HV, int IPT, int TILE>
__device__ __forceinline__ void merge_tile_outputs(const typename KO::T *sk, int d, int la, int lb,
                                                   typename KO::T (&k)[IPT], int (&srcix)[IPT])
{
    const int ai = merge_path_lds<KO>(d, la, lb, [&](int i) { return sk[lpad(i)]; },
                                      [&](int i) { return sk[lpad(la + i)]; });
    serial_merge<KO, IPT, HV>(sk, 0, la, la, lb, ai, d - ai, TILE, k, srcix);
}

template <class KT, class V, int NT, int IPT, int WAVES>
__global__ __launch_bounds__(NT, WAVES) void merge_kernel(typename KT::T *Dk, typename KT::T *Hk, V *Dv, V *Hv,
                                                   Forest F, int round, int64_t nt_host,
                                                   const TileDesc *__restrict__ desc,
                                                   unsigned *ticket_ctr, unsigned *status, unsigned epoch,
                                                   unsigned *err, uint64_t *moved, Gate gate)
{
    using K = typename KT::T;
    constexpr bool HV = ValOps<V>::has;
    using VS = typename std::conditional<HV, V, char>::type;
    constexpr int TILE = NT * IPT;
    constexpr int SLOTS = lds_slots<TILE>();
    constexpr int CLAIM = GS_MERGE_CLAIM;
    __shared__ K sk[SLOTS];
    __shared__ VS sv[HV ? SLOTS : 1];
    __shared__ unsigned s_next;
    if (gate.closed()) return;

    // tiles of this round: from the device table, else the count the host
    // passes (it knows it for one problem)
    const int64_t ntiles = F.probs ? (int64_t)F.tbase[(int64_t)round * F.stride + *F.nprob] : nt_host;
    const int tid = threadIdx.x;
    const int grp = (int)(blockIdx.x % kMergeGroups);
    unsigned *my_ctr = ticket_ctr + 32 * grp;
    // first ticket of the chunk a claim returns
    auto chunk_start = [&](unsigned c) -> int64_t { return ((int64_t)c * kMergeGroups + grp) * CLAIM; };
    if (tid == 0) s_next = atomicAdd(my_ctr, 1u);
    lds_barrier();
    int64_t cur_t = chunk_start(__builtin_amdgcn_readfirstlane(s_next));
    int slot = 0;                        // position of cur_t within its chunk
    if (cur_t >= ntiles) return;

    // (descriptors and problems are uniform per tile and read-only here: the
    // restrict qualifiers let them come through the scalar unit, so waiting
    // for them never waits for the tile data in flight)
    using ConstProb = const __attribute__((address_space(4))) Prob;
    ConstProb *const probs = (ConstProb *)(uintptr_t)F.probs;
    auto prob_of = [&](int s) -> Prob {
        if (!probs) return F.p0;
        ConstProb &q = probs[s];
        return Prob{q.doff, q.hoff, q.n, q.depth, q.pad};
    };
    TileDesc cur = desc[cur_t];
    Prob cur_p = prob_of(cur.prob);
    K lk[IPT];
    VS lv[IPT];
    // Straight-line loads: indices past the tile are clamped to its last input
    // (an empty tile reads its problem's slot 0), so every load is valid and
    // none needs a branch; the values loaded for clamped indices are never
    // stored.
    auto issue_loads = [&](const TileDesc &T, const Prob &P) {
        const int last = T.cnt > 0 ? T.cnt - 1 : 0;
        const Space<K> ks{Dk + P.doff, Hk + P.hoff, P.n};
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            const int i = min(tid + r * NT, last);
            const int64_t p = i < T.la ? T.pa + i : T.pb + (i - T.la);
            lk[r] = GS_MERGE_LOAD(ks.at(p));
            if constexpr (HV) {
                const Space<V> vs{Dv + P.doff, Hv + P.hoff, P.n};
                lv[r] = *vs.at(p);
            }
        }
    };
    if (!(cur.flags & TF_SKIP)) issue_loads(cur, cur_p);
    unsigned my_moved = 0;

    for (;;) {
        const bool skip = (cur.flags & TF_SKIP) != 0, copy = (cur.flags & TF_COPY) != 0;
        // stage the current tile in LDS and publish that its inputs are read
        // (slots past the tile receive ignored values); a view read from its
        // end is staged in reverse
        if (!skip) {
#pragma unroll
            for (int r = 0; r < IPT; ++r) {
                const int i = tid + r * NT;
                sk[lpad(i)] = lk[r];
                if constexpr (HV) sv[lpad(i)] = lv[r];
            }
        }
        lds_barrier();
        if (!skip && (cur.flags & (TF_AREV | TF_BREV))) {
            // a view read from its end: its slots came in upwards, so its
            // segment of the staged inputs is reversed in place
            const int la = cur.la, lb = cur.cnt - cur.la;
            if (cur.flags & TF_AREV) reverse_lds<K, VS, HV, NT>(sk, sv, 0, la);
            if (cur.flags & TF_BREV) reverse_lds<K, VS, HV, NT>(sk, sv, la, lb);
            lds_barrier();
        }
        const bool last_of_claim = slot == CLAIM - 1;
        unsigned nt = 0;
        if (tid == 0) {
            st_status(status + cur_t, (epoch << 2) | ST_LOADED);
            if (last_of_claim) nt = atomicAdd(my_ctr, 1u);
        }

        // merge: thread tid produces outputs [tid*IPT, tid*IPT + nout)
        K k[IPT];
        VS v[IPT];
        int srcix[IPT];
        const int d = tid * IPT;
        int nout = skip || copy ? 0 : cur.cnt - d;
        nout = nout < 0 ? 0 : (nout > IPT ? IPT : nout);
        const int la = cur.la, lb = cur.cnt - cur.la;
        if (nout > 0) {
            merge_tile_outputs<KT, VS, HV, IPT, TILE>(sk, d, la, lb, k, srcix);
            if constexpr (HV) {
#pragma unroll
                for (int i = 0; i < IPT; ++i) v[i] = sv[lpad(min(srcix[i], TILE))];
            }
        }
        if (last_of_claim) {
            if (tid == 0) s_next = nt;
            lds_barrier();
        }
        // where this tile's outputs go, fixed before the next tile's loads are
        // issued (so the stores wait for none of them): output i lands in
        // the caller's array below logical slot n, in the half buffer above
        const int64_t out_o = cur.o, out_split = cur_p.n - cur.o;
        K *const out_d = Dk + cur_p.doff + out_o;
        K *const out_h = Hk + cur_p.hoff + (out_o - cur_p.n);
        V *const vout_d = HV ? Dv + cur_p.doff + out_o : nullptr;
        V *const vout_h = HV ? Hv + cur_p.hoff + (out_o - cur_p.n) : nullptr;
        const int out_cnt = cur.cnt;
        // wait for the window before issuing the next tile's loads: a poll
        // of a status word has to wait for every load issued before it, so
        // polling after the prefetch would drain the prefetch
        if (!skip && tid < 64) wait_window(status, cur.dlo, cur.dhi, cur_t, epoch, err);

        // prefetch the next tile while this one is written back and stored
        const int64_t t2 = last_of_claim ? chunk_start(__builtin_amdgcn_readfirstlane(s_next)) : cur_t + 1;
        const bool more = t2 < ntiles;
        TileDesc nxt;
        Prob nxt_p;
        if (more) {
            nxt = desc[t2];
            nxt_p = prob_of(nxt.prob);
            if (!(nxt.flags & TF_SKIP)) issue_loads(nxt, nxt_p);
        }
        // the run samples of this tile's outputs (first or last key of each
        // stretch of samp_tile ranks), for the next round's partition: from
        // the registers of the threads that merged them (a whole tile), from
        // LDS (a short tile or a concatenation), or from memory (outputs
        // already in their slots)
        K *const samp_p = F.samp && cur.prob >= 0 && out_cnt > 0
                              ? reinterpret_cast<K *>(F.samp) + (int64_t)(cur.prob >> 1) * kSampPerTile
                              : nullptr;
        const bool samp_last = cur.prob & 1;
        constexpr int ST = TILE / kSampPerTile;                              // ranks per stretch
        const int samp_n = (out_cnt + ST - 1) / ST;                              // stretches of this tile
        // rank of stretch s's sample (s < samp_n)
        auto samp_rank = [&](int s) { return samp_last ? min((s + 1) * ST, out_cnt) - 1 : s * ST; };
        if (skip && samp_p && tid < samp_n) {
            const Space<K> ks{Dk + cur_p.doff, Hk + cur_p.hoff, cur_p.n};
            samp_p[tid] = *ks.at(out_o + samp_rank(tid));
        }
        if (!skip) {
            my_moved += (unsigned)cur.cnt;
            lds_barrier();             // the merge's reads are done and the window has been waited for
            // (a concatenation has no outputs to write back: its outputs are
            // its staged inputs, in order)
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                if (i < nout) {
                    sk[lpad(d + i)] = k[i];
                    if constexpr (HV) sv[lpad(d + i)] = v[i];
                }
            }
            lds_barrier();
            if (samp_p) {
                // a whole merged tile: the thread of rank s T holds it in k[0],
                // the one of rank (s + 1) T - 1 in k[IPT - 1]
                constexpr int TPS = NT / kSampPerTile;                      // threads per stretch
                const bool in_regs = !copy && out_cnt == TILE;
                if (in_regs) {
                    if (samp_last ? tid % TPS == TPS - 1 : tid % TPS == 0)
                        samp_p[tid / TPS] = samp_last ? k[IPT - 1] : k[0];
                } else if (tid < samp_n) {
                    samp_p[tid] = sk[lpad(samp_rank(tid))];
                }
            }
#pragma unroll
            for (int r = 0; r < IPT; ++r) {
                const int i = tid + r * NT;
                if (i < out_cnt) {
                    GS_MERGE_STORE(sk[lpad(i)], i < out_split ? out_d + i : out_h + i);
                    if constexpr (HV) *(i < out_split ? vout_d + i : vout_h + i) = sv[lpad(i)];
                }
            }
        }
        if (!more) break;
        lds_barrier();                 // LDS reads done before the next staging
        cur = nxt;
        cur_p = nxt_p;
        cur_t = t2;
        slot = last_of_claim ? 0 : slot + 1;
    }
    if (tid == 0 && moved && my_moved) atomicAdd((unsigned long long *)moved, (unsigned long long)my_moved);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
template <class KT, class V>
struct SortCfg;
#ifndef GS_F64_LEAF_NT
#define GS_F64_LEAF_NT 512
#endif
#ifndef GS_F64_LEAF_IPT
#define GS_F64_LEAF_IPT 16
#endif
#ifndef GS_F64_LEAF_WAVES
#define GS_F64_LEAF_WAVES 4
#endif
#ifndef GS_F64_MERGE_NT
#define GS_F64_MERGE_NT 256
#endif
#ifndef GS_F64_MERGE_IPT
#define GS_F64_MERGE_IPT 16
#endif
#ifndef GS_F64_MERGE_WAVES
#define GS_F64_MERGE_WAVES 3
#endif
// LEAF_WAVES / MERGE_WAVES: waves per SIMD each kernel is compiled to allow
// (the register budget), chosen so that the LDS, not the registers, limits
// the work-groups per compute unit.
template <>
struct SortCfg<KeyF64, NoVal> {
    static constexpr int LEAF_NT = GS_F64_LEAF_NT, LEAF_IPT = GS_F64_LEAF_IPT, LEAF_WAVES = GS_F64_LEAF_WAVES;
    static constexpr int MERGE_NT = GS_F64_MERGE_NT, MERGE_IPT = GS_F64_MERGE_IPT, MERGE_WAVES = GS_F64_MERGE_WAVES;
};
// the same f64 comparison with 2048-output merge tiles (a shape the
// segmented sort's tuner can choose)
struct KeyF64T8 : KeyF64 {};
template <>
struct FastKey<KeyF64T8> {
    using type = KeyF64NoNaN;
};
template <>
struct SortCfg<KeyF64T8, NoVal> {
    static constexpr int LEAF_NT = GS_F64_LEAF_NT, LEAF_IPT = GS_F64_LEAF_IPT, LEAF_WAVES = 4;
    static constexpr int MERGE_NT = 256, MERGE_IPT = 8, MERGE_WAVES = 4;
};
#ifndef GS_KV_LEAF_NT
#define GS_KV_LEAF_NT 512
#endif
#ifndef GS_KV_LEAF_WAVES
#define GS_KV_LEAF_WAVES 6
#endif
#ifndef GS_KV_LEAF_IPT
#define GS_KV_LEAF_IPT 8
#endif
#ifndef GS_KV_MERGE_IPT
#define GS_KV_MERGE_IPT 16
#endif
#ifndef GS_KV_MERGE_WAVES
#define GS_KV_MERGE_WAVES 2
#endif
template <>
struct SortCfg<KeyU64, uint32_t> {
    static constexpr int LEAF_NT = GS_KV_LEAF_NT, LEAF_IPT = GS_KV_LEAF_IPT, LEAF_WAVES = GS_KV_LEAF_WAVES;
    static constexpr int MERGE_NT = 256, MERGE_IPT = GS_KV_MERGE_IPT, MERGE_WAVES = GS_KV_MERGE_WAVES;
};
// descending orders: the same shapes as their ascending counterparts
template <>
struct SortCfg<KeyF64Desc, NoVal> : SortCfg<KeyF64, NoVal> {};
template <>
struct SortCfg<KeyU64Desc, uint32_t> : SortCfg<KeyU64, uint32_t> {};

template <class KT, class V>
constexpr int64_t leaf_size()
{
    return (int64_t)SortCfg<KT, V>::LEAF_NT * SortCfg<KT, V>::LEAF_IPT;
}
template <class KT, class V>
constexpr int64_t tile_size()
{
    return (int64_t)SortCfg<KT, V>::MERGE_NT * SortCfg<KT, V>::MERGE_IPT;
}

static int64_t align256(int64_t b) { return (b + 255) & ~(int64_t)255; }

// Control block, status words, splits, tile descriptors and (for a problem
// table) the per-round prefix rows, laid out from offset 0.
static ForestPlan layout_forest(int64_t max_probs, int rounds, int64_t max_tickets, int64_t max_status,
                                int64_t max_splits, int64_t leaf, int64_t tile, int64_t dir_nodes = 0,
                                int64_t samp_slots = 0)
{
    ForestPlan f{};
    f.max_probs = max_probs;
    f.rounds = rounds;
    f.leaf = leaf;
    f.tile = tile;
    f.stride = max_probs + 1;
    f.max_tickets = max_tickets;
    f.max_status = max_status;
    f.max_splits = max_splits;
    f.off_ctrl = 0;
    f.off_status = align256(forest_ctrl_words(rounds) * 4);
    f.dir_nodes = dir_nodes;
    f.off_dirs = f.off_status + align256(max_status * 4);
    f.off_modes = f.off_dirs + align256(dir_nodes);
    f.off_splits = f.off_modes + align256(dir_nodes / 2);
    f.off_desc = f.off_splits + align256(max_splits * 8);
    f.samp_slots = samp_slots;
    f.off_samp = f.off_desc + align256(max_tickets * (int64_t)sizeof(TileDesc));
    f.off_probs = f.off_samp + align256(samp_slots * 8);
    f.off_tbase = f.off_probs + (max_probs > 0 ? align256(max_probs * (int64_t)sizeof(Prob)) : 0);
    f.off_sbase = f.off_tbase + (max_probs > 0 ? align256((rounds + 1) * f.stride * 4) : 0);
    f.bytes = f.off_sbase + (max_probs > 0 ? align256((rounds + 1) * f.stride * 4) : 0);
    f.off_f2 = f.bytes;
    f.f2_bytes = 0;
    return f;
}

template <class KT, class V>
ForestPlan forest_plan_one(int64_t n)
{
    constexpr int64_t LEAF = leaf_size<KT, V>(), TILE = tile_size<KT, V>();
    Forest F{};
    F.p0 = Prob{0, 0, n, n > 1 ? frog_depth(n, LEAF) : 0, 0};
    int64_t mt = 1, ms = 1;
    const int D = F.p0.depth;
    const int64_t leaves = (int64_t)1 << D;
    for (int r = 1; r <= D; ++r) {
        const int64_t t = forest_tickets<TILE>(F, F.p0, r), s = forest_splits<TILE>(F, F.p0, r);
        if (t > mt) mt = t;
        if (s > ms) ms = s;
    }
    // Squidsort directions of every node (heap order, 2^(D+1) - 1 of them);
    // run samples of the leaves and of every merge round
    constexpr int64_t ST = TILE / kSampPerTile;                  // ranks per sample stretch
    const int64_t leaf_slots = leaves * ((LEAF + ST - 1) / ST), merge_slots = mt * kSampPerTile;
    return layout_forest(0, D, mt, mt > leaves ? mt : leaves, ms, LEAF, TILE, (int64_t)2 << D,
                         merge_slots > leaf_slots ? merge_slots : leaf_slots);
}

// Capacity for any set of at most max_probs problems of at most max_len keys
// each and num_keys keys in total.  At a merge depth d of a problem of n keys
// the 2^d nodes hold at most ceil(n/2^d) keys each, so its tickets are
// 2^d * ceil(ceil(n/2^d) / TILE) <= n / TILE + 2^d, and 2^d < n / LEAF
// because a node above the leaf level holds more than LEAF keys; the splits
// add one per node.  A problem has 1 leaf or fewer than 2n / LEAF.
template <class KT, class V>
ForestPlan forest_plan_many(int64_t num_keys, int64_t max_len, int64_t max_probs)
{
    constexpr int64_t LEAF = leaf_size<KT, V>(), TILE = tile_size<KT, V>();
    const int rounds = max_len > 1 ? frog_depth(max_len, LEAF) : 0;
    const int64_t mt = num_keys / TILE + num_keys / LEAF + 64;
    const int64_t ms = num_keys / TILE + 2 * (num_keys / LEAF) + 64;
    const int64_t leaves = 2 * (num_keys / LEAF) + max_probs + 64;
    return layout_forest(max_probs, rounds, mt, mt > leaves ? mt : leaves, ms, LEAF, TILE);
}

// Resident work-groups of a kernel over the whole device (cached by caller).
template <class F>
static int64_t resident_groups(F kernel, int threads, int64_t &cache)
{
    if (cache > 0) return cache;
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
        per_cu <= 0)
        per_cu = 1;
    cache = (int64_t)cus * per_cu;
    return cache;
}

static unsigned grid_for(int64_t items, int threads, int64_t cap)
{
    int64_t g = (items + threads - 1) / threads;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (unsigned)g;
}

template <class V>
constexpr bool HV_of() { return ValOps<V>::has; }

// Reversal of keys[0, n) (and vals) when the top node's run came back
// descending (*top == DIR_DESC) and the gate is open; counts the moves.
template <class K, class V>
__global__ __launch_bounds__(256) void root_reverse_kernel(K *keys, V *vals, int64_t n, Gate gate, const uint8_t *top,
                                                           uint64_t *moved)
{
    if (gate.closed() || *top != (uint8_t)DIR_DESC) return;
    const int64_t half = n / 2;
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd((unsigned long long *)moved, (unsigned long long)(2 * half));
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < half;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = n - 1 - i;
        const K a = keys[i], b = keys[j];
        keys[i] = b;
        keys[j] = a;
        if constexpr (ValOps<V>::has) {
            const V va = vals[i], vb = vals[j];
            vals[i] = vb;
            vals[j] = va;
        }
    }
}

template <class K, class V>
static void launch_root_reverse(K *keys, V *vals, int64_t n, Gate gate, const uint8_t *top, uint64_t *moved,
                                hipStream_t st)
{
    hipLaunchKernelGGL((root_reverse_kernel<K, V>), dim3(grid_for(n / 2, 256, 8192)), dim3(256), 0, st, keys, vals, n,
                       gate, top, moved);
}

// Enqueues a whole forest sort (or, with use_m1, one explicit merge) on the
// forest area `fw` laid out by `fp`.  Exact launch sizes for the single
// problem; capacity-sized persistent launches for a device-side table.
template <class KT, class V>
static hipError_t run_forest(typename KT::T *Dk, typename KT::T *Hk, V *Dv, V *Hv, Forest F,
                             const ForestPlan &fp, char *fw, hipStream_t st, Gate gate, bool leaves,
                             const F2Tables *f2 = nullptr, char *f2_img = nullptr)
{
    using C = SortCfg<KT, V>;
    using K = typename KT::T;
    constexpr int TILE = C::MERGE_NT * C::MERGE_IPT;
    unsigned *ctrl = (unsigned *)(fw + fp.off_ctrl);
    unsigned *status = (unsigned *)(fw + fp.off_status);
    int64_t *splits = (int64_t *)(fw + fp.off_splits);
    TileDesc *desc = (TileDesc *)(fw + fp.off_desc);
    unsigned *errw = ctrl + kErrWord;
    uint64_t *moved = (uint64_t *)(ctrl + kMovedWord);
    const bool table = F.probs != nullptr;
    // Squidsort's run directions: the single Frogsort1 tree only
    const bool squid = !table && !f2 && !F.use_m1 && fp.dir_nodes >= ((int64_t)2 << F.p0.depth) &&
                       fp.rounds < kTurnRounds;
    if (squid) {
        F.dirs = (uint8_t *)(fw + fp.off_dirs);
        F.modes = (uint8_t *)(fw + fp.off_modes);
        if (fp.samp_slots > 0 && fp.tile == TILE) {
            F.samp = fw + fp.off_samp;
            F.samp_tile = TILE / kSampPerTile;
            F.samp_leaf_tiles = (int)((fp.leaf + F.samp_tile - 1) / F.samp_tile);
        }
    }
    if (table) {
        F.tbase = (const unsigned *)(fw + fp.off_tbase);
        F.sbase = (const unsigned *)(fw + fp.off_sbase);
        F.stride = fp.stride;
    }
    // rounds of this run: one explicit merge, the tree's own height (trees
    // of one plan differ), or the capacity the forest area was laid out for
    const int R = F.use_m1 ? 1 : f2 ? f2->rounds : fp.rounds;
    if (R > (fp.rounds > 0 ? fp.rounds : 1)) return hipErrorInvalidValue;
    if (f2) {
        // every launch of the tree must fit the area's capacities
        if ((int)f2->rt.size() != R + 1 || (int)f2->rs.size() != R + 1 || f2->nleaves > fp.max_status ||
            f2->max_tickets > fp.max_tickets || f2->max_splits > fp.max_splits)
            return hipErrorInvalidValue;
        // the tree tables travel with the call (see F2Tables), unless the
        // caller has already put them at f2_img
        char *img = f2_img ? f2_img : fw + fp.off_f2;
        if (!f2_img) {
            hipError_t e = hipMemcpyAsync(img, f2->blob.data(), f2->blob.size(), hipMemcpyHostToDevice, st);
            if (e != hipSuccess) return e;
        }
        F.use_f2 = 1;
        F.f2.leaf_c = (const int64_t *)(img + f2->off_leaf_c);
        F.f2.leaf_d = (const int64_t *)(img + f2->off_leaf_d);
        F.f2.node_s = (const int64_t *)(img + f2->off_node_s);
        F.f2.node_n = (const int64_t *)(img + f2->off_node_n);
        F.f2.node_tb = (const unsigned *)(img + f2->off_node_tb);
        F.f2.node_sb = (const unsigned *)(img + f2->off_node_sb);
        F.f2.rb = (const unsigned *)(img + f2->off_rb);
        F.f2.rt = (const unsigned *)(img + f2->off_rt);
        F.f2.rs = (const unsigned *)(img + f2->off_rs);
        F.f2.nleaves = f2->nleaves;
        F.f2.q = f2->q;
    }

    const bool tr = trace_on();
    // ticket counters and status words start at zero on every run (the
    // call's error word is kept, so it collects every run of the call)
    if (tr) trace_begin(TK_FILL, st);
    launch_fill_ctrl(ctrl, (fp.off_splits - fp.off_ctrl) / 4, st);
    if (tr) trace_end(st);
    if (table) {
        if (tr) trace_begin(TK_OTHER, st);
        hipLaunchKernelGGL((forest_scan_kernel<TILE>), dim3((unsigned)(R + 1)), dim3(1024), 0, st, F,
                           (unsigned *)(fw + fp.off_tbase), (unsigned *)(fw + fp.off_sbase), fp.max_status,
                           fp.max_tickets, fp.max_splits, errw, gate);
        if (tr) trace_end(st);
    }

    auto leaf_fn = f2 ? leaf_kernel<KT, V, C::LEAF_NT, C::LEAF_IPT, C::LEAF_WAVES, true, false>
                      : leaf_kernel<KT, V, C::LEAF_NT, C::LEAF_IPT, C::LEAF_WAVES, false, false>;
    auto leaf_table_fn = leaf_kernel<KT, V, C::LEAF_NT, C::LEAF_IPT, C::LEAF_WAVES, false, true>;
    auto merge_fn = merge_kernel<KT, V, C::MERGE_NT, C::MERGE_IPT, C::MERGE_WAVES>;
    static int64_t merge_groups = 0, leaf_groups = 0;
    unsigned epoch = 1;
    if (leaves) {
        if (tr) trace_begin(TK_LEAF, st);
        if (table) {
            // the leaf count is on the device: the resident work-groups take
            // its leaves in turn
            const int64_t lres = resident_groups(leaf_table_fn, C::LEAF_NT, leaf_groups);
            hipLaunchKernelGGL(leaf_table_fn, dim3((unsigned)(fp.max_status < lres ? fp.max_status : lres)),
                               dim3(C::LEAF_NT), 0, st, Dk, Hk, Dv, Hv, F, ctrl + 0, status, epoch, errw, moved, gate);
        } else {
            const int64_t nl = f2 ? f2->nleaves : ((int64_t)1 << F.p0.depth);
            hipLaunchKernelGGL(leaf_fn, dim3((unsigned)nl), dim3(C::LEAF_NT), 0, st, Dk, Hk, Dv, Hv, F, ctrl + 0,
                               status, epoch, errw, moved, gate);
        }
        if (tr) trace_end(st);
    }
    const int64_t mres = resident_groups(merge_fn, C::MERGE_NT, merge_groups);
    for (int r = 1; r <= R; ++r) {
        ++epoch;
        const int64_t nsplit = table ? fp.max_splits : f2 ? f2->rs[r] : forest_splits<TILE>(F, F.p0, r);
        const int64_t ntile = table ? fp.max_tickets : f2 ? f2->rt[r] : forest_tickets<TILE>(F, F.p0, r);
        if (ntile <= 0) continue;
        if (tr) trace_begin(TK_PARTITION, st);
        unsigned *turn_flag = ctrl + kTurnWord0 + (r < kTurnRounds ? r : 0);
        hipLaunchKernelGGL((partition_kernel<KT, TILE>), dim3(grid_for(nsplit, 256, 4096)), dim3(256), 0, st, Dk,
                           Hk, F, r, splits, turn_flag, gate);
        if (tr) trace_end(st);
        if (tr) trace_begin(TK_DEPWIN, st);
        // (with Squidsort the launch also turns descending outer runs around:
        // at least 512 work-groups, most of which exit at once when there is
        // nothing to turn)
        unsigned tgrid = grid_for(ntile, 256, 4096);
        if (squid && tgrid < 512) tgrid = 512;
        hipLaunchKernelGGL((tiles_kernel<K, V, TILE>), dim3(tgrid), dim3(256), 0, st, Dk, Hk, Dv, Hv, F, r,
                           (const int64_t *)splits, desc, (const unsigned *)turn_flag, moved, gate);
        if (tr) trace_end(st);
        if (tr) trace_begin(TK_MERGE, st);
        hipLaunchKernelGGL(merge_fn, dim3((unsigned)(ntile < mres ? ntile : mres)), dim3(C::MERGE_NT), 0, st, Dk,
                           Hk, Dv, Hv, F, r, ntile, (const TileDesc *)desc, ctrl + 32 * kMergeGroups * r, status, epoch,
                           errw, moved, gate);
        if (tr) trace_end(st);
    }
    if (squid && F.p0.n > 1) {
        // the wanted order is enforced once: a top run that came back
        // descending is reversed
        if (tr) trace_begin(TK_OTHER, st);
        launch_root_reverse(Dk + F.p0.doff, HV_of<V>() ? Dv + F.p0.doff : Dv, F.p0.n, gate, F.dirs, moved, st);
        if (tr) trace_end(st);
    }
    return hipGetLastError();
}

template <class KT, class V>
SortPlan make_plan(int64_t n, int64_t q, int algo, int64_t q2)
{
    using K = typename KT::T;
    constexpr bool HV = ValOps<V>::has;
    SortPlan p{};
    p.n = n;
    p.leaf = leaf_size<KT, V>();
    p.tile = tile_size<KT, V>();
    p.q = algo == kAlgoFrog1 ? 0 : q;
    if (algo == kAlgoFrog2 && n > 1) {
        p.f2 = f2_tables(n, q, p.leaf, p.tile);
        p.depth = p.f2->rounds;
        p.hlen = f2_inner(n, q);
    } else if (algo == kAlgoFrog3 && n > 1) {
        p.f3 = f3_plans(n, q, q2, p.leaf, p.tile);
        p.depth = p.f3->total_rounds;
        // b covers a spine-less tree's own buffer, and a single leaf needs none
        p.hlen = p.f3->b < f2_inner(n, q2) ? p.f3->b : f2_inner(n, q2);
    } else {
        p.depth = n > 1 ? frog_depth(n, p.leaf) : 0;
        p.hlen = n / 2;
    }
    p.off_hkeys = 0;
    p.off_hvals = align256(p.hlen * (int64_t)sizeof(K));
    p.off_forest = p.off_hvals + (HV ? align256(p.hlen * (int64_t)sizeof(V)) : 0);
    if (p.f2) {
        const F2Tables &T = *p.f2;
        const int64_t mt = T.max_tickets > 1 ? T.max_tickets : 1;
        p.forest = layout_forest(0, T.rounds, mt, mt > T.nleaves ? mt : T.nleaves,
                                 T.max_splits > 1 ? T.max_splits : 1, p.leaf, p.tile);
        p.forest.off_f2 = p.forest.bytes;
        p.forest.f2_bytes = (int64_t)T.blob.size();
        p.forest.bytes += p.forest.f2_bytes;
    } else if (p.f3) {
        const F3Plan &P3 = *p.f3;
        p.forest = layout_forest(0, P3.max_rounds, P3.max_tickets, P3.max_status, P3.max_splits, p.leaf, p.tile);
        p.forest.off_f2 = p.forest.bytes;
        p.forest.f2_bytes = align256((int64_t)P3.image.size());
        p.forest.bytes += p.forest.f2_bytes;
    } else {
        p.forest = forest_plan_one<KT, V>(n);
    }
    p.off_order = p.off_forest + p.forest.bytes;
    p.bytes = p.off_order + 256;
    if (n <= 1) p.bytes = 0;
    return p;
}

// Frogsort3: the trees in order (each placing and sorting its part), then the
// spine merges bottom up, all on the caller's stream.
template <class KT, class V>
static hipError_t run_frog3(typename KT::T *keys, V *vals, int64_t n, char *ws, const SortPlan &p,
                            hipStream_t st, Gate gate)
{
    using K = typename KT::T;
    constexpr bool HV = ValOps<V>::has;
    const F3Plan &P3 = *p.f3;
    K *Hk = (K *)(ws + p.off_hkeys);
    V *Hv = HV ? (V *)(ws + p.off_hvals) : nullptr;
    char *fw = ws + p.off_forest;
    char *img = fw + p.forest.off_f2;
    hipError_t e = hipMemcpyAsync(img, P3.image.data(), P3.image.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    for (size_t i = 0; i < P3.trees.size(); ++i) {
        Forest F{};
        F.p0 = Prob{0, 0, n, 0, 0};
        e = run_forest<KT, V>(keys, Hk, vals, Hv, F, p.forest, fw, st, gate, true, P3.trees[i].get(),
                              img + P3.tree_off[i]);
        if (e != hipSuccess) return e;
    }
    for (const FrogMerge &m : P3.spine) {
        Forest F{};
        F.p0 = Prob{0, 0, n, 1, 0};
        F.m1 = m;
        F.use_m1 = 1;
        e = run_forest<KT, V>(keys, Hk, vals, Hv, F, p.forest, fw, st, gate, false);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

template <class KT, class V>
hipError_t run_sort(typename KT::T *keys, V *vals, int64_t n, char *ws, const SortPlan &p,
                    hipStream_t st, Gate gate)
{
    using K = typename KT::T;
    constexpr bool HV = ValOps<V>::has;
    if (n <= 1) return hipSuccess;
    if (p.f3) return run_frog3<KT, V>(keys, vals, n, ws, p, st, gate);
    Forest F{};
    F.p0 = Prob{0, 0, n, p.depth, 0};
    return run_forest<KT, V>(keys, (K *)(ws + p.off_hkeys), vals, HV ? (V *)(ws + p.off_hvals) : nullptr, F,
                             p.forest, ws + p.off_forest, st, gate, true, p.f2.get());
}

// explicit instantiations used by the ABI layer
SortPlan plan_f64(int64_t n, int64_t q, int algo, int64_t q2) { return make_plan<KeyF64, NoVal>(n, q, algo, q2); }
SortPlan plan_kv(int64_t n, int64_t q, int algo, int64_t q2) { return make_plan<KeyU64, uint32_t>(n, q, algo, q2); }

ForestPlan plan_forest_f64(int64_t num_keys, int64_t max_len, int64_t max_probs, int merge_ipt)
{
    if (merge_ipt == 8) return forest_plan_many<KeyF64T8, NoVal>(num_keys, max_len, max_probs);
    return forest_plan_many<KeyF64, NoVal>(num_keys, max_len, max_probs);
}

hipError_t sort_f64_async(double *keys, int64_t n, char *ws, const SortPlan &p, hipStream_t st,
                          const unsigned *gate, unsigned run_if)
{
    return run_sort<KeyF64, NoVal>(keys, (NoVal *)nullptr, n, ws, p, st, Gate{gate, run_if});
}

hipError_t sort_kv_async(uint64_t *keys, uint32_t *vals, int64_t n, char *ws, const SortPlan &p,
                         hipStream_t st)
{
    return run_sort<KeyU64, uint32_t>(keys, vals, n, ws, p, st, Gate{nullptr, 0u});
}

// In-place reversal of keys[0, n) (and vals), one pair (i, n-1-i) per thread:
// the right-anchored targets are the left-anchored ones of the opposite
// direction read backwards, and strictly reversed input is sorted by it.
template <class K, class V>
__global__ __launch_bounds__(256) void reverse_kernel(K *keys, V *vals, int64_t n, Gate gate)
{
    if (gate.closed()) return;
    const int64_t half = n / 2;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < half;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = n - 1 - i;
        const K a = keys[i], b = keys[j];
        keys[i] = b;
        keys[j] = a;
        if constexpr (ValOps<V>::has) {
            const V va = vals[i], vb = vals[j];
            vals[i] = vb;
            vals[j] = va;
        }
    }
}

template <class K, class V>
static void launch_reverse(K *keys, V *vals, int64_t n, hipStream_t st, Gate gate = Gate{nullptr, 0u})
{
    if (n < 2) return;
    const int64_t half = n / 2;
    hipLaunchKernelGGL((reverse_kernel<K, V>), dim3(grid_for(half, 256, 8192)), dim3(256), 0, st, keys, vals, n,
                       gate);
}

// ---------------------------------------------------------------------------
// input already in order, or reversed
// ---------------------------------------------------------------------------
// "Octosort", "Squidsort": bi-adaptive to presorted and reverse-sorted input.
// Before the tree runs, the call decides on the device whether the keys are
// already in the sort's order (every neighbour pair non-decreasing: nothing
// to do) or reversed (every pair strictly decreasing, or -- keys without
// values only -- non-increasing with every tie between bit-identical keys,
// i.e. no NaN and no zero: either way the reversal is the stable result);
// anything else is sorted.  4096 sampled pairs decide first, so unsorted
// input pays one small launch; the pass over every pair runs only when the
// sample finds no counter-example.  The decision (word 0) gates every later
// launch of the call; word 1 holds the properties still possible (the bits
// of order_bits).

template <class KT>
__global__ __launch_bounds__(256) void order_sample_kernel(const typename KT::T *keys, int64_t n, unsigned *word,
                                                           int keys_only, uint64_t *moved)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *moved = 0;     // the call's move count starts here
    const int64_t m = n - 1;             // pairs
    unsigned bits = 15u;
    for (int j = threadIdx.x; j < 4096; j += 256) {
        const int64_t i = (int64_t)j * m / 4096;
        bits &= order_bits<KT>(keys[i], keys[i + 1]);
    }
    __shared__ unsigned s_bits;
    if (threadIdx.x == 0) s_bits = 15u;
    __syncthreads();
    atomicAnd(&s_bits, bits);
    __syncthreads();
    if (threadIdx.x == 0) {
        word[1] = s_bits;
        word[0] = order_decisive<KT>(s_bits, keys_only != 0) ? (unsigned)ORD_CANDIDATE : (unsigned)ORD_SORT;
    }
}

template <class KT>
__global__ __launch_bounds__(256) void order_check_kernel(const typename KT::T *keys, int64_t n, unsigned *word,
                                                          int keys_only)
{
    if (word[0] != ORD_CANDIDATE) return;
    unsigned bits = word[1];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
         i < n - 1 && order_decisive<KT>(bits, keys_only != 0); i += (int64_t)gridDim.x * blockDim.x)
        bits &= order_bits<KT>(keys[i], keys[i + 1]);
    __shared__ unsigned s_bits;
    if (threadIdx.x == 0) s_bits = 15u;
    __syncthreads();
    atomicAnd(&s_bits, bits);
    __syncthreads();
    if (threadIdx.x == 0 && s_bits != 15u) atomicAnd(word + 1, s_bits);
}

__global__ void order_decide_kernel(unsigned *word, int keys_only)
{
    if (word[0] != ORD_CANDIDATE) return;
    const unsigned b = word[1];
    word[0] = (b & 1u)                                        ? (unsigned)ORD_IN_ORDER
              : ((b & 2u) || (keys_only && (b & 4u) && (b & 8u))) ? (unsigned)ORD_REVERSED
                                                                : (unsigned)ORD_SORT;
}

template <class KT>
static void launch_order_check(const typename KT::T *keys, int64_t n, unsigned *word, bool keys_only,
                               uint64_t *moved, hipStream_t st)
{
    const int ko = keys_only ? 1 : 0;
    hipLaunchKernelGGL((order_sample_kernel<KT>), dim3(1), dim3(256), 0, st, keys, n, word, ko, moved);
    hipLaunchKernelGGL((order_check_kernel<KT>), dim3(grid_for(n - 1, 256, 8192)), dim3(256), 0, st, keys, n,
                       word, ko);
    hipLaunchKernelGGL(order_decide_kernel, dim3(1), dim3(1), 0, st, word, ko);
}

// One stable sort with its order check: KT is the key order the tree sorts
// in; its result is left in place, or the input reversed, or the input kept.
template <class KT, class V>
static hipError_t run_sort_adaptive(typename KT::T *keys, V *vals, int64_t n, char *ws, const SortPlan &p,
                                    hipStream_t st)
{
    if (n <= 1) return hipSuccess;
    unsigned *word = (unsigned *)(ws + p.off_order);
    uint64_t *moved = (uint64_t *)(ws + p.off_forest + p.forest.off_ctrl + 4 * kMovedWord);
    launch_order_check<KT>(keys, n, word, !ValOps<V>::has, moved, st);
    hipError_t e = run_sort<KT, V>(keys, vals, n, ws, p, st, Gate{word, (unsigned)ORD_SORT});
    if (e != hipSuccess) return e;
    launch_reverse(keys, vals, n, st, Gate{word, (unsigned)ORD_REVERSED});
    return hipGetLastError();
}

ErrWords plain_err_words(char *ws, const SortPlan &p)
{
    ErrWords e{};
    e.add((unsigned *)(ws + p.off_forest + p.forest.off_ctrl) + kErrWord, DEVERR_WAIT);
    return e;
}

hipError_t sort_f64_target_async(double *keys, int64_t n, int target, char *ws, const SortPlan &p, hipStream_t st)
{
    if (n <= 1) return hipSuccess;
    const ErrWords ew = plain_err_words(ws, p);
    hipError_t e = err_words_begin(ew, st);
    if (e != hipSuccess) return e;
    // targets: 0 AscLeft, 1 AscRight = reversed DescLeft, 2 DescLeft,
    // 3 DescRight = reversed AscLeft
    e = (target == 1 || target == 2) ? run_sort_adaptive<KeyF64Desc, NoVal>(keys, (NoVal *)nullptr, n, ws, p, st)
                                     : run_sort_adaptive<KeyF64, NoVal>(keys, (NoVal *)nullptr, n, ws, p, st);
    if (e != hipSuccess) return e;
    if (target == 1 || target == 3) launch_reverse(keys, (NoVal *)nullptr, n, st);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return err_words_end(ew, st);
}

hipError_t sort_kv_target_async(uint64_t *keys, uint32_t *vals, int64_t n, int target, char *ws, const SortPlan &p,
                                hipStream_t st)
{
    if (n <= 1) return hipSuccess;
    const ErrWords ew = plain_err_words(ws, p);
    hipError_t e = err_words_begin(ew, st);
    if (e != hipSuccess) return e;
    e = (target == 1 || target == 2) ? run_sort_adaptive<KeyU64Desc, uint32_t>(keys, vals, n, ws, p, st)
                                     : run_sort_adaptive<KeyU64, uint32_t>(keys, vals, n, ws, p, st);
    if (e != hipSuccess) return e;
    if (target == 1 || target == 3) launch_reverse(keys, vals, n, st);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return err_words_end(ew, st);
}

hipError_t forest_f64_async(double *D, double *H, const Prob *probs, const unsigned *nprob, const ForestPlan &fp,
                            char *fw, hipStream_t st, const unsigned *gate, unsigned run_if, int merge_ipt)
{
    Forest F{};
    F.probs = probs;
    F.nprob = nprob;
    if (merge_ipt == 8)
        return run_forest<KeyF64T8, NoVal>(D, H, (NoVal *)nullptr, (NoVal *)nullptr, F, fp, fw, st,
                                           Gate{gate, run_if}, true);
    return run_forest<KeyF64, NoVal>(D, H, (NoVal *)nullptr, (NoVal *)nullptr, F, fp, fw, st, Gate{gate, run_if},
                                     true);
}

hipError_t merge_one_f64_async(double *D, double *H, int64_t n_space, const FrogMerge &m, char *ws,
                               const SortPlan &p, hipStream_t st, const unsigned *gate, unsigned run_if)
{
    using C = SortCfg<KeyF64, NoVal>;
    constexpr int TILE = C::MERGE_NT * C::MERGE_IPT;
    const int64_t n = m.nl + m.nr;
    if (n <= 0) return hipSuccess;
    Forest F{};
    F.p0 = Prob{0, 0, n_space, 1, 0};
    F.m1 = m;
    F.use_m1 = 1;
    // the plain plan's forest area holds the node's tiles when it covers
    // a sort of at least n keys
    if (forest_tickets<TILE>(F, F.p0, 1) > p.forest.max_tickets ||
        forest_splits<TILE>(F, F.p0, 1) > p.forest.max_splits)
        return hipErrorInvalidValue;
    return run_forest<KeyF64, NoVal>(D, H, (NoVal *)nullptr, (NoVal *)nullptr, F, p.forest, ws + p.off_forest, st,
                                     Gate{gate, run_if}, false);
}

}  // namespace gs
