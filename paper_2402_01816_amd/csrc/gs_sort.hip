// Plain frog mergesort for one array: leaf block sort fused with the setup
// placement, merge-path partition, dependency windows, and the in-place frog
// merge per level.
//
// Paper: "Symmetric merging" (mirrored child placement, merge from the inner
// ends outward), "Frogsort1" (rule 1: surplus to the outer side; rule 2:
// buffer floor(n/2); the setup recursion that places elements before merging).
#include <hip/hip_runtime.h>

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

// ---------------------------------------------------------------------------
// leaf kernel: sort each leaf's input chunk and place it at its frog slot
// ---------------------------------------------------------------------------
// Leaf i takes the i-th contiguous chunk of the input (the order the setup
// recursion visits elements) and leaves it sorted at its data start, which is
// never before its input offset.  A leaf's output can therefore only cover
// input chunks of leaves with a larger index: leaves take tickets in
// descending index order, and each waits for the leaves whose chunks its
// output covers.
template <class KT, class V, int NT, int IPT>
__global__ __launch_bounds__(NT) void leaf_kernel(Space<typename KT::T> keys, Space<V> vals,
                                                  int64_t n_total, int depth, int64_t nleaves,
                                                  unsigned *ticket_ctr, unsigned *status,
                                                  unsigned epoch, unsigned *err, Gate gate)
{
    using K = typename KT::T;
    using KF = typename FastKey<KT>::type;
    constexpr bool HV = ValOps<V>::has;
    using VS = typename std::conditional<HV, V, char>::type;
    constexpr int TILE = NT * IPT;
    constexpr int SLOTS = lds_slots<TILE>();
    __shared__ K sk[SLOTS];
    __shared__ VS sv[HV ? SLOTS : 1];
    __shared__ unsigned s_ticket;
    if (gate.closed()) return;

    const int tid = threadIdx.x;
    if (tid == 0) s_ticket = atomicAdd(ticket_ctr, 1u);
    __syncthreads();
    const int64_t t = __builtin_amdgcn_readfirstlane(s_ticket);
    const int64_t leaf = nleaves - 1 - t;
    const FrogNode f = frog_node(n_total, depth, leaf);
    const int len = (int)f.n;
    const int64_t src = f.in_off;
    const int64_t dst = frog_data_start(f);

    // load the chunk (input elements all live in the caller's array) with
    // straight-line loads from clamped indices, all issued before the first
    // LDS write
    bool nan_here = false;
    {
        K lk[IPT];
        VS lv[IPT];
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            const int i = tid + r * NT;
            const int ic = min(i, len - 1);
            lk[r] = keys.D[src + ic];
            if constexpr (HV) lv[r] = vals.D[src + ic];
        }
#pragma unroll
        for (int r = 0; r < IPT; ++r) nan_here |= is_nan_key(lk[r]);
        const bool any_nan = __syncthreads_or(nan_here) != 0;
        // slots past the chunk get a padding key that sorts after every real
        // key (ties with it stay behind the real keys)
        const K pad = any_nan ? KT::pad() : KF::pad();
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            const int i = tid + r * NT;
            sk[lpad(i)] = i < len ? lk[r] : pad;
            if constexpr (HV) sv[lpad(i)] = i < len ? lv[r] : VS();
        }
        nan_here = any_nan;
    }
    __syncthreads();
    if (tid == 0) st_status(status + t, (epoch << 2) | ST_LOADED);

    if (nan_here) block_sort_lds<KT, VS, HV, NT, IPT>(sk, sv);
    else block_sort_lds<KF, VS, HV, NT, IPT>(sk, sv);

    // wait for the leaves whose input chunks the destination covers
    if (tid < 64 && dst < n_total) {
        const int64_t end = (dst + len < n_total ? dst + len : n_total) - 1;
        const int64_t lo_leaf = frog_leaf_of(n_total, depth, dst);
        const int64_t hi_leaf = frog_leaf_of(n_total, depth, end);
        wait_window(status, nleaves - 1 - hi_leaf, nleaves - 1 - lo_leaf, t, epoch, err);
    }
    __syncthreads();

#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const int i = tid + r * NT;
        if (i < len) {
            *keys.at(dst + i) = sk[lpad(i)];
            if constexpr (HV) *vals.at(dst + i) = sv[lpad(i)];
        }
    }
}

// ---------------------------------------------------------------------------
// partition kernel: merge-path splits at every tile boundary of every node
// ---------------------------------------------------------------------------
// One thread per (node, boundary j): binary search for the number of left-run
// elements among the first j*TILE outputs of the node's stable merge.  (The
// searches are bound by the rate of random reads, so one probe per step is
// the cheapest form.)
template <class KT, int TILE>
__global__ __launch_bounds__(256) void partition_kernel(Space<typename KT::T> keys, MergeGeo geo,
                                                        int64_t nnodes, int64_t tpn, int64_t *splits,
                                                        Gate gate)
{
    if (gate.closed()) return;
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nnodes * (tpn + 1)) return;
    const int64_t node = w / (tpn + 1);
    const int64_t j = w - node * (tpn + 1);
    const FrogMerge m = geo.node(node);
    const int64_t nn = m.nl + m.nr;
    int64_t kk = j * TILE;
    if (kk > nn) kk = nn;
    int64_t lo = kk > m.nr ? kk - m.nr : 0;
    int64_t hi = kk < m.nl ? kk : m.nl;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (KT::less(*keys.at(m.r0 + (kk - 1 - mid)), *keys.at(m.l0 + mid))) hi = mid;
        else lo = mid + 1;
    }
    splits[w] = lo;
}

// ---------------------------------------------------------------------------
// dependency windows of every merge tile
// ---------------------------------------------------------------------------
// A left node's tile with output ranks [k0,k1) overwrites the outer-run (left
// child) elements with indices [k0, min(k1,nl)); a right node's tile overwrites
// the outer-run (right child) elements with indices [k0-nl, k1-nl) clipped to
// [0,nr).  The tiles that read those elements follow from the splits; their
// tickets form one contiguous range that never starts after the tile's own.
__device__ __forceinline__ int64_t upper_bound_splits(const int64_t *sp, int64_t count, int64_t x)
{
    int64_t lo = 0, hi = count;          // first j with sp[j] > x
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (sp[mid] > x) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

template <int TILE>
__device__ __forceinline__ int64_t upper_bound_bsplits(const int64_t *sp, int64_t count, int64_t n,
                                                       int64_t x)
{
    int64_t lo = 0, hi = count;          // first j with min(j*TILE,n) - sp[j] > x
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        const int64_t k = mid * TILE < n ? mid * TILE : n;
        if (k - sp[mid] > x) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

template <int TILE>
__global__ __launch_bounds__(256) void depwin_kernel(MergeGeo geo, int64_t nnodes, int64_t tpn,
                                                     const int64_t *splits, int64_t *deps, Gate gate)
{
    if (gate.closed()) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nnodes * tpn) return;
    const int64_t node = t / tpn;
    const int64_t q = t - node * tpn;
    const int64_t first = node * tpn;
    const FrogMerge m = geo.node(node);
    const int64_t nn = m.nl + m.nr;
    const int64_t j = m.left ? (tpn - 1 - q) : q;
    int64_t k0 = j * TILE;
    if (k0 > nn) k0 = nn;
    int64_t k1 = k0 + TILE;
    if (k1 > nn) k1 = nn;
    const int64_t *sp = splits + node * (tpn + 1);
    int64_t lo = 1, hi = 0;              // empty window
    if (k0 < k1) {
        if (m.outer == 0) {              // first run at [out0, out0+nl), top-down
            if (k0 < m.nl) {
                const int64_t e = (k1 < m.nl ? k1 : m.nl) - 1;
                const int64_t j0 = upper_bound_splits(sp, tpn + 1, k0) - 1;
                const int64_t j1 = upper_bound_splits(sp, tpn + 1, e) - 1;
                lo = first + (tpn - 1 - j1);
                hi = first + (tpn - 1 - j0);
            }
        } else if (m.outer == 1) {       // second run at [out0+nl, out0+n), bottom-up
            if (k1 > m.nl) {
                const int64_t b0 = k0 > m.nl ? k0 - m.nl : 0;
                const int64_t b1 = (k1 - m.nl < m.nr ? k1 - m.nl : m.nr) - 1;
                const int64_t j0 = upper_bound_bsplits<TILE>(sp, tpn + 1, nn, b0) - 1;
                const int64_t j1 = upper_bound_bsplits<TILE>(sp, tpn + 1, nn, b1) - 1;
                lo = first + j0;
                hi = first + j1;
            }
        } else {                         // first run at [out0+nr, out0+n), bottom-up
            if (k1 > m.nr) {
                const int64_t a0 = k0 > m.nr ? k0 - m.nr : 0;
                const int64_t a1 = (k1 - m.nr < m.nl ? k1 - m.nr : m.nl) - 1;
                const int64_t j0 = upper_bound_splits(sp, tpn + 1, a0) - 1;
                const int64_t j1 = upper_bound_splits(sp, tpn + 1, a1) - 1;
                lo = first + j0;
                hi = first + j1;
            }
        }
    }
    deps[2 * t] = lo;
    deps[2 * t + 1] = hi;
}

// ---------------------------------------------------------------------------
// merge kernel: persistent work-groups, one output tile per iteration
// ---------------------------------------------------------------------------
// A left node writes its output top-down (its outer run is the left child's
// data, which only moves right); a right node bottom-up (its outer run is the
// right child's data, which only moves left).  Inner runs lie outside the
// output.  Tickets are handed out in each node's write order.  A work-group
// takes the next ticket and issues that tile's loads while it merges and
// stores the current one.
struct MergeTile {
    int64_t t;        // ticket
    int64_t pa, pb;   // logical slots of the first left-run / right-run input
    int64_t o;        // logical slot of the first output
    int64_t dlo, dhi; // dependency window (tickets)
    int la, cnt;      // left-run inputs, total inputs (= outputs)
};

template <int TILE>
__device__ __forceinline__ MergeTile merge_tile_setup(int64_t t, const MergeGeo &geo, int64_t tpn,
                                                      const int64_t *splits, const int64_t *deps)
{
    MergeTile T;
    T.t = t;
    const int64_t node = (int64_t)((uint64_t)t / (uint64_t)tpn);
    const int64_t q = t - node * tpn;
    const FrogMerge m = geo.node(node);
    const int64_t nn = m.nl + m.nr;
    const int64_t j = m.left ? (tpn - 1 - q) : q;
    int64_t k0 = j * TILE;
    if (k0 > nn) k0 = nn;
    int64_t k1 = k0 + TILE;
    if (k1 > nn) k1 = nn;
    T.cnt = (int)(k1 - k0);
    T.la = 0;
    T.pa = T.pb = T.o = 0;
    T.dlo = 1;
    T.dhi = 0;
    if (T.cnt > 0) {
        const int64_t a0 = splits[node * (tpn + 1) + j];
        const int64_t a1 = splits[node * (tpn + 1) + j + 1];
        T.la = (int)(a1 - a0);
        T.pa = m.l0 + a0;
        T.pb = m.r0 + (k0 - a0);
        T.o = m.out0 + k0;
        T.dlo = deps[2 * t];
        T.dhi = deps[2 * t + 1];
    }
    return T;
}

template <class KT, class V, int NT, int IPT>
__global__ __launch_bounds__(NT) void merge_kernel(Space<typename KT::T> keys, Space<V> vals,
                                                   MergeGeo geo, int64_t tpn, int64_t ntiles,
                                                   const int64_t *splits, const int64_t *deps,
                                                   unsigned *ticket_ctr, unsigned *status,
                                                   unsigned epoch, unsigned *err, Gate gate)
{
    using K = typename KT::T;
    constexpr bool HV = ValOps<V>::has;
    using VS = typename std::conditional<HV, V, char>::type;
    constexpr int TILE = NT * IPT;
    constexpr int SLOTS = lds_slots<TILE>();
    __shared__ K sk[SLOTS];
    __shared__ VS sv[HV ? SLOTS : 1];
    __shared__ unsigned s_next;
    if (gate.closed()) return;

    const int tid = threadIdx.x;
    if (tid == 0) s_next = atomicAdd(ticket_ctr, 1u);
    __syncthreads();
    int64_t t = __builtin_amdgcn_readfirstlane(s_next);
    if (t >= ntiles) return;

    MergeTile cur = merge_tile_setup<TILE>(t, geo, tpn, splits, deps);
    K lk[IPT];
    VS lv[IPT];
    // Straight-line loads: indices past the tile are clamped to its last input
    // (an empty tile reads slot 0), so every load is valid and none needs a
    // branch; the values loaded for clamped indices are never stored.
    auto issue_loads = [&](const MergeTile &T) {
        const int last = T.cnt > 0 ? T.cnt - 1 : 0;
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            const int i = min(tid + r * NT, last);
            const int64_t p = i < T.la ? T.pa + i : T.pb + (i - T.la);
            lk[r] = *keys.at(p);
            if constexpr (HV) lv[r] = *vals.at(p);
        }
    };
    issue_loads(cur);

    for (;;) {
        // stage the current tile in LDS and publish that its inputs are read
        // (slots past the tile receive ignored values)
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            const int i = tid + r * NT;
            sk[lpad(i)] = lk[r];
            if constexpr (HV) sv[lpad(i)] = lv[r];
        }
        __syncthreads();
        unsigned nt = 0;
        if (tid == 0) {
            st_status(status + cur.t, (epoch << 2) | ST_LOADED);
            nt = atomicAdd(ticket_ctr, 1u);
        }

        // merge: thread tid produces outputs [tid*IPT, tid*IPT + nout)
        K k[IPT];
        VS v[IPT];
        int srcix[IPT];
        const int d = tid * IPT;
        int nout = cur.cnt - d;
        nout = nout < 0 ? 0 : (nout > IPT ? IPT : nout);
        const int la = cur.la, lb = cur.cnt - cur.la;
        if (nout > 0) {
            const int ai = merge_path_lds<KT>(d, la, lb, [&](int i) { return sk[lpad(i)]; },
                                              [&](int i) { return sk[lpad(la + i)]; });
            serial_merge<KT, IPT, HV>(sk, 0, la, la, lb, ai, d - ai, TILE, k, srcix);
            if constexpr (HV) {
#pragma unroll
                for (int i = 0; i < IPT; ++i) v[i] = sv[lpad(min(srcix[i], TILE))];
            }
        }
        if (tid == 0) s_next = nt;
        __syncthreads();

        // prefetch the next tile while this one waits and stores
        const int64_t t2 = __builtin_amdgcn_readfirstlane(s_next);
        const bool more = t2 < ntiles;
        MergeTile nxt;
        if (more) {
            nxt = merge_tile_setup<TILE>(t2, geo, tpn, splits, deps);
            issue_loads(nxt);
        }
        if (tid < 64) wait_window(status, cur.dlo, cur.dhi, cur.t, epoch, err);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            if (i < nout) {
                sk[lpad(d + i)] = k[i];
                if constexpr (HV) sv[lpad(d + i)] = v[i];
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            const int i = tid + r * NT;
            if (i < cur.cnt) {
                *keys.at(cur.o + i) = sk[lpad(i)];
                if constexpr (HV) *vals.at(cur.o + i) = sv[lpad(i)];
            }
        }
        if (!more) break;
        __syncthreads();                 // LDS reads done before the next staging
        cur = nxt;
    }
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
#ifndef GS_F64_MERGE_NT
#define GS_F64_MERGE_NT 256
#endif
#ifndef GS_F64_MERGE_IPT
#define GS_F64_MERGE_IPT 16
#endif
template <>
struct SortCfg<KeyF64, NoVal> {
    static constexpr int LEAF_NT = GS_F64_LEAF_NT, LEAF_IPT = GS_F64_LEAF_IPT;
    static constexpr int MERGE_NT = GS_F64_MERGE_NT, MERGE_IPT = GS_F64_MERGE_IPT;
};
template <>
struct SortCfg<KeyU64, uint32_t> {
    static constexpr int LEAF_NT = 256, LEAF_IPT = 16;
    static constexpr int MERGE_NT = 256, MERGE_IPT = 8;
};

template <class KT, class V>
int64_t leaf_size()
{
    return (int64_t)SortCfg<KT, V>::LEAF_NT * SortCfg<KT, V>::LEAF_IPT;
}

static int64_t align256(int64_t b) { return (b + 255) & ~(int64_t)255; }

template <class KT, class V>
SortPlan make_plan(int64_t n)
{
    using K = typename KT::T;
    constexpr bool HV = ValOps<V>::has;
    constexpr int TILE = SortCfg<KT, V>::MERGE_NT * SortCfg<KT, V>::MERGE_IPT;
    SortPlan p{};
    p.n = n;
    p.leaf = leaf_size<KT, V>();
    p.tile = TILE;
    p.depth = n > 1 ? frog_depth(n, p.leaf) : 0;
    int64_t max_tickets = (int64_t)1 << p.depth;     // leaf launch
    int64_t max_splits = 0;
    for (int d = 0; d < p.depth; ++d) {
        const int64_t tpn = (frog_max_node(n, d) + TILE - 1) / TILE;
        const int64_t nn = (int64_t)1 << d;
        if (nn * tpn > max_tickets) max_tickets = nn * tpn;
        if (nn * (tpn + 1) > max_splits) max_splits = nn * (tpn + 1);
    }
    const int64_t h = n / 2;
    p.off_hkeys = 0;
    p.off_hvals = align256(h * (int64_t)sizeof(K));
    p.off_tickets = p.off_hvals + (HV ? align256(h * (int64_t)sizeof(V)) : 0);
    p.n_tickets = 64;
    p.off_status = p.off_tickets + align256(p.n_tickets * 4);
    p.n_status = max_tickets;
    p.off_splits = p.off_status + align256(max_tickets * 4);
    p.off_deps = p.off_splits + align256(max_splits * 8);
    p.bytes = p.off_deps + align256(max_tickets * 16);
    if (n <= 1) p.bytes = 0;
    return p;
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

// Enqueues partition, dependency windows and the merge for one level (or one
// explicit node) whose control words start at `tickets`.
template <class KT, class V>
static void launch_level(Space<typename KT::T> sk, Space<V> sv, const MergeGeo &geo, int64_t nn, int64_t tpn,
                         int64_t *splits, int64_t *deps, unsigned *ticket, unsigned *status,
                         unsigned *errw, unsigned epoch, Gate gate, hipStream_t st)
{
    using C = SortCfg<KT, V>;
    constexpr int TILE = C::MERGE_NT * C::MERGE_IPT;
    auto merge_fn = merge_kernel<KT, V, C::MERGE_NT, C::MERGE_IPT>;
    static int64_t merge_groups = 0;
    const int64_t resident = resident_groups(merge_fn, C::MERGE_NT, merge_groups);
    const bool tr = trace_on();
    const int64_t nsplit = nn * (tpn + 1);
    const int64_t ntiles = nn * tpn;
    if (tr) trace_begin(TK_PARTITION, st);
    hipLaunchKernelGGL((partition_kernel<KT, TILE>), dim3((unsigned)((nsplit + 255) / 256)), dim3(256), 0, st,
                       sk, geo, nn, tpn, splits, gate);
    if (tr) trace_end(st);
    if (tr) trace_begin(TK_DEPWIN, st);
    hipLaunchKernelGGL((depwin_kernel<TILE>), dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, st, geo, nn,
                       tpn, (const int64_t *)splits, deps, gate);
    if (tr) trace_end(st);
    if (tr) trace_begin(TK_MERGE, st);
    const int64_t grid = ntiles < resident ? ntiles : resident;
    hipLaunchKernelGGL(merge_fn, dim3((unsigned)grid), dim3(C::MERGE_NT), 0, st, sk, sv, geo, tpn, ntiles,
                       (const int64_t *)splits, (const int64_t *)deps, ticket, status, epoch, errw, gate);
    if (tr) trace_end(st);
}

template <class KT, class V>
hipError_t run_sort(typename KT::T *keys, V *vals, int64_t n, char *ws, const SortPlan &p,
                    hipStream_t st, Gate gate)
{
    using K = typename KT::T;
    using C = SortCfg<KT, V>;
    constexpr bool HV = ValOps<V>::has;
    constexpr int TILE = C::MERGE_NT * C::MERGE_IPT;
    if (n <= 1) return hipSuccess;
    Space<K> sk{keys, (K *)(ws + p.off_hkeys), n};
    Space<V> sv{vals, HV ? (V *)(ws + p.off_hvals) : nullptr, n};
    unsigned *tickets = (unsigned *)(ws + p.off_tickets);
    unsigned *status = (unsigned *)(ws + p.off_status);
    int64_t *splits = (int64_t *)(ws + p.off_splits);
    int64_t *deps = (int64_t *)(ws + p.off_deps);

    const bool tr = trace_on();
    // tickets and status words start at zero on every call
    if (tr) trace_begin(TK_FILL, st);
    launch_fill_u32(tickets, (p.off_splits - p.off_tickets) / 4, 0u, st);
    if (tr) trace_end(st);

    const int D = p.depth;
    unsigned epoch = 1;
    if (tr) trace_begin(TK_LEAF, st);
    hipLaunchKernelGGL((leaf_kernel<KT, V, C::LEAF_NT, C::LEAF_IPT>), dim3((unsigned)((int64_t)1 << D)),
                       dim3(C::LEAF_NT), 0, st, sk, sv, n, D, (int64_t)1 << D, tickets + 0, status,
                       epoch, tickets + kErrWord, gate);
    if (tr) trace_end(st);
    for (int d = D - 1; d >= 0; --d) {
        ++epoch;
        MergeGeo geo{};
        geo.n_total = n;
        geo.depth = d;
        geo.single = 0;
        const int64_t nn = (int64_t)1 << d;
        const int64_t tpn = (frog_max_node(n, d) + TILE - 1) / TILE;
        launch_level<KT, V>(sk, sv, geo, nn, tpn, splits, deps, tickets + (D - d), status,
                            tickets + kErrWord, epoch, gate, st);
    }
    return hipGetLastError();
}

// explicit instantiations used by the ABI layer
SortPlan plan_f64(int64_t n) { return make_plan<KeyF64, NoVal>(n); }
SortPlan plan_kv(int64_t n) { return make_plan<KeyU64, uint32_t>(n); }

hipError_t sort_f64_async(double *keys, int64_t n, char *ws, const SortPlan &p, hipStream_t st,
                          const unsigned *gate, unsigned run_if)
{
    return run_sort<KeyF64, NoVal>(keys, nullptr, n, ws, p, st, Gate{gate, run_if});
}

hipError_t sort_kv_async(uint64_t *keys, uint32_t *vals, int64_t n, char *ws, const SortPlan &p,
                         hipStream_t st)
{
    return run_sort<KeyU64, uint32_t>(keys, vals, n, ws, p, st, Gate{nullptr, 0u});
}

hipError_t merge_one_f64_async(double *D, double *H, int64_t n_space, const FrogMerge &m, char *ws,
                               const SortPlan &p, hipStream_t st, const unsigned *gate, unsigned run_if)
{
    using C = SortCfg<KeyF64, NoVal>;
    constexpr int TILE = C::MERGE_NT * C::MERGE_IPT;
    const int64_t n = m.nl + m.nr;
    if (n <= 0) return hipSuccess;
    Space<double> sk{D, H, n_space};
    Space<NoVal> sv{nullptr, nullptr, n_space};
    unsigned *tickets = (unsigned *)(ws + p.off_tickets);
    unsigned *status = (unsigned *)(ws + p.off_status);
    int64_t *splits = (int64_t *)(ws + p.off_splits);
    int64_t *deps = (int64_t *)(ws + p.off_deps);
    launch_fill_u32(tickets, (p.off_splits - p.off_tickets) / 4, 0u, st);
    MergeGeo geo{};
    geo.n_total = n;
    geo.depth = 0;
    geo.single = 1;
    geo.m1 = m;
    const int64_t tpn = (n + TILE - 1) / TILE;
    launch_level<KeyF64, NoVal>(sk, sv, geo, 1, tpn, splits, deps, tickets + 1, status, tickets + kErrWord, 1u,
                                Gate{gate, run_if}, st);
    return hipGetLastError();
}

}  // namespace gs
