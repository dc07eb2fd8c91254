// Plain frog mergesort for one array: leaf block sort fused with the setup
// placement, merge-path partition, and the in-place frog merge per level.
//
// Paper: "Symmetric merging" (mirrored child placement, merge from the inner
// ends outward), "Frogsort1" (rule 1: surplus to the outer side; rule 2:
// buffer floor(n/2); the setup recursion that places elements before merging).
#include <hip/hip_runtime.h>

#include <type_traits>

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

template <class V>
struct ValOps {
    static constexpr bool has = true;
};
template <>
struct ValOps<NoVal> {
    static constexpr bool has = false;
};

// ---------------------------------------------------------------------------
// leaf kernel: sort each leaf's input chunk and place it at its frog slot
// ---------------------------------------------------------------------------
// Leaf i takes the i-th contiguous chunk of the input (the order the setup
// recursion visits elements) and leaves it sorted at its data start, which is
// never before its input offset.  A leaf's output can therefore only cover
// input chunks of leaves with a larger index, so leaves are processed in
// descending index order under the ordered-store protocol.
template <class KT, class V, int NT, int IPT>
__global__ __launch_bounds__(NT) void leaf_kernel(Space<typename KT::T> keys, Space<V> vals,
                                                  int64_t n_total, int depth, int64_t nleaves,
                                                  unsigned *ticket_ctr, unsigned *status,
                                                  unsigned epoch, unsigned *err)
{
    using K = typename KT::T;
    constexpr bool HV = ValOps<V>::has;
    constexpr int TILE = NT * IPT;
    __shared__ K sk[TILE];
    __shared__ typename std::conditional<HV, V, char>::type sv[HV ? TILE : 1];
    __shared__ unsigned s_ticket;

    const int tid = threadIdx.x;
    if (tid == 0) s_ticket = atomicAdd(ticket_ctr, 1u);
    __syncthreads();
    const int64_t t = s_ticket;
    const int64_t leaf = nleaves - 1 - t;
    const FrogNode f = frog_node(n_total, depth, leaf);
    const int len = (int)f.n;
    const int64_t src = f.in_off;
    const int64_t dst = frog_data_start(f);

    // load the chunk (input elements all live in the caller's array)
    for (int i = tid; i < TILE; i += NT) {
        if (i < len) {
            sk[i] = keys.D[src + i];
            if constexpr (HV) sv[i] = vals.D[src + i];
        } else {
            sk[i] = KT::pad();
            if constexpr (HV) sv[i] = V();
        }
    }
    __syncthreads();
    if (tid == 0) st_status(status + t, (epoch << 2) | ST_LOADED);

    // per-thread odd-even transposition sort: only adjacent strict inversions
    // are exchanged, so equal keys keep their order
    K k[IPT];
    typename std::conditional<HV, V, char>::type v[IPT];
    const int base = tid * IPT;
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        k[i] = sk[base + i];
        if constexpr (HV) v[i] = sv[base + i];
    }
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
#pragma unroll
        for (int i = (r & 1); i + 1 < IPT; i += 2) {
            if (KT::less(k[i + 1], k[i])) {
                K tk = k[i]; k[i] = k[i + 1]; k[i + 1] = tk;
                if constexpr (HV) { auto tv = v[i]; v[i] = v[i + 1]; v[i + 1] = tv; }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        sk[base + i] = k[i];
        if constexpr (HV) sv[base + i] = v[i];
    }
    __syncthreads();

    // merge rounds in LDS: runs of w -> 2w
    for (int w = IPT; w < TILE; w *= 2) {
        const int pair = base / (2 * w);
        const int a0 = pair * 2 * w;
        const int b0 = a0 + w;
        const int kd = base - a0;
        int ai = merge_path_lds<KT>(kd, w, w, [&](int i) { return sk[a0 + i]; },
                                    [&](int i) { return sk[b0 + i]; });
        int bi = kd - ai;
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            bool takeB;
            if (ai >= w) takeB = true;
            else if (bi >= w) takeB = false;
            else takeB = KT::less(sk[b0 + bi], sk[a0 + ai]);
            const int idx = takeB ? b0 + bi : a0 + ai;
            k[i] = sk[idx];
            if constexpr (HV) v[i] = sv[idx];
            if (takeB) ++bi; else ++ai;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            sk[base + i] = k[i];
            if constexpr (HV) sv[base + i] = v[i];
        }
        __syncthreads();
    }

    // wait until every leaf with a larger index has loaded its chunk
    if (tid < 64) lookback_wait(status, 0, t, epoch, err);
    __syncthreads();

    for (int i = tid; i < len; i += NT) {
        *keys.at(dst + i) = sk[i];
        if constexpr (HV) *vals.at(dst + i) = sv[i];
    }
}

// ---------------------------------------------------------------------------
// partition kernel: merge-path splits at every tile boundary of every node
// ---------------------------------------------------------------------------
// One wavefront per (node, boundary j): a 64-ary search for the number of
// left-run elements among the first j*TILE outputs of the node's stable merge.
template <class KT, int TILE>
__global__ __launch_bounds__(256) void partition_kernel(Space<typename KT::T> keys, int64_t n_total,
                                                        int depth, int64_t nnodes, int64_t tpn,
                                                        int64_t *splits)
{
    using K = typename KT::T;
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= nnodes * (tpn + 1)) return;
    const int64_t node = w / (tpn + 1);
    const int64_t j = w % (tpn + 1);
    const FrogNode f = frog_node(n_total, depth, node);
    const FrogMerge m = frog_merge_of(f);
    int64_t kk = j * TILE;
    if (kk > f.n) kk = f.n;
    int64_t lo = kk > m.nr ? kk - m.nr : 0;
    int64_t hi = kk < m.nl ? kk : m.nl;
    while (lo < hi) {
        const int64_t span = hi - lo;
        const int64_t step = (span + 63) / 64;
        const int64_t a = lo + (int64_t)lane * step;
        bool need_more_a = false;
        if (a < hi) {
            const K av = *keys.at(m.l0 + a);
            const K bv = *keys.at(m.r0 + (kk - 1 - a));
            need_more_a = !KT::less(bv, av);
        }
        const int c = __popcll(__ballot(need_more_a));
        if (step == 1) { lo += c; break; }
        if (c == 0) break;                      // first candidate already settles it
        const int64_t nlo = lo + (int64_t)(c - 1) * step + 1;
        const int64_t nhi = lo + (int64_t)c * step;
        lo = nlo;
        hi = nhi < hi ? nhi : hi;
    }
    if (lane == 0) splits[w] = lo;
}

// ---------------------------------------------------------------------------
// merge kernel: one output tile of one node per work-group
// ---------------------------------------------------------------------------
// A left node writes its output top-down (its outer run is the left child's
// data, which only moves right); a right node bottom-up (its outer run is the
// right child's data, which only moves left).  Inner runs lie outside the
// output.  Tickets are handed out in each node's write order.
template <class KT, class V, int NT, int IPT>
__global__ __launch_bounds__(NT) void merge_kernel(Space<typename KT::T> keys, Space<V> vals,
                                                   int64_t n_total, int depth, int64_t tpn,
                                                   const int64_t *splits, unsigned *ticket_ctr,
                                                   unsigned *status, unsigned epoch, unsigned *err)
{
    using K = typename KT::T;
    constexpr bool HV = ValOps<V>::has;
    constexpr int TILE = NT * IPT;
    __shared__ K sk[TILE];
    __shared__ typename std::conditional<HV, V, char>::type sv[HV ? TILE : 1];
    __shared__ unsigned s_ticket;

    const int tid = threadIdx.x;
    if (tid == 0) s_ticket = atomicAdd(ticket_ctr, 1u);
    __syncthreads();
    const int64_t t = s_ticket;
    const int64_t node = t / tpn;
    const int64_t q = t - node * tpn;
    const int64_t first = node * tpn;
    const FrogNode f = frog_node(n_total, depth, node);
    const FrogMerge m = frog_merge_of(f);
    const int64_t j = m.left ? (tpn - 1 - q) : q;
    int64_t k0 = j * TILE;
    if (k0 > f.n) k0 = f.n;
    int64_t k1 = k0 + TILE;
    if (k1 > f.n) k1 = f.n;
    if (k0 >= k1) {                              // empty tile (node shorter than tpn tiles)
        if (tid == 0) st_status(status + t, (epoch << 2) | ST_LOADED);
        return;
    }
    const int64_t a0 = splits[node * (tpn + 1) + j];
    const int64_t a1 = splits[node * (tpn + 1) + j + 1];
    const int la = (int)(a1 - a0);
    const int lb = (int)((k1 - a1) - (k0 - a0));
    const int64_t b0 = k0 - a0;
    const int cnt = la + lb;

    for (int i = tid; i < cnt; i += NT) {
        const int64_t p = i < la ? m.l0 + a0 + i : m.r0 + b0 + (i - la);
        sk[i] = *keys.at(p);
        if constexpr (HV) sv[i] = *vals.at(p);
    }
    __syncthreads();
    if (tid == 0) st_status(status + t, (epoch << 2) | ST_LOADED);

    K k[IPT];
    typename std::conditional<HV, V, char>::type v[IPT];
    const int d = tid * IPT;
    int nout = cnt - d;
    nout = nout < 0 ? 0 : (nout > IPT ? IPT : nout);
    if (nout > 0) {
        int ai = merge_path_lds<KT>(d, la, lb, [&](int i) { return sk[i]; },
                                    [&](int i) { return sk[la + i]; });
        int bi = d - ai;
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            if (i < nout) {
                bool takeB;
                if (ai >= la) takeB = true;
                else if (bi >= lb) takeB = false;
                else takeB = KT::less(sk[la + bi], sk[ai]);
                const int idx = takeB ? la + bi : ai;
                k[i] = sk[idx];
                if constexpr (HV) v[i] = sv[idx];
                if (takeB) ++bi; else ++ai;
            }
        }
    }

    if (tid < 64) lookback_wait(status, first, t, epoch, err);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        if (i < nout) {
            sk[d + i] = k[i];
            if constexpr (HV) sv[d + i] = v[i];
        }
    }
    __syncthreads();
    const int64_t o = m.out0 + k0;
    for (int i = tid; i < cnt; i += NT) {
        *keys.at(o + i) = sk[i];
        if constexpr (HV) *vals.at(o + i) = sv[i];
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
template <class KT, class V>
struct SortCfg;
template <>
struct SortCfg<KeyF64, NoVal> {
    static constexpr int LEAF_NT = 256, LEAF_IPT = 16;
    static constexpr int MERGE_NT = 256, MERGE_IPT = 16;
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
    p.bytes = p.off_splits + align256(max_splits * 8);
    if (n <= 1) p.bytes = 0;
    return p;
}

template <class KT, class V>
hipError_t run_sort(typename KT::T *keys, V *vals, int64_t n, char *ws, const SortPlan &p,
                    hipStream_t st)
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
                       epoch, tickets + kErrWord);
    if (tr) trace_end(st);
    for (int d = D - 1; d >= 0; --d) {
        ++epoch;
        const int64_t nn = (int64_t)1 << d;
        const int64_t tpn = (frog_max_node(n, d) + TILE - 1) / TILE;
        const int64_t nsplit = nn * (tpn + 1);
        if (tr) trace_begin(TK_PARTITION, st);
        hipLaunchKernelGGL((partition_kernel<KT, TILE>), dim3((unsigned)((nsplit + 3) / 4)), dim3(256),
                           0, st, sk, n, d, nn, tpn, splits);
        if (tr) trace_end(st);
        if (tr) trace_begin(TK_MERGE, st);
        hipLaunchKernelGGL((merge_kernel<KT, V, C::MERGE_NT, C::MERGE_IPT>), dim3((unsigned)(nn * tpn)),
                           dim3(C::MERGE_NT), 0, st, sk, sv, n, d, tpn, (const int64_t *)splits,
                           tickets + (D - d), status, epoch, tickets + kErrWord);
        if (tr) trace_end(st);
    }
    return hipGetLastError();
}

// explicit instantiations used by the ABI layer
SortPlan plan_f64(int64_t n) { return make_plan<KeyF64, NoVal>(n); }
SortPlan plan_kv(int64_t n) { return make_plan<KeyU64, uint32_t>(n); }

hipError_t sort_f64_async(double *keys, int64_t n, char *ws, const SortPlan &p, hipStream_t st)
{
    return run_sort<KeyF64, NoVal>(keys, nullptr, n, ws, p, st);
}

hipError_t sort_kv_async(uint64_t *keys, uint32_t *vals, int64_t n, char *ws, const SortPlan &p,
                         hipStream_t st)
{
    return run_sort<KeyU64, uint32_t>(keys, vals, n, ws, p, st);
}

}  // namespace gs
