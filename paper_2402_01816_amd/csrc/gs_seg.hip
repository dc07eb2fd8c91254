// Segmented sort: many independent arrays of uneven length, one persistent
// launch.
//
// Every segment is sorted on its own by the same stable method as the plain
// path ("Definition of sorting": ascending, ties in input order; "Frogsort1":
// half buffer, mirrored children, merges from the inner ends outward).
// Segments are grouped by size class on the device.  A work item is either a
// batch of short segments of one class, each placed in its own aligned
// power-of-two block of one LDS tile and block-sorted together, or one long
// segment that a single work-group frog-sorts end to end: leaves in LDS, then
// every node's merge streamed through LDS windows in the node's write order,
// which is the order in which in-place frog merging is safe.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "gs_block.h"
#include "gs_device.h"
#include "gs_internal.h"

namespace gs {

namespace {

constexpr int SEG_NT = 256;
constexpr int SEG_IPT = 16;
constexpr int SEG_TILE = SEG_NT * SEG_IPT;         // 4096 keys per LDS tile
constexpr int SEG_LOG_TILE = 12;
constexpr int SEG_MIPT = 8;                         // merge outputs per thread
constexpr int SEG_WIN = SEG_NT * SEG_MIPT;          // 2048-key window per run
constexpr int SEG_SLOTS = lds_slots<SEG_TILE>();
constexpr int SEG_CLASS_LONG = 13;                  // longer than one tile

// control words at the start of the segment workspace
constexpr int C_INVALID = 0;
constexpr int C_TICKET = 1;
constexpr int C_HIST = 16;                          // 16 class counters

__device__ __forceinline__ int seg_class(int64_t len)
{
    if (len <= 1) return 0;
    if (len > SEG_TILE) return SEG_CLASS_LONG;
    int c = 4;                                      // at least 16 keys per block
    while (((int64_t)1 << c) < len) ++c;
    return c;
}

}  // namespace

// ---------------------------------------------------------------------------
// 1. validate the offsets and count segments per class
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void seg_classify_kernel(const int64_t *offsets, int64_t nseg,
                                                           int64_t num_keys, unsigned *ctrl,
                                                           int *cls, int *rank, Gate gate)
{
    if (gate.closed()) return;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nseg) return;
    const int64_t lo = offsets[s], hi = offsets[s + 1];
    if (lo < 0 || hi < lo || hi > num_keys) {
        atomicOr(ctrl + C_INVALID, 1u);
        cls[s] = 0;
        return;
    }
    const int c = seg_class(hi - lo);
    cls[s] = c;
    rank[s] = (int)atomicAdd(ctrl + C_HIST + c, 1u);
}

// ---------------------------------------------------------------------------
// 2. place segment ids into one list ordered by class
// ---------------------------------------------------------------------------
// First list position of class c (classes in work-list order).
__device__ __forceinline__ int64_t class_base(const unsigned *ctrl, int c)
{
    int64_t acc = 0;
    for (int pos = 0; pos <= 9; ++pos) {
        const int cc = pos == 0 ? SEG_CLASS_LONG : 12 - (pos - 1);
        if (cc == c) return acc;
        acc += ctrl[C_HIST + cc];
    }
    return acc;
}

__global__ __launch_bounds__(256) void seg_scatter_kernel(int64_t nseg, const unsigned *ctrl,
                                                          const int *cls, const int *rank,
                                                          int *list, Gate gate)
{
    if (gate.closed()) return;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nseg || ctrl[C_INVALID]) return;
    const int c = cls[s];
    if (c == 0) return;
    list[class_base(ctrl, c) + rank[s]] = (int)s;
}

// ---------------------------------------------------------------------------
// 3. the persistent sorter
// ---------------------------------------------------------------------------

// Load keys [src, src+cnt) of a space into logical LDS slots [dst, dst+cnt);
// cnt <= SEG_WIN and uniform across the work-group.  Straight-line loads from
// clamped indices; nothing is read when cnt is 0 (src may then be one past
// the run).
template <class K>
__device__ __forceinline__ void load_window(K *sk, const Space<K> &sp, int64_t src, int cnt, int dst)
{
    if (cnt <= 0) return;
    const int last = cnt - 1;
    K r[SEG_MIPT];
#pragma unroll
    for (int q = 0; q < SEG_MIPT; ++q) {
        const int i = min((int)threadIdx.x + q * SEG_NT, last);
        r[q] = *sp.at(src + i);
    }
#pragma unroll
    for (int q = 0; q < SEG_MIPT; ++q) {
        const int i = (int)threadIdx.x + q * SEG_NT;
        if (i < cnt) sk[lpad(dst + i)] = r[q];
    }
}

// Stable merge of c outputs from LDS: A = logical [a_base, a_base+na),
// B = [b_base, b_base+nb), na + nb = c <= SEG_WIN; written to the space at
// logical slots [o, o+c) (through LDS for coalesced stores).
template <class KT>
__device__ __forceinline__ void merge_window_out(typename KT::T *sk, int a_base, int na, int b_base,
                                                 int nb, const Space<typename KT::T> &sp, int64_t o)
{
    using K = typename KT::T;
    const int tid = threadIdx.x;
    const int c = na + nb;
    const int d = tid * SEG_MIPT;
    K k[SEG_MIPT];
    int srcix[SEG_MIPT];
    int nout = c - d;
    nout = nout < 0 ? 0 : (nout > SEG_MIPT ? SEG_MIPT : nout);
    if (nout > 0) {
        const int ai = merge_path_lds<KT>(d, na, nb, [&](int i) { return sk[lpad(a_base + i)]; },
                                          [&](int i) { return sk[lpad(b_base + i)]; });
        serial_merge<KT, SEG_MIPT, false>(sk, a_base, na, b_base, nb, ai, d - ai, 2 * SEG_WIN, k,
                                          srcix);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < SEG_MIPT; ++i)
        if (i < nout) sk[lpad(d + i)] = k[i];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < SEG_MIPT; ++q) {
        const int i = tid + q * SEG_NT;
        if (i < c) *sp.at(o + i) = sk[lpad(i)];
    }
    __syncthreads();
}

// Merge-path split of the first `dd` outputs of merging LDS runs
// A = [a_base, a_base+na) and B = [b_base, b_base+nb); found by thread 0 and
// broadcast.
template <class KT>
__device__ __forceinline__ int window_split(const typename KT::T *sk, int a_base, int na, int b_base,
                                            int nb, int dd, int *s_bcast)
{
    if (threadIdx.x == 0)
        *s_bcast = merge_path_lds<KT>(dd, na, nb, [&](int i) { return sk[lpad(a_base + i)]; },
                                      [&](int i) { return sk[lpad(b_base + i)]; });
    __syncthreads();
    const int r = *s_bcast;
    __syncthreads();
    return r;
}

// One frog node's merge by a single work-group, streamed in the node's write
// order.  A left node produces its largest outputs first and writes them from
// the top of its output down; a right node produces its smallest outputs
// first and writes them upward.  Every output step overwrites only outer-run
// slots whose elements were already consumed, so re-reading the windows
// from memory at the next step always sees untouched input.
template <class KT>
__device__ void wg_stream_merge(typename KT::T *sk, const Space<typename KT::T> &sp,
                                const FrogMerge &m, int *s_bcast)
{
    const int64_t n = m.nl + m.nr;
    if (m.left) {
        int64_t ta = m.nl, tb = m.nr, rem = n;     // unconsumed prefixes, outputs left
        while (rem > 0) {
            const int wl = (int)(ta < SEG_WIN ? ta : SEG_WIN);
            const int wr = (int)(tb < SEG_WIN ? tb : SEG_WIN);
            load_window(sk, sp, m.l0 + ta - wl, wl, 0);
            load_window(sk, sp, m.r0 + tb - wr, wr, SEG_WIN);
            __syncthreads();
            const int c = (int)(rem < SEG_WIN ? rem : SEG_WIN);
            const int da = window_split<KT>(sk, 0, wl, SEG_WIN, wr, wl + wr - c, s_bcast);
            const int db = wl + wr - c - da;
            merge_window_out<KT>(sk, da, wl - da, SEG_WIN + db, wr - db, sp, m.out0 + rem - c);
            ta -= wl - da;
            tb -= wr - db;
            rem -= c;
        }
    } else {
        int64_t ia = 0, ib = 0, done = 0;           // consumed counts, outputs done
        while (done < n) {
            const int wl = (int)(m.nl - ia < SEG_WIN ? m.nl - ia : SEG_WIN);
            const int wr = (int)(m.nr - ib < SEG_WIN ? m.nr - ib : SEG_WIN);
            load_window(sk, sp, m.l0 + ia, wl, 0);
            load_window(sk, sp, m.r0 + ib, wr, SEG_WIN);
            __syncthreads();
            const int c = (int)(n - done < SEG_WIN ? n - done : SEG_WIN);
            const int ca = window_split<KT>(sk, 0, wl, SEG_WIN, wr, c, s_bcast);
            merge_window_out<KT>(sk, 0, ca, SEG_WIN, c - ca, sp, m.out0 + done);
            ia += ca;
            ib += c - ca;
            done += c;
        }
    }
}

// Load up to SEG_TILE keys [src, src+len) of `keys` into the LDS tile (slots
// past len padded), report whether any is NaN.
template <class KT>
__device__ __forceinline__ bool load_tile_padded(typename KT::T *sk, const typename KT::T *src, int len,
                                                 int P_log)
{
    using K = typename KT::T;
    using KF = typename FastKey<KT>::type;
    K r[SEG_IPT];
    bool nan_here = false;
    const int last = len > 0 ? len - 1 : 0;
#pragma unroll
    for (int q = 0; q < SEG_IPT; ++q) {
        const int i = min((int)threadIdx.x + q * SEG_NT, last);
        r[q] = src[i];
        nan_here |= ((int)threadIdx.x + q * SEG_NT < len) && is_nan_key(r[q]);
    }
    const bool any_nan = __syncthreads_or(nan_here) != 0;
    const K pad = any_nan ? KT::pad() : KF::pad();
#pragma unroll
    for (int q = 0; q < SEG_IPT; ++q) {
        const int i = (int)threadIdx.x + q * SEG_NT;
        sk[lpad(i)] = i < len ? r[q] : pad;
    }
    (void)P_log;
    return any_nan;
}

template <class KT>
__device__ __forceinline__ void sort_tile(typename KT::T *sk, bool any_nan, int maxw)
{
    using KF = typename FastKey<KT>::type;
    char dummy[1];
    __syncthreads();
    if (any_nan) block_sort_lds<KT, char, false, SEG_NT, SEG_IPT>(sk, dummy, maxw);
    else block_sort_lds<KF, char, false, SEG_NT, SEG_IPT>(sk, dummy, maxw);
}

// A whole frog sort of one segment by one work-group.
template <class KT>
__device__ void wg_frog_sort(typename KT::T *sk, const Space<typename KT::T> &sp, int *s_bcast)
{
    const int64_t n = sp.n;
    const int depth = frog_depth(n, SEG_TILE);
    // leaves in descending order: a leaf's slot only covers input chunks of
    // leaves with a larger index, which are already in place by then
    for (int64_t leaf = ((int64_t)1 << depth) - 1; leaf >= 0; --leaf) {
        const FrogNode f = frog_node(n, depth, leaf);
        const int len = (int)f.n;
        const bool any_nan = load_tile_padded<KT>(sk, sp.D + f.in_off, len, SEG_LOG_TILE);
        sort_tile<KT>(sk, any_nan, SEG_TILE);
        const int64_t dst = frog_data_start(f);
#pragma unroll
        for (int q = 0; q < SEG_IPT; ++q) {
            const int i = (int)threadIdx.x + q * SEG_NT;
            if (i < len) *sp.at(dst + i) = sk[lpad(i)];
        }
        __syncthreads();
    }
    for (int d = depth - 1; d >= 0; --d) {
        for (int64_t node = 0; node < ((int64_t)1 << d); ++node) {
            const FrogMerge m = frog_merge_of(frog_node(n, d, node));
            wg_stream_merge<KT>(sk, sp, m, s_bcast);
        }
    }
}

template <class KT>
__global__ __launch_bounds__(SEG_NT) void seg_sort_kernel(typename KT::T *keys, const int64_t *offsets,
                                                          typename KT::T *hbuf, unsigned *ctrl,
                                                          const int *list, Gate gate)
{
    using K = typename KT::T;
    __shared__ K sk[SEG_SLOTS];
    __shared__ int s_item;
    __shared__ int s_bcast;
    __shared__ int64_t s_off[SEG_NT];
    __shared__ int s_len[SEG_NT];
    __shared__ int64_t s_base[10], s_end[10];     // per work-list position
    if (gate.closed() || ctrl[C_INVALID]) return;

    // list start and cumulative work items of every class (work-list order)
    if (threadIdx.x == 0) {
        int64_t lacc = 0, iacc = 0;
        for (int pos = 0; pos <= 9; ++pos) {
            const int c = pos == 0 ? SEG_CLASS_LONG : 12 - (pos - 1);
            const int64_t cnt = ctrl[C_HIST + c];
            const int64_t per = pos == 0 ? 1 : (SEG_TILE >> c);
            s_base[pos] = lacc;
            lacc += cnt;
            iacc += (cnt + per - 1) / per;
            s_end[pos] = iacc;
        }
    }
    __syncthreads();
    const int64_t total = s_end[9];
    const int64_t off0 = offsets[0];

    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(ctrl + C_TICKET, 1u);
        __syncthreads();
        const int64_t item = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (item >= total) break;
        int pos = 0;
        while (item >= s_end[pos]) ++pos;
        const int64_t idx = item - (pos == 0 ? 0 : s_end[pos - 1]);
        const int c = pos == 0 ? SEG_CLASS_LONG : 12 - (pos - 1);
        if (c == SEG_CLASS_LONG) {
            const int64_t s = list[s_base[pos] + idx];
            const int64_t lo = offsets[s], hi = offsets[s + 1];
            Space<K> sp{keys + lo, hbuf + (lo - off0) / 2, hi - lo};
            wg_frog_sort<KT>(sk, sp, &s_bcast);
            continue;
        }
        // a batch of short segments of class c, one per aligned block of P keys
        const int P_log = c;
        const int per = SEG_TILE >> P_log;
        const int64_t first = idx * per;
        const int64_t cnt_c = ctrl[C_HIST + c];
        const int nb = (int)(cnt_c - first < per ? cnt_c - first : per);
        if ((int)threadIdx.x < nb) {
            const int64_t s = list[s_base[pos] + first + threadIdx.x];
            s_off[threadIdx.x] = offsets[s];
            s_len[threadIdx.x] = (int)(offsets[s + 1] - offsets[s]);
        }
        __syncthreads();
        using KF = typename FastKey<KT>::type;
        K r[SEG_IPT];
        bool nan_here = false;
#pragma unroll
        for (int q = 0; q < SEG_IPT; ++q) {
            const int i = (int)threadIdx.x + q * SEG_NT;
            const int b = i >> P_log, j = i & ((1 << P_log) - 1);
            const bool real = b < nb && j < s_len[b < nb ? b : 0];
            const int64_t p = real ? s_off[b] + j : s_off[0];
            r[q] = keys[p];
            nan_here |= real && is_nan_key(r[q]);
        }
        const bool any_nan = __syncthreads_or(nan_here) != 0;
        const K pad = any_nan ? KT::pad() : KF::pad();
#pragma unroll
        for (int q = 0; q < SEG_IPT; ++q) {
            const int i = (int)threadIdx.x + q * SEG_NT;
            const int b = i >> P_log, j = i & ((1 << P_log) - 1);
            const bool real = b < nb && j < s_len[b < nb ? b : 0];
            sk[lpad(i)] = real ? r[q] : pad;
        }
        sort_tile<KT>(sk, any_nan, 1 << P_log);
#pragma unroll
        for (int q = 0; q < SEG_IPT; ++q) {
            const int i = (int)threadIdx.x + q * SEG_NT;
            const int b = i >> P_log, j = i & ((1 << P_log) - 1);
            if (b < nb && j < s_len[b]) keys[s_off[b] + j] = sk[lpad(i)];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int64_t align256s(int64_t b) { return (b + 255) & ~(int64_t)255; }

SegPlan plan_seg(int64_t num_keys, int64_t nseg)
{
    SegPlan p{};
    p.num_keys = num_keys;
    p.nseg = nseg;
    p.off_h = 0;
    p.off_ctrl = align256s((num_keys / 2) * 8);
    p.off_cls = p.off_ctrl + 256;
    p.off_rank = p.off_cls + align256s(nseg * 4);
    p.off_list = p.off_rank + align256s(nseg * 4);
    p.bytes = p.off_list + align256s(nseg * 4);
    p.tile = SEG_TILE;
    return p;
}

hipError_t segsort_core_async(double *keys, const int64_t *offsets, int64_t nseg, int64_t num_keys,
                              double *hbuf, unsigned *ctrl, int *cls, int *rank, int *list,
                              const unsigned *gate, unsigned run_if, hipStream_t st)
{
    if (nseg <= 0) return hipSuccess;
    const Gate g{gate, run_if};
    const bool tr = trace_on();
    if (tr) trace_begin(TK_OTHER, st);
    launch_fill_u32(ctrl, 64, 0u, st);
    const unsigned grid = (unsigned)((nseg + 255) / 256);
    hipLaunchKernelGGL(seg_classify_kernel, dim3(grid), dim3(256), 0, st, offsets, nseg, num_keys, ctrl, cls,
                       rank, g);
    hipLaunchKernelGGL(seg_scatter_kernel, dim3(grid), dim3(256), 0, st, nseg, (const unsigned *)ctrl,
                       (const int *)cls, (const int *)rank, list, g);
    if (tr) trace_end(st);
    static int64_t groups = 0;
    if (groups <= 0) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, seg_sort_kernel<KeyF64>, SEG_NT, 0) !=
                hipSuccess || per_cu <= 0)
            per_cu = 1;
        groups = (int64_t)cus * per_cu;
    }
    if (tr) trace_begin(TK_SEGSORT, st);
    hipLaunchKernelGGL(seg_sort_kernel<KeyF64>, dim3((unsigned)groups), dim3(SEG_NT), 0, st, keys, offsets, hbuf,
                       ctrl, (const int *)list, g);
    if (tr) trace_end(st);
    return hipGetLastError();
}

hipError_t segsort_f64_async(double *keys, const int64_t *offsets, const SegPlan &p, char *ws,
                             hipStream_t st)
{
    return segsort_core_async(keys, offsets, p.nseg, p.num_keys, (double *)(ws + p.off_h),
                              (unsigned *)(ws + p.off_ctrl), (int *)(ws + p.off_cls), (int *)(ws + p.off_rank),
                              (int *)(ws + p.off_list), nullptr, 0u, st);
}

}  // namespace gs
