// Segmented sort: many independent arrays of uneven length.
//
// Every segment is sorted on its own by the same stable method as the plain
// path ("Definition of sorting": ascending, ties in input order; "Frogsort1":
// half buffer, mirrored children, merges from the inner ends outward).
// Segments are grouped by size class on the device.  Short segments (up to one
// LDS tile) are sorted by one persistent launch, several per work-group, each
// in its own aligned power-of-two block of the tile.  Every longer segment
// becomes one problem of a forest sort: its own frog tree over its own slice of
// the half buffer, with the leaves of all long segments sorted in one launch and
// the merges of all segments at the same height above the leaves done by one
// set of merge launches, every tile of every segment spread over the device.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "gs_block.h"
#include "gs_device.h"
#include "gs_internal.h"

namespace gs {

namespace {

constexpr int SEG_CLASS_LONG = 15;                  // longer than one short tile
constexpr int SEG_MAX_POS = 16;                     // work-list positions (long + short classes)

// control words at the start of the segment workspace
constexpr int C_INVALID = 0;
constexpr int C_TICKET = 1;
constexpr int C_CAND = 2;                           // some segment is an order candidate
constexpr int C_REV = 3;                            // some segment is to be reversed
constexpr int C_HIST = 16;                          // 16 class counters
constexpr int C_NLONG = 48;                         // long segments handed to the forest

// Class of a segment for short tiles of 2^logt keys: 0 for at most one key,
// c in [4, logt] for lengths in (2^(c-1), 2^c] (at least 16 keys per block),
// SEG_CLASS_LONG above one tile.
__device__ __forceinline__ int seg_class(int64_t len, int logt)
{
    if (len <= 1) return 0;
    if (len > ((int64_t)1 << logt)) return SEG_CLASS_LONG;
    int c = 4;
    while (((int64_t)1 << c) < len) ++c;
    return c;
}

// A segment's order code, held in its rank word until the classification
// overwrites it (ranks are never negative): sort it, nothing to do, reverse
// it, or still to be decided from the order bits in its class word.
constexpr int SEG_SORT = 0;
constexpr int SEG_DONE = kSegDone;
constexpr int SEG_REVERSE = -2;
constexpr int SEG_CANDIDATE = -3;
constexpr int64_t SEG_RANGE = 16384;                // keys per work-group of the range passes
constexpr int64_t SEG_WAVE_CHECK = 8192;            // pairs of a segment its wave checks itself

__host__ __device__ inline int64_t seg_ranges(int64_t num_keys) { return (num_keys + SEG_RANGE - 1) / SEG_RANGE; }

// Work-list order: the long class first, then the short classes from the
// largest blocks down.
__device__ __forceinline__ int class_at(int pos, int logt) { return pos == 0 ? SEG_CLASS_LONG : logt - (pos - 1); }
__device__ __forceinline__ int num_pos(int logt) { return logt - 2; }

}  // namespace

// ---------------------------------------------------------------------------
// 0. per segment: already in order, or reversed ("Octosort", "Squidsort")
// ---------------------------------------------------------------------------
// The whole-array order check of the plain path, applied to every segment:
// a segment whose neighbour pairs are all in order needs nothing, one whose
// pairs all strictly decrease (or, these being keys without values, do not
// increase and tie only bit-identical keys) is sorted by one reversal.
// Nothing moves in these passes (the offsets are validated only by the
// classification; a segment with bad offsets reads nothing).
//
// 0a. One wave per segment reads its first SEG_WAVE_CHECK pairs in order,
// 512 at a time, and stops as soon as the pairs seen rule out both orders
// (for unsorted data, after the first 512).  A segment still possibly in
// order past those pairs becomes a candidate: its order bits so far are in
// cls[s], the range pass completes them, and cand[r] marks every range r of
// SEG_RANGE keys that holds some of its remaining pairs (ctrl[C_CAND]: some
// segment is a candidate).
template <class KT>
__global__ __launch_bounds__(256) void seg_order_sample_kernel(const typename KT::T *keys, const int64_t *offsets,
                                                               int64_t nseg, int64_t num_keys, int *cls,
                                                               int *rank, unsigned *ctrl, unsigned char *cand,
                                                               Gate gate)
{
    if (gate.closed()) return;
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * 4;
    for (int64_t s = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); s < nseg; s += waves) {
        const int64_t lo = offsets[s], hi = offsets[s + 1];
        if (lo < 0 || hi < lo || hi > num_keys) {
            if (lane == 0) rank[s] = SEG_SORT;
            continue;
        }
        const int64_t pairs = hi - lo - 1;
        const int64_t lim = pairs < SEG_WAVE_CHECK ? pairs : SEG_WAVE_CHECK;
        unsigned all = 15u;
        for (int64_t base = 0; base < lim; base += 512) {
            unsigned bits = 15u;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int64_t j = base + r * 64 + lane;
                if (j < lim) bits &= order_bits<KT>(keys[lo + j], keys[lo + j + 1]);
            }
            // and of the four order bits over the wave
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (__ballot(((bits >> b) & 1u) == 0u) != 0ull) all &= ~(1u << b);
            if (!order_decisive<KT>(all, true)) break;
        }
        int code;
        if (pairs > lim && order_decisive<KT>(all, true)) {
            code = SEG_CANDIDATE;
            const int64_t r0 = (lo + lim) / SEG_RANGE, r1 = (hi - 2) / SEG_RANGE;   // ranges of pairs [lo+lim, hi-1)
            for (int64_t r = r0 + lane; r <= r1; r += 64) cand[r] = 1;
            if (lane == 0) atomicOr(ctrl + C_CAND, 1u);
        } else {
            code = (all & 1u) ? SEG_DONE : ((all & 2u) || ((all & 4u) && (all & 8u))) ? SEG_REVERSE : SEG_SORT;
        }
        if (lane == 0) {
            rank[s] = code;
            cls[s] = (int)all;
        }
    }
}

// First segment that ends past key r0 (offsets non-decreasing; with bad
// offsets any segment index comes back, and the keys read stay inside the
// segment's own checked bounds).
__device__ __forceinline__ int64_t seg_first_after(const int64_t *offsets, int64_t nseg, int64_t r0)
{
    int64_t a = 0, b = nseg;                        // first s with offsets[s + 1] > r0
    while (a < b) {
        const int64_t m = (a + b) >> 1;
        if (offsets[m + 1] > r0) b = m;
        else a = m + 1;
    }
    return a;
}

// Last of the empty segments at offset o that start with segment s (the
// loop then continues after it); never moves backwards, whatever the offsets.
__device__ __forceinline__ int64_t seg_skip_empty(const int64_t *offsets, int64_t nseg, int64_t s, int64_t o)
{
    const int64_t next = seg_first_after(offsets, nseg, o);   // first segment ending past o
    return next - 1 > s ? next - 1 : s;
}

// 0b. One work-group per SEG_RANGE keys of the array: the pairs of every
// candidate segment past the ones its wave checked that start in the range
// are checked and their order bits and-ed into cls[s], so a long segment is
// read by many work-groups at once.  A range that holds no such pairs
// (cand[range] clear) has nothing to do.
template <class KT>
__global__ __launch_bounds__(256) void seg_order_range_kernel(const typename KT::T *keys, const int64_t *offsets,
                                                              int64_t nseg, int64_t num_keys, int *cls,
                                                              const int *rank, const unsigned *ctrl,
                                                              const unsigned char *cand, int64_t range0, Gate gate)
{
    __shared__ unsigned s_bits;
    const int64_t range = range0 + blockIdx.x;
    if (gate.closed() || !ctrl[C_CAND] || !cand[range]) return;
    const int64_t r0 = range * SEG_RANGE;
    const int64_t r1 = r0 + SEG_RANGE < num_keys ? r0 + SEG_RANGE : num_keys;
    for (int64_t s = seg_first_after(offsets, nseg, r0); s < nseg; ++s) {
        const int64_t lo = offsets[s], hi = offsets[s + 1];
        if (lo >= r1) break;
        if (hi == lo) {                              // past a run of empty segments at once
            s = seg_skip_empty(offsets, nseg, s, lo);
            continue;
        }
        if (rank[s] != SEG_CANDIDATE || lo < 0 || hi < lo || hi > num_keys) continue;
        const int64_t pairs = hi - lo - 1;
        const int64_t from = lo + (pairs < SEG_WAVE_CHECK ? pairs : SEG_WAVE_CHECK);   // past the wave's pairs
        const int64_t a = from > r0 ? from : r0;
        const int64_t b = hi - 1 < r1 ? hi - 1 : r1;  // pairs (i, i+1) with i in [a, b)
        if (a >= b) continue;
        if (threadIdx.x == 0) s_bits = 15u;
        __syncthreads();
        unsigned bits = 15u;
        for (int64_t i0 = a + threadIdx.x; i0 < b; i0 += 4 * 256) {   // four pairs in flight per thread
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + r * 256;
                if (i < b) bits &= order_bits<KT>(keys[i], keys[i + 1]);
            }
        }
        atomicAnd(&s_bits, bits);
        __syncthreads();
        if (threadIdx.x == 0 && s_bits != 15u) atomicAnd((unsigned *)cls + s, s_bits);
        __syncthreads();                            // s_bits read before the next segment resets it
    }
}

// ---------------------------------------------------------------------------
// 1. validate the offsets and count segments per class
// ---------------------------------------------------------------------------
// With the order codes (order_codes != 0), a candidate's code is decided from
// its order bits, and a segment already in order or to be reversed takes
// class 0 (no sorting work) and keeps its code (ctrl[C_REV] says some segment
// is reversed, revmap[r] that range r holds pairs of one to swap; order codes
// come with a revmap).  A segment's rank is its place among its class: counted per
// work-group in LDS, then one device atomic per class and work-group.
__global__ __launch_bounds__(256) void seg_classify_kernel(const int64_t *offsets, int64_t nseg,
                                                           int64_t num_keys, int logt, unsigned *ctrl,
                                                           int *cls, int *rank, int order_codes,
                                                           unsigned char *revmap, Gate gate)
{
    __shared__ unsigned s_cnt[SEG_MAX_POS], s_base[SEG_MAX_POS];
    if (gate.closed()) return;
    if (threadIdx.x < SEG_MAX_POS) s_cnt[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int c = -1;                                     // class of a segment that needs sorting
    unsigned local = 0u;
    if (s < nseg) {
        const int64_t lo = offsets[s], hi = offsets[s + 1];
        if (lo < 0 || hi < lo || hi > num_keys) {
            atomicOr(ctrl + C_INVALID, 1u);
            cls[s] = 0;
        } else {
            int code = SEG_SORT;
            if (order_codes) {
                code = rank[s];
                if (code == SEG_CANDIDATE) {
                    const unsigned b = (unsigned)cls[s];
                    code = (b & 1u) ? SEG_DONE : ((b & 2u) || ((b & 4u) && (b & 8u))) ? SEG_REVERSE : SEG_SORT;
                    rank[s] = code;
                }
                if (code == SEG_REVERSE && hi - lo > 1) {
                    // the ranges that hold the lower half [lo, mid), whose pairs the reversal swaps
                    atomicOr(ctrl + C_REV, 1u);
                    const int64_t mid = lo + (hi - lo) / 2;
                    for (int64_t r = lo / SEG_RANGE; r <= (mid - 1) / SEG_RANGE; ++r) revmap[r] = 1;
                }
            }
            if (code != SEG_SORT) {
                cls[s] = 0;
            } else {
                c = seg_class(hi - lo, logt);
                cls[s] = c;
                local = atomicAdd(&s_cnt[c], 1u);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < SEG_MAX_POS && s_cnt[threadIdx.x])
        s_base[threadIdx.x] = atomicAdd(ctrl + C_HIST + threadIdx.x, s_cnt[threadIdx.x]);
    __syncthreads();
    if (c >= 0) rank[s] = (int)(s_base[c] + local);
}

// Reverses, in place, every segment whose code says so, once every segment's
// offsets passed the classification.  One work-group per SEG_RANGE keys
// swaps the pairs (i, lo + hi - 1 - i) whose lower index i lies in its range.
// Nothing to do in a range without such pairs (revmap[range] clear).
template <class K>
__global__ __launch_bounds__(256) void seg_reverse_kernel(K *keys, const int64_t *offsets, int64_t nseg,
                                                          int64_t num_keys, const unsigned *ctrl, const int *cls,
                                                          const int *rank, const unsigned char *revmap,
                                                          int64_t range0, Gate gate)
{
    const int64_t range = range0 + blockIdx.x;
    if (gate.closed() || ctrl[C_INVALID] || !ctrl[C_REV] || !revmap[range]) return;
    const int64_t r0 = range * SEG_RANGE;
    const int64_t r1 = r0 + SEG_RANGE < num_keys ? r0 + SEG_RANGE : num_keys;
    for (int64_t s = seg_first_after(offsets, nseg, r0); s < nseg; ++s) {
        const int64_t lo = offsets[s], hi = offsets[s + 1];
        if (lo >= r1) break;
        if (hi == lo) {                              // past a run of empty segments at once
            s = seg_skip_empty(offsets, nseg, s, lo);
            continue;
        }
        if (cls[s] != 0 || rank[s] != SEG_REVERSE) continue;
        const int64_t mid = lo + (hi - lo) / 2;     // lower halves: [lo, mid)
        const int64_t a = lo > r0 ? lo : r0;
        const int64_t b = mid < r1 ? mid : r1;
        for (int64_t i0 = a + threadIdx.x; i0 < b; i0 += 4 * 256) {   // four swaps in flight per thread
            K x[4], y[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + r * 256;
                if (i < b) {
                    x[r] = keys[i];
                    y[r] = keys[lo + hi - 1 - i];
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + r * 256;
                if (i < b) {
                    keys[i] = y[r];
                    keys[lo + hi - 1 - i] = x[r];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// 2. place segment ids into one list ordered by class
// ---------------------------------------------------------------------------
// First list position of class c (classes in work-list order).
__device__ __forceinline__ int64_t class_base(const unsigned *ctrl, int c, int logt)
{
    int64_t acc = 0;
    for (int pos = 0; pos < num_pos(logt); ++pos) {
        const int cc = class_at(pos, logt);
        if (cc == c) return acc;
        acc += ctrl[C_HIST + cc];
    }
    return acc;
}

__global__ __launch_bounds__(256) void seg_scatter_kernel(int64_t nseg, int logt, const unsigned *ctrl,
                                                          const int *cls, const int *rank, int *list, Gate gate)
{
    if (gate.closed()) return;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nseg || ctrl[C_INVALID]) return;
    const int c = cls[s];
    if (c == 0) return;
    list[class_base(ctrl, c, logt) + rank[s]] = (int)s;
}

// ---------------------------------------------------------------------------
// 3. the persistent sorter of the short classes
// ---------------------------------------------------------------------------

// Long segments (class SEG_CLASS_LONG, first in the work list) as forest
// problems: the segment's keys and its slice of the half buffer, which starts
// at floor((offset - offsets[0]) / 2) (slices of consecutive segments never
// overlap since floor(a/2) + floor(b/2) <= floor((a+b)/2)).
__global__ __launch_bounds__(256) void seg_probs_kernel(const int64_t *offsets, unsigned *ctrl, const int *list,
                                                        Prob *probs, int64_t max_probs, int64_t leaf, Gate gate)
{
    if (gate.closed()) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool invalid = ctrl[C_INVALID] != 0;
    const int64_t L = ctrl[C_HIST + SEG_CLASS_LONG];
    const bool fits = L <= max_probs;
    if (i == 0) ctrl[C_NLONG] = (invalid || !fits) ? 0u : (unsigned)L;
    if (invalid || !fits || i >= L) return;
    const int64_t s = list[i];
    const int64_t lo = offsets[s], hi = offsets[s + 1];
    Prob P;
    P.doff = lo;
    P.hoff = (lo - offsets[0]) / 2;
    P.n = hi - lo;
    P.depth = frog_depth(P.n, leaf);
    P.pad = 0;
    probs[i] = P;
}

// Work items: batches of segments of one short class c, TILE >> c of them
// (one per aligned block of 2^c keys of the LDS tile), sorted together.
template <class KT, int NT, int IPT>
__global__ __launch_bounds__(NT) void seg_sort_kernel(typename KT::T *keys, const int64_t *offsets,
                                                      unsigned *ctrl, const int *list, Gate gate)
{
    using K = typename KT::T;
    using KF = typename FastKey<KT>::type;
    constexpr int TILE = NT * IPT;
    constexpr int LOGT = TILE == 2048 ? 11 : (TILE == 4096 ? 12 : (TILE == 8192 ? 13 : -1));
    static_assert(LOGT > 0, "short tiles of 2048, 4096 or 8192 keys");
    static_assert(TILE / 16 <= NT, "one thread per segment of the smallest class");
    __shared__ K sk[lds_slots<TILE>()];
    __shared__ int s_item;
    __shared__ int64_t s_off[NT];
    __shared__ int s_len[NT];
    __shared__ int64_t s_base[SEG_MAX_POS], s_end[SEG_MAX_POS];   // per work-list position
    if (gate.closed() || ctrl[C_INVALID]) return;
    const int npos = num_pos(LOGT);

    // list start and cumulative work items of every class (work-list order)
    if (threadIdx.x == 0) {
        int64_t lacc = 0, iacc = 0;
        for (int pos = 0; pos < npos; ++pos) {
            const int c = class_at(pos, LOGT);
            const int64_t cnt = ctrl[C_HIST + c];
            const int64_t per = pos == 0 ? 1 : (TILE >> c);
            s_base[pos] = lacc;
            lacc += cnt;
            if (pos > 0) iacc += (cnt + per - 1) / per;     // long segments: forest
            s_end[pos] = iacc;
        }
    }
    __syncthreads();
    const int64_t total = s_end[npos - 1];

    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(ctrl + C_TICKET, 1u);
        __syncthreads();
        const int64_t item = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (item >= total) break;
        int pos = 1;
        while (item >= s_end[pos]) ++pos;
        const int64_t idx = item - s_end[pos - 1];
        const int c = class_at(pos, LOGT);
        // a batch of short segments of class c, one per aligned block of P keys
        const int P_log = c;
        const int per = TILE >> P_log;
        const int64_t first = idx * per;
        const int64_t cnt_c = ctrl[C_HIST + c];
        const int nb = (int)(cnt_c - first < per ? cnt_c - first : per);
        if ((int)threadIdx.x < nb) {
            const int64_t s = list[s_base[pos] + first + threadIdx.x];
            s_off[threadIdx.x] = offsets[s];
            s_len[threadIdx.x] = (int)(offsets[s + 1] - offsets[s]);
        }
        __syncthreads();
        K r[IPT];
        bool nan_here = false, differ = false;
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            const int i = (int)threadIdx.x + q * NT;
            const int b = i >> P_log, j = i & ((1 << P_log) - 1);
            const bool real = b < nb && j < s_len[b < nb ? b : 0];
            const int64_t p = real ? s_off[b] + j : s_off[0];
            r[q] = keys[p];
            nan_here |= real && is_nan_key(r[q]);
            differ |= real && tie_bits_may_differ(r[q]);
        }
        const bool any_nan = __syncthreads_or(nan_here) != 0;
        // equal keys bit for bit equal: the order among them cannot be seen
        const bool ties_identical = __syncthreads_or(differ) == 0;
        const K pad = any_nan ? KT::pad() : KF::pad();
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            const int i = (int)threadIdx.x + q * NT;
            const int b = i >> P_log, j = i & ((1 << P_log) - 1);
            const bool real = b < nb && j < s_len[b < nb ? b : 0];
            sk[lpad(i)] = real ? r[q] : pad;
        }
        // only the blocks that hold segments are sorted
        const int active = nb << P_log;
        char dummy[1];
        __syncthreads();
        if (any_nan) block_sort_lds<KT, char, false, NT, IPT, true>(sk, dummy, 1 << P_log, active);
        else block_sort_lds<KF, char, false, NT, IPT, true>(sk, dummy, 1 << P_log, active, ties_identical);
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            const int i = (int)threadIdx.x + q * NT;
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

static int log2_exact(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

// The configurations the tuner tries: short-tile shape and forest merge tile.
static const SegConfig kSegConfigs[] = {
    {256, 16, 16}, {256, 8, 16}, {512, 8, 16}, {512, 16, 16}, {1024, 8, 16},
    {256, 16, 8}, {256, 8, 8}, {512, 8, 8}, {512, 16, 8}, {1024, 8, 8},
};

int seg_config_count() { return (int)(sizeof kSegConfigs / sizeof kSegConfigs[0]); }
SegConfig seg_config_at(int i) { return kSegConfigs[i]; }
SegConfig seg_default_config() { return kSegConfigs[0]; }

bool seg_config_valid(const SegConfig &c)
{
    for (int i = 0; i < seg_config_count(); ++i)
        if (kSegConfigs[i].short_threads == c.short_threads && kSegConfigs[i].short_ipt == c.short_ipt &&
            kSegConfigs[i].merge_ipt == c.merge_ipt)
            return true;
    return false;
}

// Most long segments a call can have: every one holds more than a short tile.
static int64_t max_long(int64_t num_keys, int64_t nseg, int64_t tile)
{
    const int64_t m = num_keys / (tile + 1);
    return m < nseg ? m : nseg;
}

SegPlan plan_seg(int64_t num_keys, int64_t nseg, const SegConfig &cfg, int64_t q, int algo, int64_t q2)
{
    SegPlan p{};
    p.num_keys = num_keys;
    p.nseg = nseg;
    p.cfg = cfg;
    p.tile = (int64_t)cfg.short_threads * cfg.short_ipt;
    p.q = q > 0 && q < 32768 ? q : 0;
    p.algo = algo;
    p.q2 = q2;
    p.hlen = p.q ? (int64_t)(((__int128)p.q * num_keys) >> 16) : num_keys / 2;
    // The long segments of one pass have disjoint half buffers inside the
    // buffer, so they hold at most 2 hlen keys plus one per segment, and each
    // holds more than a tile: at most 2 hlen + 2 hlen / tile + 1 keys.
    p.pass_keys = p.q ? 2 * p.hlen + 2 * p.hlen / p.tile + 1 : num_keys;
    if (p.pass_keys > num_keys) p.pass_keys = num_keys;
    p.off_h = 0;
    p.off_ctrl = align256s(p.hlen * 8);
    p.off_cls = p.off_ctrl + 256;
    p.off_rank = p.off_cls + align256s(nseg * 4);
    p.off_list = p.off_rank + align256s(nseg * 4);
    p.off_maps = p.off_list + align256s(nseg * 4);
    p.off_forest = p.off_maps + align256s(2 * seg_ranges(num_keys));
    p.forest = plan_forest_f64(p.pass_keys, p.pass_keys, max_long(p.pass_keys, nseg, p.tile), cfg.merge_ipt);
    p.bytes = p.off_forest + p.forest.bytes;
    // a segment sorted alone is longer than a tile and than 2 hlen + 1 keys.
    // The plain sort's workspace at the call's fraction grows with the keys,
    // but not strictly: its control area for a length just below a power of
    // two can exceed that of the power by a few KiB.  The whole array's, with
    // its control area grown by 1/8 + 8 KiB, bounds every segment's (and the
    // call checks each segment's own before anything runs).
    p.alone_bytes = 0;
    if (p.q && num_keys > p.tile && num_keys > 2 * p.hlen + 1) {
        const SortPlan a = plan_f64(num_keys, p.q, algo, q2);
        const int64_t ctrl = a.bytes - align256s(a.hlen * 8);
        p.alone_bytes = align256s(a.bytes + ctrl / 8 + 8192);
    }
    if (p.alone_bytes > p.bytes) p.bytes = p.alone_bytes;
    return p;
}

std::vector<SegStep> seg_schedule(const int64_t *off, int64_t nseg, int64_t tile, int64_t hlen)
{
    std::vector<SegStep> steps;
    int64_t s0 = 0;
    while (s0 < nseg) {
        int64_t s = s0;
        const int64_t base = off[s0];
        for (; s < nseg; ++s) {
            const int64_t len = off[s + 1] - off[s];
            if (len <= tile) continue;                       // sorted in LDS: no buffer
            if ((off[s] - base) / 2 + len / 2 <= hlen) continue;
            break;
        }
        if (s > s0) {
            steps.push_back(SegStep{s0, s, false});
            s0 = s;
        } else {
            // the first segment alone overflows the buffer
            steps.push_back(SegStep{s0, s0 + 1, true});
            s0 = s0 + 1;
        }
    }
    return steps;
}


// The forest of segsort_core_async, which runs the default shape.
ForestPlan plan_forest_seg(int64_t num_keys, int64_t max_len, int64_t nseg)
{
    const SegConfig c = seg_default_config();
    return plan_forest_f64(num_keys, max_len, max_long(num_keys, nseg, (int64_t)c.short_threads * c.short_ipt),
                           c.merge_ipt);
}

template <int NT, int IPT>
static void launch_short(double *keys, const int64_t *offsets, unsigned *ctrl, const int *list, Gate g,
                         hipStream_t st)
{
    static int64_t groups = 0;
    if (groups <= 0) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, seg_sort_kernel<KeyF64, NT, IPT>, NT, 0) !=
                hipSuccess || per_cu <= 0)
            per_cu = 1;
        groups = (int64_t)cus * per_cu;
    }
    hipLaunchKernelGGL((seg_sort_kernel<KeyF64, NT, IPT>), dim3((unsigned)groups), dim3(NT), 0, st, keys, offsets,
                       ctrl, list, g);
}

// work-groups for a one-segment-per-group pass (each walks segments with a
// stride of the grid)
static unsigned seg_groups(int64_t nseg)
{
    return (unsigned)(nseg < 65536 ? nseg : 65536);
}

// maps: 2 x seg_ranges(num_keys) bytes (candidate and reversal range maps),
// needed with order_check only.
static hipError_t segsort_run(double *keys, const int64_t *offsets, int64_t nseg, int64_t num_keys, double *hbuf,
                              unsigned *ctrl, int *cls, int *rank, int *list, unsigned char *maps, char *forest,
                              const ForestPlan &fp, const SegConfig &cfg, bool order_check, const unsigned *gate,
                              unsigned run_if, hipStream_t st, bool preset_codes = false, int64_t key_lo = 0,
                              int64_t key_hi = -1)
{
    if (nseg <= 0) return hipSuccess;
    const Gate g{gate, run_if};
    const int logt = log2_exact(cfg.short_threads * cfg.short_ipt);
    const bool tr = trace_on();
    if (tr) trace_begin(TK_OTHER, st);
    launch_fill_u32(ctrl, 64, 0u, st);
    const unsigned grid = (unsigned)((nseg + 255) / 256);
    const unsigned ranges = (unsigned)((num_keys + SEG_RANGE - 1) / SEG_RANGE);
    unsigned char *cand = maps, *revmap = maps ? maps + ranges : nullptr;
    // the range passes cover the ranges of keys [key_lo, key_hi) the
    // segments hold (all of them by default)
    if (key_hi < 0) key_hi = num_keys;
    const int64_t range0 = key_lo / SEG_RANGE;
    const int64_t range1 = (key_hi + SEG_RANGE - 1) / SEG_RANGE;
    const unsigned span = (unsigned)(range1 > range0 ? range1 - range0 : 0);
    if (order_check) {
        if (ranges > 0) launch_fill_u32((unsigned *)maps, (2 * (int64_t)ranges + 3) / 4, 0u, st);
        hipLaunchKernelGGL((seg_order_sample_kernel<KeyF64>), dim3(seg_groups((nseg + 3) / 4)), dim3(256), 0, st,
                           (const double *)keys, offsets, nseg, num_keys, cls, rank, ctrl, cand, g);
        if (span > 0)
            hipLaunchKernelGGL((seg_order_range_kernel<KeyF64>), dim3(span), dim3(256), 0, st,
                               (const double *)keys, offsets, nseg, num_keys, cls, (const int *)rank,
                               (const unsigned *)ctrl, (const unsigned char *)cand, range0, g);
    }
    hipLaunchKernelGGL(seg_classify_kernel, dim3(grid), dim3(256), 0, st, offsets, nseg, num_keys, logt, ctrl, cls,
                       rank, order_check || preset_codes ? 1 : 0, revmap, g);
    if (order_check && span > 0)
        hipLaunchKernelGGL((seg_reverse_kernel<double>), dim3(span), dim3(256), 0, st, keys, offsets, nseg,
                           num_keys, (const unsigned *)ctrl, (const int *)cls, (const int *)rank,
                           (const unsigned char *)revmap, range0, g);
    hipLaunchKernelGGL(seg_scatter_kernel, dim3(grid), dim3(256), 0, st, nseg, logt, (const unsigned *)ctrl,
                       (const int *)cls, (const int *)rank, list, g);
    Prob *probs = (Prob *)(forest + fp.off_probs);
    const int64_t maxp = fp.max_probs;
    hipLaunchKernelGGL(seg_probs_kernel, dim3((unsigned)((maxp + 255) / 256 > 0 ? (maxp + 255) / 256 : 1)),
                       dim3(256), 0, st, offsets, ctrl, (const int *)list, probs, maxp, fp.leaf, g);
    if (tr) trace_end(st);
    if (tr) trace_begin(TK_SEGSORT, st);
    const int key = cfg.short_threads * 100 + cfg.short_ipt;
    switch (key) {
    case 25608: launch_short<256, 8>(keys, offsets, ctrl, list, g, st); break;
    case 25616: launch_short<256, 16>(keys, offsets, ctrl, list, g, st); break;
    case 51208: launch_short<512, 8>(keys, offsets, ctrl, list, g, st); break;
    case 51216: launch_short<512, 16>(keys, offsets, ctrl, list, g, st); break;
    case 102408: launch_short<1024, 8>(keys, offsets, ctrl, list, g, st); break;
    default: return hipErrorInvalidValue;
    }
    if (tr) trace_end(st);
    if (maxp <= 0) return hipGetLastError();
    return forest_f64_async(keys, hbuf, probs, ctrl + C_NLONG, fp, forest, st, gate, run_if, cfg.merge_ipt);
}

hipError_t segsort_core_async(double *keys, const int64_t *offsets, int64_t nseg, int64_t num_keys,
                              double *hbuf, unsigned *ctrl, int *cls, int *rank, int *list, char *forest,
                              const ForestPlan &fp, const unsigned *gate, unsigned run_if, hipStream_t st,
                              bool preset_codes)
{
    return segsort_run(keys, offsets, nseg, num_keys, hbuf, ctrl, cls, rank, list, nullptr, forest, fp,
                       seg_default_config(), false, gate, run_if, st, preset_codes);
}

hipError_t segsort_f64_async(double *keys, const int64_t *offsets, const SegPlan &p, char *ws,
                             hipStream_t st)
{
    // the forest's error word; the offsets flag (control word 0) is set by
    // the run itself before anything else reads it
    ErrWords ew{};
    ew.add((unsigned *)(ws + p.off_forest + p.forest.off_ctrl) + kErrWord, DEVERR_WAIT);
    hipError_t e = err_words_begin(ew, st);
    if (e != hipSuccess) return e;
    e = segsort_run(keys, offsets, p.nseg, p.num_keys, (double *)(ws + p.off_h), (unsigned *)(ws + p.off_ctrl),
                    (int *)(ws + p.off_cls), (int *)(ws + p.off_rank), (int *)(ws + p.off_list),
                    (unsigned char *)(ws + p.off_maps), ws + p.off_forest, p.forest, p.cfg, true, nullptr, 0u, st);
    if (e != hipSuccess) return e;
    ew.add((unsigned *)(ws + p.off_ctrl), DEVERR_OFFSETS);
    return err_words_end(ew, st);
}

hipError_t segsort_passes_async(double *keys, const int64_t *offsets, const int64_t *h_off, const SegPlan &p,
                                const std::vector<SegStep> &steps, char *ws, hipStream_t st)
{
    // every pass's forest shares one control block, so its error word
    ErrWords ew{};
    ew.add((unsigned *)(ws + p.off_forest + p.forest.off_ctrl) + kErrWord, DEVERR_WAIT);
    hipError_t e = err_words_begin(ew, st);
    if (e != hipSuccess) return e;
    for (const SegStep &t : steps) {
        if (t.alone) continue;
        // the forest sized to this pass's long segments (fewer rounds and
        // smaller launches than the capacity of any pass); its areas lie
        // inside the reserved one, whose control block comes first
        int64_t keys_long = 0, max_len = 0, nlong = 0;
        for (int64_t s = t.s0; s < t.s1; ++s) {
            const int64_t len = h_off[s + 1] - h_off[s];
            if (len <= p.tile) continue;
            keys_long += len;
            nlong += 1;
            if (len > max_len) max_len = len;
        }
        ForestPlan fp = plan_forest_f64(keys_long, max_len, nlong, p.cfg.merge_ipt);
        if (fp.bytes > p.forest.bytes || fp.off_ctrl != p.forest.off_ctrl) fp = p.forest;
        e = segsort_run(keys, offsets + t.s0, t.s1 - t.s0, p.num_keys, (double *)(ws + p.off_h),
                        (unsigned *)(ws + p.off_ctrl), (int *)(ws + p.off_cls), (int *)(ws + p.off_rank),
                        (int *)(ws + p.off_list), (unsigned char *)(ws + p.off_maps), ws + p.off_forest, fp,
                        p.cfg, true, nullptr, 0u, st, false, h_off[t.s0], h_off[t.s1]);
        if (e != hipSuccess) return e;
    }
    return err_words_end(ew, st);
}

}  // namespace gs
