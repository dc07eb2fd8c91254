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

// Descending orders of the same keys (the DescLeft target: the greater key
// first, ties still in input order): less is the ascending less with its
// arguments swapped; padding sorts after every key in this order.
struct KeyF64Desc {
    using T = double;
    static __device__ __forceinline__ bool less(double a, double b) { return KeyF64::less(b, a); }
    static __device__ __forceinline__ double pad() { return -__builtin_inf(); }
};
struct KeyF64DescNoNaN {
    using T = double;
    static __device__ __forceinline__ bool less(double a, double b) { return b < a; }
    static __device__ __forceinline__ double pad() { return -__builtin_inf(); }
};
struct KeyU64Desc {
    using T = uint64_t;
    static __device__ __forceinline__ bool less(uint64_t a, uint64_t b) { return b < a; }
    static __device__ __forceinline__ uint64_t pad() { return 0; }
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
// a forest of independent frog sorts processed level-synchronously
// ---------------------------------------------------------------------------
// Every problem (one array, one segment, one bucket) is a frog tree of its own
// over its own logical space: slots [0, n) at D + doff, slots [n, n + n/2) at
// H + hoff.  Round 0 sorts every leaf of every problem; round r >= 1 performs
// the merges at depth (depth - r) of every problem that deep, so all problems
// reach their roots together.  Work items (tickets) of a round are numbered
// problem after problem; per problem, leaves in descending index order and
// merge tiles node after node, each node's tiles in its write order.
struct Prob {
    int64_t doff;     // first key in the caller's array
    int64_t hoff;     // first slot in the half buffer
    int64_t n;        // keys
    int32_t depth;    // depth of the leaf level
    int32_t pad;
};

// ---------------------------------------------------------------------------
// Frogsort2: one irregular tree from host-built tables (geometry in
// frog_geometry.h)
// ---------------------------------------------------------------------------
struct F2View {
    const int64_t *leaf_c;     // input offset of every leaf, in input order (+ a final n)
    const int64_t *leaf_d;     // data start of every leaf
    const int64_t *node_s;     // region start of every merge node (grouped by round)
    const int64_t *node_n;     // its elements, | kF2LeftBit for a left node
    const unsigned *node_tb;   // its first ticket within its round
    const unsigned *node_sb;   // its first split within its round
    const unsigned *rb;        // first node of every round (rounds + 2 entries)
    const unsigned *rt, *rs;   // tickets and splits of every round
    int64_t nleaves;
    int64_t q;
};

// Last index i in [0, L) with c[i] <= x (c ascending, c[0] <= x).
__device__ __forceinline__ int64_t locate_i64(const int64_t *c, int64_t L, int64_t x)
{
    int64_t lo = 0, hi = L;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (c[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

struct Forest {
    const Prob *probs;        // problem table, or nullptr: the single problem p0
    const unsigned *nprob;    // number of problems in the table (device word)
    const unsigned *tbase;    // per round, prefix sums of tickets over problems
    const unsigned *sbase;    // per round, prefix sums of merge-path splits
    int64_t stride;           // row length of tbase / sbase (>= problems + 1)
    Prob p0;
    FrogMerge m1;             // with use_m1: round 1 of p0 is this one merge
    int use_m1;
    int use_f2;               // with use_f2: p0 is sorted by the Frogsort2 tree in f2
    F2View f2;
    // Squidsort (the single Frogsort1 tree only, else null): the direction
    // (DIR_*) of every node's run, heap order (depth d, node i at
    // 2^d - 1 + i), and the packed mode of every node of the current round
    uint8_t *dirs;
    uint8_t *modes;
    // Run samples (the single Frogsort1 tree only, else null): for every run
    // a round produces, one key per stretch of samp_tile ranks (kSampPerTile
    // stretches per merge tile) at slot (node * stretches per node +
    // stretch): the stretch's first key for a left child (the run its
    // parent's merge takes first), its last key for a right child.  The next
    // round's partition reads them before its merge overwrites them with its
    // own.  The leaves have samp_leaf_tiles stretches each.
    void *samp;
    int samp_tile, samp_leaf_tiles;
};

// Run-sample stretches per merge tile (a power of two).
#ifndef GS_SAMP_PER_TILE
#define GS_SAMP_PER_TILE 8
#endif
constexpr int kSampPerTile = GS_SAMP_PER_TILE;

GS_HD int64_t forest_nodes(const Forest &F, const Prob &P, int round)
{
    if (F.use_m1) return 1;
    return round <= P.depth ? ((int64_t)1 << (P.depth - round)) : 0;
}

template <int TILE>
GS_HD int64_t forest_tpn(const Forest &F, const Prob &P, int round)
{
    if (F.use_m1) return (F.m1.nl + F.m1.nr + TILE - 1) / TILE;
    return (frog_max_node(P.n, P.depth - round) + TILE - 1) / TILE;
}

// tickets of one problem in a round (round 0: its leaves)
template <int TILE>
GS_HD int64_t forest_tickets(const Forest &F, const Prob &P, int round)
{
    if (round == 0) return (int64_t)1 << P.depth;
    return forest_nodes(F, P, round) * forest_tpn<TILE>(F, P, round);
}

template <int TILE>
GS_HD int64_t forest_splits(const Forest &F, const Prob &P, int round)
{
    if (round == 0) return 0;
    return forest_nodes(F, P, round) * (forest_tpn<TILE>(F, P, round) + 1);
}

GS_HD FrogMerge forest_merge(const Forest &F, const Prob &P, int round, int64_t node)
{
    return F.use_m1 ? F.m1 : frog_merge_of(frog_node(P.n, P.depth - round, node));
}

// Problem whose range of a prefix row holds x: the last s in [0, L) with
// row[s] <= x (then row[s+1] > x, so the problem is not empty).
__device__ __forceinline__ Prob forest_prob(const Forest &F, int64_t s) { return F.probs ? F.probs[s] : F.p0; }

__device__ __forceinline__ int64_t forest_locate(const unsigned *row, int64_t L, int64_t x)
{
    int64_t lo = 0, hi = L;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)row[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// The same search done by every lane of a wave together, x uniform: each
// round probes 63 evenly spaced rows at once and keeps the interval between
// the last probe <= x and the next, so about log64(L) rounds of loads.
__device__ __forceinline__ int64_t forest_locate_wave(const unsigned *row, int64_t L, int64_t x)
{
    const int lane = threadIdx.x & 63;
    int64_t lo = 0, hi = L;
    while (hi - lo > 1) {
        const int64_t step = (hi - lo + 63) / 64;
        const int64_t idx = lo + (int64_t)(lane + 1) * step;
        const bool le = idx < hi && (int64_t)row[idx] <= x;
        const int k = __popcll(__ballot(le));           // probes <= x form a prefix of the lanes
        const int64_t nlo = lo + (int64_t)k * step;
        const int64_t nhi = lo + (int64_t)(k + 1) * step;
        lo = nlo;
        hi = nhi < hi ? nhi : hi;
    }
    return lo;
}

// One merge output tile, resolved before the merge launch: the runs it reads,
// where it writes, and the tickets it must wait for before storing.  Its
// inputs are la elements of view a, stored at slots [pa, pa + la), then
// cnt - la elements of view b at [pb, pb + cnt - la); a view read from its
// end (TF_AREV / TF_BREV) has its slots loaded upwards all the same and
// staged in reverse; its outputs are their stable merge (a first on ties),
// or simply the inputs in that order (TF_COPY: a concatenation node).
enum : int { TF_SKIP = 1, TF_COPY = 2, TF_AREV = 8, TF_BREV = 16 };
struct TileDesc {
    int64_t pa, pb;   // lowest logical slots of its view-a / view-b inputs
    int64_t o;        // logical slot of its first output
    unsigned dlo, dhi;       // dependency window (tickets, inclusive; empty if dlo > dhi)
    int la, cnt;      // view-a inputs, total inputs (= outputs)
    // its problem (row of the table) in a table run; for the single tree
    // with run samples, 2 * (its sample slot) + (1: the node is a right child,
    // its sample is the stretch's last key; 0: a left child, the first key),
    // or -1
    int prob;
    int flags;        // TF_*; TF_SKIP: empty, or every output already sits in its slot
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

// Every wait is bounded: a wait whose status has not arrived after
// kSpinLimit polls sets *err (the call then reports a device error) and gives
// up, so no wave spins forever.  The word before *err is a test setting
// written from the host: with bit 0 set, every wait that checks another work
// item still waits as usual but then sets *err as if it had given up (the
// error paths run while the output stays correct).
constexpr unsigned kSpinLimit = 1u << 22;

// Called by one full wavefront: returns once every ticket in [lo, hi] other
// than `self` has published its loaded status for `epoch`, or the limit ran
// out.
__device__ __forceinline__ void wait_window(const unsigned *status, int64_t lo, int64_t hi,
                                            int64_t self, unsigned epoch, unsigned *err)
{
    const int lane = threadIdx.x & 63;
    const unsigned want = epoch << 2;
    const bool force_fail = (ld_status(err - 1) & 1u) != 0;
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
            if ((st & ~3u) != want || force_fail)
                __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// A work-group barrier that orders LDS accesses only: the fences are limited
// to the local address space, so global loads in flight (a prefetched tile)
// stay in flight across it.  For barriers whose only job is LDS reuse.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
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
