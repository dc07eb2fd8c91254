// Geometry of the Frogsort1 tree ("Symmetric merging", "Frogsort1") and of
// one Frogsort2 node ("Frogsort2", at the end).
//
// A node sorts `n` data elements inside a region of m(n) = n + floor(n/2)
// slots of the logical frog space.  A left node leaves its data at the left
// end of its region, a right node at the right end.  Its outer child (left
// child of a left node, right child of a right node) takes ceil(n/2) elements
// (rule 1: the surplus goes outward); the inner child takes floor(n/2), which
// always fits the floor(n/2)-slot gap between the two children's data (rule 2:
// the buffer is floor(n/2)).  The left child is a left node at the start of
// the region, the right child a right node at its end.  The top node is a left
// node over [0, m(n)), so the sorted result ends in slots [0, n) with no copy.
//
// The GPU path processes the tree breadth first: all leaves (depth D, at most
// `leaf_max` elements each) in one launch, then one merge launch per level from
// depth D-1 up to 0.  Every node's geometry is recomputed on the fly by walking
// from the root, so Frogsort1 needs no descriptor table.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define GS_HD __host__ __device__ __forceinline__
#else
#define GS_HD inline
#endif

namespace gs {

GS_HD int64_t frog_region(int64_t n) { return n + n / 2; }

struct FrogNode {
    int64_t s;        // region start (logical slot)
    int64_t n;        // data elements
    int64_t in_off;   // offset of its elements in the input order
    int     left;     // 1: data at the left end of the region, 0: right end
};

// Node `idx` (0 = leftmost) at depth `depth` of the tree over `n_total`.
GS_HD FrogNode frog_node(int64_t n_total, int depth, int64_t idx)
{
    FrogNode f{0, n_total, 0, 1};
    for (int d = depth - 1; d >= 0; --d) {
        int64_t nl = f.left ? (f.n + 1) / 2 : f.n / 2;
        int64_t nr = f.n - nl;
        if ((idx >> d) & 1) {
            f.s += frog_region(f.n) - frog_region(nr);
            f.in_off += nl;
            f.n = nr;
            f.left = 0;
        } else {
            f.n = nl;
            f.left = 1;
        }
    }
    return f;
}

// First slot of the node's data.
GS_HD int64_t frog_data_start(const FrogNode &f)
{
    return f.left ? f.s : f.s + frog_region(f.n) - f.n;
}

// The merge a node performs: the two runs and where the output goes.  The
// first run wins ties (it holds the earlier input).  One run may lie inside
// the output ("outer"); its elements only move away from the side the output
// is written from:
//   outer 0: first run at [out0, out0+nl), output written top-down (left node)
//   outer 1: second run at [out0+nl, out0+n), written bottom-up (right node)
//   outer 2: first run at [out0+nr, out0+n), written bottom-up
struct FrogMerge {
    int64_t l0, nl;   // first run  [l0, l0+nl)
    int64_t r0, nr;   // second run [r0, r0+nr)
    int64_t out0;     // output     [out0, out0+nl+nr)
    int     left;     // 1 = output written top-down
    int     outer;    // which run lies inside the output (see above)
};

GS_HD FrogMerge frog_merge_of(const FrogNode &f)
{
    FrogMerge m;
    m.nl = f.left ? (f.n + 1) / 2 : f.n / 2;
    m.nr = f.n - m.nl;
    m.l0 = f.s;
    m.r0 = f.s + frog_region(f.n) - m.nr;
    m.out0 = frog_data_start(f);
    m.left = f.left;
    m.outer = f.left ? 0 : 1;
    return m;
}

// ---------------------------------------------------------------------------
// Squidsort: directions of runs and how a node forms its run
// ---------------------------------------------------------------------------
// "Squidsort" combines Frogsort with the non-overlap test of "Full
// adaptivity" and the data-driven order of Octosort.  A run comes back
// ascending, or descending (it then holds the stable ascending result of its
// node reversed); DIR_NONE is a run of one element.  A node whose children
// both come back in one direction and do not overlap is their concatenation
// in that direction (only the inner run moves).  Every other node merges into
// an ascending run: a descending inner run is read from its end, and a
// descending outer run -- which lies inside the output, where only a run read
// in its own storage order moves away from the side the output is written
// from -- is first turned around in place (NODE_MERGE_REV).  The top run is
// reversed once if it comes back descending.
enum : int { DIR_NONE = 0, DIR_ASC = 1, DIR_DESC = 2 };
enum : int { NODE_MERGE = 0, NODE_MERGE_REV = 1, NODE_CONCAT = 2 };

// Element i of a view sits at slot start + step * i.
struct RunView {
    int64_t start;
    int64_t step;     // +1 or -1
    int64_t n;
};

GS_HD int64_t view_slot(const RunView &v, int64_t i) { return v.start + v.step * i; }
GS_HD RunView view_of(int64_t first, int64_t n, bool reversed)
{
    RunView v;
    v.start = reversed ? first + n - 1 : first;
    v.step = reversed ? -1 : 1;
    v.n = n;
    return v;
}

// The two input sequences a node's tiles read, in output order: the output
// is the stable merge of a and b (a, the first run, wins ties), or their
// plain concatenation (copy).  turned: the outer run has already been turned
// around in place (the tiles see it ascending; the merge-path splits, taken
// before, read it from its end, which is the same sequence).
struct NodeViews {
    RunView a, b;
    int copy;
};

GS_HD NodeViews node_views(const FrogMerge &m, int kind, int dL, int dR, bool turned)
{
    NodeViews v;
    v.copy = kind == NODE_CONCAT;
    if (kind == NODE_CONCAT) {
        v.a = view_of(m.l0, m.nl, false);
        v.b = view_of(m.r0, m.nr, false);
    } else {
        const bool outer_first = m.outer != 1;
        const bool revL = dL == DIR_DESC && !(turned && outer_first);
        const bool revR = dR == DIR_DESC && !(turned && !outer_first);
        v.a = view_of(m.l0, m.nl, revL);
        v.b = view_of(m.r0, m.nr, revR);
    }
    return v;
}

// Packed per-node mode: kind | dL << 2 | dR << 4.
GS_HD unsigned node_mode_pack(int kind, int dL, int dR) { return (unsigned)(kind | dL << 2 | dR << 4); }
GS_HD int node_mode_kind(unsigned w) { return (int)(w & 3u); }
GS_HD int node_mode_dl(unsigned w) { return (int)((w >> 2) & 3u); }
GS_HD int node_mode_dr(unsigned w) { return (int)((w >> 4) & 3u); }

// Dependency window of one merge tile ("Symmetric merging" made into an
// ordered-store protocol).  Tile j of a node (tpn tiles; its outputs are
// ranks [min(j*tile, n), min((j+1)*tile, n)) written at out0 + rank) may
// store only after every tile that reads an element in a slot it overwrites
// has loaded.  sp holds the node's tpn + 1 merge-path splits (sp[j] = first
// elements of view a among the outputs before tile j; for a concatenation
// sp[j] = min(j*tile, na)).  Tiles take tickets first + j (the output written
// bottom-up) or first + tpn - 1 - j (top-down, a left node).  Returns the
// window [*lo, *hi] (empty when *lo > *hi), the tile's own ticket included
// when it reads slots it writes.
GS_HD int64_t ub_a(const int64_t *sp, int64_t count, int64_t x)
{
    int64_t lo = 0, hi = count;          // first j with sp[j] > x
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (sp[mid] > x) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}
GS_HD int64_t ub_b(const int64_t *sp, int64_t count, int64_t tile, int64_t n, int64_t x)
{
    int64_t lo = 0, hi = count;          // first j with min(j*tile, n) - sp[j] > x
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        const int64_t k = mid * tile < n ? mid * tile : n;
        if (k - sp[mid] > x) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

GS_HD void tile_window(const NodeViews &v, int64_t out0, int left, const int64_t *sp, int64_t tpn,
                       int64_t tile, int64_t j, int64_t first, int64_t *lo, int64_t *hi)
{
    const int64_t n = v.a.n + v.b.n;
    int64_t k0 = j * tile, k1 = k0 + tile;
    k0 = k0 < n ? k0 : n;
    k1 = k1 < n ? k1 : n;
    int64_t wlo = 1, whi = 0;
    for (int r = 0; r < 2 && k0 < k1; ++r) {
        const RunView &x = r == 0 ? v.a : v.b;
        if (x.n <= 0) continue;
        // slots of x the tile overwrites
        const int64_t xs = x.step > 0 ? x.start : x.start - (x.n - 1);
        const int64_t p0 = out0 + k0 > xs ? out0 + k0 : xs;
        const int64_t p1 = out0 + k1 < xs + x.n ? out0 + k1 : xs + x.n;
        if (p0 >= p1) continue;
        int64_t va = (p0 - x.start) * x.step, vb = (p1 - 1 - x.start) * x.step;
        if (va > vb) {
            const int64_t t = va;
            va = vb;
            vb = t;
        }
        // the tiles reading view elements [va, vb]
        int64_t j0, j1;
        if (r == 0) {
            j0 = ub_a(sp, tpn + 1, va) - 1;
            j1 = ub_a(sp, tpn + 1, vb) - 1;
        } else {
            j0 = ub_b(sp, tpn + 1, tile, n, va) - 1;
            j1 = ub_b(sp, tpn + 1, tile, n, vb) - 1;
        }
        j0 = j0 < 0 ? 0 : j0 > tpn - 1 ? tpn - 1 : j0;
        j1 = j1 < 0 ? 0 : j1 > tpn - 1 ? tpn - 1 : j1;
        const int64_t tl = left ? first + (tpn - 1 - j1) : first + j0;
        const int64_t th = left ? first + (tpn - 1 - j0) : first + j1;
        if (wlo > whi) {
            wlo = tl;
            whi = th;
        } else {
            wlo = tl < wlo ? tl : wlo;
            whi = th > whi ? th : whi;
        }
    }
    *lo = wlo;
    *hi = whi;
}

// Leaf (node index at `depth`) whose input chunk holds input position p.
GS_HD int64_t frog_leaf_of(int64_t n_total, int depth, int64_t p)
{
    int64_t n = n_total, in_off = 0, idx = 0;
    int left = 1;
    for (int d = 0; d < depth; ++d) {
        const int64_t nl = left ? (n + 1) / 2 : n / 2;
        if (p < in_off + nl) {
            n = nl;
            left = 1;
            idx = idx * 2;
        } else {
            in_off += nl;
            n -= nl;
            left = 0;
            idx = idx * 2 + 1;
        }
    }
    return idx;
}

// Ordered-store window of a leaf of the Frogsort1 tree (depth `depth` over n
// elements): the leaf sorts input chunk `leaf` and stores it at its data
// start, overwriting the input chunks of the leaves whose chunks its
// destination covers.  Leaves take tickets in descending index order
// (ticket = leaves - 1 - index), so those leaves -- never one with a smaller
// index, as every data start is at or after its chunk -- hold tickets up to
// its own.  [*lo, *hi] is empty (lo > hi) when the destination lies past the
// caller's array.
GS_HD void leaf_window(int64_t n, int depth, int64_t leaf, int64_t *lo, int64_t *hi)
{
    const FrogNode f = frog_node(n, depth, leaf);
    const int64_t dst = frog_data_start(f), len = f.n;
    const int64_t nleaves = (int64_t)1 << depth;
    *lo = 1;
    *hi = 0;
    if (dst < n && len > 0) {
        const int64_t end = (dst + len < n ? dst + len : n) - 1;
        *lo = nleaves - 1 - frog_leaf_of(n, depth, end);
        *hi = nleaves - 1 - frog_leaf_of(n, depth, dst);
    }
}

// Depth at which every node holds at most leaf_max elements (sizes at depth d
// are floor(n/2^d) or ceil(n/2^d)).
GS_HD int frog_depth(int64_t n, int64_t leaf_max)
{
    int d = 0;
    while (((n + ((int64_t)1 << d) - 1) >> d) > leaf_max) ++d;
    return d;
}

// Largest node size at depth d.
GS_HD int64_t frog_max_node(int64_t n, int d)
{
    return (n + ((int64_t)1 << d) - 1) >> d;
}

// ---------------------------------------------------------------------------
// Frogsort2
// ---------------------------------------------------------------------------
// The inner child of a node of n elements takes floor(q n / 2^16) of them and
// the outer child the rest; the node's region is n + floor(q n / 2^16) slots
// ("Frogsort2": inner branch and buffer both the fraction p = q / 2^16).  The
// children sit as in Frogsort1, so a node's merge is a FrogMerge of the same
// two kinds (outer 0 for a left node, outer 1 for a right node).
constexpr int64_t kF2LeftBit = (int64_t)1 << 62;

GS_HD int64_t f2_inner(int64_t n, int64_t q) { return (n * q) >> 16; }

GS_HD FrogMerge f2_merge(int64_t s, int64_t n_left, int64_t q)
{
    const int64_t n = n_left & (kF2LeftBit - 1);
    const int64_t ni = f2_inner(n, q);
    FrogMerge m;
    m.l0 = s;
    if (n_left & kF2LeftBit) {           // outer run: left child's data at [s, s + n - ni)
        m.nl = n - ni;
        m.nr = ni;
        m.r0 = s + n;                    // inner run just past the output
        m.out0 = s;
        m.left = 1;
        m.outer = 0;
    } else {                             // inner run at [s, s + ni), just before the output
        m.nl = ni;
        m.nr = n - ni;
        m.r0 = s + 2 * ni;
        m.out0 = s + ni;
        m.left = 0;
        m.outer = 1;
    }
    return m;
}

}  // namespace gs
