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
