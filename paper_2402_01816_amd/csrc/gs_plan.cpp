// Host planning of the irregular trees (Frogsort2, Frogsort3 / Frogsort6):
// walks each tree once and keeps the tables of the last few plans.
#include <hip/hip_runtime.h>
#include <string.h>

#include <list>
#include <memory>
#include <mutex>
#include <vector>

#include "frog_geometry.h"
#include "gs_internal.h"

namespace gs {

static int64_t align256(int64_t b) { return (b + 255) & ~(int64_t)255; }

// ---------------------------------------------------------------------------
// Frogsort2 planning (host)
// ---------------------------------------------------------------------------
// The tree of an imbalanced split has leaves at many depths and no closed form
// for "node i of level d", so the host walks it once (O(n / leaf) nodes) and
// keeps the tables of the last few (n, q, leaf, tile) it planned.
namespace {

struct F2Walk {
    int64_t q, leaf;
    std::vector<int64_t> leaf_c, leaf_d;   // leaves in input order
    std::vector<int64_t> ns, nn;           // merge nodes in post order
    std::vector<int> nh;                   // their heights
};

int64_t f2_region(int64_t n, int64_t q) { return n + f2_inner(n, q); }

// The node over [s, s + region) that holds input [c, c + n); returns its
// height (0 for a leaf).  A left leaf's data start at its region's start, a
// right leaf's at its end minus n.
int f2_walk(F2Walk &W, int64_t s, int64_t n, int64_t c, int left)
{
    if (n <= W.leaf) {
        W.leaf_c.push_back(c);
        W.leaf_d.push_back(left ? s : s + f2_inner(n, W.q));
        return 0;
    }
    const int64_t ni = f2_inner(n, W.q);
    const int64_t nl = left ? n - ni : ni, nr = n - nl;
    const int hl = f2_walk(W, s, nl, c, 1);
    const int hr = f2_walk(W, s + f2_region(n, W.q) - f2_region(nr, W.q), nr, c + nl, 0);
    const int h = 1 + (hl > hr ? hl : hr);
    W.ns.push_back(s);
    W.nn.push_back(n | (left ? kF2LeftBit : 0));
    W.nh.push_back(h);
    return h;
}

template <class T>
int64_t f2_put(std::vector<char> &blob, const std::vector<T> &v)
{
    const int64_t off = align256((int64_t)blob.size());
    blob.resize((size_t)(off + (int64_t)(v.size() * sizeof(T))));
    if (!v.empty()) memcpy(blob.data() + off, v.data(), v.size() * sizeof(T));
    return off;
}

// Tables of the tree whose root (left or right node) has its region at s0 and
// its n input elements at [c0, c0 + n).
std::shared_ptr<const F2Tables> f2_build(int64_t s0, int64_t n, int64_t c0, int left0, int64_t q, int64_t leaf,
                                         int64_t tile)
{
    F2Walk W;
    W.q = q;
    W.leaf = leaf;
    const int H = f2_walk(W, s0, n, c0, left0);
    auto T = std::make_shared<F2Tables>();
    T->n = n;
    T->q = q;
    T->leaf = leaf;
    T->tile = tile;
    T->rounds = H;
    T->nleaves = (int64_t)W.leaf_c.size();
    T->nnodes = (int64_t)W.ns.size();
    // merge nodes grouped by height, post order within a height
    std::vector<unsigned> rb((size_t)H + 2, 0u);
    for (int h : W.nh) rb[(size_t)h + 1]++;
    for (int r = 1; r <= H; ++r) rb[(size_t)r + 1] += rb[(size_t)r];
    std::vector<unsigned> fill(rb.begin(), rb.end());
    std::vector<int64_t> ns((size_t)T->nnodes), nn((size_t)T->nnodes);
    for (size_t i = 0; i < W.ns.size(); ++i) {
        const unsigned k = fill[(size_t)W.nh[i]]++;
        ns[k] = W.ns[i];
        nn[k] = W.nn[i];
    }
    std::vector<unsigned> tb((size_t)T->nnodes), sb((size_t)T->nnodes);
    T->rt.assign((size_t)H + 1, 0u);
    T->rs.assign((size_t)H + 1, 0u);
    T->max_tickets = T->max_splits = 0;
    T->merged = 0;
    for (size_t i = 0; i < nn.size(); ++i) T->merged += nn[i] & (kF2LeftBit - 1);
    for (int r = 1; r <= H; ++r) {
        int64_t t = 0, sp = 0;
        for (unsigned k = rb[(size_t)r]; k < rb[(size_t)r + 1]; ++k) {
            const int64_t tpn = ((nn[k] & (kF2LeftBit - 1)) + tile - 1) / tile;
            tb[k] = (unsigned)t;
            sb[k] = (unsigned)sp;
            t += tpn;
            sp += tpn + 1;
        }
        T->rt[(size_t)r] = (unsigned)t;
        T->rs[(size_t)r] = (unsigned)sp;
        if (t > T->max_tickets) T->max_tickets = t;
        if (sp > T->max_splits) T->max_splits = sp;
    }
    std::vector<int64_t> lc = W.leaf_c;
    lc.push_back(c0 + n);
    T->off_leaf_c = f2_put(T->blob, lc);
    T->off_leaf_d = f2_put(T->blob, W.leaf_d);
    T->off_node_s = f2_put(T->blob, ns);
    T->off_node_n = f2_put(T->blob, nn);
    T->off_node_tb = f2_put(T->blob, tb);
    T->off_node_sb = f2_put(T->blob, sb);
    T->off_rb = f2_put(T->blob, rb);
    T->off_rt = f2_put(T->blob, T->rt);
    T->off_rs = f2_put(T->blob, T->rs);
    T->blob.resize((size_t)align256((int64_t)T->blob.size()));
    return T;
}

std::mutex g_plan_mu;
std::list<std::shared_ptr<const F2Tables>> g_f2_cache;   // most recently used first
constexpr size_t kF2CacheEntries = 8;

// Entries are immutable; a call holds its own reference for as long as it
// reads one, so dropping an entry from the list never frees tables in use.
}  // namespace

std::shared_ptr<const F2Tables> f2_tables(int64_t n, int64_t q, int64_t leaf, int64_t tile)
{
    {
        std::lock_guard<std::mutex> g(g_plan_mu);
        for (auto it = g_f2_cache.begin(); it != g_f2_cache.end(); ++it) {
            const F2Tables &t = **it;
            if (t.n == n && t.q == q && t.leaf == leaf && t.tile == tile) {
                auto hit = *it;
                g_f2_cache.erase(it);
                g_f2_cache.push_front(hit);
                return hit;
            }
        }
    }
    auto t = f2_build(0, n, 0, 1, q, leaf, tile);
    std::lock_guard<std::mutex> g(g_plan_mu);
    g_f2_cache.push_front(t);
    if (g_f2_cache.size() > kF2CacheEntries) g_f2_cache.pop_back();
    return t;
}

namespace {

std::shared_ptr<const F3Plan> f3_build(int64_t n, int64_t q, int64_t q2, int64_t leaf, int64_t tile)
{
    auto P = std::make_shared<F3Plan>();
    P->n = n;
    P->q = q;
    P->q2 = q2;
    P->leaf = leaf;
    P->tile = tile;
    const int64_t b = f2_inner(n, q);
    P->b = b;
    std::vector<int64_t> sizes;                 // spine nodes that split
    int64_t m = n;
    while (m > leaf && f2_inner(m, q2) > b) {
        // inner child: the last b elements, a right node whose sub-tree
        // region (b + floor(q2 b / 2^16) slots) ends at m + b
        const int64_t s0 = m + b - f2_region(b, q2);
        P->trees.push_back(f2_build(s0, b, m - b, 0, q2, leaf, tile));
        P->root_s.push_back(s0);
        P->root_n.push_back(b);
        P->root_c.push_back(m - b);
        P->root_left.push_back(0);
        sizes.push_back(m);
        m -= b;
    }
    P->trees.push_back(f2_build(0, m, 0, 1, q2, leaf, tile));
    P->root_s.push_back(0);
    P->root_n.push_back(m);
    P->root_c.push_back(0);
    P->root_left.push_back(1);
    for (size_t k = sizes.size(); k-- > 0;) {
        const int64_t mk = sizes[k];
        FrogMerge fm;
        fm.l0 = 0;
        fm.nl = mk - b;
        fm.r0 = mk;
        fm.nr = b;
        fm.out0 = 0;
        fm.left = 1;
        fm.outer = 0;
        P->spine.push_back(fm);
    }
    P->max_rounds = 0;
    P->total_rounds = (int)P->spine.size();
    P->max_tickets = P->max_splits = P->max_status = 1;
    P->merged = 0;
    for (const auto &t : P->trees) {
        P->merged += t->merged;
        const int64_t off = align256((int64_t)P->image.size());
        P->tree_off.push_back(off);
        P->image.resize((size_t)(off + (int64_t)t->blob.size()));
        memcpy(P->image.data() + off, t->blob.data(), t->blob.size());
        P->max_rounds = t->rounds > P->max_rounds ? t->rounds : P->max_rounds;
        P->total_rounds += t->rounds;
        P->max_tickets = t->max_tickets > P->max_tickets ? t->max_tickets : P->max_tickets;
        P->max_splits = t->max_splits > P->max_splits ? t->max_splits : P->max_splits;
        P->max_status = t->nleaves > P->max_status ? t->nleaves : P->max_status;
    }
    for (const FrogMerge &fm : P->spine) {
        P->merged += fm.nl + fm.nr;
        const int64_t tiles = (fm.nl + fm.nr + tile - 1) / tile;
        P->max_tickets = tiles > P->max_tickets ? tiles : P->max_tickets;
        P->max_splits = tiles + 1 > P->max_splits ? tiles + 1 : P->max_splits;
    }
    P->max_status = P->max_tickets > P->max_status ? P->max_tickets : P->max_status;
    return P;
}

std::list<std::shared_ptr<const F3Plan>> g_f3_cache;     // most recently used first

}  // namespace

std::shared_ptr<const F3Plan> f3_plans(int64_t n, int64_t q, int64_t q2, int64_t leaf, int64_t tile)
{
    {
        std::lock_guard<std::mutex> g(g_plan_mu);
        for (auto it = g_f3_cache.begin(); it != g_f3_cache.end(); ++it) {
            const F3Plan &t = **it;
            if (t.n == n && t.q == q && t.q2 == q2 && t.leaf == leaf && t.tile == tile) {
                auto hit = *it;
                g_f3_cache.erase(it);
                g_f3_cache.push_front(hit);
                return hit;
            }
        }
    }
    auto t = f3_build(n, q, q2, leaf, tile);
    std::lock_guard<std::mutex> g(g_plan_mu);
    g_f3_cache.push_front(t);
    if (g_f3_cache.size() > kF2CacheEntries) g_f3_cache.pop_back();
    return t;
}

}  // namespace gs
