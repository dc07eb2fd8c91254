/*
 * CPU oracle for the greeNsort stable-sorting path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  It shares no
 * code, header, helper or constant with the GPU library and must never be
 * used as a fallback for it.
 *
 * Everything here is written to be slow and obviously correct:
 *
 *   - oracle_sort_*  : the result the paper's task defines ("Definition of
 *     sorting": stable ascending order with ties kept in input order read from
 *     left to right, the AscLeft target; "Values and principles / Stability").
 *     oracle_sort_*_target: the four stable targets (AscLeft, AscRight,
 *     DescLeft, DescRight) written as one composite (key, index) order.
 *     It is computed by the prototypical stable mergesort of the section
 *     "Merging or partitioning?" (one full-size buffer, top-down, take the left
 *     element unless the right one is strictly smaller).  Frogsort reaches this
 *     same result; the oracle does not implement Frogsort.
 *   - oracle_rank_*  : the same definition written as a count, usable one
 *     element at a time on arrays too large to sort on the CPU in a test.
 *   - oracle_frog_*  : an instrumented model of the paper's Frogsort0/Frogsort1
 *     recursion ("Symmetric merging", "Frogsort0", "Frogsort1") used only to
 *     pin the memory layout and the adaptivity counts the paper states.
 *   - oracle_squid_* : the same for Squidsort1 ("Squidsort": Frogsort1 with the
 *     non-overlap test of "Full adaptivity" and Octosort's data-driven,
 *     lazily enforced order), checking every write against unread elements.
 *   - oracle_frog2_* : the same for Frogsort2 ("Frogsort2": imbalanced splits,
 *     buffer p), checking on every write that the smaller buffer suffices.
 *   - oracle_frog3_* : the same for Frogsort3 / Frogsort6 (the buffer shared by
 *     the two branches in turn), with the input placed in place.
 *   - oracle_mlp_*   : an fp64 forward pass, MSE loss, backward pass and Adam
 *     step for the 1-64-64-1 ReLU network used by the learned bucket path
 *     (not part of the paper; parity of the GPU gradients is checked here).
 *
 * Comparison (the paper only asks for comparison sorting of doubles): less(a,b)
 * is IEEE a<b, except that every NaN is greater than every non-NaN and NaNs tie
 * with each other.  -0.0 and +0.0 therefore tie and keep their input order.
 * Unsigned 64-bit keys compare with unsigned <.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* comparison                                                                */
/* ------------------------------------------------------------------------ */

int oracle_less_f64(double a, double b)
{
    if (isnan(a)) return 0;          /* NaN is never less than anything */
    if (isnan(b)) return 1;          /* non-NaN is less than NaN        */
    return a < b;                    /* IEEE: -0 < +0 is false          */
}

static int less_u64(uint64_t a, uint64_t b) { return a < b; }

/* ------------------------------------------------------------------------ */
/* prototypical stable mergesort with a 100% buffer                          */
/* ------------------------------------------------------------------------ */

/* Sort x[lo,hi) stably using tmp[lo,hi) as scratch. */
static void msort_f64(double *x, double *tmp, int64_t lo, int64_t hi)
{
    if (hi - lo < 2) return;
    int64_t mid = lo + (hi - lo) / 2;
    msort_f64(x, tmp, lo, mid);
    msort_f64(x, tmp, mid, hi);
    int64_t i = lo, j = mid, k = lo;
    while (i < mid && j < hi) {
        /* a right element is taken only if it is strictly smaller: ties keep
           the left (earlier) element first */
        if (oracle_less_f64(x[j], x[i])) tmp[k++] = x[j++];
        else                             tmp[k++] = x[i++];
    }
    while (i < mid) tmp[k++] = x[i++];
    while (j < hi)  tmp[k++] = x[j++];
    memcpy(x + lo, tmp + lo, (size_t)(hi - lo) * sizeof(double));
}

static void msort_kv(uint64_t *k, uint32_t *v, uint64_t *tk, uint32_t *tv,
                     int64_t lo, int64_t hi)
{
    if (hi - lo < 2) return;
    int64_t mid = lo + (hi - lo) / 2;
    msort_kv(k, v, tk, tv, lo, mid);
    msort_kv(k, v, tk, tv, mid, hi);
    int64_t i = lo, j = mid, o = lo;
    while (i < mid && j < hi) {
        if (less_u64(k[j], k[i])) { tk[o] = k[j]; tv[o] = v[j]; o++; j++; }
        else                      { tk[o] = k[i]; tv[o] = v[i]; o++; i++; }
    }
    while (i < mid) { tk[o] = k[i]; tv[o] = v[i]; o++; i++; }
    while (j < hi)  { tk[o] = k[j]; tv[o] = v[j]; o++; j++; }
    memcpy(k + lo, tk + lo, (size_t)(hi - lo) * sizeof(uint64_t));
    memcpy(v + lo, tv + lo, (size_t)(hi - lo) * sizeof(uint32_t));
}

/* Returns 0 on success, -1 if the scratch buffer could not be allocated. */
int oracle_sort_f64(double *x, int64_t n)
{
    if (n < 2) return 0;
    double *tmp = (double *)malloc((size_t)n * sizeof(double));
    if (!tmp) return -1;
    msort_f64(x, tmp, 0, n);
    free(tmp);
    return 0;
}

int oracle_sort_kv(uint64_t *k, uint32_t *v, int64_t n)
{
    if (n < 2) return 0;
    uint64_t *tk = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    uint32_t *tv = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    if (!tk || !tv) { free(tk); free(tv); return -1; }
    msort_kv(k, v, tk, tv, 0, n);
    free(tk); free(tv);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* the four stable targets ("Definition of sorting")                          */
/* ------------------------------------------------------------------------ */
/* Target t: bit 1 = descending key order, bit 0 = ties in reverse input order
   (read from the right) instead of input order (read from the left):
   0 AscLeft, 1 AscRight, 2 DescLeft, 3 DescRight.  Written as the plain
   definition: element i comes before element j iff its key comes first in
   the target's key order, or the keys tie and its index comes first in the
   target's index order.  That order is total, so any correct sort of the
   indices by it gives the result. */
static int before_f64(const double *x, int64_t i, int64_t j, int t)
{
    const int desc = (t >> 1) & 1, right = t & 1;
    const double a = x[i], b = x[j];
    if (desc ? oracle_less_f64(b, a) : oracle_less_f64(a, b)) return 1;
    if (desc ? oracle_less_f64(a, b) : oracle_less_f64(b, a)) return 0;
    return right ? i > j : i < j;
}

static int before_u64(const uint64_t *k, int64_t i, int64_t j, int t)
{
    const int desc = (t >> 1) & 1, right = t & 1;
    const uint64_t a = k[i], b = k[j];
    if (desc ? less_u64(b, a) : less_u64(a, b)) return 1;
    if (desc ? less_u64(a, b) : less_u64(b, a)) return 0;
    return right ? i > j : i < j;
}

/* mergesort of an index array by the order `before` (keys of one type) */
static void msort_idx(int64_t *ix, int64_t *tmp, int64_t lo, int64_t hi, const void *keys, int is_f64, int t)
{
    if (hi - lo < 2) return;
    int64_t mid = lo + (hi - lo) / 2;
    msort_idx(ix, tmp, lo, mid, keys, is_f64, t);
    msort_idx(ix, tmp, mid, hi, keys, is_f64, t);
    int64_t i = lo, j = mid, k = lo;
    while (i < mid && j < hi) {
        const int jb = is_f64 ? before_f64((const double *)keys, ix[j], ix[i], t)
                              : before_u64((const uint64_t *)keys, ix[j], ix[i], t);
        tmp[k++] = jb ? ix[j++] : ix[i++];
    }
    while (i < mid) tmp[k++] = ix[i++];
    while (j < hi)  tmp[k++] = ix[j++];
    memcpy(ix + lo, tmp + lo, (size_t)(hi - lo) * sizeof(int64_t));
}

/* x sorted in place for target t; -1 on allocation failure, -2 bad target. */
int oracle_sort_f64_target(double *x, int64_t n, int t)
{
    if (t < 0 || t > 3) return -2;
    if (n < 2) return 0;
    int64_t *ix = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *tmp = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    double *y = (double *)malloc((size_t)n * sizeof(double));
    if (!ix || !tmp || !y) { free(ix); free(tmp); free(y); return -1; }
    for (int64_t i = 0; i < n; ++i) ix[i] = i;
    msort_idx(ix, tmp, 0, n, x, 1, t);
    for (int64_t i = 0; i < n; ++i) y[i] = x[ix[i]];
    memcpy(x, y, (size_t)n * sizeof(double));
    free(ix); free(tmp); free(y);
    return 0;
}

int oracle_sort_kv_target(uint64_t *k, uint32_t *v, int64_t n, int t)
{
    if (t < 0 || t > 3) return -2;
    if (n < 2) return 0;
    int64_t *ix = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *tmp = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    uint64_t *yk = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    uint32_t *yv = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    if (!ix || !tmp || !yk || !yv) { free(ix); free(tmp); free(yk); free(yv); return -1; }
    for (int64_t i = 0; i < n; ++i) ix[i] = i;
    msort_idx(ix, tmp, 0, n, k, 0, t);
    for (int64_t i = 0; i < n; ++i) { yk[i] = k[ix[i]]; yv[i] = v[ix[i]]; }
    memcpy(k, yk, (size_t)n * sizeof(uint64_t));
    memcpy(v, yv, (size_t)n * sizeof(uint32_t));
    free(ix); free(tmp); free(yk); free(yv);
    return 0;
}

/* Segment i is x[off[i], off[i+1]); each segment is sorted on its own.
   Returns -2 if the offsets are not non-decreasing or off[0] < 0. */
int oracle_segsort_f64(double *x, const int64_t *off, int64_t nseg)
{
    if (nseg <= 0) return 0;
    if (off[0] < 0) return -2;
    int64_t maxlen = 0;
    for (int64_t s = 0; s < nseg; s++) {
        if (off[s + 1] < off[s]) return -2;
        if (off[s + 1] - off[s] > maxlen) maxlen = off[s + 1] - off[s];
    }
    if (maxlen < 2) return 0;
    double *tmp = (double *)malloc((size_t)maxlen * sizeof(double));
    if (!tmp) return -1;
    for (int64_t s = 0; s < nseg; s++) {
        int64_t lo = off[s], len = off[s + 1] - off[s];
        if (len >= 2) msort_f64(x + lo, tmp, 0, len);
    }
    free(tmp);
    return 0;
}

int oracle_segsort_kv(uint64_t *k, uint32_t *v, const int64_t *off, int64_t nseg)
{
    if (nseg <= 0) return 0;
    if (off[0] < 0) return -2;
    int64_t maxlen = 0;
    for (int64_t s = 0; s < nseg; s++) {
        if (off[s + 1] < off[s]) return -2;
        if (off[s + 1] - off[s] > maxlen) maxlen = off[s + 1] - off[s];
    }
    if (maxlen < 2) return 0;
    uint64_t *tk = (uint64_t *)malloc((size_t)maxlen * sizeof(uint64_t));
    uint32_t *tv = (uint32_t *)malloc((size_t)maxlen * sizeof(uint32_t));
    if (!tk || !tv) { free(tk); free(tv); return -1; }
    for (int64_t s = 0; s < nseg; s++) {
        int64_t lo = off[s], len = off[s + 1] - off[s];
        if (len >= 2) msort_kv(k + lo, v + lo, tk, tv, 0, len);
    }
    free(tk); free(tv);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* the definition as a count                                                 */
/* ------------------------------------------------------------------------ */

/* Output position of input element j under the stable ascending definition:
   the number of elements strictly less than x[j], plus the number of earlier
   elements tied with x[j].  One pass over x answers m queries at once. */
void oracle_rank_f64(const double *x, int64_t n, const int64_t *idx, int64_t m,
                     int64_t *rank)
{
    for (int64_t q = 0; q < m; q++) rank[q] = 0;
    for (int64_t i = 0; i < n; i++) {
        double xi = x[i];
        for (int64_t q = 0; q < m; q++) {
            double xq = x[idx[q]];
            if (oracle_less_f64(xi, xq)) rank[q]++;
            else if (i < idx[q] && !oracle_less_f64(xq, xi)) rank[q]++;
        }
    }
}

void oracle_rank_u64(const uint64_t *x, int64_t n, const int64_t *idx, int64_t m,
                     int64_t *rank)
{
    for (int64_t q = 0; q < m; q++) rank[q] = 0;
    for (int64_t i = 0; i < n; i++) {
        uint64_t xi = x[i];
        for (int64_t q = 0; q < m; q++) {
            uint64_t xq = x[idx[q]];
            if (xi < xq || (xi == xq && i < idx[q])) rank[q]++;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* instrumented model of the Frogsort recursion                             */
/* ------------------------------------------------------------------------ */
/*
 * Memory is a logical array of slots.  Data elements are carried as (key,
 * label) pairs so that the layout tables of the paper can be reproduced: the
 * label of an element is the position it had after setup.  Slot contents that
 * are buffer hold label -1.
 *
 * A node covers `u` units; a unit is `g` data slots (g = 1: Frogsort1, single
 * elements; g = 2: Frogsort0 triplets, two data and one buffer slot).  A node
 * of u units has n = g*u data elements and a region of n + floor(n/2) slots
 * (for g = 2 this is 3u slots, one buffer slot per triplet).
 *
 * A left node leaves its sorted data at the left end of its region, a right
 * node at the right end.  Its outer child (the left child of a left node, the
 * right child of a right node) receives the surplus unit when u is odd
 * (Frogsort1 rule 1; Frogsort0 rule), so the inner child is never larger than
 * the gap between the two children's data (Frogsort1 rule 2: the buffer is
 * floor(n/2)).  Merging proceeds from the inner ends of the two runs towards
 * the outer border ("Symmetric merging"): a left node writes its output from
 * the top (next to the gap) down to its left border, a right node from the
 * bottom up to its right border.
 */

typedef struct {
    double  *key;      /* slot keys                                          */
    int64_t *lab;      /* slot labels (-1 = buffer)                           */
    int64_t  cmp;      /* merge comparisons                                   */
    int64_t  mov;      /* merge element moves (writes to a different slot)    */
    int      g;        /* data slots per unit                                 */
    /* trace: after every merge, a snapshot of the labels if trace != NULL   */
    int64_t *trace;    /* [max_snap][nslots]                                   */
    int64_t  nslots, nsnap, max_snap;
} frog_model;

static int64_t frog_region(const frog_model *M, int64_t u)
{
    int64_t n = (int64_t)M->g * u;
    return n + n / 2;
}

static void frog_snapshot(frog_model *M)
{
    if (!M->trace || M->nsnap >= M->max_snap) return;
    memcpy(M->trace + M->nsnap * M->nslots, M->lab, (size_t)M->nslots * sizeof(int64_t));
    M->nsnap++;
}

static void frog_put(frog_model *M, int64_t dst, int64_t src)
{
    if (dst != src) {
        M->key[dst] = M->key[src];
        M->lab[dst] = M->lab[src];
        M->mov++;
    }
}

static void frog_left(frog_model *M, int64_t s, int64_t u);
static void frog_right(frog_model *M, int64_t s, int64_t u);

/* A leaf unit: for g = 1 a single element, already in place.  For g = 2 the
   unit is a triplet whose two data slots are sorted to the left (left leaf) or
   to the right (right leaf); its middle slot is the buffer. */
static void frog_leaf(frog_model *M, int64_t s, int left)
{
    if (M->g == 1) return;
    /* setup put the two data elements at s and s+2, buffer at s+1 */
    int64_t a = s, b = s + 2;
    M->cmp++;
    int swap = oracle_less_f64(M->key[b], M->key[a]);
    double ka = M->key[a], kb = M->key[b];
    int64_t la = M->lab[a], lb = M->lab[b];
    if (swap) { double t = ka; ka = kb; kb = t; int64_t tl = la; la = lb; lb = tl; }
    if (left) {   /* data to s, s+1 */
        M->key[s] = ka; M->lab[s] = la; M->key[s + 1] = kb; M->lab[s + 1] = lb;
        M->lab[s + 2] = -1;
    } else {      /* data to s+1, s+2 */
        M->key[s + 1] = ka; M->lab[s + 1] = la; M->key[s + 2] = kb; M->lab[s + 2] = lb;
        M->lab[s] = -1;
    }
    M->mov += 1 + (swap ? 1 : 0);
    frog_snapshot(M);
}

/* Left node over [s, s+region): outer = left child gets ceil(u/2) units. */
static void frog_left(frog_model *M, int64_t s, int64_t u)
{
    if (u == 1) { frog_leaf(M, s, 1); return; }
    int64_t ul = (u + 1) / 2, ur = u / 2;
    int64_t nl = (int64_t)M->g * ul, nr = (int64_t)M->g * ur, n = nl + nr;
    int64_t reg = frog_region(M, u);
    frog_left(M, s, ul);                                   /* L at [s, s+nl)     */
    frog_right(M, s + reg - frog_region(M, ur), ur);       /* R at [s+reg-nr, .) */
    int64_t Lb = s, Rb = s + reg - nr;
    int64_t i = nl - 1, j = nr - 1, w = s + n - 1;
    /* descending: the larger element goes to the top; on a tie the later
       (right-run) element takes the higher slot */
    while (j >= 0) {
        if (i < 0) { frog_put(M, w--, Rb + j); j--; continue; }
        M->cmp++;
        if (oracle_less_f64(M->key[Rb + j], M->key[Lb + i])) { frog_put(M, w--, Lb + i); i--; }
        else                                                 { frog_put(M, w--, Rb + j); j--; }
    }
    /* L's remaining prefix is already in place */
    for (int64_t p = s + n; p < s + reg; p++) M->lab[p] = -1;
    frog_snapshot(M);
}

/* Right node over [s, s+region): outer = right child gets ceil(u/2) units. */
static void frog_right(frog_model *M, int64_t s, int64_t u)
{
    if (u == 1) { frog_leaf(M, s, 0); return; }
    int64_t ul = u / 2, ur = (u + 1) / 2;
    int64_t nl = (int64_t)M->g * ul, nr = (int64_t)M->g * ur, n = nl + nr;
    int64_t reg = frog_region(M, u);
    frog_left(M, s, ul);
    frog_right(M, s + reg - frog_region(M, ur), ur);
    int64_t Lb = s, Rb = s + reg - nr;
    int64_t i = 0, j = 0, w = s + reg - n;
    /* ascending: the smaller element goes to the bottom; on a tie the earlier
       (left-run) element takes the lower slot */
    while (i < nl) {
        if (j >= nr) { frog_put(M, w++, Lb + i); i++; continue; }
        M->cmp++;
        if (oracle_less_f64(M->key[Rb + j], M->key[Lb + i])) { frog_put(M, w++, Rb + j); j++; }
        else                                                 { frog_put(M, w++, Lb + i); i++; }
    }
    for (int64_t p = s; p < s + reg - n; p++) M->lab[p] = -1;
    frog_snapshot(M);
}

/* Setup recursion: place the input elements (in input order) into the leaf
   slots of the frog tree.  For g = 1 a leaf is one slot; for g = 2 a leaf is a
   triplet whose data go to its first and last slot. */
static int64_t frog_setup(frog_model *M, const double *in, int64_t next,
                          int64_t s, int64_t u, int left)
{
    if (u == 1) {
        if (M->g == 1) {
            M->key[s] = in[next]; M->lab[s] = next; return next + 1;
        }
        M->key[s] = in[next]; M->lab[s] = next;
        M->lab[s + 1] = -1;
        M->key[s + 2] = in[next + 1]; M->lab[s + 2] = next + 1;
        return next + 2;
    }
    int64_t ul = left ? (u + 1) / 2 : u / 2;
    int64_t ur = u - ul;
    int64_t reg = frog_region(M, u);
    next = frog_setup(M, in, next, s, ul, 1);
    next = frog_setup(M, in, next, s + reg - frog_region(M, ur), ur, 0);
    return next;
}

/*
 * Run the model on `in[0, g*u)` as a top-level left node.
 *   out_key   : n sorted keys (the data region after the top merge)
 *   out_label : n labels: the input index each output element came from
 *   setup_lab : nslots labels right after setup (may be NULL)
 *   trace     : max_snap x nslots label snapshots after every merge (may be NULL)
 *   counts    : {comparisons, moves, snapshots taken}
 * Returns the number of slots (n + floor(n/2)), or -1 on allocation failure.
 */
int64_t oracle_frog_model(const double *in, int64_t u, int g, double *out_key,
                          int64_t *out_label, int64_t *setup_lab, int64_t *trace,
                          int64_t max_snap, int64_t *counts)
{
    frog_model M;
    memset(&M, 0, sizeof M);
    M.g = g;
    if (u <= 0) { if (counts) counts[0] = counts[1] = counts[2] = 0; return 0; }
    M.nslots = frog_region(&M, u);
    M.key = (double *)calloc((size_t)M.nslots, sizeof(double));
    M.lab = (int64_t *)malloc((size_t)M.nslots * sizeof(int64_t));
    if (!M.key || !M.lab) { free(M.key); free(M.lab); return -1; }
    for (int64_t p = 0; p < M.nslots; p++) M.lab[p] = -1;
    frog_setup(&M, in, 0, 0, u, 1);
    if (setup_lab) memcpy(setup_lab, M.lab, (size_t)M.nslots * sizeof(int64_t));
    M.trace = trace; M.max_snap = max_snap;
    frog_left(&M, 0, u);
    int64_t n = (int64_t)g * u;
    if (out_key) memcpy(out_key, M.key, (size_t)n * sizeof(double));
    if (out_label) memcpy(out_label, M.lab, (size_t)n * sizeof(int64_t));
    if (counts) { counts[0] = M.cmp; counts[1] = M.mov; counts[2] = M.nsnap; }
    int64_t ns = M.nslots;
    free(M.key); free(M.lab);
    return ns;
}

/* Geometry of the Frogsort1 tree (g = 1) walked down to depth `depth`:
   for every node at that depth, in left-to-right order, writes
   {region start, data elements, is_left, data start, input offset}.
   Returns the number of nodes written (2^depth). */
static int64_t frog_geom(int64_t s, int64_t n, int left, int depth, int64_t in_off,
                         int64_t *out, int64_t k)
{
    if (depth == 0) {
        int64_t reg = n + n / 2;
        out[5 * k + 0] = s;
        out[5 * k + 1] = n;
        out[5 * k + 2] = left;
        out[5 * k + 3] = left ? s : s + reg - n;
        out[5 * k + 4] = in_off;
        return k + 1;
    }
    int64_t nl = left ? (n + 1) / 2 : n / 2, nr = n - nl;
    int64_t reg = n + n / 2, regr = nr + nr / 2;
    k = frog_geom(s, nl, 1, depth - 1, in_off, out, k);
    k = frog_geom(s + reg - regr, nr, 0, depth - 1, in_off + nl, out, k);
    return k;
}

int64_t oracle_frog_geometry(int64_t n, int depth, int64_t *out)
{
    return frog_geom(0, n, 1, depth, 0, out, 0);
}

/* ------------------------------------------------------------------------ */
/* instrumented model of Squidsort1 (Frogsort1 + non-overlap test + lazy order) */
/* ------------------------------------------------------------------------ */
/*
 * "Squidsort": Frogsort1 combined with the non-overlap test of "Full
 * adaptivity" (Omitsort: a merge whose two inputs do not overlap is left out)
 * and the data-driven order of Octosort (a run may come back ascending or
 * descending, and the wanted order is enforced lazily).
 *
 * Every node returns the direction of its run: SQ_NONE for a single element,
 * SQ_ASC (the run holds the stable ascending result of the node's input) or
 * SQ_DESC (the run holds that result reversed).  With the two children's
 * ascending views SL and SR (a descending run is read from its end):
 *   - both not descending and SR[0] not less than SL[last]: the node is the
 *     concatenation, ascending; nothing is compared beyond the test and only
 *     the inner run moves (next to the outer one);
 *   - else, both not ascending and SR[last] less than SL[0]: the
 *     concatenation of the two stored runs is the reversed result, so the
 *     node is descending, again moving only the inner run;
 *   - else the node merges.  Its direction is the outer child's (ascending
 *     if that is a single element): the paper enforces the wanted order when
 *     the children's directions differ, but in the frog layout the outer run
 *     lies inside the output, and only a merge in the outer run's own
 *     direction moves its elements away from the side the output is written
 *     from.  The inner run is read in whichever direction the merge needs.
 *     The wanted order is then enforced once, by reversing the whole array if
 *     the top node ends descending.
 * mode 1 enforces ascending at every merge instead (the literal reading);
 * the write check then finds outer elements overwritten before they are read.
 * mode 2 keeps a descending run only through concatenations: before a merge
 * a descending outer run is turned around in place (a reversal within its
 * own slots, counted with the moves), and every merge is ascending -- on a
 * device that pays the same for a move whether or not it compares, this
 * avoids merges that keep a run descending only for the final reversal to
 * turn it around again.
 *
 * Writes go in the frog order (left node top-down, right node bottom-up) and
 * every write is checked: a slot that still holds an element not yet read is
 * a violation (counted; the model carries on).
 */
enum { SQ_NONE = 0, SQ_ASC = 1, SQ_DESC = 2 };

typedef struct {
    double  *key;
    int64_t *lab;
    char    *live;      /* slot holds a run element not yet read */
    int64_t  cmp;       /* merge comparisons                      */
    int64_t  test;      /* non-overlap test comparisons           */
    int64_t  mov;       /* moves of merges and concatenations      */
    int64_t  bad;       /* writes over an element not yet read     */
    int      mode;
} squid_model;

static double sq_view(const squid_model *M, int64_t base, int64_t n, int dir, int64_t i)
{
    return M->key[dir == SQ_DESC ? base + n - 1 - i : base + i];
}

static int64_t sq_slot(int64_t base, int64_t n, int dir, int64_t i)
{
    return dir == SQ_DESC ? base + n - 1 - i : base + i;
}

static void sq_put(squid_model *M, int64_t dst, int64_t src)
{
    M->live[src] = 0;                   /* read first: a run element may stay */
    if (M->live[dst]) M->bad++;
    if (dst != src) {
        M->key[dst] = M->key[src];
        M->lab[dst] = M->lab[src];
        M->mov++;
    }
}

static int squid_node(squid_model *M, int64_t s, int64_t n, int left)
{
    if (n == 1) return SQ_NONE;
    const int64_t nl = left ? (n + 1) / 2 : n / 2, nr = n - nl;
    const int64_t reg = n + n / 2;
    const int dL = squid_node(M, s, nl, 1);
    const int dR = squid_node(M, s + reg - (nr + nr / 2), nr, 0);
    const int64_t Lb = s, Rb = s + reg - nr, out0 = left ? s : s + reg - n;
    for (int64_t p = Lb; p < Lb + nl; p++) M->live[p] = 1;
    for (int64_t p = Rb; p < Rb + nr; p++) M->live[p] = 1;
    int dir = SQ_ASC, concat = 0;
    if (dL != SQ_DESC && dR != SQ_DESC) {
        M->test++;
        if (!oracle_less_f64(sq_view(M, Rb, nr, dR, 0), sq_view(M, Lb, nl, dL, nl - 1))) concat = 1;
    }
    if (!concat && dL != SQ_ASC && dR != SQ_ASC) {
        M->test++;
        if (oracle_less_f64(sq_view(M, Rb, nr, dR, nr - 1), sq_view(M, Lb, nl, dL, 0))) {
            concat = 1;
            dir = SQ_DESC;
        }
    }
    if (concat) {
        /* the stored runs side by side: the outer one stays, the inner moves */
        if (left) for (int64_t j = nr - 1; j >= 0; j--) sq_put(M, s + nl + j, Rb + j);
        else      for (int64_t i = 0; i < nl; i++) sq_put(M, out0 + i, Lb + i);
        for (int64_t p = Lb; p < Lb + nl; p++) M->live[p] = 0;
        for (int64_t p = Rb; p < Rb + nr; p++) M->live[p] = 0;
        return dir;
    }
    int douter = left ? dL : dR;
    int dLm = dL, dRm = dR;
    if (M->mode == 2 && douter == SQ_DESC) {
        /* turn the outer run around in its own slots */
        const int64_t x0 = left ? Lb : Rb, nx = left ? nl : nr;
        for (int64_t a = x0, b = x0 + nx - 1; a < b; a++, b--) {
            double tk = M->key[a]; M->key[a] = M->key[b]; M->key[b] = tk;
            int64_t tl = M->lab[a]; M->lab[a] = M->lab[b]; M->lab[b] = tl;
            M->mov += 2;
        }
        if (left) dLm = SQ_ASC; else dRm = SQ_ASC;
        douter = SQ_ASC;
    }
    dir = (M->mode == 0 && douter == SQ_DESC) ? SQ_DESC : SQ_ASC;
    /* The stable ascending merge M of SL and SR takes SL first on ties; slot
       out0+k receives M[k] (ascending) or M[n-1-k] (descending).  The write
       order decides which end of M is produced first. */
    const int smallest_first = left ? (dir == SQ_DESC) : (dir == SQ_ASC);
    int64_t i, j, ie, je, step;
    if (smallest_first) { i = 0; j = 0; ie = nl; je = nr; step = 1; }
    else                { i = nl - 1; j = nr - 1; ie = -1; je = -1; step = -1; }
    for (int64_t k = 0; k < n; k++) {
        int takeL;
        if (i == ie) takeL = 0;
        else if (j == je) takeL = 1;
        else {
            M->cmp++;
            const double a = sq_view(M, Lb, nl, dLm, i), b = sq_view(M, Rb, nr, dRm, j);
            /* from the small end L wins ties; from the large end R's tied
               elements come out first (they follow L's in M) */
            takeL = smallest_first ? !oracle_less_f64(b, a) : oracle_less_f64(b, a);
        }
        const int64_t mpos = smallest_first ? k : n - 1 - k;           /* position in M */
        const int64_t w = (dir == SQ_ASC) ? out0 + mpos : out0 + (n - 1 - mpos);
        const int64_t src = takeL ? sq_slot(Lb, nl, dLm, i) : sq_slot(Rb, nr, dRm, j);
        sq_put(M, w, src);
        if (takeL) i += step; else j += step;
    }
    for (int64_t p = Lb; p < Lb + nl; p++) M->live[p] = 0;
    for (int64_t p = Rb; p < Rb + nr; p++) M->live[p] = 0;
    return dir;
}

/*
 * Run the Squidsort1 model on in[0, n) (elements placed by the Frogsort1 setup
 * recursion, one element per leaf).  mode 0: the reading above; mode 1:
 * ascending enforced at every merge; mode 2: descending outer runs turned
 * around before their merge.
 *   out_key, out_label: the n results and the input index of each (after the
 *                       final reversal when the top node is descending)
 *   counts: {merge comparisons, test comparisons, merge and concatenation
 *            moves, final-reversal moves, direction of the top node,
 *            overwrites of unread elements}
 * Returns the number of slots, or -1 on allocation failure.
 */
int64_t oracle_squid_model(const double *in, int64_t n, int mode, double *out_key, int64_t *out_label,
                           int64_t *counts)
{
    for (int c = 0; c < 6; c++) counts[c] = 0;
    if (n <= 0) return 0;
    frog_model F;
    memset(&F, 0, sizeof F);
    F.g = 1;
    F.nslots = frog_region(&F, n);
    F.key = (double *)calloc((size_t)F.nslots, sizeof(double));
    F.lab = (int64_t *)malloc((size_t)F.nslots * sizeof(int64_t));
    char *live = (char *)calloc((size_t)F.nslots, 1);
    if (!F.key || !F.lab || !live) { free(F.key); free(F.lab); free(live); return -1; }
    for (int64_t p = 0; p < F.nslots; p++) F.lab[p] = -1;
    frog_setup(&F, in, 0, 0, n, 1);
    squid_model M;
    memset(&M, 0, sizeof M);
    M.key = F.key; M.lab = F.lab; M.live = live; M.mode = mode;
    const int dir = squid_node(&M, 0, n, 1);
    int64_t rev = 0;
    if (dir == SQ_DESC) {
        for (int64_t a = 0, b = n - 1; a < b; a++, b--) {
            double tk = M.key[a]; M.key[a] = M.key[b]; M.key[b] = tk;
            int64_t tl = M.lab[a]; M.lab[a] = M.lab[b]; M.lab[b] = tl;
            rev += 2;
        }
    }
    if (out_key) memcpy(out_key, M.key, (size_t)n * sizeof(double));
    if (out_label) memcpy(out_label, M.lab, (size_t)n * sizeof(int64_t));
    counts[0] = M.cmp; counts[1] = M.test; counts[2] = M.mov; counts[3] = rev;
    counts[4] = dir; counts[5] = M.bad;
    int64_t ns = F.nslots;
    free(F.key); free(F.lab); free(live);
    return ns;
}

/* ------------------------------------------------------------------------ */
/* instrumented model of Frogsort2 (imbalanced split, smaller buffer)        */
/* ------------------------------------------------------------------------ */
/*
 * "Frogsort2": the inner child of every node takes a fraction p of the node's
 * elements, and symmetric merging then needs a buffer of only that fraction.
 * Here p = q / 65536 for an integer q in [1, 32768]: a node of n elements has
 * an inner child of floor(q*n/65536) elements, an outer child with the rest,
 * and a region of n + floor(q*n/65536) slots.  A split is only defined when the
 * inner child is not empty; the model reports a node where it would be.  The
 * children sit as in Frogsort1 (the left child is a left node at the start of
 * the region, the right child a right node at its end; the outer child is the
 * left child of a left node and the right child of a right node), and merging
 * runs from the runs' inner ends outward.  Nodes of at most leaf_max elements
 * are leaves: the setup recursion copies their chunk of the input (in input
 * order) to their data slots, at the left end of the region for a left leaf and
 * at the right end for a right leaf, where a stable insertion sort orders them.
 * With q = 32768 and leaf_max = 1 this is the Frogsort1 model above, step for
 * step (the paper notes Frogsort1 is Frogsort2 with p = 0.5).
 *
 * The model checks that the buffer suffices: a write to a slot that still holds
 * an element nobody has read sets bit 0 of `bad`; an empty inner child sets
 * bit 1.  gap_shrink > 0 shrinks every region by that many slots (only so that a
 * test can see the check fire).
 *
 * With in == NULL only the geometry is walked (no slots are allocated).
 */
typedef struct {
    double  *key;
    int64_t *lab;
    int64_t  q, leaf_max, gap_shrink;
    int64_t  cmp, mov, bad;
    int64_t *trace;
    int64_t  nslots, nsnap, max_snap;
    int64_t *leaves, max_leaves, nleaves;   /* {input offset, data start, len}      */
    int64_t *nodes, max_nodes, nnodes;      /* {region start, n, is_left, height}   */
} frog2_model;

static int64_t f2_inner(const frog2_model *M, int64_t n) { return n * M->q / 65536; }

static int64_t f2_region(const frog2_model *M, int64_t n)
{
    int64_t r = n + f2_inner(M, n) - M->gap_shrink;
    return r < n ? n : r;
}

static void f2_snapshot(frog2_model *M)
{
    if (!M->key || !M->trace || M->nsnap >= M->max_snap) return;
    memcpy(M->trace + M->nsnap * M->nslots, M->lab, (size_t)M->nslots * sizeof(int64_t));
    M->nsnap++;
}

/* Move the element in slot src to slot dst: src becomes free, and dst must
   not hold an element that has not been read yet. */
static void f2_put(frog2_model *M, int64_t dst, int64_t src)
{
    if (dst == src) return;
    double k = M->key[src];
    int64_t l = M->lab[src];
    M->lab[src] = -1;
    if (M->lab[dst] >= 0) M->bad |= 1;
    M->key[dst] = k;
    M->lab[dst] = l;
    M->mov++;
}

/* Setup: place the input chunk of every leaf (in input order) at its data
   slots and sort it there.  Returns the next input position. */
static int64_t f2_setup(frog2_model *M, const double *in, int64_t next, int64_t s, int64_t n, int left)
{
    if (n <= M->leaf_max) {
        int64_t d = left ? s : s + f2_region(M, n) - n;
        if (M->nleaves < M->max_leaves) {
            M->leaves[3 * M->nleaves + 0] = next;
            M->leaves[3 * M->nleaves + 1] = d;
            M->leaves[3 * M->nleaves + 2] = n;
        }
        M->nleaves++;
        if (M->key) {
            for (int64_t i = 0; i < n; i++) {
                if (M->lab[d + i] >= 0) M->bad |= 1;
                M->key[d + i] = in[next + i];
                M->lab[d + i] = next + i;
            }
            /* stable insertion sort: an element moves below another only
               if it is strictly smaller */
            for (int64_t i = 1; i < n; i++) {
                double k = M->key[d + i];
                int64_t l = M->lab[d + i], j = i - 1;
                while (j >= 0 && oracle_less_f64(k, M->key[d + j])) {
                    M->key[d + j + 1] = M->key[d + j];
                    M->lab[d + j + 1] = M->lab[d + j];
                    j--;
                }
                M->key[d + j + 1] = k;
                M->lab[d + j + 1] = l;
            }
        }
        return next + n;
    }
    int64_t ni = f2_inner(M, n);
    if (ni < 1) { M->bad |= 2; return next + n; }
    int64_t nl = left ? n - ni : ni, nr = n - nl;
    next = f2_setup(M, in, next, s, nl, 1);
    next = f2_setup(M, in, next, s + f2_region(M, n) - f2_region(M, nr), nr, 0);
    return next;
}

/* Merge recursion over a node placed by f2_setup; returns the node's height
   (0 for a leaf). */
static int64_t f2_node(frog2_model *M, int64_t s, int64_t n, int left)
{
    if (n <= M->leaf_max) return 0;
    int64_t ni = f2_inner(M, n);
    if (ni < 1) { M->bad |= 2; return 0; }
    int64_t nl = left ? n - ni : ni, nr = n - nl;
    int64_t reg = f2_region(M, n);
    int64_t hl = f2_node(M, s, nl, 1);
    int64_t hr = f2_node(M, s + reg - f2_region(M, nr), nr, 0);
    int64_t h = 1 + (hl > hr ? hl : hr);
    if (M->key) {
        int64_t Lb = s, Rb = s + reg - nr;
        if (left) {
            /* descending from the top slot of the output; on a tie the
               right-run element takes the higher slot */
            int64_t i = nl - 1, j = nr - 1, w = s + n - 1;
            while (j >= 0) {
                if (i < 0) { f2_put(M, w--, Rb + j); j--; continue; }
                M->cmp++;
                if (oracle_less_f64(M->key[Rb + j], M->key[Lb + i])) { f2_put(M, w--, Lb + i); i--; }
                else                                                 { f2_put(M, w--, Rb + j); j--; }
            }
        } else {
            /* ascending from the bottom slot of the output; on a tie the
               left-run element takes the lower slot */
            int64_t i = 0, j = 0, w = s + reg - n;
            while (i < nl) {
                if (j >= nr) { f2_put(M, w++, Lb + i); i++; continue; }
                M->cmp++;
                if (oracle_less_f64(M->key[Rb + j], M->key[Lb + i])) { f2_put(M, w++, Rb + j); j++; }
                else                                                 { f2_put(M, w++, Lb + i); i++; }
            }
        }
        f2_snapshot(M);
    }
    if (M->nnodes < M->max_nodes) {
        M->nodes[4 * M->nnodes + 0] = s;
        M->nodes[4 * M->nnodes + 1] = n;
        M->nodes[4 * M->nnodes + 2] = left;
        M->nodes[4 * M->nnodes + 3] = h;
    }
    M->nnodes++;
    return h;
}

/*
 * Run the model on in[0, n) as a top-level left node (in may be NULL: geometry
 * only).  Outputs as for oracle_frog_model, plus the leaves in input order and
 * the merge nodes in post order (each array written up to its capacity).
 *   counts: {comparisons, moves, snapshots, leaves, nodes, bad}
 * Returns the number of slots, n + floor(q*n/65536) (minus gap_shrink), or -1
 * on allocation failure.
 */
int64_t oracle_frog2_model(const double *in, int64_t n, int64_t q, int64_t leaf_max, int64_t gap_shrink,
                           double *out_key, int64_t *out_label, int64_t *setup_lab,
                           int64_t *trace, int64_t max_snap,
                           int64_t *leaves, int64_t max_leaves, int64_t *nodes, int64_t max_nodes,
                           int64_t *counts)
{
    frog2_model M;
    memset(&M, 0, sizeof M);
    M.q = q;
    M.leaf_max = leaf_max < 1 ? 1 : leaf_max;
    M.gap_shrink = gap_shrink;
    M.leaves = leaves; M.max_leaves = leaves ? max_leaves : 0;
    M.nodes = nodes;   M.max_nodes = nodes ? max_nodes : 0;
    for (int i = 0; i < 6; i++) counts[i] = 0;
    if (n <= 0) return 0;
    M.nslots = f2_region(&M, n);
    if (in) {
        M.key = (double *)calloc((size_t)M.nslots, sizeof(double));
        M.lab = (int64_t *)malloc((size_t)M.nslots * sizeof(int64_t));
        if (!M.key || !M.lab) { free(M.key); free(M.lab); return -1; }
        for (int64_t p = 0; p < M.nslots; p++) M.lab[p] = -1;
    }
    f2_setup(&M, in, 0, 0, n, 1);
    if (in && setup_lab) memcpy(setup_lab, M.lab, (size_t)M.nslots * sizeof(int64_t));
    M.trace = trace; M.max_snap = max_snap;
    f2_node(&M, 0, n, 1);
    if (in) {
        if (out_key) memcpy(out_key, M.key, (size_t)n * sizeof(double));
        if (out_label) memcpy(out_label, M.lab, (size_t)n * sizeof(int64_t));
    }
    counts[0] = M.cmp; counts[1] = M.mov; counts[2] = M.nsnap;
    counts[3] = M.nleaves; counts[4] = M.nnodes; counts[5] = M.bad;
    int64_t ns = M.nslots;
    free(M.key); free(M.lab);
    return ns;
}

/* ------------------------------------------------------------------------ */
/* instrumented model of Frogsort3 / Frogsort6 (one buffer shared in turn)   */
/* ------------------------------------------------------------------------ */
/*
 * "Frogsort3 and 6": Frogsort3, instead of splitting the buffer between the
 * two branches, lets the whole buffer serve one branch after the other, and a
 * branch switches to Frogsort1 once the buffer is at least half its size;
 * Frogsort6 does the
 * same but switches to Frogsort2 (inner fraction p2) once that fits; Frogsort1,
 * 2 and 3 are its special cases.  Reading: the input sits in slots [0, n), the
 * buffer is b = floor(q*n/65536) slots [n, n+b), and the sub-trees are
 * Frogsort2 trees with inner child floor(q2*m/65536) (q2 = 32768: Frogsort1,
 * i.e. Frogsort3).  A node of m elements over slots [0, m + b) whose sub-tree
 * would need more than b (floor(q2*m/65536) > b) splits into an inner child of
 * b elements (its last b input elements) and an outer child of m - b.  The
 * inner child is sorted first, by a sub-tree whose root is a right node with
 * its region ending at slot m + b, so its data end at [m, m + b) (its setup
 * moves its chunk there; the space it passes through is free).  The outer
 * child is then the same problem on m - b elements over [0, m), and the node
 * finishes with a left-node merge of [0, m-b) and [m, m+b) into [0, m),
 * written from the top.  A node whose sub-tree fits the buffer is one sub-tree
 * over [0, m + floor(q2*m/65536)), and so is a node of at most leaf_max
 * elements: that tree is a single leaf, sorted where it lies, which needs no
 * buffer at all.
 *
 * Every placement and merge write is checked as in the Frogsort2 model (bit 0
 * of `bad`; bit 1: an empty buffer where the node still has to split).
 * gap_shrink > 0 ends every inner child that many slots early, so a test can
 * see the check fire.
 */
static int64_t f3_r1(const frog2_model *M, int64_t m) { return m + f2_inner(M, m); }

/* In-place setup of a sub-tree over [s, s + f3_r1(n)) whose input sits at
   [c, c + n): leaves from right to left, each chunk moved from its top
   element down (every destination is at or after its source), then sorted
   in place. */
static void f3_place(frog2_model *M, int64_t s, int64_t n, int64_t c, int left)
{
    if (n <= M->leaf_max) {
        int64_t d = left ? s : s + f3_r1(M, n) - n;
        if (M->nleaves < M->max_leaves) {
            M->leaves[3 * M->nleaves + 0] = c;
            M->leaves[3 * M->nleaves + 1] = d;
            M->leaves[3 * M->nleaves + 2] = n;
        }
        M->nleaves++;
        if (!M->key) return;
        int64_t mov = M->mov;
        for (int64_t i = n - 1; i >= 0; i--) f2_put(M, d + i, c + i);
        M->mov = mov;                        /* placement is not counted as merge moves */
        for (int64_t i = 1; i < n; i++) {
            double k = M->key[d + i];
            int64_t l = M->lab[d + i], j = i - 1;
            while (j >= 0 && oracle_less_f64(k, M->key[d + j])) {
                M->key[d + j + 1] = M->key[d + j];
                M->lab[d + j + 1] = M->lab[d + j];
                j--;
            }
            M->key[d + j + 1] = k;
            M->lab[d + j + 1] = l;
        }
        return;
    }
    int64_t ni = f2_inner(M, n);
    if (ni < 1) { M->bad |= 2; return; }
    int64_t nl = left ? n - ni : ni, nr = n - nl;
    f3_place(M, s + f3_r1(M, n) - f3_r1(M, nr), nr, c + nl, 0);
    f3_place(M, s, nl, c, 1);
}

/* The spine: a node of m elements over [0, m + b).  spine[] receives
   {outer elements, inner start, inner elements} of every spine merge, bottom
   up; tree[] {region start, elements, input offset, is_left} of every
   sub-tree in the order they run. */
typedef struct {
    int64_t *spine, max_spine, nspine;
    int64_t *tree, max_tree, ntree;
    int64_t shrink;
} frog3_sched;

static void f3_tree(frog2_model *M, frog3_sched *S, int64_t s, int64_t n, int64_t c, int left)
{
    if (S->ntree < S->max_tree) {
        S->tree[4 * S->ntree + 0] = s;
        S->tree[4 * S->ntree + 1] = n;
        S->tree[4 * S->ntree + 2] = c;
        S->tree[4 * S->ntree + 3] = left;
    }
    S->ntree++;
    f3_place(M, s, n, c, left);
    f2_node(M, s, n, left);
}

static void f3_node(frog2_model *M, frog3_sched *S, int64_t m, int64_t b)
{
    if (f2_inner(M, m) <= b || m <= M->leaf_max) { f3_tree(M, S, 0, m, 0, 1); return; }
    if (b < 1) { M->bad |= 2; return; }              /* no buffer to share */
    int64_t end = m + b - S->shrink;                 /* the inner child's region end */
    f3_tree(M, S, end - f3_r1(M, b), b, m - b, 0);
    f3_node(M, S, m - b, b);
    int64_t nl = m - b, nr = b, Lb = 0, Rb = end - b;
    int64_t i = nl - 1, j = nr - 1, w = m - 1;
    while (M->key && j >= 0) {
        if (i < 0) { f2_put(M, w--, Rb + j); j--; continue; }
        M->cmp++;
        if (oracle_less_f64(M->key[Rb + j], M->key[Lb + i])) { f2_put(M, w--, Lb + i); i--; }
        else                                                 { f2_put(M, w--, Rb + j); j--; }
    }
    if (S->nspine < S->max_spine) {
        S->spine[3 * S->nspine + 0] = nl;
        S->spine[3 * S->nspine + 1] = Rb;
        S->spine[3 * S->nspine + 2] = nr;
    }
    S->nspine++;
}

/*
 * Run the model on in[0, n) (in == NULL: geometry only); q2 = 32768 is
 * Frogsort3.  Outputs as for oracle_frog2_model, plus the spine merges and the
 * sub-trees.
 *   counts: {comparisons, moves, leaves, nodes, bad, spine merges, trees}
 * Returns the number of slots, n + min(b, the whole tree's buffer), or -1 on
 * allocation failure.
 */
int64_t oracle_frog3_model(const double *in, int64_t n, int64_t q, int64_t q2, int64_t leaf_max, int64_t gap_shrink,
                           double *out_key, int64_t *out_label,
                           int64_t *leaves, int64_t max_leaves, int64_t *nodes, int64_t max_nodes,
                           int64_t *spine, int64_t max_spine, int64_t *tree, int64_t max_tree,
                           int64_t *counts)
{
    frog2_model M;
    frog3_sched S;
    memset(&M, 0, sizeof M);
    memset(&S, 0, sizeof S);
    for (int i = 0; i < 7; i++) counts[i] = 0;
    if (n <= 0) return 0;
    int64_t b = n * q / 65536;
    M.q = q2;                                        /* the sub-trees' split */
    M.leaf_max = leaf_max < 1 ? 1 : leaf_max;
    M.leaves = leaves; M.max_leaves = leaves ? max_leaves : 0;
    M.nodes = nodes;   M.max_nodes = nodes ? max_nodes : 0;
    S.spine = spine;   S.max_spine = spine ? max_spine : 0;
    S.tree = tree;     S.max_tree = tree ? max_tree : 0;
    S.shrink = gap_shrink;
    M.nslots = n + (f2_inner(&M, n) <= b ? f2_inner(&M, n) : b);
    if (in) {
        M.key = (double *)calloc((size_t)M.nslots, sizeof(double));
        M.lab = (int64_t *)malloc((size_t)M.nslots * sizeof(int64_t));
        if (!M.key || !M.lab) { free(M.key); free(M.lab); return -1; }
        for (int64_t p = 0; p < M.nslots; p++) M.lab[p] = -1;
        for (int64_t p = 0; p < n; p++) { M.key[p] = in[p]; M.lab[p] = p; }
    }
    f3_node(&M, &S, n, b);
    if (in && out_key) memcpy(out_key, M.key, (size_t)n * sizeof(double));
    if (in && out_label) memcpy(out_label, M.lab, (size_t)n * sizeof(int64_t));
    counts[0] = M.cmp; counts[1] = M.mov; counts[2] = M.nleaves; counts[3] = M.nnodes;
    counts[4] = M.bad; counts[5] = S.nspine; counts[6] = S.ntree;
    int64_t ns = M.nslots;
    free(M.key); free(M.lab);
    return ns;
}

/* ------------------------------------------------------------------------ */
/* fp64 reference for the 1-64-64-1 ReLU network (learned bucket path)       */
/* ------------------------------------------------------------------------ */
/*
 * Parameter vector layout (4353 values), for hidden width H = 64:
 *   W1[H]      first layer weights (input is a scalar)
 *   b1[H]
 *   W2[H*H]    row-major: W2[i*H + j] multiplies hidden-1 unit j into unit i
 *   b2[H]
 *   w3[H]
 *   b3[1]
 * y(u) = w3 . relu(W2 relu(W1 u + b1) + b2) + b3
 * loss = mean over the batch of (y - t)^2
 */
#define MLP_H 64
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + MLP_H)
#define OFF_W2 (OFF_B1 + MLP_H)
#define OFF_B2 (OFF_W2 + MLP_H * MLP_H)
#define OFF_W3 (OFF_B2 + MLP_H)
#define OFF_B3 (OFF_W3 + MLP_H)
#define MLP_NP (OFF_B3 + 1)

int oracle_mlp_num_params(void) { return MLP_NP; }

static double relu(double v) { return v > 0.0 ? v : 0.0; }

void oracle_mlp_forward(const double *p, const double *u, int64_t B, double *y)
{
    double h1[MLP_H], h2[MLP_H];
    for (int64_t b = 0; b < B; b++) {
        for (int i = 0; i < MLP_H; i++) h1[i] = relu(p[OFF_W1 + i] * u[b] + p[OFF_B1 + i]);
        for (int i = 0; i < MLP_H; i++) {
            double a = p[OFF_B2 + i];
            for (int j = 0; j < MLP_H; j++) a += p[OFF_W2 + i * MLP_H + j] * h1[j];
            h2[i] = relu(a);
        }
        double out = p[OFF_B3];
        for (int i = 0; i < MLP_H; i++) out += p[OFF_W3 + i] * h2[i];
        y[b] = out;
    }
}

/* Loss and its gradient with respect to every parameter (same layout).
   ReLU'(0) is taken as 0. */
double oracle_mlp_loss_grad(const double *p, const double *u, const double *t,
                            int64_t B, double *grad)
{
    double h1[MLP_H], z1[MLP_H], h2[MLP_H], z2[MLP_H], g2[MLP_H], g1[MLP_H];
    double loss = 0.0;
    if (grad) for (int k = 0; k < MLP_NP; k++) grad[k] = 0.0;
    for (int64_t b = 0; b < B; b++) {
        for (int i = 0; i < MLP_H; i++) {
            z1[i] = p[OFF_W1 + i] * u[b] + p[OFF_B1 + i];
            h1[i] = relu(z1[i]);
        }
        for (int i = 0; i < MLP_H; i++) {
            double a = p[OFF_B2 + i];
            for (int j = 0; j < MLP_H; j++) a += p[OFF_W2 + i * MLP_H + j] * h1[j];
            z2[i] = a;
            h2[i] = relu(a);
        }
        double y = p[OFF_B3];
        for (int i = 0; i < MLP_H; i++) y += p[OFF_W3 + i] * h2[i];
        double r = y - t[b];
        loss += r * r;
        if (!grad) continue;
        double dy = 2.0 * r / (double)B;
        grad[OFF_B3] += dy;
        for (int i = 0; i < MLP_H; i++) {
            grad[OFF_W3 + i] += dy * h2[i];
            g2[i] = (z2[i] > 0.0) ? dy * p[OFF_W3 + i] : 0.0;   /* d loss / d z2 */
        }
        for (int j = 0; j < MLP_H; j++) g1[j] = 0.0;
        for (int i = 0; i < MLP_H; i++) {
            grad[OFF_B2 + i] += g2[i];
            for (int j = 0; j < MLP_H; j++) {
                grad[OFF_W2 + i * MLP_H + j] += g2[i] * h1[j];
                g1[j] += p[OFF_W2 + i * MLP_H + j] * g2[i];
            }
        }
        for (int j = 0; j < MLP_H; j++) {
            double d = (z1[j] > 0.0) ? g1[j] : 0.0;               /* d loss / d z1 */
            grad[OFF_B1 + j] += d;
            grad[OFF_W1 + j] += d * u[b];
        }
    }
    return loss / (double)B;
}

/* One Adam step (Kingma & Ba 2015) at step number `step` (1-based). */
void oracle_adam_step(double *p, const double *g, double *m, double *v, int64_t np,
                      int64_t step, double lr, double beta1, double beta2, double eps)
{
    double c1 = 1.0 - pow(beta1, (double)step);
    double c2 = 1.0 - pow(beta2, (double)step);
    for (int64_t k = 0; k < np; k++) {
        m[k] = beta1 * m[k] + (1.0 - beta1) * g[k];
        v[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k];
        double mh = m[k] / c1, vh = v[k] / c2;
        p[k] -= lr * mh / (sqrt(vh) + eps);
    }
}
