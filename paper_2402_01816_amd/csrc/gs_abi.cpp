// C ABI of libgs.so: argument checks, workspace accounting, dispatch, reports.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gs.h"
#include "frog_geometry.h"
#include "gs_internal.h"
#include "gs_learned.h"
#include "gs_mlp.h"

namespace {

thread_local std::string g_detail = "";

gs_status fail(gs_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
gs_status fail(gs_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_detail = buf;
    return s;
}

gs_status hip_fail(hipError_t e, const char *where)
{
    return fail(GS_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

// 0 if a HIP device is visible
gs_status check_device()
{
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return fail(GS_ENODEVICE, "no HIP device visible (%s)",
                    e == hipSuccess ? "count is 0" : hipGetErrorString(e));
    }
    return GS_OK;
}

// Which tree a call runs.  buffer_fraction >= 0.5 with GS_ALGO_AUTO (or
// GS_ALGO_FROGSORT1): Frogsort1, buffer floor(n/2).  Below 0.5 the fraction is
// rounded down to q / 2^16 (so the buffer never exceeds it) and AUTO runs
// Frogsort3, the faster of the small-buffer trees on this device; Frogsort2,
// Frogsort3 and Frogsort6 can be asked for by name (at a fraction >= 0.5 they
// run with q = 2^15).  Frogsort6's sub-tree fraction is rounded the same way
// into q2 (2^15 at >= 0.5: Frogsort3).  Below 1/64 the trees grow too deep to
// be worth running.
constexpr int kAutoSmallBuffer = gs::kAlgoFrog3;

gs_status fraction_q(double f, const char *what, int64_t *q)
{
    if (!(f > 0.0)) return fail(GS_EINVAL, "%s must be > 0 (got %g)", what, f);
    const int64_t v = f >= 0.5 ? 32768 : (int64_t)floor(f * 65536.0);
    if (v < gs::kF2MinQ) return fail(GS_EUNSUPPORTED, "%s %g is below the smallest supported, 1/64", what, f);
    *q = v;
    return GS_OK;
}

gs_status resolve_algo(double f, int algo, double sub, int *out, int64_t *q, int64_t *q2)
{
    *q = 0;
    *q2 = 32768;
    *out = gs::kAlgoFrog1;
    if (algo < GS_ALGO_AUTO || algo > GS_ALGO_FROGSORT6) return fail(GS_EINVAL, "unknown algorithm %d", algo);
    if (!(f > 0.0)) return fail(GS_EINVAL, "buffer_fraction must be > 0 (got %g)", f);
    if (algo == GS_ALGO_FROGSORT1 || (algo == GS_ALGO_AUTO && f >= 0.5)) {
        if (f < 0.5) return fail(GS_EINVAL, "Frogsort1 needs buffer_fraction >= 0.5 (got %g)", f);
        return GS_OK;
    }
    gs_status s = fraction_q(f, "buffer_fraction", q);
    if (s != GS_OK) return s;
    if (algo == GS_ALGO_FROGSORT6 && (s = fraction_q(sub, "sub_fraction", q2)) != GS_OK) return s;
    *out = algo == GS_ALGO_FROGSORT2 ? gs::kAlgoFrog2 : algo == GS_ALGO_AUTO ? kAutoSmallBuffer : gs::kAlgoFrog3;
    return GS_OK;
}

// The segmented sort's buffer: q = 0 at buffer_fraction >= 0.5 (Frogsort1 on
// every segment in one pass); below, q/2^16 and the plain sort's algorithm
// for a segment sorted alone.
struct SegFraction {
    int64_t q = 0, q2 = 32768;
    int algo = gs::kAlgoFrog1;
};
gs_status seg_fraction(double f, SegFraction *out)
{
    return resolve_algo(f, GS_ALGO_AUTO, 0.5, &out->algo, &out->q, &out->q2);
}

// A Frogsort2 call copies its host-built tree tables into the workspace, which
// a graph capture cannot record safely.
gs_status check_not_capturing(hipStream_t st)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return GS_OK;
    }
    if (cs != hipStreamCaptureStatusNone)
        return fail(GS_EUNSUPPORTED, "buffer_fraction < 0.5 cannot be captured into a graph");
    return GS_OK;
}

bool aligned256(const void *p) { return ((uintptr_t)p & 255u) == 0; }

// Optional timing/report around an asynchronous body.
struct Reporter {
    gs_report *rep;
    hipStream_t st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    Reporter(gs_report *r, hipStream_t s) : rep(r), st(s)
    {
        if (!rep) return;
        memset(rep, 0, sizeof *rep);
        if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess)
            (void)hipEventRecord(e0, st);
    }
    gs_status finish(gs_status s)
    {
        if (!rep) return s;
        if (e1) (void)hipEventRecord(e1, st);
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess && s == GS_OK) s = hip_fail(e, "hipStreamSynchronize");
        float ms = 0.f;
        if (e0 && e1 && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) rep->elapsed_ms = ms;
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        return s;
    }
};

// Reads the kernels' error word (a bounded wait that gave up, or a work
// capacity exceeded) of a forest control block after the stream is
// synchronised.
gs_status check_err_word(const char *ctrl)
{
    unsigned w = 0;
    hipError_t e = hipMemcpy(&w, ctrl + 4 * gs::kErrWord, 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "reading the error word");
    if (w) return fail(GS_EDEVICE, "a bounded device wait gave up or a work capacity was exceeded");
    return GS_OK;
}

gs_status check_err_word(const char *ws, const gs::SortPlan &p)
{
    return check_err_word(ws + p.off_forest + p.forest.off_ctrl);
}

// The order check's decision of a plain sort and the call's element moves,
// after the stream is synchronised (target: the extra reversal of the
// right-anchored targets).
gs_status read_order(const char *ws, const gs::SortPlan &p, int64_t n, int target, gs_report *rep)
{
    unsigned w = 0;
    uint64_t moved = 0;
    hipError_t e = hipMemcpy(&w, ws + p.off_order, 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess)
        e = hipMemcpy(&moved, ws + p.off_forest + p.forest.off_ctrl + 4 * gs::kMovedWord, 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "reading the order word");
    const uint64_t rev = (uint64_t)(n - (n & 1));
    rep->order = w;
    rep->keys_moved = (w == gs::ORD_IN_ORDER ? 0 : w == gs::ORD_REVERSED ? rev : moved) +
                      ((target == GS_ASC_RIGHT || target == GS_DESC_RIGHT) ? rev : 0);
    return GS_OK;
}

struct TraceRec {
    int kind;
    hipEvent_t a, b;
};
thread_local int g_trace = 0;          // 0 off, 1 every launch, 2 merge launches only
thread_local bool g_open = false;      // a record waits for its end event
thread_local std::vector<TraceRec> g_recs;

}  // namespace

namespace gs {
bool trace_on() { return g_trace != 0; }
// Timing-only events: without the system-scope fence an event record would
// write back and invalidate the caches between the launches it brackets,
// slowing the work it measures.
void trace_begin(int kind, hipStream_t st)
{
    g_open = false;
    if (g_trace == 2 && kind != TK_MERGE) return;
    TraceRec r{kind, nullptr, nullptr};
    if (hipEventCreateWithFlags(&r.a, hipEventDisableSystemFence) != hipSuccess ||
        hipEventCreateWithFlags(&r.b, hipEventDisableSystemFence) != hipSuccess)
        return;
    (void)hipEventRecord(r.a, st);
    g_recs.push_back(r);
    g_open = true;
}
void trace_end(hipStream_t st)
{
    if (g_open && !g_recs.empty()) (void)hipEventRecord(g_recs.back().b, st);
    g_open = false;
}
}  // namespace gs

extern "C" {

int gs_trace_enable(int on)
{
    const int was = g_trace;
    g_trace = on == 2 ? 2 : on != 0 ? 1 : 0;
    return was;
}

gs_status gs_copy_f64(const double *src, double *dst, int64_t n, void *hip_stream)
{
    g_detail.clear();
    if (n < 0) return fail(GS_EINVAL, "n < 0");
    if (n == 0) return GS_OK;
    if (!src || !dst) return fail(GS_EINVAL, "src or dst is NULL");
    gs_status s = check_device();
    if (s != GS_OK) return s;
    hipError_t e = gs::copy_f64_async(src, dst, n, (hipStream_t)hip_stream);
    return e == hipSuccess ? GS_OK : hip_fail(e, "gs_copy_f64 launch");
}

int gs_trace_read(int *kinds, double *ms, int max)
{
    int k = 0;
    for (auto &r : g_recs) {
        float t = 0.f;
        (void)hipEventSynchronize(r.b);
        if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) t = -1.f;
        if (k < max) {
            kinds[k] = r.kind;
            ms[k] = t;
        }
        ++k;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_recs.clear();
    return k < max ? k : max;
}

gs_status gs_device_errors(int device, uint32_t *flags, int clear)
{
    g_detail.clear();
    if (!flags) return fail(GS_EINVAL, "flags is NULL");
    *flags = 0;
    gs_status s = check_device();
    if (s != GS_OK) return s;
    int count = 0, cur = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return fail(GS_EINVAL, "no device %d", device);
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != device) e = hipSetDevice(device);
    if (e != hipSuccess) return hip_fail(e, "selecting the device");
    unsigned f = 0;
    e = gs::sticky_errors_read(&f, clear != 0);
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return hip_fail(e, "reading the device error flags");
    *flags = f;
    return GS_OK;
}

int gs_test_fail_waits(int on)
{
    const unsigned was = gs::test_wait_word();
    gs::set_test_wait_word(on ? 1u : 0u);
    return (was & 1u) ? 1 : 0;
}

const char *gs_status_string(gs_status s)
{
    switch (s) {
        case GS_OK: return "GS_OK";
        case GS_EINVAL: return "GS_EINVAL";
        case GS_EUNSUPPORTED: return "GS_EUNSUPPORTED";
        case GS_EWORKSPACE: return "GS_EWORKSPACE";
        case GS_ENODEVICE: return "GS_ENODEVICE";
        case GS_EDEVICE: return "GS_EDEVICE";
    }
    return "GS_UNKNOWN";
}

const char *gs_last_error_detail(void) { return g_detail.c_str(); }

const char *gs_version(void) { return "0.1.0 gfx950"; }

size_t gs_workspace_bytes_f64_ex(int64_t n, double buffer_fraction, int algo, double sub_fraction)
{
    int64_t q = 0, q2 = 0;
    int a = 0;
    if (n < 0 || n > ((int64_t)1 << 40) || resolve_algo(buffer_fraction, algo, sub_fraction, &a, &q, &q2) != GS_OK)
        return SIZE_MAX;
    if (n <= 1) return 0;
    return (size_t)gs::plan_f64(n, q, a, q2).bytes;
}

size_t gs_workspace_bytes_kv_ex(int64_t n, double buffer_fraction, int algo, double sub_fraction)
{
    int64_t q = 0, q2 = 0;
    int a = 0;
    if (n < 0 || n > ((int64_t)1 << 40) || resolve_algo(buffer_fraction, algo, sub_fraction, &a, &q, &q2) != GS_OK)
        return SIZE_MAX;
    if (n <= 1) return 0;
    return (size_t)gs::plan_kv(n, q, a, q2).bytes;
}

size_t gs_workspace_bytes_f64(int64_t n, double buffer_fraction)
{
    return gs_workspace_bytes_f64_ex(n, buffer_fraction, GS_ALGO_AUTO, 0.5);
}

size_t gs_workspace_bytes_kv(int64_t n, double buffer_fraction)
{
    return gs_workspace_bytes_kv_ex(n, buffer_fraction, GS_ALGO_AUTO, 0.5);
}

int gs_plan_depth(int64_t n, int is_kv, int64_t *leaf_max)
{
    gs::SortPlan p = is_kv ? gs::plan_kv(n > 1 ? n : 2) : gs::plan_f64(n > 1 ? n : 2);
    if (leaf_max) *leaf_max = p.leaf;
    return n > 1 ? p.depth : 0;
}

void gs_plan_node(int64_t n, int depth, int64_t idx, int64_t *out)
{
    gs::FrogNode f = gs::frog_node(n, depth, idx);
    out[0] = f.s;
    out[1] = f.n;
    out[2] = f.left;
    out[3] = gs::frog_data_start(f);
    out[4] = f.in_off;
}

int gs_plan_leaf_window(int64_t n, int depth, int64_t leaf, int64_t *lo_hi)
{
    if (n < 1 || depth < 0 || depth > 40 || leaf < 0 || leaf >= ((int64_t)1 << depth) || !lo_hi) return -1;
    gs::leaf_window(n, depth, leaf, lo_hi, lo_hi + 1);
    return 0;
}

int gs_plan_tile_windows(const int64_t *merge, int kind, int dir_first, int dir_second, int turned, int64_t tile,
                         const int64_t *splits, int64_t *windows)
{
    if (!merge || !splits || !windows || tile < 1 || kind < gs::NODE_MERGE || kind > gs::NODE_CONCAT) return -1;
    gs::FrogMerge m{};
    m.l0 = merge[0];
    m.nl = merge[1];
    m.r0 = merge[2];
    m.nr = merge[3];
    m.out0 = merge[4];
    m.left = (int)merge[5];
    m.outer = (int)merge[6];
    if (m.nl < 0 || m.nr < 0 || m.outer < 0 || m.outer > 2) return -1;
    const gs::NodeViews v = gs::node_views(m, kind, dir_first, dir_second, turned != 0);
    const int64_t n = m.nl + m.nr, tpn = (n + tile - 1) / tile;
    for (int64_t q = 0; q < tpn; ++q) {
        const int64_t j = m.left ? tpn - 1 - q : q;
        int64_t lo, hi;
        gs::tile_window(v, m.out0, m.left, splits, tpn, tile, j, 0, &lo, &hi);
        if (lo <= hi) {
            lo = lo < 0 ? 0 : lo;
            hi = hi > q ? q : hi;
        }
        windows[2 * q] = lo;
        windows[2 * q + 1] = hi;
    }
    return (int)tpn;
}

int gs_plan_frog2(int64_t n, double buffer_fraction, int is_kv, int64_t *leaves, int64_t max_leaves,
                  int64_t *nodes, int64_t max_nodes, int64_t *counts)
{
    int64_t q = 0, q2 = 0;
    int a = 0;
    if (n < 2 || n > ((int64_t)1 << 32) ||
        resolve_algo(buffer_fraction, GS_ALGO_FROGSORT2, 0.5, &a, &q, &q2) != GS_OK)
        return -1;
    const gs::SortPlan p = is_kv ? gs::plan_kv(n, q, a) : gs::plan_f64(n, q, a);
    const gs::F2Tables &T = *p.f2;
    const char *b = T.blob.data();
    const int64_t *lc = (const int64_t *)(b + T.off_leaf_c), *ld = (const int64_t *)(b + T.off_leaf_d);
    const int64_t *ns = (const int64_t *)(b + T.off_node_s), *nn = (const int64_t *)(b + T.off_node_n);
    const unsigned *rb = (const unsigned *)(b + T.off_rb);
    for (int64_t i = 0; i < T.nleaves && i < max_leaves; ++i) {
        leaves[3 * i + 0] = lc[i];
        leaves[3 * i + 1] = ld[i];
        leaves[3 * i + 2] = lc[i + 1] - lc[i];
    }
    for (int r = 1; r <= T.rounds; ++r)
        for (unsigned k = rb[r]; k < rb[r + 1] && (int64_t)k < max_nodes; ++k) {
            nodes[4 * k + 0] = ns[k];
            nodes[4 * k + 1] = nn[k] & (gs::kF2LeftBit - 1);
            nodes[4 * k + 2] = (nn[k] & gs::kF2LeftBit) ? 1 : 0;
            nodes[4 * k + 3] = r;
        }
    counts[0] = T.nleaves;
    counts[1] = T.nnodes;
    counts[2] = T.rounds;
    counts[3] = p.hlen;
    counts[4] = T.max_tickets;
    counts[5] = T.max_splits;
    counts[6] = T.merged;
    return 0;
}

int gs_plan_frog3(int64_t n, double buffer_fraction, double sub_fraction, int is_kv, int64_t *trees,
                  int64_t max_trees, int64_t *spine, int64_t max_spine, int64_t *leaves, int64_t max_leaves,
                  int64_t *counts)
{
    int64_t q = 0, q2 = 0;
    int a = 0;
    if (n < 2 || n > ((int64_t)1 << 32) ||
        resolve_algo(buffer_fraction, GS_ALGO_FROGSORT6, sub_fraction, &a, &q, &q2) != GS_OK)
        return -1;
    const gs::SortPlan p = is_kv ? gs::plan_kv(n, q, a, q2) : gs::plan_f64(n, q, a, q2);
    const gs::F3Plan &P = *p.f3;
    int64_t nl = 0;
    for (size_t i = 0; i < P.trees.size(); ++i) {
        const gs::F2Tables &T = *P.trees[i];
        const char *b = T.blob.data();
        const int64_t *lc = (const int64_t *)(b + T.off_leaf_c), *ld = (const int64_t *)(b + T.off_leaf_d);
        if ((int64_t)i < max_trees) {
            trees[4 * i + 0] = P.root_s[i];
            trees[4 * i + 1] = P.root_n[i];
            trees[4 * i + 2] = P.root_c[i];
            trees[4 * i + 3] = P.root_left[i];
        }
        for (int64_t k = 0; k < T.nleaves; ++k, ++nl)
            if (nl < max_leaves) {
                leaves[3 * nl + 0] = lc[k];
                leaves[3 * nl + 1] = ld[k];
                leaves[3 * nl + 2] = lc[k + 1] - lc[k];
            }
    }
    for (size_t k = 0; k < P.spine.size() && (int64_t)k < max_spine; ++k) {
        spine[3 * k + 0] = P.spine[k].nl;
        spine[3 * k + 1] = P.spine[k].r0;
        spine[3 * k + 2] = P.spine[k].nr;
    }
    counts[0] = (int64_t)P.trees.size();
    counts[1] = (int64_t)P.spine.size();
    counts[2] = nl;
    counts[3] = P.total_rounds;
    counts[4] = p.hlen;
    counts[5] = P.b;
    counts[6] = P.merged;
    return 0;
}

int64_t gs_plan_seg_steps(const int64_t *offsets, int64_t num_segments, int64_t num_keys, double buffer_fraction,
                          int64_t *steps, int64_t max_steps, int64_t *buffer)
{
    if (num_segments < 0 || num_keys < 0 || (num_segments > 0 && !offsets) || (max_steps > 0 && !steps))
        return -1;
    SegFraction fr;
    if (seg_fraction(buffer_fraction, &fr) != GS_OK) return -1;
    if (!fr.q) return -2;
    for (int64_t i = 0; i < num_segments; ++i)
        if (offsets[i] < 0 || offsets[i + 1] < offsets[i] || offsets[i + 1] > num_keys) return -1;
    const gs::SegPlan p = gs::plan_seg(num_keys, num_segments, gs::seg_default_config(), fr.q, fr.algo, fr.q2);
    if (buffer) *buffer = p.hlen;
    const std::vector<gs::SegStep> st = gs::seg_schedule(offsets, num_segments, p.tile, p.hlen);
    for (size_t k = 0; k < st.size() && (int64_t)k < max_steps; ++k) {
        steps[3 * k + 0] = st[k].s0;
        steps[3 * k + 1] = st[k].s1;
        steps[3 * k + 2] = st[k].alone ? 1 : 0;
    }
    return (int64_t)st.size();
}

gs_status gs_sort_f64(double *keys, int64_t n, double buffer_fraction, void *ws, size_t ws_bytes,
                      void *hip_stream, gs_report *rep)
{
    return gs_sort_f64_target(keys, n, GS_ASC_LEFT, buffer_fraction, ws, ws_bytes, hip_stream, rep);
}

gs_status gs_sort_f64_target(double *keys, int64_t n, int target, double buffer_fraction, void *ws,
                             size_t ws_bytes, void *hip_stream, gs_report *rep)
{
    return gs_sort_f64_ex(keys, n, target, buffer_fraction, GS_ALGO_AUTO, 0.5, ws, ws_bytes, hip_stream, rep);
}

gs_status gs_sort_f64_ex(double *keys, int64_t n, int target, double buffer_fraction, int algo, double sub_fraction,
                         void *ws, size_t ws_bytes, void *hip_stream, gs_report *rep)
{
    g_detail.clear();
    if (target < GS_ASC_LEFT || target > GS_DESC_RIGHT) return fail(GS_EINVAL, "unknown target %d", target);
    if (n < 0) return fail(GS_EINVAL, "n < 0");
    if (n > 0 && !keys) return fail(GS_EINVAL, "keys is NULL");
    int64_t q = 0, q2 = 0;
    int a = 0;
    gs_status s = resolve_algo(buffer_fraction, algo, sub_fraction, &a, &q, &q2);
    if (s != GS_OK) return s;
    if (n > ((int64_t)1 << 40)) return fail(GS_EINVAL, "n above 2^40");
    gs::SortPlan p = gs::plan_f64(n, q, a, q2);
    if (n > 1) {
        if ((int64_t)ws_bytes < p.bytes || !ws)
            return fail(GS_EWORKSPACE, "workspace %zu bytes, need %lld", ws_bytes, (long long)p.bytes);
        if (!aligned256(ws)) return fail(GS_EINVAL, "workspace not 256-byte aligned");
    }
    if (n <= 1) {
        if (rep) { memset(rep, 0, sizeof *rep); rep->ram_fraction = 1.0; }
        return GS_OK;
    }
    if ((s = check_device()) != GS_OK) return s;
    hipStream_t st = (hipStream_t)hip_stream;
    if ((p.f2 || p.f3) && (s = check_not_capturing(st)) != GS_OK) return s;
    Reporter r(rep, st);
    hipError_t e = gs::sort_f64_target_async(keys, n, target, (char *)ws, p, st);
    if (e != hipSuccess) return r.finish(hip_fail(e, "gs_sort_f64 launch"));
    if (rep) {
        rep->levels = (uint32_t)p.depth;
        rep->workspace_bytes_used = (uint64_t)p.bytes;
        rep->ram_fraction = n > 0 ? 1.0 + (double)p.bytes / (8.0 * (double)n) : 1.0;
    }
    s = r.finish(GS_OK);
    if (rep && s == GS_OK) s = check_err_word((const char *)ws, p);
    if (rep && s == GS_OK) s = read_order((const char *)ws, p, n, target, rep);
    return s;
}

gs_status gs_sort_f64_noalloc(double *keys, int64_t n, void *hip_stream)
{
    g_detail.clear();
    if (n < 0) return fail(GS_EINVAL, "n < 0");
    if (n > 0 && !keys) return fail(GS_EINVAL, "keys is NULL");
    if (n > gs::kNoAllocMaxKeys)
        return fail(GS_EINVAL, "gs_sort_f64_noalloc: n = %lld is above its static workspace's limit of %lld keys",
                    (long long)n, (long long)gs::kNoAllocMaxKeys);
    if (n <= 1) return GS_OK;
    gs::SortPlan p = gs::plan_f64(n);
    if (p.bytes > gs::kNoAllocScratchBytes)
        return fail(GS_EUNSUPPORTED, "gs_sort_f64_noalloc: n = %lld needs %lld workspace bytes, above the static %lld",
                    (long long)n, (long long)p.bytes, (long long)gs::kNoAllocScratchBytes);
    gs_status s = check_device();
    if (s != GS_OK) return s;
    char *ws = nullptr;
    hipError_t e = gs::noalloc_scratch(&ws);
    if (e != hipSuccess) return hip_fail(e, "looking up the static workspace");
    e = gs::sort_f64_target_async(keys, n, GS_ASC_LEFT, ws, p, (hipStream_t)hip_stream);
    return e == hipSuccess ? GS_OK : hip_fail(e, "gs_sort_f64_noalloc launch");
}

static bool to_seg_config(const gs_seg_config *c, gs::SegConfig *out)
{
    if (!c) {
        *out = gs::seg_default_config();
        return true;
    }
    out->short_threads = (int)c->short_threads;
    out->short_ipt = (int)c->short_ipt;
    out->merge_ipt = (int)c->merge_ipt;
    return c->reserved == 0 && gs::seg_config_valid(*out);
}

}  // extern "C"

// ---- tuning cache: the shape gs_segsort_autotune found, per device
// architecture and size class (floor(log2) of the keys and of the segments);
// kept for the process and, when GS_TUNE_CACHE names a file, read from it on
// first use and written back after every tuning run -------------------------
namespace {
struct TuneKey {
    std::string arch;
    int lk, ls;
    bool operator<(const TuneKey &o) const
    {
        return arch != o.arch ? arch < o.arch : lk != o.lk ? lk < o.lk : ls < o.ls;
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, gs_seg_config> g_tune;
bool g_tune_env_read = false;

int floor_log2(int64_t v)
{
    int r = 0;
    while (v > 1) {
        v >>= 1;
        ++r;
    }
    return r;
}

// the current device's architecture name without its feature suffixes
// (queried once per device)
std::string current_arch()
{
    static std::mutex mu;
    static std::map<int, std::string> names;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return std::string();
    }
    std::lock_guard<std::mutex> lk(mu);
    const auto it = names.find(dev);
    if (it != names.end()) return it->second;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return std::string();
    }
    std::string a(prop.gcnArchName);
    const size_t c = a.find(':');
    if (c != std::string::npos) a = a.substr(0, c);
    names[dev] = a;
    return a;
}

// value of "key": <int> inside one JSON object's text; false if absent
bool json_int(const std::string &obj, const char *key, long long *out)
{
    const std::string k = std::string("\"") + key + "\"";
    size_t p = obj.find(k);
    if (p == std::string::npos) return false;
    p = obj.find(':', p + k.size());
    if (p == std::string::npos) return false;
    char *end = nullptr;
    const long long v = strtoll(obj.c_str() + p + 1, &end, 10);
    if (end == obj.c_str() + p + 1) return false;
    *out = v;
    return true;
}

bool json_str(const std::string &obj, const char *key, std::string *out)
{
    const std::string k = std::string("\"") + key + "\"";
    size_t p = obj.find(k);
    if (p == std::string::npos) return false;
    p = obj.find('"', obj.find(':', p + k.size()));
    if (p == std::string::npos) return false;
    const size_t q = obj.find('"', p + 1);
    if (q == std::string::npos) return false;
    *out = obj.substr(p + 1, q - p - 1);
    return true;
}

// reads {"entries": [{...}, ...]} (every valid entry; others are skipped);
// caller holds the lock
int tune_load_locked(const char *path)
{
    FILE *f = fopen(path, "rb");
    if (!f) return -1;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    fclose(f);
    int n = 0;
    size_t p = text.find('[');
    while (p != std::string::npos) {
        const size_t a = text.find('{', p);
        if (a == std::string::npos) break;
        const size_t b = text.find('}', a);
        if (b == std::string::npos) break;
        const std::string obj = text.substr(a, b - a + 1);
        p = b + 1;
        std::string arch;
        long long lk, ls, st, si, mi;
        if (!json_str(obj, "arch", &arch) || !json_int(obj, "log2_keys", &lk) ||
            !json_int(obj, "log2_segments", &ls) || !json_int(obj, "short_threads", &st) ||
            !json_int(obj, "short_ipt", &si) || !json_int(obj, "merge_ipt", &mi))
            continue;
        gs_seg_config c{(uint32_t)st, (uint32_t)si, (uint32_t)mi, 0u};
        gs::SegConfig sc;
        if (!to_seg_config(&c, &sc) || lk < 0 || lk > 62 || ls < 0 || ls > 62) continue;
        g_tune[TuneKey{arch, (int)lk, (int)ls}] = c;
        ++n;
    }
    return n;
}

int tune_save_locked(const char *path)
{
    FILE *f = fopen(path, "wb");
    if (!f) return -1;
    fprintf(f, "{\"entries\": [");
    bool first = true;
    for (const auto &kv : g_tune) {
        fprintf(f, "%s\n  {\"arch\": \"%s\", \"log2_keys\": %d, \"log2_segments\": %d, \"short_threads\": %u, "
                   "\"short_ipt\": %u, \"merge_ipt\": %u}",
                first ? "" : ",", kv.first.arch.c_str(), kv.first.lk, kv.first.ls, kv.second.short_threads,
                kv.second.short_ipt, kv.second.merge_ipt);
        first = false;
    }
    fprintf(f, "\n]}\n");
    return fclose(f) == 0 ? (int)g_tune.size() : -1;
}

void tune_env_locked()
{
    if (g_tune_env_read) return;
    g_tune_env_read = true;
    const char *path = getenv("GS_TUNE_CACHE");
    if (path && *path) (void)tune_load_locked(path);
}

bool tune_lookup(const std::string &arch, int64_t n, int64_t nseg, gs_seg_config *out)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_env_locked();
    const auto it = g_tune.find(TuneKey{arch, floor_log2(n), floor_log2(nseg)});
    if (it == g_tune.end()) return false;
    *out = it->second;
    return true;
}

void tune_record(const std::string &arch, int64_t n, int64_t nseg, const gs_seg_config &c)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_env_locked();
    g_tune[TuneKey{arch, floor_log2(n), floor_log2(nseg)}] = c;
    const char *path = getenv("GS_TUNE_CACHE");
    if (path && *path) (void)tune_save_locked(path);
}
}  // namespace

extern "C" {

int gs_tune_cache_get(const char *arch, int64_t num_keys, int64_t num_segments, gs_seg_config *out)
{
    if (!out || num_keys < 1 || num_segments < 1) return -1;
    const std::string a = arch ? std::string(arch) : current_arch();
    return tune_lookup(a, num_keys, num_segments, out) ? 1 : 0;
}

gs_status gs_tune_cache_put(const char *arch, int64_t num_keys, int64_t num_segments, const gs_seg_config *cfg)
{
    g_detail.clear();
    gs::SegConfig sc;
    if (!arch || !*arch || !cfg || num_keys < 1 || num_segments < 1 || !to_seg_config(cfg, &sc))
        return fail(GS_EINVAL, "bad tuning-cache entry");
    tune_record(arch, num_keys, num_segments, *cfg);
    return GS_OK;
}

int gs_tune_cache_load(const char *path)
{
    if (!path) return -1;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_env_read = true;
    return tune_load_locked(path);
}

int gs_tune_cache_save(const char *path)
{
    if (!path) return -1;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return tune_save_locked(path);
}

void gs_tune_cache_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    g_tune_env_read = true;
}

int gs_seg_config_count(void) { return gs::seg_config_count(); }

gs_status gs_seg_config_get(int i, gs_seg_config *out)
{
    g_detail.clear();
    if (!out || i < 0 || i >= gs::seg_config_count()) return fail(GS_EINVAL, "no shape %d", i);
    const gs::SegConfig c = gs::seg_config_at(i);
    out->short_threads = (uint32_t)c.short_threads;
    out->short_ipt = (uint32_t)c.short_ipt;
    out->merge_ipt = (uint32_t)c.merge_ipt;
    out->reserved = 0;
    return GS_OK;
}

void gs_seg_default_config(gs_seg_config *out)
{
    if (out) (void)gs_seg_config_get(0, out);
}

size_t gs_workspace_bytes_seg_ex(int64_t num_keys, int64_t num_segments, double buffer_fraction,
                                 const gs_seg_config *cfg)
{
    if (num_keys < 0 || num_segments < 0 || !(buffer_fraction > 0.0)) return SIZE_MAX;
    SegFraction fr;
    if (seg_fraction(buffer_fraction, &fr) != GS_OK) return SIZE_MAX;
    if (num_segments == 0) return 0;
    gs::SegConfig c;
    if (!to_seg_config(cfg, &c)) return SIZE_MAX;
    return (size_t)gs::plan_seg(num_keys, num_segments, c, fr.q, fr.algo, fr.q2).bytes;
}

size_t gs_workspace_bytes_seg(int64_t num_keys, int64_t num_segments, double buffer_fraction)
{
    if (num_keys < 0 || num_segments < 0 || !(buffer_fraction > 0.0)) return SIZE_MAX;
    SegFraction fr;
    if (seg_fraction(buffer_fraction, &fr) != GS_OK) return SIZE_MAX;
    if (num_segments == 0) return 0;
    int64_t most = 0;
    for (int i = 0; i < gs::seg_config_count(); ++i) {
        const int64_t b = gs::plan_seg(num_keys, num_segments, gs::seg_config_at(i), fr.q, fr.algo, fr.q2).bytes;
        if (b > most) most = b;
    }
    return (size_t)most;
}

// Checks shared by the segmented entry points; fills the plan.
static gs_status seg_checks(double *keys, int64_t num_keys, const int64_t *offsets, int64_t num_segments,
                            double buffer_fraction, const gs_seg_config *cfg, void *ws, size_t ws_bytes,
                            gs::SegPlan *p)
{
    if (num_keys < 0 || num_segments < 0) return fail(GS_EINVAL, "num_keys or num_segments < 0");
    if (num_segments > ((int64_t)1 << 31) - 2) return fail(GS_EINVAL, "num_segments above 2^31-2");
    if (num_keys > ((int64_t)1 << 40)) return fail(GS_EINVAL, "num_keys above 2^40");
    SegFraction fr;
    gs_status s = seg_fraction(buffer_fraction, &fr);
    if (s != GS_OK) return s;
    gs::SegConfig c;
    if (!to_seg_config(cfg, &c)) return fail(GS_EINVAL, "unknown segmented-sort shape");
    if (num_segments == 0) return GS_OK;
    if (!offsets) return fail(GS_EINVAL, "offsets is NULL");
    if (num_keys > 0 && !keys) return fail(GS_EINVAL, "keys is NULL");
    *p = gs::plan_seg(num_keys, num_segments, c, fr.q, fr.algo, fr.q2);
    if ((int64_t)ws_bytes < p->bytes || !ws)
        return fail(GS_EWORKSPACE, "workspace %zu bytes, need %lld", ws_bytes, (long long)p->bytes);
    if (!aligned256(ws)) return fail(GS_EINVAL, "workspace not 256-byte aligned");
    return GS_OK;
}

// buffer_fraction < 0.5: the offsets come to the host (the call waits for
// the work queued before it on the stream), the buffer serves runs of
// consecutive segments in turn, and a segment whose half buffer does not fit
// is sorted alone by the plain sort, with the largest fraction whose buffer
// fits in the workspace.
static gs_status segsort_small_buffer(double *keys, int64_t num_keys, const int64_t *offsets, int64_t nseg,
                                      const gs::SegPlan &p, void *ws, size_t ws_bytes, hipStream_t st,
                                      gs_report *rep)
{
    gs_status s = check_not_capturing(st);
    if (s != GS_OK) return s;
    std::vector<int64_t> off((size_t)nseg + 1);
    hipError_t e = hipMemcpyAsync(off.data(), offsets, (size_t)(nseg + 1) * sizeof(int64_t), hipMemcpyDeviceToHost,
                                  st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "reading the segment offsets");
    for (int64_t i = 0; i < nseg; ++i) {
        if (off[i] < 0 || off[i + 1] < off[i] || off[i + 1] > num_keys) {
            if (rep) {
                memset(rep, 0, sizeof *rep);
                rep->ram_fraction = 1.0;
                rep->invalid_offsets = 1u;
            }
            return fail(GS_EINVAL, "offsets not non-decreasing within [0, num_keys]");
        }
    }
    const std::vector<gs::SegStep> steps = gs::seg_schedule(off.data(), nseg, p.tile, p.hlen);
    // every plan of a segment sorted alone is made before anything runs
    std::vector<gs::SortPlan> alone;
    int64_t used = p.off_forest + p.forest.bytes;
    for (const gs::SegStep &t : steps) {
        if (!t.alone) continue;
        const int64_t len = off[(size_t)t.s0 + 1] - off[(size_t)t.s0];
        const int64_t qa = (int64_t)(((__int128)p.hlen << 16) / len);   // floor(qa len / 2^16) <= hlen
        gs::SortPlan a{};
        bool fits = false;
        if (qa >= gs::kF2MinQ && qa < 32768) {
            a = gs::plan_f64(len, qa, p.algo, p.q2);
            fits = a.bytes <= (int64_t)ws_bytes;
        }
        if (!fits) {
            a = gs::plan_f64(len, p.q, p.algo, p.q2);
            if (a.bytes > (int64_t)ws_bytes)
                return fail(GS_EWORKSPACE, "workspace %zu bytes, a segment of %lld keys needs %lld", ws_bytes,
                            (long long)len, (long long)a.bytes);
        }
        if (a.bytes > used) used = a.bytes;
        alone.push_back(std::move(a));
    }
    Reporter r(rep, st);
    size_t k = 0;
    for (const gs::SegStep &t : steps) {
        if (!t.alone) continue;
        const gs::SortPlan &a = alone[k++];
        e = gs::sort_f64_target_async(keys + off[(size_t)t.s0], a.n, GS_ASC_LEFT, (char *)ws, a, st);
        if (e != hipSuccess) return r.finish(hip_fail(e, "gs_segsort launch"));
        if (rep) {
            // the passes below reuse this sort's control area
            e = hipStreamSynchronize(st);
            s = e != hipSuccess ? hip_fail(e, "hipStreamSynchronize") : check_err_word((const char *)ws, a);
            if (s != GS_OK) return r.finish(s);
        }
    }
    e = gs::segsort_passes_async(keys, offsets, off.data(), p, steps, (char *)ws, st);
    if (e != hipSuccess) return r.finish(hip_fail(e, "gs_segsort launch"));
    s = r.finish(GS_OK);
    if (rep && s == GS_OK) {
        rep->workspace_bytes_used = (uint64_t)used;
        rep->ram_fraction = num_keys > 0 ? 1.0 + (double)used / (8.0 * (double)num_keys) : 1.0;
        s = check_err_word((const char *)ws + p.off_forest + p.forest.off_ctrl);
    }
    return s;
}

gs_status gs_segsort_ex(double *keys, int64_t num_keys, const int64_t *offsets, int64_t num_segments,
                        double buffer_fraction, const gs_seg_config *cfg, void *ws, size_t ws_bytes,
                        void *hip_stream, gs_report *rep)
{
    g_detail.clear();
    // no shape given: the tuned one of this architecture and size class, if
    // the tuning cache holds one and the workspace fits it
    gs_seg_config tuned;
    if (!cfg && num_keys > 0 && num_segments > 0 && tune_lookup(current_arch(), num_keys, num_segments, &tuned)) {
        const size_t need = gs_workspace_bytes_seg_ex(num_keys, num_segments, buffer_fraction, &tuned);
        if (need != SIZE_MAX && need <= ws_bytes) cfg = &tuned;
    }
    gs::SegPlan p{};
    gs_status s = seg_checks(keys, num_keys, offsets, num_segments, buffer_fraction, cfg, ws, ws_bytes, &p);
    if (s != GS_OK) return s;
    if (num_segments == 0) {
        if (rep) { memset(rep, 0, sizeof *rep); rep->ram_fraction = 1.0; }
        return GS_OK;
    }
    if ((s = check_device()) != GS_OK) return s;
    hipStream_t st = (hipStream_t)hip_stream;
    if (p.q) return segsort_small_buffer(keys, num_keys, offsets, num_segments, p, ws, ws_bytes, st, rep);
    Reporter r(rep, st);
    hipError_t e = gs::segsort_f64_async(keys, offsets, p, (char *)ws, st);
    if (e != hipSuccess) return r.finish(hip_fail(e, "gs_segsort launch"));
    s = r.finish(GS_OK);
    if (rep && s == GS_OK) {
        rep->workspace_bytes_used = (uint64_t)p.bytes;
        rep->ram_fraction = num_keys > 0 ? 1.0 + (double)p.bytes / (8.0 * (double)num_keys) : 1.0;
        unsigned inval = 0;
        hipError_t e2 = hipMemcpy(&inval, (const char *)ws + p.off_ctrl, 4, hipMemcpyDeviceToHost);
        if (e2 != hipSuccess) return hip_fail(e2, "reading the offsets flag");
        rep->invalid_offsets = inval ? 1u : 0u;
        if (inval) return fail(GS_EINVAL, "offsets not non-decreasing within [0, num_keys]");
        s = check_err_word((const char *)ws + p.off_forest + p.forest.off_ctrl);
    }
    return s;
}

gs_status gs_segsort(double *keys, int64_t num_keys, const int64_t *offsets, int64_t num_segments,
                     double buffer_fraction, void *ws, size_t ws_bytes, void *hip_stream,
                     gs_report *rep)
{
    return gs_segsort_ex(keys, num_keys, offsets, num_segments, buffer_fraction, nullptr, ws, ws_bytes,
                         hip_stream, rep);
}

gs_status gs_segsort_autotune(const double *keys, int64_t num_keys, const int64_t *offsets,
                              int64_t num_segments, double *scratch, void *ws, size_t ws_bytes,
                              void *hip_stream, int reps, gs_seg_config *best, float *times_ms)
{
    g_detail.clear();
    if (!best) return fail(GS_EINVAL, "best is NULL");
    if (reps < 1) return fail(GS_EINVAL, "reps < 1");
    if (num_keys > 0 && !scratch) return fail(GS_EINVAL, "scratch is NULL");
    const int nc = gs::seg_config_count();
    gs::SegPlan p{};
    for (int i = 0; i < nc; ++i) {
        gs_seg_config c;
        (void)gs_seg_config_get(i, &c);
        gs_status s = seg_checks(scratch, num_keys, offsets, num_segments, 0.5, &c, ws, ws_bytes, &p);
        if (s != GS_OK) return s;
    }
    gs_seg_default_config(best);
    if (num_segments == 0 || num_keys == 0) return GS_OK;
    gs_status s = check_device();
    if (s != GS_OK) return s;
    hipStream_t st = (hipStream_t)hip_stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(GS_EDEVICE, "hipEventCreate failed");
    }
    float best_ms = 0.f;
    s = GS_OK;
    for (int i = 0; i < nc && s == GS_OK; ++i) {
        gs_seg_config c;
        (void)gs_seg_config_get(i, &c);
        float fastest = 0.f;
        for (int r = 0; r <= reps && s == GS_OK; ++r) {           // run 0 warms up
            hipError_t e = hipMemcpyAsync(scratch, keys, (size_t)num_keys * 8, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess) e = hipEventRecord(e0, st);
            if (e == hipSuccess) {
                p = gs::plan_seg(num_keys, num_segments, gs::seg_config_at(i));
                e = gs::segsort_f64_async(scratch, offsets, p, (char *)ws, st);
            }
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                s = hip_fail(e, "timing a segmented-sort shape");
                break;
            }
            if (r > 0 && (r == 1 || ms < fastest)) fastest = ms;
        }
        if (s != GS_OK) break;
        unsigned inval = 0;
        hipError_t e2 = hipMemcpy(&inval, (const char *)ws + p.off_ctrl, 4, hipMemcpyDeviceToHost);
        if (e2 != hipSuccess) s = hip_fail(e2, "reading the offsets flag");
        else if (inval) s = fail(GS_EINVAL, "offsets not non-decreasing within [0, num_keys]");
        else s = check_err_word((const char *)ws + p.off_forest + p.forest.off_ctrl);
        if (s != GS_OK) break;
        if (times_ms) times_ms[i] = fastest;
        if (i == 0 || fastest < best_ms) {
            best_ms = fastest;
            *best = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s == GS_OK && num_keys > 0 && num_segments > 0) {
        const std::string arch = current_arch();
        if (!arch.empty()) tune_record(arch, num_keys, num_segments, *best);
    }
    return s;
}

gs_status gs_sort_kv(uint64_t *keys, uint32_t *vals, int64_t n, double buffer_fraction, void *ws,
                     size_t ws_bytes, void *hip_stream, gs_report *rep)
{
    return gs_sort_kv_target(keys, vals, n, GS_ASC_LEFT, buffer_fraction, ws, ws_bytes, hip_stream, rep);
}

gs_status gs_sort_kv_target(uint64_t *keys, uint32_t *vals, int64_t n, int target, double buffer_fraction,
                            void *ws, size_t ws_bytes, void *hip_stream, gs_report *rep)
{
    return gs_sort_kv_ex(keys, vals, n, target, buffer_fraction, GS_ALGO_AUTO, 0.5, ws, ws_bytes, hip_stream, rep);
}

gs_status gs_sort_kv_ex(uint64_t *keys, uint32_t *vals, int64_t n, int target, double buffer_fraction, int algo,
                        double sub_fraction, void *ws, size_t ws_bytes, void *hip_stream, gs_report *rep)
{
    g_detail.clear();
    if (target < GS_ASC_LEFT || target > GS_DESC_RIGHT) return fail(GS_EINVAL, "unknown target %d", target);
    if (n < 0) return fail(GS_EINVAL, "n < 0");
    if (n > 0 && (!keys || !vals)) return fail(GS_EINVAL, "keys or vals is NULL");
    int64_t q = 0, q2 = 0;
    int a = 0;
    gs_status s = resolve_algo(buffer_fraction, algo, sub_fraction, &a, &q, &q2);
    if (s != GS_OK) return s;
    if (n > ((int64_t)1 << 40)) return fail(GS_EINVAL, "n above 2^40");
    gs::SortPlan p = gs::plan_kv(n, q, a, q2);
    if (n > 1) {
        if ((int64_t)ws_bytes < p.bytes || !ws)
            return fail(GS_EWORKSPACE, "workspace %zu bytes, need %lld", ws_bytes, (long long)p.bytes);
        if (!aligned256(ws)) return fail(GS_EINVAL, "workspace not 256-byte aligned");
    }
    if (n <= 1) {
        if (rep) { memset(rep, 0, sizeof *rep); rep->ram_fraction = 1.0; }
        return GS_OK;
    }
    if ((s = check_device()) != GS_OK) return s;
    hipStream_t st = (hipStream_t)hip_stream;
    if ((p.f2 || p.f3) && (s = check_not_capturing(st)) != GS_OK) return s;
    Reporter r(rep, st);
    hipError_t e = gs::sort_kv_target_async(keys, vals, n, target, (char *)ws, p, st);
    if (e != hipSuccess) return r.finish(hip_fail(e, "gs_sort_kv launch"));
    if (rep) {
        rep->levels = (uint32_t)p.depth;
        rep->workspace_bytes_used = (uint64_t)p.bytes;
        rep->ram_fraction = n > 0 ? 1.0 + (double)p.bytes / (12.0 * (double)n) : 1.0;
    }
    s = r.finish(GS_OK);
    if (rep && s == GS_OK) s = check_err_word((const char *)ws, p);
    if (rep && s == GS_OK) s = read_order((const char *)ws, p, n, target, rep);
    return s;
}

}  // extern "C"

// ---- learned path -----------------------------------------------------------
extern "C" {

void gs_learned_default_params(gs_learned_params *p)
{
    memset(p, 0, sizeof *p);
    p->num_buckets = 4096;
    p->sample_size = 65536;
    p->train_steps = 8;
    p->batch = 2048;
    p->knots = 4096;
    p->lr = 4e-2f;
    p->seed = 0x5eed;
    p->mode = 0;
    p->buffer_fraction = 0.5;
}

// The learned path at buffer fraction 0 (the default) or >= 0.5; below, the
// plain sort's algorithm and q (*q = 0: the learned path).
static gs_status learned_fraction(const gs_learned_params &p, int *algo, int64_t *q, int64_t *q2)
{
    *q = 0;
    if (p.buffer_fraction == 0.0 || p.buffer_fraction >= 0.5) return GS_OK;
    return resolve_algo(p.buffer_fraction, GS_ALGO_AUTO, 0.5, algo, q, q2);
}

static gs_status check_learned_params(const gs_learned_params &p)
{
    auto pow2 = [](uint32_t v) { return v >= 2 && (v & (v - 1)) == 0; };
    if (!pow2(p.num_buckets) || p.num_buckets > 4096)
        return fail(GS_EINVAL, "num_buckets must be a power of two in [2, 4096]");
    if (p.sample_size < 1024 || p.sample_size > (1u << 24)) return fail(GS_EINVAL, "sample_size out of [1024, 2^24]");
    if (p.knots < 2 || p.knots > 16384) return fail(GS_EINVAL, "knots out of [2, 16384]");
    if (p.batch < 32 || p.batch % 32 || p.batch > 8192) return fail(GS_EINVAL, "batch must be a multiple of 32 in [32, 8192]");
    if (p.mode > 2) return fail(GS_EINVAL, "mode must be 0, 1 or 2");
    if (p.screen > 1) return fail(GS_EINVAL, "screen must be 0 or 1");
    if (!(p.lr > 0.f) || !(p.lr < 1.f)) return fail(GS_EINVAL, "lr out of (0, 1)");
    if (p.train_steps > 100000) return fail(GS_EINVAL, "train_steps above 100000");
    int a = 0;
    int64_t q = 0, q2 = 0;
    return learned_fraction(p, &a, &q, &q2);
}

size_t gs_workspace_bytes_learned(int64_t n, const gs_learned_params *p)
{
    gs_learned_params d;
    gs_learned_default_params(&d);
    const gs_learned_params &q = p ? *p : d;
    if (n < 0) return SIZE_MAX;
    if (n <= 1) return 0;
    if (check_learned_params(q) != GS_OK) return SIZE_MAX;
    int a = 0;
    int64_t fq = 0, fq2 = 0;
    (void)learned_fraction(q, &a, &fq, &fq2);
    if (fq) return (size_t)gs::plan_f64(n, fq, a, fq2).bytes;
    return (size_t)gs::plan_learned(n, q).bytes;
}

gs_status gs_learned_sort(double *keys, int64_t n, const gs_learned_params *p, void *ws, size_t ws_bytes,
                          void *hip_stream, gs_report *rep)
{
    g_detail.clear();
    gs_learned_params d;
    gs_learned_default_params(&d);
    const gs_learned_params &q = p ? *p : d;
    if (n < 0) return fail(GS_EINVAL, "n < 0");
    if (n > 0 && !keys) return fail(GS_EINVAL, "keys is NULL");
    gs_status s = check_learned_params(q);
    if (s != GS_OK) return s;
    if (n > ((int64_t)1 << 40)) return fail(GS_EINVAL, "n above 2^40");
    if (n <= 1) {
        if (rep) { memset(rep, 0, sizeof *rep); rep->ram_fraction = 1.0; }
        return GS_OK;
    }
    int fa = 0;
    int64_t fq = 0, fq2 = 0;
    (void)learned_fraction(q, &fa, &fq, &fq2);
    if (fq) {
        // the distribution passes need a half buffer: the plain path at the
        // caller's fraction sorts instead
        s = gs_sort_f64_ex(keys, n, GS_ASC_LEFT, q.buffer_fraction, GS_ALGO_AUTO, 0.5, ws, ws_bytes, hip_stream,
                           rep);
        if (rep && s == GS_OK) rep->fallback = 3;
        return s;
    }
    gs::LearnedPlan L = gs::plan_learned(n, q);
    if ((int64_t)ws_bytes < L.bytes || !ws)
        return fail(GS_EWORKSPACE, "workspace %zu bytes, need %lld", ws_bytes, (long long)L.bytes);
    if (!aligned256(ws)) return fail(GS_EINVAL, "workspace not 256-byte aligned");
    if ((s = check_device()) != GS_OK) return s;
    hipStream_t st = (hipStream_t)hip_stream;
    Reporter r(rep, st);
    hipError_t e = gs::learned_sort_async(keys, n, q, (char *)ws, L, st);
    if (e != hipSuccess) return r.finish(hip_fail(e, "gs_learned_sort launch"));
    s = r.finish(GS_OK);
    if (rep && s == GS_OK) {
        gs::LearnedReport lr{};
        hipError_t e2 = gs::learned_read_report((const char *)ws, L, &lr);
        if (e2 != hipSuccess) return hip_fail(e2, "reading the learned report");
        rep->levels = (uint32_t)L.plain.depth;
        rep->workspace_bytes_used = (uint64_t)L.bytes;
        rep->ram_fraction = 1.0 + (double)L.bytes / (8.0 * (double)n);
        rep->fallback = lr.fallback;
        rep->overflow_buckets = lr.overflow_buckets;
        rep->max_bucket = lr.max_bucket;
        rep->train_loss_first = lr.loss_first;
        rep->train_loss_last = lr.loss_last;
        rep->feature = lr.feature;
        rep->heavy_values = lr.heavy;
        unsigned any = 0;
        hipError_t e3 = gs::learned_errors((const char *)ws, L, &any);
        if (e3 != hipSuccess) return hip_fail(e3, "reading the error words");
        if (any) return fail(GS_EDEVICE, "a bounded device wait gave up or a work capacity was exceeded");
    }
    return s;
}

// ---- test hooks for the network (device pointers) ---------------------------
gs_status gs_mlp_loss_grad(const float *params, const float *u, const float *t, int batch, float *grad,
                           float *loss, void *work, size_t work_bytes, void *hip_stream)
{
    if (!params || !u || !t || !grad || !loss || batch < 32 || batch % 32)
        return fail(GS_EINVAL, "bad gs_mlp_loss_grad arguments");
    const size_t need = (size_t)(batch / 32) * (gs::kMlpParams + 1) * 4;
    if (!work || work_bytes < need) return fail(GS_EWORKSPACE, "gs_mlp_loss_grad needs %zu bytes", need);
    gs_status s = check_device();
    if (s != GS_OK) return s;
    hipError_t e = gs::mlp_loss_grad(params, u, t, batch, (float *)work, grad, loss, (hipStream_t)hip_stream);
    return e == hipSuccess ? GS_OK : hip_fail(e, "gs_mlp_loss_grad");
}

gs_status gs_mlp_train(float *params, float *adam_m, float *adam_v, const float *u, const float *t,
                       int64_t count, int steps, int batch, float lr, uint64_t seed, int full_batch,
                       float *losses, void *work, size_t work_bytes, void *hip_stream)
{
    if (!params || !adam_m || !adam_v || !u || !t || count < 1 || steps < 0 || batch < 32 || batch % 32 ||
        batch > 8192 || !(lr > 0.f))
        return fail(GS_EINVAL, "bad gs_mlp_train arguments");
    const size_t need = (size_t)(batch / 32) * (gs::kMlpParams + 1) * 4 + 256;
    if (!work || work_bytes < need) return fail(GS_EWORKSPACE, "gs_mlp_train needs %zu bytes", need);
    gs_status s = check_device();
    if (s != GS_OK) return s;
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e = gs::mlp_train(params, adam_m, adam_v, u, t, count, steps, batch, lr, seed, full_batch,
                                 (float *)work, losses, nullptr, st);
    return e == hipSuccess ? GS_OK : hip_fail(e, "gs_mlp_train");
}

gs_status gs_mlp_forward(const float *params, const float *u, int64_t count, float *y, void *hip_stream)
{
    if (!params || !u || !y || count < 0) return fail(GS_EINVAL, "bad gs_mlp_forward arguments");
    if (count == 0) return GS_OK;
    gs_status s = check_device();
    if (s != GS_OK) return s;
    hipError_t e = gs::mlp_forward(params, u, count, y, 0, nullptr, (hipStream_t)hip_stream);
    return e == hipSuccess ? GS_OK : hip_fail(e, "gs_mlp_forward");
}

}  // extern "C"
