/*
 * gs.h -- C ABI of the MI355X (gfx950) greeNsort library, libgs.so.
 *
 * The library sorts contiguous device arrays stably and in ascending order
 * (the paper's "Definition of sorting": the AscLeft target, ties kept in input
 * order read from left to right; "Values and principles / Stability"), by the
 * half-buffer symmetric mergesort of the sections "Symmetric merging" and
 * "Frogsort1": the extra memory is a buffer of floor(n/2) elements, and the two
 * children of every merge are sorted into mirrored positions (data left/buffer
 * right vs buffer left/data right) so that merging needs no extra moves.
 *
 * Conventions for every call below
 *   - Pointers named `keys`, `vals`, `offsets`, `ws` are DEVICE pointers
 *     (hipMalloc / torch CUDA tensors) on the current HIP device; pointers in
 *     structs are device pointers unless their comment says host.
 *   - `hip_stream` is a hipStream_t (NULL = the default stream).  Every call is
 *     asynchronous on that stream unless `rep` is non-NULL, in which case the
 *     call synchronises the stream before filling the report (gs_learned_sort
 *     also synchronises once mid-call; see there).
 *   - Sorting is in place: the result replaces `keys` (and `vals`).
 *   - The caller owns all memory.  The library makes no device allocation; the
 *     workspace `ws` (at least gs_workspace_bytes_*() bytes, 256-byte aligned)
 *     holds the half buffer and a small control area, so the paper's %RAM KPI
 *     ("Sustainability measures") is exactly 1 + ws_bytes / data_bytes.
 *   - Errors are returned, never thrown.  Argument errors are detected before
 *     any device work is enqueued, so the input is untouched on any error.
 *   - `buffer_fraction` p caps the element buffer (the half buffer of keys,
 *     and of values) as a fraction of the data.  The workspace holds a control
 *     area on top of it (status words, merge-path splits, tile descriptors,
 *     run directions and run samples, plan tables): for the single-array
 *     sorts under 0.4% of the data at 2^28 keys (about 32 bytes per 1024
 *     keys), more for small n, where its fixed part dominates.  %RAM
 *     (ram_fraction in the report) counts both, so it exceeds 1 + p by that
 *     overhead.
 *     p >= 0.5 selects Frogsort1 (buffer floor(n/2); never more).  For p in
 *     [1/64, 0.5) the fraction is rounded down to q/65536 (q = floor(65536 p))
 *     and the sort runs Frogsort3 ("Frogsort3 and 6": one buffer of floor(q n/65536)
 *     elements serving the branches in turn) unless gs_sort_*_ex asks for
 *     Frogsort2 ("Frogsort2": every inner branch, and the buffer, the fraction
 *     p).  p in (0, 1/64) -> GS_EUNSUPPORTED (the trees get hundreds of levels
 *     deep); NaN, <= 0 -> GS_EINVAL.  The segmented sort below 0.5: see
 *     gs_segsort.
 *   - A call with p < 0.5 plans its tree on the host and copies the plan's
 *     tables into the workspace on the stream (hipMemcpyAsync from host
 *     memory the library keeps), so it returns GS_EUNSUPPORTED while the
 *     stream is capturing a graph.
 *   - Calls on different streams with different workspaces may run
 *     concurrently; two calls sharing one workspace must be ordered.
 *   - Failures found on the device after a call has returned (a bounded wait
 *     that gave up, a work capacity exceeded, rejected segment offsets) reach
 *     the caller through the call's status when it asks for a report, and in
 *     every case through the per-device flags of gs_device_errors (below).
 *
 * Comparison: float64 keys compare as IEEE `<` except that NaNs are greater
 * than every other value and tie with each other; -0.0 and +0.0 tie.  Keys are
 * moved bit for bit and never rounded or transformed.  uint64 keys compare
 * unsigned.
 */
#ifndef GS_H
#define GS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GS_OK = 0,
    GS_EINVAL = 1,        /* bad argument (null pointer with n > 0, n < 0, bad fraction, bad offsets) */
    GS_EUNSUPPORTED = 2,  /* valid request this version does not implement (buffer_fraction < 1/64, ...) */
    GS_EWORKSPACE = 3,    /* ws_bytes below the size the matching gs_workspace_bytes_* returns */
    GS_ENODEVICE = 4,     /* no HIP device visible */
    GS_EDEVICE = 5        /* a HIP runtime call failed; see gs_last_error_detail() */
} gs_status;

/* Optional out-parameter.  If non-NULL the call synchronises its stream. */
typedef struct {
    double   ram_fraction;          /* %RAM = (data bytes + workspace bytes) / data bytes */
    uint64_t workspace_bytes_used;  /* bytes of ws the call may touch */
    uint32_t levels;                /* merge levels (tree depth) of the largest sort done */
    uint32_t fallback;              /* learned: 1 the bucket table failed verification (order,
                                       overflow), 2 the sample predicted too uneven buckets,
                                       3 a buffer fraction below 0.5 */
    uint32_t overflow_buckets;      /* learned: buckets above the in-LDS capacity */
    uint32_t max_bucket;            /* learned: largest bucket (keys) */
    float    train_loss_first;      /* learned: training loss of the first / last step */
    float    train_loss_last;
    uint32_t feature;               /* learned: bit 0: 0 = linear in x, 1 = linear in the key bits;
                                       bit 1: the knot table is the sample's CDF (mode 2, or the
                                       trained table failed the sample screening) */
    uint32_t invalid_offsets;       /* segsort: 1 if the device check rejected the offsets */
    double   elapsed_ms;            /* wall time of the call measured with HIP events */
    uint32_t order;                 /* plain sorts: 0 sorted, 1 input already in order (nothing
                                       moved), 2 input strictly reversed (one reversal pass) */
    uint32_t heavy_values;          /* learned: key values of the sample's long runs of equal keys
                                       given buckets of their own (not sorted further) */
    uint64_t keys_moved;            /* plain sorts: element moves of the call (leaf stores, merge
                                       and concatenation stores, reversals), the bytes a pass
                                       writes divided by the element size */
} gs_report;

/* Parameters of the learned CDF bucket path (not from the paper). */
typedef struct {
    uint32_t num_buckets;    /* buckets, power of two in [2, 4096]; default 4096 */
    uint32_t sample_size;    /* keys sampled for training, in [1024, 2^24]; default 65536 */
    uint32_t train_steps;    /* Adam steps; default 8 */
    uint32_t batch;          /* minibatch per step, multiple of 32 in [32, 8192]; default 2048 */
    uint32_t knots;          /* knots of the tabulated model, in [2, 16384]; default 4096 */
    float    lr;             /* Adam learning rate; default 4e-2 */
    uint64_t seed;           /* sample positions, weight init and minibatches */
    uint32_t mode;           /* 0 = trained network, 1 = untrained linear CDF (table[i] = i/knots),
                                2 = the sorted sample's CDF at the knots (no network) */
    uint32_t screen;         /* 0 = trained mode screens its table on the sample before any key
                                moves (default); 1 = skip that early screening (the checks on
                                the full bucket totals still apply) */
    const float *weights_override;    /* device, 4353 floats: skip training, use these weights; may be NULL */
    const float *test_bucket_table;   /* device, `knots`+1 floats: raw table, bypasses the running max
                                         (test hook to force an order violation); may be NULL */
    double   buffer_fraction; /* 0 or >= 0.5 (default 0.5): the learned path, whose distribution
                                 passes write each half out of place into the half buffer;
                                 [1/64, 0.5): that buffer does not fit, and the call sorts with the
                                 plain path at this fraction instead (Frogsort3, as gs_sort_f64
                                 does; report.fallback = 3); below 1/64 GS_EUNSUPPORTED */
} gs_learned_params;

/* Fills `p` with the defaults above. */
void gs_learned_default_params(gs_learned_params *p);

/* Workspace sizes in bytes (0 for n <= 1); SIZE_MAX for invalid arguments. */
size_t gs_workspace_bytes_f64(int64_t n, double buffer_fraction);
size_t gs_workspace_bytes_kv(int64_t n, double buffer_fraction);
size_t gs_workspace_bytes_seg(int64_t num_keys, int64_t num_segments, double buffer_fraction);
size_t gs_workspace_bytes_learned(int64_t n, const gs_learned_params *p);

/* Stable ascending sort of n float64 keys in place ("Frogsort1").  The top
   merge writes the result straight into `keys`; ws holds the floor(n/2)
   half buffer.  Every plain sort (these, the targets, the _ex calls) first
   checks on the device whether the keys are already in order (then nothing
   moves) or strictly reversed (then one reversal pass is the whole sort):
   the bi-adaptivity of "Octosort" and "Squidsort" at the level of the whole
   array; 4096 sampled pairs keep the check to one small launch on other
   input. */
gs_status gs_sort_f64(double *keys, int64_t n, double buffer_fraction,
                      void *ws, size_t ws_bytes, void *hip_stream, gs_report *rep);

/* gs_sort_f64 at buffer_fraction 0.5 that allocates nothing and takes no
   workspace: for callers that cannot allocate device memory (code under HIP
   graph capture, tight serving loops, harnesses that forbid allocation).  The
   half buffer and control area live in a static device array of
   GS_NOALLOC_SCRATCH_BYTES that every device the library runs on holds until
   the process ends; n above GS_NOALLOC_MAX_KEYS -> GS_EINVAL with nothing
   enqueued.  Same result, order check and error reporting (gs_device_errors)
   as gs_sort_f64; asynchronous on `hip_stream`.  All calls on one device share
   that device's array: two calls that can overlap on one device (different
   streams, or host threads without ordering) race and give wrong results;
   calls ordered on one stream are safe.  The array is not cleared between
   calls and needs no clearing: each call initialises what it reads. */
#define GS_NOALLOC_MAX_KEYS ((int64_t)1 << 22)
#define GS_NOALLOC_SCRATCH_BYTES ((int64_t)17 << 20)
gs_status gs_sort_f64_noalloc(double *keys, int64_t n, void *hip_stream);

/* Stable ascending sort of n uint64 keys; vals[i] (uint32) travels with
   keys[i].  Stability is observable through vals ("Stability"). */
gs_status gs_sort_kv(uint64_t *keys, uint32_t *vals, int64_t n, double buffer_fraction,
                     void *ws, size_t ws_bytes, void *hip_stream, gs_report *rep);

/* The four stable targets ("Definition of sorting"): keys ascending (Asc) or
   descending (Desc); tied keys in input order (Left, read from the left) or in
   reverse input order (Right, read from the right).  DescLeft is sorted
   directly (the greater key first, ties in input order); AscRight and
   DescRight are DescLeft and AscLeft read backwards (one extra reversal
   pass).  AscLeft is gs_sort_f64 / gs_sort_kv.  Same workspace as those. */
typedef enum { GS_ASC_LEFT = 0, GS_ASC_RIGHT = 1, GS_DESC_LEFT = 2, GS_DESC_RIGHT = 3 } gs_target;
gs_status gs_sort_f64_target(double *keys, int64_t n, int target, double buffer_fraction,
                             void *ws, size_t ws_bytes, void *hip_stream, gs_report *rep);
gs_status gs_sort_kv_target(uint64_t *keys, uint32_t *vals, int64_t n, int target, double buffer_fraction,
                            void *ws, size_t ws_bytes, void *hip_stream, gs_report *rep);

/* The same with the tree named (sections "Frogsort1", "Frogsort2",
   "Frogsort3 and 6").  GS_ALGO_AUTO is what the calls above run: Frogsort1 for
   p >= 0.5, Frogsort3 below.  GS_ALGO_FROGSORT1 with p < 0.5 -> GS_EINVAL;
   the others with p >= 0.5 run their own tree at p = 0.5 (Frogsort3 is then
   one Frogsort1 tree).  Frogsort6 shares the buffer like Frogsort3 but its
   sub-trees are Frogsort2 trees at sub_fraction (rounded down to a multiple
   of 1/65536; >= 0.5 is Frogsort3, <= buffer_fraction a single Frogsort2
   tree); sub_fraction is ignored by the other trees.  The workspace depends
   on the tree: size it with the _ex queries.  rep->levels counts every merge
   round of the call. */
typedef enum {
    GS_ALGO_AUTO = 0,
    GS_ALGO_FROGSORT1 = 1,
    GS_ALGO_FROGSORT2 = 2,
    GS_ALGO_FROGSORT3 = 3,
    GS_ALGO_FROGSORT6 = 4
} gs_algo;
size_t gs_workspace_bytes_f64_ex(int64_t n, double buffer_fraction, int algo, double sub_fraction);
size_t gs_workspace_bytes_kv_ex(int64_t n, double buffer_fraction, int algo, double sub_fraction);
gs_status gs_sort_f64_ex(double *keys, int64_t n, int target, double buffer_fraction, int algo,
                         double sub_fraction, void *ws, size_t ws_bytes, void *hip_stream, gs_report *rep);
gs_status gs_sort_kv_ex(uint64_t *keys, uint32_t *vals, int64_t n, int target, double buffer_fraction, int algo,
                        double sub_fraction, void *ws, size_t ws_bytes, void *hip_stream, gs_report *rep);

/* Sort every segment keys[offsets[i], offsets[i+1]) on its own, for
   i in [0, num_segments); `offsets` holds num_segments+1 int64 values (device).
   Offsets must be non-decreasing with offsets[0] >= 0 and
   offsets[num_segments] <= num_keys; keys outside every segment are untouched.
   The offsets are checked on the device: on a violation nothing is written and
   the report (if any) shows invalid_offsets = 1 and the call returns GS_EINVAL;
   without a report the call returns GS_OK and the keys are left unchanged.
   Every segment first gets the order check of the plain path ("Octosort",
   "Squidsort"): one already in order is left as it is, one whose neighbours
   all strictly decrease (or do not increase and tie only bit-identical keys)
   is reversed in place -- in both cases the stable result -- and only the
   others are sorted.
   buffer_fraction >= 0.5: every segment is frog-sorted (Frogsort1) with a
   half buffer of its own, all in one pass.  buffer_fraction p in [1/64, 0.5):
   one buffer of floor(q num_keys / 2^16) doubles (q = floor(65536 p)) serves
   the segments in turn, the way Frogsort3 lets one buffer serve its branches
   in turn ("Frogsort3 and 6"): each pass takes consecutive segments while the
   half buffers of its long ones (placed side by side) fit, and a segment whose
   own half buffer does not fit is sorted alone by the plain sort (Frogsort3)
   with the largest fraction whose buffer fits.  Such a call first copies the
   offsets to the host (it waits for the stream's earlier work), checks them
   there (a violation returns GS_EINVAL before anything runs, with
   invalid_offsets = 1 in the report), and returns GS_EUNSUPPORTED while the
   stream is capturing a graph. */
gs_status gs_segsort(double *keys, int64_t num_keys, const int64_t *offsets,
                     int64_t num_segments, double buffer_fraction,
                     void *ws, size_t ws_bytes, void *hip_stream, gs_report *rep);

/* Shape of a segmented sort (the result does not depend on it).  Segments of
   at most short_threads * short_ipt keys are sorted in LDS, several per
   work-group; longer ones are frog-sorted together, their merges cut into
   tiles of 256 * merge_ipt outputs. */
typedef struct {
    uint32_t short_threads;  /* work-group size of the short-segment sort */
    uint32_t short_ipt;      /* keys per thread of the short-segment sort */
    uint32_t merge_ipt;      /* merge outputs per thread of the long segments (8 or 16) */
    uint32_t reserved;       /* 0 */
} gs_seg_config;

/* The shapes gs_segsort_autotune tries (count, then the i-th) and the one
   gs_segsort uses. */
int gs_seg_config_count(void);
gs_status gs_seg_config_get(int i, gs_seg_config *out);
void gs_seg_default_config(gs_seg_config *out);

/* gs_workspace_bytes_seg covers every shape; this one a given shape. */
size_t gs_workspace_bytes_seg_ex(int64_t num_keys, int64_t num_segments, double buffer_fraction,
                                 const gs_seg_config *cfg);

/* gs_segsort with a given shape (host pointer; GS_EINVAL for a shape that is
   not one of gs_seg_config_get's). */
gs_status gs_segsort_ex(double *keys, int64_t num_keys, const int64_t *offsets, int64_t num_segments,
                        double buffer_fraction, const gs_seg_config *cfg, void *ws, size_t ws_bytes,
                        void *hip_stream, gs_report *rep);

/* Times every shape on the caller's input and returns the fastest in *best.
   keys (num_keys doubles) is only read: each timed run sorts a copy in
   `scratch` (num_keys doubles, device, caller-owned); ws is sized by
   gs_workspace_bytes_seg.  reps >= 1 runs per shape, the fastest counts;
   times_ms (host, gs_seg_config_count() floats, may be NULL) receives each
   shape's time.  Synchronises the stream; allocates no device memory. */
gs_status gs_segsort_autotune(const double *keys, int64_t num_keys, const int64_t *offsets,
                              int64_t num_segments, double *scratch, void *ws, size_t ws_bytes,
                              void *hip_stream, int reps, gs_seg_config *best, float *times_ms);

/* Tuning cache (host only): the shape gs_segsort_autotune found, kept per
   device architecture (e.g. "gfx950") and size class (floor(log2) of
   num_keys and of num_segments) for the life of the process.  gs_segsort and
   gs_segsort_ex without a shape use the cached shape of the current device's
   architecture and the call's size class when there is one and the workspace
   fits it (gs_workspace_bytes_seg covers every shape); the result never
   depends on the shape.  When the environment variable GS_TUNE_CACHE names a
   file, the cache is read from it on first use and written back (JSON:
   {"entries": [{"arch", "log2_keys", "log2_segments", "short_threads",
   "short_ipt", "merge_ipt"}, ...]}) after every tuning run. */
/* 1 and *out filled if the cache holds a shape for arch (NULL: the current
   device's) and the size class of (num_keys, num_segments), 0 if not, -1 on
   bad arguments. */
int gs_tune_cache_get(const char *arch, int64_t num_keys, int64_t num_segments, gs_seg_config *out);
/* Records a shape (one of gs_seg_config_get's; else GS_EINVAL). */
gs_status gs_tune_cache_put(const char *arch, int64_t num_keys, int64_t num_segments, const gs_seg_config *cfg);
/* Reads entries from a file written by gs_tune_cache_save (or the
   GS_TUNE_CACHE file) into the cache; returns the valid entries read, -1 if
   the file cannot be read.  Entries that are not valid shapes are skipped. */
int gs_tune_cache_load(const char *path);
/* Writes the whole cache; returns the entries written, -1 on failure. */
int gs_tune_cache_save(const char *path);
/* Empties the cache (GS_TUNE_CACHE is not read again). */
void gs_tune_cache_clear(void);

/* Stable ascending sort of n float64 keys with the same result as
   gs_sort_f64, using a small FP32 CDF network trained on the device to bucket
   the keys first.  The key-to-bucket map is verified monotone before any key
   moves; if it is not, or a bucket would exceed max(2^20, a quarter of its
   half), or the sample has no usable range, the plain path sorts the
   untouched input (report.fallback = 1).  Before that, the trained table
   buckets the sorted sample: a bucket predicted above max(2^19, 16 x the
   average) replaces the table by the sample's CDF at the knots, and if that
   one fails too (keys packed closer than a knot resolves) the call goes to
   the plain path at once (report.fallback = 2), as it does when a run of
   equal sample keys too long for one bucket is not among the heavy values.
   Heavy values: the values of the longest runs of equal keys in the sorted
   sample (at least 4 average buckets' share; at most 31 and num_buckets/8)
   get buckets of their own, which are not sorted (report.heavy_values).
   Unless the stream is capturing a graph, the call synchronises the stream
   once, after training, to read that decision and enqueue only the path that
   runs; under capture both paths are enqueued, gated on the device.  Inputs
   shorter than 4 * sample_size run the plain path directly.  Extra memory
   stays at the half buffer (plus per-tile digit counters and the network's
   state).  `p` is a host pointer (NULL = defaults). */
gs_status gs_learned_sort(double *keys, int64_t n, const gs_learned_params *p,
                          void *ws, size_t ws_bytes, void *hip_stream, gs_report *rep);

/* ---- device-side failures ------------------------------------------------ */
/* Some failures happen on the device after a call has returned GS_OK, since
   the calls are asynchronous:
     GS_DEVERR_WAIT     a bounded wait of the ordered-store protocol gave up
                        (the waiting work item stored anyway, so the output may
                        be wrong), or a work capacity of the device-side plan was
                        exceeded (that work was skipped); the in-place merges
                        make such an output unusable;
     GS_DEVERR_OFFSETS  a segmented sort rejected its offsets on the device
                        (nothing was written).
   A call made with a report synchronises and returns GS_EDEVICE (GS_EINVAL for
   offsets).  Every call, with or without a report, also ORs what it met into
   sticky flags kept in device memory, one set per device, for the life of the
   process; this needs no workspace and no allocation. */
#define GS_DEVERR_WAIT 1u
#define GS_DEVERR_OFFSETS 2u
/* Reads the flags of `device` into *flags and, with clear != 0, resets them.
   Synchronous copies: call it after synchronising the streams of the calls it
   is meant to cover.  GS_EINVAL for a device that does not exist. */
gs_status gs_device_errors(int device, uint32_t *flags, int clear);
/* Test hook, process-wide, for calls enqueued from now on: with on != 0 every
   bounded wait that checks another work item waits as usual and is then
   recorded as one that gave up, so the calls report GS_DEVERR_WAIT (and
   GS_EDEVICE with a report) while their output stays correct; 0 restores
   normal operation.  Returns the previous setting. */
int gs_test_fail_waits(int on);

const char *gs_status_string(gs_status s);
/* Detail of the last error on the calling thread (never NULL). */
const char *gs_last_error_detail(void);
/* Library version string, e.g. "0.1.0 gfx950". */
const char *gs_version(void);

/* ---- measurement ---------------------------------------------------------- */

/* Launch tracing for profiling tools: while enabled on the calling thread
   (on = 1), every kernel launch made by the calls above is bracketed by HIP
   events on the call's stream; with on = 2 only the merge launches are (the
   fewest events for timing the dominant kernel inside a timed run).  The
   events skip the system-scope fence, so they do not write back the caches
   between the launches they bracket.  Returns the previous setting. */
int gs_trace_enable(int on);
/* Streaming copy of n float64 values from src to dst (device, not
   overlapping), asynchronous on the stream: the empirical bandwidth ceiling a
   sorting pass is measured against (a pass reads and writes every key once;
   16-byte non-temporal loads and stores when both pointers are 16-byte
   aligned).  GS_EINVAL for n < 0 or a NULL pointer with n > 0. */
gs_status gs_copy_f64(const double *src, double *dst, int64_t n, void *hip_stream);
/* Waits for the recorded events, writes up to `max` records (host arrays):
   kinds[i] (0 fill, 1 leaf sort, 2 partition, 3 merge, 4 other, 5 dependency windows) and ms[i]
   (launch duration), clears the record list and returns the count written. */
int gs_trace_read(int *kinds, double *ms, int max);

/* ---- the CDF network on its own (device pointers; for tests and tools) --- */
/* Loss (mean squared error) and gradient of the 1-64-64-1 ReLU network
   (4353 parameters: W1[64] b1[64] W2[64*64] row-major b2[64] w3[64] b3) on a
   batch (multiple of 32) of inputs u and targets t; the reductions run in a
   fixed order.  work: (batch/32)*4354 floats. */
gs_status gs_mlp_loss_grad(const float *params, const float *u, const float *t, int batch,
                           float *grad, float *loss, void *work, size_t work_bytes, void *hip_stream);
/* `steps` Adam steps (beta 0.9/0.999, eps 1e-8) in place on params/m/v over
   `count` samples; full_batch = 1 takes the first `batch` samples every step,
   else 32 per work-group drawn by a seeded hash.  losses[0], losses[1]: mean
   loss of the first and last step.  work: (batch/32)*4354 floats + 256 bytes. */
gs_status gs_mlp_train(float *params, float *adam_m, float *adam_v, const float *u, const float *t,
                       int64_t count, int steps, int batch, float lr, uint64_t seed, int full_batch,
                       float *losses, void *work, size_t work_bytes, void *hip_stream);
/* y[i] = network(u[i]) for i < count. */
gs_status gs_mlp_forward(const float *params, const float *u, int64_t count, float *y, void *hip_stream);

/* ---- introspection for tests (host only, no device work) ---------------- */

/* Depth of the frog tree the plain path builds for n keys with leaves of at
   most the library's leaf size (elements); *leaf_max receives that size. */
int gs_plan_depth(int64_t n, int is_kv, int64_t *leaf_max);
/* Geometry of node `idx` at `depth` of the frog tree over n elements:
   out[0..4] = region start, data size, is_left, data start, input offset. */
void gs_plan_node(int64_t n, int depth, int64_t idx, int64_t *out);
/* The ordered-store protocol's windows, computed by the code the kernels run.
   Leaf `leaf` of the Frogsort1 tree of `depth` over n keys: lo_hi[0..1] =
   the leaf tickets (ticket = 2^depth - 1 - leaf index) whose input chunks its
   destination covers (empty when lo > hi).  Returns 0, -1 on bad arguments. */
int gs_plan_leaf_window(int64_t n, int depth, int64_t leaf, int64_t *lo_hi);
/* One merge: merge[0..6] = first run start, its size, second run start, its
   size, output start, written top-down (1) or bottom-up (0), which run lies
   inside the output (0 first at the output start, 1 second at its end, 2
   first at its end); kind 0 merge, 1 merge after turning a descending outer
   run around (turned: 1 once that has happened), 2 concatenation; dir_first /
   dir_second: 1 ascending, 2 descending runs; splits[0..tiles]: the merge-path
   splits at every tile boundary (first-view elements among the first
   j * tile outputs).  windows[2 t], windows[2 t + 1] = the tickets ticket t
   waits for before storing (tiles take tickets in write order).  Returns the
   number of tiles, -1 on bad arguments. */
int gs_plan_tile_windows(const int64_t *merge, int kind, int dir_first, int dir_second, int turned, int64_t tile,
                         const int64_t *splits, int64_t *windows);
/* The Frogsort2 tree for n keys at buffer_fraction (is_kv: the key/value leaf
   size): leaves[3*i..] = input offset, data start, length (input order);
   nodes[4*j..] = region start, elements, is_left, merge round; counts[0..6] =
   leaves, nodes, rounds, buffer elements, tiles and splits of the largest
   round, elements merged over all rounds.  Arrays are filled up to their
   capacities.  -1 on bad arguments. */
int gs_plan_frog2(int64_t n, double buffer_fraction, int is_kv, int64_t *leaves, int64_t max_leaves,
                  int64_t *nodes, int64_t max_nodes, int64_t *counts);
/* The Frogsort6 schedule (sub_fraction 0.5: Frogsort3): trees[4*i..] = root
   region start, elements, input offset, is_left (running order);
   spine[3*k..] = outer elements, inner start, inner elements (bottom up);
   leaves[3*i..] of every tree; counts[0..6] = trees, spine merges, leaves,
   merge rounds, buffer elements, b, elements merged over all rounds. */
int gs_plan_frog3(int64_t n, double buffer_fraction, double sub_fraction, int is_kv, int64_t *trees,
                  int64_t max_trees, int64_t *spine, int64_t max_spine, int64_t *leaves, int64_t max_leaves,
                  int64_t *counts);
/* The steps of gs_segsort at buffer_fraction < 0.5 with the default shape,
   for host offsets[0..num_segments] (checked as gs_segsort checks them):
   steps[3*i..] = first segment, one past the last, 1 if that one segment is
   sorted alone by the plain sort (0: a pass).  *buffer receives the buffer's
   elements.  Returns the number of steps (steps filled up to max_steps), -1
   on bad arguments or offsets, -2 for a fraction of 0.5 or more (one pass). */
int64_t gs_plan_seg_steps(const int64_t *offsets, int64_t num_segments, int64_t num_keys, double buffer_fraction,
                          int64_t *steps, int64_t max_steps, int64_t *buffer);

#ifdef __cplusplus
}
#endif

#endif /* GS_H */
