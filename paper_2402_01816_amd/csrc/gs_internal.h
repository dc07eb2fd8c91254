// Internal interface between the C ABI layer and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <vector>

#include "frog_geometry.h"

namespace gs {

// Index (in the ticket-counter block) of the word the kernels set when a
// bounded wait gave up or a work capacity was exceeded.  The clearing at the
// start of every forest run keeps it, so it collects every run of a call; the
// call clears it once when it starts (err_words_begin).
constexpr int kErrWord = 63;
// Words 60-61: elements moved by the call's leaf, merge and reversal launches
// (a 64-bit count, cleared by the plain sort's first kernel; kept across the
// runs of a call like the error word).
constexpr int kMovedWord = 60;
// Words 16 + r: set when a node of merge round r turns its outer run around
// first (Squidsort, the single Frogsort1 tree; rounds up to 40).
constexpr int kTurnWord0 = 16;
constexpr int kTurnRounds = 40;
// The word before it: the test setting of the bounded waits (bit 0: record
// every wait that checked another work item as failed).  Every forest run
// writes it from the host's setting.
constexpr int kTestWord = kErrWord - 1;

// Flags of the device-side failures a call can meet (gs_device_errors).
enum : unsigned { DEVERR_WAIT = 1u, DEVERR_OFFSETS = 2u };

// The error words of one call: cleared by err_words_begin before the call's
// first kernel; err_words_end ORs bit[i] into the device's sticky flags for
// every word that is set once the call's kernels have run.
struct ErrWords {
    unsigned *w[4];
    unsigned bit[4];
    int count;
    void add(unsigned *word, unsigned b)
    {
        if (count < 4) {
            w[count] = word;
            bit[count] = b;
            ++count;
        }
    }
};
hipError_t err_words_begin(const ErrWords &e, hipStream_t st);
hipError_t err_words_end(const ErrWords &e, hipStream_t st);
// The device's sticky flags (current device); read and optionally clear them.
hipError_t sticky_errors_read(unsigned *flags, bool clear);
// Test setting of the bounded waits (the value of kTestWord).
unsigned test_wait_word();
void set_test_wait_word(unsigned w);
// Clears a forest control block of `count` words except kTestWord, which
// gets the test setting, and kErrWord and the moved count, which are kept.
void launch_fill_ctrl(unsigned *ctrl, int64_t count, hipStream_t st);

// Control words of a forest run: the leaf ticket counter (word 0), the
// error word, and per merge round r >= 1 kMergeGroups ticket counters, each on
// its own 128-byte line starting at word 32 * (kMergeGroups * r + g).
#ifndef GS_MERGE_GROUPS
#define GS_MERGE_GROUPS 8
#endif
constexpr int kMergeGroups = GS_MERGE_GROUPS;
inline int64_t forest_ctrl_words(int rounds)
{
    return (int64_t)32 * kMergeGroups * ((rounds > 0 ? rounds : 1) + 1);
}

// Layout of the area a forest run (one or many frog trees) works in, from
// offset 0 of that area.
struct ForestPlan {
    int64_t max_probs;    // rows of the problem table (0: one problem given inline)
    int rounds;           // merge rounds launched
    int64_t leaf, tile;   // largest leaf, merge output tile (elements)
    int64_t stride;       // row length of the prefix tables
    int64_t max_tickets;  // work items of one merge round (capacity)
    int64_t max_status;   // status words (capacity over all rounds)
    int64_t max_splits;   // merge-path splits of one round (capacity)
    int64_t off_ctrl;     // forest_ctrl_words(rounds) words
    int64_t off_status;
    int64_t off_dirs;     // Squidsort run directions, heap order (dir_nodes bytes; 0 = none)
    int64_t off_modes;    // node modes of the current round (dir_nodes / 2 bytes)
    int64_t dir_nodes;
    int64_t off_splits;
    int64_t off_desc;     // tile descriptors of the current round
    int64_t off_samp;     // run samples, samp_slots key pairs (0 slots = none)
    int64_t samp_slots;
    int64_t off_probs;    // problem table (table runs only)
    int64_t off_tbase, off_sbase;   // per-round prefix rows (table runs only)
    int64_t off_f2, f2_bytes;       // Frogsort2 tree tables (imbalanced plans only)
    int64_t bytes;
};

// Frogsort2 ("Frogsort2": the inner child of a node of n elements takes
// floor(q n / 2^16) of them, q / 2^16 = p < 1/2, and the buffer shrinks to the
// same fraction).  The tree is irregular, so the host walks it once and the
// call uploads these tables into the workspace: the leaves in input order and
// the merge nodes grouped by height (round r merges every node of height r).
struct F2Tables {
    int64_t n, q, leaf, tile;
    int rounds;                          // height of the root
    int64_t nleaves, nnodes;
    int64_t max_tickets, max_splits;     // largest round
    int64_t merged;                      // elements merged over all rounds (sum of node sizes)
    std::vector<unsigned> rt, rs;        // tickets / splits per round (host copy)
    std::vector<char> blob;              // device image, offsets below
    int64_t off_leaf_c, off_leaf_d, off_node_s, off_node_n, off_node_tb, off_node_sb, off_rb, off_rt, off_rs;
};

// Frogsort3 ("Frogsort3 and 6": one buffer of b = floor(q n / 2^16) elements serves
// the branches in turn) and Frogsort6 (the same, switching to Frogsort2 trees
// at fraction q2 / 2^16 instead of Frogsort1; q2 = 2^15 is Frogsort3).  While
// a sub-tree over the m elements left would need more than b, the last b of
// them form an inner child, sorted by a sub-tree whose root is a right node
// with its region ending at slot m + b (its data land at [m, m + b)); then the
// rest is the same problem on m - b.  What remains (its sub-tree fits b, or it
// is a single leaf) is one sub-tree at slot 0, and the spine merges [0, m - b)
// with [m, m + b) into [0, m), bottom up.  Every sub-tree runs from F2Tables;
// all their tables go up in one image.
struct F3Plan {
    int64_t n, q, b, leaf, tile;
    int64_t q2;                                           // the sub-trees' split (2^15: Frogsort1)
    std::vector<std::shared_ptr<const F2Tables>> trees;   // in running order
    std::vector<int64_t> root_s, root_n, root_c;           // their roots: region start, size, input offset
    std::vector<int> root_left;
    std::vector<int64_t> tree_off;                        // their tables' offsets in `image`
    std::vector<FrogMerge> spine;                         // bottom up
    std::vector<char> image;
    int max_rounds;                                       // deepest tree
    int total_rounds;                                     // merge rounds of the whole sort
    int64_t max_tickets, max_splits, max_status;
    int64_t merged;                                       // elements merged (trees and spine)
};

enum : int { kAlgoFrog1 = 1, kAlgoFrog2 = 2, kAlgoFrog3 = 3 };

// Workspace layout and tree shape of one plain sort.
struct SortPlan {
    int64_t n;            // keys
    int64_t leaf;         // largest leaf (elements)
    int64_t tile;         // merge output tile (elements)
    int depth;            // number of merge rounds
    int64_t q;            // 0: Frogsort1; else Frogsort2 with inner child floor(q n / 2^16)
    int64_t hlen;         // buffer elements: floor(n/2), or floor(q n / 2^16)
    int64_t off_hkeys;    // buffer for keys
    int64_t off_hvals;    // buffer for values (kv only)
    int64_t off_forest;   // control area of the run
    ForestPlan forest;
    std::shared_ptr<const F2Tables> f2;   // Frogsort2 tables
    std::shared_ptr<const F3Plan> f3;     // Frogsort3 schedule
    int64_t off_order;    // the order check's two words (see ORD_*)
    int64_t bytes;        // total workspace
};

// The order check's decision (word 0 at off_order): sort, keys already in
// order, keys strictly reversed; candidate while the full check runs.
enum : unsigned { ORD_SORT = 0, ORD_IN_ORDER = 1, ORD_REVERSED = 2, ORD_CANDIDATE = 3 };

// Shape of a segmented sort: the work-group size and keys per thread of the
// batched short-segment sort (their product is the LDS tile and the length
// above which a segment goes to the forest) and the merge outputs per thread
// of the forest's merge tiles (256 threads).
struct SegConfig {
    int short_threads, short_ipt, merge_ipt;
};
int seg_config_count();
SegConfig seg_config_at(int i);
SegConfig seg_default_config();
bool seg_config_valid(const SegConfig &c);

// Workspace layout of one segmented sort.  With q = 0 every segment is
// sorted in one pass over a half buffer of floor(num_keys/2) doubles.  With a
// buffer fraction q/2^16 below one half the buffer holds
// floor(q num_keys / 2^16) doubles and serves runs of consecutive segments in
// turn (the passes of seg_schedule); a segment whose own half buffer does not
// fit is sorted alone by the plain sort (algo and q2 as for a plain sort at
// that fraction), which needs at most alone_bytes.
struct SegPlan {
    int64_t num_keys, nseg;
    SegConfig cfg;
    int64_t tile;         // keys per short LDS tile
    int64_t q;            // 0, or the buffer fraction q/2^16 < 1/2
    int algo;             // plain-sort algorithm of a segment sorted alone
    int64_t q2;           // its sub-fraction (Frogsort6)
    int64_t hlen;         // buffer elements
    int64_t pass_keys;    // most keys the long segments of one pass can hold
    int64_t alone_bytes;  // workspace of the largest segment sorted alone (0: none can be)
    int64_t off_h;        // the buffer: hlen doubles
    int64_t off_ctrl;     // 64 control words
    int64_t off_cls, off_rank, off_list;   // per-segment class, rank in class, class-ordered list
    int64_t off_maps;     // order-check range maps (2 bytes per range of keys)
    int64_t off_forest;   // forest area for the long segments of one pass
    ForestPlan forest;
    int64_t bytes;
};
SegPlan plan_seg(int64_t num_keys, int64_t nseg, const SegConfig &cfg, int64_t q = 0, int algo = 0,
                 int64_t q2 = 0);
// One step of a segmented sort with a buffer below one half: the segments
// [s0, s1) sorted together in one pass, the long ones' half buffers side by
// side in the buffer, or (alone) the one segment s0 too long for that, sorted
// by the plain sort.
struct SegStep {
    int64_t s0, s1;
    bool alone;
};
// The steps for host offsets off[0..nseg] (validated) and a buffer of hlen
// doubles: greedy, each pass taking consecutive segments while every long
// segment's half buffer, placed at (its first key - the pass's first key) / 2,
// ends within the buffer.
std::vector<SegStep> seg_schedule(const int64_t *off, int64_t nseg, int64_t tile, int64_t hlen);
// Runs the passes of a schedule (the steps that are not alone) with one
// error-word bracket; offsets stays the caller's device array, h_off is its
// host copy.
hipError_t segsort_passes_async(double *keys, const int64_t *offsets, const int64_t *h_off, const SegPlan &p,
                                const std::vector<SegStep> &steps, char *ws, hipStream_t st);
// Forest area for the long segments of up to nseg segments of at most max_len
// keys each, num_keys keys in total.
ForestPlan plan_forest_seg(int64_t num_keys, int64_t max_len, int64_t nseg);
hipError_t segsort_f64_async(double *keys, const int64_t *offsets, const SegPlan &p, char *ws,
                             hipStream_t st);
// The same with every buffer given: hbuf holds floor((offsets[nseg]-offsets[0])/2)
// doubles, ctrl 64 words, cls/rank/list nseg ints each, forest an area laid
// out by fp (from plan_forest_seg for these sizes).  With preset_codes the
// caller has written every segment's order code into rank[] (0: to be sorted,
// kSegDone: already in order) on the stream before the call.
constexpr int kSegDone = -1;
// Streaming copy of n doubles (16-byte non-temporal accesses when both
// pointers allow them); skipped on the device while *skip_if != 0.
hipError_t copy_f64_async(const double *src, double *dst, int64_t n, hipStream_t st,
                          const unsigned *skip_if = nullptr);
hipError_t segsort_core_async(double *keys, const int64_t *offsets, int64_t nseg, int64_t num_keys,
                              double *hbuf, unsigned *ctrl, int *cls, int *rank, int *list, char *forest,
                              const ForestPlan &fp, const unsigned *gate, unsigned run_if, hipStream_t st,
                              bool preset_codes = false);

struct Prob;
// Capacity of a forest area for up to max_probs f64 problems of at most
// max_len keys each, num_keys keys in total.
// merge_ipt: merge outputs per thread of the forest's 256-thread merge tiles
// (8 or 16).
ForestPlan plan_forest_f64(int64_t num_keys, int64_t max_len, int64_t max_probs, int merge_ipt = 16);
// Frog-sorts every problem of a device table (nprob: device word with the
// number of rows) over D (keys) and H (half buffers); area fw laid out by fp
// (planned with the same merge_ipt).
hipError_t forest_f64_async(double *D, double *H, const Prob *probs, const unsigned *nprob, const ForestPlan &fp,
                            char *fw, hipStream_t st, const unsigned *gate, unsigned run_if, int merge_ipt = 16);

// algo kAlgoFrog1: buffer floor(n/2) (q unused).  kAlgoFrog2 / kAlgoFrog3:
// the buffer fraction is q / 2^16, q in [kF2MinQ, 2^15]; kAlgoFrog3 with
// q2 < 2^15 is Frogsort6.
constexpr int64_t kF2MinQ = 1024;       // p >= 1/64
SortPlan plan_f64(int64_t n, int64_t q = 0, int algo = kAlgoFrog1, int64_t q2 = 32768);
SortPlan plan_kv(int64_t n, int64_t q = 0, int algo = kAlgoFrog1, int64_t q2 = 32768);
// Tables of the Frogsort2 tree over n elements, and the Frogsort3 / 6
// schedule (gs_plan.cpp; cached, immutable once built).
std::shared_ptr<const F2Tables> f2_tables(int64_t n, int64_t q, int64_t leaf, int64_t tile);
std::shared_ptr<const F3Plan> f3_plans(int64_t n, int64_t q, int64_t q2, int64_t leaf, int64_t tile);
// gate (may be null): every launch exits at once unless *gate == run_if.
hipError_t sort_f64_async(double *keys, int64_t n, char *ws, const SortPlan &p, hipStream_t st,
                          const unsigned *gate = nullptr, unsigned run_if = 0u);
hipError_t sort_kv_async(uint64_t *keys, uint32_t *vals, int64_t n, char *ws, const SortPlan &p,
                         hipStream_t st);
// Targets of "Definition of sorting": 0 AscLeft, 1 AscRight, 2 DescLeft,
// 3 DescRight (plan from plan_f64 / plan_kv: the shapes are shared).
hipError_t sort_f64_target_async(double *keys, int64_t n, int target, char *ws, const SortPlan &p, hipStream_t st);
hipError_t sort_kv_target_async(uint64_t *keys, uint32_t *vals, int64_t n, int target, char *ws, const SortPlan &p,
                                hipStream_t st);
void launch_fill_u32(unsigned *p, int64_t count, unsigned v, hipStream_t st);
// The error word of a plain plan's control area.
ErrWords plain_err_words(char *ws, const SortPlan &p);

// The static workspace of gs_sort_f64_noalloc (gs_noalloc.hip): the device
// address of the current device's copy, looked up on the first call there.
constexpr int64_t kNoAllocMaxKeys = (int64_t)1 << 22;
constexpr int64_t kNoAllocScratchBytes = (int64_t)17 << 20;
hipError_t noalloc_scratch(char **out);

// One explicit merge node over the logical space {D, H, n_space}, using the
// control area of a plain plan at least as large as the node.
hipError_t merge_one_f64_async(double *D, double *H, int64_t n_space, const FrogMerge &m, char *ws,
                               const SortPlan &p, hipStream_t st, const unsigned *gate, unsigned run_if);

// Launch tracing (measurement only).  When enabled on the calling thread,
// launchers bracket every kernel launch with HIP events on its stream.
enum TraceKind : int { TK_FILL = 0, TK_LEAF = 1, TK_PARTITION = 2, TK_MERGE = 3, TK_OTHER = 4, TK_DEPWIN = 5, TK_SEGSORT = 6,
                       TK_LEARN_PREP = 7, TK_LEARN_TRAIN = 8, TK_LEARN_BUCKET = 9 };
bool trace_on();
void trace_begin(int kind, hipStream_t st);
void trace_end(hipStream_t st);

}  // namespace gs
