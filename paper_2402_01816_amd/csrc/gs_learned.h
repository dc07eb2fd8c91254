// Learned CDF bucket path: plan, launcher and report.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gs.h"
#include "gs_internal.h"

namespace gs {

// Monotone feature phi(x) in [0,1] over the sample range (device struct).
struct Feature {
    double lo, hi, range;       // linear: (x - lo) * inv, inv = 1 / range
    double inv;
    uint64_t klo, khi;          // bits: (key(x) - klo) * kinv, kinv = 1 / krange
    double krange, kinv;
    double scale, kscale;       // G / range, G / krange (knot coordinates)
    int bits;                   // 1: use the key bits
    int valid;                  // 0: the sample gave no usable range
};

struct LearnedPlan {
    int64_t n, S;
    int B, G, batch;
    int use_learned;            // 0: input too small, the plain path runs
    int64_t limit;              // largest bucket the learned path accepts
    int64_t ntiles;             // tiles of one distribution pass
    SortPlan plain;             // plain plan (fallback, final-merge control words)
    SortPlan splan;             // plan of the sample sort
    int64_t off_sample, off_sample_ws, off_u, off_t, off_feat, off_ctrl;
    int64_t off_params, off_m, off_v, off_partial, off_losses, off_raw, off_tab;
    int64_t off_totals, off_starts, off_offsets, off_dstart, off_tilecnt;
    int64_t off_segctrl, off_seglists;
    int64_t off_heavy;          // the sample's heavy values (kHeavyMax doubles, ascending, NaN past the count)
    int64_t off_runs;           // the sample's long runs of equal keys (start, length)
    int64_t off_segforest;      // forest area of the bucket sorts (both halves in turn)
    ForestPlan segforest;
    int64_t bytes;
};

struct LearnedReport {
    unsigned fallback, order_violation, overflow_buckets, max_bucket, big_buckets, err, feature, heavy;
    float loss_first, loss_last;
};

LearnedPlan plan_learned(int64_t n, const gs_learned_params &prm);
hipError_t learned_sort_async(double *keys, int64_t n, const gs_learned_params &prm, char *ws,
                              const LearnedPlan &L, hipStream_t st);
hipError_t learned_read_report(const char *ws, const LearnedPlan &L, LearnedReport *r);
// After the stream is synchronised: the DEVERR_* flags of every error word
// of the call (0: none set).
hipError_t learned_errors(const char *ws, const LearnedPlan &L, unsigned *any);

}  // namespace gs
