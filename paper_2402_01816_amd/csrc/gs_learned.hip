// Learned CDF bucket path (not part of the paper): the same stable ascending
// result as the plain frog sort, with most merge levels replaced by two
// stable 64-way distribution passes and per-bucket sorts.
//
//   1. sample keys at strided positions, sort the sample with the plain path;
//   2. pick a monotone feature phi (linear in x, or linear in the key's
//      order-preserving bit pattern); from the ranks of the sorted sample, the
//      log of the sample's local density in phi: over a window of 2h ranks,
//      log(2h / (S * (phi[i+h] - phi[i-h])));
//   3. train the 1-64-64-1 network on the device to fit that log density
//      (its output layer starts at zero: an untrained network is the uniform
//      density, i.e. the linear CDF);
//   4. tabulate the CDF the network implies: the cumulative trapezoid
//      integral of exp(network) over G+1 knots, normalised to end at 1 --
//      monotone by construction, and its slope follows the estimated density,
//      which is what evens out the buckets;
//   5. bucket(x) = floor(B * interp(table, G * phi(x))): every step is monotone
//      non-decreasing in x, so a key in a higher bucket is strictly greater
//      than every key in a lower one; the table is checked for monotonicity
//      before any key moves (a non-monotone table -- only possible through the
//      test hook -- sends the call to the plain path on the untouched input);
//      values that fill long runs of the sorted sample (heavy values: equal
//      keys always share a bucket, so no network can spread them) get buckets
//      of their own, which need no sort -- the stable distribution leaves
//      their keys in input order;
//   6. bucket totals of both halves before any key moves (the overflow
//      check sends the call to the plain path on the untouched input); then
//      for the second half and then the first: per-tile digit counts, a
//      stable pass by the bucket id's low digit into the half buffer and one
//      by its high digit back, which leaves the half grouped by bucket in
//      input order, and every bucket frog-sorted in place with the half
//      buffer as its buffer;
//   7. the sorted first half moves into the half buffer, and one frog merge
//      (a right node: the second half is its outer run and stays or moves
//      left) writes the output bottom-up.
// Memory stays at the half buffer throughout.
#include <hip/hip_runtime.h>

#include "gs_block.h"
#include "gs_device.h"
#include "gs_internal.h"
#include "gs_learned.h"
#include "gs_mlp.h"

namespace gs {

namespace {

constexpr int FEAT_BINS = 4096;          // bins for choosing the feature
constexpr int kDensH = 32;               // half window (ranks) of the density targets
// A bucket larger than max(kBucketLimit, a quarter of its half) sends the call
// to the plain path: the network failed to spread the keys.
constexpr int64_t kBucketLimit = (int64_t)1 << 20;

// control words of the learned path
constexpr int L_FALLBACK = 0;            // 1: take the plain path
constexpr int L_ORDER = 1;               // table not monotone
constexpr int L_OVERFLOW = 2;            // buckets above the limit
constexpr int L_MAXB = 3;                // largest bucket
constexpr int L_ERR = 5;                 // training's error word (it has no waits: stays 0)
constexpr int L_BIGB = 6;                // buckets larger than one LDS tile
constexpr int L_FEAT = 7;                // chosen feature
constexpr int L_SCREENED = 8;              // the sample predicted too uneven buckets
constexpr int L_HEAVY = 9;                 // heavy values found in the sample
constexpr int L_RUNS = 10;                 // long runs of equal keys recorded in the sample
constexpr int L_RESCUE = 11;               // the trained table failed the screening: sample table
constexpr int L_SAMPTAB = 12;              // the knot table is the sample's CDF

// Heavy values: at most kHeavyMax, kept ascending in kHeavySlots doubles with
// NaN past the count (a NaN slot compares as greater than every key).  A
// heavy value fills a run of at least kHeavySkew x the average bucket's share
// of the sorted sample.
#ifndef GS_HEAVY_SLOTS
#define GS_HEAVY_SLOTS 32
#endif
constexpr int kHeavySlots = GS_HEAVY_SLOTS;              // a power of two
static_assert((kHeavySlots & (kHeavySlots - 1)) == 0 && kHeavySlots <= 256, "heavy slots");
constexpr int kHeavyMax = kHeavySlots - 1;
constexpr int64_t kHeavySkew = 4;
constexpr int kHeavyCand = 256;           // long runs of the sample recorded at most

// The plain path screens the learned form before any key moves: a bucket
// predicted (from the sample, scaled to a half) above max(kScreenMin, 16 x the
// average bucket) means the network did not spread the keys well enough for
// the bucket sorts to beat the merge passes they replace.
constexpr int64_t kScreenMin = (int64_t)1 << 19;
constexpr int64_t kScreenSkew = 16;

__device__ __forceinline__ uint64_t mix64d(uint64_t z)
{
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Order-preserving integer image of a float64 key under the sort's
// comparison: -0 and +0 map together, every NaN maps to the maximum.
__device__ __forceinline__ uint64_t ckey(double x)
{
    uint64_t u = (uint64_t)__double_as_longlong(x);
    u = (u << 1) == 0 ? 0ull : u;
    const uint64_t m = (u >> 63) ? ~u : (u | (1ull << 63));
    return x != x ? ~0ull : m;
}

__device__ __forceinline__ double phi_of(double x, const Feature &F)
{
    if (F.bits) {
        const uint64_t k = ckey(x);
        const double num = k >= F.klo ? (double)(k - F.klo) : -(double)(F.klo - k);
        return num * F.kinv;
    }
    return (x - F.lo) * F.inv;
}

// With hc heavy values h_1 < ... < h_hc (hv, ascending), key x's bucket is
// its table bucket t(x) (the table spread over B - 2 hc buckets) plus
// c(x) + c'(x), where c(x) counts the heavy values at or below x and c'(x)
// those below it.  That stays monotone (t and both counts are), gives h_k the
// bucket t(h_k) + 2k - 1, and no other key can land there: a key below h_k
// has at most k - 1 heavy values at or below it and t no larger, a key above
// it at least k and t no smaller, and both offsets 2c are even.
// heavy_shift returns c(x) + c'(x) (x not NaN): a search over the kHeavySlots
// slots in powers of two, the NaN slots past the count never at or below x.
__device__ __forceinline__ int heavy_shift(double x, const double *hv)
{
    int pos = 0;
#pragma unroll
    for (int step = kHeavySlots / 2; step >= 1; step >>= 1) pos += hv[pos + step - 1] <= x ? step : 0;
    const bool eq = pos > 0 && hv[pos - 1] == x;
    return 2 * pos - (eq ? 1 : 0);
}

// Bucket of key x.  Monotone non-decreasing in x whenever `tab` is
// non-decreasing: the knot coordinate u is monotone (correctly rounded
// subtraction, conversion, multiplication by a positive constant and
// rounding to float), the knot index and the fraction are monotone in u, the
// interpolation is clamped to the next knot.  NaN keys take the last bucket
// (they sort last).  With heavy values (hc > 0) the table spreads over
// B - 2 hc buckets and heavy_shift places the rest.
// Knot coordinate of key x, clamped to [0, G] (a NaN coordinate becomes 0).
__device__ __forceinline__ float knot_coord(double x, const Feature &F, int G)
{
    float u;
    if (F.bits) {
        const uint64_t k = ckey(x);
        const uint64_t dk = k > F.klo ? k - F.klo : 0ull;
        u = (float)((double)dk * F.kscale);
    } else {
        u = (float)((x - F.lo) * F.scale);
    }
    return fminf(fmaxf(u, 0.f), (float)G);
}

__device__ __forceinline__ int bucket_of(double x, const Feature &F, const float *tab, int G, int B,
                                         const double *hv = nullptr, int hc = 0)
{
    // knot index and fraction
    const float uc = knot_coord(x, F, G);
    const int i = min((int)uc, G - 1);
    const float f = uc - (float)i;
    const float a = tab[i], b = tab[i + 1];
    const float v = fminf(fmaf(f, b - a, a), b);
    const int Bt = B - 2 * hc;
    int bk = (int)(v * (float)Bt);
    bk = bk < 0 ? 0 : (bk > Bt - 1 ? Bt - 1 : bk);
    if (hc > 0 && x == x) bk += heavy_shift(x, hv);
    return x != x ? B - 1 : bk;
}

// bucket_of for N keys at once, step for step the same arithmetic: every
// knot coordinate first, then all table reads, then the interpolations, so
// that the keys' LDS reads are in flight together.
template <int N>
__device__ __forceinline__ void buckets_of(const double *x, int *bk, const Feature &F, const float *tab, int G, int B,
                                           const double *hv = nullptr, int hc = 0)
{
    float uc[N];
    if (F.bits) {
#pragma unroll
        for (int r = 0; r < N; ++r) {
            const uint64_t k = ckey(x[r]);
            const uint64_t dk = k > F.klo ? k - F.klo : 0ull;
            const float u = (float)((double)dk * F.kscale);
            uc[r] = fminf(fmaxf(u, 0.f), (float)G);
        }
    } else {
#pragma unroll
        for (int r = 0; r < N; ++r) {
            const float u = (float)((x[r] - F.lo) * F.scale);
            uc[r] = fminf(fmaxf(u, 0.f), (float)G);
        }
    }
    int ix[N];
    float a[N], b[N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        ix[r] = min((int)uc[r], G - 1);
        a[r] = tab[ix[r]];
        b[r] = tab[ix[r] + 1];
    }
    const int Bt = B - 2 * hc;
#pragma unroll
    for (int r = 0; r < N; ++r) {
        const float f = uc[r] - (float)ix[r];
        const float v = fminf(fmaf(f, b[r] - a[r], a[r]), b[r]);
        int k = (int)(v * (float)Bt);
        k = k < 0 ? 0 : (k > Bt - 1 ? Bt - 1 : k);
        bk[r] = k;
    }
    if (hc > 0) {
#pragma unroll
        for (int r = 0; r < N; ++r)
            if (x[r] == x[r]) bk[r] += heavy_shift(x[r], hv);
    }
#pragma unroll
    for (int r = 0; r < N; ++r) bk[r] = x[r] != x[r] ? B - 1 : bk[r];
}

}  // namespace

// ---------------------------------------------------------------------------
// 1. sample: key j*stride + hash(seed, j) mod stride for j < S
// ---------------------------------------------------------------------------
__global__ void learned_sample_kernel(const double *keys, int64_t n, int64_t S, uint64_t seed, double *out)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= S) return;
    const int64_t stride = n / S;
    const uint64_t h = mix64d(seed ^ (0x9E3779B97F4A7C15ull * (uint64_t)(j + 1)));
    out[j] = keys[j * stride + (int64_t)(h % (uint64_t)stride)];
}

// ---------------------------------------------------------------------------
// 2. feature choice, training inputs and targets from the sorted sample
// ---------------------------------------------------------------------------
// One work-group of 1024 threads.  lo/hi: smallest and largest non-NaN sample
// key.  The feature whose FEAT_BINS-bin histogram of the sample has the
// smaller largest bin wins (ties: linear).  (The training inputs and targets
// follow in learned_targets_kernel.)
//
// The sorted sample's runs of equal keys come first.  A run of at least
// kHeavySkew x the average bucket's share of the sample is a heavy value:
// equal keys always share a bucket, so no network can spread them, and the
// kHeavyMax longest (NaN excepted) get buckets of their own (hv, ascending,
// NaN past the count; the count in ctrl[L_HEAVY]), which need no sort.  Every
// such run found (at most kHeavyCand) is recorded for the density targets
// (runs: start, length; the count in ctrl[L_RUNS]).  With `screen_half` > 0 (the half size the screening scales to) a run that is not
// among them -- or NaNs -- long enough that it alone scales past the screening
// limit sends the call to the plain path before any training (the training
// and tabulation launches are gated on the fallback word).
__global__ __launch_bounds__(1024) void learned_prep_kernel(const double *xs, int64_t S, int G, Feature *feat,
                                                            unsigned *ctrl, int64_t screen_half, int B, double *hv,
                                                            int64_t *runs)
{
    {
        __shared__ unsigned s_cnt, s_fail;
        __shared__ int64_t s_len[kHeavyCand], s_start[kHeavyCand];
        __shared__ double s_val[kHeavyCand];
        const int64_t half = screen_half > 0 ? screen_half : S;
        const int64_t avg = half / B;
        const int64_t limit = kScreenSkew * avg > kScreenMin ? kScreenSkew * avg : kScreenMin;
        // shortest run whose scaled size run * half / S exceeds the limit
        const int64_t m = ((limit + 1) * S + half - 1) / half;
        // shortest heavy run
        int64_t mh = (kHeavySkew * S + B - 1) / B;
        mh = mh < 2 ? 2 : mh;
        if (threadIdx.x == 0) s_cnt = s_fail = 0u;
        __syncthreads();
        auto same = [&](double a, double b) { return a == b || (a != a && b != b); };
        for (int64_t i = threadIdx.x; i + mh - 1 < S; i += 1024) {
            // a long run starting here: measure it (its end by binary search)
            if (same(xs[i], xs[i + mh - 1]) && (i == 0 || !same(xs[i - 1], xs[i]))) {
                int64_t lo = i + mh - 1, hi = S;         // last index of the run: lo
                while (hi - lo > 1) {
                    const int64_t mid = (lo + hi) >> 1;
                    if (same(xs[i], xs[mid])) lo = mid;
                    else hi = mid;
                }
                const int64_t len = lo - i + 1;
                if (xs[i] != xs[i]) {
                    if (screen_half > 0 && len >= m) atomicOr(&s_fail, 1u);
                } else {
                    const unsigned c = atomicAdd(&s_cnt, 1u);
                    if (c < (unsigned)kHeavyCand) {
                        s_len[c] = len;
                        s_start[c] = i;
                        s_val[c] = xs[i];
                    }
                }
            }
        }
        __syncthreads();
        const int nc = s_cnt < (unsigned)kHeavyCand ? (int)s_cnt : kHeavyCand;
        const int hmax = kHeavyMax < B / 8 ? kHeavyMax : B / 8;
        const int hc = nc < hmax ? nc : hmax;
        // the hmax longest runs: candidate c's place among all by length
        // (longer first, ties by the smaller value: the choice does not depend
        // on the order the candidates were recorded in), then the chosen ones'
        // place by value (candidates hold distinct values)
        __shared__ int s_pick[kHeavyCand];
        __shared__ int64_t s_rest;
        if (threadIdx.x == 0) s_rest = 0;
        __syncthreads();
        for (int c = threadIdx.x; c < nc; c += 1024) {
            runs[2 * c] = s_start[c];
            runs[2 * c + 1] = s_len[c];
            int place = 0;
            for (int e = 0; e < nc; ++e)
                place += (s_len[e] > s_len[c] || (s_len[e] == s_len[c] && s_val[e] < s_val[c])) ? 1 : 0;
            s_pick[c] = place;
            if (place >= hc) atomicMax((unsigned long long *)&s_rest, (unsigned long long)s_len[c]);
        }
        __syncthreads();
        for (int c = threadIdx.x; c < nc; c += 1024) {
            if (s_pick[c] >= hc) continue;
            int place = 0;
            for (int e = 0; e < nc; ++e) place += (s_pick[e] < hc && s_val[e] < s_val[c]) ? 1 : 0;
            hv[place] = s_val[c];
        }
        for (int c = hc + (int)threadIdx.x; c < kHeavySlots; c += 1024) hv[c] = __builtin_nan("");
        if (threadIdx.x == 0) {
            ctrl[L_RUNS] = (unsigned)nc;
            const int64_t rest = s_rest;                // longest run left out
            const bool lost = s_cnt > (unsigned)kHeavyCand;   // candidates not recorded
            ctrl[L_HEAVY] = (unsigned)hc;
            if (screen_half > 0 && (s_fail || lost || rest >= m)) {
                const int64_t worst = rest > m ? rest : m;
                const int64_t predicted = worst * screen_half / S;
                ctrl[L_SCREENED] = 1u;
                ctrl[L_MAXB] = (unsigned)(predicted < 0xffffffffll ? predicted : 0xffffffffll);
                ctrl[L_FALLBACK] = 1u;
            }
        }
        __syncthreads();
    }
    __shared__ unsigned h_lin[FEAT_BINS], h_bits[FEAT_BINS];
    __shared__ int64_t s_nn;
    __shared__ unsigned s_max[2];
    const int tid = threadIdx.x;
    for (int i = tid; i < FEAT_BINS; i += 1024) h_lin[i] = h_bits[i] = 0u;
    if (tid == 0) {
        int64_t lo = 0, hi = S;                    // first NaN (NaNs sort last)
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (xs[mid] != xs[mid]) hi = mid;
            else lo = mid + 1;
        }
        s_nn = lo;
        s_max[0] = s_max[1] = 0u;
    }
    __syncthreads();
    const int64_t nn = s_nn;
    Feature F{};
    F.valid = 0;
    if (nn > 0) {
        F.lo = xs[0];
        F.hi = xs[nn - 1];
        F.range = F.hi - F.lo;
        F.klo = ckey(F.lo);
        F.khi = ckey(F.hi);
        F.krange = (double)(F.khi - F.klo);
        F.inv = 1.0 / F.range;
        F.kinv = 1.0 / F.krange;
        F.scale = (double)G / F.range;
        F.kscale = (double)G / F.krange;
    }
    const bool lin_ok = nn > 0 && F.range > 0.0 && F.range < __builtin_inf() && F.inv < __builtin_inf() &&
                        F.scale < __builtin_inf();
    const bool bits_ok = nn > 0 && F.khi > F.klo;
    for (int64_t i = tid; i < nn; i += 1024) {
        if (lin_ok) {
            F.bits = 0;
            int b = (int)(phi_of(xs[i], F) * FEAT_BINS);
            b = b < 0 ? 0 : (b >= FEAT_BINS ? FEAT_BINS - 1 : b);
            atomicAdd(&h_lin[b], 1u);
        }
        if (bits_ok) {
            F.bits = 1;
            int b = (int)(phi_of(xs[i], F) * FEAT_BINS);
            b = b < 0 ? 0 : (b >= FEAT_BINS ? FEAT_BINS - 1 : b);
            atomicAdd(&h_bits[b], 1u);
        }
    }
    __syncthreads();
    for (int i = tid; i < FEAT_BINS; i += 1024) {
        atomicMax(&s_max[0], h_lin[i]);
        atomicMax(&s_max[1], h_bits[i]);
    }
    __syncthreads();
    if (tid == 0) {
        F.valid = (lin_ok || bits_ok) ? 1 : 0;
        F.bits = (!lin_ok || (bits_ok && s_max[1] < s_max[0])) ? 1 : 0;
        *feat = F;
        ctrl[L_FEAT] = (unsigned)F.bits;
    }
}

// Training input of sample key i: phi (NaN keys at the top), clamped to
// [0, 1] and rounded to float.
__device__ __forceinline__ float train_input(double x, const Feature &F)
{
    double p = F.valid ? phi_of(x, F) : 0.0;
    if (x != x) p = 1.0;
    p = p < 0.0 ? 0.0 : (p > 1.0 ? 1.0 : p);
    return (float)p;
}

// Inputs and log-density targets, one thread per sample key: the sample keys
// in a window of +-kDensH ranks over the width of their inputs (the two ends'
// inputs recomputed from their keys, so no pass waits on another).  The runs
// of equal keys recorded by the prep kernel do not count: a run is a point
// mass that no density expresses (its keys share one bucket whatever the
// table does), and counted it would crowd the rest of the table.  A key
// inside a run takes the window around the whole run, so the run's value
// gets the density of the keys next to it.  Without runs this is the plain
// window density.
__global__ __launch_bounds__(256) void learned_targets_kernel(const double *xs, int64_t S, const Feature *feat,
                                                              float *u, float *t, const int64_t *runs,
                                                              const unsigned *ctrl)
{
    __shared__ int64_t s_run[2 * kHeavyCand];
    const unsigned nrec = ctrl[L_RUNS];
    const int nr = nrec < (unsigned)kHeavyCand ? (int)nrec : kHeavyCand;
    for (int k = threadIdx.x; k < 2 * nr; k += blockDim.x) s_run[k] = runs[k];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S) return;
    const Feature F = *feat;
    u[i] = train_input(xs[i], F);
    int64_t lo = i - kDensH, hi = i + kDensH, in_runs = 0;
    for (int k = 0; k < nr; ++k) {
        const int64_t st = s_run[2 * k], ln = s_run[2 * k + 1];
        in_runs += ln;
        if (i >= st && i < st + ln) {
            lo = st - kDensH;
            hi = st + ln - 1 + kDensH;
        }
    }
    lo = lo > 0 ? lo : 0;
    hi = hi < S - 1 ? hi : S - 1;
    // sample keys in [lo, hi) outside the runs
    int64_t cnt = hi - lo;
    for (int k = 0; k < nr; ++k) {
        const int64_t st = s_run[2 * k], en = st + s_run[2 * k + 1];
        const int64_t a = st > lo ? st : lo, b = en < hi ? en : hi;
        cnt -= b > a ? b - a : 0;
    }
    const int64_t rest = S - in_runs > 1 ? S - in_runs : 1;
    double w = (double)train_input(xs[hi], F) - (double)train_input(xs[lo], F);
    w = w > 1e-7 ? w : 1e-7;
    t[i] = (float)log((double)(cnt > 1 ? cnt : 1) / ((double)rest * w));
}

// ---------------------------------------------------------------------------
// 4. knot table: normalised cumulative integral of exp(network) (or the
//    linear CDF, or the sample's own CDF, or the raw test table); verified
//    monotone
// ---------------------------------------------------------------------------
// The sample's CDF at the knots: table[i] is the share of the sample keys
// whose knot coordinate lies below i, counted without NaNs and without the
// heavy values' runs (their keys have buckets of their own), so the keys of
// every knot interval spread evenly over the table's share of buckets.  The
// other long runs count: each keeps the table's room for its keys, which
// stops two of them close in value from sharing a bucket.  Monotone by
// construction (counts of a sorted sample below rising bounds).  With
// `rescue` the kernel runs only if the screening rejected the trained table.
// Sets ctrl[L_SAMPTAB].
__global__ __launch_bounds__(1024) void learned_sample_table_kernel(const double *xs, int64_t S, const Feature *feat,
                                                                    int G, float *tab, const int64_t *runs,
                                                                    const double *hv, unsigned *ctrl, int rescue)
{
    __shared__ int64_t s_run[2 * kHeavyCand];     // the heavy values' runs: start, length
    __shared__ int64_t s_nn;
    __shared__ unsigned s_nh;
    if (ctrl[L_FALLBACK] || (rescue && !ctrl[L_RESCUE])) return;
    const int tid = threadIdx.x;
    const unsigned nrec = ctrl[L_RUNS];
    const int nrall = nrec < (unsigned)kHeavyCand ? (int)nrec : kHeavyCand;
    const int hc = (int)ctrl[L_HEAVY];
    if (tid == 0) s_nh = 0u;
    __syncthreads();
    for (int k = tid; k < nrall; k += 1024) {
        const int64_t st = runs[2 * k];
        bool heavy = false;
        for (int h = 0; h < hc; ++h) heavy = heavy || hv[h] == xs[st];
        if (heavy) {
            const unsigned slot = atomicAdd(&s_nh, 1u);
            s_run[2 * slot] = st;
            s_run[2 * slot + 1] = runs[2 * k + 1];
        }
    }
    if (tid == 0) {
        int64_t a = 0, b = S;                      // first NaN (NaNs sort last)
        while (a < b) {
            const int64_t m = (a + b) >> 1;
            if (xs[m] != xs[m]) b = m;
            else a = m + 1;
        }
        s_nn = a;
    }
    __syncthreads();
    const Feature F = *feat;
    const int64_t nn = s_nn;
    const int nr = (int)s_nh;
    auto outside = [&](int64_t j) {               // keys of [0, j) in no heavy value's run
        int64_t c = j;
        for (int k = 0; k < nr; ++k) {
            const int64_t st = s_run[2 * k], en = st + s_run[2 * k + 1];
            const int64_t e = en < j ? en : j;
            c -= e > st ? e - st : 0;
        }
        return c;
    };
    const int64_t total = outside(nn);
    if (tid == 0) ctrl[L_SAMPTAB] = 1u;
    for (int i = tid; i <= G; i += 1024) {
        int64_t a = 0, b = nn;                     // first key with coordinate >= i
        while (a < b) {
            const int64_t m = (a + b) >> 1;
            if (knot_coord(xs[m], F, G) < (float)i) a = m + 1;
            else b = m;
        }
        tab[i] = i == G || total <= 0 ? (i == G ? 1.0f : 0.0f) : (float)((double)outside(a) / (double)total);
    }
}

__global__ __launch_bounds__(1024) void learned_table_kernel(const float *raw, const float *test_table, int mode,
                                                             int G, float *tab, unsigned *ctrl, const Feature *feat)
{
    __shared__ double s_part[1024];
    __shared__ float s_mx[1024];
    __shared__ unsigned s_bad;
    if (ctrl[L_FALLBACK]) return;        // screened out before training
    const int tid = threadIdx.x;
    const int cnt = G + 1;
    const int per = (cnt + 1023) / 1024;
    const int b0 = tid * per, b1 = b0 + per < cnt ? b0 + per : cnt;
    if (tid == 0) s_bad = 0u;
    if (test_table) {
        for (int i = b0; i < b1; ++i) tab[i] = test_table[i];
    } else if (mode == 1) {
        for (int i = b0; i < b1; ++i) tab[i] = (float)((double)i / (double)G);
    } else if (mode == 2) {
        // written by learned_sample_table_kernel: only verified here
    } else {
        // largest log density (NaN counts as very small)
        float mx = -3.0e38f;
        for (int i = b0; i < b1; ++i) {
            const float r = raw[i];
            if (r == r && r > mx) mx = r;
        }
        s_mx[tid] = mx;
        __syncthreads();
        if (tid == 0) {
            float m = s_mx[0];
            for (int k = 1; k < 1024; ++k) m = s_mx[k] > m ? s_mx[k] : m;
            s_mx[0] = m;
        }
        __syncthreads();
        const float top = s_mx[0];
        auto dens = [&](int i) -> double {
            const float r = raw[i];
            double e = (r == r) ? (double)(r - top) : -30.0;
            e = e < -30.0 ? -30.0 : (e > 0.0 ? 0.0 : e);
            return exp(e);
        };
        // trapezoid areas of the knot intervals ending at each knot, summed per
        // thread chunk, then an exclusive prefix over chunks
        double acc = 0.0;
        for (int i = b0; i < b1; ++i)
            if (i > 0) acc += 0.5 * (dens(i) + dens(i - 1));
        s_part[tid] = acc;
        __syncthreads();
        if (tid == 0)
            for (int k = 1; k < 1024; ++k) s_part[k] += s_part[k - 1];
        __syncthreads();
        const double total = s_part[1023];
        double run = tid > 0 ? s_part[tid - 1] : 0.0;
        for (int i = b0; i < b1; ++i) {
            if (i > 0) run += 0.5 * (dens(i) + dens(i - 1));
            tab[i] = i == G ? 1.0f : (float)(run / total);
        }
    }
    __syncthreads();
    __threadfence_block();
    for (int i = b0; i < b1; ++i) {
        const float a = tab[i];
        const bool ok = a >= 0.f && a <= 1.f && (i + 1 >= cnt || a <= tab[i + 1]);
        if (!ok) atomicOr(&s_bad, 1u);
    }
    __syncthreads();
    if (tid == 0) {
        if (s_bad) ctrl[L_ORDER] = 1u;
        if (s_bad || !feat->valid) ctrl[L_FALLBACK] = 1u;
    }
}

// ---------------------------------------------------------------------------
// 6a. digit counts per tile (and bucket totals) of one half
// ---------------------------------------------------------------------------
// Tiles are SW_TILE consecutive keys.  Every work-group takes tiles
// [blockIdx.x, blockIdx.x + gridDim.x, ...), counts the digit (bucket id >>
// shift, dbits bits) of each of its keys into tilecnt[d * ntiles + tile] and,
// if totals is given, every bucket id into a work-group histogram that is
// added into totals[] with integer atomics at the end (the totals do not
// depend on the order of the additions).
constexpr int SW_NT = 256;
// work-groups of a counting pass
#ifndef GS_LEARN_CGRID
#define GS_LEARN_CGRID 1024
#endif
// keys per thread of a tile: 14 (3584-key tiles) lets the distribution pass's
// knot table and staged tile fit three work-groups into a compute unit's LDS
#ifndef GS_LEARN_ROUNDS
#define GS_LEARN_ROUNDS 14
#endif
constexpr int SW_ROUNDS = GS_LEARN_ROUNDS;
static_assert(SW_ROUNDS % 2 == 0, "the counting pass computes buckets in two halves of the rounds");
constexpr int SW_TILE = SW_NT * SW_ROUNDS;           // 3584 keys by default
// waves per SIMD the distribution pass's registers are sized for: as many
// work-groups as its LDS (knot table + staged tile) lets a compute unit hold
#ifndef GS_LEARN_SCATTER_WAVES
#define GS_LEARN_SCATTER_WAVES (SW_ROUNDS >= 16 ? 2 : SW_ROUNDS >= 12 ? 3 : 4)
#endif

// The sorted sample through the knot table: its largest bucket, scaled to a
// half of the input, decides whether the call goes on with the learned form.
// First pass (the trained table): a table that fails is replaced by the
// sample's CDF (ctrl[L_RESCUE]).  Second pass, only after such a rescue: a
// table that still fails (keys no knot resolves) sends the call to the plain
// path at once.
__global__ __launch_bounds__(1024) void learned_screen_kernel(const double *sample, int64_t S, const Feature *feat,
                                                             const float *tab, int G, int B, int64_t half,
                                                             unsigned *ctrl, const double *hv, int second)
{
    extern __shared__ unsigned char s_raw[];
    float *s_tab = (float *)s_raw;                       // G + 1 knots
    unsigned *s_hist = (unsigned *)(s_tab + G + 1);      // B buckets
    __shared__ unsigned s_max;
    __shared__ double s_hv[kHeavySlots];
    if (ctrl[L_FALLBACK] || (second && !ctrl[L_RESCUE])) return;
    const int tid = threadIdx.x;
    const int hc = (int)ctrl[L_HEAVY];
    for (int i = tid; i <= G; i += 1024) s_tab[i] = tab[i];
    for (int i = tid; i < B; i += 1024) s_hist[i] = 0u;
    if (tid < kHeavySlots) s_hv[tid] = hv[tid];
    if (tid == 0) s_max = 0u;
    __syncthreads();
    const Feature F = *feat;
    for (int64_t i = tid; i < S; i += 1024) atomicAdd(&s_hist[bucket_of(sample[i], F, s_tab, G, B, s_hv, hc)], 1u);
    __syncthreads();
    // the heavy values' own buckets need no sort: they do not count
    if (tid < hc) s_hist[bucket_of(s_hv[tid], F, s_tab, G, B, s_hv, hc)] = 0u;
    __syncthreads();
    unsigned m = 0u;
    for (int i = tid; i < B; i += 1024) m = s_hist[i] > m ? s_hist[i] : m;
    atomicMax(&s_max, m);
    __syncthreads();
    if (tid == 0) {
        const int64_t predicted = (int64_t)s_max * half / S;
        const int64_t avg = half / B;
        const int64_t limit = kScreenSkew * avg > kScreenMin ? kScreenSkew * avg : kScreenMin;
        if (predicted > limit && !second) {
            ctrl[L_RESCUE] = 1u;
        } else if (predicted > limit) {
            ctrl[L_SCREENED] = 1u;
            ctrl[L_MAXB] = (unsigned)(predicted < 0xffffffffll ? predicted : 0xffffffffll);
            ctrl[L_FALLBACK] = 1u;
        }
    }
}

__global__ __launch_bounds__(SW_NT, 4) void learned_count_kernel(const double *src, int64_t len, const Feature *feat,
                                                              const float *tab, int G, int B, int shift, int dbits,
                                                              unsigned *tilecnt, unsigned *totals,
                                                              const unsigned *ctrl, const double *hv)
{
    extern __shared__ unsigned char lds_raw[];
    float *s_tab = (float *)lds_raw;
    unsigned *s_tot = (unsigned *)(lds_raw + (size_t)(G + 1) * 4);
    __shared__ unsigned s_dc[64];
    __shared__ double s_hv[kHeavySlots];
    if (ctrl[L_FALLBACK] || len <= 0) return;
    const Feature F = *feat;
    const int tid = threadIdx.x;
    const int D = 1 << dbits;
    const int hc = (int)ctrl[L_HEAVY];
    const int64_t ntiles = (len + SW_TILE - 1) / SW_TILE;
    for (int i = tid; i <= G; i += SW_NT) s_tab[i] = tab[i];
    if (tid < kHeavySlots) s_hv[tid] = hv[tid];
    if (totals)
        for (int i = tid; i < B; i += SW_NT) s_tot[i] = 0u;
    // keys of tile t (indices past the input read its last key)
    double x[SW_ROUNDS];
    auto load_tile = [&](int64_t t) {
        const double *p = src + t * SW_TILE + tid;
        if ((t + 1) * SW_TILE <= len) {
#pragma unroll
            for (int r = 0; r < SW_ROUNDS; ++r) x[r] = p[r * SW_NT];
        } else {
#pragma unroll
            for (int r = 0; r < SW_ROUNDS; ++r) {
                const int64_t i = t * SW_TILE + r * SW_NT + tid;
                x[r] = src[i < len ? i : len - 1];
            }
        }
    };
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        load_tile(t);
        if (tid < 64) s_dc[tid] = 0u;
        __syncthreads();
        const int64_t base = t * SW_TILE;
        int bk[SW_ROUNDS];
        buckets_of<SW_ROUNDS / 2>(x, bk, F, s_tab, G, B, s_hv, hc);    // two halves: fewer live registers
        buckets_of<SW_ROUNDS / 2>(x + SW_ROUNDS / 2, bk + SW_ROUNDS / 2, F, s_tab, G, B, s_hv, hc);
#pragma unroll
        for (int r = 0; r < SW_ROUNDS; ++r) {
            if (base + r * SW_NT + tid < len) {
                atomicAdd(&s_dc[(bk[r] >> shift) & (D - 1)], 1u);
                if (totals) atomicAdd(&s_tot[bk[r]], 1u);
            }
        }
        __syncthreads();
        if (tid < D) tilecnt[(int64_t)tid * ntiles + t] = s_dc[tid];
    }
    if (totals) {
        __syncthreads();
        for (int i = tid; i < B; i += SW_NT)
            if (s_tot[i]) atomicAdd(&totals[i], s_tot[i]);
    }
}

// Per digit (one work-group each): tilecnt[d][t] becomes the destination of
// tile t's first key of digit d: dstart[d] + the keys of digit d in tiles
// before t (an exclusive scan over the tiles, in tile order).
// The column of one digit is scanned in chunks of TS_CHUNK counts staged in
// LDS: loaded and stored back coalesced, each thread scanning 32 consecutive
// counts of the chunk (padded LDS index: conflict-free), a block scan of the
// threads' sums, and a carry from chunk to chunk.
constexpr int TS_CHUNK = 32 * 1024;
__host__ __device__ constexpr int ts_pad(int i) { return i + (i >> 5); }

__global__ __launch_bounds__(1024) void learned_tilescan_kernel(unsigned *tilecnt, int64_t ntiles,
                                                                const unsigned *dstart, const unsigned *ctrl)
{
    extern __shared__ unsigned s_col[];              // ts_pad(TS_CHUNK) words
    __shared__ unsigned s_part[1024];
    if (ctrl[L_FALLBACK]) return;
    const int d = blockIdx.x, tid = threadIdx.x;
    unsigned *col = tilecnt + (int64_t)d * ntiles;
    unsigned carry = dstart[d];
    for (int64_t c0 = 0; c0 < ntiles; c0 += TS_CHUNK) {
        const int len = (int)(ntiles - c0 < TS_CHUNK ? ntiles - c0 : TS_CHUNK);
        for (int i = tid; i < len; i += 1024) s_col[ts_pad(i)] = col[c0 + i];
        __syncthreads();
        const int b0 = 32 * tid;
        unsigned acc = 0;
        for (int i = 0; i < 32; ++i)
            if (b0 + i < len) acc += s_col[ts_pad(b0 + i)];
        s_part[tid] = acc;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const unsigned v = tid >= o ? s_part[tid - o] : 0u;
            __syncthreads();
            s_part[tid] += v;
            __syncthreads();
        }
        unsigned run = carry + s_part[tid] - acc;
        const unsigned total = s_part[1023];
        for (int i = 0; i < 32; ++i) {
            if (b0 + i < len) {
                const unsigned c = s_col[ts_pad(b0 + i)];
                s_col[ts_pad(b0 + i)] = run;
                run += c;
            }
        }
        carry += total;
        __syncthreads();
        for (int i = tid; i < len; i += 1024) col[c0 + i] = s_col[ts_pad(i)];
        __syncthreads();                             // LDS and s_part free for the next chunk
    }
}

// Bucket starts (exclusive scan of totals) of both halves, the segment
// offsets for the bucket sorts, the digit starts of the two distribution
// passes, the largest bucket and the overflow decision (the heavy values' own
// buckets are not sorted, so no size limit applies to them).  A bucket id is
// (high digit << lbits) | low digit.  Also the bucket sorts' order codes
// (codes: one row of B per half): the heavy values' buckets are done.
__global__ __launch_bounds__(1024) void learned_bucket_scan_kernel(const unsigned *totals, int B, int lbits,
                                                                   int halves, unsigned *starts, int64_t *offsets,
                                                                   unsigned *dstart, int64_t limit, unsigned *ctrl,
                                                                   const Feature *feat, const float *tab, int G,
                                                                   const double *hv, int *codes0, int *codes1)
{
    __shared__ int64_t s_part[1024];
    __shared__ unsigned s_max, s_over, s_big;
    __shared__ unsigned s_low[64];
    __shared__ unsigned char s_heavy[4096];
    __shared__ double s_hv[kHeavySlots];
    if (ctrl[L_FALLBACK]) return;
    const int tid = threadIdx.x;
    const int DL = 1 << lbits, DH = B >> lbits;
    const int hc = (int)ctrl[L_HEAVY];
    if (tid == 0) s_max = s_over = s_big = 0u;
    for (int b = tid; b < B; b += 1024) s_heavy[b] = 0;
    if (tid < kHeavySlots) s_hv[tid] = hv[tid];
    __syncthreads();
    if (tid < hc) s_heavy[bucket_of(s_hv[tid], *feat, tab, G, B, s_hv, hc)] = 1;
    __syncthreads();
    for (int b = tid; b < B; b += 1024) {
        const int code = s_heavy[b] ? kSegDone : 0;
        codes0[b] = code;
        codes1[b] = code;
    }
    for (int h = 0; h < halves; ++h) {
        const unsigned *tt = totals + (size_t)h * B;
        const int per = (B + 1023) / 1024;
        const int b0 = tid * per, b1 = b0 + per < B ? b0 + per : B;
        int64_t acc = 0;
        for (int b = b0; b < b1; ++b) {
            acc += tt[b];
            if (s_heavy[b]) continue;
            atomicMax(&s_max, tt[b]);
            if ((int64_t)tt[b] > limit) atomicAdd(&s_over, 1u);
            if (tt[b] > 4096u) atomicAdd(&s_big, 1u);
        }
        s_part[tid] = acc;
        __syncthreads();
        if (tid == 0)
            for (int k = 1; k < 1024; ++k) s_part[k] += s_part[k - 1];
        __syncthreads();
        int64_t run = tid > 0 ? s_part[tid - 1] : 0;
        for (int b = b0; b < b1; ++b) {
            starts[(size_t)h * B + b] = (unsigned)run;
            offsets[(size_t)h * (B + 1) + b] = run;
            run += tt[b];
        }
        if (tid == 1023) offsets[(size_t)h * (B + 1) + B] = s_part[1023];
        // keys per low digit, in bucket order within each digit
        if (tid < DL) {
            unsigned c = 0;
            for (int d1 = 0; d1 < DH; ++d1) c += tt[(d1 << lbits) | tid];
            s_low[tid] = c;
        }
        __syncthreads();
        unsigned *ds = dstart + (size_t)h * 128;
        if (tid == 0) {
            unsigned r = 0;
            for (int d = 0; d < DL; ++d) {
                ds[d] = r;                                  // pass 1: by low digit
                r += s_low[d];
            }
        }
        if (tid < DH) ds[64 + tid] = starts[(size_t)h * B + (tid << lbits)];   // pass 2: by high digit
        __syncthreads();
    }
    if (tid == 0) {
        ctrl[L_MAXB] = s_max;
        ctrl[L_OVERFLOW] = s_over;
        ctrl[L_BIGB] = s_big;
        if (s_over) ctrl[L_FALLBACK] = 1u;
    }
}

// ---------------------------------------------------------------------------
// 6b. one stable distribution pass by a digit of the bucket id
// ---------------------------------------------------------------------------
// One tile per work-group iteration.  Wave w ranks its keys (SW_ROUNDS rounds
// of 64 in input order): every lane of a round sets its bit in its digit's
// lane mask (LDS atomic or), so a key's place among its round's equals is a
// population count; lane d turns the counts of digit d into prefixes over
// the rounds, and a key's rank is its round's prefix plus its place among its
// round's equals.  The tile then stages its keys in LDS grouped by digit and
// writes every digit's run contiguously at the tile's offset for that digit
// (from the tile scan).  The rank scratch shares LDS with the staging area.
__global__ __launch_bounds__(SW_NT, GS_LEARN_SCATTER_WAVES) void learned_scatter_kernel(const double *src, double *dst, int64_t len,
                                                                const Feature *feat, const float *tab, int G, int B,
                                                                int shift, int dbits, const unsigned *tileoff,
                                                                const unsigned *ctrl, const double *hv)
{
    extern __shared__ unsigned char lds_raw[];
    float *s_tab = (float *)lds_raw;
    __shared__ double s_hv[kHeavySlots];
    double *s_key = (double *)(lds_raw + (((size_t)(G + 1) * 4 + 15) & ~(size_t)15));
    unsigned char *s_dig = (unsigned char *)(s_key + SW_TILE);
    __shared__ unsigned s_wcnt[SW_NT / 64][64];     // per wave and digit: keys, then staging base
    __shared__ unsigned s_goff[64];
    __shared__ int64_t s_delta[64];                 // per digit: destination minus staged position
    if (ctrl[L_FALLBACK] || len <= 0) return;
    const Feature F = *feat;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int D = 1 << dbits;
    const int hc = (int)ctrl[L_HEAVY];
    if (tid < kHeavySlots) s_hv[tid] = hv[tid];
    const int64_t ntiles = (len + SW_TILE - 1) / SW_TILE;
    // this wave's [round][digit] scratch: lane masks, then prefixes
    unsigned long long *wm = (unsigned long long *)s_key + wave * (SW_ROUNDS * 64);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int i = tid; i <= G; i += SW_NT) s_tab[i] = tab[i];
    // tile t's destination of every digit (thread d < D holds digit d's),
    // then a wave's keys of the tile (indices past the input read its last
    // key)
    double x[SW_ROUNDS];
    unsigned goff = 0u;
    auto load_tile = [&](int64_t t) {
        if (tid < D) goff = tileoff[(int64_t)tid * ntiles + t];
        const int64_t base = t * SW_TILE + (int64_t)wave * (SW_TILE / 4);
        if ((t + 1) * SW_TILE <= len) {
            const double *q = src + base + lane;
#pragma unroll
            for (int r = 0; r < SW_ROUNDS; ++r) x[r] = q[r * 64];
        } else {
#pragma unroll
            for (int r = 0; r < SW_ROUNDS; ++r) {
                const int64_t p = base + r * 64 + lane;
                x[r] = src[p < len ? p : len - 1];
            }
        }
    };
    if ((int64_t)blockIdx.x < ntiles) load_tile(blockIdx.x);
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t base = t * SW_TILE + (int64_t)wave * (SW_TILE / 4);
#pragma unroll
        for (int r = 0; r < SW_ROUNDS; ++r) wm[r * 64 + lane] = 0ull;
        if (tid < D) s_goff[tid] = goff;
        __syncthreads();
        int dg[SW_ROUNDS];
        buckets_of<SW_ROUNDS>(x, dg, F, s_tab, G, B, s_hv, hc);
#pragma unroll
        for (int r = 0; r < SW_ROUNDS; ++r) {
            const bool valid = base + r * 64 + lane < len;
            dg[r] = valid ? ((dg[r] >> shift) & (D - 1)) : -1;
        }
        // lanes of a round with equal digits: each sets its bit in the digit's
        // mask (bitwise or, so the order of the updates does not matter)
        // (a key past the input sets no bit: it ors 0 into digit 0's mask)
#pragma unroll
        for (int r = 0; r < SW_ROUNDS; ++r)
            atomicOr(&wm[r * 64 + (dg[r] >= 0 ? dg[r] : 0)], dg[r] >= 0 ? 1ull << lane : 0ull);
        __builtin_amdgcn_wave_barrier();
        unsigned rk[SW_ROUNDS];
#pragma unroll
        for (int r = 0; r < SW_ROUNDS; ++r)
            rk[r] = (unsigned)__popcll(wm[r * 64 + (dg[r] >= 0 ? dg[r] : 0)] & below);
        unsigned cnt[SW_ROUNDS];
#pragma unroll
        for (int r = 0; r < SW_ROUNDS; ++r) cnt[r] = (unsigned)__popcll(wm[r * 64 + lane]);   // lane = digit
        __builtin_amdgcn_wave_barrier();
        {
            unsigned run = 0;
#pragma unroll
            for (int r = 0; r < SW_ROUNDS; ++r) {
                wm[r * 64 + lane] = run;                    // keys of digit `lane` in earlier rounds
                run += cnt[r];
            }
            s_wcnt[wave][lane] = run;
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int r = 0; r < SW_ROUNDS; ++r) rk[r] += (unsigned)wm[r * 64 + (dg[r] >= 0 ? dg[r] : 0)];
        __syncthreads();
        if (tid < 64) {
            const int d = tid;
            unsigned run = 0;
            unsigned woff[SW_NT / 64];
#pragma unroll
            for (int w = 0; w < SW_NT / 64; ++w) {          // wave offsets per digit
                woff[w] = run;
                run += s_wcnt[w][d];
            }
            // tile-local start of every digit: exclusive scan over the digits
            unsigned inc = run;
            for (int o = 1; o < 64; o <<= 1) {
                const unsigned v = __shfl_up(inc, o);
                if (lane >= o) inc += v;
            }
            const unsigned toff = inc - run;
            // staging base of each wave's keys of digit d, and the shift from a
            // staged position to the destination
#pragma unroll
            for (int w = 0; w < SW_NT / 64; ++w) s_wcnt[w][d] = toff + woff[w];
            s_delta[d] = (int64_t)s_goff[d] - (int64_t)toff;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < SW_ROUNDS; ++r) {
            if (dg[r] >= 0) {
                const unsigned pos = s_wcnt[wave][dg[r]] + rk[r];
                s_key[pos] = x[r];
                s_dig[pos] = (unsigned char)dg[r];
            }
        }
        // the keys are staged: load the next tile while this one is written
        if (t + gridDim.x < ntiles) load_tile(t + gridDim.x);
        __syncthreads();
        const int64_t rem = len - t * SW_TILE;
        const int nvalid = rem < SW_TILE ? (int)rem : SW_TILE;
        for (int i = tid; i < nvalid; i += SW_NT) {
            const int64_t g = s_delta[s_dig[i]] + i;
            if ((uint64_t)g < (uint64_t)len) dst[g] = s_key[i];
        }
        __syncthreads();                                    // LDS free for the next tile
    }
}

// Work-groups of a distribution pass: as many as the device holds at once
// with `slds` bytes of dynamic LDS each (each walks tiles with a stride of the
// grid, so none waits for a slot behind the others), cached per device.
static int64_t scatter_groups(size_t slds)
{
    static int64_t cache[16] = {};
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) dev = 0;
    const int slot = dev < 16 ? dev : 15;
    if (dev < 16 && cache[slot] > 0) return cache[slot];
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, learned_scatter_kernel, SW_NT, slds) != hipSuccess ||
        per_cu <= 0)
        per_cu = 1;
    const int64_t g = (int64_t)cus * per_cu;
    if (dev < 16) cache[slot] = g;
    return g;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int64_t al256(int64_t b) { return (b + 255) & ~(int64_t)255; }

LearnedPlan plan_learned(int64_t n, const gs_learned_params &prm)
{
    LearnedPlan L{};
    L.n = n;
    L.S = prm.sample_size;
    L.B = (int)prm.num_buckets;
    L.G = (int)prm.knots;
    L.batch = (int)prm.batch;
    L.use_learned = n >= 4 * (int64_t)L.S && n >= (1 << 16) && n < ((int64_t)1 << 32) && L.S >= 1024 &&
                    L.B >= 2 && L.G >= 2 && L.batch >= 32;
    L.plain = plan_f64(n);
    // half buffer with one extra slot (the second half has ceil(n/2) keys)
    const int64_t hb = al256((n / 2 + 1) * 8);
    const int64_t shift = hb - L.plain.off_forest;
    L.plain.off_forest += shift;
    L.plain.bytes += shift;
    int64_t o = al256(L.plain.bytes);
    if (!L.use_learned) {
        L.bytes = o;
        return L;
    }
    const int64_t half = n - n / 2;
    L.limit = half / 4 > kBucketLimit ? half / 4 : kBucketLimit;
    L.ntiles = (half + SW_TILE - 1) / SW_TILE;        // tiles of the larger half
    L.splan = plan_f64(L.S);
    L.off_sample = o; o = al256(o + L.S * 8);
    L.off_sample_ws = o; o = al256(o + L.splan.bytes);
    L.off_u = o; o = al256(o + L.S * 4);
    L.off_t = o; o = al256(o + L.S * 4);
    L.off_feat = o; o = al256(o + (int64_t)sizeof(Feature));
    L.off_ctrl = o; o = al256(o + 64 * 4);
    L.off_params = o; o = al256(o + kMlpParams * 4);
    L.off_m = o; o = al256(o + kMlpParams * 4);
    L.off_v = o; o = al256(o + kMlpParams * 4);
    const int nwg = L.batch / mlp_samples_per_group();
    L.off_partial = o; o = al256(o + (int64_t)nwg * (kMlpParams + 1) * 4);
    L.off_losses = o; o = al256(o + 2 * 4);
    L.off_raw = o; o = al256(o + (int64_t)(L.G + 1) * 4);
    L.off_tab = o; o = al256(o + (int64_t)(L.G + 1) * 4);
    L.off_totals = o; o = al256(o + 2 * (int64_t)L.B * 4);
    L.off_starts = o; o = al256(o + 2 * (int64_t)L.B * 4);
    L.off_offsets = o; o = al256(o + 2 * (int64_t)(L.B + 1) * 8);
    L.off_dstart = o; o = al256(o + 2 * 128 * 4);
    L.off_tilecnt = o; o = al256(o + 2 * L.ntiles * 64 * 4);
    L.off_segctrl = o; o = al256(o + 2 * 64 * 4);
    L.off_seglists = o; o = al256(o + 2 * 3 * (int64_t)L.B * 4);
    L.off_heavy = o; o = al256(o + kHeavySlots * 8);
    L.off_runs = o; o = al256(o + kHeavyCand * 16);
    L.segforest = plan_forest_seg(half, half < L.limit ? half : L.limit, L.B);
    L.off_segforest = o; o = al256(o + L.segforest.bytes);
    L.bytes = o;
    return L;
}

static hipError_t learned_sort_body(double *keys, int64_t n, const gs_learned_params &prm, char *ws,
                                    const LearnedPlan &L, hipStream_t st)
{
    if (!L.use_learned) return sort_f64_async(keys, n, ws, L.plain, st);
    const int B = L.B, G = L.G;
    int bbits = 0;
    while ((1 << bbits) < B) ++bbits;
    unsigned *ctrl = (unsigned *)(ws + L.off_ctrl);
    double *H = (double *)ws;                      // floor(n/2)+1 slots
    double *sample = (double *)(ws + L.off_sample);
    float *u = (float *)(ws + L.off_u), *t = (float *)(ws + L.off_t);
    Feature *feat = (Feature *)(ws + L.off_feat);
    float *params = (float *)(ws + L.off_params);
    float *m = (float *)(ws + L.off_m), *v = (float *)(ws + L.off_v);
    float *partial = (float *)(ws + L.off_partial), *losses = (float *)(ws + L.off_losses);
    float *raw = (float *)(ws + L.off_raw), *tab = (float *)(ws + L.off_tab);
    int64_t *offsets = (int64_t *)(ws + L.off_offsets);
    unsigned *segctrl = (unsigned *)(ws + L.off_segctrl);
    int *seglists = (int *)(ws + L.off_seglists);
    double *hv = (double *)(ws + L.off_heavy);
    int64_t *runs = (int64_t *)(ws + L.off_runs);
    const bool tr = trace_on();

    launch_fill_u32(ctrl, 64, 0u, st);
    launch_fill_u32((unsigned *)m, kMlpParams, 0u, st);
    launch_fill_u32((unsigned *)v, kMlpParams, 0u, st);
    launch_fill_u32((unsigned *)losses, 2, 0u, st);

    // 1-2. sample, sort it with the plain path, feature and targets
    if (tr) trace_begin(TK_LEARN_PREP, st);
    hipLaunchKernelGGL(learned_sample_kernel, dim3((unsigned)((L.S + 255) / 256)), dim3(256), 0, st,
                       (const double *)keys, n, L.S, prm.seed, sample);
    if (tr) trace_end(st);
    hipError_t e = sort_f64_async(sample, L.S, ws + L.off_sample_ws, L.splan, st);
    if (e != hipSuccess) return e;
    if (tr) trace_begin(TK_LEARN_PREP, st);
    const bool screening = prm.mode == 0 && !prm.test_bucket_table && prm.screen == 0;
    hipLaunchKernelGGL(learned_prep_kernel, dim3(1), dim3(1024), 0, st, (const double *)sample, L.S, G, feat, ctrl,
                       screening ? n - n / 2 : (int64_t)0, B, hv, runs);
    hipLaunchKernelGGL(learned_targets_kernel, dim3((unsigned)((L.S + 255) / 256)), dim3(256), 0, st,
                       (const double *)sample, L.S, (const Feature *)feat, u, t, (const int64_t *)runs,
                       (const unsigned *)ctrl);
    if (tr) trace_end(st);

    // 3-4. network and knot table
    if (tr) trace_begin(TK_LEARN_TRAIN, st);
    if (prm.mode == 0 && !prm.test_bucket_table) {
        if (prm.weights_override) {
            e = hipMemcpyAsync(params, prm.weights_override, kMlpParams * 4, hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess) return e;
        } else {
            e = mlp_init(params, prm.seed, st);
            if (e != hipSuccess) return e;
            if (prm.train_steps > 0) {
                e = mlp_train(params, m, v, u, t, L.S, (int)prm.train_steps, L.batch, prm.lr, prm.seed, 0, partial,
                              losses, ctrl + L_FALLBACK, st);
                if (e != hipSuccess) return e;
            }
        }
        e = mlp_forward(params, nullptr, G + 1, raw, G, ctrl + L_FALLBACK, st);
        if (e != hipSuccess) return e;
    }
    if (tr) trace_end(st);
    if (prm.mode == 2 && !prm.test_bucket_table)
        hipLaunchKernelGGL(learned_sample_table_kernel, dim3(1), dim3(1024), 0, st, (const double *)sample, L.S,
                           (const Feature *)feat, G, tab, (const int64_t *)runs, (const double *)hv, ctrl, 0);
    hipLaunchKernelGGL(learned_table_kernel, dim3(1), dim3(1024), 0, st, (const float *)raw, prm.test_bucket_table,
                       (int)prm.mode, G, tab, ctrl, (const Feature *)feat);
    if (screening) {
        const size_t jlds = (size_t)(G + 1) * 4 + (size_t)B * 4;
        (void)hipFuncSetAttribute((const void *)learned_screen_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)jlds);
        for (int second = 0; second < 2; ++second) {
            hipLaunchKernelGGL(learned_screen_kernel, dim3(1), dim3(1024), jlds, st, (const double *)sample, L.S,
                               (const Feature *)feat, (const float *)tab, G, B, n - n / 2, ctrl,
                               (const double *)hv, second);
            if (!second)
                hipLaunchKernelGGL(learned_sample_table_kernel, dim3(1), dim3(1024), 0, st, (const double *)sample,
                                   L.S, (const Feature *)feat, G, tab, (const int64_t *)runs, (const double *)hv,
                                   ctrl, 1);
        }
    }
    // Unless the stream is being captured, the host reads the decision once
    // and enqueues only the path that runs (the gated launches of the other
    // one cost about a millisecond); under capture every launch stays gated
    // on the device word.
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
        (void)hipGetLastError();
        cs = hipStreamCaptureStatusActive;
    }
    if (cs == hipStreamCaptureStatusNone) {
        unsigned fb = 0u;
        e = hipMemcpyAsync(&fb, ctrl + L_FALLBACK, 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return e;
        if (fb) return sort_f64_async(keys, n, ws, L.plain, st, ctrl + L_FALLBACK, 1u);
    }

    // 6. bucket totals of both halves (and the first pass's tile counts)
    //    before anything moves
    const int64_t nA = n / 2, nB = n - nA;                 // first and second half
    const int lbits = bbits / 2, hbits = bbits - lbits;    // bucket id = (high << lbits) | low
    const int64_t tA = (nA + SW_TILE - 1) / SW_TILE, tB = (nB + SW_TILE - 1) / SW_TILE;
    if (tA > L.ntiles || tB > L.ntiles) return hipErrorInvalidValue;   // the plan sized the tile counts
    unsigned *totals = (unsigned *)(ws + L.off_totals);
    unsigned *starts = (unsigned *)(ws + L.off_starts);
    unsigned *dstart = (unsigned *)(ws + L.off_dstart);
    unsigned *cntA = (unsigned *)(ws + L.off_tilecnt);
    unsigned *cntB = cntA + 64 * tA;
    const size_t clds = (size_t)(G + 1) * 4 + (size_t)B * 4;
    const size_t slds = (((size_t)(G + 1) * 4 + 15) & ~(size_t)15) + (size_t)SW_TILE * 9;
    (void)hipFuncSetAttribute((const void *)learned_count_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)clds);
    (void)hipFuncSetAttribute((const void *)learned_scatter_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)slds);
    const unsigned cgrid = GS_LEARN_CGRID;
    const size_t tslds = (size_t)ts_pad(TS_CHUNK) * 4;
    (void)hipFuncSetAttribute((const void *)learned_tilescan_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)tslds);
    if (tr) trace_begin(TK_LEARN_BUCKET, st);
    launch_fill_u32(totals, 2 * (int64_t)B, 0u, st);
    hipLaunchKernelGGL(learned_count_kernel, dim3(cgrid), dim3(SW_NT), clds, st, (const double *)keys, nA,
                       (const Feature *)feat, (const float *)tab, G, B, 0, lbits, cntA, totals,
                       (const unsigned *)ctrl, (const double *)hv);
    hipLaunchKernelGGL(learned_count_kernel, dim3(cgrid), dim3(SW_NT), clds, st, (const double *)(keys + nA), nB,
                       (const Feature *)feat, (const float *)tab, G, B, 0, lbits, cntB, totals + B,
                       (const unsigned *)ctrl, (const double *)hv);
    // (order codes of the bucket sorts: rank rows of both halves' segment lists)
    hipLaunchKernelGGL(learned_bucket_scan_kernel, dim3(1), dim3(1024), 0, st, (const unsigned *)totals, B, lbits,
                       2, starts, offsets, dstart, L.limit, ctrl, (const Feature *)feat, (const float *)tab, G,
                       (const double *)hv, seglists + B, seglists + 4 * B);
    if (tr) trace_end(st);

    // 7. each half: two stable distribution passes (low digit into the half
    //    buffer, high digit back), which leave its keys grouped by bucket in
    //    input order in place; then every bucket sorted, with the half buffer
    //    as frog buffer.  Second half first, then the first.
    const int64_t sres = scatter_groups(slds);
    auto distribute = [&](double *region, int64_t len, int64_t ntiles, unsigned *cnt, int h) {
        if (ntiles == 0) return;
        const unsigned sgrid = (unsigned)(ntiles < sres ? ntiles : sres);
        hipLaunchKernelGGL(learned_tilescan_kernel, dim3(1u << lbits), dim3(1024), tslds, st, cnt, ntiles,
                           (const unsigned *)(dstart + h * 128), (const unsigned *)ctrl);
        hipLaunchKernelGGL(learned_scatter_kernel, dim3(sgrid), dim3(SW_NT), slds, st,
                           (const double *)region, H, len, (const Feature *)feat, (const float *)tab, G, B, 0, lbits,
                           (const unsigned *)cnt, (const unsigned *)ctrl, (const double *)hv);
        hipLaunchKernelGGL(learned_count_kernel, dim3(cgrid), dim3(SW_NT), clds, st, (const double *)H, len,
                           (const Feature *)feat, (const float *)tab, G, B, lbits, hbits, cnt, (unsigned *)nullptr,
                           (const unsigned *)ctrl, (const double *)hv);
        hipLaunchKernelGGL(learned_tilescan_kernel, dim3(1u << hbits), dim3(1024), tslds, st, cnt, ntiles,
                           (const unsigned *)(dstart + h * 128 + 64), (const unsigned *)ctrl);
        hipLaunchKernelGGL(learned_scatter_kernel, dim3(sgrid), dim3(SW_NT), slds, st, (const double *)H,
                           region, len, (const Feature *)feat, (const float *)tab, G, B, lbits, hbits,
                           (const unsigned *)cnt, (const unsigned *)ctrl, (const double *)hv);
    };
    if (tr) trace_begin(TK_LEARN_BUCKET, st);
    distribute(keys + nA, nB, tB, cntB, 1);
    if (tr) trace_end(st);
    e = segsort_core_async(keys + nA, offsets + (B + 1), B, nB, H, segctrl + 64, seglists + 3 * B,
                           seglists + 4 * B, seglists + 5 * B, ws + L.off_segforest, L.segforest,
                           ctrl + L_FALLBACK, 0u, st, true);
    if (e != hipSuccess) return e;
    if (tr) trace_begin(TK_LEARN_BUCKET, st);
    distribute(keys, nA, tA, cntA, 0);
    if (tr) trace_end(st);
    e = segsort_core_async(keys, offsets, B, nA, H, segctrl, seglists, seglists + B, seglists + 2 * B,
                           ws + L.off_segforest, L.segforest, ctrl + L_FALLBACK, 0u, st, true);
    if (e != hipSuccess) return e;

    // 8. merge: the sorted first half moves to the half buffer (logical
    //    [n, n+nA)); the second run stays at [nA, n) inside the output [0, n),
    //    which is written bottom-up
    if (tr) trace_begin(TK_LEARN_BUCKET, st);
    e = copy_f64_async(keys, H, nA, st, ctrl + L_FALLBACK);
    if (e != hipSuccess) return e;
    if (tr) trace_end(st);
    FrogMerge fm{};
    fm.l0 = n;
    fm.nl = nA;
    fm.r0 = nA;
    fm.nr = nB;
    fm.out0 = 0;
    fm.left = 0;
    fm.outer = 1;
    e = merge_one_f64_async(keys, H, n, fm, ws, L.plain, st, ctrl + L_FALLBACK, 0u);
    if (e != hipSuccess) return e;

    // plain path on the untouched input if the bucketing was rejected
    e = sort_f64_async(keys, n, ws, L.plain, st, ctrl + L_FALLBACK, 1u);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

// The error words of every control area the call uses: the plain plan's
// (fallback sort and final merge), the sample sort's, the bucket forest's and
// the training barrier's.
static ErrWords learned_err_words(char *ws, const LearnedPlan &L)
{
    ErrWords ew = plain_err_words(ws, L.plain);
    if (L.use_learned) {
        ew.add((unsigned *)(ws + L.off_sample_ws + L.splan.off_forest + L.splan.forest.off_ctrl) + kErrWord,
               DEVERR_WAIT);
        ew.add((unsigned *)(ws + L.off_segforest + L.segforest.off_ctrl) + kErrWord, DEVERR_WAIT);
        ew.add((unsigned *)(ws + L.off_ctrl) + L_ERR, DEVERR_WAIT);
    }
    return ew;
}

hipError_t learned_sort_async(double *keys, int64_t n, const gs_learned_params &prm, char *ws,
                              const LearnedPlan &L, hipStream_t st)
{
    const ErrWords ew = learned_err_words(ws, L);
    hipError_t e = err_words_begin(ew, st);
    if (e != hipSuccess) return e;
    e = learned_sort_body(keys, n, prm, ws, L, st);
    if (e != hipSuccess) return e;
    return err_words_end(ew, st);
}

hipError_t learned_errors(const char *ws, const LearnedPlan &L, unsigned *any)
{
    const ErrWords ew = learned_err_words((char *)ws, L);
    *any = 0;
    for (int i = 0; i < ew.count; ++i) {
        unsigned w = 0;
        hipError_t e = hipMemcpy(&w, ew.w[i], 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return e;
        *any |= w ? ew.bit[i] : 0u;
    }
    return hipSuccess;
}

hipError_t learned_read_report(const char *ws, const LearnedPlan &L, LearnedReport *r)
{
    if (!L.use_learned) {
        *r = LearnedReport{};
        return hipSuccess;
    }
    unsigned c[64];
    float loss[2];
    hipError_t e = hipMemcpy(c, ws + L.off_ctrl, sizeof c, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(loss, ws + L.off_losses, sizeof loss, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    r->fallback = c[L_FALLBACK] ? (c[L_SCREENED] ? 2u : 1u) : 0u;
    r->order_violation = c[L_ORDER];
    r->overflow_buckets = c[L_OVERFLOW];
    r->max_bucket = c[L_MAXB];
    r->big_buckets = c[L_BIGB];
    r->err = c[L_ERR];
    r->feature = c[L_FEAT] | (c[L_SAMPTAB] ? 2u : 0u);
    r->heavy = c[L_FALLBACK] ? 0u : c[L_HEAVY];
    r->loss_first = loss[0];
    r->loss_last = loss[1];
    return hipSuccess;
}

}  // namespace gs
