// Learned CDF bucket path (not part of the paper): the same stable ascending
// result as the plain frog sort, with most merge levels replaced by one
// bucketing scatter and per-bucket sorts.
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
//   6. for the second half then the first half of the input: per-wave bucket
//      counts, a stable ranked scatter into free memory, per-bucket sorts;
//   7. one frog-style in-place merge of the two sorted halves into the input.
// Memory stays at the half buffer: the second half is scattered into the half
// buffer, sorted there using its own vacated input region as scratch; the
// first half is scattered into that vacated region, sorted using its own
// vacated region; the final merge writes bottom-up over the first half's run.
#include <hip/hip_runtime.h>

#include "gs_block.h"
#include "gs_device.h"
#include "gs_internal.h"
#include "gs_learned.h"
#include "gs_mlp.h"

namespace gs {

namespace {

constexpr int HNT = 256;                 // histogram / scatter work-group size
constexpr int HIPT = 16;                 // keys per lane per batch
constexpr int FEAT_BINS = 4096;          // bins for choosing the feature
constexpr int kDensH = 32;               // half window (ranks) of the density targets

// control words of the learned path
constexpr int L_FALLBACK = 0;            // 1: take the plain path
constexpr int L_ORDER = 1;               // table not monotone
constexpr int L_OVERFLOW = 2;            // buckets above the limit
constexpr int L_MAXB = 3;                // largest bucket
constexpr int L_BAR = 4;                 // training grid barrier
constexpr int L_ERR = 5;
constexpr int L_BIGB = 6;                // buckets larger than one LDS tile
constexpr int L_FEAT = 7;                // chosen feature

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
    if (x != x) return ~0ull;
    uint64_t u = (uint64_t)__double_as_longlong(x);
    if ((u << 1) == 0) u = 0;
    return (u >> 63) ? ~u : (u | (1ull << 63));
}

__device__ __forceinline__ double phi_of(double x, const Feature &F)
{
    if (F.bits) {
        const uint64_t k = ckey(x);
        const double num = k >= F.klo ? (double)(k - F.klo) : -(double)(F.klo - k);
        return num / F.krange;
    }
    return (x - F.lo) / F.range;
}

// Bucket of key x.  Monotone non-decreasing in x whenever `tab` is
// non-decreasing: phi is monotone (correctly rounded subtraction, conversion
// and division by a positive constant), the knot index and the fraction are
// monotone in phi, the interpolation is clamped to the next knot.
__device__ __forceinline__ int bucket_of(double x, const Feature &F, const float *tab, int G, int B)
{
    if (x != x) return B - 1;
    const double u = phi_of(x, F) * (double)G;
    int i;
    float f;
    if (!(u > 0.0)) {
        i = 0;
        f = 0.f;
    } else if (u >= (double)G) {
        i = G - 1;
        f = 1.f;
    } else {
        i = (int)u;
        f = (float)(u - (double)i);
    }
    const float a = tab[i], b = tab[i + 1];
    const float v = fminf(fmaf(f, b - a, a), b);
    const int bk = (int)(v * (float)B);
    return bk < 0 ? 0 : (bk > B - 1 ? B - 1 : bk);
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
// smaller largest bin wins (ties: linear).  Targets: log of the local density
// of the sample in phi over a window of +-kDensH ranks.
__global__ __launch_bounds__(1024) void learned_prep_kernel(const double *xs, int64_t S, Feature *feat,
                                                            float *u, float *t, unsigned *ctrl)
{
    __shared__ unsigned h_lin[FEAT_BINS], h_bits[FEAT_BINS];
    __shared__ int64_t s_nn;
    __shared__ unsigned s_max[2];
    __shared__ Feature sF;
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
    }
    const bool lin_ok = nn > 0 && F.range > 0.0 && F.range < __builtin_inf();
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
        sF = F;
        *feat = F;
        ctrl[L_FEAT] = (unsigned)F.bits;
    }
    __syncthreads();
    F = sF;
    // inputs phi (NaN keys at the top), then log-density targets from the
    // rank differences of the (non-decreasing) inputs
    for (int64_t i = tid; i < S; i += 1024) {
        double p = F.valid ? phi_of(xs[i], F) : 0.0;
        if (xs[i] != xs[i]) p = 1.0;
        p = p < 0.0 ? 0.0 : (p > 1.0 ? 1.0 : p);
        u[i] = (float)p;
    }
    __syncthreads();
    __threadfence_block();
    for (int64_t i = tid; i < S; i += 1024) {
        const int64_t lo = i - kDensH > 0 ? i - kDensH : 0;
        const int64_t hi = i + kDensH < S - 1 ? i + kDensH : S - 1;
        double w = (double)u[hi] - (double)u[lo];
        w = w > 1e-7 ? w : 1e-7;
        t[i] = (float)log((double)(hi - lo) / ((double)S * w));
    }
}

// ---------------------------------------------------------------------------
// 4. knot table: normalised cumulative integral of exp(network) (or the
//    linear CDF, or the raw test table); verified monotone
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void learned_table_kernel(const float *raw, const float *test_table, int mode,
                                                             int G, float *tab, unsigned *ctrl, const Feature *feat)
{
    __shared__ double s_part[1024];
    __shared__ float s_mx[1024];
    __shared__ unsigned s_bad;
    const int tid = threadIdx.x;
    const int cnt = G + 1;
    const int per = (cnt + 1023) / 1024;
    const int b0 = tid * per, b1 = b0 + per < cnt ? b0 + per : cnt;
    if (tid == 0) s_bad = 0u;
    if (test_table) {
        for (int i = b0; i < b1; ++i) tab[i] = test_table[i];
    } else if (mode == 1) {
        for (int i = b0; i < b1; ++i) tab[i] = (float)((double)i / (double)G);
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
// 6a. per-wave bucket counts of one half
// ---------------------------------------------------------------------------
// Wave w of the half takes keys [w*chunk, min((w+1)*chunk, len)); counts go
// to counts[w*B + b].
__global__ __launch_bounds__(HNT) void learned_hist_kernel(const double *src, int64_t len, int64_t chunk,
                                                           int64_t nwaves, const Feature *feat, const float *tab,
                                                           int G, int B, unsigned *counts, const unsigned *ctrl)
{
    extern __shared__ unsigned char lds_raw[];
    float *s_tab = (float *)lds_raw;
    unsigned *s_cnt = (unsigned *)(lds_raw + (size_t)(G + 1) * 4);
    if (ctrl[L_FALLBACK]) return;
    const Feature F = *feat;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i <= G; i += HNT) s_tab[i] = tab[i];
    unsigned *mycnt = s_cnt + (size_t)wave * B;
    for (int i = lane; i < B; i += 64) mycnt[i] = 0u;
    __syncthreads();
    const int64_t w = (int64_t)blockIdx.x * (HNT / 64) + wave;
    if (w < nwaves) {
        const int64_t c0 = w * chunk;
        const int64_t c1 = c0 + chunk < len ? c0 + chunk : len;
        for (int64_t base = c0; base < c1; base += 64 * HIPT) {
            double x[HIPT];
#pragma unroll
            for (int r = 0; r < HIPT; ++r) {
                const int64_t i = base + r * 64 + lane;
                x[r] = src[i < c1 ? i : c1 - 1];
            }
#pragma unroll
            for (int r = 0; r < HIPT; ++r) {
                const int64_t i = base + r * 64 + lane;
                if (i < c1) atomicAdd(&mycnt[bucket_of(x[r], F, s_tab, G, B)], 1u);
            }
        }
    }
    __syncthreads();
    if (w < nwaves)
        for (int i = lane; i < B; i += 64) counts[w * B + i] = mycnt[i];
}

// ---------------------------------------------------------------------------
// 6b. per bucket: exclusive prefix over waves (in place) and the total
// ---------------------------------------------------------------------------
// Work-group of 256 threads = 64 buckets x 4 quarters of the waves: each
// thread sums its quarter, the quarters are prefixed in LDS, then each thread
// rewrites its quarter as exclusive prefixes (all in wave order).
__global__ __launch_bounds__(256) void learned_colscan_kernel(unsigned *counts, int64_t nwaves, int B,
                                                              unsigned *totals, const unsigned *ctrl)
{
    __shared__ unsigned s_q[4][64];
    if (ctrl[L_FALLBACK]) return;
    const int bl = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int b = blockIdx.x * 64 + bl;
    const int64_t per = (nwaves + 3) / 4;
    const int64_t w0 = q * per, w1 = w0 + per < nwaves ? w0 + per : nwaves;
    unsigned acc = 0;
    if (b < B) {
#pragma unroll 8
        for (int64_t w = w0; w < w1; ++w) acc += counts[w * B + b];
    }
    s_q[q][bl] = acc;
    __syncthreads();
    unsigned run = 0;
    for (int k = 0; k < q; ++k) run += s_q[k][bl];
    if (b < B) {
#pragma unroll 8
        for (int64_t w = w0; w < w1; ++w) {
            const unsigned c = counts[w * B + b];
            counts[w * B + b] = run;
            run += c;
        }
        if (q == 3) totals[b] = run;
    }
}

// Bucket starts (exclusive scan of totals) of both halves, the segment
// offsets for the bucket sorts, the largest bucket and the overflow decision.
__global__ __launch_bounds__(1024) void learned_bucket_scan_kernel(const unsigned *totals, int B, int halves,
                                                                   unsigned *starts, int64_t *offsets,
                                                                   int64_t limit, unsigned *ctrl)
{
    __shared__ int64_t s_part[1024];
    __shared__ unsigned s_max, s_over, s_big;
    if (ctrl[L_FALLBACK]) return;
    const int tid = threadIdx.x;
    if (tid == 0) s_max = s_over = s_big = 0u;
    __syncthreads();
    for (int h = 0; h < halves; ++h) {
        const unsigned *tt = totals + (size_t)h * B;
        const int per = (B + 1023) / 1024;
        const int b0 = tid * per, b1 = b0 + per < B ? b0 + per : B;
        int64_t acc = 0;
        for (int b = b0; b < b1; ++b) {
            acc += tt[b];
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
// 6c. stable ranked scatter of one half
// ---------------------------------------------------------------------------
// Each wave walks its chunk in input order, 64 keys per step.  Lanes holding
// the same bucket find each other with one ballot per bucket bit; a lane's
// rank among them plus the wave's running count for the bucket (kept in LDS,
// started at the bucket start plus the counts of all earlier waves) is its
// destination, so equal buckets keep input order.
__global__ __launch_bounds__(HNT) void learned_scatter_kernel(const double *src, int64_t len, int64_t chunk,
                                                              int64_t nwaves, const Feature *feat,
                                                              const float *tab, int G, int B, int bbits,
                                                              const unsigned *counts, const unsigned *starts,
                                                              double *dst, const unsigned *ctrl)
{
    extern __shared__ unsigned char lds_raw[];
    float *s_tab = (float *)lds_raw;
    unsigned *s_cnt = (unsigned *)(lds_raw + (size_t)(G + 1) * 4);
    if (ctrl[L_FALLBACK]) return;
    const Feature F = *feat;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i <= G; i += HNT) s_tab[i] = tab[i];
    const int64_t w = (int64_t)blockIdx.x * (HNT / 64) + wave;
    unsigned *mycnt = s_cnt + (size_t)wave * B;
    if (w < nwaves)
        for (int i = lane; i < B; i += 64) mycnt[i] = counts[w * B + i] + starts[i];
    __syncthreads();
    if (w >= nwaves) return;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t c0 = w * chunk;
    const int64_t c1 = c0 + chunk < len ? c0 + chunk : len;
    for (int64_t base = c0; base < c1; base += 64 * HIPT) {
        double x[HIPT];
#pragma unroll
        for (int r = 0; r < HIPT; ++r) {
            const int64_t i = base + r * 64 + lane;
            x[r] = src[i < c1 ? i : c1 - 1];
        }
#pragma unroll
        for (int r = 0; r < HIPT; ++r) {
            const int64_t i = base + r * 64 + lane;
            const bool valid = i < c1;
            const int b = valid ? bucket_of(x[r], F, s_tab, G, B) : B;   // B: no bucket
            uint64_t peers = __ballot(valid);
            for (int k = 0; k < bbits + 1; ++k) {
                const uint64_t m = __ballot((b >> k) & 1);
                peers &= ((b >> k) & 1) ? m : ~m;
            }
            const int rank = __popcll(peers & below);
            const int cnt = __popcll(peers);
            unsigned pos = 0;
            if (valid) pos = mycnt[b];
            // every lane has read its count before any leader writes
            __builtin_amdgcn_wave_barrier();
            if (valid && rank == 0) mycnt[b] = pos + (unsigned)cnt;
            __builtin_amdgcn_wave_barrier();
            const int64_t d = (int64_t)pos + rank;
            if (valid && d < len) dst[d] = x[r];
        }
    }
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
    const int64_t shift = hb - L.plain.off_tickets;
    L.plain.off_tickets += shift;
    L.plain.off_status += shift;
    L.plain.off_splits += shift;
    L.plain.off_deps += shift;
    L.plain.bytes += shift;
    int64_t o = al256(L.plain.bytes);
    if (!L.use_learned) {
        L.bytes = o;
        return L;
    }
    const int64_t half = n - n / 2;
    L.nwaves = (half + (1 << 14) - 1) >> 14;      // chunks of >= 2^14 keys per wave
    if (L.nwaves < 1) L.nwaves = 1;
    if (L.nwaves > 2048) L.nwaves = 2048;
    L.chunk = (half + L.nwaves - 1) / L.nwaves;
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
    L.off_counts = o; o = al256(o + 2 * L.nwaves * L.B * 4);
    L.off_totals = o; o = al256(o + 2 * (int64_t)L.B * 4);
    L.off_starts = o; o = al256(o + 2 * (int64_t)L.B * 4);
    L.off_offsets = o; o = al256(o + 2 * (int64_t)(L.B + 1) * 8);
    L.off_segctrl = o; o = al256(o + 2 * 64 * 4);
    L.off_seglists = o; o = al256(o + 2 * 3 * (int64_t)L.B * 4);
    L.bytes = o;
    return L;
}

hipError_t learned_sort_async(double *keys, int64_t n, const gs_learned_params &prm, char *ws,
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
    unsigned *counts = (unsigned *)(ws + L.off_counts);
    unsigned *totals = (unsigned *)(ws + L.off_totals);
    unsigned *starts = (unsigned *)(ws + L.off_starts);
    int64_t *offsets = (int64_t *)(ws + L.off_offsets);
    unsigned *segctrl = (unsigned *)(ws + L.off_segctrl);
    int *seglists = (int *)(ws + L.off_seglists);
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
    hipLaunchKernelGGL(learned_prep_kernel, dim3(1), dim3(1024), 0, st, (const double *)sample, L.S, feat, u, t,
                       ctrl);
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
                              losses, ctrl + L_BAR, ctrl + L_ERR, nullptr, st);
                if (e != hipSuccess) return e;
            }
        }
        e = mlp_forward(params, nullptr, G + 1, raw, G, nullptr, st);
        if (e != hipSuccess) return e;
    }
    if (tr) trace_end(st);
    hipLaunchKernelGGL(learned_table_kernel, dim3(1), dim3(1024), 0, st, (const float *)raw, prm.test_bucket_table,
                       (int)prm.mode, G, tab, ctrl, (const Feature *)feat);

    // 6a-b. counts of both halves before anything moves
    const int64_t nA = n / 2, nB = n - nA;                 // first and second half
    const size_t lds = (size_t)(G + 1) * 4 + (size_t)(HNT / 64) * B * 4;
    (void)hipFuncSetAttribute((const void *)learned_hist_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    (void)hipFuncSetAttribute((const void *)learned_scatter_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    const unsigned hgrid = (unsigned)((L.nwaves + (HNT / 64) - 1) / (HNT / 64));
    const int64_t chunkA = (nA + L.nwaves - 1) / L.nwaves;
    const int64_t chunkB = (nB + L.nwaves - 1) / L.nwaves;
    unsigned *countsA = counts, *countsB = counts + L.nwaves * B;
    if (tr) trace_begin(TK_LEARN_BUCKET, st);
    hipLaunchKernelGGL(learned_hist_kernel, dim3(hgrid), dim3(HNT), lds, st, (const double *)keys, nA, chunkA,
                       L.nwaves, (const Feature *)feat, (const float *)tab, G, B, countsA, (const unsigned *)ctrl);
    hipLaunchKernelGGL(learned_hist_kernel, dim3(hgrid), dim3(HNT), lds, st, (const double *)(keys + nA), nB,
                       chunkB, L.nwaves, (const Feature *)feat, (const float *)tab, G, B, countsB,
                       (const unsigned *)ctrl);
    hipLaunchKernelGGL(learned_colscan_kernel, dim3((unsigned)((B + 63) / 64)), dim3(256), 0, st, countsA,
                       L.nwaves, B, totals, (const unsigned *)ctrl);
    hipLaunchKernelGGL(learned_colscan_kernel, dim3((unsigned)((B + 63) / 64)), dim3(256), 0, st, countsB,
                       L.nwaves, B, totals + B, (const unsigned *)ctrl);
    const int64_t limit = (int64_t)1 << 20;
    hipLaunchKernelGGL(learned_bucket_scan_kernel, dim3(1), dim3(1024), 0, st, (const unsigned *)totals, B, 2,
                       starts, offsets, limit, ctrl);
    if (tr) trace_end(st);

    // 6c. second half -> half buffer, sorted there with its vacated region as scratch
    if (tr) trace_begin(TK_LEARN_BUCKET, st);
    hipLaunchKernelGGL(learned_scatter_kernel, dim3(hgrid), dim3(HNT), lds, st, (const double *)(keys + nA), nB,
                       chunkB, L.nwaves, (const Feature *)feat, (const float *)tab, G, B, bbits,
                       (const unsigned *)countsB, (const unsigned *)(starts + B), H, (const unsigned *)ctrl);
    if (tr) trace_end(st);
    e = segsort_core_async(H, offsets + (B + 1), B, nB, keys + nA, segctrl + 64, seglists + 3 * B,
                           seglists + 4 * B, seglists + 5 * B, ctrl + L_FALLBACK, 0u, st);
    if (e != hipSuccess) return e;
    // first half -> the top nA slots of the vacated second-half region
    if (tr) trace_begin(TK_LEARN_BUCKET, st);
    hipLaunchKernelGGL(learned_scatter_kernel, dim3(hgrid), dim3(HNT), lds, st, (const double *)keys, nA, chunkA,
                       L.nwaves, (const Feature *)feat, (const float *)tab, G, B, bbits, (const unsigned *)countsA,
                       (const unsigned *)starts, keys + nB, (const unsigned *)ctrl);
    if (tr) trace_end(st);
    e = segsort_core_async(keys + nB, offsets, B, nA, keys, segctrl, seglists, seglists + B, seglists + 2 * B,
                           ctrl + L_FALLBACK, 0u, st);
    if (e != hipSuccess) return e;

    // 7. merge: first run (sorted first half) at [nB, n), second run in the
    //    half buffer (logical [n, n+nB)), output [0, n) written bottom-up
    FrogMerge fm{};
    fm.l0 = nB;
    fm.nl = nA;
    fm.r0 = n;
    fm.nr = nB;
    fm.out0 = 0;
    fm.left = 0;
    fm.outer = 2;
    e = merge_one_f64_async(keys, H, n, fm, ws, L.plain, st, ctrl + L_FALLBACK, 0u);
    if (e != hipSuccess) return e;

    // plain path on the untouched input if the bucketing was rejected
    e = sort_f64_async(keys, n, ws, L.plain, st, ctrl + L_FALLBACK, 1u);
    if (e != hipSuccess) return e;
    return hipGetLastError();
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
    r->fallback = c[L_FALLBACK];
    r->order_violation = c[L_ORDER];
    r->overflow_buckets = c[L_OVERFLOW];
    r->max_bucket = c[L_MAXB];
    r->big_buckets = c[L_BIGB];
    r->err = c[L_ERR];
    r->feature = c[L_FEAT];
    r->loss_first = loss[0];
    r->loss_last = loss[1];
    return hipSuccess;
}

}  // namespace gs
