// Second CPU reference (test and benchmark infrastructure, like the rest of
// this directory; nothing of the GPU library calls or links it): the C++
// standard library's stable sort under the key order the paper's definition
// of sorting fixes -- IEEE less on numbers, every NaN after every number, and
// ties (the two zeros, equal NaN ranks) kept in input order.  It serves as a
// pin of the oracle (same bits out on every input) and as a timed CPU
// baseline beside it.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <utility>
#include <vector>

namespace {

bool less_f64(double a, double b)
{
    if (std::isnan(a)) return false;
    if (std::isnan(b)) return true;
    return a < b;
}

}  // namespace

extern "C" void stdsort_stable_f64(double *x, int64_t n)
{
    if (n > 1) std::stable_sort(x, x + n, less_f64);
}

// keys compared as unsigned 64-bit integers, each value travelling with its key
extern "C" void stdsort_stable_kv(uint64_t *k, uint32_t *v, int64_t n)
{
    if (n <= 1) return;
    std::vector<std::pair<uint64_t, uint32_t>> p((size_t)n);
    for (int64_t i = 0; i < n; ++i) p[(size_t)i] = {k[i], v[i]};
    std::stable_sort(p.begin(), p.end(),
                     [](const std::pair<uint64_t, uint32_t> &a, const std::pair<uint64_t, uint32_t> &b) {
                         return a.first < b.first;
                     });
    for (int64_t i = 0; i < n; ++i) {
        k[i] = p[(size_t)i].first;
        v[i] = p[(size_t)i].second;
    }
}
