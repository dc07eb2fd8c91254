"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws numbers.  It holds none of the sorting method's
arithmetic: no comparison, merge, layout or bucketing.  Both the CPU oracle and
the GPU library receive the arrays built here.

Random bits come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used as a counter-based
generator: draw i of stream s is mix64(s + (i + 1) * GAMMA), with GAMMA the
golden-ratio increment and mix64 the Stafford variant-13 finaliser from that
paper.  Streams are keyed by (workload id, pattern id, seed), so every array is
reproducible from its recipe alone.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_CHUNK = 1 << 22


def _threads() -> int:
    return max(1, min(8, os.cpu_count() or 1))


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (in place on a uint64 array, also returned)."""
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def stream_seed(workload: int, pattern: int, seed: int) -> int:
    """One 64-bit stream key per (workload id, pattern id, seed)."""
    z = np.array([(workload << 32) + (pattern << 16) + seed], dtype=np.uint64)
    return int(mix64(z)[0])


def _fill(n: int, fn, dtype) -> np.ndarray:
    out = np.empty(n, dtype=dtype)
    starts = list(range(0, n, _CHUNK))
    if len(starts) <= 1:
        if n:
            fn(0, n, out)
        return out
    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(lambda a: fn(a, min(a + _CHUNK, n), out), starts))
    return out


def u64(n: int, key: int, offset: int = 0) -> np.ndarray:
    """n raw 64-bit draws of stream `key`, starting at draw `offset`."""
    k = np.uint64(key % (1 << 64))

    def fn(a, b, out):
        with np.errstate(over="ignore"):
            z = (np.arange(a + offset + 1, b + offset + 1, dtype=np.uint64) * GAMMA) + k
        out[a:b] = mix64(z)

    return _fill(n, fn, np.uint64)


def uniform01(n: int, key: int, offset: int = 0) -> np.ndarray:
    """U[0,1) doubles: the top 53 bits times 2^-53 (exact; never -0, NaN or 1)."""
    k = np.uint64(key % (1 << 64))

    def fn(a, b, out):
        with np.errstate(over="ignore"):
            z = (np.arange(a + offset + 1, b + offset + 1, dtype=np.uint64) * GAMMA) + k
        z = mix64(z) >> np.uint64(11)
        out[a:b] = z.astype(np.float64) * (1.0 / 9007199254740992.0)

    return _fill(n, fn, np.float64)


def _chunked(n: int, fn, dtype) -> np.ndarray:
    """out[a:b] = fn(a, b) over chunks, on a thread pool (numpy releases the GIL)."""
    def fill(a, b, out):
        out[a:b] = fn(a, b)
    return _fill(n, fill, dtype)


def normal(n: int, key: int) -> np.ndarray:
    """Standard normal deviates by Box-Muller from two uniform streams."""
    u1 = uniform01(n, key, 0)
    u2 = uniform01(n, key ^ 0x5DEECE66D, 0)
    # (0, 1] for the log: 1 - u1
    return _chunked(n, lambda a, b: np.sqrt(-2.0 * np.log(1.0 - u1[a:b]))
                    * np.cos(2.0 * math.pi * u2[a:b]), np.float64)


def permute_indices(j: np.ndarray, n: int, key: int) -> np.ndarray:
    """A seeded bijection of [0, n), applied to the indices j.

    Rounds of (x * odd + c) mod 2^b and x ^= x >> (b/2) are bijections of
    [0, 2^b); cycle walking restricts the permutation to [0, n).
    """
    if n <= 1:
        return np.zeros_like(j, dtype=np.int64)
    bits = max(2, int(math.ceil(math.log2(n))))
    mask = np.uint64((1 << bits) - 1)
    consts = u64(8, key)
    x = np.asarray(j, dtype=np.uint64).copy()

    def rounds(v):
        with np.errstate(over="ignore"):
            for r in range(4):
                v = (v * (consts[2 * r] | np.uint64(1)) + consts[2 * r + 1]) & mask
                v ^= v >> np.uint64(bits // 2)
        return v

    x = rounds(x)
    bad = x >= np.uint64(n)
    while bad.any():
        x[bad] = rounds(x[bad])
        bad = x >= np.uint64(n)
    return x.astype(np.int64)


# ---------------------------------------------------------------------------
# plain f64 patterns (uniform, tied, presorted, reversed, perturbed)
# ---------------------------------------------------------------------------
PATTERNS = ("uniform", "tied", "presorted", "reversed", "perturbed")
_PATTERN_ID = {p: i for i, p in enumerate(PATTERNS + ("zeros_signed", "lognormal",
                                                      "gaussmix", "zipf_ints",
                                                      "zipf", "uniform_u64", "few"))}


def f64_pattern(pattern: str, n: int, seed: int = 0, workload: int = 2,
                distinct: int = 1 << 14, perturb: float = 0.1) -> np.ndarray:
    """float64 keys of one of the named patterns.

    uniform      i.i.d. U[0,1)
    tied         keys drawn uniformly from `distinct` distinct U[0,1) values
    presorted    ascending: x_i = (i + u_i) / n with u_i ~ U[0,1)
    reversed     the presorted array in descending order
    perturbed    presorted, then floor(perturb*n) positions (distinct, chosen by
                 a seeded permutation) replaced by fresh U[0,1)
    zeros_signed 30% zeros of random sign, the rest from 64 distinct small
                 values of either sign (ties and -0/+0 everywhere)
    """
    key = stream_seed(workload, _PATTERN_ID[pattern], seed)
    if pattern == "uniform":
        return uniform01(n, key)
    if pattern == "tied":
        table = np.unique(uniform01(4 * distinct, key ^ 0xA5A5))
        if table.size < distinct:
            raise RuntimeError("not enough distinct table values")
        table = table[permute_indices(np.arange(distinct), table.size, key)[:distinct]]
        idx = (u64(n, key) >> np.uint64(64 - int(math.log2(distinct)))).astype(np.int64) \
            if distinct & (distinct - 1) == 0 else (u64(n, key) % np.uint64(distinct)).astype(np.int64)
        return table[idx]
    if pattern in ("presorted", "reversed", "perturbed"):
        x = (np.arange(n, dtype=np.float64) + uniform01(n, key)) / float(max(n, 1))
        if pattern == "reversed":
            return x[::-1].copy()
        if pattern == "perturbed":
            k = int(math.floor(perturb * n))
            pos = permute_indices(np.arange(k), n, key ^ 0x1234)
            x[pos] = uniform01(k, key ^ 0x4321)
        return x
    if pattern == "zeros_signed":
        u = u64(n, key)
        vals = np.concatenate([np.arange(1, 33, dtype=np.float64) / 8.0,
                               -np.arange(1, 33, dtype=np.float64) / 8.0])
        x = vals[(u & np.uint64(63)).astype(np.int64)]
        zero = ((u >> np.uint64(8)) % np.uint64(10)) < np.uint64(3)
        neg = ((u >> np.uint64(20)) & np.uint64(1)) == np.uint64(1)
        x[zero] = np.where(neg[zero], -0.0, 0.0)
        return x
    raise ValueError(pattern)


# ---------------------------------------------------------------------------
# the paper's measurement patterns ("Methods and measurement")
# ---------------------------------------------------------------------------
PAPER_PATTERNS = ("permut", "tielog2", "ascall", "descall", "asclocal", "ascglobal",
                  "desclocal", "descglobal")
_PAPER_ID = {p: 32 + i for i, p in enumerate(PAPER_PATTERNS)}


def permute_in_groups(idx: np.ndarray, group: np.ndarray, size: int, key: int) -> np.ndarray:
    """For every element, a seeded bijection of [0, size) chosen by its group
    id, applied to idx (in [0, size)): each group gets its own permutation.
    Same construction as permute_indices, with round constants drawn per
    group."""
    if size <= 1:
        return np.zeros_like(idx, dtype=np.int64)
    bits = max(2, int(math.ceil(math.log2(size))))
    mask = np.uint64((1 << bits) - 1)
    g = np.asarray(group, dtype=np.uint64)
    consts = []
    with np.errstate(over="ignore"):
        for r in range(8):
            consts.append(mix64(g * GAMMA + np.uint64((key + 0x51ED * (r + 1)) & 0xFFFFFFFFFFFFFFFF)))
    x = np.asarray(idx, dtype=np.uint64).copy()

    def rounds(v, sel):
        with np.errstate(over="ignore"):
            for r in range(4):
                v = (v * (consts[2 * r][sel] | np.uint64(1)) + consts[2 * r + 1][sel]) & mask
                v ^= v >> np.uint64(bits // 2)
        return v

    allsel = np.ones(x.size, dtype=bool)
    x = rounds(x, allsel)
    bad = x >= np.uint64(size)
    while bad.any():
        x[bad] = rounds(x[bad], bad)
        bad = x >= np.uint64(size)
    return x.astype(np.int64)


def paper_pattern(pattern: str, n: int, seed: int = 0, workload: int = 2) -> np.ndarray:
    """float64 keys of the paper's measurement patterns (distinct integers
    unless tied), with sqrt(n) runs of length L = round(sqrt(n)) (the last
    run shorter when L does not divide n):

    permut      a random permutation of 1..n
    tielog2     draws from ceil(log2 n) distinct random values
    ascall      1..n ascending;  descall: n..1
    asclocal    L-long ascending runs whose values are spread at random over
                the whole range: run b, place j holds j*B + s_j(b) + 1, with B
                runs and s_j a random permutation of the runs for every place j
    ascglobal   run b holds the b-th quantile b*L+1 .. (b+1)*L, in random order
    desclocal   as asclocal with every run descending
    descglobal  as ascglobal with the quantiles in descending order
    """
    key = stream_seed(workload, _PAPER_ID[pattern], seed)
    if n == 0:
        return np.zeros(0, dtype=np.float64)
    pos = np.arange(n, dtype=np.int64) if n <= 1 << 24 else None
    if pattern == "permut":
        pos = np.arange(n, dtype=np.int64)
        return (permute_indices(pos, n, key) + 1).astype(np.float64)
    if pattern == "tielog2":
        d = max(1, int(math.ceil(math.log2(max(n, 2)))))
        table = np.unique(uniform01(4 * d + 16, key ^ 0xA5A5))[:d]
        return table[(u64(n, key) % np.uint64(table.size)).astype(np.int64)]
    if pattern == "ascall":
        return np.arange(1, n + 1, dtype=np.float64)
    if pattern == "descall":
        return np.arange(n, 0, -1, dtype=np.float64)
    if pattern not in ("asclocal", "desclocal", "ascglobal", "descglobal"):
        raise ValueError(pattern)
    L = max(1, int(round(math.sqrt(n))))
    B = -(-n // L)

    def fill(a, e, out):
        p = np.arange(a, e, dtype=np.int64)
        b, j = p // L, p % L
        if pattern in ("asclocal", "desclocal"):
            jj = j if pattern == "asclocal" else (L - 1 - j)
            out[a:e] = jj * B + permute_in_groups(b, jj, B, key) + 1
        else:
            q = b if pattern == "ascglobal" else (B - 1 - b)
            out[a:e] = q * L + permute_in_groups(j, b, L, key) + 1
    return _fill(n, fill, np.float64)


# ---------------------------------------------------------------------------
# key-value workloads (uint64 keys, uint32 payload = original index)
# ---------------------------------------------------------------------------
def zipf_cdf(values: int, s: float) -> np.ndarray:
    """Cumulative Zipf(s) weights over ranks 1..values, normalised to end at 1."""
    w = np.arange(1, values + 1, dtype=np.float64) ** (-s)
    c = np.cumsum(w)
    return c / c[-1]


def zipf_ranks(n: int, key: int, values: int = 1 << 20, s: float = 1.1) -> np.ndarray:
    """Zipf(s) ranks in [0, values) by inverse CDF (binary search on U)."""
    cdf = zipf_cdf(values, s)
    u = uniform01(n, key)
    return _chunked(n, lambda a, b: np.minimum(np.searchsorted(cdf, u[a:b], side="right"),
                                               values - 1), np.int64)


def kv_pattern(pattern: str, n: int, seed: int = 0, workload: int = 3,
               values: int = 1 << 20, s: float = 1.1):
    """(uint64 keys, uint32 payload = original index)."""
    key = stream_seed(workload, _PATTERN_ID[pattern if pattern != "uniform" else "uniform_u64"], seed)
    if pattern == "uniform":
        k = u64(n, key)
    elif pattern == "zipf":
        table = u64(values, key ^ 0xBEEF)            # distinct with overwhelming odds
        k = table[zipf_ranks(n, key, values, s)]
    elif pattern == "few":
        k = u64(n, key) & np.uint64(7)
    else:
        raise ValueError(pattern)
    return k, np.arange(n, dtype=np.uint32)


# ---------------------------------------------------------------------------
# segmented workloads
# ---------------------------------------------------------------------------
def seg_lengths(num_segments: int, lo: int, hi: int, key: int, total: int | None = None):
    """Log-uniform integer lengths in [lo, hi]; if `total` is given all lengths
    are rescaled (by a factor close to 1) so that they sum to it exactly."""
    u = uniform01(num_segments, key)
    lens = np.floor(np.exp(math.log(lo) + u * (math.log(hi + 1) - math.log(lo)))).astype(np.int64)
    lens = np.clip(lens, lo, hi)
    if total is not None and lens.size:
        # rescale to the exact total, then hand out the rounding remainder one
        # key at a time to the first segments
        lens = np.floor(lens * (total / float(lens.sum()))).astype(np.int64)
        rem = total - int(lens.sum())
        lens[: rem] += 1
    return lens


def seg_lengths_until(total: int, lo: int, hi: int, key: int):
    """Log-uniform integer lengths in [lo, hi] drawn until they reach `total`
    keys; the last length is cut so that they sum to it exactly."""
    mean = (hi + 1 - lo) / (math.log(hi + 1) - math.log(lo))
    m = int(total / mean * 1.2) + 64
    while True:
        u = uniform01(m, key)
        lens = np.clip(np.floor(np.exp(math.log(lo) + u * (math.log(hi + 1) - math.log(lo)))).astype(np.int64),
                       lo, hi)
        c = np.cumsum(lens)
        if c[-1] >= total:
            k = int(np.searchsorted(c, total))          # first prefix reaching the total
            lens = lens[: k + 1].copy()
            lens[k] -= int(c[k]) - total
            return lens
        m *= 2


def segmented(num_segments: int | None, lo: int, hi: int, seed: int = 0, total: int | None = None,
              workload: int = 4, patterns=("uniform", "tied", "presorted", "reversed")):
    """(keys, int64 offsets): segments of log-uniform length, each filled with a
    pattern drawn uniformly from `patterns`.  With num_segments None, lengths
    are drawn until they hold `total` keys (the last one cut to fit).

    uniform   i.i.d. U[0,1)
    tied      draws from 1024 distinct U[0,1) values
    presorted ascending within the segment: (position + u) / length
    reversed  1 - presorted (descending within the segment)
    """
    key = stream_seed(workload, 0, seed)
    if num_segments is None:
        lens = seg_lengths_until(int(total), lo, hi, key)
        num_segments = lens.size
    else:
        lens = seg_lengths(num_segments, lo, hi, key, total)
    off = np.zeros(num_segments + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    n = int(off[-1])
    pat = (u64(num_segments, key ^ 0x77) % np.uint64(len(patterns))).astype(np.int64)
    pat_of = np.repeat(pat, lens)
    x = uniform01(n, key ^ 0x99)
    if "tied" in patterns:
        tab = np.unique(uniform01(1 << 12, key ^ 0x3C3C))[: 1 << 10]
        sel = pat_of == patterns.index("tied")
        tix = (u64(n, key ^ 0x55) >> np.uint64(54)).astype(np.int64)
        x[sel] = tab[tix[sel] % tab.size]
    ordered = [patterns.index(p) for p in ("presorted", "reversed") if p in patterns]
    if ordered:
        pos = np.arange(n, dtype=np.float64) - np.repeat(off[:-1], lens).astype(np.float64)
        ln = np.repeat(np.maximum(lens, 1), lens).astype(np.float64)
        v = (pos + x) / ln
        if "presorted" in patterns:
            sel = pat_of == patterns.index("presorted")
            x[sel] = v[sel]
        if "reversed" in patterns:
            sel = pat_of == patterns.index("reversed")
            x[sel] = 1.0 - v[sel]
    return x, off


# ---------------------------------------------------------------------------
# learned-path distributions
# ---------------------------------------------------------------------------
def learned_pattern(pattern: str, n: int, seed: int = 0, workload: int = 5):
    """lognormal(0,2); a mixture of 8 Gaussians (means U[-100,100], std
    log-uniform in [0.1,10], equal weights); Zipf(1.1) ranks over 2^20 mapped
    through a seeded permutation of [1, 2^20] and cast to float64."""
    key = stream_seed(workload, _PATTERN_ID[pattern], seed)
    if pattern == "lognormal":
        z = normal(n, key)
        return _chunked(n, lambda a, b: np.exp(2.0 * z[a:b]), np.float64)
    if pattern == "gaussmix":
        prm = uniform01(16, key ^ 0xF00D)
        mu = -100.0 + 200.0 * prm[:8]
        sd = np.exp(math.log(0.1) + prm[8:] * (math.log(10.0) - math.log(0.1)))
        comp = (u64(n, key ^ 0xC0) >> np.uint64(61)).astype(np.int64)
        return mu[comp] + sd[comp] * normal(n, key)
    if pattern == "zipf_ints":
        values = 1 << 20
        r = zipf_ranks(n, key, values, 1.1)
        perm = permute_indices(np.arange(values), values, key ^ 0xABCD) + 1
        return perm[r].astype(np.float64)
    raise ValueError(pattern)
