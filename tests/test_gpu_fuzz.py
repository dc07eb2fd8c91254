"""Seeded random mix of calls against the oracle.

Each case draws a size log-uniform over [2, 2^21], a pattern (NaN and
infinities sprinkled into some), a target and a tree (Frogsort1, Frogsort3,
Frogsort2, Frogsort6 at random buffer fractions); segmented cases draw a
random layout (empty segments, keys outside every segment, some segments
presorted or reversed).  Every result is compared bit for bit with the
oracle's definition.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import announce, bits, need_gpu, to_dev

pytestmark = pytest.mark.gpu

F64_PATTERNS = ["uniform", "tied", "presorted", "reversed", "perturbed", "zeros_signed"]
KV_PATTERNS = ["uniform", "zipf", "few"]
TARGETS = ("AscLeft", "AscRight", "DescLeft", "DescRight")


@pytest.fixture(scope="module")
def gs():
    need_gpu()
    import paper_2402_01816_amd as g
    return g


def _size(rng, hi=1 << 21):
    return int(np.exp(rng.uniform(np.log(2), np.log(hi))))


def _tree(rng):
    c = int(rng.integers(4))
    if c == 1:
        return dict(buffer_fraction=float(rng.choice([0.3, 0.25, 0.1])))            # Frogsort3
    if c == 2:
        return dict(buffer_fraction=float(rng.choice([0.25, 0.1])), algo="frogsort2")
    if c == 3:
        return dict(buffer_fraction=0.1, algo="frogsort6", sub_fraction=0.25)
    return {}


@pytest.mark.parametrize("seed", range(24))
def test_fuzz_sort_f64(gs, orc, seed):
    rng = np.random.default_rng(7000 + seed)
    n = _size(rng)
    pattern = F64_PATTERNS[int(rng.integers(len(F64_PATTERNS)))]
    target = TARGETS[int(rng.integers(4))]
    x = W.f64_pattern(pattern, n, seed=seed)
    if rng.random() < 0.3:
        m = max(1, n // 97)
        x[rng.integers(0, n, m)] = rng.choice([np.nan, np.inf, -np.inf], m)
    kw = _tree(rng)
    announce("fuzz f64", seed, pattern, target, n, kw)
    t = to_dev(x)
    gs.gs_sort_f64(t, target=target, **kw)
    assert np.array_equal(bits(t), bits(orc.sort_f64_target(x, target)))


@pytest.mark.parametrize("seed", range(12))
def test_fuzz_sort_kv(gs, orc, seed):
    rng = np.random.default_rng(8000 + seed)
    n = _size(rng)
    pattern = KV_PATTERNS[int(rng.integers(len(KV_PATTERNS)))]
    target = TARGETS[int(rng.integers(4))]
    k, v = W.kv_pattern(pattern, n, seed=seed)
    kw = _tree(rng)
    announce("fuzz kv", seed, pattern, target, n, kw)
    tk = to_dev(k.view(np.int64))
    tv = to_dev(v.view(np.int32))
    gs.gs_sort_kv(tk, tv, target=target, **kw)
    rk, rv = orc.sort_kv_target(k, v, target)
    assert np.array_equal(tk.cpu().numpy().view(np.uint64), rk)
    assert np.array_equal(tv.cpu().numpy().view(np.uint32), rv)


@pytest.mark.parametrize("seed", range(12))
def test_fuzz_segsort(gs, orc, seed):
    rng = np.random.default_rng(9000 + seed)
    nseg = int(rng.integers(1, 3000))
    lens = np.floor(np.exp(rng.uniform(0, np.log(1 << 17), nseg))).astype(np.int64) - 1
    lens[rng.random(nseg) < 0.05] = 0
    head, tail = int(rng.integers(0, 100)), int(rng.integers(0, 100))
    off = np.zeros(nseg + 1, dtype=np.int64)
    off[0] = head
    off[1:] = head + np.cumsum(lens)
    n = int(off[-1]) + tail
    pattern = F64_PATTERNS[int(rng.integers(len(F64_PATTERNS)))]
    x = W.f64_pattern(pattern, n, seed=seed)
    for s in np.flatnonzero(rng.random(nseg) < 0.3):
        seg = np.sort(x[off[s]:off[s + 1]])
        x[off[s]:off[s + 1]] = seg[::-1] if rng.random() < 0.5 else seg
    announce("fuzz segsort", seed, pattern, nseg, n)
    t = to_dev(x)
    gs.gs_segsort(t, to_dev(off))
    assert np.array_equal(bits(t), bits(orc.segsort_f64(x, off)))
