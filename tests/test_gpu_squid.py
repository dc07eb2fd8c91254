"""Squidsort on the GPU: run directions carried up the single Frogsort1 tree,
the non-overlap test, descending outer runs turned around before their
parent's merge and the final reversal, checked element by element against
the oracle on the paper's
measurement patterns ("Methods and measurement") and on mixtures of
ascending, descending and tied runs of every length from a few keys to
several leaves; at the full size on sampled outputs."""
import numpy as np
import pytest

import workloads as W
from gpu_util import announce, bits, multiset_hash_dev, need_gpu, to_dev

pytestmark = pytest.mark.gpu

PAPER = ["permut", "tielog2", "asclocal", "ascglobal", "desclocal", "descglobal"]
SIZES = [8193, 100_003, (1 << 20) + 7, 1 << 22]


@pytest.fixture(scope="module")
def gs():
    need_gpu()
    import paper_2402_01816_amd as g
    return g


@pytest.mark.parametrize("pattern", PAPER)
@pytest.mark.parametrize("n", SIZES)
def test_paper_patterns_f64(gs, orc, pattern, n):
    announce("squid f64", pattern, n)
    x = W.paper_pattern(pattern, n, seed=41)
    t = to_dev(x)
    rep = gs.gs_sort_f64(t, report=True)
    assert np.array_equal(bits(t), bits(orc.sort_f64(x)))
    assert rep["order"] == 0
    assert 0 < rep["keys_moved"] <= n * (rep["levels"] + 2)


@pytest.mark.parametrize("pattern", PAPER)
@pytest.mark.parametrize("target", ["AscLeft", "AscRight", "DescLeft", "DescRight"])
def test_paper_patterns_kv_targets(gs, orc, pattern, target):
    """Key/value with payload = index (stability visible) on every target:
    DescLeft sorts in the reversed key order, so the roles of the ascending
    and descending patterns swap."""
    n = (1 << 20) + 3
    announce("squid kv", pattern, target, n)
    x = W.paper_pattern(pattern, n, seed=42)
    k = (x * 4).astype(np.uint64) // np.uint64(5)            # some ties
    v = np.arange(n, dtype=np.uint32)
    tk, tv = to_dev(k.view(np.int64)), to_dev(v.view(np.int32))
    gs.gs_sort_kv(tk, tv, target=target)
    rk, rv = orc.sort_kv_target(k, v, target)
    assert np.array_equal(tk.cpu().numpy().view(np.uint64), rk)
    assert np.array_equal(tv.cpu().numpy().view(np.uint32), rv)


def _mixed_runs(rng, n, max_run, values):
    parts, total = [], 0
    while total < n:
        m = int(rng.integers(1, max_run + 1))
        kind = int(rng.integers(0, 5))
        if kind == 0:                                    # strictly descending
            r = np.sort(rng.choice(values, size=min(m, values), replace=False))[::-1]
        elif kind == 1:                                  # descending with ties
            r = np.sort(rng.integers(0, values, m))[::-1]
        elif kind == 2:                                  # ascending with ties
            r = np.sort(rng.integers(0, values, m))
        elif kind == 3:                                  # constant
            r = np.full(m, rng.integers(0, values))
        else:                                            # random
            r = rng.integers(0, values, m)
        parts.append(r.astype(np.float64))
        total += r.size
    return np.concatenate(parts)[:n]


@pytest.mark.parametrize("seed", range(16))
def test_mixed_runs_f64(gs, orc, seed):
    """Runs of every kind and length (up to several leaves), ties as signed
    zeros and repeated values, occasional NaN: every node mode is taken."""
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.choice([8193, 40_000, 300_001, (1 << 20) + 5, 3_000_017]))
    max_run = int(rng.choice([50, 3000, 20_000, 200_000]))
    values = int(rng.choice([4, 1000, 1 << 40]))
    x = _mixed_runs(rng, n, max_run, values)
    x[(x == 0) & (rng.random(n) < 0.5)] = -0.0
    if seed % 4 == 3:
        x[rng.integers(0, n, 5)] = np.nan
    announce("squid mixed f64", seed, n, max_run, values)
    t = to_dev(x)
    gs.gs_sort_f64(t)
    assert np.array_equal(bits(t), bits(orc.sort_f64(x)))
    t = to_dev(x)
    gs.gs_sort_f64(t, target="DescLeft")
    assert np.array_equal(bits(t), bits(orc.sort_f64_target(x, "DescLeft")))


@pytest.mark.parametrize("blocks", [2, 4, 8, 64, 512])
def test_descending_blocks(gs, orc, blocks):
    """Strictly descending blocks of 2^22 / blocks keys, the blocks in
    ascending or in descending order of their values, or shuffled: whole
    descending sub-trees concatenate, their parents turn a descending outer
    run around and merge, and a top run that ends descending is reversed
    once.  The moves never exceed the plain tree's."""
    n = 1 << 22
    L = n // blocks
    base = np.arange(n, 0, -1, dtype=np.float64).reshape(blocks, L)    # each row strictly descending
    rng = np.random.default_rng(blocks)
    for order in ("desc", "asc", "shuffled"):
        rows = {"desc": np.arange(blocks), "asc": np.arange(blocks)[::-1],
                "shuffled": rng.permutation(blocks)}[order]
        x = base[rows].reshape(-1).copy()
        x[-1], x[-2] = x[-2], x[-1]                        # not the whole-array reversal
        announce("squid desc blocks", blocks, order)
        t = to_dev(x)
        rep = gs.gs_sort_f64(t, report=True)
        assert rep["order"] == 0
        assert np.array_equal(bits(t), bits(orc.sort_f64(x))), order
        assert rep["keys_moved"] <= n * (rep["levels"] + 1)


@pytest.mark.parametrize("k", [20, 22])
def test_ascglobal_moves_closed_form(gs, k):
    """ascglobal with quantile runs shorter than a leaf: every leaf comes back
    ascending and no two leaves overlap, so every node is a concatenation:
    the leaves move n keys and each level moves only its inner runs, n/2."""
    n = 1 << k
    x = W.paper_pattern("ascglobal", n, seed=43)
    t = to_dev(x)
    rep = gs.gs_sort_f64(t, report=True)
    depth = rep["levels"]
    assert rep["keys_moved"] == n + depth * (n // 2)
    assert np.array_equal(bits(t), bits(np.arange(1, n + 1, dtype=np.float64)))


def test_full_merge_moves(gs):
    """Uniform keys: every leaf and every level moves every key."""
    n = 1 << 22
    x = W.f64_pattern("uniform", n, seed=44)
    rep = gs.gs_sort_f64(to_dev(x), report=True)
    assert rep["keys_moved"] == n * (rep["levels"] + 1)


@pytest.mark.parametrize("pattern", ["asclocal", "ascglobal", "desclocal", "descglobal"])
def test_paper_patterns_full_size(gs, orc, pattern):
    """n = 2^28: sampled output positions against the oracle's counting form
    of the definition, sortedness and the multiset of the bits."""
    torch = need_gpu()
    n = 1 << 28
    announce("squid full size", pattern, n)
    x = W.paper_pattern(pattern, n, seed=45)
    t = torch.from_numpy(x).to("cuda")
    h0 = multiset_hash_dev(t)
    rep = gs.gs_sort_f64(t, report=True)
    assert bool((t[1:] >= t[:-1]).all().item())
    assert multiset_hash_dev(t) == h0
    idx = np.concatenate([[0, n - 1], np.random.default_rng(1).integers(0, n, 14)])
    ranks = orc.rank_f64(x, idx)
    got = t[torch.from_numpy(ranks).to("cuda")].cpu().numpy()
    assert np.array_equal(bits(got), bits(x[idx]))
    assert rep["keys_moved"] <= n * (rep["levels"] + 1)
    del t
    torch.cuda.empty_cache()
