"""Pins of the CPU oracle against facts fixed outside it.

Each test checks the oracle against something other than itself: the paper's
worked layout tables, closed-form counts the paper states, brute force over all
permutations, an exhaustive enumeration of weak orders checked against the
counting form of the definition, numpy's stable sort (a library routine that
implements the same ordering), finite differences and closed forms for the
network gradients.
"""
import itertools
import math
import os

import numpy as np
import pytest

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# comparison semantics
# --------------------------------------------------------------------------
def test_less_semantics(orc):
    nan, inf = float("nan"), float("inf")
    assert not orc.less_f64(-0.0, 0.0) and not orc.less_f64(0.0, -0.0)
    assert orc.less_f64(-1.0, -0.0) and orc.less_f64(0.0, 5e-324)
    assert orc.less_f64(5e-324, 1e-323)                   # denormals compare exactly
    assert orc.less_f64(inf, nan) and not orc.less_f64(nan, inf)
    assert not orc.less_f64(nan, nan)
    assert orc.less_f64(-inf, -1e308) and not orc.less_f64(1.0, 1.0)


# --------------------------------------------------------------------------
# the result: brute force, exhaustive weak orders, library routine
# --------------------------------------------------------------------------
def _definition_by_brute_force(keys):
    """The unique permutation that orders keys ascending and keeps tied keys
    in input order, found by trying every permutation."""
    n = len(keys)
    found = []
    for perm in itertools.permutations(range(n)):
        ok = True
        for a, b in zip(perm, perm[1:]):
            if keys[b] < keys[a] or (keys[a] == keys[b] and b < a):
                ok = False
                break
        if ok:
            found.append(perm)
    assert len(found) == 1
    return np.array(found[0], dtype=np.int64)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5, 6])
def test_brute_force_small(orc, n):
    rng = np.random.default_rng(100 + n)
    for trial in range(40 if n > 3 else 10):
        keys = rng.integers(0, max(1, n // 2 + 1), size=n).astype(np.uint64)
        k, v = orc.sort_kv(keys, np.arange(n, dtype=np.uint32))
        perm = _definition_by_brute_force(list(keys))
        assert np.array_equal(v, perm.astype(np.uint32))
        assert np.array_equal(k, keys[perm])


def _weak_orders(n):
    """All arrays of length n whose value set is exactly {0..k-1} for some k
    (one representative per weak order; Fubini-many)."""
    if n == 0:
        return np.zeros((1, 0), dtype=np.int64)
    grid = np.indices((n,) * n).reshape(n, -1).T          # n^n candidate arrays
    mx = grid.max(axis=1)
    present = np.zeros((grid.shape[0], n), dtype=bool)
    np.put_along_axis(present, grid, True, axis=1)
    ok = present.sum(axis=1) == mx + 1
    return grid[ok]


FUBINI = [1, 1, 3, 13, 75, 541, 4683, 47293, 545835]


@pytest.mark.parametrize("n", range(0, 9))
def test_exhaustive_weak_orders(orc, n):
    arrs = _weak_orders(n)
    assert arrs.shape[0] == FUBINI[n]
    m = arrs.shape[0]
    keys = arrs.reshape(-1).astype(np.uint64)
    vals = np.tile(np.arange(n, dtype=np.uint32), m)
    off = np.arange(0, m * n + 1, n, dtype=np.int64) if n else np.zeros(m + 1, dtype=np.int64)
    k, v = orc.segsort_kv(keys, vals, off)
    if n == 0:
        return
    # counting form of the definition, vectorised over all arrays
    a = arrs[:, :, None]           # element j
    b = arrs[:, None, :]           # element i
    idx = np.arange(n)
    less = b < a
    tie_before = (b == a) & (idx[None, None, :] < idx[None, :, None])
    rank = (less | tie_before).sum(axis=2)                # [m, n]
    expect_v = np.empty_like(rank)
    np.put_along_axis(expect_v, rank, np.broadcast_to(idx, rank.shape).copy(), axis=1)
    assert np.array_equal(v.reshape(m, n), expect_v.astype(np.uint32))
    assert np.array_equal(k.reshape(m, n), np.take_along_axis(arrs, expect_v, axis=1))
    # the f64 path on the same weak orders, tie class 0 written as signed zeros
    x = arrs.astype(np.float64).reshape(-1)
    sign = (np.arange(x.size) * 2654435761 >> 3) & 1
    x[(x == 0) & (sign == 1)] = -0.0
    y = orc.segsort_f64(x, off).reshape(m, n)
    expect = np.take_along_axis(x.reshape(m, n), expect_v, axis=1)
    assert np.array_equal(y.view(np.uint64), expect.view(np.uint64))


@pytest.mark.parametrize("pattern", ["uniform", "tied", "presorted", "reversed",
                                     "perturbed", "zeros_signed"])
@pytest.mark.parametrize("n", [0, 1, 2, 3, 7, 8, 1000, 4097, 1 << 16])
def test_matches_library_stable_sort(orc, pattern, n):
    x = W.f64_pattern(pattern, n, seed=3)
    y = orc.sort_f64(x)
    ref = x[np.argsort(x, kind="stable")]
    assert np.array_equal(y.view(np.uint64), ref.view(np.uint64))


@pytest.mark.parametrize("pattern", ["uniform", "tied", "presorted", "reversed",
                                     "perturbed", "zeros_signed"])
@pytest.mark.parametrize("n", [0, 1, 2, 1000, 4097, 1 << 16])
def test_matches_std_stable_sort(orc, pattern, n):
    """The C++ standard library's stable sort under the same key order gives
    the same bits (NaN payloads and signed zeros included)."""
    x = W.f64_pattern(pattern, n, seed=4)
    if n > 8:
        rng = np.random.default_rng(n)
        x[rng.integers(0, n, 5)] = np.nan
        x[rng.integers(0, n, 5)] = np.frombuffer(np.uint64(0x7FF8000000000077).tobytes(), dtype=np.float64)[0]
    y = orc.sort_f64(x)
    ref = orc.std_stable_sort_f64(x)
    assert np.array_equal(y.view(np.uint64), ref.view(np.uint64))


@pytest.mark.parametrize("pattern", ["uniform", "zipf", "few"])
def test_kv_matches_std_stable_sort(orc, pattern):
    k0, v0 = W.kv_pattern(pattern, 50_000, seed=2)
    k, v = orc.sort_kv(k0, v0)
    rk, rv = orc.std_stable_sort_kv(k0, v0)
    assert np.array_equal(k, rk) and np.array_equal(v, rv)


def test_nan_inf_denormal_order(orc):
    x = np.array([np.nan, 1.0, -np.inf, 5e-324, -0.0, np.inf, 0.0, -5e-324,
                  np.float64(np.nan), -0.0, 1.0], dtype=np.float64)
    x[8] = np.frombuffer(np.uint64(0x7FF8000000000123).tobytes(), dtype=np.float64)[0]
    y = orc.sort_f64(x)
    ref = x[np.argsort(x, kind="stable")]
    assert np.array_equal(y.view(np.uint64), ref.view(np.uint64))
    # NaNs last with payload bits preserved and in input order
    assert np.isnan(y[-2:]).all()
    assert y[-1].view(np.uint64) == np.uint64(0x7FF8000000000123)


@pytest.mark.parametrize("pattern", ["uniform", "zipf", "few"])
def test_kv_matches_library(orc, pattern):
    k0, v0 = W.kv_pattern(pattern, 50_000, seed=1)
    k, v = orc.sort_kv(k0, v0)
    p = np.argsort(k0, kind="stable")
    assert np.array_equal(k, k0[p]) and np.array_equal(v, v0[p].astype(np.uint32))


def test_segsort_matches_library(orc):
    x, off = W.segmented(300, 1, 3000, seed=5)
    y = orc.segsort_f64(x, off)
    for s in range(off.size - 1):
        seg = x[off[s]:off[s + 1]]
        ref = seg[np.argsort(seg, kind="stable")]
        assert np.array_equal(y[off[s]:off[s + 1]].view(np.uint64), ref.view(np.uint64))


def test_segsort_rejects_bad_offsets(orc):
    with pytest.raises(ValueError):
        orc.segsort_f64(np.zeros(10), np.array([0, 5, 3, 10]))


def test_rank_matches_library(orc):
    x = W.f64_pattern("zeros_signed", 20_000, seed=9)
    pos = np.empty(x.size, dtype=np.int64)
    pos[np.argsort(x, kind="stable")] = np.arange(x.size)
    idx = np.arange(0, x.size, 997)
    assert np.array_equal(orc.rank_f64(x, idx), pos[idx])
    k, _ = W.kv_pattern("few", 20_000, seed=2)
    pos[np.argsort(k, kind="stable")] = np.arange(k.size)
    assert np.array_equal(orc.rank_u64(k, idx), pos[idx])


# --------------------------------------------------------------------------
# the frog model: paper tables, rules, adaptivity counts
# --------------------------------------------------------------------------
def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split()[1:])
    return rows


def _letters(labels, names):
    return [names[lab] if lab >= 0 else "_" for lab in labels]


def _matches(row, got):
    for want, have in zip(row, got):
        if want == ".":
            continue
        if want.islower():
            if have != "_":
                return False
        elif want != have:
            return False
    return True


def test_golden_frogsort1_n3(orc):
    rows = _read_golden("frogsort1_n3.txt")
    names = ["A", "C", "D"]
    r = orc.frog_model(np.array([1.0, 2.0, 3.0]), g=1, max_snap=8)
    assert r["nslots"] == 4                              # n + floor(n/2)
    assert _matches(rows[0], _letters(r["setup"], names))
    assert r["trace"].shape[0] == 2
    assert _matches(rows[1], _letters(r["trace"][0], names))
    assert _matches(rows[2], _letters(r["trace"][1], names))
    # a layout that misplaces the surplus element would fail here
    assert list(r["setup"]) == [0, -1, 1, 2]


def test_golden_frogsort0_triplets(orc):
    rows = _read_golden("frogsort0_triplets.txt")
    names = ["A", "C", "D", "F", "G", "I"]
    r = orc.frog_model(np.arange(1.0, 7.0), g=2, max_snap=16)
    assert r["nslots"] == 9
    assert _matches(rows[0], _letters(r["setup"], names))
    snaps = [_letters(t, names) for t in r["trace"]]
    # snapshots: triplet 1, triplet 2, merge(1,2), triplet 3, top merge
    assert len(snaps) == 5
    assert _matches(rows[1], snaps[1])
    assert _matches(rows[2], snaps[3])
    assert _matches(rows[3], snaps[4])


@pytest.mark.parametrize("n", list(range(1, 70)) + [255, 256, 1000, 1023, 4097])
def test_frog_model_sorts_stably(orc, n):
    rng = np.random.default_rng(n)
    x = rng.integers(0, max(2, n // 3), size=n).astype(np.float64)
    x[rng.random(n) < 0.2] = -0.0
    r = orc.frog_model(x, g=1)
    p = np.argsort(x, kind="stable")
    assert np.array_equal(r["labels"], p)
    assert np.array_equal(r["keys"].view(np.uint64), x[p].view(np.uint64))


@pytest.mark.parametrize("k", range(1, 15))
def test_frog_presorted_counts(orc, k):
    """Presorted input: every merge touches only its inner run, so compares and
    moves are (n/2) log2 n in total for n = 2^k ("Symmetric merging": 50% of
    the compares and moves of a full merge)."""
    n = 1 << k
    r = orc.frog_model(np.arange(n, dtype=np.float64), g=1)
    assert r["compares"] == (n // 2) * k
    assert r["moves"] == (n // 2) * k


@pytest.mark.parametrize("k", range(1, 13))
def test_frog_reversed_moves(orc, k):
    """Strictly descending input: every merge moves its whole output."""
    n = 1 << k
    r = orc.frog_model(np.arange(n, 0, -1, dtype=np.float64), g=1)
    assert r["moves"] == n * k
    assert np.array_equal(r["keys"], np.arange(1, n + 1, dtype=np.float64))


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 13, 100, 1000, 4097, 1 << 12])
def test_frog_geometry_rules(orc, n):
    """Rule 1 (surplus to the outer side) and rule 2 (buffer floor(n/2)) at
    every depth: children fit their parent's region, the inner child's data
    fit the gap, and every leaf's data start is at or after its input offset."""
    depth = 0
    while (n >> depth) > 1 and depth < 12:
        depth += 1
    for d in range(depth + 1):
        g = orc.frog_geometry(n, d)
        assert g.shape[0] == 1 << d
        assert g[:, 1].sum() == n
        assert (g[:, 3] >= g[:, 4]).all()
        assert np.array_equal(np.cumsum(g[:, 1])[:-1], g[1:, 4])
        for s, size, left, ds, _ in g:
            reg = size + size // 2
            assert s <= ds and ds + size <= s + reg
            assert ds == (s if left else s + reg - size)
        assert g[:, 0].max() + 1 <= n + n // 2
    g = orc.frog_geometry(n, 1)
    if n >= 2:
        (s0, n0, l0, d0, _), (s1, n1, l1, d1, _) = g
        assert l0 == 1 and l1 == 0 and n0 == (n + 1) // 2 and n1 == n // 2
        assert d1 == n                                   # inner run right after the output
        assert d1 - (d0 + n0) == n // 2                 # the gap holds the inner child


# --------------------------------------------------------------------------
# Frogsort2 model: the special case, the definition, the buffer check
# --------------------------------------------------------------------------
F2_QS = [1024, 3277, 6553, 13107, 16384, 21845, 29491, 32767, 32768]


@pytest.mark.parametrize("n", list(range(1, 40)) + [100, 255, 1000, 1023])
def test_frog2_half_is_frogsort1(orc, n):
    """The paper notes that Frogsort1 is Frogsort2 with p = 0.5: with q = 32768
    and one-element leaves the Frogsort2 model places, compares and moves
    exactly as the Frogsort1 model, merge for merge."""
    rng = np.random.default_rng(7000 + n)
    x = rng.integers(0, max(2, n // 4), size=n).astype(np.float64)
    a = orc.frog2_model(x, 32768, 1, max_snap=2 * n + 2)
    b = orc.frog_model(x, g=1, max_snap=2 * n + 2)
    assert a["bad"] == 0 and a["nslots"] == b["nslots"] == n + n // 2
    assert np.array_equal(a["setup"], b["setup"])
    assert np.array_equal(a["trace"], b["trace"])
    assert (a["compares"], a["moves"]) == (b["compares"], b["moves"])
    assert np.array_equal(a["labels"], b["labels"])


@pytest.mark.parametrize("q", F2_QS)
@pytest.mark.parametrize("leaf_max", [1, 2, 7, 64])
def test_frog2_sorts_stably_within_its_buffer(orc, q, leaf_max):
    """For every fraction the model reaches the definition (stable ascending,
    checked against numpy's stable argsort) with n + floor(q n / 65536) slots
    and never writes over an element that has not been read."""
    rng = np.random.default_rng(q * 131 + leaf_max)
    if q * (leaf_max + 1) < 65536:
        # a node just above the leaf size would get an empty inner child
        r = orc.frog2_model(rng.random(leaf_max + 1), q, leaf_max)
        assert r["bad"] & 2
        return
    for n in [1, leaf_max, leaf_max + 1, 97, 300, 1000, 2049]:
        x = rng.integers(0, max(2, n // 5), size=n).astype(np.float64)
        x[rng.random(n) < 0.1] = -0.0
        x[rng.random(n) < 0.05] = np.nan
        r = orc.frog2_model(x, q, leaf_max)
        assert r["bad"] == 0, (q, leaf_max, n)
        assert r["nslots"] == n + (q * n) // 65536 <= n + n * q / 65536
        p = _stable_order(x)
        assert np.array_equal(r["labels"], p)
        assert np.array_equal(r["keys"].view(np.uint64), x[p].view(np.uint64))


def _stable_order(x):
    """Stable ascending order with NaN last (numpy's argsort puts NaN last and
    is stable with kind='stable'); -0.0 and +0.0 tie."""
    return np.argsort(x, kind="stable")


@pytest.mark.parametrize("q", [3277, 6553, 16384, 32767])
def test_frog2_check_fires_on_a_short_buffer(orc, q):
    """The model's buffer check is live: one slot fewer per region makes some
    write land on an element that has not been read."""
    rng = np.random.default_rng(q)
    x = rng.random(2000)
    assert orc.frog2_model(x, q, 32)["bad"] == 0
    assert orc.frog2_model(x, q, 32, gap_shrink=1)["bad"] & 1


def _children(q, s, n, left):
    ni = (q * n) // 65536
    nl = n - ni if left else ni
    nr = n - nl
    reg = n + ni
    return (s, nl, 1), (s + reg - (nr + (q * nr) // 65536), nr, 0)


@pytest.mark.parametrize("q", F2_QS)
@pytest.mark.parametrize("n", [5000, 65537, 1 << 20])
def test_frog2_geometry_rules(orc, q, n):
    """The inner child holds floor(q n / 65536) elements and the outer child
    the rest; children fit their parent's region side by side; leaves cover
    the input in order, none larger than the leaf size, each starting at or
    after its input offset; a node's height is one more than its higher
    child's."""
    leaf_max = 512
    g = orc.frog2_geometry(n, q, leaf_max)
    lv, nd = g["leaves"], g["nodes"]
    assert g["bad"] == 0
    assert lv[:, 2].sum() == n and (lv[:, 2] <= leaf_max).all() and (lv[:, 2] >= 1).all()
    assert np.array_equal(np.concatenate([[0], np.cumsum(lv[:, 2])[:-1]]), lv[:, 0])
    assert (lv[:, 1] >= lv[:, 0]).all()
    assert lv[:, 1].max() + lv[lv[:, 1].argmax(), 2] <= g["nslots"]
    height = {(int(s), int(m), int(l)): int(h) for s, m, l, h in nd}
    assert height[(0, n, 1)] == nd[:, 3].max()
    for (s, m, l), h in height.items():
        assert m > leaf_max
        c0, c1 = _children(q, s, m, l)
        h0 = height.get(c0, 0 if c0[1] <= leaf_max else None)
        h1 = height.get(c1, 0 if c1[1] <= leaf_max else None)
        assert h0 is not None and h1 is not None
        assert h == 1 + max(h0, h1)
        reg0 = c0[1] + (q * c0[1]) // 65536
        assert c0[0] + reg0 <= c1[0]                       # side by side
    assert len(height) == nd.shape[0] == lv.shape[0] - 1   # a binary tree


@pytest.mark.parametrize("q", [3277, 6553, 13107, 32768])
def test_frog2_presorted_and_reversed_counts(orc, q):
    """Presorted input: a merge compares and moves only its inner run
    ("Symmetric merging"), so both counts are the sum of the inner children.
    Strictly descending input: every merge moves its whole output."""
    n = 3000
    inner = lambda nd: int(sum((q * m) // 65536 for m in nd[:, 1]))
    leaf = 65536 // q                     # the smallest leaf size that always splits
    r = orc.frog2_model(np.arange(n, dtype=np.float64), q, leaf)
    assert r["compares"] == r["moves"] == inner(r["nodes"])
    r = orc.frog2_model(np.arange(n, 0, -1, dtype=np.float64), q, leaf)
    assert r["moves"] == int(r["nodes"][:, 1].sum())
    assert np.array_equal(r["keys"], np.arange(1, n + 1, dtype=np.float64))


# --------------------------------------------------------------------------
# Frogsort3 model: one buffer shared by the branches in turn
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 3, 10, 33, 100, 257, 1000])
def test_frog3_with_enough_buffer_is_frogsort1(orc, n):
    """With a buffer of at least half the data the top node switches to
    Frogsort1 at once: the same result, compares and moves as the Frogsort1
    special case of the Frogsort2 model."""
    rng = np.random.default_rng(8000 + n)
    x = rng.integers(0, max(2, n // 4), size=n).astype(np.float64)
    a = orc.frog3_model(x, 32768, 4)
    b = orc.frog2_model(x, 32768, 4)
    assert a["bad"] == 0 and a["spine"].shape[0] == 0 and a["trees"].shape[0] == 1
    assert a["nslots"] == b["nslots"] == n + n // 2
    assert (a["compares"], a["moves"]) == (b["compares"], b["moves"])
    assert np.array_equal(a["labels"], b["labels"])


@pytest.mark.parametrize("q", F2_QS)
@pytest.mark.parametrize("leaf_max", [1, 5, 64])
def test_frog3_sorts_stably_within_its_buffer(orc, q, leaf_max):
    """Every fraction reaches the definition in place with n + min(b, n/2)
    slots, b = floor(q n / 65536), and no write lands on an unread element."""
    rng = np.random.default_rng(q * 7 + leaf_max)
    for n in [2, 3, 64, 65, 300, 1000, 2049, 5000]:
        b = (q * n) // 65536
        x = rng.integers(0, max(2, n // 5), size=n).astype(np.float64)
        x[rng.random(n) < 0.1] = -0.0
        x[rng.random(n) < 0.05] = np.nan
        r = orc.frog3_model(x, q, leaf_max)
        if b < 1 and n // 2 > b and n > leaf_max:
            assert r["bad"] & 2
            continue
        assert r["bad"] == 0, (q, leaf_max, n)
        assert r["nslots"] == n + min(b, n // 2)
        p = _stable_order(x)
        assert np.array_equal(r["labels"], p)
        assert np.array_equal(r["keys"].view(np.uint64), x[p].view(np.uint64))


@pytest.mark.parametrize("q", [1024, 6553, 16384])
def test_frog3_check_fires_on_a_short_gap(orc, q):
    rng = np.random.default_rng(q)
    x = rng.random(3000)
    assert orc.frog3_model(x, q, 16)["bad"] == 0
    assert orc.frog3_model(x, q, 16, gap_shrink=1)["bad"] & 1


@pytest.mark.parametrize("q", [1024, 3277, 6553, 13107, 21845, 32767])
@pytest.mark.parametrize("n", [5000, 1 << 16, (1 << 20) + 3])
def test_frog3_schedule_rules(orc, q, n):
    """The spine takes b = floor(q n / 65536) elements at a time off the end
    of the input until the buffer covers half of what is left; each piece is
    one Frogsort1 tree, a right node whose region ends b slots past its input;
    the rest is one Frogsort1 tree at slot 0; the spine merges run bottom up."""
    b = (q * n) // 65536
    g = orc.frog3_geometry(n, q, 512)
    assert g["bad"] == 0
    sizes = []
    m = n
    while m // 2 > b and m > 512:
        sizes.append(m)
        m -= b
    K = len(sizes)
    assert g["spine"].shape[0] == K and g["trees"].shape[0] == K + 1
    for k, mk in enumerate(sizes):
        s, size, c, left = g["trees"][k]
        assert (size, c, left) == (b, mk - b, 0)
        assert s + b + b // 2 == mk + b                   # the region ends at mk + b
    assert tuple(g["trees"][K]) == (0, m, 0, 1)
    for k, (nl, r0, nr) in enumerate(g["spine"]):
        mk = sizes[K - 1 - k]
        assert (nl, r0, nr) == (mk - b, mk, b)
    assert g["nslots"] == n + (b if K else n // 2)


@pytest.mark.parametrize("q", [3277, 6553, 32767])
def test_frog3_presorted_counts(orc, q):
    """Presorted input: every merge, in the Frogsort1 trees and on the spine,
    compares and moves only its inner run."""
    n = 3000
    r = orc.frog3_model(np.arange(n, dtype=np.float64), q, 8)
    inner = int(sum(m // 2 for m in r["nodes"][:, 1])) + int(r["spine"][:, 2].sum())
    assert r["compares"] == r["moves"] == inner


@pytest.mark.parametrize("q2", [6553, 16384, 21845])
@pytest.mark.parametrize("n", [100, 1000, 4097])
def test_frog6_with_enough_buffer_is_frogsort2(orc, q2, n):
    """Frogsort1, 2 and 3 are instances of Frogsort6 ("Frogsort3 and 6"): when the shared
    buffer already covers the whole tree's Frogsort2 buffer (p3 >= p2), the
    sort is one Frogsort2 tree at p2, merge for merge."""
    rng = np.random.default_rng(q2 + n)
    x = rng.integers(0, max(2, n // 4), size=n).astype(np.float64)
    leaf = 65536 // q2 + 1
    a = orc.frog3_model(x, q2, leaf, q2=q2)
    b = orc.frog2_model(x, q2, leaf)
    assert a["bad"] == 0 and a["spine"].shape[0] == 0 and a["trees"].shape[0] == 1
    assert a["nslots"] == b["nslots"] == n + (q2 * n) // 65536
    assert (a["compares"], a["moves"]) == (b["compares"], b["moves"])
    assert np.array_equal(a["labels"], b["labels"])


@pytest.mark.parametrize("q", [1024, 3277, 6553, 13107])
@pytest.mark.parametrize("q2", [6553, 16384, 32767])
def test_frog6_sorts_stably_within_its_buffer(orc, q, q2):
    """Frogsort6 (shared buffer b = floor(q n / 65536), Frogsort2 sub-trees
    at q2) reaches the definition with no write on an unread element, in at
    most n + b slots; the spine runs while a sub-tree would need more than b."""
    rng = np.random.default_rng(q * 3 + q2)
    leaf = 65536 // min(q, q2) + 1
    for n in [leaf + 1, 300, 1000, 4097, 20000]:
        b = (q * n) // 65536
        x = rng.integers(0, max(2, n // 5), size=n).astype(np.float64)
        x[rng.random(n) < 0.1] = -0.0
        r = orc.frog3_model(x, q, leaf, q2=q2)
        assert r["bad"] == 0, (q, q2, n)
        assert r["nslots"] <= n + b
        p = _stable_order(x)
        assert np.array_equal(r["labels"], p)
        m, K = n, 0
        while m > leaf and (q2 * m) // 65536 > b:
            m -= b
            K += 1
        assert r["spine"].shape[0] == K
        if K and b >= 2:       # one slot short: the first spine write lands on the inner run
            assert orc.frog3_model(x, q, leaf, q2=q2, gap_shrink=1)["bad"] & 1


# --------------------------------------------------------------------------
# network reference: forward closed forms, finite differences, Adam
# --------------------------------------------------------------------------
def test_mlp_forward_closed_form(orc):
    sl = orc.mlp_slices()
    p = np.zeros(orc.MLP_NUM_PARAMS)
    # y = w3[i] * relu(W2[i, j] * relu(W1[j] * u + b1[j]) + b2[i]) + b3
    i, j = 5, 17
    p[sl["W1"]][j] = 1.5
    p[sl["b1"]][j] = 0.25
    p[sl["W2"]][i * 64 + j] = -2.0          # row i (output unit), column j (input unit)
    p[sl["b2"]][i] = 3.0
    p[sl["w3"]][i] = 0.5
    p[sl["b3"]][0] = -0.125
    u = np.array([-1.0, -0.1, 0.0, 0.3, 1.0, 2.0])
    h1 = np.maximum(1.5 * u + 0.25, 0.0)
    h2 = np.maximum(-2.0 * h1 + 3.0, 0.0)
    assert np.allclose(orc.mlp_forward(p, u), 0.5 * h2 - 0.125, rtol=0, atol=1e-15)
    # the transposed index must not contribute
    p2 = p.copy()
    p2[sl["W2"]][i * 64 + j] = 0.0
    p2[sl["W2"]][j * 64 + i] = -2.0
    assert np.allclose(orc.mlp_forward(p2, u), 0.5 * 3.0 - 0.125)


def _rand_params(orc, seed):
    rng = np.random.default_rng(seed)
    sl = orc.mlp_slices()
    p = np.zeros(orc.MLP_NUM_PARAMS)
    p[sl["W1"]] = rng.normal(0, math.sqrt(2.0), 64)
    p[sl["b1"]] = rng.normal(0, 0.1, 64)
    p[sl["W2"]] = rng.normal(0, math.sqrt(2.0 / 64), 64 * 64)
    p[sl["b2"]] = rng.normal(0, 0.1, 64)
    p[sl["w3"]] = rng.normal(0, math.sqrt(2.0 / 64), 64)
    p[sl["b3"]] = rng.normal(0, 0.1, 1)
    return p


def test_mlp_loss_matches_forward(orc):
    p = _rand_params(orc, 1)
    rng = np.random.default_rng(2)
    u, t = rng.random(100), rng.random(100)
    loss, _ = orc.mlp_loss_grad(p, u, t)
    assert math.isclose(loss, float(np.mean((orc.mlp_forward(p, u) - t) ** 2)), rel_tol=1e-13)


def test_mlp_gradient_finite_differences(orc):
    p = _rand_params(orc, 3)
    rng = np.random.default_rng(4)
    u, t = rng.random(64), rng.random(64)
    _, g = orc.mlp_loss_grad(p, u, t)
    h = 1e-6
    # every first-layer, second-layer bias, output parameter and a sample of W2
    sl = orc.mlp_slices()
    idx = list(range(0, 128)) + list(range(sl["b2"].start, orc.MLP_NUM_PARAMS))
    idx += list(rng.choice(np.arange(sl["W2"].start, sl["W2"].stop), 400, replace=False))
    for k in idx:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (orc.mlp_loss_grad(pp, u, t, want_grad=False)[0]
              - orc.mlp_loss_grad(pm, u, t, want_grad=False)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])


def test_adam_first_step_closed_form(orc):
    """After one step from m = v = 0 the bias-corrected update is
    lr * g / (|g| + eps) for every parameter."""
    rng = np.random.default_rng(5)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    m, v = np.zeros(50), np.zeros(50)
    p0 = p.copy()
    orc.adam_step(p, g, m, v, 1, lr=1e-2)
    assert np.allclose(p, p0 - 1e-2 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
    # second step with the same gradient: m and v keep their EMA closed forms
    orc.adam_step(p, g, m, v, 2, lr=1e-2)
    assert np.allclose(m, (0.9 * 0.1 + 0.1) * g)
    assert np.allclose(v, (0.999 * 0.001 + 0.001) * g * g)


# --------------------------------------------------------------------------
# the four stable targets ("Definition of sorting")
# --------------------------------------------------------------------------
TARGETS = ("AscLeft", "AscRight", "DescLeft", "DescRight")


def _target_by_brute_force(keys, target):
    """The unique permutation meeting the target, by trying every permutation:
    keys in ascending (Asc) or descending (Desc) order, tied keys in input
    order (Left) or reverse input order (Right)."""
    desc, right = target.startswith("Desc"), target.endswith("Right")
    n = len(keys)
    found = []
    for perm in itertools.permutations(range(n)):
        ok = True
        for a, b in zip(perm, perm[1:]):
            ka, kb = keys[a], keys[b]
            wrong_keys = (kb > ka) if desc else (kb < ka)
            wrong_ties = ka == kb and ((b > a) if right else (b < a))
            if wrong_keys or wrong_ties:
                ok = False
                break
        if ok:
            found.append(perm)
    assert len(found) == 1
    return np.array(found[0], dtype=np.int64)


@pytest.mark.parametrize("target", TARGETS)
@pytest.mark.parametrize("n", [0, 1, 2, 3, 5, 6])
def test_targets_brute_force(orc, target, n):
    rng = np.random.default_rng(300 + n)
    for trial in range(25 if n > 3 else 8):
        keys = rng.integers(0, max(1, n // 2 + 1), size=n).astype(np.uint64)
        k, v = orc.sort_kv_target(keys, np.arange(n, dtype=np.uint32), target)
        perm = _target_by_brute_force(keys.tolist(), target)
        assert np.array_equal(v.astype(np.int64), perm)
        assert np.array_equal(k, keys[perm])


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_targets_exhaustive_weak_orders(orc, n):
    """Every weak order of n keys, as ±0-labelled doubles: the f64 targets
    keep or reverse the input order of ties exactly as the kv payload shows."""
    for w in itertools.product(range(n), repeat=n):
        if set(w) != set(range(max(w) + 1)):
            continue
        keys = np.array(w, dtype=np.uint64)
        for target in TARGETS:
            k, v = orc.sort_kv_target(keys, np.arange(n, dtype=np.uint32), target)
            desc, right = target.startswith("Desc"), target.endswith("Right")
            ks = k.astype(np.int64)
            d = np.diff(ks)
            assert np.all(d <= 0) if desc else np.all(d >= 0)
            tie = d == 0
            dv = np.diff(v.astype(np.int64))[tie]
            assert np.all(dv < 0) if right else np.all(dv > 0)


@pytest.mark.parametrize("pattern", ["uniform", "tied", "zeros_signed"])
def test_targets_match_lexsort(orc, pattern):
    """numpy's lexsort on (index, key) implements each target for NaN-free
    keys (it compares -0.0 and 0.0 as equal, as the targets do)."""
    x = W.f64_pattern(pattern, 3001, seed=8)
    idx = np.arange(x.size)
    for target in TARGETS:
        desc, right = target.startswith("Desc"), target.endswith("Right")
        order = np.lexsort((-idx if right else idx, -x if desc else x))
        got = orc.sort_f64_target(x, target)
        assert np.array_equal(got.view(np.uint64), x[order].view(np.uint64)), target


def test_target_identities(orc):
    """AscLeft is the plain stable sort; the right-anchored targets are the
    left-anchored ones of the opposite direction read backwards."""
    x = W.f64_pattern("zeros_signed", 5000, seed=9)
    x[::97] = np.nan
    b = lambda a: a.view(np.uint64)
    asc_l = orc.sort_f64_target(x, "AscLeft")
    assert np.array_equal(b(asc_l), b(orc.sort_f64(x)))
    assert np.array_equal(b(orc.sort_f64_target(x, "DescRight")), b(asc_l[::-1]))
    assert np.array_equal(b(orc.sort_f64_target(x, "AscRight")),
                          b(orc.sort_f64_target(x, "DescLeft")[::-1]))
    d = orc.sort_f64_target(x, "DescLeft")
    assert np.isnan(d[: np.isnan(x).sum()]).all()             # NaN is the largest key


# ---------------------------------------------------------------------------
# Squidsort1 model ("Squidsort", "Full adaptivity", Octosort's lazy order)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("k", range(1, 15))
def test_squid_presorted_and_reversed_counts(orc, k):
    """"Squidsort": no merge comparisons and 50 % of the moves on presorted and
    on reverse-sorted input.  For n = 2^k the moves are (n/2) log2 n, the
    inner runs of every node; reversed input adds one final reversal of n."""
    n = 1 << k
    for x, top, rev in ((np.arange(1, n + 1, dtype=np.float64), orc.SQUID_ASC, 0),
                        (np.arange(n, 0, -1, dtype=np.float64), orc.SQUID_DESC, n)):
        y, lab, c = orc.squid_model(x)
        assert c["merge_cmp"] == 0
        assert c["moves"] == (n // 2) * k
        assert c["rev_moves"] == rev
        assert c["top_dir"] == (top if n > 1 else orc.SQUID_NONE)
        assert c["overwrites"] == 0
        assert c["test_cmp"] <= 2 * (n - 1)
        assert np.array_equal(y, np.arange(1, n + 1, dtype=np.float64))


@pytest.mark.parametrize("n", [3, 5, 7, 100, 1000, 1023, 4097, 12345])
def test_squid_moves_equal_frogsort_presorted(orc, n):
    """For any n the moves on presorted input are the inner runs of every
    node, which the Frogsort1 model also moves on presorted input (pinned by
    its own closed form above); reversed input moves the same plus the final
    reversal."""
    x = np.arange(n, dtype=np.float64)
    frog = orc.frog_model(x, g=1)
    _, _, c = orc.squid_model(x)
    assert c["merge_cmp"] == 0 and c["moves"] == frog["moves"]
    _, _, c = orc.squid_model(x[::-1].copy())
    assert c["merge_cmp"] == 0 and c["moves"] == frog["moves"]
    assert c["rev_moves"] == n - (n & 1)


@pytest.mark.parametrize("mode", [0, 2])
@pytest.mark.parametrize("n", range(0, 8))
def test_squid_exhaustive_weak_orders(orc, n, mode):
    """Every weak order of n keys (tie class 0 as signed zeros, so stability
    is visible in the bits): the model's output is the definition's, element
    by element, and no write lands on an unread element -- for the reading
    above (mode 0) and for the rule the GPU runs (mode 2)."""
    arrs = _weak_orders(n)
    for row in arrs:
        x = row.astype(np.float64)
        x[(x == 0) & ((np.arange(n) & 1) == 1)] = -0.0
        y, lab, c = orc.squid_model(x, mode=mode)
        p = np.argsort(row, kind="stable")
        assert np.array_equal(lab, p), row
        assert np.array_equal(y.view(np.uint64), x[p].view(np.uint64))
        assert c["overwrites"] == 0


def _runs(rng, n, max_run, tie_values):
    """Ascending and descending runs of random lengths (strict, non-strict and
    tied), concatenated."""
    out = []
    while sum(map(len, out)) < n:
        m = int(rng.integers(1, max_run + 1))
        kind = rng.integers(0, 4)
        if kind == 0:
            r = np.sort(rng.integers(0, tie_values, m))
        elif kind == 1:
            r = np.sort(rng.integers(0, tie_values, m))[::-1]
        elif kind == 2:
            r = np.sort(rng.permutation(10 * n)[:m])[::-1]       # strictly descending
        else:
            r = rng.integers(0, tie_values, m)
        out.append(r.astype(np.float64))
    return np.concatenate(out)[:n]


@pytest.mark.parametrize("mode", [0, 2])
@pytest.mark.parametrize("seed", range(12))
def test_squid_sorts_mixed_runs_stably(orc, seed, mode):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 5000))
    x = _runs(rng, n, int(rng.integers(2, 300)), int(rng.integers(2, 50)))
    x[(x == 0) & (rng.random(n) < 0.5)] = -0.0
    y, lab, c = orc.squid_model(x, mode=mode)
    p = np.argsort(x, kind="stable")
    assert np.array_equal(lab, p)
    assert np.array_equal(y.view(np.uint64), x[p].view(np.uint64))
    assert c["overwrites"] == 0
    frog = orc.frog_model(x, g=1)
    assert c["moves"] <= frog["moves"] + x.size


@pytest.mark.parametrize("k", range(1, 13))
def test_squid_turning_rule_counts(orc, k):
    """The GPU's rule (mode 2) on presorted and reversed input is the
    model's: no merge, 50 % moves, one final reversal for reversed input.  On
    descending runs of 2^j that the tree then has to merge, it moves at most
    what Frogsort1 moves (each turn costs half of the node it precedes, and
    the concatenations below it saved half of every node)."""
    n = 1 << k
    for x, rev in ((np.arange(1, n + 1, dtype=np.float64), 0), (np.arange(n, 0, -1, dtype=np.float64), n)):
        _, _, c = orc.squid_model(x, mode=2)
        assert c["merge_cmp"] == 0 and c["moves"] == (n // 2) * k and c["rev_moves"] == (rev if n > 1 else 0)
    rng = np.random.default_rng(k)
    for j in range(1, k):
        runs = np.arange(n, dtype=np.float64).reshape(-1, 1 << j)[:, ::-1]      # descending runs
        x = runs[rng.permutation(runs.shape[0])].reshape(-1).copy()
        _, lab, c = orc.squid_model(x, mode=2)
        assert np.array_equal(lab, np.argsort(x, kind="stable"))
        assert c["moves"] <= orc.frog_model(x, g=1)["moves"] + n


@pytest.mark.parametrize("pattern", ["asclocal", "ascglobal", "desclocal", "descglobal",
                                     "permut", "tielog2"])
def test_squid_on_paper_patterns(orc, pattern):
    """The paper's patterns: the model sorts them and, where runs are
    presorted, needs fewer merge comparisons than Frogsort1."""
    import workloads as W
    n = 1 << 12
    x = W.paper_pattern(pattern, n, seed=2)
    y, lab, c = orc.squid_model(x)
    assert np.array_equal(lab, np.argsort(x, kind="stable"))
    assert c["overwrites"] == 0
    frog = orc.frog_model(x, g=1)
    if pattern in ("asclocal", "desclocal", "ascglobal"):
        assert c["merge_cmp"] < frog["compares"]


def test_squid_literal_reading_overwrites(orc):
    """Planted on the CPU: enforcing ascending at a merge whose outer run is
    descending (the literal reading of Octosort's rule) overwrites outer
    elements before they are read; the model's reading (merge in the outer
    run's direction) never does."""
    x = np.concatenate([np.arange(64, 0, -1), np.arange(100, 164), np.arange(300, 236, -1)]).astype(np.float64)
    x = np.concatenate([x, np.arange(500, 692).astype(np.float64)])
    _, lab, c1 = orc.squid_model(x, mode=1)
    assert c1["overwrites"] > 0
    _, lab, c0 = orc.squid_model(x, mode=0)
    assert c0["overwrites"] == 0
    assert np.array_equal(lab, np.argsort(x, kind="stable"))


def test_paper_patterns_shapes():
    """The generators make what the paper's patterns describe: distinct
    values (tielog2: ceil(log2 n) of them), runs of L = sqrt(n) ascending
    (asclocal) or descending (desclocal) spread over the whole range,
    quantile runs in ascending (ascglobal) or descending (descglobal)
    order."""
    import workloads as W
    n, L = 1 << 14, 1 << 7
    for p in W.PAPER_PATTERNS:
        x = W.paper_pattern(p, n, seed=5)
        assert np.unique(x).size == (14 if p == "tielog2" else n), p
    r = W.paper_pattern("asclocal", n, seed=5).reshape(-1, L)
    assert (np.diff(r, axis=1) > 0).all() and (r[:, 0] < n / 2).all() and (r[:, -1] > n / 2).all()
    r = W.paper_pattern("desclocal", n, seed=5).reshape(-1, L)
    assert (np.diff(r, axis=1) < 0).all()
    r = W.paper_pattern("ascglobal", n, seed=5).reshape(-1, L)
    assert (r.max(axis=1)[:-1] < r.min(axis=1)[1:]).all() and not (np.diff(r, axis=1) > 0).all()
    r = W.paper_pattern("descglobal", n, seed=5).reshape(-1, L)
    assert (r.min(axis=1)[:-1] > r.max(axis=1)[1:]).all()
