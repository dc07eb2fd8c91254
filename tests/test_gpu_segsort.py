"""Parity of gs_segsort (through the C ABI) with the CPU oracle's segmented sort.

Lengths cover every size class of the device path (empty, single, short
batched blocks, exactly one tile, multi-leaf frog sorts), ragged tails, NaN and
signed-zero ties.  The full workload (100,000 segments, 2^28 keys, mixed
patterns) is compared element by element with the oracle.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import announce, bits, need_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    need_gpu()
    import paper_2402_01816_amd as g
    return g


def _run(gs, x, off, **kw):
    t = to_dev(x)
    o = to_dev(off.astype(np.int64))
    rep = gs.gs_segsort(t, o, **kw)
    return t, rep


def _check(orc, t, x, off):
    ref = orc.segsort_f64(x, off)
    assert np.array_equal(bits(t), bits(ref))


@pytest.mark.parametrize("lengths", [
    [0], [1], [2], [3, 0, 1, 2],
    [15, 16, 17, 31, 32, 33, 255, 256, 257],
    [4095, 4096, 4097],
    [8191, 8192, 8193, 12289],
    [20000, 1, 0, 5, 40000],
    [65537],
])
@pytest.mark.parametrize("pattern", ["uniform", "zeros_signed", "tied"])
def test_segsort_lengths(gs, orc, lengths, pattern):
    announce("segsort", pattern, lengths)
    n = int(sum(lengths))
    x = W.f64_pattern(pattern, n, seed=len(lengths) + n)
    off = np.zeros(len(lengths) + 1, dtype=np.int64)
    off[1:] = np.cumsum(lengths)
    t, _ = _run(gs, x, off)
    _check(orc, t, x, off)


@pytest.mark.parametrize("lengths", [
    [1 << 20, (1 << 20) - 1, 300001, 5, 0, 70000, 8193, 4097],
    [(1 << 22) + 3],
    [4097] * 300 + [9000] * 50 + [17] * 200,
])
def test_segsort_long_segments(gs, orc, lengths):
    """Segments above one LDS tile go through the forest sort: many frog
    trees of different depths merged level by level in shared launches."""
    announce("segsort long", len(lengths), max(lengths))
    n = int(sum(lengths))
    x = W.f64_pattern("zeros_signed", n, seed=n % 1000)
    off = np.zeros(len(lengths) + 1, dtype=np.int64)
    off[1:] = np.cumsum(lengths)
    t, _ = _run(gs, x, off)
    _check(orc, t, x, off)


def test_segsort_draw_until_total(gs, orc):
    """Lengths log-uniform in [16, 2^20] drawn until 2^24 keys, mixed
    patterns per segment."""
    announce("segsort until-total")
    x, off = W.segmented(None, 16, 1 << 20, seed=5, total=1 << 24)
    x = x.copy()
    x[::97] = -0.0
    x[::89] = 0.0
    t, _ = _run(gs, x, off)
    _check(orc, t, x, off)


@pytest.mark.parametrize("shape", range(10))
def test_segsort_every_shape(gs, orc, shape):
    """Every shape the tuner can pick gives the same (oracle) result on a mix
    of short and long segments, ±0 ties included."""
    cfg = gs.gs_seg_configs()[shape]
    announce("segsort shape", cfg)
    x, off = W.segmented(1500, 1, 40000, seed=20 + shape)
    x = x.copy()
    x[::7] = -0.0
    x[::11] = 0.0
    t, _ = _run(gs, x, off, config=cfg)
    _check(orc, t, x, off)


def test_segsort_autotune(gs, orc):
    """The tuner leaves the input untouched, times every shape and returns one
    of them; sorting with it matches the oracle."""
    announce("segsort autotune")
    x, off = W.segmented(3000, 16, 30000, seed=31)
    keys = to_dev(x)
    offs = to_dev(off)
    best, times = gs.gs_segsort_autotune(keys, offs, reps=1)
    assert np.array_equal(bits(keys), bits(x))
    assert best in gs.gs_seg_configs()
    assert len(times) == len(gs.gs_seg_configs()) and all(v > 0 for v in times.values())
    assert times[gs.gs_seg_configs().index(best)] == min(times.values())
    gs.gs_segsort(keys, offs, config=best)
    _check(orc, keys, x, off)
    # the tuned shape is kept for this architecture and size class, and a
    # call without a shape takes it
    assert gs.gs_tune_cache_get(x.size, off.size - 1) == best
    keys2 = to_dev(x)
    gs.gs_segsort(keys2, offs)
    _check(orc, keys2, x, off)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_segsort_random_mix(gs, orc, seed):
    announce("segsort mix", seed)
    x, off = W.segmented(3000, 1, 30000, seed=seed)
    x = x.copy()
    x[::101] = -0.0
    x[::103] = 0.0
    t, _ = _run(gs, x, off)
    _check(orc, t, x, off)


def test_segsort_special_values(gs, orc):
    announce("segsort special")
    rng = np.random.default_rng(3)
    pool = np.array([np.nan, np.inf, -np.inf, 0.0, -0.0, 5e-324, 1.0, -1.0])
    lens = rng.integers(0, 9000, 60)
    off = np.zeros(lens.size + 1, dtype=np.int64)
    off[1:] = np.cumsum(lens)
    x = pool[rng.integers(0, pool.size, int(off[-1]))]
    t, _ = _run(gs, x, off)
    _check(orc, t, x, off)


def test_segsort_leaves_outside_untouched(gs, orc):
    announce("segsort outside")
    x = W.f64_pattern("uniform", 30000, seed=4)
    off = np.array([1000, 1000, 5000, 5001, 22000], dtype=np.int64)
    t, rep = _run(gs, x, off, report=True)
    got = t.cpu().numpy()
    assert np.array_equal(bits(got[:1000]), bits(x[:1000]))
    assert np.array_equal(bits(got[22000:]), bits(x[22000:]))
    ref = orc.segsort_f64(x, off)
    assert np.array_equal(bits(got), bits(ref))
    assert rep["invalid_offsets"] == 0


@pytest.mark.parametrize("bad", [[0, 5, 3, 10], [-1, 4, 10], [0, 4, 10 + 1]])
def test_segsort_invalid_offsets_reported(gs, bad):
    announce("segsort invalid", bad)
    x = W.f64_pattern("uniform", 10, seed=5)
    t = to_dev(x)
    o = to_dev(np.array(bad, dtype=np.int64))
    with pytest.raises(gs.GsError) as e:
        gs.gs_segsort(t, o, report=True)
    assert e.value.status == gs.GS_EINVAL
    assert np.array_equal(bits(t), bits(x))


ORDER_LENGTHS = [2, 3, 17, 1000, 4097, 8193, 8194, 20000, 70001]


def _ordered_segment(kind, m, rng):
    u = np.sort(rng.random(m))
    if kind == "sorted":
        return u
    if kind == "reversed":
        return u[::-1].copy()
    if kind == "reversed_ties":                 # non-increasing, ties bit-identical
        return np.sort(rng.integers(0, 16, m).astype(np.float64))[::-1].copy()
    if kind == "reversed_signed_zero_ties":     # non-increasing, but +0 and -0 tie
        v = np.sort(rng.integers(-3, 4, m).astype(np.float64))[::-1].copy()
        z = np.flatnonzero(v == 0)
        v[z[::2]] = -0.0
        return v
    if kind == "reversed_nan_first":            # one NaN, then strictly decreasing
        v = u[::-1].copy()
        v[0] = np.nan
        return v
    if kind == "reversed_two_nans":             # NaN ties NaN: not strictly decreasing
        v = u[::-1].copy()
        v[: min(2, m)] = np.nan
        return v
    if kind == "almost_sorted":
        v = u.copy()
        v[m - 2], v[m - 1] = v[m - 1], v[m - 2]
        return v
    if kind == "almost_reversed":
        v = u[::-1].copy()
        v[m - 2], v[m - 1] = v[m - 1], v[m - 2]
        return v
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["sorted", "reversed", "reversed_ties", "reversed_signed_zero_ties",
                                  "reversed_nan_first", "reversed_two_nans", "almost_sorted", "almost_reversed"])
def test_segsort_ordered_segments(gs, orc, kind):
    """Segments already in order are left alone and reversed ones reversed
    (the order check's shortcut); near misses in the last pair, signed-zero
    ties and tied NaNs must still be sorted.  Lengths span the short classes
    and the forest, and 8193 / 8194 keys put the last pair at the end of the
    pairs a segment's wave checks (8192) and just past it, where the range
    pass takes over; a uniform segment sits between every two."""
    announce("segsort ordered", kind)
    rng = np.random.default_rng(11)
    parts, lens = [], []
    for m in ORDER_LENGTHS:
        parts += [_ordered_segment(kind, m, rng), rng.random(m // 2 + 1)]
        lens += [m, m // 2 + 1]
    x = np.concatenate(parts)
    off = np.zeros(len(lens) + 1, dtype=np.int64)
    off[1:] = np.cumsum(lens)
    t, rep = _run(gs, x, off, report=True)
    _check(orc, t, x, off)
    assert rep["invalid_offsets"] == 0


def test_segsort_many_empty_segments(gs, orc):
    """Runs of hundreds of thousands of empty segments around long presorted,
    reversed and unsorted ones (the range passes jump over each run)."""
    announce("segsort many empty")
    rng = np.random.default_rng(5)
    parts, lens = [], []
    for kind in ("reversed", "sorted", "uniform", "reversed"):
        lens += [0] * 200_000
        m = int(rng.integers(40_000, 90_000))
        u = np.sort(rng.random(m))
        parts.append(u[::-1].copy() if kind == "reversed" else u if kind == "sorted" else rng.random(m))
        lens.append(m)
    lens += [0] * 1000
    x = np.concatenate(parts)
    off = np.zeros(len(lens) + 1, dtype=np.int64)
    off[1:] = np.cumsum(lens)
    t, rep = _run(gs, x, off, report=True)
    _check(orc, t, x, off)
    assert rep["invalid_offsets"] == 0


def test_segsort_invalid_offsets_with_reversed_segments(gs):
    """Valid reversed segments around an invalid one: the call fails and
    nothing moves (the reversal waits for every segment's offsets)."""
    announce("segsort invalid reversed")
    x = np.arange(100, 0, -1, dtype=np.float64)
    t = to_dev(x)
    o = to_dev(np.array([0, 50, 40, 100], dtype=np.int64))
    with pytest.raises(gs.GsError) as e:
        gs.gs_segsort(t, o, report=True)
    assert e.value.status == gs.GS_EINVAL
    assert np.array_equal(bits(t), bits(x))


def _weak_orders(n):
    grid = np.indices((n,) * n).reshape(n, -1).T
    present = np.zeros((grid.shape[0], n), dtype=bool)
    np.put_along_axis(present, grid, True, axis=1)
    return grid[present.sum(axis=1) == grid.max(axis=1) + 1]


def test_segsort_exhaustive_weak_orders(gs, orc):
    """Every weak order of n <= 8 keys (598,445 arrays) as one segmented call;
    tie class 0 written as mixed-sign zeros so stability is visible."""
    announce("segsort exhaustive")
    xs, lens = [], []
    for n in range(0, 9):
        a = _weak_orders(n) if n else np.zeros((1, 0), dtype=np.int64)
        xs.append(a.reshape(-1).astype(np.float64))
        lens.extend([n] * a.shape[0])
    x = np.concatenate(xs)
    sign = (np.arange(x.size) * 2654435761 >> 3) & 1
    x[(x == 0) & (sign == 1)] = -0.0
    off = np.zeros(len(lens) + 1, dtype=np.int64)
    off[1:] = np.cumsum(lens)
    assert len(lens) == 1 + 1 + 3 + 13 + 75 + 541 + 4683 + 47293 + 545835
    t, _ = _run(gs, x, off)
    _check(orc, t, x, off)


def test_segsort_graph_capture_replay(gs, orc):
    """gs_segsort captured once into a HIP graph (torch's graph API) and
    replayed on fresh inputs copied into the captured buffer; every replay is
    checked against the oracle, with eager work between replays."""
    torch = need_gpu()
    announce("segsort graph")
    x0, off = W.segmented(2000, 1, 20000, seed=7)
    n = x0.size
    keys = to_dev(x0)
    offs = to_dev(off)
    need = gs.gs_workspace_bytes_seg(n, off.size - 1)
    ws_raw = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    o = (-ws_raw.data_ptr()) % 256
    ws = ws_raw[o:o + need]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):                      # warm-up outside capture
        gs.gs_segsort(keys, offs, workspace=ws, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        gs.gs_segsort(keys, offs, workspace=ws, stream=s)
    for seed in (11, 12, 13):
        x, off2 = W.segmented(2000, 1, 20000, seed=7)
        x = x + seed                                # same offsets, new keys
        keys.copy_(torch.from_numpy(x))
        _ = (keys * 2).sum()                        # unrelated eager work
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _check(orc, keys, x, off)


def test_segsort_full_workload(gs, orc):
    """100,000 segments, log-uniform lengths in [16, 19023] rescaled to total
    2^28 keys, patterns uniform/tied/presorted/reversed per segment."""
    announce("segsort full")
    x, off = W.segmented(100_000, 16, 19023, seed=0, total=1 << 28)
    t, rep = _run(gs, x, off, report=True)
    assert rep["invalid_offsets"] == 0
    got = t.cpu().numpy()
    del t
    ref = orc.segsort_f64(x, off)
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
