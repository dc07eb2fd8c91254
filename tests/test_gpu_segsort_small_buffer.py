"""Parity of gs_segsort below buffer fraction 0.5 (through the C ABI) with the
CPU oracle's segmented sort.

One buffer of floor(q n / 2^16) doubles serves runs of consecutive segments
in turn; a segment whose own half buffer does not fit is sorted alone by the
plain sort (Frogsort3).  The cases make several passes, segments sorted alone
(first, last and in between), presorted and reversed segments, empty and
short segments, ragged lengths and ±0 / NaN ties, at every fraction from the
smallest (1/64) up to just below one half.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import announce, bits, need_gpu, to_dev

pytestmark = pytest.mark.gpu

FRACTIONS = [1 / 64, 0.1, 0.25, 0.45]


@pytest.fixture(scope="module")
def gs():
    need_gpu()
    import paper_2402_01816_amd as g
    return g


def _offsets(lengths):
    off = np.zeros(len(lengths) + 1, dtype=np.int64)
    off[1:] = np.cumsum(lengths)
    return off


def _ties(x):
    x = x.copy()
    x[::97] = -0.0
    x[::89] = 0.0
    x[::1009] = np.nan
    return x


def _sort_check(gs, orc, x, off, p):
    t = to_dev(x)
    rep = gs.gs_segsort(t, to_dev(off), buffer_fraction=p, report=True)
    assert rep["invalid_offsets"] == 0
    n = x.size
    assert rep["workspace_bytes_used"] <= gs.gs_workspace_bytes_seg(n, off.size - 1, p)
    assert np.array_equal(bits(t), bits(orc.segsort_f64(x, off)))
    return rep


@pytest.mark.parametrize("p", FRACTIONS)
@pytest.mark.parametrize("seed", [0, 1])
def test_small_buffer_segsort_mix(gs, orc, p, seed):
    """Log-uniform lengths in [1, 40000]: many passes at the small fractions."""
    announce("segsort small buffer mix", p, seed)
    x, off = W.segmented(1500, 1, 40000, seed=40 + seed)
    rows, _ = gs.plan_seg_steps(off, x.size, p)
    assert rows.shape[0] >= 2 or p >= 0.45
    _sort_check(gs, orc, _ties(x), off, p)


@pytest.mark.parametrize("p", FRACTIONS)
@pytest.mark.parametrize("where", ["first", "middle", "last", "only"])
def test_small_buffer_segsort_alone(gs, orc, p, where):
    """A segment too long for the buffer's half, sorted alone by the plain
    sort, next to segments sorted in passes."""
    announce("segsort small buffer alone", p, where)
    rng = np.random.default_rng(10 * ["first", "middle", "last", "only"].index(where) + FRACTIONS.index(p))
    rest = [int(v) for v in rng.integers(0, 20000, 40)]
    big = 3 * sum(rest) + 12345 if where != "only" else 300001
    lengths = {"first": [big] + rest, "middle": rest[:20] + [big] + rest[20:],
               "last": rest + [big], "only": [big]}[where]
    off = _offsets(lengths)
    x = _ties(W.f64_pattern("uniform", int(off[-1]), seed=len(lengths)))
    rows, _ = gs.plan_seg_steps(off, x.size, p)
    if p < 0.3:
        assert rows[:, 2].any()
    _sort_check(gs, orc, x, off, p)


@pytest.mark.parametrize("p", [1 / 64, 0.25])
def test_small_buffer_segsort_ordered(gs, orc, p):
    """Presorted, reversed and tied segments take the order check in every
    pass; a reversed segment sorted alone takes the plain sort's."""
    announce("segsort small buffer ordered", p)
    rng = np.random.default_rng(9)
    parts = []
    for k, m in enumerate([5000, 260000, 9000, 30000, 70001, 17, 8193, 3]):
        v = rng.standard_normal(m)
        kind = k % 3
        if kind == 0:
            v = np.sort(v)
        elif kind == 1:
            v = np.sort(v)[::-1].copy()
        else:
            v = np.round(v * 3)
        parts.append(v)
    x = np.concatenate(parts)
    off = _offsets([v.size for v in parts])
    _sort_check(gs, orc, x, off, p)


def test_small_buffer_segsort_outside_untouched(gs, orc):
    announce("segsort small buffer outside")
    x = W.f64_pattern("uniform", 300000, seed=4)
    off = np.array([1000, 1000, 5000, 205001, 220000], dtype=np.int64)
    t = to_dev(x)
    gs.gs_segsort(t, to_dev(off), buffer_fraction=0.1)
    got = t.cpu().numpy()
    assert np.array_equal(bits(got[:1000]), bits(x[:1000]))
    assert np.array_equal(bits(got[220000:]), bits(x[220000:]))
    assert np.array_equal(bits(got), bits(orc.segsort_f64(x, off)))


@pytest.mark.parametrize("bad", [[0, 5, 3, 10], [-1, 4, 10], [0, 4, 10 + 1]])
def test_small_buffer_segsort_invalid_offsets(gs, bad):
    """Checked on the host before anything runs: GS_EINVAL with or without a
    report, keys unchanged."""
    announce("segsort small buffer invalid", bad)
    x = W.f64_pattern("uniform", 10, seed=5)
    t = to_dev(x)
    o = to_dev(np.array(bad, dtype=np.int64))
    for report in (True, False):
        with pytest.raises(gs.GsError) as e:
            gs.gs_segsort(t, o, buffer_fraction=0.25, report=report)
        assert e.value.status == gs.GS_EINVAL
    assert np.array_equal(bits(t), bits(x))


@pytest.mark.filterwarnings("ignore:The CUDA Graph is empty")   # nothing may be recorded
def test_small_buffer_segsort_rejects_capture(gs):
    """The call reads the offsets on the host, so it refuses to be recorded
    into a graph (and enqueues nothing)."""
    torch = need_gpu()
    x, off = W.segmented(500, 1, 20000, seed=3)
    t = to_dev(x)
    o = to_dev(off)
    need = gs.gs_workspace_bytes_seg(x.size, off.size - 1, 0.25)
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    a = (-ws.data_ptr()) % 256
    ws = ws[a: a + need]
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    err = None
    with torch.cuda.stream(s):
        g.capture_begin()
        try:
            gs.gs_segsort(t, o, buffer_fraction=0.25, workspace=ws, stream=s)
        except gs.GsError as e:
            err = e
        finally:
            g.capture_end()
    assert err is not None and err.status == gs.GS_EUNSUPPORTED


@pytest.mark.parametrize("p", [1 / 64])
def test_small_buffer_segsort_full_workload(gs, orc, p):
    """100,000 segments, log-uniform lengths rescaled to 2^28 keys (the
    segmented benchmark's input), every key compared with the oracle; the
    buffer and control stay within p + 1 % of the keys' bytes."""
    announce("segsort small buffer full", p)
    x, off = W.segmented(100_000, 16, 19023, seed=0, total=1 << 28)
    t = to_dev(x)
    rep = gs.gs_segsort(t, to_dev(off), buffer_fraction=p, report=True)
    assert rep["invalid_offsets"] == 0
    assert rep["ram_fraction"] < 1 + p + 0.01
    got = t.cpu().numpy()
    del t
    ref = orc.segsort_f64(x, off)
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
