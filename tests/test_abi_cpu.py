"""Host-side checks of libgs.so that need no GPU: it loads, exports every
symbol include/gs.h declares, validates arguments before touching the device,
reports GS_ENODEVICE without a device, and its planner reproduces the oracle's
frog geometry."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2402_01816_amd as g

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "gs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(gs_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_exports_every_declared_symbol():
    names = _declared_symbols()
    assert "gs_sort_f64" in names and "gs_learned_sort" in names
    lib = ctypes.CDLL(g.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_strings():
    assert "gfx950" in g.version()
    for s in range(6):
        assert g.lib.gs_status_string(s).decode() == g.STATUS_NAMES[s]


def test_workspace_sizes():
    assert g.gs_workspace_bytes_f64(0) == 0 and g.gs_workspace_bytes_f64(1) == 0
    for n in [2, 3, 1000, 4097, 1 << 20, 1 << 28]:
        b = g.gs_workspace_bytes_f64(n)
        assert b >= 8 * (n // 2)
        # the control area on top of the half buffer: at most 34 bytes per
        # 1024 keys (16 of them the run samples, one key per 512 ranks) plus
        # a fixed part
        assert b <= 8 * (n // 2) + 4096 + 34 * n // 1024 + 64 * 1024
    n = 1 << 28
    assert 1.5 < 1 + g.gs_workspace_bytes_f64(n) / (8 * n) < 1.5042
    assert g.gs_workspace_bytes_kv(n) >= 12 * (n // 2)
    assert g.gs_workspace_bytes_f64(-1) == g.SIZE_MAX


@pytest.mark.parametrize("field,value,ok", [("mode", 2, True), ("mode", 3, False), ("num_buckets", 3, False),
                                             ("num_buckets", 8192, False), ("knots", 1, False),
                                             ("batch", 48, False), ("screen", 2, False)])
def test_learned_params_checked(field, value, ok):
    """Learned-path parameters are validated on the host: an invalid set has no
    workspace size (SIZE_MAX) and the call returns GS_EINVAL before any device
    work; mode 2 (the sample's CDF as the knot table) is valid."""
    p = g.gs_learned_default_params()
    setattr(p, field, value)
    n = 1 << 20
    b = g.gs_workspace_bytes_learned(n, p)
    if ok:
        assert 8 * (n // 2) <= b < g.SIZE_MAX
    else:
        assert b == g.SIZE_MAX
        fake = ctypes.c_void_p(0x100000)
        assert g.lib.gs_learned_sort(fake, n, ctypes.byref(p), fake, 1 << 30, None, None) == g.GS_EINVAL


def test_learned_buffer_fraction():
    """The learned call's buffer fraction: 0 and >= 0.5 keep the learned
    path's half buffer; [1/64, 0.5) sizes the plain sort's workspace at that
    fraction; below 1/64 is unsupported, negative or NaN invalid."""
    n = 1 << 22
    p = g.gs_learned_default_params()
    assert p.buffer_fraction == 0.5
    half = g.gs_workspace_bytes_learned(n, p)
    p.buffer_fraction = 0.0
    assert g.gs_workspace_bytes_learned(n, p) == half
    p.buffer_fraction = 0.9
    assert g.gs_workspace_bytes_learned(n, p) == half
    for f in (0.25, 0.1, 1 / 64):
        p.buffer_fraction = f
        assert g.gs_workspace_bytes_learned(n, p) == g.gs_workspace_bytes_f64(n, f)
    fake = ctypes.c_void_p(0x100000)
    for f, st in ((1 / 64 - 1e-9, g.GS_EUNSUPPORTED), (-0.5, g.GS_EINVAL), (float("nan"), g.GS_EINVAL)):
        p.buffer_fraction = f
        assert g.gs_workspace_bytes_learned(n, p) == g.SIZE_MAX
        assert g.lib.gs_learned_sort(fake, n, ctypes.byref(p), fake, 1 << 30, None, None) == st
    p.buffer_fraction = 0.25
    need = g.gs_workspace_bytes_learned(n, p)
    assert g.lib.gs_learned_sort(fake, n, ctypes.byref(p), fake, need - 1, None, None) == g.GS_EWORKSPACE


def _call_f64(keys, n, frac, ws, wsb):
    return g.lib.gs_sort_f64(keys, n, frac, ws, wsb, None, None)


def test_argument_errors_before_device():
    fake = ctypes.c_void_p(0x100000)
    need = g.gs_workspace_bytes_f64(1000)
    assert _call_f64(fake, -1, 0.5, fake, need) == g.GS_EINVAL
    assert _call_f64(None, 10, 0.5, fake, need) == g.GS_EINVAL
    assert _call_f64(fake, 1000, 0.0, fake, need) == g.GS_EINVAL
    assert _call_f64(fake, 1000, float("nan"), fake, need) == g.GS_EINVAL
    assert _call_f64(fake, 1000, 0.01, fake, need) == g.GS_EUNSUPPORTED      # below 1/64
    assert g.gs_workspace_bytes_f64(1000, 0.01) == g.SIZE_MAX
    assert _call_f64(fake, 1000, 0.5, fake, need - 1) == g.GS_EWORKSPACE
    assert _call_f64(fake, 1000, 0.5, None, need) == g.GS_EWORKSPACE
    assert _call_f64(fake, 1000, 0.5, ctypes.c_void_p(0x100010), need) == g.GS_EINVAL
    assert "aligned" in g.lib.gs_last_error_detail().decode()
    assert g.lib.gs_sort_kv(fake, None, 10, 0.5, fake, 1 << 20, None, None) == g.GS_EINVAL
    # the streaming copy: argument errors before any device work
    assert g.lib.gs_copy_f64(fake, fake, -1, None) == g.GS_EINVAL
    assert g.lib.gs_copy_f64(None, fake, 10, None) == g.GS_EINVAL
    assert g.lib.gs_copy_f64(fake, None, 10, None) == g.GS_EINVAL
    assert g.lib.gs_copy_f64(None, None, 0, None) == g.GS_OK
    # n <= 1 is a no-op that needs no workspace and no device
    assert _call_f64(None, 0, 0.5, None, 0) == g.GS_OK
    assert _call_f64(fake, 1, 0.5, None, 0) == g.GS_OK


def test_no_device_reported():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is visible")
    except ImportError:
        pass
    fake = ctypes.c_void_p(0x100000)
    need = g.gs_workspace_bytes_f64(1000)
    assert _call_f64(fake, 1000, 0.5, fake, need) == g.GS_ENODEVICE


@pytest.mark.parametrize("n", [2, 3, 5, 100, 4096, 4097, 12345, 1 << 20, (1 << 20) + 7,
                               (1 << 28) + 3])
def test_planner_matches_oracle_geometry(orc, n):
    depth, leaf = g.plan_depth(n)
    assert -(-n // (1 << depth)) <= leaf
    assert depth == 0 or -(-n // (1 << (depth - 1))) > leaf
    for d in range(min(depth, 12) + 1):
        geo = orc.frog_geometry(n, d)
        step = max(1, geo.shape[0] // 200)
        for i in range(0, geo.shape[0], step):
            assert tuple(int(v) for v in geo[i]) == g.plan_node(n, d, i)


def test_segsort_argument_errors():
    fake = ctypes.c_void_p(0x100000)
    need = g.gs_workspace_bytes_seg(1000, 10)
    assert need >= 8 * 500 and need != g.SIZE_MAX
    f = g.lib.gs_segsort
    assert f(fake, 1000, None, 10, 0.5, fake, need, None, None) == g.GS_EINVAL
    assert f(fake, 1000, fake, -1, 0.5, fake, need, None, None) == g.GS_EINVAL
    assert f(fake, -5, fake, 10, 0.5, fake, need, None, None) == g.GS_EINVAL
    assert f(fake, 1000, fake, 10, 0.01, fake, need, None, None) == g.GS_EUNSUPPORTED
    need3 = g.gs_workspace_bytes_seg(1000, 10, 0.3)
    assert need3 != g.SIZE_MAX
    assert f(fake, 1000, fake, 10, 0.3, fake, need3 - 1, None, None) == g.GS_EWORKSPACE
    assert f(fake, 1000, fake, 10, 0.3, fake, need3, None, None) == g.GS_ENODEVICE
    assert f(fake, 1000, fake, 10, 0.5, fake, need - 1, None, None) == g.GS_EWORKSPACE
    assert f(None, 0, None, 0, 0.5, None, 0, None, None) == g.GS_OK
    assert g.gs_workspace_bytes_seg(10, 0) == 0
    assert g.gs_workspace_bytes_seg(-1, 3) == g.SIZE_MAX


def _forest_counts(n, leaf, tile, rnd):
    """Exact work items of one problem of n keys in a round of the forest
    sort (round 0: leaves; round r: merge tiles and splits at depth D - r)."""
    D = 0
    while -(-n // (1 << D)) > leaf:
        D += 1
    if rnd == 0:
        return 1 << D, 0
    if rnd > D:
        return 0, 0
    d = D - rnd
    nodes = 1 << d
    tpn = -(-(-(-n // nodes)) // tile)
    return nodes * tpn, nodes * (tpn + 1)


@pytest.mark.parametrize("seed", range(6))
def test_forest_capacity_bounds(seed):
    """The workspace capacities of the forest sort (tickets, splits, leaves per
    round) bound the exact counts for random sets of problems of every size."""
    leaf, tile = 8192, 4096
    rng = np.random.default_rng(seed)
    lo = [4097, 2, 8193, 4097, 2, 100000][seed]
    hi = [9000, 70000, 1 << 20, 1 << 17, 5000, 1 << 22][seed]
    lens = np.exp(rng.uniform(np.log(lo), np.log(hi), rng.integers(1, 3000))).astype(np.int64)
    K, P = int(lens.sum()), lens.size
    cap_t = K // tile + K // leaf + 64
    cap_s = K // tile + 2 * (K // leaf) + 64
    cap_leaves = max(cap_t, 2 * (K // leaf) + P + 64)
    for rnd in range(0, 20):
        t = s = 0
        for n in lens:
            a, b = _forest_counts(int(n), leaf, tile, rnd)
            t += a
            s += b
        assert t <= (cap_leaves if rnd == 0 else cap_t)
        assert s <= cap_s


def test_segsort_shapes_and_errors():
    shapes = g.gs_seg_configs()
    assert len(shapes) == g.lib.gs_seg_config_count() >= 2
    assert shapes[0] == {"short_threads": 256, "short_ipt": 16, "merge_ipt": 16}
    c = g.GsSegConfig()
    assert g.lib.gs_seg_config_get(len(shapes), ctypes.byref(c)) == g.GS_EINVAL
    assert g.lib.gs_seg_config_get(-1, ctypes.byref(c)) == g.GS_EINVAL
    top = g.gs_workspace_bytes_seg(1 << 24, 5000)
    for s in shapes:
        cs = g._seg_config(s)
        b = g.lib.gs_workspace_bytes_seg_ex(1 << 24, 5000, 0.5, ctypes.byref(cs))
        assert 8 * (1 << 23) <= b <= top
    bad = g.GsSegConfig(300, 16, 16, 0)
    assert g.lib.gs_workspace_bytes_seg_ex(1 << 20, 10, 0.5, ctypes.byref(bad)) == g.SIZE_MAX
    fake = ctypes.c_void_p(0x100000)
    need = g.gs_workspace_bytes_seg(1000, 10)
    assert g.lib.gs_segsort_ex(fake, 1000, fake, 10, 0.5, ctypes.byref(bad), fake, need, None,
                               None) == g.GS_EINVAL
    reserved = g.GsSegConfig(256, 16, 16, 1)
    assert g.lib.gs_segsort_ex(fake, 1000, fake, 10, 0.5, ctypes.byref(reserved), fake, need, None,
                               None) == g.GS_EINVAL
    best = g.GsSegConfig()
    assert g.lib.gs_segsort_autotune(fake, 1000, fake, 10, None, fake, need, None, 1,
                                     ctypes.byref(best), None) == g.GS_EINVAL
    assert g.lib.gs_segsort_autotune(fake, 1000, fake, 10, fake, fake, need, None, 0,
                                     ctypes.byref(best), None) == g.GS_EINVAL


def test_target_argument_errors():
    fake = ctypes.c_void_p(0x100000)
    need = g.gs_workspace_bytes_f64(1000)
    for bad in (-1, 4, 99):
        assert g.lib.gs_sort_f64_target(fake, 1000, bad, 0.5, fake, need, None, None) == g.GS_EINVAL
        assert g.lib.gs_sort_kv_target(fake, fake, 1000, bad, 0.5, fake, 1 << 20, None, None) == g.GS_EINVAL
    assert g.lib.gs_sort_f64_target(None, 0, 2, 0.5, None, 0, None, None) == g.GS_OK


FRACTIONS = [1 / 64, 0.05, 0.1, 0.2, 0.25, 1 / 3, 0.45, 0.4999]


@pytest.mark.parametrize("kv", [False, True])
@pytest.mark.parametrize("p", FRACTIONS)
def test_frog2_plan_matches_oracle(orc, kv, p):
    """The library's Frogsort2 planner walks the same tree as the oracle's
    model: the same leaves (input offset, data start, length) in input order,
    the same merge nodes, each merged in the round of its height, and a buffer
    of floor(q n / 65536) elements."""
    _, leaf = g.plan_depth(1 << 20, kv=kv)
    q = orc.frog2_fraction_q(p)
    for n in [2, leaf, leaf + 1, 3 * leaf + 7, 1000003, (1 << 22) + 12345]:
        lv, nd, counts = g.plan_frog2(n, p, kv)
        r = orc.frog2_geometry(n, q, leaf)
        assert np.array_equal(lv, r["leaves"]), n
        mine = sorted(map(tuple, nd.tolist()))
        theirs = sorted(map(tuple, r["nodes"].tolist()))
        assert mine == theirs, n
        assert counts[2] == (r["nodes"][:, 3].max() if r["nodes"].size else 0)
        assert counts[3] == (q * n) // 65536 == r["nslots"] - n


@pytest.mark.parametrize("p", FRACTIONS)
def test_small_buffer_workspace(p):
    """%RAM follows the fraction for both small-buffer trees: the buffer is at
    most floor(q n / 65536) elements (never above p n) and the control area
    and tree tables stay a small fraction of the data; the default below 0.5
    is Frogsort3."""
    import oracle
    q = oracle.frog2_fraction_q(p)
    for n in [5000, 1 << 20, (1 << 24) + 5]:
        h = (q * n) // 65536
        assert h <= p * n
        for algo in ("frogsort2", "frogsort3"):
            b = g.gs_workspace_bytes_f64(n, p, algo)
            assert 8 * min(h, n // 2) <= b <= 8 * h + 0.02 * 8 * n + (1 << 20)
            bk = g.gs_workspace_bytes_kv(n, p, algo)
            assert 12 * min(h, n // 2) <= bk <= 12 * h + 0.02 * 12 * n + (1 << 20)
    assert g.gs_workspace_bytes_f64(1 << 24, p) == g.gs_workspace_bytes_f64(1 << 24, p, "frogsort3")
    if p <= 0.45:
        for algo in ("frogsort2", "frogsort3"):
            assert g.gs_workspace_bytes_f64(1 << 24, p, algo) < g.gs_workspace_bytes_f64(1 << 24, 0.5)


def test_frog2_fraction_bounds():
    assert g.gs_workspace_bytes_f64(1 << 20, 1 / 64) != g.SIZE_MAX
    assert g.gs_workspace_bytes_f64(1 << 20, 1 / 64 - 1e-9) == g.SIZE_MAX
    assert g.gs_workspace_bytes_f64(1 << 20, 0.5) == g.gs_workspace_bytes_f64(1 << 20, 0.9)
    fake = ctypes.c_void_p(0x100000)
    need = g.gs_workspace_bytes_seg(1000, 10)
    assert g.lib.gs_segsort(fake, 1000, fake, 10, 1 / 64 - 1e-9, fake, need, None, None) == g.GS_EUNSUPPORTED
    assert g.gs_workspace_bytes_seg(1 << 20, 10, 1 / 64 - 1e-9) == g.SIZE_MAX
    assert g.gs_workspace_bytes_seg(1 << 20, 10, 1 / 64) != g.SIZE_MAX


def _default_tile():
    c = g.GsSegConfig()
    g.lib.gs_seg_default_config(ctypes.byref(c))
    return c.short_threads * c.short_ipt


def _seg_offsets(rng, n_target, tile, giant=False):
    """Segment lengths mixing empty, short (at most a tile), long and, with
    giant, one segment of 60 % of the keys."""
    lens = []
    while sum(lens) < n_target:
        u = rng.random()
        lens.append(0 if u < 0.05 else int(rng.integers(1, tile + 1)) if u < 0.6
                    else int(rng.integers(tile + 1, 6 * tile)))
    if giant:
        lens.insert(int(rng.integers(0, len(lens))), int(1.5 * sum(lens)))
    return np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("p", [1 / 64, 0.1, 0.25, 0.45])
def test_seg_small_buffer_steps(seed, p):
    """Below buffer fraction 0.5 the segmented sort's steps cover every
    segment once, in order; every pass's long segments have their half
    buffers, placed at (first key - the pass's first key) / 2, inside the
    buffer; a pass ends only at a long segment that would overflow it; a
    segment sorted alone is long and its own half buffer overflows it."""
    rng = np.random.default_rng(seed)
    tile = _default_tile()
    off = _seg_offsets(rng, 40 * tile, tile, giant=seed % 2 == 1)
    n = int(off[-1]) + int(rng.integers(0, 50))
    rows, hlen = g.plan_seg_steps(off, n, p)
    assert hlen == (int(p * 65536) * n) >> 16
    nseg = off.shape[0] - 1
    assert rows[0, 0] == 0 and rows[-1, 1] == nseg
    assert (rows[1:, 0] == rows[:-1, 1]).all() and (rows[:, 1] > rows[:, 0]).all()
    ln = np.diff(off)
    for s0, s1, alone in rows:
        if alone:
            assert s1 == s0 + 1 and ln[s0] > tile and ln[s0] // 2 > hlen
            continue
        for s in range(s0, s1):
            if ln[s] > tile:
                assert (off[s] - off[s0]) // 2 + ln[s] // 2 <= hlen
        if s1 < nseg:
            assert ln[s1] > tile and (off[s1] - off[s0]) // 2 + ln[s1] // 2 > hlen
    if seed % 2 == 1 and p < 0.3:
        assert rows[:, 2].any()
    bad = off.copy()
    bad[3] = bad[2] - 1
    with pytest.raises(ValueError):
        g.plan_seg_steps(bad, n, p)
    with pytest.raises(ValueError):
        g.plan_seg_steps(off, n, 0.5)


@pytest.mark.parametrize("p", [1 / 64, 0.1, 0.25, 0.45])
def test_seg_small_buffer_workspace(p):
    """The segmented workspace below 0.5 is the buffer plus control, smaller
    than the half buffer's, and covers the plain sort's workspace of any
    segment that may have to be sorted alone (any length up to the keys)."""
    n = 1 << 24
    ws = g.gs_workspace_bytes_seg(n, 5000, p)
    assert ws < g.gs_workspace_bytes_seg(n, 5000, 0.5)
    assert ws / (8 * n) < p + 0.01
    rng = np.random.default_rng(7)
    for N in [100003, 1 << 20, 3000017]:
        top = g.gs_workspace_bytes_seg(N, 9, p)
        lens = np.unique(np.concatenate([rng.integers(2, N + 1, 40), N - np.arange(40)]))
        assert max(g.gs_workspace_bytes_f64(int(L), p) for L in lens) <= top


@pytest.mark.parametrize("kv", [False, True])
@pytest.mark.parametrize("p", FRACTIONS)
@pytest.mark.parametrize("p2", [0.5, 0.2, 1 / 64])
def test_frog3_plan_matches_oracle(orc, kv, p, p2):
    """The library's Frogsort3 (p2 = 0.5) and Frogsort6 (Frogsort2 sub-trees
    at p2) schedules are the oracle model's: the same sub-trees (root, size,
    input offset, side) in running order, the same spine merges bottom up, the
    same leaves, and the same buffer."""
    _, leaf = g.plan_depth(1 << 20, kv=kv)
    q = orc.frog2_fraction_q(p)
    q2 = 32768 if p2 >= 0.5 else orc.frog2_fraction_q(p2)
    for n in [2, leaf, leaf + 1, 3 * leaf + 7, 1000003, (1 << 22) + 12345]:
        trees, spine, leaves, counts = g.plan_frog3(n, p, kv, sub_fraction=p2)
        r = orc.frog3_geometry(n, q, leaf, q2=q2)
        assert np.array_equal(trees, r["trees"]), n
        assert np.array_equal(spine, r["spine"]), n
        assert sorted(map(tuple, leaves.tolist())) == sorted(map(tuple, r["leaves"].tolist()))
        assert counts[4] == r["nslots"] - n
        assert counts[4] <= p * n


def test_algo_argument_errors():
    fake = ctypes.c_void_p(0x100000)
    need = g.gs_workspace_bytes_f64(1000, 0.5)
    f = g.lib.gs_sort_f64_ex
    assert f(fake, 1000, 0, 0.5, 7, 0.5, fake, need, None, None) == g.GS_EINVAL
    assert f(fake, 1000, 0, 0.25, 1, 0.5, fake, need, None, None) == g.GS_EINVAL     # Frogsort1 needs 0.5
    assert f(fake, 1000, 0, 0.01, 3, 0.5, fake, need, None, None) == g.GS_EUNSUPPORTED
    assert f(fake, 1000, 0, 0.1, 4, 0.01, fake, need, None, None) == g.GS_EUNSUPPORTED
    assert f(fake, 1000, 0, 0.1, 4, 0.0, fake, need, None, None) == g.GS_EINVAL
    assert f(fake, 1000, 0, 0.1, 4, float("nan"), fake, need, None, None) == g.GS_EINVAL
    assert g.gs_workspace_bytes_f64(1000, 0.25, "frogsort1") == g.SIZE_MAX
    assert g.gs_workspace_bytes_f64(1 << 20, 0.9, "frogsort3") == g.gs_workspace_bytes_f64(1 << 20, 0.5, "frogsort3")
    # Frogsort6 at sub-fraction 0.5 is Frogsort3; at or below the fraction, one Frogsort2 tree
    n = (1 << 22) + 5
    assert g.gs_workspace_bytes_f64(n, 0.1, "frogsort6", 0.5) == g.gs_workspace_bytes_f64(n, 0.1, "frogsort3")
    assert g.plan_frog3(n, 0.25, sub_fraction=0.2)[3][1] == 0


def test_device_error_query_without_device():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is visible")
    except ImportError:
        pass
    flags = ctypes.c_uint32(7)
    assert g.lib.gs_device_errors(0, ctypes.byref(flags), 0) == g.GS_ENODEVICE
    assert flags.value == 0
    assert g.lib.gs_device_errors(0, None, 0) == g.GS_EINVAL


def test_fail_waits_hook_toggles():
    was = g.gs_test_fail_waits(True)
    try:
        assert g.gs_test_fail_waits(True) is True
    finally:
        g.gs_test_fail_waits(was)
    assert g.gs_test_fail_waits(was) is was


def test_noalloc_limits():
    """The static workspace of gs_sort_f64_noalloc holds the workspace of
    every size up to its limit; above it, and on bad arguments, the call
    fails before touching a device."""
    src = open(os.path.join(ROOT, "include", "gs.h")).read()
    max_keys = int(re.search(r"#define GS_NOALLOC_MAX_KEYS \(\(int64_t\)1 << (\d+)\)", src).group(1))
    scratch = int(re.search(r"#define GS_NOALLOC_SCRATCH_BYTES \(\(int64_t\)(\d+) << 20\)", src).group(1)) << 20
    assert 1 << max_keys == g.NOALLOC_MAX_KEYS
    rng = np.random.default_rng(5)
    sizes = {2, 3, 4097, 8192, 8193, (1 << max_keys) - 1, 1 << max_keys}
    sizes |= {int(v) for v in rng.integers(2, (1 << max_keys) + 1, 300)}
    sizes |= {(1 << k) + d for k in range(1, max_keys) for d in (-1, 0, 1)}
    for n in sorted(sizes):
        if 2 <= n <= 1 << max_keys:
            assert g.gs_workspace_bytes_f64(n) <= scratch, n
    fake = ctypes.c_void_p(0x100000)
    assert g.lib.gs_sort_f64_noalloc(fake, (1 << max_keys) + 1, None) == g.GS_EINVAL
    assert "limit" in g.lib.gs_last_error_detail().decode()
    assert g.lib.gs_sort_f64_noalloc(fake, -1, None) == g.GS_EINVAL
    assert g.lib.gs_sort_f64_noalloc(None, 10, None) == g.GS_EINVAL
    assert g.lib.gs_sort_f64_noalloc(None, 0, None) == g.GS_OK
    assert g.lib.gs_sort_f64_noalloc(fake, 1, None) == g.GS_OK


# ---------------------------------------------------------------------------
# the in-place protocol's windows against brute force ("Symmetric merging")
# ---------------------------------------------------------------------------
ASC, DESC = 1, 2
MERGE, MERGE_REV, CONCAT = 0, 1, 2


def _merge_case(rng, outer, kind, tile):
    """A random merge of the frog kinds: the outer run inside the output
    (outer 0: first run at its start, written top-down; 1: second run at its
    end, bottom-up; 2: first run at its end, bottom-up), the inner run
    outside; random sizes (ragged against the tile), ties, and run
    directions fitting the node kind."""
    nl, nr = (int(v) for v in rng.integers(1, 5 * tile, 2))
    n = nl + nr
    out0 = int(rng.integers(0, 3 * tile))
    gap = int(rng.integers(0, tile))
    if outer == 0:
        l0, r0 = out0, out0 + n + gap
    elif outer == 1:
        if rng.random() < 0.5:              # inner run just before the output (a right node)
            out0 += nl + gap
            l0 = out0 - nl - gap
        else:                               # inner run past the output (an explicit merge)
            l0 = out0 + n + gap
        r0 = out0 + nl
    else:
        l0 = out0 + nr
        r0 = out0 + n + gap
    left = 1 if outer == 0 else 0
    vals = int(rng.choice([3, 50, 10 ** 6]))
    sl = np.sort(rng.integers(0, vals, nl))
    sr = np.sort(rng.integers(0, vals, nr))
    outer_first = outer != 1
    if kind == CONCAT:
        dl = dr = ASC if rng.random() < 0.5 else DESC
        if dl == ASC:
            sr = sr + sl[-1]                        # ties across the seam allowed
        else:
            sl = sl + sr[-1] + 1                    # strictly above
    else:
        d_outer = DESC if kind == MERGE_REV else ASC
        d_inner = ASC if rng.random() < 0.5 else DESC
        dl, dr = (d_outer, d_inner) if outer_first else (d_inner, d_outer)
    return dict(merge=np.array([l0, nl, r0, nr, out0, left, outer], dtype=np.int64),
                sl=sl, sr=sr, dl=dl, dr=dr, n=n, outer_first=outer_first)


def _brute_windows(c, kind, tile):
    """Tickets each tile must wait for, from the slots every tile reads and
    writes (the outer run already turned for MERGE_REV), and the splits."""
    l0, nl, r0, nr, out0, left, outer = (int(v) for v in c["merge"])
    n = c["n"]
    # storage direction of each run when the tiles run
    st_l = c["dl"] == DESC and not (kind == MERGE_REV and c["outer_first"])
    st_r = c["dr"] == DESC and not (kind == MERGE_REV and not c["outer_first"])
    slot_l = (lambda i: l0 + nl - 1 - i) if st_l else (lambda i: l0 + i)
    slot_r = (lambda i: r0 + nr - 1 - i) if st_r else (lambda i: r0 + i)
    if kind == CONCAT:
        # stored orders side by side
        src = [l0 + i for i in range(nl)] + [r0 + i for i in range(nr)]
        from_a = [True] * nl + [False] * nr
    else:
        i = j = 0
        src, from_a = [], []
        sl, sr = c["sl"], c["sr"]
        while i < nl or j < nr:
            if j >= nr or (i < nl and not sr[j] < sl[i]):
                src.append(slot_l(i)); from_a.append(True); i += 1
            else:
                src.append(slot_r(j)); from_a.append(False); j += 1
    tpn = -(-n // tile)
    splits = np.array([sum(from_a[: min(k * tile, n)]) for k in range(tpn + 1)], dtype=np.int64)
    ticket = (lambda jj: tpn - 1 - jj) if left else (lambda jj: jj)
    reads = [set(src[jj * tile: min((jj + 1) * tile, n)]) for jj in range(tpn)]
    windows = {}
    for jj in range(tpn):
        writes = set(range(out0 + jj * tile, out0 + min((jj + 1) * tile, n)))
        windows[ticket(jj)] = sorted(ticket(k) for k in range(tpn) if reads[k] & writes)
    return splits, windows, tpn


@pytest.mark.parametrize("outer", [0, 1, 2])
@pytest.mark.parametrize("kind", [MERGE, MERGE_REV, CONCAT])
@pytest.mark.parametrize("seed", range(20))
def test_tile_windows_match_brute_force(outer, kind, seed):
    """Every merge tile's window, as the kernels compute it, is the smallest
    ticket range holding every ticket whose inputs include a slot the tile
    writes, and never passes the tile's own ticket: the outer run only moves away
    from the side the output is written from.  Both frog node kinds, the
    third kind of the explicit merges, concatenations, inner runs read from
    their end and outer runs turned around first, with ties."""
    rng = np.random.default_rng(100 * seed + 10 * outer + kind)
    tile = int(rng.choice([4, 7, 16]))
    c = _merge_case(rng, outer, kind, tile)
    splits, want, tpn = _brute_windows(c, kind, tile)
    got = np.zeros(2 * tpn, dtype=np.int64)
    r = g.lib.gs_plan_tile_windows(c["merge"].ctypes.data, kind, c["dl"], c["dr"], 1, tile,
                                   splits.ctypes.data, got.ctypes.data)
    assert r == tpn
    for t in range(tpn):
        w = want[t]
        assert not w or w[-1] <= t, (t, w)                        # never a later ticket
        # the window is the smallest ticket range holding that set (a tile
        # in between that reads none of those slots may be waited for too)
        lo, hi = int(got[2 * t]), int(got[2 * t + 1])
        assert ((lo, hi) == (w[0], w[-1])) if w else lo > hi, (t, lo, hi, w)


@pytest.mark.parametrize("n", [8193, 12345, 65536, (1 << 20) + 7, 3_000_017])
def test_leaf_windows_match_brute_force(n):
    """Every leaf's window is exactly the set of leaf tickets whose input
    chunks its destination covers, never past its own ticket."""
    depth, _ = g.plan_depth(n)
    L = 1 << depth
    nodes = [g.plan_node(n, depth, i) for i in range(L)]        # (s, n, left, data start, input offset)
    chunk_lo = np.array([nd[4] for nd in nodes])
    lo_hi = np.zeros(2, dtype=np.int64)
    for i, nd in enumerate(nodes):
        dst, ln = nd[3], nd[1]
        cover = set()
        if dst < n:
            for p in (dst, min(dst + ln, n) - 1):
                cover.add(int(np.searchsorted(chunk_lo, p, side="right") - 1))
            cover = set(range(min(cover), max(cover) + 1))
        want = sorted(L - 1 - k for k in cover)
        assert g.lib.gs_plan_leaf_window(n, depth, i, lo_hi.ctypes.data) == 0
        lo, hi = int(lo_hi[0]), int(lo_hi[1])
        assert (list(range(lo, hi + 1)) if lo <= hi else []) == want
        assert not want or want[-1] <= L - 1 - i


def test_tile_windows_check_sees_a_wrong_layout():
    """The brute-force check above is not blind: windows computed as if a
    turned outer run were still stored descending disagree with it."""
    bad = 0
    for seed in range(20):
        for outer in (0, 1, 2):
            rng = np.random.default_rng(100 * seed + 10 * outer + MERGE_REV)
            tile = int(rng.choice([4, 7, 16]))
            c = _merge_case(rng, outer, MERGE_REV, tile)
            splits, want, tpn = _brute_windows(c, MERGE_REV, tile)
            got = np.zeros(2 * tpn, dtype=np.int64)
            g.lib.gs_plan_tile_windows(c["merge"].ctypes.data, MERGE_REV, c["dl"], c["dr"], 0, tile,
                                       splits.ctypes.data, got.ctypes.data)
            for t in range(tpn):
                w = want[t]
                lo, hi = int(got[2 * t]), int(got[2 * t + 1])
                bad += (((lo, hi) != (w[0], w[-1])) if w else lo <= hi)
    assert bad > 0


def test_tune_cache_roundtrip(tmp_path):
    """The tuning cache keys shapes by architecture and size class
    (floor(log2) of keys and segments), rejects shapes that are not the
    tuner's, and survives a save / clear / load round trip; a file's invalid
    entries are skipped."""
    g.lib.gs_tune_cache_clear()
    shapes = g.gs_seg_configs()
    g.gs_tune_cache_put("gfx950", 1 << 20, 5000, shapes[3])
    assert g.gs_tune_cache_get((1 << 21) - 1, 4096, arch="gfx950") == shapes[3]   # same class
    assert g.gs_tune_cache_get(1 << 21, 5000, arch="gfx950") is None               # next class
    assert g.gs_tune_cache_get(1 << 20, 5000, arch="gfx942") is None
    bad = g.GsSegConfig(); bad.short_threads, bad.short_ipt, bad.merge_ipt = 512, 16, 12
    assert g.lib.gs_tune_cache_put(b"gfx950", 1 << 20, 5000, ctypes.byref(bad)) == g.GS_EINVAL
    path = str(tmp_path / "tune.json")
    assert g.lib.gs_tune_cache_save(path.encode()) == 1
    g.lib.gs_tune_cache_clear()
    assert g.gs_tune_cache_get(1 << 20, 5000, arch="gfx950") is None
    assert g.lib.gs_tune_cache_load(path.encode()) == 1
    assert g.gs_tune_cache_get(1 << 20, 5000, arch="gfx950") == shapes[3]
    with open(path, "w") as f:
        f.write('{"entries": [{"arch": "gfx950", "log2_keys": 10, "log2_segments": 2, "short_threads": 512, '
                '"short_ipt": 16, "merge_ipt": 12}, {"arch": "gfx950", "log2_keys": 11, "log2_segments": 2, '
                '"short_threads": %d, "short_ipt": %d, "merge_ipt": %d}]}'
                % (shapes[1]["short_threads"], shapes[1]["short_ipt"], shapes[1]["merge_ipt"]))
    assert g.lib.gs_tune_cache_load(path.encode()) == 1
    assert g.gs_tune_cache_get(1 << 11, 4, arch="gfx950") == shapes[1]
    assert g.gs_tune_cache_get(1 << 10, 4, arch="gfx950") is None
    assert g.lib.gs_tune_cache_load(str(tmp_path / "missing.json").encode()) == -1
    g.lib.gs_tune_cache_clear()


def test_tune_cache_read_from_environment(tmp_path):
    """GS_TUNE_CACHE names a file read on the cache's first use."""
    import subprocess
    import sys
    shapes = g.gs_seg_configs()
    path = tmp_path / "tune.json"
    s = shapes[2]
    path.write_text('{"entries": [{"arch": "gfx950", "log2_keys": 24, "log2_segments": 12, "short_threads": %d, '
                    '"short_ipt": %d, "merge_ipt": %d}]}' % (s["short_threads"], s["short_ipt"], s["merge_ipt"]))
    code = ("import paper_2402_01816_amd as g; c = g.gs_tune_cache_get(1 << 24, 5000, arch='gfx950'); "
            "print(c['short_threads'], c['short_ipt'], c['merge_ipt'])")
    env = dict(os.environ, GS_TUNE_CACHE=str(path), PYTHONPATH=ROOT)
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split() == [str(s["short_threads"]), str(s["short_ipt"]), str(s["merge_ipt"])]
