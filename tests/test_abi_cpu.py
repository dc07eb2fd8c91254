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
        assert b <= 8 * (n // 2) + 4096 + n // 64 + 64 * 1024
    n = 1 << 28
    assert 1.5 < 1 + g.gs_workspace_bytes_f64(n) / (8 * n) < 1.502
    assert g.gs_workspace_bytes_kv(n) >= 12 * (n // 2)
    assert g.gs_workspace_bytes_f64(-1) == g.SIZE_MAX


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
    assert f(fake, 1000, fake, 10, 0.3, fake, need, None, None) == g.GS_EUNSUPPORTED
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
    assert g.lib.gs_segsort(fake, 1000, fake, 10, 0.25, fake, need, None, None) == g.GS_EUNSUPPORTED


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
