"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Small and medium sizes are compared element by element, bit for bit, with the
oracle's full result.  Sizes span one leaf, several leaves and merge tiles, and
ragged tails.  At the full benchmark size the oracle's counting form of the
definition fixes sampled output positions, and the rest is checked by
properties (sorted, same multiset).
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import announce, bits, multiset_hash_dev, need_gpu, to_dev

pytestmark = pytest.mark.gpu

SIZES = [0, 1, 2, 3, 17, 255, 4095, 4096, 4097, 8191, 8193, 12345, 65536, 100003,
         1 << 20, (1 << 20) + 7]
PATTERNS = ["uniform", "tied", "presorted", "reversed", "perturbed", "zeros_signed"]


@pytest.fixture(scope="module")
def gs():
    need_gpu()
    import paper_2402_01816_amd as g
    return g


@pytest.mark.parametrize("pattern", PATTERNS)
@pytest.mark.parametrize("n", SIZES)
def test_sort_f64_parity(gs, orc, pattern, n):
    announce("sort_f64", pattern, n)
    x = W.f64_pattern(pattern, n, seed=11)
    t = to_dev(x)
    gs.gs_sort_f64(t)
    ref = orc.sort_f64(x)
    assert np.array_equal(bits(t), bits(ref))


def test_sort_f64_special_values(gs, orc):
    announce("sort_f64 special")
    rng = np.random.default_rng(7)
    n = 50_000
    pool = np.array([np.nan, -np.nan, np.inf, -np.inf, 0.0, -0.0, 5e-324, -5e-324,
                     2.2250738585072014e-308, 1.0, -1.0, 1e308], dtype=np.float64)
    x = pool[rng.integers(0, pool.size, n)]
    x[::97] = np.frombuffer(np.uint64(0x7FF0000000000ABC).tobytes(), dtype=np.float64)[0]
    t = to_dev(x)
    gs.gs_sort_f64(t)
    assert np.array_equal(bits(t), bits(orc.sort_f64(x)))


def test_sort_f64_report_and_ram(gs):
    torch = need_gpu()
    n = 1 << 20
    t = to_dev(W.f64_pattern("uniform", n))
    rep = gs.gs_sort_f64(t, report=True)
    assert rep["levels"] == gs.plan_depth(n)[0]
    assert 1.5 <= rep["ram_fraction"] < 1.52
    assert rep["workspace_bytes_used"] == gs.gs_workspace_bytes_f64(n)
    assert rep["elapsed_ms"] > 0
    del torch


@pytest.mark.parametrize("pattern", ["uniform", "zipf", "few"])
@pytest.mark.parametrize("n", [0, 1, 2, 5, 2047, 2048, 2049, 4097, 10000, 65537, 1 << 20])
def test_sort_kv_parity(gs, orc, pattern, n):
    announce("sort_kv", pattern, n)
    k, v = W.kv_pattern(pattern, n, seed=5)
    tk = to_dev(k.view(np.int64))
    tv = to_dev(v.view(np.int32))
    gs.gs_sort_kv(tk, tv)
    rk, rv = orc.sort_kv(k, v)
    assert np.array_equal(tk.cpu().numpy().view(np.uint64), rk)
    assert np.array_equal(tv.cpu().numpy().view(np.uint32), rv)


def test_repeated_calls_share_workspace(gs, orc):
    torch = need_gpu()
    n = 300_001
    need = gs.gs_workspace_bytes_f64(n)
    ws = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    off = (-ws.data_ptr()) % 256
    wsv = ws[off:off + need]
    for seed in range(3):
        x = W.f64_pattern("zeros_signed", n, seed=seed)
        t = to_dev(x)
        gs.gs_sort_f64(t, workspace=wsv)
        assert np.array_equal(bits(t), bits(orc.sort_f64(x)))
    # a smaller sort afterwards on the same workspace
    x = W.f64_pattern("tied", 5000, seed=9)
    t = to_dev(x)
    gs.gs_sort_f64(t, workspace=wsv[: gs.gs_workspace_bytes_f64(5000)])
    assert np.array_equal(bits(t), bits(orc.sort_f64(x)))


@pytest.mark.parametrize("n", [1 << 24, (1 << 24) + 4097])
def test_sort_f64_many_tiles_visible_ties(gs, orc, n):
    """Element by element at sizes whose top merges hold thousands of tiles,
    more than the merge launch's resident work-groups, so every work-group
    takes several tiles in turn; ±0 ties and NaNs with different payloads
    make every tie order visible."""
    announce("sort_f64 many tiles ties", n)
    x = W.f64_pattern("zeros_signed", n, seed=n % 977)
    x[::509] = np.float64(np.nan)
    x[::1021] = -np.float64(np.nan)
    t = to_dev(x)
    gs.gs_sort_f64(t)
    assert np.array_equal(bits(t), bits(orc.sort_f64(x)))


FULL_N = 1 << 28


@pytest.mark.parametrize("pattern", W.PATTERNS)
def test_sort_f64_full_size_sampled(gs, orc, pattern):
    """n = 2^28: sampled positions from the oracle's counting definition, plus
    sortedness and multiset equality over the whole output."""
    torch = need_gpu()
    announce("sort_f64 full", pattern, FULL_N)
    x = W.f64_pattern(pattern, FULL_N, seed=0)
    t = to_dev(x)
    h_in = multiset_hash_dev(t)
    gs.gs_sort_f64(t)
    torch.cuda.synchronize()
    assert multiset_hash_dev(t) == h_in
    assert bool((t[1:] >= t[:-1]).all().item())
    rng = np.random.default_rng(1)
    idx = np.concatenate([[0, FULL_N - 1], rng.integers(0, FULL_N, 14)])
    ranks = orc.rank_f64(x, idx)
    got = t[torch.from_numpy(ranks).to("cuda")].cpu().numpy()
    assert np.array_equal(bits(got), bits(x[idx]))


KV_FULL_N = 1 << 29


@pytest.mark.parametrize("pattern", ["uniform", "zipf"])
def test_sort_kv_full_size(gs, orc, pattern):
    """n = 2^29 key/value pairs with payload = input index.  Every output pair
    is checked on the device: keys non-decreasing as unsigned integers, the
    payload a permutation of the input indices that carries each key with it,
    and equal keys in increasing payload order -- together exactly the
    stable definition.  Sampled positions also come from the oracle's
    counting form."""
    torch = need_gpu()
    n = KV_FULL_N
    announce("sort_kv full", pattern, n)
    k, v = W.kv_pattern(pattern, n, seed=0)
    tk_in = to_dev(k.view(np.int64))
    tk = tk_in.clone()
    tv = to_dev(v.view(np.int32))
    gs.gs_sort_kv(tk, tv)
    torch.cuda.synchronize()
    ks = tk ^ (-(1 << 63))               # unsigned order as signed order
    assert bool((ks[1:] >= ks[:-1]).all().item())
    del ks
    vi = tv.to(torch.int64)
    seen = torch.zeros(n, dtype=torch.bool, device="cuda")
    seen[vi] = True
    assert bool(seen.all().item())
    del seen
    assert torch.equal(tk_in[vi], tk)
    bad = (tk[1:] == tk[:-1]) & (vi[1:] <= vi[:-1])
    assert not bool(bad.any().item())
    del bad, tk_in
    rng = np.random.default_rng(2)
    idx = np.concatenate([[0, n - 1], rng.integers(0, n, 6)])
    ranks = orc.rank_u64(k, idx)
    got = tv[torch.from_numpy(ranks).to("cuda")].cpu().numpy().view(np.uint32)
    assert np.array_equal(got, v[idx])


TARGETS = ("AscLeft", "AscRight", "DescLeft", "DescRight")


@pytest.mark.parametrize("target", TARGETS)
@pytest.mark.parametrize("n", [2, 3, 4097, 12345, 1 << 20, (1 << 20) + 7])
def test_sort_f64_targets(gs, orc, target, n):
    """The four stable targets, bit for bit (±0 ties show the tie order;
    NaNs and infinities included)."""
    announce("sort_f64 target", target, n)
    x = W.f64_pattern("zeros_signed", n, seed=21 + n)
    x[::61] = np.nan
    x[::67] = -np.inf
    x[::71] = np.inf
    t = to_dev(x)
    gs.gs_sort_f64(t, target=target)
    assert np.array_equal(bits(t), bits(orc.sort_f64_target(x, target)))


@pytest.mark.parametrize("target", TARGETS)
@pytest.mark.parametrize("pattern", ["uniform", "tied"])
@pytest.mark.parametrize("n", [300, 4097, 100003, 1 << 20])
def test_sort_f64_targets_identical_ties(gs, orc, target, pattern, n):
    """The four targets on keys without NaN or zeros, where every tie is
    between bit-identical keys: the blocks take the register network and the
    merge rounds across lanes, ascending and descending."""
    announce("sort_f64 target identical ties", target, pattern, n)
    x = W.f64_pattern(pattern, n, seed=5 + n) + 1.0
    t = to_dev(x)
    gs.gs_sort_f64(t, target=target)
    assert np.array_equal(bits(t), bits(orc.sort_f64_target(x, target)))


@pytest.mark.parametrize("target", TARGETS)
@pytest.mark.parametrize("pattern", ["uniform", "few"])
def test_sort_kv_targets(gs, orc, target, pattern):
    """Key/value targets: payload = input index, so the tie order is visible
    for every tie."""
    torch = need_gpu()
    n = (1 << 20) + 13
    announce("sort_kv target", target, pattern)
    k0, v0 = W.kv_pattern(pattern, n, seed=5)
    K = to_dev(k0.view(np.int64))
    V = to_dev(v0.view(np.int32))
    gs.gs_sort_kv(K, V, target=target)
    rk, rv = orc.sort_kv_target(k0, v0, target)
    assert np.array_equal(K.cpu().numpy().view(np.uint64), rk)
    assert np.array_equal(V.cpu().numpy().view(np.uint32), rv)


# --------------------------------------------------------------------------
# input already in order or strictly reversed ("Octosort", "Squidsort")
# --------------------------------------------------------------------------
def _order_cases(n, seed):
    rng = np.random.default_rng(seed)
    base = np.sort(rng.random(n))
    ties = np.sort(rng.integers(0, 50, n).astype(np.float64))
    cases = {
        "in order": (base, 1),
        "in order, ties": (ties, 1),
        "in order, ±0 and NaN tail": (np.concatenate([[-1.0], [0.0, -0.0, 0.0, -0.0], np.full(3, 7.0),
                                                     np.full(max(n - 11, 0), np.inf), [np.nan, np.nan, np.nan]]), 1),
        "strictly reversed": (base[::-1].copy(), 2),
        "strictly reversed, NaN first": (np.concatenate([[np.nan], base[::-1]]), 2),
        "reversed with ties, zeros among them": (ties[::-1].copy(), 0),
        # equal keys bit for bit equal: the reversal is the stable result
        "reversed with ties, no zero or NaN": ((ties + 1.0)[::-1].copy(), 2),
        "two NaNs then reversed": (np.concatenate([[np.nan, np.nan], base[::-1]]), 0),
    }
    # one inversion between two sampled pairs (the sample sees pairs at
    # floor(j (n-1) / 4096)): only the full check finds it
    if n > 16:
        x = base.copy()
        k = 5 * (n - 1) // 4096 + 3
        x[k], x[k + 1] = x[k + 1], x[k]
        cases["one hidden inversion"] = (x, 0)
    return cases


@pytest.mark.parametrize("n", [3, 4097, 1_000_003])
def test_order_fast_paths(gs, orc, n):
    for name, (x, want) in _order_cases(n, seed=n).items():
        announce("order", name, x.size)
        t = to_dev(x)
        rep = gs.gs_sort_f64(t, report=True)
        assert np.array_equal(bits(t), bits(orc.sort_f64(x))), name
        if x.size > 3:
            assert rep["order"] == want, name


@pytest.mark.parametrize("target", TARGETS)
def test_order_fast_paths_targets(gs, orc, target):
    n = 200_003
    for name, (x, _) in _order_cases(n, seed=7).items():
        announce("order target", target, name)
        t = to_dev(x)
        gs.gs_sort_f64(t, target=target)
        assert np.array_equal(bits(t), bits(orc.sort_f64_target(x, target))), name


def test_order_fast_paths_kv(gs, orc):
    n = 300_001
    rng = np.random.default_rng(3)
    base = np.sort(rng.integers(0, 1 << 62, n, dtype=np.int64).astype(np.uint64))
    ties = np.sort(rng.integers(1, 9, n).astype(np.uint64))
    for name, k, want in (("in order", base, 1), ("strictly reversed", base[::-1].copy(), 2),
                          ("in order, ties", ties, 1),
                          # the payload shows the order of ties: no reversal shortcut
                          ("reversed with ties", ties[::-1].copy(), 0)):
        announce("order kv", name)
        v = np.arange(n, dtype=np.uint32)
        tk = to_dev(k.view(np.int64))
        tv = to_dev(v.view(np.int32))
        rep = gs.gs_sort_kv(tk, tv, report=True)
        rk, rv = orc.sort_kv(k, v)
        assert rep["order"] == want, name
        assert np.array_equal(tk.cpu().numpy().view(np.uint64), rk)
        assert np.array_equal(tv.cpu().numpy().view(np.uint32), rv)


@pytest.mark.parametrize("algo,p", [("frogsort2", 0.1), ("frogsort3", 0.25), ("frogsort6", 0.1)])
def test_order_fast_paths_small_buffer(gs, orc, algo, p):
    n = 1_000_003
    for name, (x, want) in _order_cases(n, seed=11).items():
        announce("order small buffer", algo, name)
        t = to_dev(x)
        rep = gs.gs_sort_f64(t, buffer_fraction=p, algo=algo, sub_fraction=0.25, report=True)
        assert np.array_equal(bits(t), bits(orc.sort_f64(x))), name
        assert rep["order"] == want, name


def test_concurrent_streams(gs, orc):
    """Calls on different streams with different workspaces run at the same
    time: a plain sort, a Frogsort3 sort (with its table upload) and a
    key/value sort, each on its own stream, all bit for bit right."""
    torch = need_gpu()
    n = 3_000_017
    announce("concurrent streams", n)
    xs = [W.f64_pattern("uniform", n, seed=s) for s in (31, 32)]
    k, v = W.kv_pattern("few", n, seed=33)
    ts = [to_dev(x) for x in xs]
    tk, tv = to_dev(k.view(np.int64)), to_dev(v.view(np.int32))
    streams = [torch.cuda.Stream() for _ in range(3)]

    def ws(nbytes):
        w = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        return w[(-w.data_ptr()) % 256:][:nbytes]
    w0 = ws(gs.gs_workspace_bytes_f64(n))
    w1 = ws(gs.gs_workspace_bytes_f64(n, 0.2))
    w2 = ws(gs.gs_workspace_bytes_kv(n))
    torch.cuda.synchronize()
    for _ in range(2):
        gs.gs_sort_f64(ts[0], workspace=w0, stream=streams[0])
        gs.gs_sort_f64(ts[1], 0.2, workspace=w1, stream=streams[1])
        gs.gs_sort_kv(tk, tv, workspace=w2, stream=streams[2])
    torch.cuda.synchronize()
    for t, x in zip(ts, xs):
        assert np.array_equal(bits(t), bits(orc.sort_f64(x)))
    rk, rv = orc.sort_kv(k, v)
    assert np.array_equal(tk.cpu().numpy().view(np.uint64), rk)
    assert np.array_equal(tv.cpu().numpy().view(np.uint32), rv)


@pytest.mark.parametrize("kv", [False, True])
def test_graph_capture_replay(gs, orc, kv):
    """The plain sort (Frogsort1) captured once into a HIP graph and replayed
    on fresh inputs copied into the captured buffers -- unsorted, presorted
    and reversed, so every replay takes a different branch of the on-device
    order decision -- with eager work between replays; every replay is
    checked against the oracle."""
    torch = need_gpu()
    n = (1 << 20) + 7
    announce("graph capture", "kv" if kv else "f64", n)
    if kv:
        k0, v0 = W.kv_pattern("uniform", n, seed=3)
        keys, vals = to_dev(k0.view(np.int64)), to_dev(v0.view(np.int32))
        need = gs.gs_workspace_bytes_kv(n)
    else:
        keys, vals = to_dev(W.f64_pattern("uniform", n, seed=3)), None
        need = gs.gs_workspace_bytes_f64(n)
    ws_raw = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    o = (-ws_raw.data_ptr()) % 256
    ws = ws_raw[o:o + need]

    def call(stream):
        if kv:
            gs.gs_sort_kv(keys, vals, workspace=ws, stream=stream)
        else:
            gs.gs_sort_f64(keys, workspace=ws, stream=stream)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):                      # warm-up outside capture
        call(s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        call(s)
    for pattern in ("uniform", "presorted", "reversed", "tied"):
        if kv:
            k, v = W.kv_pattern("few" if pattern == "tied" else "uniform", n, seed=17)
            if pattern == "presorted":
                k = np.sort(k)
            elif pattern == "reversed":
                k = np.sort(k)[::-1].copy()
            keys.copy_(torch.from_numpy(k.view(np.int64)))
            vals.copy_(torch.from_numpy(v.view(np.int32)))
        else:
            x = W.f64_pattern(pattern, n, seed=17)
            keys.copy_(torch.from_numpy(x))
        _ = (keys * 2).sum()                        # unrelated eager work
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        if kv:
            rk, rv = orc.sort_kv(k, v)
            assert np.array_equal(keys.cpu().numpy().view(np.uint64), rk), pattern
            assert np.array_equal(vals.cpu().numpy().view(np.uint32), rv), pattern
        else:
            assert np.array_equal(bits(keys), bits(orc.sort_f64(x))), pattern
