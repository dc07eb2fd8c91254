"""The small-buffer trees on the GPU: Frogsort2 ("Frogsort2": inner branch and
buffer both a fraction p < 1/2 of the data) and Frogsort3 ("Frogsort3 and 6": one
buffer of that fraction serving the branches in turn).  Parity with the CPU
oracle through the C ABI, bit for bit, for fractions from 1/64 to just under
1/2, sizes from one leaf to many rounds with ragged tails, both key types and
all four targets; at 2^28 the oracle's counting definition fixes sampled
positions."""
import numpy as np
import pytest

import workloads as W
from gpu_util import announce, bits, multiset_hash_dev, need_gpu, to_dev

pytestmark = pytest.mark.gpu

FRACTIONS = [1 / 64, 0.05, 0.1, 0.2, 1 / 3, 0.4999]
ALGOS = ["frogsort2", "frogsort3"]
SIZES = [2, 17, 8192, 8193, 12345, 65537, 100003, (1 << 20) + 7]
PATTERNS = ["uniform", "tied", "presorted", "reversed", "zeros_signed"]


@pytest.fixture(scope="module")
def gs():
    need_gpu()
    import paper_2402_01816_amd as g
    return g


@pytest.mark.parametrize("pattern", PATTERNS)
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("p", FRACTIONS)
@pytest.mark.parametrize("algo", ALGOS)
def test_small_buffer_f64_parity(gs, orc, algo, p, n, pattern):
    announce("small-buffer f64", algo, p, n, pattern)
    x = W.f64_pattern(pattern, n, seed=31 + n)
    t = to_dev(x)
    gs.gs_sort_f64(t, buffer_fraction=p, algo=algo)
    assert np.array_equal(bits(t), bits(orc.sort_f64(x)))


@pytest.mark.parametrize("pattern", ["uniform", "few"])
@pytest.mark.parametrize("n", [4097, 65537, (1 << 20) + 3])
@pytest.mark.parametrize("p", [1 / 64, 0.1, 0.25, 0.45])
@pytest.mark.parametrize("algo", ALGOS)
def test_small_buffer_kv_parity(gs, orc, algo, p, n, pattern):
    announce("small-buffer kv", algo, p, n, pattern)
    k, v = W.kv_pattern(pattern, n, seed=9)
    tk = to_dev(k.view(np.int64))
    tv = to_dev(v.view(np.int32))
    gs.gs_sort_kv(tk, tv, buffer_fraction=p, algo=algo)
    rk, rv = orc.sort_kv(k, v)
    assert np.array_equal(tk.cpu().numpy().view(np.uint64), rk)
    assert np.array_equal(tv.cpu().numpy().view(np.uint32), rv)


@pytest.mark.parametrize("target", ("AscLeft", "AscRight", "DescLeft", "DescRight"))
@pytest.mark.parametrize("algo", ALGOS)
def test_small_buffer_targets(gs, orc, algo, target):
    n = (1 << 20) + 7
    announce("small-buffer target", algo, target, n)
    x = W.f64_pattern("zeros_signed", n, seed=3)
    x[::61] = np.nan
    x[::67] = -np.inf
    t = to_dev(x)
    gs.gs_sort_f64(t, buffer_fraction=0.1, target=target, algo=algo)
    assert np.array_equal(bits(t), bits(orc.sort_f64_target(x, target)))
    k, v = W.kv_pattern("few", n, seed=4)
    tk = to_dev(k.view(np.int64))
    tv = to_dev(v.view(np.int32))
    gs.gs_sort_kv(tk, tv, buffer_fraction=0.2, target=target, algo=algo)
    rk, rv = orc.sort_kv_target(k, v, target)
    assert np.array_equal(tk.cpu().numpy().view(np.uint64), rk)
    assert np.array_equal(tv.cpu().numpy().view(np.uint32), rv)


@pytest.mark.parametrize("p", [0.05, 0.25])
@pytest.mark.parametrize("algo", ALGOS)
def test_small_buffer_report(gs, orc, algo, p):
    """The report carries the merge rounds and %RAM = 1 + at most the buffer
    fraction + a small control area."""
    n = 1 << 22
    t = to_dev(W.f64_pattern("uniform", n, seed=2))
    rep = gs.gs_sort_f64(t, buffer_fraction=p, report=True, algo=algo)
    counts = gs.plan_frog2(n, p)[2] if algo == "frogsort2" else gs.plan_frog3(n, p)[3]
    assert rep["levels"] == (counts[2] if algo == "frogsort2" else counts[3])
    assert rep["workspace_bytes_used"] == gs.gs_workspace_bytes_f64(n, p, algo)
    assert 1 + p - 0.002 <= rep["ram_fraction"] < 1 + p + 0.02
    assert np.array_equal(bits(t), bits(orc.sort_f64(W.f64_pattern("uniform", n, seed=2))))


def test_small_buffer_repeated_calls(gs, orc):
    """Calls with different trees, fractions and sizes in a row, most reusing
    one workspace: the plan caches and the uploaded tables never mix."""
    torch = need_gpu()
    big = 2 * gs.gs_workspace_bytes_f64(300_001, 0.1, "frogsort2")
    ws = torch.empty(big + 256, dtype=torch.uint8, device="cuda")
    off = (-ws.data_ptr()) % 256
    ws = ws[off: off + big]
    for i, (p, n) in enumerate([(0.1, 300_001), (0.3, 200_000), (0.05, 123_457), (0.1, 300_001),
                                (0.49, 250_000), (0.2, 100_000)]):
        for algo in ALGOS:
            announce("small-buffer repeated", algo, p, n)
            x = W.f64_pattern("uniform", n, seed=40 + i)
            t = to_dev(x)
            need = gs.gs_workspace_bytes_f64(n, p, algo)
            gs.gs_sort_f64(t, buffer_fraction=p, algo=algo, workspace=ws if need <= big else None)
        assert np.array_equal(bits(t), bits(orc.sort_f64(x)))


@pytest.mark.parametrize("p", [0.1, 0.25])
@pytest.mark.parametrize("algo", ALGOS)
def test_small_buffer_full_size_sampled(gs, orc, algo, p):
    """n = 2^28: sampled positions from the oracle's counting definition,
    plus sortedness and multiset equality over the whole output."""
    torch = need_gpu()
    n = 1 << 28
    announce("small-buffer full", algo, p, n)
    x = W.f64_pattern("uniform", n, seed=0)
    t = to_dev(x)
    h_in = multiset_hash_dev(t)
    gs.gs_sort_f64(t, buffer_fraction=p, algo=algo)
    torch.cuda.synchronize()
    assert multiset_hash_dev(t) == h_in
    assert bool((t[1:] >= t[:-1]).all().item())
    rng = np.random.default_rng(2)
    idx = np.concatenate([[0, n - 1], rng.integers(0, n, 14)])
    ranks = orc.rank_f64(x, idx)
    got = t[torch.from_numpy(ranks).to("cuda")].cpu().numpy()
    assert np.array_equal(bits(got), bits(x[idx]))


@pytest.mark.parametrize("n", [8193, 100003, (1 << 20) + 7, (1 << 22) + 3])
@pytest.mark.parametrize("p,p2", [(0.1, 0.25), (0.05, 0.2), (1 / 64, 0.1), (0.25, 0.2), (0.3, 0.45)])
def test_frog6_parity(gs, orc, p, p2, n):
    """Frogsort6: the buffer shared as in Frogsort3 with Frogsort2 sub-trees
    at p2 (a single Frogsort2 tree once p >= p2)."""
    announce("frog6", p, p2, n)
    x = W.f64_pattern("tied", n, seed=n)
    t = to_dev(x)
    gs.gs_sort_f64(t, buffer_fraction=p, algo="frogsort6", sub_fraction=p2)
    assert np.array_equal(bits(t), bits(orc.sort_f64(x)))
    k, v = W.kv_pattern("few", n, seed=n)
    tk = to_dev(k.view(np.int64))
    tv = to_dev(v.view(np.int32))
    gs.gs_sort_kv(tk, tv, buffer_fraction=p, algo="frogsort6", sub_fraction=p2)
    rk, rv = orc.sort_kv(k, v)
    assert np.array_equal(tk.cpu().numpy().view(np.uint64), rk)
    assert np.array_equal(tv.cpu().numpy().view(np.uint32), rv)


@pytest.mark.filterwarnings("ignore:The CUDA Graph is empty")   # nothing may be recorded
def test_small_buffer_rejects_capture(gs):
    """A small-buffer call uploads host-built tables, so it refuses to be
    recorded into a graph (and enqueues nothing)."""
    torch = need_gpu()
    n = 100_000
    t = to_dev(W.f64_pattern("uniform", n, seed=1))
    need = gs.gs_workspace_bytes_f64(n, 0.1)
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    off = (-ws.data_ptr()) % 256
    ws = ws[off: off + need]
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    err = None
    with torch.cuda.stream(s):
        g.capture_begin()
        try:
            gs.gs_sort_f64(t, buffer_fraction=0.1, workspace=ws, stream=s)
        except gs.GsError as e:
            err = e
        finally:
            g.capture_end()
    assert err is not None and err.status == gs.GS_EUNSUPPORTED
