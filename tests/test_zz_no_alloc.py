"""gs_sort_f64_noalloc: the plain sort with the library's static device
workspace, compared bit for bit with gs_sort_f64 (the same sort with a caller
workspace) and with the oracle, on two calls in a row, the second smaller.
Called through the C ABI (ctypes), as every entry point is."""
import ctypes

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


def _noalloc(gs, t, stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return gs.lib.gs_sort_f64_noalloc(ctypes.c_void_p(t.data_ptr()) if t.numel() else None, t.numel(),
                                      ctypes.c_void_p(s.cuda_stream))


def test_noalloc_matches_workspace_entry_point(gs, orc):
    torch = need_gpu()
    torch.cuda.synchronize()
    gs.gs_device_errors(clear=True)
    # the largest size first, then a smaller one: the second call reuses the
    # static array as the first left it
    for n, pattern, seed in ((gs.NOALLOC_MAX_KEYS, "zeros_signed", 21), (100_003, "uniform", 22),
                             ((1 << 20) + 7, "tied", 23)):
        announce("noalloc", pattern, n)
        x = W.f64_pattern(pattern, n, seed=seed)
        a, b = to_dev(x), to_dev(x)
        assert _noalloc(gs, a) == gs.GS_OK
        gs.gs_sort_f64(b)
        torch.cuda.synchronize()
        assert np.array_equal(bits(a), bits(b)), (pattern, n)
        assert np.array_equal(bits(a), bits(orc.sort_f64(x))), (pattern, n)
    assert gs.gs_device_errors() == 0


def test_noalloc_order_check_and_small(gs, orc):
    """Presorted and reversed input take the order check's branches; n <= 1
    is a no-op; the binding's wrapper gives the same result."""
    torch = need_gpu()
    for pattern in ("presorted", "reversed", "perturbed"):
        x = W.f64_pattern(pattern, 300_001, seed=24)
        a = to_dev(x)
        gs.gs_sort_f64_noalloc(a)
        torch.cuda.synchronize()
        assert np.array_equal(bits(a), bits(orc.sort_f64(x))), pattern
    for n in (0, 1, 2, 3):
        x = W.f64_pattern("uniform", n, seed=25)
        a = to_dev(x)
        assert _noalloc(gs, a) == gs.GS_OK
        torch.cuda.synchronize()
        assert np.array_equal(bits(a), bits(orc.sort_f64(x)))


def test_noalloc_rejects_above_limit(gs):
    """One key above the limit: GS_EINVAL before anything is enqueued."""
    torch = need_gpu()
    n = gs.NOALLOC_MAX_KEYS + 1
    x = W.f64_pattern("uniform", n, seed=26)
    a = to_dev(x)
    assert _noalloc(gs, a) == gs.GS_EINVAL
    assert "limit" in gs.lib.gs_last_error_detail().decode()
    torch.cuda.synchronize()
    assert np.array_equal(bits(a), bits(x))


def test_noalloc_under_graph_capture(gs, orc):
    """Captured into a HIP graph (no allocation inside the capture) and
    replayed on new inputs copied into the captured buffer, with eager work
    between the replays."""
    torch = need_gpu()
    n = 500_009
    keys = to_dev(W.f64_pattern("uniform", n, seed=27))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        assert _noalloc(gs, keys, s) == gs.GS_OK
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        assert _noalloc(gs, keys, s) == gs.GS_OK
    for pattern in ("uniform", "reversed", "zeros_signed"):
        x = W.f64_pattern(pattern, n, seed=28)
        keys.copy_(torch.from_numpy(x))
        _ = (keys * 3).sum()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(bits(keys), bits(orc.sort_f64(x))), pattern
