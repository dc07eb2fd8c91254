"""Device-side failures reach the caller with and without a report, and the
binding's temporary workspaces stay valid on the caller's stream.

The failures are forced from the host: the test setting makes every bounded
wait of the ordered-store protocol complete as usual and then record itself as
one that gave up, so every kernel ends normally and the outputs stay right
(checked against the oracle) while the error paths run.
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


@pytest.fixture
def forced_failures(gs):
    torch = need_gpu()
    torch.cuda.synchronize()
    gs.gs_device_errors(clear=True)
    was = gs.gs_test_fail_waits(True)
    yield
    gs.gs_test_fail_waits(was)
    torch.cuda.synchronize()
    gs.gs_device_errors(clear=True)


def test_normal_calls_leave_no_flags(gs, orc):
    torch = need_gpu()
    announce("device errors: clean run")
    torch.cuda.synchronize()
    gs.gs_device_errors(clear=True)
    x = W.f64_pattern("uniform", (1 << 20) + 7, seed=5)
    t = to_dev(x)
    rep = gs.gs_sort_f64(t, report=True)
    assert rep["levels"] > 0
    t = to_dev(x)
    gs.gs_sort_f64(t)
    torch.cuda.synchronize()
    assert gs.gs_device_errors() == 0
    assert np.array_equal(bits(t), bits(orc.sort_f64(x)))


def test_forced_wait_failure_with_report(gs, orc, forced_failures):
    announce("device errors: report")
    x = W.f64_pattern("uniform", (1 << 20) + 7, seed=6)
    t = to_dev(x)
    with pytest.raises(gs.GsError) as ei:
        gs.gs_sort_f64(t, report=True)
    assert ei.value.status == gs.GS_EDEVICE
    assert np.array_equal(bits(t), bits(orc.sort_f64(x)))       # the waits did complete
    k, v = W.kv_pattern("uniform", (1 << 19) + 3, seed=6)
    tk, tv = to_dev(k.view(np.int64)), to_dev(v.view(np.int32))
    with pytest.raises(gs.GsError) as ei:
        gs.gs_sort_kv(tk, tv, report=True)
    assert ei.value.status == gs.GS_EDEVICE


@pytest.mark.parametrize("call", ["f64", "f64_frogsort3", "kv", "segsort", "learned"])
def test_forced_wait_failure_without_report(gs, orc, forced_failures, call):
    """Without a report the calls return normally; the device's sticky flags
    show the failure once the stream is synchronised."""
    torch = need_gpu()
    announce("device errors: no report", call)
    n = (1 << 20) + 7
    if call in ("f64", "f64_frogsort3"):
        x = W.f64_pattern("uniform", n, seed=7)
        t = to_dev(x)
        gs.gs_sort_f64(t, 0.25 if call == "f64_frogsort3" else 0.5)
        torch.cuda.synchronize()
        assert np.array_equal(bits(t), bits(orc.sort_f64(x)))
    elif call == "kv":
        k, v = W.kv_pattern("zipf", n, seed=7)
        tk, tv = to_dev(k.view(np.int64)), to_dev(v.view(np.int32))
        gs.gs_sort_kv(tk, tv)
        torch.cuda.synchronize()
        rk, rv = orc.sort_kv(k, v)
        assert np.array_equal(tk.cpu().numpy().view(np.uint64), rk)
        assert np.array_equal(tv.cpu().numpy().view(np.uint32), rv)
    elif call == "segsort":
        x, off = W.segmented(40, 16, 200_000, seed=7)
        t, to = to_dev(x), to_dev(off)
        gs.gs_segsort(t, to)
        torch.cuda.synchronize()
        assert np.array_equal(bits(t), bits(orc.segsort_f64(x, off)))
    else:
        x = W.learned_pattern("lognormal", 1 << 20, seed=7)
        t = to_dev(x)
        gs.gs_learned_sort(t)
        torch.cuda.synchronize()
        assert np.array_equal(bits(t), bits(orc.sort_f64(x)))
    assert gs.gs_device_errors(clear=True) & gs.GS_DEVERR_WAIT
    assert gs.gs_device_errors() == 0


def test_rejected_offsets_without_report(gs):
    """Offsets that decrease: nothing is written; without a report the call
    returns normally and the sticky flags name the offsets."""
    torch = need_gpu()
    announce("device errors: offsets")
    torch.cuda.synchronize()
    gs.gs_device_errors(clear=True)
    x = W.f64_pattern("uniform", 10_000, seed=8)
    off = np.array([0, 5000, 3000, 10_000], dtype=np.int64)
    t = to_dev(x)
    gs.gs_segsort(t, to_dev(off))
    torch.cuda.synchronize()
    assert np.array_equal(bits(t), bits(x))
    assert gs.gs_device_errors(clear=True) == gs.GS_DEVERR_OFFSETS


def test_errors_of_unknown_device(gs):
    torch = need_gpu()
    with pytest.raises(gs.GsError) as ei:
        gs.gs_device_errors(torch.cuda.device_count())
    assert ei.value.status == gs.GS_EINVAL


@pytest.mark.parametrize("call", ["f64", "kv", "learned"])
def test_side_stream_without_workspace(gs, orc, call):
    """A call on a side stream with no workspace given: the binding allocates
    the workspace on the current stream, so it must keep that memory from
    being handed out again while the side stream still sorts.  A tensor of the
    same size is allocated and filled on the current stream right after the
    call returns; the sort must still come out right."""
    torch = need_gpu()
    announce("side stream, binding-owned workspace", call)
    n = (1 << 22) + 5
    side = torch.cuda.Stream()
    if call == "kv":
        k, v = W.kv_pattern("uniform", n, seed=9)
        tk, tv = to_dev(k.view(np.int64)), to_dev(v.view(np.int32))
        need = gs.gs_workspace_bytes_kv(n)
    else:
        x = W.learned_pattern("lognormal", n, seed=9) if call == "learned" else W.f64_pattern("uniform", n, seed=9)
        t = to_dev(x)
        need = gs.gs_workspace_bytes_learned(n) if call == "learned" else gs.gs_workspace_bytes_f64(n)
    side.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    if call == "kv":
        gs.gs_sort_kv(tk, tv, stream=side)
    elif call == "learned":
        gs.gs_learned_sort(t, stream=side)
    else:
        gs.gs_sort_f64(t, stream=side)
    junk = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    junk.fill_(0x5A)
    torch.cuda.synchronize()
    del junk
    if call == "kv":
        rk, rv = orc.sort_kv(k, v)
        assert np.array_equal(tk.cpu().numpy().view(np.uint64), rk)
        assert np.array_equal(tv.cpu().numpy().view(np.uint32), rv)
    else:
        assert np.array_equal(bits(t), bits(orc.sort_f64(x)))
