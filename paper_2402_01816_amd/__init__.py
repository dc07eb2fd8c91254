"""Python binding of libgs.so (include/gs.h): argument marshalling only.

Every sorting step runs in the library's HIP kernels; this module only turns
torch tensors into device pointers, allocates the caller-owned workspace with
torch, passes the current HIP stream and converts status codes into
exceptions.  There is no fallback: if libgs.so is missing, importing this
module raises.

The functions carry the C names: gs_sort_f64, gs_sort_kv, gs_segsort,
gs_learned_sort and the gs_workspace_bytes_* queries.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgs.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is not built; run `python paper_2402_01816_amd/build.py` "
        "(hipcc, gfx950) first")

# torch brings its own copy of the HIP runtime (same soname as the system one).
# Loading torch first makes libgs.so bind to that already-loaded runtime, so the
# process holds exactly one HIP runtime and torch's memory and streams are valid
# handles for the library.
import torch  # noqa: E402,F401  (must precede loading libgs.so)

_lib = ctypes.CDLL(LIB_PATH)

GS_OK, GS_EINVAL, GS_EUNSUPPORTED, GS_EWORKSPACE, GS_ENODEVICE, GS_EDEVICE = range(6)
STATUS_NAMES = {0: "GS_OK", 1: "GS_EINVAL", 2: "GS_EUNSUPPORTED", 3: "GS_EWORKSPACE",
                4: "GS_ENODEVICE", 5: "GS_EDEVICE"}
MLP_NUM_PARAMS = 4353
SIZE_MAX = ctypes.c_size_t(-1).value


class GsReport(ctypes.Structure):
    _fields_ = [
        ("ram_fraction", ctypes.c_double),
        ("workspace_bytes_used", ctypes.c_uint64),
        ("levels", ctypes.c_uint32),
        ("fallback", ctypes.c_uint32),
        ("overflow_buckets", ctypes.c_uint32),
        ("max_bucket", ctypes.c_uint32),
        ("train_loss_first", ctypes.c_float),
        ("train_loss_last", ctypes.c_float),
        ("feature", ctypes.c_uint32),
        ("invalid_offsets", ctypes.c_uint32),
        ("elapsed_ms", ctypes.c_double),
        ("order", ctypes.c_uint32),
        ("heavy_values", ctypes.c_uint32),
        ("keys_moved", ctypes.c_uint64),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class GsLearnedParams(ctypes.Structure):
    _fields_ = [
        ("num_buckets", ctypes.c_uint32),
        ("sample_size", ctypes.c_uint32),
        ("train_steps", ctypes.c_uint32),
        ("batch", ctypes.c_uint32),
        ("knots", ctypes.c_uint32),
        ("lr", ctypes.c_float),
        ("seed", ctypes.c_uint64),
        ("mode", ctypes.c_uint32),
        ("screen", ctypes.c_uint32),
        ("weights_override", ctypes.c_void_p),
        ("test_bucket_table", ctypes.c_void_p),
        ("buffer_fraction", ctypes.c_double),
    ]


class GsSegConfig(ctypes.Structure):
    """Shape of a segmented sort (mirrors gs_seg_config)."""
    _fields_ = [
        ("short_threads", ctypes.c_uint32),
        ("short_ipt", ctypes.c_uint32),
        ("merge_ipt", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]

    def as_dict(self):
        return {"short_threads": self.short_threads, "short_ipt": self.short_ipt,
                "merge_ipt": self.merge_ipt}


class GsError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        self.status_name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{where}: {self.status_name}: {detail}")


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_D = ctypes.c_double
_SZ = ctypes.c_size_t

_SIGS = {
    "gs_workspace_bytes_f64": ([_I64, _D], _SZ),
    "gs_workspace_bytes_kv": ([_I64, _D], _SZ),
    "gs_sort_f64": ([_P, _I64, _D, _P, _SZ, _P, ctypes.POINTER(GsReport)], ctypes.c_int),
    "gs_sort_kv": ([_P, _P, _I64, _D, _P, _SZ, _P, ctypes.POINTER(GsReport)], ctypes.c_int),
    "gs_sort_f64_target": ([_P, _I64, ctypes.c_int, _D, _P, _SZ, _P, ctypes.POINTER(GsReport)],
                           ctypes.c_int),
    "gs_sort_kv_target": ([_P, _P, _I64, ctypes.c_int, _D, _P, _SZ, _P, ctypes.POINTER(GsReport)],
                          ctypes.c_int),
    "gs_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "gs_last_error_detail": ([], ctypes.c_char_p),
    "gs_version": ([], ctypes.c_char_p),
    "gs_plan_depth": ([_I64, ctypes.c_int, ctypes.POINTER(_I64)], ctypes.c_int),
    "gs_plan_node": ([_I64, ctypes.c_int, _I64, ctypes.POINTER(_I64)], None),
    "gs_plan_leaf_window": ([_I64, ctypes.c_int, _I64, ctypes.c_void_p], ctypes.c_int),
    "gs_plan_tile_windows": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _I64,
                              ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "gs_plan_frog2": ([_I64, ctypes.c_double, ctypes.c_int, ctypes.c_void_p, _I64, ctypes.c_void_p, _I64,
                       ctypes.c_void_p], ctypes.c_int),
    "gs_plan_frog3": ([_I64, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_void_p, _I64,
                       ctypes.c_void_p, _I64, ctypes.c_void_p, _I64, ctypes.c_void_p], ctypes.c_int),
    "gs_tune_cache_get": ([ctypes.c_char_p, _I64, _I64, ctypes.POINTER(GsSegConfig)], ctypes.c_int),
    "gs_tune_cache_put": ([ctypes.c_char_p, _I64, _I64, ctypes.POINTER(GsSegConfig)], ctypes.c_int),
    "gs_tune_cache_load": ([ctypes.c_char_p], ctypes.c_int),
    "gs_tune_cache_save": ([ctypes.c_char_p], ctypes.c_int),
    "gs_tune_cache_clear": ([], None),
    "gs_plan_seg_steps": ([ctypes.c_void_p, _I64, _I64, _D, ctypes.c_void_p, _I64, ctypes.c_void_p], _I64),
    "gs_workspace_bytes_f64_ex": ([_I64, _D, ctypes.c_int, _D], _SZ),
    "gs_workspace_bytes_kv_ex": ([_I64, _D, ctypes.c_int, _D], _SZ),
    "gs_sort_f64_ex": ([_P, _I64, ctypes.c_int, _D, ctypes.c_int, _D, _P, _SZ, _P, ctypes.POINTER(GsReport)],
                       ctypes.c_int),
    "gs_sort_kv_ex": ([_P, _P, _I64, ctypes.c_int, _D, ctypes.c_int, _D, _P, _SZ, _P,
                       ctypes.POINTER(GsReport)], ctypes.c_int),
}
_OPTIONAL = {
    "gs_workspace_bytes_seg": ([_I64, _I64, _D], _SZ),
    "gs_workspace_bytes_learned": ([_I64, ctypes.POINTER(GsLearnedParams)], _SZ),
    "gs_segsort": ([_P, _I64, _P, _I64, _D, _P, _SZ, _P, ctypes.POINTER(GsReport)], ctypes.c_int),
    "gs_seg_config_count": ([], ctypes.c_int),
    "gs_seg_config_get": ([ctypes.c_int, ctypes.POINTER(GsSegConfig)], ctypes.c_int),
    "gs_seg_default_config": ([ctypes.POINTER(GsSegConfig)], None),
    "gs_workspace_bytes_seg_ex": ([_I64, _I64, _D, ctypes.POINTER(GsSegConfig)], _SZ),
    "gs_segsort_ex": ([_P, _I64, _P, _I64, _D, ctypes.POINTER(GsSegConfig), _P, _SZ, _P,
                       ctypes.POINTER(GsReport)], ctypes.c_int),
    "gs_segsort_autotune": ([_P, _I64, _P, _I64, _P, _P, _SZ, _P, ctypes.c_int,
                             ctypes.POINTER(GsSegConfig), ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
    "gs_learned_sort": ([_P, _I64, ctypes.POINTER(GsLearnedParams), _P, _SZ, _P,
                         ctypes.POINTER(GsReport)], ctypes.c_int),
    "gs_learned_default_params": ([ctypes.POINTER(GsLearnedParams)], None),
    "gs_mlp_loss_grad": ([_P, _P, _P, ctypes.c_int, _P, _P, _P, _SZ, _P], ctypes.c_int),
    "gs_mlp_train": ([_P, _P, _P, _P, _P, _I64, ctypes.c_int, ctypes.c_int, ctypes.c_float,
                      ctypes.c_uint64, ctypes.c_int, _P, _P, _SZ, _P], ctypes.c_int),
    "gs_mlp_forward": ([_P, _P, _I64, _P, _P], ctypes.c_int),
    "gs_sort_f64_noalloc": ([_P, _I64, _P], ctypes.c_int),
    "gs_device_errors": ([ctypes.c_int, ctypes.POINTER(ctypes.c_uint32), ctypes.c_int], ctypes.c_int),
    "gs_test_fail_waits": ([ctypes.c_int], ctypes.c_int),
    "gs_trace_enable": ([ctypes.c_int], ctypes.c_int),
    "gs_copy_f64": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p], ctypes.c_int),
    "gs_trace_read": ([ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double), ctypes.c_int],
                      ctypes.c_int),
}
for _name, (_args, _res) in {**_SIGS, **_OPTIONAL}.items():
    if _name in _SIGS or hasattr(_lib, _name):
        _fn = getattr(_lib, _name)
        _fn.argtypes = _args
        _fn.restype = _res

lib = _lib


def version() -> str:
    return _lib.gs_version().decode()


def _detail() -> str:
    return _lib.gs_last_error_detail().decode(errors="replace")


def _check(status: int, where: str):
    if status != GS_OK:
        raise GsError(status, where, _detail())


# ---------------------------------------------------------------------------
# workspace queries
# ---------------------------------------------------------------------------
ALGOS = {"auto": 0, "frogsort1": 1, "frogsort2": 2, "frogsort3": 3, "frogsort6": 4}


def _algo(algo) -> int:
    if isinstance(algo, str):
        return ALGOS[algo.lower()]
    return int(algo)


def gs_workspace_bytes_f64(n: int, buffer_fraction: float = 0.5, algo="auto", sub_fraction: float = 0.5) -> int:
    return int(_lib.gs_workspace_bytes_f64_ex(n, buffer_fraction, _algo(algo), sub_fraction))


def gs_workspace_bytes_kv(n: int, buffer_fraction: float = 0.5, algo="auto", sub_fraction: float = 0.5) -> int:
    return int(_lib.gs_workspace_bytes_kv_ex(n, buffer_fraction, _algo(algo), sub_fraction))


def gs_workspace_bytes_seg(num_keys: int, num_segments: int, buffer_fraction: float = 0.5) -> int:
    return int(_lib.gs_workspace_bytes_seg(num_keys, num_segments, buffer_fraction))


def gs_learned_default_params() -> GsLearnedParams:
    p = GsLearnedParams()
    _lib.gs_learned_default_params(ctypes.byref(p))
    return p


def gs_workspace_bytes_learned(n: int, params: GsLearnedParams | None = None) -> int:
    p = params if params is not None else gs_learned_default_params()
    return int(_lib.gs_workspace_bytes_learned(n, ctypes.byref(p)))


def plan_depth(n: int, kv: bool = False):
    leaf = _I64(0)
    d = _lib.gs_plan_depth(n, 1 if kv else 0, ctypes.byref(leaf))
    return d, leaf.value


def plan_node(n: int, depth: int, idx: int):
    out = (_I64 * 5)()
    _lib.gs_plan_node(n, depth, idx, out)
    return tuple(out)


def plan_frog2(n: int, buffer_fraction: float, kv: bool = False):
    """The library's Frogsort2 plan for n keys (host only): leaves as rows
    (input offset, data start, length) in input order, merge nodes as rows
    (region start, n, is_left, round), and the counts
    (leaves, nodes, rounds, buffer elements, largest round's tiles, splits,
    elements merged)."""
    import numpy as np
    counts = np.zeros(7, dtype=np.int64)
    if _lib.gs_plan_frog2(n, buffer_fraction, 1 if kv else 0, None, 0, None, 0, counts.ctypes.data) != 0:
        raise ValueError("no Frogsort2 plan for these arguments")
    leaves = np.zeros((int(counts[0]), 3), dtype=np.int64)
    nodes = np.zeros((max(int(counts[1]), 1), 4), dtype=np.int64)
    _lib.gs_plan_frog2(n, buffer_fraction, 1 if kv else 0, leaves.ctypes.data, leaves.shape[0],
                       nodes.ctypes.data, int(counts[1]), counts.ctypes.data)
    return leaves, nodes[: int(counts[1])], tuple(int(c) for c in counts)


def plan_frog3(n: int, buffer_fraction: float, kv: bool = False, sub_fraction: float = 0.5):
    """The library's Frogsort3 schedule for n keys (Frogsort6 with
    sub_fraction < 0.5; host only): trees as rows
    (root region start, elements, input offset, is_left) in running order,
    spine merges as rows (outer elements, inner start, inner elements) bottom
    up, every tree's leaves (input offset, data start, length), and the counts
    (trees, spine merges, leaves, merge rounds, buffer elements, b, elements
    merged)."""
    import numpy as np
    counts = np.zeros(7, dtype=np.int64)
    if _lib.gs_plan_frog3(n, buffer_fraction, sub_fraction, 1 if kv else 0, None, 0, None, 0, None, 0,
                          counts.ctypes.data) != 0:
        raise ValueError("no Frogsort3 plan for these arguments")
    trees = np.zeros((int(counts[0]), 4), dtype=np.int64)
    spine = np.zeros((max(int(counts[1]), 1), 3), dtype=np.int64)
    leaves = np.zeros((int(counts[2]), 3), dtype=np.int64)
    _lib.gs_plan_frog3(n, buffer_fraction, sub_fraction, 1 if kv else 0, trees.ctypes.data, trees.shape[0],
                       spine.ctypes.data, int(counts[1]), leaves.ctypes.data, leaves.shape[0],
                       counts.ctypes.data)
    return trees, spine[: int(counts[1])], leaves, tuple(int(c) for c in counts)


def gs_tune_cache_get(num_keys: int, num_segments: int, arch: str | None = None):
    """The segmented-sort shape the tuning cache holds for this size class
    (arch None: the current device's), as a dict, or None."""
    c = GsSegConfig()
    r = _lib.gs_tune_cache_get(arch.encode() if arch else None, num_keys, num_segments, ctypes.byref(c))
    if r < 0:
        raise ValueError("bad tuning-cache query")
    return dict(short_threads=c.short_threads, short_ipt=c.short_ipt, merge_ipt=c.merge_ipt) if r else None


def gs_tune_cache_put(arch: str, num_keys: int, num_segments: int, config):
    _check(_lib.gs_tune_cache_put(arch.encode(), num_keys, num_segments, ctypes.byref(_seg_config(config))),
           "gs_tune_cache_put")


def plan_seg_steps(offsets, num_keys: int, buffer_fraction: float):
    """The segmented sort's steps below buffer fraction 0.5 (host only): rows
    (first segment, one past the last, 1 if sorted alone by the plain sort)
    and the buffer's elements, for host int64 offsets."""
    import numpy as np
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    nseg = max(off.shape[0] - 1, 0)
    buf = _I64(0)
    cnt = _lib.gs_plan_seg_steps(off.ctypes.data, nseg, num_keys, buffer_fraction, None, 0, ctypes.byref(buf))
    if cnt < 0:
        raise ValueError("no segmented steps for these arguments")
    rows = np.zeros((max(cnt, 1), 3), dtype=np.int64)
    _lib.gs_plan_seg_steps(off.ctypes.data, nseg, num_keys, buffer_fraction, rows.ctypes.data, cnt, None)
    return rows[:cnt], buf.value


# ---------------------------------------------------------------------------
# torch marshalling
# ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _on_stream(stream, *tensors):
    """Temporaries allocated here on the current stream but used by a call
    on another stream: tell torch's caching allocator, so it does not hand
    their memory out again before the work queued on that stream is done."""
    if stream is None:
        return
    for t in tensors:
        if t is not None:
            t.record_stream(stream)


def _workspace(nbytes: int, device, workspace=None, stream=None):
    torch = _torch()
    if nbytes == 0:
        return None, 0
    if workspace is not None:
        if workspace.device != device or workspace.dtype != torch.uint8:
            raise ValueError("workspace must be a uint8 tensor on the keys' device")
        return workspace, workspace.numel()
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    _on_stream(stream, ws)
    off = (-ws.data_ptr()) % 256
    return ws[off: off + nbytes], nbytes


def _stream_ptr(stream, device):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t, what, dtypes):
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if t.dtype not in dtypes:
        raise TypeError(f"{what} must have dtype in {dtypes}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr()) if t.numel() else ctypes.c_void_p(0)


def _rep(report):
    return GsReport() if report else None


def _rep_ptr(r):
    return ctypes.byref(r) if r is not None else ctypes.POINTER(GsReport)()


TARGETS = {"AscLeft": 0, "AscRight": 1, "DescLeft": 2, "DescRight": 3}


def _target(target) -> int:
    if isinstance(target, str):
        return TARGETS[target]
    return int(target)


def gs_sort_f64(keys, buffer_fraction: float = 0.5, workspace=None, stream=None, report=False,
                target="AscLeft", algo="auto", sub_fraction: float = 0.5):
    """Stable in-place sort of a contiguous float64 device tensor; target one
    of AscLeft (default), AscRight, DescLeft, DescRight; algo one of auto,
    frogsort1, frogsort2, frogsort3, frogsort6 (sub_fraction: Frogsort6's
    sub-tree fraction)."""
    torch = _torch()
    kp = _dev_ptr(keys, "keys", (torch.float64,))
    n = keys.numel()
    need = gs_workspace_bytes_f64(n, buffer_fraction, algo, sub_fraction)
    if need == SIZE_MAX:
        need = 0
    ws, wsb = _workspace(need, keys.device, workspace, stream)
    r = _rep(report)
    st = _lib.gs_sort_f64_ex(kp, n, _target(target), buffer_fraction, _algo(algo), sub_fraction,
                             ctypes.c_void_p(ws.data_ptr()) if ws is not None else None, wsb,
                             _stream_ptr(stream, keys.device), _rep_ptr(r))
    _check(st, "gs_sort_f64")
    return r.as_dict() if r is not None else None


NOALLOC_MAX_KEYS = 1 << 22


def gs_sort_f64_noalloc(keys, stream=None):
    """gs_sort_f64 at buffer fraction 0.5 with the library's static device
    workspace: no allocation at all (at most NOALLOC_MAX_KEYS keys; calls
    that can overlap on one device race)."""
    torch = _torch()
    kp = _dev_ptr(keys, "keys", (torch.float64,))
    st = _lib.gs_sort_f64_noalloc(kp, keys.numel(), _stream_ptr(stream, keys.device))
    _check(st, "gs_sort_f64_noalloc")


def gs_sort_kv(keys, vals, buffer_fraction: float = 0.5, workspace=None, stream=None, report=False,
               target="AscLeft", algo="auto", sub_fraction: float = 0.5):
    """Stable in-place sort of 64-bit keys (int64 or uint64 storage, compared
    as unsigned) carrying 32-bit values (int32 or uint32 storage); target as
    for gs_sort_f64."""
    torch = _torch()
    k64 = tuple(d for d in (torch.int64, getattr(torch, "uint64", None)) if d is not None)
    v32 = tuple(d for d in (torch.int32, getattr(torch, "uint32", None)) if d is not None)
    kp = _dev_ptr(keys, "keys", k64)
    vp = _dev_ptr(vals, "vals", v32)
    if keys.numel() != vals.numel():
        raise ValueError("keys and vals differ in length")
    n = keys.numel()
    need = gs_workspace_bytes_kv(n, buffer_fraction, algo, sub_fraction)
    if need == SIZE_MAX:
        need = 0
    ws, wsb = _workspace(need, keys.device, workspace, stream)
    r = _rep(report)
    st = _lib.gs_sort_kv_ex(kp, vp, n, _target(target), buffer_fraction, _algo(algo), sub_fraction,
                            ctypes.c_void_p(ws.data_ptr()) if ws is not None else None, wsb,
                            _stream_ptr(stream, keys.device), _rep_ptr(r))
    _check(st, "gs_sort_kv")
    return r.as_dict() if r is not None else None


def gs_seg_configs():
    """Every segmented-sort shape the tuner tries, as dicts (the first is the
    default)."""
    out = []
    for i in range(_lib.gs_seg_config_count()):
        c = GsSegConfig()
        _check(_lib.gs_seg_config_get(i, ctypes.byref(c)), "gs_seg_config_get")
        out.append(c.as_dict())
    return out


def _seg_config(config):
    if config is None:
        return None
    c = GsSegConfig()
    c.short_threads, c.short_ipt, c.merge_ipt = (int(config[k]) for k in
                                                 ("short_threads", "short_ipt", "merge_ipt"))
    return c


def gs_segsort(keys, offsets, buffer_fraction: float = 0.5, workspace=None, stream=None,
               report=False, config=None):
    """Sort every segment keys[offsets[i]:offsets[i+1]] of a float64 device
    tensor in place; offsets is an int64 device tensor of num_segments+1.
    config: a shape from gs_seg_configs() / gs_segsort_autotune (None: the
    default)."""
    torch = _torch()
    kp = _dev_ptr(keys, "keys", (torch.float64,))
    op = _dev_ptr(offsets, "offsets", (torch.int64,))
    nseg = max(offsets.numel() - 1, 0)
    n = keys.numel()
    cfg = _seg_config(config)
    need = gs_workspace_bytes_seg(n, nseg, buffer_fraction)
    if need == SIZE_MAX:
        need = 0
    ws, wsb = _workspace(need, keys.device, workspace, stream)
    r = _rep(report)
    st = _lib.gs_segsort_ex(kp, n, op, nseg, buffer_fraction,
                            ctypes.byref(cfg) if cfg is not None else None,
                            ctypes.c_void_p(ws.data_ptr()) if ws is not None else None, wsb,
                            _stream_ptr(stream, keys.device), _rep_ptr(r))
    _check(st, "gs_segsort")
    return r.as_dict() if r is not None else None


def gs_segsort_autotune(keys, offsets, reps: int = 2, workspace=None, scratch=None, stream=None):
    """Time every segmented-sort shape on these keys (left unchanged; the runs
    sort copies in `scratch`) and return (fastest shape, {shape index: ms})."""
    torch = _torch()
    kp = _dev_ptr(keys, "keys", (torch.float64,))
    op = _dev_ptr(offsets, "offsets", (torch.int64,))
    nseg = max(offsets.numel() - 1, 0)
    n = keys.numel()
    need = gs_workspace_bytes_seg(n, nseg, 0.5)
    if need == SIZE_MAX:
        need = 0
    ws, wsb = _workspace(need, keys.device, workspace, stream)
    if scratch is None:
        scratch = torch.empty_like(keys)
        _on_stream(stream, scratch)
    count = _lib.gs_seg_config_count()
    times = (ctypes.c_float * count)()
    best = GsSegConfig()
    st = _lib.gs_segsort_autotune(kp, n, op, nseg, ctypes.c_void_p(scratch.data_ptr()),
                                  ctypes.c_void_p(ws.data_ptr()) if ws is not None else None, wsb,
                                  _stream_ptr(stream, keys.device), reps, ctypes.byref(best), times)
    _check(st, "gs_segsort_autotune")
    return best.as_dict(), {i: float(times[i]) for i in range(count)}


def gs_learned_sort(keys, params: GsLearnedParams | None = None, workspace=None, stream=None,
                    report=False, **overrides):
    """Stable ascending in-place sort of a float64 device tensor through the
    learned CDF bucket path (same result as gs_sort_f64)."""
    torch = _torch()
    kp = _dev_ptr(keys, "keys", (torch.float64,))
    p = params if params is not None else gs_learned_default_params()
    for k, v in overrides.items():
        setattr(p, k, v)
    n = keys.numel()
    need = gs_workspace_bytes_learned(n, p)
    if need == SIZE_MAX:
        need = 0
    ws, wsb = _workspace(need, keys.device, workspace, stream)
    r = _rep(report)
    st = _lib.gs_learned_sort(kp, n, ctypes.byref(p),
                              ctypes.c_void_p(ws.data_ptr()) if ws is not None else None, wsb,
                              _stream_ptr(stream, keys.device), _rep_ptr(r))
    _check(st, "gs_learned_sort")
    return r.as_dict() if r is not None else None


# ---------------------------------------------------------------------------
# device-side failures
# ---------------------------------------------------------------------------
GS_DEVERR_WAIT = 1
GS_DEVERR_OFFSETS = 2


def gs_copy_f64(src, dst, stream=None):
    """Streaming copy of a float64 device tensor into another of the same size
    (the bandwidth ceiling a sorting pass is measured against)."""
    torch = _torch()
    sp = _dev_ptr(src, "src", (torch.float64,))
    dp = _dev_ptr(dst, "dst", (torch.float64,))
    if src.numel() != dst.numel():
        raise ValueError("src and dst differ in size")
    _check(_lib.gs_copy_f64(sp, dp, src.numel(), _stream_ptr(stream, src.device)), "gs_copy_f64")


def gs_device_errors(device=0, clear=False) -> int:
    """The device's sticky failure flags (GS_DEVERR_*) of every call so far;
    synchronise the calls' streams first."""
    flags = ctypes.c_uint32(0)
    _check(_lib.gs_device_errors(int(device), ctypes.byref(flags), 1 if clear else 0), "gs_device_errors")
    return int(flags.value)


def gs_test_fail_waits(on: bool) -> bool:
    """Test hook: record every ordered-store wait as failed (the waits still
    complete, the output stays correct); returns the previous setting."""
    return bool(_lib.gs_test_fail_waits(1 if on else 0))


# ---------------------------------------------------------------------------
# the CDF network on its own (float32 device tensors)
# ---------------------------------------------------------------------------
def _f32(t, what):
    torch = _torch()
    return _dev_ptr(t, what, (torch.float32,))


def gs_mlp_loss_grad(params, u, t, stream=None):
    """(loss tensor [1], grad tensor [4353]) of the network on a batch."""
    torch = _torch()
    batch = u.numel()
    grad = torch.empty(MLP_NUM_PARAMS, dtype=torch.float32, device=params.device)
    loss = torch.empty(1, dtype=torch.float32, device=params.device)
    work = torch.empty((batch // 32 + 1) * (MLP_NUM_PARAMS + 1), dtype=torch.float32, device=params.device)
    _on_stream(stream, grad, loss, work)
    st = _lib.gs_mlp_loss_grad(_f32(params, "params"), _f32(u, "u"), _f32(t, "t"), batch,
                               _f32(grad, "grad"), _f32(loss, "loss"), _f32(work, "work"),
                               work.numel() * 4, _stream_ptr(stream, params.device))
    _check(st, "gs_mlp_loss_grad")
    return loss, grad


def gs_mlp_train(params, adam_m, adam_v, u, t, steps, batch, lr, seed=0, full_batch=False,
                 stream=None):
    """In-place Adam training; returns a [2] tensor (first, last step loss)."""
    torch = _torch()
    losses = torch.zeros(2, dtype=torch.float32, device=params.device)
    work = torch.empty((batch // 32) * (MLP_NUM_PARAMS + 1) + 64, dtype=torch.float32,
                       device=params.device)
    _on_stream(stream, losses, work)
    st = _lib.gs_mlp_train(_f32(params, "params"), _f32(adam_m, "m"), _f32(adam_v, "v"),
                           _f32(u, "u"), _f32(t, "t"), u.numel(), steps, batch, lr, seed,
                           1 if full_batch else 0, _f32(losses, "losses"), _f32(work, "work"),
                           work.numel() * 4, _stream_ptr(stream, params.device))
    _check(st, "gs_mlp_train")
    return losses


def gs_mlp_forward(params, u, stream=None):
    torch = _torch()
    y = torch.empty_like(u)
    _on_stream(stream, y)
    st = _lib.gs_mlp_forward(_f32(params, "params"), _f32(u, "u"), u.numel(), _f32(y, "y"),
                             _stream_ptr(stream, params.device))
    _check(st, "gs_mlp_forward")
    return y
