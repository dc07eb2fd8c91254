"""CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it, and the
two share no code.  The C source is ``oracle.c``; this module compiles it with
gcc into ``liboracle.so`` next to it and wraps it with ctypes.  ``stdsort.cpp``
(g++, ``libstdsort.so``) holds a second reference: the C++ standard library's
stable sort under the same key order.

Every function computes what the paper's definition of sorting fixes (stable,
ascending, ties in input order) by the plainest available route; see the header
comment of ``oracle.c`` for the section each part follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_STD_SRC = os.path.join(_HERE, "stdsort.cpp")
_STD_LIB = os.path.join(_HERE, "libstdsort.so")
_lib = None
_stdlib = None

MLP_HIDDEN = 64
MLP_NUM_PARAMS = 4353


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` with gcc (fp64, no fast-math) and ``stdsort.cpp``
    with g++."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-std=c11",
             "-shared", "-fPIC", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    if force or not os.path.exists(_STD_LIB):
        tmp = _STD_LIB + ".tmp"
        subprocess.check_call(
            ["g++", "-O2", "-fno-fast-math", "-std=c++17", "-shared", "-fPIC", "-Wall", "-Wextra",
             "-o", tmp, _STD_SRC])
        os.replace(tmp, _STD_LIB)
    return _LIB


def _load_std():
    global _stdlib
    if _stdlib is not None:
        return _stdlib
    if not os.path.exists(_STD_LIB) or os.path.getmtime(_STD_LIB) < os.path.getmtime(_STD_SRC):
        build(force=True)
    lib = ctypes.CDLL(_STD_LIB)
    lib.stdsort_stable_f64.argtypes = [ctypes.c_void_p, ctypes.c_int64]
    lib.stdsort_stable_f64.restype = None
    lib.stdsort_stable_kv.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
    lib.stdsort_stable_kv.restype = None
    _stdlib = lib
    return lib


def std_stable_sort_f64(x: np.ndarray) -> np.ndarray:
    """std::stable_sort of a copy of x under the oracle's key order."""
    y = np.ascontiguousarray(x, dtype=np.float64).copy()
    _load_std().stdsort_stable_f64(y.ctypes.data, y.size)
    return y


def std_stable_sort_kv(k: np.ndarray, v: np.ndarray):
    """std::stable_sort of copies of (k, v) by unsigned key."""
    kk = np.ascontiguousarray(k, dtype=np.uint64).copy()
    vv = np.ascontiguousarray(v, dtype=np.uint32).copy()
    _load_std().stdsort_stable_kv(kk.ctypes.data, vv.ctypes.data, kk.size)
    return kk, vv


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    lib.oracle_less_f64.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.oracle_less_f64.restype = ctypes.c_int
    lib.oracle_sort_f64.argtypes = [P, I64]
    lib.oracle_sort_f64.restype = ctypes.c_int
    lib.oracle_sort_kv.argtypes = [P, P, I64]
    lib.oracle_sort_kv.restype = ctypes.c_int
    lib.oracle_sort_f64_target.argtypes = [P, I64, ctypes.c_int]
    lib.oracle_sort_f64_target.restype = ctypes.c_int
    lib.oracle_sort_kv_target.argtypes = [P, P, I64, ctypes.c_int]
    lib.oracle_sort_kv_target.restype = ctypes.c_int
    lib.oracle_segsort_f64.argtypes = [P, P, I64]
    lib.oracle_segsort_f64.restype = ctypes.c_int
    lib.oracle_segsort_kv.argtypes = [P, P, P, I64]
    lib.oracle_segsort_kv.restype = ctypes.c_int
    lib.oracle_rank_f64.argtypes = [P, I64, P, I64, P]
    lib.oracle_rank_f64.restype = None
    lib.oracle_rank_u64.argtypes = [P, I64, P, I64, P]
    lib.oracle_rank_u64.restype = None
    lib.oracle_frog_model.argtypes = [P, I64, ctypes.c_int, P, P, P, P, I64, P]
    lib.oracle_frog_model.restype = I64
    lib.oracle_squid_model.argtypes = [P, I64, ctypes.c_int, P, P, P]
    lib.oracle_squid_model.restype = I64
    lib.oracle_frog_geometry.argtypes = [I64, ctypes.c_int, P]
    lib.oracle_frog_geometry.restype = I64
    lib.oracle_frog2_model.argtypes = [P, I64, I64, I64, I64, P, P, P, P, I64, P, I64, P, I64, P]
    lib.oracle_frog2_model.restype = I64
    lib.oracle_frog3_model.argtypes = [P, I64, I64, I64, I64, I64, P, P, P, I64, P, I64, P, I64, P, I64, P]
    lib.oracle_frog3_model.restype = I64
    lib.oracle_mlp_num_params.argtypes = []
    lib.oracle_mlp_num_params.restype = ctypes.c_int
    lib.oracle_mlp_forward.argtypes = [P, P, I64, P]
    lib.oracle_mlp_forward.restype = None
    lib.oracle_mlp_loss_grad.argtypes = [P, P, P, I64, P]
    lib.oracle_mlp_loss_grad.restype = ctypes.c_double
    lib.oracle_adam_step.argtypes = [P, P, P, P, I64, I64, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_double]
    lib.oracle_adam_step.restype = None
    assert lib.oracle_mlp_num_params() == MLP_NUM_PARAMS
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


def less_f64(a: float, b: float) -> bool:
    """The comparison every f64 result is defined by (NaN last, -0 == +0)."""
    return bool(_load().oracle_less_f64(float(a), float(b)))


def sort_f64(x: np.ndarray) -> np.ndarray:
    """Stable ascending sort of float64 keys; returns a new array."""
    y = np.array(x, dtype=np.float64, copy=True, order="C")
    if _load().oracle_sort_f64(_ptr(y), y.size) != 0:
        raise MemoryError("oracle_sort_f64: allocation failed")
    return y


def sort_kv(keys: np.ndarray, vals: np.ndarray):
    """Stable ascending sort of uint64 keys carrying uint32 values."""
    k = np.array(keys, dtype=np.uint64, copy=True, order="C")
    v = np.array(vals, dtype=np.uint32, copy=True, order="C")
    if k.shape != v.shape:
        raise ValueError("keys and vals differ in shape")
    if _load().oracle_sort_kv(_ptr(k), _ptr(v), k.size) != 0:
        raise MemoryError("oracle_sort_kv: allocation failed")
    return k, v


TARGETS = {"AscLeft": 0, "AscRight": 1, "DescLeft": 2, "DescRight": 3}


def sort_f64_target(x: np.ndarray, target: str) -> np.ndarray:
    """One of the four stable targets ("Definition of sorting"): ascending or
    descending keys, ties in input order (Left) or reverse input order
    (Right); returns a new array."""
    y = np.array(x, dtype=np.float64, copy=True, order="C")
    if _load().oracle_sort_f64_target(_ptr(y), y.size, TARGETS[target]) != 0:
        raise MemoryError("oracle_sort_f64_target failed")
    return y


def sort_kv_target(keys: np.ndarray, vals: np.ndarray, target: str):
    k = np.array(keys, dtype=np.uint64, copy=True, order="C")
    v = np.array(vals, dtype=np.uint32, copy=True, order="C")
    if k.shape != v.shape:
        raise ValueError("keys and vals differ in shape")
    if _load().oracle_sort_kv_target(_ptr(k), _ptr(v), k.size, TARGETS[target]) != 0:
        raise MemoryError("oracle_sort_kv_target failed")
    return k, v


def segsort_f64(x: np.ndarray, offsets: np.ndarray) -> np.ndarray:
    """Sort every segment x[offsets[i]:offsets[i+1]] on its own."""
    y = np.array(x, dtype=np.float64, copy=True, order="C")
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    if off.size and off[-1] > y.size:
        raise ValueError("offsets beyond the array")
    rc = _load().oracle_segsort_f64(_ptr(y), _ptr(off), max(off.size - 1, 0))
    if rc == -2:
        raise ValueError("offsets must be non-decreasing and start at >= 0")
    if rc != 0:
        raise MemoryError("oracle_segsort_f64: allocation failed")
    return y


def segsort_kv(keys: np.ndarray, vals: np.ndarray, offsets: np.ndarray):
    k = np.array(keys, dtype=np.uint64, copy=True, order="C")
    v = np.array(vals, dtype=np.uint32, copy=True, order="C")
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    if off.size and off[-1] > k.size:
        raise ValueError("offsets beyond the array")
    rc = _load().oracle_segsort_kv(_ptr(k), _ptr(v), _ptr(off), max(off.size - 1, 0))
    if rc == -2:
        raise ValueError("offsets must be non-decreasing and start at >= 0")
    if rc != 0:
        raise MemoryError("oracle_segsort_kv: allocation failed")
    return k, v


def rank_f64(x: np.ndarray, idx) -> np.ndarray:
    """Output position of each x[idx[q]] under the stable ascending definition."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.zeros(idx.size, dtype=np.int64)
    _load().oracle_rank_f64(_ptr(x), x.size, _ptr(idx), idx.size, _ptr(out))
    return out


def rank_u64(x: np.ndarray, idx) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.uint64)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.zeros(idx.size, dtype=np.int64)
    _load().oracle_rank_u64(_ptr(x), x.size, _ptr(idx), idx.size, _ptr(out))
    return out


def frog_model(keys: np.ndarray, g: int = 1, max_snap: int = 0):
    """Run the instrumented Frogsort model (g=1: Frogsort1, g=2: Frogsort0
    triplets) as a top-level left node.

    Returns a dict with the sorted keys, the input index of every output
    element, the slot labels after setup, the label snapshots taken after every
    merge (and, for g=2, every triplet), and the comparison/move counts.
    """
    keys = np.ascontiguousarray(keys, dtype=np.float64)
    n = keys.size
    if n % g:
        raise ValueError("n must be a multiple of g")
    u = n // g
    nslots = n + n // 2
    out_k = np.zeros(n, dtype=np.float64)
    out_l = np.zeros(n, dtype=np.int64)
    setup = np.zeros(max(nslots, 1), dtype=np.int64)
    trace = np.zeros((max(max_snap, 1), max(nslots, 1)), dtype=np.int64)
    counts = np.zeros(3, dtype=np.int64)
    ns = _load().oracle_frog_model(_ptr(keys), u, g, _ptr(out_k), _ptr(out_l),
                                   _ptr(setup), _ptr(trace), max_snap, _ptr(counts))
    if ns < 0:
        raise MemoryError("oracle_frog_model: allocation failed")
    return {
        "keys": out_k, "labels": out_l, "setup": setup[:nslots],
        "trace": trace[: int(counts[2]), :nslots], "compares": int(counts[0]),
        "moves": int(counts[1]), "nslots": int(ns),
    }


SQUID_NONE, SQUID_ASC, SQUID_DESC = 0, 1, 2


def squid_model(keys: np.ndarray, mode: int = 0):
    """Run the instrumented Squidsort1 model (one element per leaf).

    Returns (sorted keys, input index of each output, counts) with counts a
    dict: merge_cmp, test_cmp, moves (merges and concatenations), rev_moves
    (final reversal), top_dir (SQUID_*), overwrites (writes over unread
    elements).  mode 1 enforces ascending at every merge (the literal
    reading; shows why the model merges in the outer run's direction); mode 2
    turns a descending outer run around in place before an ascending merge
    (the rule the GPU path runs)."""
    lib = _load()
    x = np.ascontiguousarray(keys, dtype=np.float64)
    n = x.size
    out = np.zeros(n, dtype=np.float64)
    lab = np.zeros(n, dtype=np.int64)
    c = np.zeros(6, dtype=np.int64)
    r = lib.oracle_squid_model(_ptr(x), n, int(mode), _ptr(out), _ptr(lab), _ptr(c))
    if r < 0:
        raise MemoryError("oracle_squid_model")
    names = ("merge_cmp", "test_cmp", "moves", "rev_moves", "top_dir", "overwrites")
    return out, lab, {k: int(v) for k, v in zip(names, c)}


def frog_geometry(n: int, depth: int) -> np.ndarray:
    """Nodes of the Frogsort1 tree at `depth` (left to right), each as
    (region start, data size, is_left, data start, input offset)."""
    out = np.zeros((1 << depth, 5), dtype=np.int64)
    k = _load().oracle_frog_geometry(n, depth, _ptr(out))
    return out[:k]


def frog2_fraction_q(p: float) -> int:
    """The fraction p as q / 65536, rounded down (so the buffer never exceeds
    p of the data): the reading the Frogsort2 model and the library share."""
    return int(np.floor(float(p) * 65536.0))


def frog2_model(keys, q: int, leaf_max: int, max_snap: int = 0, gap_shrink: int = 0):
    """Run the instrumented Frogsort2 model (inner child floor(q*n/65536),
    leaves of at most leaf_max elements) as a top-level left node.  With keys
    None only the geometry is walked.

    Returns a dict with the sorted keys and their input indices, the slot
    labels after setup, the label snapshots after every merge, the leaves
    (input offset, data start, length) in input order, the merge nodes
    (region start, n, is_left, height) in post order, the comparison / move
    counts, the slot count and the violation bits."""
    geo_only = keys is None
    if geo_only:
        raise ValueError("use frog2_geometry")
    keys = np.ascontiguousarray(keys, dtype=np.float64)
    return _frog2(keys, keys.size, q, leaf_max, max_snap, gap_shrink)


def frog2_geometry(n: int, q: int, leaf_max: int):
    """Leaves and merge nodes of the Frogsort2 tree over n elements (see
    frog2_model), without moving any data."""
    return _frog2(None, int(n), q, leaf_max, 0, 0)


def _frog2(keys, n, q, leaf_max, max_snap, gap_shrink):
    lib = _load()
    counts = np.zeros(6, dtype=np.int64)
    # first pass: sizes only
    lib.oracle_frog2_model(None, n, q, leaf_max, gap_shrink, None, None, None, None, 0,
                           None, 0, None, 0, _ptr(counts))
    nl, nn = int(counts[3]), int(counts[4])
    leaves = np.zeros((max(nl, 1), 3), dtype=np.int64)
    nodes = np.zeros((max(nn, 1), 4), dtype=np.int64)
    nslots = n + (n * q) // 65536 if n > 0 else 0
    nslots = max(nslots - gap_shrink, n)
    res = {"n": n}
    if keys is None:
        ns = lib.oracle_frog2_model(None, n, q, leaf_max, gap_shrink, None, None, None, None, 0,
                                    _ptr(leaves), nl, _ptr(nodes), nn, _ptr(counts))
    else:
        out_k = np.zeros(max(n, 1), dtype=np.float64)
        out_l = np.zeros(max(n, 1), dtype=np.int64)
        setup = np.zeros(max(nslots, 1), dtype=np.int64)
        trace = np.zeros((max(max_snap, 1), max(nslots, 1)), dtype=np.int64)
        ns = lib.oracle_frog2_model(_ptr(keys), n, q, leaf_max, gap_shrink, _ptr(out_k), _ptr(out_l),
                                    _ptr(setup), _ptr(trace), max_snap, _ptr(leaves), nl,
                                    _ptr(nodes), nn, _ptr(counts))
        if ns < 0:
            raise MemoryError("oracle_frog2_model: allocation failed")
        res.update(keys=out_k[:n], labels=out_l[:n], setup=setup[:ns],
                   trace=trace[: int(counts[2]), :ns])
    res.update(leaves=leaves[:nl], nodes=nodes[:nn], compares=int(counts[0]), moves=int(counts[1]),
               nslots=int(ns), bad=int(counts[5]))
    return res


def frog3_model(keys, q: int, leaf_max: int, gap_shrink: int = 0, q2: int = 32768):
    """Run the instrumented Frogsort3 model (shared buffer floor(q*n/65536),
    sub-trees with leaves of at most leaf_max elements: Frogsort1 for
    q2 = 32768, Frogsort2 at q2 / 65536 otherwise, i.e. Frogsort6) in place on
    keys; keys None walks the geometry only.

    Returns a dict with the sorted keys and their input indices, the leaves
    (input offset, data start, length) in placement order, the merge nodes of
    the Frogsort1 trees (region start, n, is_left, height), the spine merges
    (outer elements, inner start, inner elements) bottom up, the Frogsort1
    trees in running order (region start, n, input offset, is_left), the merge
    comparison / move counts, the slot count and the violation bits."""
    lib = _load()
    n = 0 if keys is None else np.asarray(keys).size
    return _frog3(lib, keys, n, q, leaf_max, gap_shrink, q2)


def frog3_geometry(n: int, q: int, leaf_max: int, q2: int = 32768):
    return _frog3(_load(), None, int(n), q, leaf_max, 0, q2)


def _frog3(lib, keys, n, q, leaf_max, gap_shrink, q2):
    counts = np.zeros(7, dtype=np.int64)
    lib.oracle_frog3_model(None, n, q, q2, leaf_max, gap_shrink, None, None, None, 0, None, 0,
                           None, 0, None, 0, _ptr(counts))
    sizes = [int(c) for c in counts]
    leaves = np.zeros((max(sizes[2], 1), 3), dtype=np.int64)
    nodes = np.zeros((max(sizes[3], 1), 4), dtype=np.int64)
    spine = np.zeros((max(sizes[5], 1), 3), dtype=np.int64)
    trees = np.zeros((max(sizes[6], 1), 4), dtype=np.int64)
    res = {"n": n}
    if keys is not None:
        keys = np.ascontiguousarray(keys, dtype=np.float64)
        out_k = np.zeros(max(n, 1), dtype=np.float64)
        out_l = np.zeros(max(n, 1), dtype=np.int64)
        ns = lib.oracle_frog3_model(_ptr(keys), n, q, q2, leaf_max, gap_shrink, _ptr(out_k), _ptr(out_l),
                                    _ptr(leaves), sizes[2], _ptr(nodes), sizes[3], _ptr(spine), sizes[5],
                                    _ptr(trees), sizes[6], _ptr(counts))
        if ns < 0:
            raise MemoryError("oracle_frog3_model: allocation failed")
        res.update(keys=out_k[:n], labels=out_l[:n])
    else:
        ns = lib.oracle_frog3_model(None, n, q, q2, leaf_max, gap_shrink, None, None,
                                    _ptr(leaves), sizes[2], _ptr(nodes), sizes[3], _ptr(spine), sizes[5],
                                    _ptr(trees), sizes[6], _ptr(counts))
    res.update(leaves=leaves[: sizes[2]], nodes=nodes[: sizes[3]], spine=spine[: sizes[5]],
               trees=trees[: sizes[6]], compares=int(counts[0]), moves=int(counts[1]),
               nslots=int(ns), bad=int(counts[4]))
    return res


def mlp_forward(params: np.ndarray, u: np.ndarray) -> np.ndarray:
    p = np.ascontiguousarray(params, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    assert p.size == MLP_NUM_PARAMS
    y = np.zeros(u.size, dtype=np.float64)
    _load().oracle_mlp_forward(_ptr(p), _ptr(u), u.size, _ptr(y))
    return y


def mlp_loss_grad(params: np.ndarray, u: np.ndarray, t: np.ndarray, want_grad=True):
    p = np.ascontiguousarray(params, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    t = np.ascontiguousarray(t, dtype=np.float64)
    assert p.size == MLP_NUM_PARAMS and u.size == t.size
    g = np.zeros(MLP_NUM_PARAMS, dtype=np.float64) if want_grad else None
    loss = _load().oracle_mlp_loss_grad(_ptr(p), _ptr(u), _ptr(t), u.size,
                                        _ptr(g) if want_grad else ctypes.c_void_p(0))
    return loss, g


def adam_step(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam update of float64 arrays params, m, v."""
    for a in (params, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = np.ascontiguousarray(grad, dtype=np.float64)
    _load().oracle_adam_step(_ptr(params), _ptr(g), _ptr(m), _ptr(v), params.size,
                             int(step), lr, beta1, beta2, eps)


# parameter slices (same layout as the C code)
def mlp_slices(h: int = MLP_HIDDEN):
    o = 0
    sl = {}
    for name, size in (("W1", h), ("b1", h), ("W2", h * h), ("b2", h), ("w3", h), ("b3", 1)):
        sl[name] = slice(o, o + size)
        o += size
    return sl
