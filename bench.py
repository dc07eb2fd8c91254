#!/usr/bin/env python3
"""Benchmark: stable float64 sort of n = 2^28 keys on one MI355X.

One step = one call of gs_sort_f64 (leaf sort + every frog merge level) over
one resident 2 GiB array of synthetic keys.  Each timed step sorts its own
pre-made copy of the input, so the timed region holds nothing but sorting.

Prints one JSON line (see the keys below).  Run with --help for options.
"""
from __future__ import annotations

import argparse
import ctypes

import numpy as np
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
METRIC = "Gkeys/s stable f64 sort n=2^28 (learned vs plain merge), %HBM BW, %RAM footprint"
COUNTERS = os.path.join(ROOT, "profiles", "merge_kernel_f64_2p28_uniform_hbm_counters.md")


def merge_traffic():
    """HBM bytes per merge-kernel launch from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE passes, scaled by a copy kernel of known size),
    or None when the merge kernel's sources no longer hash to the value the
    counters were taken on."""
    import hashlib
    try:
        kv = dict(l.split(": ", 1) for l in open(COUNTERS).read().splitlines()
                  if l.startswith(("traffic_bytes_per_launch:", "sources_sha256_16:", "sources:")))
        h = hashlib.sha256()
        for f in kv["sources"].split():
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest()[:16] != kv["sources_sha256_16"].strip():
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def log(msg):
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


def _host():
    """The host the CPU baselines ran on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = None
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline(n_sample: int, pattern: str, full_n: int = 0, full_reps: int = 1):
    """The CPU oracle (single thread) on a bounded contiguous sample, with the
    C++ standard library's stable sort (single thread) on the same sample
    beside it; with full_n, both on the whole input as well, full_reps times
    each (median reported)."""
    import oracle
    import workloads as W

    def timed(fn, x):
        t0 = time.perf_counter()
        fn(x)
        return time.perf_counter() - t0

    x = W.f64_pattern(pattern, n_sample, seed=0)
    dt = timed(oracle.sort_f64, x)
    ds = timed(oracle.std_stable_sort_f64, x)
    del x
    out = {"value": n_sample / dt / 1e9, "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
           "sample": f"{n_sample} keys ({pattern}, seed 0), one single-threaded call of the "
                     f"oracle's stable mergesort, {dt:.2f} s",
           "seconds": dt, "host": _host(),
           "std_stable_sort": {"value": n_sample / ds / 1e9, "unit": "Gkeys/s", "cores": 1,
                               "seconds": ds, "sample": "the same keys, one std::stable_sort call"}}
    if full_n:
        x = W.f64_pattern(pattern, full_n, seed=0)
        dfs, dss = [], []
        for r in range(max(1, full_reps)):
            dfs.append(timed(oracle.sort_f64, x))
            dss.append(timed(oracle.std_stable_sort_f64, x))
            print(f"cpu full input, run {r + 1}: oracle {dfs[-1]:.2f} s, std::stable_sort {dss[-1]:.2f} s",
                  file=sys.stderr, flush=True)
        df = sorted(dfs)[len(dfs) // 2]
        dsf = sorted(dss)[len(dss) // 2]
        out["full_input"] = {"n": full_n, "runs": len(dfs), "oracle_s": df, "oracle_s_all": dfs,
                             "oracle_gkeys_per_s": full_n / df / 1e9, "std_stable_sort_s": dsf,
                             "std_stable_sort_s_all": dss, "std_stable_sort_gkeys_per_s": full_n / dsf / 1e9}
    return out


def _time_calls(torch, stream, fn, reps):
    """Median of `reps` HIP-event timings of fn(i) (input restored outside)."""
    times = []
    for i in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        fn(i, None)
        e0.record(stream)
        fn(i, True)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2]


SECTIONS = ("patterns", "learned", "segmented", "kv", "buffer")
LEARNED_PATTERNS = ("lognormal", "gaussmix", "zipf_ints")
LEARNED_CALLS = ("plain", "learned", "learned_untrained", "learned_sample_table")
KV_PATTERNS = ("uniform", "zipf")
SEG_WORKLOADS = ("100k_arrays", "until_total_16_to_2^20")
SEG_FRACTIONS = (0.25, 0.1, 1 / 64)     # the segmented sort below the half buffer


def extras(gs, torch, W, log2n, dev, sections=SECTIONS, learned_patterns=LEARNED_PATTERNS,
           learned_calls=LEARNED_CALLS, kv_patterns=KV_PATTERNS, seg_workloads=SEG_WORKLOADS,
           seg_per_array=True):
    """Side measurements on the same device: the plain sort on the other input
    patterns, the learned path against the plain path on the learned
    workloads, the segmented sort against per-array plain calls, the
    key-value sort and the smaller buffers.  Medians of a few HIP-event timed
    reps.  `sections` (and the learned filters) choose a subset, e.g. to
    profile one workload on its own."""
    stream = torch.cuda.current_stream(dev)
    n = 1 << log2n
    res = {}
    if "patterns" in sections:
        res["plain_patterns"] = _extras_patterns(gs, torch, W, n, dev, stream)
    if "learned" in sections:
        res["learned_vs_plain"] = _extras_learned(gs, torch, W, n, dev, stream, learned_patterns, learned_calls)
    if "segmented" in sections:
        res["segmented"] = _extras_segmented(gs, torch, W, n, dev, stream, seg_workloads, seg_per_array)
    if "kv" in sections:
        res["key_value"] = _extras_kv(gs, torch, W, log2n, dev, stream, kv_patterns)
    if "buffer" in sections:
        res["buffer_fraction"] = _extras_buffer(gs, torch, W, n, dev, stream)
    return res


def _extras_patterns(gs, torch, W, n, dev, stream):
    """The plain sort on the other input patterns of the same size."""
    pats = {}
    need = gs.gs_workspace_bytes_f64(n)
    ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    ws = ws[(-ws.data_ptr()) % 256:][:need]
    # the build's own patterns, then the paper's ("Methods and measurement")
    plan = [(p, lambda p=p: W.f64_pattern(p, n, seed=0)) for p in ("tied", "presorted", "reversed", "perturbed")]
    plan += [(p, lambda p=p: W.paper_pattern(p, n, seed=0)) for p in W.PAPER_PATTERNS]
    for pat, make in plan:
        log(f"extras: plain {pat}")
        x = torch.from_numpy(make()).to(dev)
        buf = torch.empty_like(x)

        def fn_p(i, timed):
            if timed is None:
                buf.copy_(x)
            else:
                gs.gs_sort_f64(buf, workspace=ws)
        rep = gs.gs_sort_f64(buf.copy_(x), workspace=ws, report=True)
        ms = _time_calls(torch, stream, fn_p, 3)
        # element moves of the call (16 B per move: one 8-byte read and one
        # 8-byte write), against the 16n(levels+1) of a sort that merges
        # every level in full
        moved = int(rep["keys_moved"])
        pats[pat] = {"ms": round(ms, 3), "gkeys_per_s": round(n / (ms * 1e-3) / 1e9, 3),
                     "keys_moved": moved, "moved_bytes_gb": round(16.0 * moved / 1e9, 3),
                     "moves_vs_full_merge": round(moved / (n * (rep["levels"] + 1)), 4),
                     "order": int(rep["order"])}
        del x, buf
    del ws
    return pats


def _extras_learned(gs, torch, W, n, dev, stream, patterns, calls):
    """Learned vs plain on the learned workloads."""
    every = {"plain": lambda b: gs.gs_sort_f64(b),
             "learned": lambda b: gs.gs_learned_sort(b),
             "learned_untrained": lambda b: gs.gs_learned_sort(b, mode=1),
             "learned_sample_table": lambda b: gs.gs_learned_sort(b, mode=2)}
    lr = {}
    for pat in patterns:
        log(f"extras: learned {pat}")
        x = torch.from_numpy(W.learned_pattern(pat, n, seed=0)).to(dev)
        buf = torch.empty_like(x)
        row = {}
        for name in calls:
            call = every[name]

            def fn(i, timed, call=call):
                if timed is None:
                    buf.copy_(x)
                else:
                    call(buf)
            call(buf)                                  # warm-up (and workspace)
            ms = _time_calls(torch, stream, fn, 3)
            row[name] = {"ms": round(ms, 3), "gkeys_per_s": round(n / (ms * 1e-3) / 1e9, 3)}
        buf.copy_(x)
        rep = gs.gs_learned_sort(buf, report=True)
        row["learned_report"] = {k: rep[k] for k in ("fallback", "max_bucket", "overflow_buckets",
                                                    "train_loss_first", "train_loss_last", "feature",
                                                    "heavy_values")}
        row["learned_sorted"] = bool((buf[1:] >= buf[:-1]).all().item())
        lr[pat] = row
        del x, buf
    return lr


def _extras_segmented(gs, torch, W, n, dev, stream, workloads, per_array):
    """Segmented: 100,000 arrays, log-uniform lengths rescaled to total n,
    mixed patterns; and lengths log-uniform in [16, 2^20] drawn until n."""
    segres = {}
    shapes = {"100k_arrays": (100_000, 16, 19023), "until_total_16_to_2^20": (None, 16, 1 << 20)}
    for name in workloads:
        nseg, lo, hi = shapes[name]
        log(f"extras: segmented {name}")
        xs, off = W.segmented(nseg, lo, hi, seed=0, total=n)
        nseg = off.size - 1
        x = torch.from_numpy(xs).to(dev)
        o = torch.from_numpy(off).to(dev)
        buf = torch.empty_like(x)
        need = gs.gs_workspace_bytes_seg(n, nseg)
        ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
        ws = ws[(-ws.data_ptr()) % 256:][:need]
        best, times = gs.gs_segsort_autotune(x, o, reps=2, workspace=ws, scratch=buf)

        def timed(cfg):
            def fn_seg(i, t):
                if t is None:
                    buf.copy_(x)
                else:
                    gs.gs_segsort(buf, o, workspace=ws, config=cfg)
            gs.gs_segsort(buf.copy_(x), o, workspace=ws, config=cfg)
            return _time_calls(torch, stream, fn_seg, 3)
        ms_default = timed(gs.gs_seg_configs()[0])   # (no shape would now take the tuned one)
        ms_best = timed(best)
        # the tuned call captured once in a HIP graph and replayed
        side = torch.cuda.Stream(dev)
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            gs.gs_segsort(buf.copy_(x), o, workspace=ws, config=best, stream=side)
        stream.wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=side):
            gs.gs_segsort(buf, o, workspace=ws, config=best, stream=side)

        def fn_graph(i, t):
            if t is None:
                buf.copy_(x)
            else:
                graph.replay()
        ms_graph = _time_calls(torch, stream, fn_graph, 3)
        # smaller buffers: one buffer serving runs of segments in turn
        fractions = {}
        for frac in SEG_FRACTIONS:
            need_f = gs.gs_workspace_bytes_seg(n, nseg, frac)
            ws_f = torch.empty(need_f + 256, dtype=torch.uint8, device=dev)
            ws_f = ws_f[(-ws_f.data_ptr()) % 256:][:need_f]

            def fn_frac(i, t, ws_f=ws_f, frac=frac):
                if t is None:
                    buf.copy_(x)
                else:
                    gs.gs_segsort(buf, o, buffer_fraction=frac, workspace=ws_f)
            gs.gs_segsort(buf.copy_(x), o, buffer_fraction=frac, workspace=ws_f)
            ms_f = _time_calls(torch, stream, fn_frac, 3)
            rep_f = gs.gs_segsort(buf.copy_(x), o, buffer_fraction=frac, workspace=ws_f, report=True)
            fractions[f"{frac:.4g}"] = {"ms": round(ms_f, 3), "ram_fraction": round(rep_f["ram_fraction"], 5),
                                        "steps": int(gs.plan_seg_steps(off, n, frac)[0].shape[0])}
            del ws_f
        buf.copy_(x)
        graph.replay()
        torch.cuda.synchronize()
        ok = True
        for k in range(0, nseg, max(1, nseg // 50)):
            seg = buf[int(off[k]):int(off[k + 1])]
            if seg.numel() > 1 and not bool((seg[1:] >= seg[:-1]).all().item()):
                ok = False
        del graph
        row = {
            "arrays": nseg, "keys": n, "min_len": int(np.diff(off).min()), "max_len": int(np.diff(off).max()),
            "ms_default_shape": round(ms_default, 3), "ms_tuned": round(ms_best, 3),
            "ms_tuned_graph": round(ms_graph, 3),
            "gkeys_per_s_tuned": round(n / (ms_best * 1e-3) / 1e9, 3),
            "tuned_shape": best, "shape_ms": {str(i): round(v, 3) for i, v in times.items()},
            "buffer_fractions": fractions, "sorted_spot_check": ok}
        segres[name] = row
        if not per_array:
            del x, buf, o, ws
            continue
        # one plain call per array, every array
        k = nseg
        sub = [buf[int(off[i]):int(off[i + 1])] for i in range(k)]
        wsmax = max(gs.gs_workspace_bytes_f64(t.numel()) for t in sub)
        ws1 = torch.empty(wsmax + 256, dtype=torch.uint8, device=dev)
        ws1 = ws1[(-ws1.data_ptr()) % 256:][:wsmax]

        def fn_each(i, t):
            if t is None:
                buf.copy_(x)
            else:
                for a in sub:
                    if a.numel() > 1:
                        gs.gs_sort_f64(a, workspace=ws1[: gs.gs_workspace_bytes_f64(a.numel())])
        ms_each = _time_calls(torch, stream, fn_each, 1)
        row["per_array_launches_ms"] = round(ms_each, 1)
        row["per_array_note"] = f"{k} separate gs_sort_f64 calls, one per array, timed together"
        del x, buf, o, sub, ws, ws1
    return segres


def _extras_kv(gs, torch, W, log2n, dev, stream, patterns):
    """Key-value: 2^(log2n+1) uint64 keys with uint32 payload."""
    log("extras: key-value")
    nk = 1 << (log2n + 1)
    kv = {}
    for pat in patterns:
        k0, v0 = W.kv_pattern(pat, nk, seed=0)
        K = torch.from_numpy(k0.view(np.int64)).to(dev)
        V = torch.from_numpy(v0.view(np.int32)).to(dev)
        Kb, Vb = torch.empty_like(K), torch.empty_like(V)

        def fn_kv(i, timed):
            if timed is None:
                Kb.copy_(K)
                Vb.copy_(V)
            else:
                gs.gs_sort_kv(Kb, Vb)
        gs.gs_sort_kv(Kb.copy_(K), Vb.copy_(V))
        ms = _time_calls(torch, stream, fn_kv, 3)
        kv[pat] = {"n": nk, "ms": round(ms, 3), "gkeys_per_s": round(nk / (ms * 1e-3) / 1e9, 3)}
        del K, V, Kb, Vb
    return kv


def _extras_buffer(gs, torch, W, n, dev, stream):
    """Smaller buffers on the headline input (Frogsort3, the default below
    0.5, and Frogsort2); %RAM is 1 + workspace / data and tFootprint =
    %RAM x runTime (the paper's sustainability measures)."""
    x = torch.from_numpy(W.f64_pattern("uniform", n, seed=0)).to(dev)
    buf = torch.empty_like(x)
    small = {}
    for algo, fracs in (("frogsort1", (0.5,)), ("frogsort3", (0.45, 0.25, 0.1, 1 / 64)),
                        ("frogsort2", (0.25, 0.1))):
        for p in fracs:
            log(f"extras: {algo} buffer_fraction {p}")
            need = gs.gs_workspace_bytes_f64(n, p, algo)
            ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
            ws = ws[(-ws.data_ptr()) % 256:][:need]

            def fn_small(i, timed, p=p, ws=ws, algo=algo):
                if timed is None:
                    buf.copy_(x)
                else:
                    gs.gs_sort_f64(buf, buffer_fraction=p, workspace=ws, algo=algo)
            gs.gs_sort_f64(buf.copy_(x), buffer_fraction=p, workspace=ws, algo=algo)
            ms = _time_calls(torch, stream, fn_small, 3)
            ram = 1.0 + need / (8.0 * n)
            small[f"{algo}_p{p:.4g}"] = {"ms": round(ms, 3), "gkeys_per_s": round(n / (ms * 1e-3) / 1e9, 3),
                                         "ram_fraction": round(ram, 4), "t_footprint_ms": round(ram * ms, 3)}
            del ws
    del x, buf
    return small


def _names(arg, allowed):
    names = tuple(a for a in arg.split(",") if a)
    bad = [a for a in names if a not in allowed]
    if bad:
        print(f"unknown name(s) {bad}; choose from {list(allowed)}", file=sys.stderr)
        sys.exit(2)
    return names


def run_extras(args, gs, torch, W, dev):
    return extras(gs, torch, W, args.log2n, dev, _names(args.extras, SECTIONS),
                  _names(args.learned_patterns, LEARNED_PATTERNS), _names(args.learned_calls, LEARNED_CALLS),
                  _names(args.kv_patterns, KV_PATTERNS), _names(args.seg_workloads, SEG_WORKLOADS),
                  not args.no_seg_per_array)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--pattern", default="uniform")
    ap.add_argument("--cpu-sample-log2", type=int, default=26)
    ap.add_argument("--cpu-full", action="store_true",
                    help="also time both CPU references on the whole input (about a minute)")
    ap.add_argument("--cpu-full-reps", type=int, default=1,
                    help="runs of each CPU reference on the whole input with --cpu-full (median reported)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the learned / segmented / key-value side measurements")
    ap.add_argument("--extras", default=",".join(SECTIONS),
                    help="comma-separated side measurements to run, from " + ", ".join(SECTIONS))
    ap.add_argument("--learned-patterns", default=",".join(LEARNED_PATTERNS))
    ap.add_argument("--learned-calls", default=",".join(LEARNED_CALLS))
    ap.add_argument("--kv-patterns", default=",".join(KV_PATTERNS))
    ap.add_argument("--seg-workloads", default=",".join(SEG_WORKLOADS))
    ap.add_argument("--no-seg-per-array", action="store_true",
                    help="skip the per-array plain launches the segmented sort is compared with")
    ap.add_argument("--extras-only", action="store_true",
                    help="run only the chosen side measurements (to profile one workload) and print "
                         "them; no headline line")
    ap.add_argument("--buffer-fraction", type=float, default=0.5,
                    help="time this buffer fraction instead (below 0.5: Frogsort3 unless --algo)")
    ap.add_argument("--algo", default="auto", choices=["auto", "frogsort1", "frogsort2", "frogsort3"])
    args = ap.parse_args()
    frac, algo = args.buffer_fraction, args.algo
    for arg, allowed in ((args.extras, SECTIONS), (args.learned_patterns, LEARNED_PATTERNS),
                         (args.learned_calls, LEARNED_CALLS), (args.kv_patterns, KV_PATTERNS),
                         (args.seg_workloads, SEG_WORKLOADS)):
        _names(arg, allowed)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sort of one array runs on one device). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2402_01816_amd as gs
    import workloads as W

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(3)
    dev = torch.device("cuda:0")
    if args.extras_only:
        print(json.dumps({"extras": run_extras(args, gs, torch, W, dev)}), flush=True)
        return
    n = 1 << args.log2n
    log(f"generating {args.pattern} n=2^{args.log2n}")
    x = W.f64_pattern(args.pattern, n, seed=0)
    pristine = torch.from_numpy(x).to(dev)
    del x
    need = gs.gs_workspace_bytes_f64(n, frac, algo)
    ws_raw = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    off = (-ws_raw.data_ptr()) % 256
    ws = ws_raw[off: off + need]
    stream = torch.cuda.current_stream(dev)

    log(f"warmup {args.warmup}")
    buf = torch.empty_like(pristine)
    for _ in range(args.warmup):
        buf.copy_(pristine)
        gs.gs_sort_f64(buf, frac, workspace=ws, algo=algo)
    torch.cuda.synchronize()
    rep = None
    if args.warmup > 0:
        buf.copy_(pristine)
        rep = gs.gs_sort_f64(buf, frac, workspace=ws, report=True, algo=algo)
    del buf

    # empirical ceilings: a copy moves the same 16n bytes as one merge pass
    # (8n read + 8n write): the library's streaming copy kernel and the
    # runtime's device-to-device copy
    dst = torch.empty_like(pristine)

    def copy_rate(fn):
        for _ in range(2):
            fn()
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        c0.record(stream)
        for _ in range(5):
            fn()
        c1.record(stream)
        torch.cuda.synchronize()
        return 16.0 * n / (c0.elapsed_time(c1) / 5 * 1e-3) / 1e9
    copy_gbs = copy_rate(lambda: gs.gs_copy_f64(pristine, dst))
    runtime_copy_gbs = copy_rate(lambda: dst.copy_(pristine))
    del dst

    log(f"preparing {args.steps} input copies")
    copies = [pristine.clone() for _ in range(args.steps)]
    torch.cuda.synchronize()

    gs.lib.gs_trace_enable.argtypes = [ctypes.c_int]
    gs.lib.gs_trace_read.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                                     ctypes.c_int]
    # the timed steps bracket only the merge launches with events (the fewest
    # events that time the dominant kernel); the other kernels are timed in a
    # separate traced pass below
    gs.lib.gs_trace_enable(2)
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for c in copies:
        gs.gs_sort_f64(c, frac, workspace=ws, algo=algo)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gs.lib.gs_trace_enable(0)
    maxrec = 64 * (args.steps + 1)
    kinds = (ctypes.c_int * maxrec)()
    mss = (ctypes.c_double * maxrec)()
    nrec = gs.lib.gs_trace_read(kinds, mss, maxrec)
    gpu_ms = e0.elapsed_time(e1)
    ms_per_step = gpu_ms / args.steps

    # spot check of every timed output (sorted, same multiset as the input)
    for c in copies[:2]:
        assert bool((c[1:] >= c[:-1]).all().item()), "bench output not sorted"
    del copies

    names = {0: "fill", 1: "leaf", 2: "partition", 3: "merge", 4: "other", 5: "depwin"}
    merge_ms = [mss[i] for i in range(nrec) if kinds[i] == 3]

    # every kernel kind of a step, from an untimed pass with every launch traced
    trace_steps = min(2, args.steps)
    trace_copies = [pristine.clone() for _ in range(trace_steps)]
    torch.cuda.synchronize()
    gs.lib.gs_trace_enable(1)
    for c in trace_copies:
        gs.gs_sort_f64(c, frac, workspace=ws, algo=algo)
    torch.cuda.synchronize()
    gs.lib.gs_trace_enable(0)
    nrec = gs.lib.gs_trace_read(kinds, mss, maxrec)
    per_kind = {}
    for i in range(nrec):
        per_kind.setdefault(names.get(kinds[i], "other"), []).append(mss[i])
    del trace_copies
    levels = len(merge_ms) // max(args.steps, 1)
    merge_avg = sum(merge_ms) / max(len(merge_ms), 1)
    default = frac >= 0.5 and algo in ("auto", "frogsort1")
    if default:
        merge_bytes = 16.0 * n                      # every key read once and written once
        merged = n * levels
    else:
        # launches differ in size: the plan's merged elements over all rounds
        # give the average bytes per launch
        cnt = gs.plan_frog2(n, frac)[2] if algo == "frogsort2" else gs.plan_frog3(n, frac)[3]
        merged = cnt[6]
        merge_bytes = 16.0 * merged / max(levels, 1)
    achieved = merge_bytes / (merge_avg * 1e-3) / 1e9 if merge_avg > 0 else 0.0
    ram = 1.0 + need / (8.0 * n)
    traffic = merge_traffic() if (n == 1 << 28 and args.pattern == "uniform" and default) else None
    value = n / (ms_per_step * 1e-3) / 1e9
    passes = 1 + merged / n
    whole_bytes = 16.0 * n * passes

    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"plain stable f64 sort, n=2^{args.log2n}, {args.pattern} keys "
                               f"(seed 0), buffer_fraction {frac:g}" + ("" if default else f", {algo}"),
                   "n": n, "pattern": args.pattern, "buffer_fraction": frac, "algo": algo,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "merge_kernel",
                     "bytes_per_launch": merge_bytes, "avg_launch_ms": round(merge_avg, 5)},
        "copy_ceiling_gbs": round(copy_gbs, 1),
        "merge_frac_of_copy": round(achieved / copy_gbs, 4) if copy_gbs > 0 else None,
        "runtime_copy_gbs": round(runtime_copy_gbs, 1),
        "merge_frac_of_runtime_copy": round(achieved / runtime_copy_gbs, 4) if runtime_copy_gbs > 0 else None,
        "ram_fraction": round(ram, 5),
        "t_footprint_ram_s": round(ram * ms_per_step * 1e-3, 6),
        "whole_sort_hbm_frac": round(whole_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "passes": round(passes, 3),
        "per_kernel_ms_per_step": {k: round(sum(v) / trace_steps, 4) for k, v in per_kind.items()},
        "per_kernel_note": f"every launch bracketed by events, {trace_steps} untimed steps",
        "wall_s": round(wall, 3),
        "report": rep,
    }
    if not args.no_extras:
        out["extras"] = run_extras(args, gs, torch, W, dev)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(1 << args.cpu_sample_log2, args.pattern,
                                           n if args.cpu_full else 0, args.cpu_full_reps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
