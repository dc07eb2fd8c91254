"""Build libgs.so (the HIP library behind include/gs.h) for gfx950 with hipcc.

Usage: python paper_2402_01816_amd/build.py   (or build() of __graft_entry__.py)
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.environ.get("GS_LIB_OUT", os.path.join(HERE, "libgs.so"))
OBJDIR = os.environ.get("GS_OBJ_DIR", os.path.join(HERE, "_build"))
ARCH = os.environ.get("GS_OFFLOAD_ARCH", "gfx950")

SOURCES = ["gs_abi.cpp", "gs_plan.cpp", "gs_sort.hip", "gs_seg.hip", "gs_mlp.hip", "gs_learned.hip",
           "gs_errors.hip", "gs_noalloc.hip", "gs_measure.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CFLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
] + os.environ.get("GS_EXTRA_CFLAGS", "").split()


def _compile(src: str) -> str:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *CFLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    # show warnings other than the host pass's note about the packed-fp32 feature
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l and l.strip())
    if msg:
        sys.stderr.write(msg + "\n")
    return obj


def build() -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    with ThreadPoolExecutor(len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
