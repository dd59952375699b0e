"""Builds librd.so (the gfx950 race checker) in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "librd.so")
DEMO_LIB = os.path.join(HERE, "librd_demo.so")
DEMO_SOURCE = "rd_demo.hip"
SOURCES = ["rd_prep.hip", "rd_sort.hip", "rd_interp.hip", "rd_engine.hip", "rd_segcheck.hip", "rd_batch.hip", "rd_host.hip",
           "rd_server.hip", "rd_kinds.hip", "rd_lockset.hip", "rd_gwcp.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
    # no packed fp32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    subprocess.check_call([HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj],
                          stderr=subprocess.DEVNULL if os.environ.get("RD_QUIET_BUILD") else None)
    return obj


def build() -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES) + 1)) as ex:
        objs = list(ex.map(_compile, SOURCES + [DEMO_SOURCE]))
    demo_obj = objs.pop()
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    # the example kernels recorded with include/rd_device.h, a library of their own
    tmp = DEMO_LIB + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-o", tmp, demo_obj])
    os.replace(tmp, DEMO_LIB)
    return LIB


if __name__ == "__main__":
    print(build())
