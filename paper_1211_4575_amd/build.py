"""Build libpp.so (the HIP library behind include/pp.h) for gfx950, in-tree.

Every .hip file under csrc/ is compiled with hipcc into an object, in parallel, and the
objects are linked into paper_1211_4575_amd/libpp.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libpp.so")
SRC_INPUTS = os.path.join(HERE, "csrc_inputs")
OUT_INPUTS = os.path.join(HERE, "libpp_inputs.so")
BUILD = os.path.join(HERE, "_build")
ARCH = os.environ.get("PP_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CFLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-munsafe-fp-atomics",
    # packed FP32 instructions are kept off in every GPU code object
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *CFLAGS, "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stdout}\n{res.stderr}")
    warn = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if warn and os.environ.get("PP_BUILD_VERBOSE"):
        print(warn, file=sys.stderr)
    return obj


def _link(objs, out):
    tmp = out + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, out)


def build(jobs: int | None = None) -> str:
    """Compile every HIP source and link libpp.so (the method) and libpp_inputs.so (the
    on-device input generator); returns the path of libpp.so.  Always rebuilds."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(SRC, "*.hip")))
    srcs_in = sorted(glob.glob(os.path.join(SRC_INPUTS, "*.hip")))
    jobs = jobs or min(8, len(srcs) + len(srcs_in))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs + srcs_in))
    _link(objs[: len(srcs)], OUT)
    _link(objs[len(srcs):], OUT_INPUTS)
    return OUT


if __name__ == "__main__":
    print(build())
