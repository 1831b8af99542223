"""Build the HIP library (libsm.so) for gfx950 with hipcc, in-tree.

    python -m paper_1012_2547_amd.build          # compile
    python -m paper_1012_2547_amd.build --asm    # also write the gfx950 ISA to _build/
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libsm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["sm_kernels.hip", "sm_batch.hip", "sm_api.cpp", "sm_batch.cpp", "sm_server.cpp"]

# Packed-FP32 instructions are disabled for every HIP translation unit.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall",
             "-Wno-unused-function", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def build(verbose: bool = False, asm: bool = False) -> str:
    bdir = os.path.join(ROOT, "_build")
    os.makedirs(bdir, exist_ok=True)
    cmds, objs = [], []
    for src in sources():
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        cmd = [HIPCC] + HIP_FLAGS + ["-c", src, "-o", obj]
        if src.endswith(".cpp"):
            cmd[1:1] = ["-x", "hip"]
        cmds.append(cmd)
        objs.append(obj)
        if asm and src.endswith(".hip"):
            s = os.path.join(bdir, os.path.basename(src) + ".gfx950.s")
            cmds.append([HIPCC] + HIP_FLAGS + ["--cuda-device-only", "-S", src, "-o", s])
    # one compiler process per translation unit, at most JOBS at a time
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", "0") or 0) or os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(jobs) as ex:
        for cmd in cmds:
            if verbose:
                print(" ".join(cmd), flush=True)
        list(ex.map(subprocess.check_call, cmds))
    tmp = LIB + ".tmp%d" % os.getpid()
    # roctx: named host ranges for rocprofv3 --marker-trace
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + [
        "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, asm="--asm" in sys.argv))
