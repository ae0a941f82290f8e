"""Build libdugks.so for gfx950 with hipcc (in-tree, next to this file)."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdugks.so")
SOURCES = [os.path.join(CSRC, "dugks_kernels.hip"), os.path.join(CSRC, "dugks_api.cpp"),
           os.path.join(CSRC, "dugks_pool.cpp")]
HEADERS = [os.path.join(CSRC, "dugks_impl.h"), os.path.join(CSRC, "dugks_host.h"),
           os.path.join(os.path.dirname(HERE), "include", "dugks.h")]
# the bandwidth probe the benchmark compares the step with (not part of libdugks)
PROBE_LIB = os.path.join(HERE, "libcopyprobe.so")
PROBE_SOURCES = [os.path.join(CSRC, "copy_probe.hip")]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def command(out: str = LIB, extra=(), sources=None) -> list[str]:
    return [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
            # packed FP32 instructions stay off (see the design notes)
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            # multiply-adds are fused within a source expression only, never
            # across statements: the same expression then rounds the same way
            # in every kernel that inlines it (the one-row kernel and the
            # march give the same bits)
            "-ffp-contract=on",
            "-Wno-unused-command-line-argument", *extra, "-o", out, *(sources or SOURCES)]


def build(verbose: bool = False) -> str:
    for lib, src in ((LIB, SOURCES), (PROBE_LIB, PROBE_SOURCES)):
        tmp = lib + ".tmp"
        cmd = command(tmp, sources=src)
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, lib)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
