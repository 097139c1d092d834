"""Builds the HIP library libeg.so in-tree for gfx950 with hipcc."""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libeg.so")
SOURCES = ["eg_kernels.hip", "eg_host.cpp"]
FLAGS = ["-std=c++17", "-O3", "--offload-arch=gfx950", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-Wno-unknown-pragmas"]


def sources():
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    hdrs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    hdrs.append(os.path.join(os.path.dirname(HERE), "include", "eg.h"))
    return srcs, hdrs


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    srcs, hdrs = sources()
    return any(os.path.getmtime(f) > t for f in srcs + hdrs)


def build(verbose: bool = False) -> str:
    srcs, _ = sources()
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *FLAGS, "-I", CSRC, *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
