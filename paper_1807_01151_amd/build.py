"""Builds the HIP library libeg.so in-tree for gfx950 with hipcc."""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libeg.so")
SOURCES = ["eg_kernels.hip", "eg_jaclu_lds.hip", "eg_noalloc.hip", "eg_peak.hip", "eg_tangent.hip", "eg_poly.hip", "eg_host.cpp"]
FLAGS_COMPILE = ["-std=c++17", "-O3", "--offload-arch=gfx950", "-fPIC",
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
    """Compiles every translation unit to an object in parallel (each keeps
    its own device code object; no relocatable device code is needed since
    every kernel is launched from the unit that defines it), then links."""
    import tempfile
    srcs, _ = sources()
    tmp = LIB + ".tmp"
    with tempfile.TemporaryDirectory(prefix="egbuild") as td:
        objs, procs = [], []
        for src in srcs:
            obj = os.path.join(td, os.path.basename(src) + ".o")
            cmd = ["hipcc", *FLAGS_COMPILE, "-I", CSRC, "-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((subprocess.Popen(cmd), cmd))
            objs.append(obj)
        bad = [cmd for p, cmd in procs if p.wait() != 0]
        if bad:
            raise subprocess.CalledProcessError(1, bad[0])
        cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
