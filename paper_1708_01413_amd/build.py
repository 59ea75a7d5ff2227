"""Build libapc.so (HIP for gfx950) in-tree with hipcc.

Every source is compiled to its own object in parallel (each file launches only
its own kernels, so no relocatable device code is needed), then the objects are
linked into one shared library."""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libapc.so")
OBJDIR = os.path.join(ROOT, "_build")
SOURCES = [os.path.join(CSRC, "apc_kernels.hip"), os.path.join(CSRC, "apc_gemm.hip"),
           os.path.join(CSRC, "apc_batch.hip"), os.path.join(CSRC, "apc_noalloc.hip"),
           os.path.join(CSRC, "apc_resident.hip"), os.path.join(CSRC, "apc_host.cpp")]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    "--offload-arch=gfx950",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def _clean(text: str) -> str:
    return "\n".join(l for l in text.splitlines()
                     if "packed-fp32-ops" not in l and "not a recognized feature" not in l)


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    out = _clean(res.stdout + res.stderr)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{out}")
    if verbose and out.strip():
        print(out)


def build_lib(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJDIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = [os.path.join(OBJDIR, os.path.basename(src) + ".o") for src in SOURCES]
    cmds = [[hipcc, *HIPCC_FLAGS, *inc, "-c", src, "-o", obj] for src, obj in zip(SOURCES, objs)]
    with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_lib(verbose="-v" in sys.argv))
