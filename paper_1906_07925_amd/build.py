"""Build the gfx950 shared library ``libmpsph.so`` in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmpsph.so")

SOURCES = ["mpsph.hip", "sort.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # multiply-adds fused only within one expression (as written), never across statements, so
    # that every kernel built from the same arithmetic (the pair-kernel variants, the batched and
    # single-domain launches) rounds it the same way
    "-ffp-contract=on",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden", "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False, out: str | None = None, defines: dict | None = None) -> str:
    """Compile the library; ``defines`` sets tuning macros (row group, batch width, waves per
    EU) for a build written to ``out`` instead of the default in-tree path."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    lib = out or LIB
    out_tmp = lib + ".tmp"
    dflags = [f"-D{k}={v}" for k, v in (defines or {}).items()]
    cmd = [hipcc, *FLAGS, *dflags, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           *[os.path.join(CSRC, s) for s in SOURCES], "-o", out_tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(out_tmp, lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
