"""Builds libbemrat.so in-tree with hipcc for gfx950.

Usage: python -m paper_1906_03938_amd.build  (or via __graft_entry__.build()).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbemrat.so")
SOURCES = ["abi.cpp", "mesh.hip", "sweep.hip", "sweep_lp.hip", "combine.hip", "assemble.hip", "nearfield.hip", "scratch.hip", "nfnet.hip", "lu.hip"]
HEADERS = ["internal.h", "generators.h", "devmath.h"]


def command(out: str = LIB, arch: str = "gfx950", extra=()):
    return [
        "hipcc",
        f"--offload-arch={arch}",
        "-O3",
        "-std=c++17",
        "-fPIC",
        "-shared",
        # keep the compiler from emitting packed FP32 instructions
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"),
        "-I", CSRC,
        *extra,
        "-o", out,
        *[os.path.join(CSRC, s) for s in SOURCES],
    ]


def build(verbose: bool = False, out: str = LIB) -> str:
    cmd = command(out)
    if verbose:
        print(" ".join(cmd), flush=True)
    tmp = out + ".tmp"
    cmd[cmd.index("-o") + 1] = tmp
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
