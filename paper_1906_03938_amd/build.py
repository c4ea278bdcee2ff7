"""Builds libbemrat.so in-tree with hipcc for gfx950.

Each source is compiled to an object of its own, the compilations running side by side,
and the objects are linked into the shared library.

Usage: python -m paper_1906_03938_amd.build  (or via __graft_entry__.build()).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbemrat.so")
SOURCES = ["abi.cpp", "mesh.hip", "sweep.hip", "sweep_lp.hip", "combine.hip", "assemble.hip", "nearfield.hip", "scratch.hip", "nfnet.hip", "lu.hip"]
HEADERS = ["internal.h", "generators.h", "devmath.h"]


def flags(arch: str = "gfx950", extra=()):
    return [
        f"--offload-arch={arch}",
        "-O3",
        "-std=c++17",
        "-fPIC",
        # keep the compiler from emitting packed FP32 instructions
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"),
        "-I", CSRC,
        *extra,
    ]


def compile_command(src: str, obj: str, arch: str = "gfx950", extra=()):
    return ["hipcc", *flags(arch, extra), "-c", "-o", obj, os.path.join(CSRC, src)]


def link_command(objs, out: str, arch: str = "gfx950"):
    return ["hipcc", f"--offload-arch={arch}", "-shared", "-fPIC", "-o", out, *objs]


def build(verbose: bool = False, out: str = LIB, jobs: int | None = None) -> str:
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1)
    tmpdir = tempfile.mkdtemp(prefix="bemrat_build_")
    try:
        objs = [os.path.join(tmpdir, s + ".o") for s in SOURCES]
        cmds = [compile_command(s, o) for s, o in zip(SOURCES, objs)]

        def run(cmd):
            if verbose:
                print(" ".join(cmd), flush=True)
            return subprocess.run(cmd, capture_output=True, text=True)

        with ThreadPoolExecutor(max_workers=jobs) as pool:
            results = list(pool.map(run, cmds))
        failed = [(c, r) for c, r in zip(cmds, results) if r.returncode != 0]
        for c, r in failed:
            sys.stderr.write(r.stdout + r.stderr)
        if failed:
            raise subprocess.CalledProcessError(failed[0][1].returncode, failed[0][0])
        tmp = out + ".tmp"
        link = link_command(objs, tmp)
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.run(link, check=True)
        os.replace(tmp, out)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
