"""Build libwstack.so (the HIP kernels and the C ABI) in-tree for gfx950.

Usage: python -m paper_2301_06061_amd.build [--jobs N]

Every HIP source is compiled with hipcc for gfx950 only; object files go to
``paper_2301_06061_amd/_build`` and the shared library to
``paper_2301_06061_amd/libwstack.so``.  The memory access-pattern probe that
``bench.py --access-probes`` runs (a separate program, not part of the
library) is built next to its source in ``probes/``.  This always
recompiles.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libwstack.so")
ARCH = "gfx950"

SOURCES = ["abi.cpp", "bin.hip", "grid.hip", "fft.hip", "clean.hip"]
PROBES = os.path.join(HERE, "probes")
PROBE_SOURCES = ["access_patterns.hip"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc",
                 shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP toolchain is required")


def _flags():
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
        # No packed-FP32 instructions: their forms are avoided on this part.
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", INCLUDE, "-I", CSRC,
        "-Wno-unused-command-line-argument",
    ]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + _flags()
    if src.endswith(".cpp"):
        cmd += ["-x", "hip"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{res.stderr}")
    return obj


def _compile_probe(src: str) -> str:
    exe = os.path.join(PROBES, os.path.splitext(src)[0])
    cmd = [hipcc()] + _flags() + [os.path.join(PROBES, src), "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compiling probe {src} failed:\n{res.stderr}")
    return exe


def build(jobs: int = 4, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        probes = ex.map(_compile_probe, PROBE_SOURCES)
        objs = list(ex.map(_compile, SOURCES))
        list(probes)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] \
        + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"linking libwstack.so failed:\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    args = ap.parse_args(argv)
    build(args.jobs, verbose=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
