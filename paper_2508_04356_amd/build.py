"""Builds libgdsw.so (HIP for gfx950) in the package directory.

Usage: python paper_2508_04356_amd/build.py   (or call build()).
Every call recompiles every source.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgdsw.so")

HIP_SOURCES = ["kernels_factor.hip", "kernels_inverse.hip", "kernels_gemv.hip", "kernels_symv.hip", "kernels_gemm.hip", "kernels_multi.hip", "kernels_ops.hip", "kernels_learned.hip", "setup.hip", "solve.hip", "solve_multi.hip", "batch.hip",
               "learned.hip", "noalloc.hip", "block.hip", "abi.hip"]
CXX_SOURCES = ["problem.cpp", "algebraic.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
          f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
HIP_FLAGS = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics"]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError("command failed:\n" + " ".join(cmd) + "\n" + p.stdout)
    return p.stdout


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compiles every source and links `out`; `defines` ("NAME=VALUE") are
    passed to every compile (launch-shape constants of the kernels)."""
    bdir = BUILD if out == LIB else out + ".build"
    os.makedirs(bdir, exist_ok=True)
    dflags = [f"-D{d}" for d in defines]
    jobs = []
    for src in HIP_SOURCES:
        obj = os.path.join(bdir, src + ".o")
        jobs.append([HIPCC, *COMMON, *HIP_FLAGS, *dflags, "-c", os.path.join(CSRC, src), "-o", obj])
    for src in CXX_SOURCES:
        obj = os.path.join(bdir, src + ".o")
        jobs.append(["g++", *COMMON, *dflags, "-c", os.path.join(CSRC, src), "-o", obj])
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
        outs = list(ex.map(_run, jobs))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    objs = [os.path.join(bdir, s + ".o") for s in HIP_SOURCES + CXX_SOURCES]
    tmp = out + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    import argparse

    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("-v", action="store_true", help="print compiler output")
    ap.add_argument("--out", default=LIB, help="library path (default: the package's libgdsw.so)")
    ap.add_argument("-D", dest="defines", action="append", default=[], help="NAME=VALUE for every compile")
    a = ap.parse_args()
    print(build(verbose=a.v, out=os.path.abspath(a.out), defines=a.defines))
