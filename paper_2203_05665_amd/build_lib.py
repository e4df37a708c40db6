"""Builds the HIP library libh2mi355x.so in-tree for gfx950.

Host-only C++ (tree construction, quadrature tables) is compiled with g++ and
-ffp-contract=off, so the decisions that shape the trees use plain IEEE double
arithmetic; HIP sources are compiled with hipcc for gfx950 with packed FP32
instructions disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libh2mi355x.so")
BUILD = os.path.join(HERE, "_build")
ARCH = os.environ.get("H2_OFFLOAD_ARCH", "gfx950")

HOST_SOURCES = ["structure.cpp", "quadrules.cpp"]
HIP_SOURCES = ["assemble.hip", "matvec.hip", "matvec_multi.hip", "ksolve.hip", "krylov.hip", "recompress.hip",
               "tune.hip", "probe.hip", "capi.hip"]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    jobs = []
    objs = []
    for s in HOST_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        objs.append(o)
        jobs.append(["g++", "-O2", "-std=c++17", "-fPIC", "-pthread", "-ffp-contract=off", "-Wall", "-c",
                     os.path.join(CSRC, s), "-o", o])
    for s in HIP_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        objs.append(o)
        jobs.append([hipcc, "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
                     "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                     "-Wno-unused-command-line-argument", "-c", os.path.join(CSRC, s), "-o", o])
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for r in ex.map(_run, jobs):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout, r.stderr)
    tmp = OUT + ".tmp"
    _run([hipcc, "-shared", "-fPIC", "-pthread", "--offload-arch=" + ARCH, "-o", tmp] + objs)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
