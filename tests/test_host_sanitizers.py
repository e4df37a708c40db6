"""The library's host code (tree and block-tree construction, symmetric halving
of the block lists, quadrature generators) built with g++ under AddressSanitizer
and UBSan and run on icosphere and cube meshes: no memory error, no undefined
behaviour, no leak, and the tree invariants hold (perm is a permutation, the
leaves cover every position)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import h2_inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2203_05665_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_tree_code_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "drive")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=undefined", "-I", CSRC, os.path.join(ROOT, "tests", "host_sanitize_driver.cpp"),
           os.path.join(CSRC, "structure.cpp"), os.path.join(CSRC, "quadrules.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    files = []
    for name, (kind, level) in {"sphere2": ("sphere", 2), "cube32": ("cube", 32), "sphere5": ("sphere", 5)}.items():
        V, T = I.mesh_for(kind, level)
        path = str(tmp_path / (name + ".bin"))
        with open(path, "wb") as f:
            np.array([V.shape[0], T.shape[0]], np.int64).tofile(f)
            np.ascontiguousarray(V, np.float64).tofile(f)
            np.ascontiguousarray(T, np.int32).tofile(f)
        files.append(path)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe] + files, capture_output=True, text=True, timeout=600, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-3000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out and "LeakSanitizer" not in out
    assert "quadrature ok" in out and out.count("m=4 leaf=64") == 3
