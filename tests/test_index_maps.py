"""Host emulation of the kernels' index maps (tests/index_emulation.cpp over csrc/qs_index.h, the functions the kernels
call): block passes own every amplitude exactly once and use every LDS slot once per phase and stage; every fused-swap
form moves amplitude i to sigma(i) and writes no index twice."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_kernel_index_maps_on_the_host(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not installed")
    exe = tmp_path / "index_emulation"
    cmd = [cxx, "-std=c++17", "-O2", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"), "-I",
           os.path.join(ROOT, "paper_2203_16044_amd", "csrc"), os.path.join(ROOT, "tests", "index_emulation.cpp"),
           "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout + r.stderr
