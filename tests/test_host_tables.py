"""The host-side projector tables (sphere rows, projector values and per-plane row ranges that the
plane pass and the projector kernels index) checked on the CPU by tests/host/check_tables.cpp,
built with AddressSanitizer and UndefinedBehaviorSanitizer: every projector shape the tests and
workloads use, plus atoms on grid points, on the cell corner, outside the cell, coincident atoms,
empty spheres and a sphere just below half the cell."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "check_tables.cpp")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_projector_tables_under_sanitizers(tmp_path):
    exe = str(tmp_path / "check_tables")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"), SRC, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
    # verify_asan_link_order=0: the sanitizer runtime need not be the first library a preload
    # list names
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok "), r.stdout
