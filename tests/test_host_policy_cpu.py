"""Host-side C++ of the library on the CPU, under the address and
undefined-behaviour sanitizers: the query server's policy (arena allocator,
cost-aware admission, driven with random sequences and a fake executor) and
the batched plans' tuning-cache format (round trips, damaged and random input)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1803_08285_amd", "csrc")


def _build_and_run(tmp_path, name):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / name
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I", CSRC, os.path.join(ROOT, "tests", "cpu", name + ".cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout


def test_serve_policy_under_sanitizers(tmp_path):
    assert "all checks passed" in _build_and_run(tmp_path, "serve_policy_test")


def test_tune_cache_under_sanitizers(tmp_path):
    assert "all checks passed" in _build_and_run(tmp_path, "tune_cache_test")
