"""The launch-time divisor of the run-time-length kernels (csrc/gp_fdiv.hpp), built for
the host with g++ under the undefined-behaviour sanitizer and checked against the
hardware division over every divisor up to 5000, the powers of two up to 2^30 and their
neighbours, and numerators across 0 .. 2^31 - 1 (no GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_fast_division_matches_integer_division(tmp_path):
    exe = str(tmp_path / "fdiv")
    cmd = ["g++", "-std=c++17", "-O2", "-D__host__=", "-D__device__=",
           "-fsanitize=undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "paper_1601_04640_amd", "csrc"),
           os.path.join(ROOT, "tests", "host", "fdiv_main.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok "), r.stdout
    assert "runtime error" not in r.stderr, r.stderr
