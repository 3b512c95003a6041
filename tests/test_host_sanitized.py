"""The plan-time host code (csrc/host_plan.hpp: frame rule, relay binning for
the spreading kernel, Gauss-Legendre quadrature, float64 FFT) built with g++
under the address and undefined-behaviour sanitizers and checked by
tests/host/host_plan_check.cpp against definitions written out there."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2501_05244_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "host", "host_plan_check.cpp")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not installed")
def test_host_plan_under_sanitizers(tmp_path):
    exe = tmp_path / "host_plan_check"
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wall", "-Werror"]
    r = subprocess.run(["g++", *flags, "-I", CSRC, SRC, "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "host plan checks ok" in r.stdout
