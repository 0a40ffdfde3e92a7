"""Host validation and plan preparation under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/host_checks.cpp is built with g++ (host code only, no device code) together with the
library's host-prep source and run: random trees in shuffled id order and random tables are
prepared and every product (slot order, level schedule, branch lengths, totals, depth-first
tip ranges and sorted entries, the tail program of the propagation) is checked against
counts walked up from each tip; malformed trees and tables must return their status codes.
"""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2005_05826_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def test_host_prep_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime.h")):
        pytest.skip("g++ or the HIP headers are not available")
    exe = str(tmp_path / "host_checks")
    build = [gxx, "-std=c++17", "-O1", "-g", "-pthread", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include",
             f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
             os.path.join(ROOT, "tests", "host_checks.cpp"), os.path.join(CSRC, "host_prep.cpp"), "-o", exe]
    r = subprocess.run(build, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, "400"], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout[-2000:])
    assert r.returncode == 0, (r.stdout[-2000:] + r.stderr[-4000:])
    assert "0 failures" in r.stdout
