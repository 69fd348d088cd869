"""Host C++ unit tests (tests/host_cpp/test_plan.cpp) of the library's pure
host code: position mapping, the stability symbol and the checkpoint
schedule, built with g++ under the address and undefined-behaviour
sanitizers and run on the CPU."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_units_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "test_plan")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-static-libasan",
           "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2502_12350_amd", "csrc"),
           os.path.join(ROOT, "tests", "host_cpp", "test_plan.cpp"),
           os.path.join(ROOT, "paper_2502_12350_amd", "csrc", "wfd_plan.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ALL PASSED" in r.stdout
