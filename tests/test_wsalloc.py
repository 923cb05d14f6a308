"""The workspace bookkeeping (paper_2509_22975_amd/csrc/mcd_wsalloc.h) on the
CPU, built with g++ under the address and undefined-behaviour sanitizers and
checked against a brute-force model of the range (tests/wsalloc_check.cc)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_workspace_bookkeeping_under_sanitizers():
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "wsalloc_check")
        cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "paper_2509_22975_amd", "csrc"),
               os.path.join(ROOT, "tests", "wsalloc_check.cc"), "-o", exe]
        subprocess.run(cmd, check=True, capture_output=True, text=True)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, r.stderr
        assert r.stdout.strip() == "ok"
