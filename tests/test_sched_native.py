"""The serving executor's pool allocator and batch planning (header-only host
code shared by the executor and its simulation), compiled on the host with
g++ under the address and undefined-behaviour sanitizers and exercised on
random operation sequences: no overlapping blocks, exact byte accounting,
a sorted and coalesced free list that returns to one block, tiles that
cover every request's rays once and in order, requests in order of
remaining work."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_sched_under_sanitizers(tmp_path):
    exe = str(tmp_path / "sched_check")
    src = os.path.join(ROOT, "tests", "native", "sched_check.cpp")
    inc = os.path.join(ROOT, "paper_2602_05081_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", inc, src, "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert "sched checks passed" in out.stdout
