"""The service's workspace allocator (csrc/mgr_arena.hpp), built with g++ and
checked against a brute-force granule map on random allocate/release
sequences.  No GPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2105_12764_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_arena_first_fit_and_coalescing(tmp_path):
    exe = tmp_path / "arena_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", CSRC, os.path.join(HERE, "arena_check.cpp"),
                    "-o", str(exe)], check=True, capture_output=True, text=True)
    for seed in (1, 2, 3):
        r = subprocess.run([str(exe), str(seed)], capture_output=True, text=True, timeout=120)
        assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
