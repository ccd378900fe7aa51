"""The plan cache's bookkeeping (csrc/mgr_plan_cache.hpp), built with g++ and
checked on random sequences: least-recently-used order and capacity, and the
lifetime rule -- a plan is destroyed only when its last owner (the cache, a
call in progress, a captured graph's holder) lets go, never inside a graph's
release callback.  No GPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2105_12764_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_plan_cache_order_and_lifetimes(tmp_path):
    exe = tmp_path / "plan_cache_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", CSRC, os.path.join(HERE, "plan_cache_check.cpp"),
                    "-o", str(exe)], check=True, capture_output=True, text=True)
    for seed in (1, 2, 3):
        r = subprocess.run([str(exe), str(seed)], capture_output=True, text=True, timeout=120)
        assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
