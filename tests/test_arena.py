"""Host test of the serving arena's bookkeeping (csrc/arena.h): the first-fit
block list of the device region and the pinned staging ring, driven through
random sequences (no GPU)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2008_11520_amd", "csrc")


def test_arena_bookkeeping_random_sequences(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "arena_check")
    subprocess.check_call([cxx, "-O2", "-std=c++17", "-Wall", "-I", CSRC, os.path.join(HERE, "arena_check.cpp"),
                           "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr
