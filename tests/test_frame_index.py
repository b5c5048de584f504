"""Host replay of the tile frame the one-launch K = 2 step hands to the rhs
kernel (csrc/frame.h, the functions both kernels call): every node is
completed once, every contribution lookup hits a slot written with that
patch's output, and the nodes written in place are read by no other tile's
defect, over meshes of 1..26 x 1..26 coarse elements."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2008_11520_amd", "csrc")


def test_tile_frame_covers_every_node_once(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "frame_check")
    subprocess.check_call([cxx, "-O2", "-std=c++17", "-Wall", "-I", CSRC,
                           os.path.join(HERE, "frame_check.cpp"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr
