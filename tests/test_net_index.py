"""Host replay of the persistent network kernels' prefetch addresses
(csrc/net_index.h, the functions those kernels call): every read of a tile's
input rows and state lies inside the rows of the flow it belongs to, for
K = 1..3, H = 64/128 and every row count of a tile's halves, and every row
whose results are stored receives its own input row and state."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2008_11520_amd", "csrc")


def test_prefetch_addresses_in_bounds(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "net_index_check")
    subprocess.check_call([cxx, "-O2", "-std=c++17", "-Wall", "-I", CSRC,
                           os.path.join(HERE, "net_index_check.cpp"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr
