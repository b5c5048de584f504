"""Host build of the fine-element code the defect kernels use (csrc/element.h):
the strip form of the element residuals against the element-by-element form,
and the tile partition (strips + halo ring, four conflict-free assembly
rounds).  The element-by-element form itself is checked against the FP64
oracle by the GPU parity tests."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2008_11520_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_strip_form_and_tile_partition(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "element_check")
    subprocess.check_call([HIPCC, "-O2", "-std=c++17", "--offload-arch=gfx950", "-I", CSRC,
                           os.path.join(HERE, "element_check.cpp"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
