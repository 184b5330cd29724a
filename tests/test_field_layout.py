"""Host-side bounds check of the BF16 field kernel's scratch-slot, encoding
and LDS addressing (tests/field_bf16_layout_check.cpp, built on the CPU from
the kernel's own index functions) over the small scene's, the room's and
the panorama's networks and a grid of other accepted shapes."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_bf16_field_addressing_in_bounds(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not (os.path.exists(hipcc) or shutil.which(hipcc)):
        pytest.skip("hipcc not available")
    exe = tmp_path / "layout_check"
    src = os.path.join(HERE, "field_bf16_layout_check.cpp")
    build = subprocess.run([hipcc, "-x", "hip", "--offload-host-only", "-std=c++17", "-O2", src,
                            "-o", str(exe)], capture_output=True, text=True)
    assert build.returncode == 0, build.stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(run.stdout)
    assert run.returncode == 0, run.stdout
    assert run.stdout.startswith("ok:")
