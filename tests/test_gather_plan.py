"""Launch shapes of the gather-form sampler, checked on the CPU: the planner
header is compiled into a small host program that walks every shape planned
for q = 2..32, L = 1..512 and a range of chain counts and CU shares, and checks
the kernel's slot, load, row, token and LDS ranges against what the shape
allocates (tests/gather_plan_check.cpp)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_gather_launch_shapes_stay_in_bounds(tmp_path):
    exe = str(tmp_path / "gather_plan_check")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-o", exe,
                           os.path.join(HERE, "gather_plan_check.cpp")])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout[-3000:]
    assert "0 failures" in out.stdout
