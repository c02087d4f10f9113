"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the FP64 oracle, driven through every routine on small ragged inputs, and the
gather sampler's launch planner with its index-range checker.  Any
out-of-bounds access, leak or undefined operation makes the run fail."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    return subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.check_call(["gcc", "-std=c11", "-ffp-contract=off", *SAN, "-o", exe,
                           os.path.join(HERE, "oracle_sanitize_main.c"),
                           os.path.join(ROOT, "oracle", "bmdca_oracle.c"), "-lm"])
    out = _run(exe)
    assert out.returncode == 0, (out.stdout + out.stderr)[-4000:]
    assert "oracle sanitizer run ok" in out.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_gather_planner_under_sanitizers(tmp_path):
    exe = str(tmp_path / "gather_plan_san")
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-o", exe,
                           os.path.join(HERE, "gather_plan_check.cpp")])
    out = _run(exe)
    assert out.returncode == 0, (out.stdout + out.stderr)[-4000:]
    assert "0 failures" in out.stdout
