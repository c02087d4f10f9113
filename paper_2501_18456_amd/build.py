"""Build libbmdca.so (HIP, gfx950) in-tree.

Every HIP source is compiled to an object file in parallel and linked into
paper_2501_18456_amd/libbmdca.so. Run as `python -m paper_2501_18456_amd.build`.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libbmdca.so")
PEAKS = os.path.join(HERE, "libbmdca_peaks.so")  # measurement aid of bench.py only
OBJDIR = os.path.join(HERE, "_build")
SOURCES = ["api.hip", "sampler.hip", "sampler_mh.hip", "sampler_w8.hip", "sampler_w12.hip", "stats.hip", "learn.hip",
           "reweight.hip", "scoring.hip", "equilibrium.hip", "decimation.hip"]

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Wall", "-Wno-unused-function",
    # packed FP32 instructions stay off everywhere (the host pass warns that it
    # does not know the feature; that is harmless)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(OBJDIR, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        text = "\n".join(ln for ln in text.splitlines() if "packed-fp32-ops" not in ln)
        if p.returncode != 0:
            failed.append(src)
            sys.stderr.write(text + "\n")
        elif verbose and text.strip():
            sys.stderr.write(text + "\n")
    if failed:
        raise RuntimeError("hipcc failed for: " + ", ".join(failed))
    tmp = OUT + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, OUT)
    # the benchmark's device throughput probe: a library of its own
    tmp = PEAKS + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC, *FLAGS, "-shared", "-o", tmp, os.path.join(CSRC, "peaks.hip")])
    os.replace(tmp, PEAKS)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
