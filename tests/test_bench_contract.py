"""Host-side parts of the benchmark contract: one GPU only, and the sweep
kernel's profiled HBM traffic reported only for the sources it was taken with."""
import hashlib
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_traffic_follows_the_source_digest(monkeypatch):
    h = hashlib.sha256()
    for f in bench.GATHER_TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    monkeypatch.setattr(bench, "GATHER_TRAFFIC", {"sha256": h.hexdigest(),
                                                  "bytes": {"precision": 123.0}})
    assert bench.gather_traffic("precision") == 123.0
    assert bench.gather_traffic("protein") is None
    monkeypatch.setattr(bench, "GATHER_TRAFFIC", {"sha256": "0" * 64,
                                                  "bytes": {"precision": 123.0}})
    assert bench.gather_traffic("precision") is None


def test_cpu_info_names_the_host():
    info = bench.cpu_info()
    assert info["nproc"] >= 1 and 1 <= info["omp_threads"] <= info["usable"]
