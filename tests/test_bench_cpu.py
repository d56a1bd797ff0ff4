"""CPU-side parts of bench.py: the one-GPU guard and the oracle baselines on tiny samples."""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_oracle_baselines_report_their_sample(orc):
    sys.path.insert(0, ROOT)
    import bench

    for r in (bench.cpu_d3q19(n=8, steps=1), bench.cpu_batched(ndom=2, steps=1)):
        assert r["value"] > 0 and r["unit"] == "MLUPS" and r["kind"] == "oracle"
        assert r["cores"] >= 1 and r["sample"]


def test_traffic_records_name_their_kernel_sources():
    sys.path.insert(0, ROOT)
    import json

    import bench

    with open(bench.TRAFFIC_FILE) as fh:
        recs = json.load(fh)
    assert recs
    for name, rec in recs.items():
        assert rec["kind"] in bench.KERNEL_SOURCES, name
        assert rec["read_bytes_per_launch"] > 0 and rec["write_bytes_per_launch"] > 0, name
        assert len(rec["source_sha"]) == 16, name


def test_cpu_model_names_the_host():
    sys.path.insert(0, ROOT)
    import bench

    m = bench.cpu_model()
    assert "logical processors visible" in m and len(m) > 30
