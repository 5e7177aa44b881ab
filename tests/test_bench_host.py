"""Host-side logic of the benchmark script: host description, the
all-core CPU baseline, the single-GPU guard and the counter-summary keys. No
GPU is used."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_host_description():
    h = bench.host_description()
    assert h["nproc"] >= 1 and 1 <= h["usable_cpus"] <= h["nproc"] and isinstance(h["cpu_model"], str)


def test_all_core_baseline_splits_whole_segments():
    # parts of whole segments on several threads round-trip exactly
    import datagen
    x = datagen.ar2_uint16(50_003, 3, seed=7)
    dec, enc, parts = bench.cpu_baseline_all_cores(x, "fire", 1024, 4)
    assert parts == 4 and dec > 0 and enc > 0


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_counter_summary_is_keyed_like_the_bench_lookup():
    # the default stream workload (4,194,304 x 8 uint16, FIRE, 1024-row
    # segments) must find its HBM traffic entry under the kernel label the
    # bench line reports
    import json
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        d = json.load(fh)
    key = "k_decode_pc|" + bench.stream_workload_name(4194304, 8, "fire", 1024)
    assert key in d
    e = d[key]
    assert e["kernel"].startswith("spz::k_decode_pc<")
    assert e["bytes_per_launch"] > 0 and len(e["source_hash"]) == 16
