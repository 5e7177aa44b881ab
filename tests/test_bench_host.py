"""Host-side logic of the benchmark script: the seg_rows autotuner's choice
rule and the single-GPU guard. No GPU is used."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_pick_fastest_within_tolerance():
    sizes = {256: 1100, 512: 1009, 1024: 1005, 2048: 1001}
    times = {256: 1.0, 512: 2.0, 1024: 3.0, 2048: 4.0}
    # 256 is fastest but 10 % larger than the unsegmented 1000 bytes
    assert bench.pick_seg_rows(sizes, times, 1000) == 512


def test_pick_boundary_is_inclusive():
    sizes = {512: 1010, 1024: 1000}
    times = {512: 1.0, 1024: 2.0}
    assert bench.pick_seg_rows(sizes, times, 1000) == 512
    assert bench.pick_seg_rows({512: 1011, 1024: 1000}, times, 1000) == 1024


def test_pick_smallest_container_when_none_qualifies():
    sizes = {256: 1300, 512: 1200, 1024: 1150, 2048: 1160}
    times = {256: 1.0, 512: 2.0, 1024: 3.0, 2048: 0.5}
    assert bench.pick_seg_rows(sizes, times, 1000) == 1024


def test_pick_ties_go_to_first_listed():
    sizes = {512: 1000, 1024: 1000}
    times = {512: 1.0, 1024: 1.0}
    assert bench.pick_seg_rows(sizes, times, 1000) == 512
    assert bench.pick_seg_rows({1024: 1000, 512: 1000}, times, 1000) == 1024


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
