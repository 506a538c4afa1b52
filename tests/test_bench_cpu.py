"""Host-side contract of bench.py (no GPU): the one-GPU refusal, the default
schedule, and the guard that withholds the memory-traffic figure once the
dominant kernel's sources differ from the ones the counters were taken on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_default_steps_fill_every_lane_equally():
    old = sys.argv
    try:
        sys.argv = ["bench.py"]
        a = bench.parse()
    finally:
        sys.argv = old
    assert a.gpus == 1 and a.inflight >= 1
    assert a.steps % a.inflight == 0


def test_traffic_reported_only_for_the_counted_sources_and_schedule(monkeypatch):
    h = bench._kernel_source_hash()
    assert len(h) == 16
    b = bench.TRAFFIC["fields_per_step"]
    monkeypatch.setitem(bench.TRAFFIC, "src_sha256_prefix", h)
    assert bench._traffic(b) == bench.TRAFFIC["bytes_per_launch"]
    # another schedule puts another number of matrices into each launch
    assert bench._traffic(b + 1) is None
    monkeypatch.setitem(bench.TRAFFIC, "src_sha256_prefix", "0" * 16 if h != "0" * 16 else "1" * 16)
    assert bench._traffic(b) is None


def test_counted_schedule_is_the_default():
    old = sys.argv
    try:
        sys.argv = ["bench.py"]
        a = bench.parse()
    finally:
        sys.argv = old
    assert a.fields_per_step == bench.TRAFFIC["fields_per_step"]


def test_committed_traffic_matches_the_current_sources():
    """The stored counters belong to the LDS reduction as it is now (else
    the bench reports null traffic, which the contract also allows: this
    test keeps the two from drifting apart unnoticed)."""
    assert bench.TRAFFIC["src_sha256_prefix"] == bench._kernel_source_hash()
