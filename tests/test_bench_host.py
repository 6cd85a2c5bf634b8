"""Host logic of bench.py, without a device: the byte model of the photon
merges, the roofline arithmetic, the rule that committed counter traffic
counts only for the sources it was taken from, and the refusal of a run
on several GPUs."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_merge_bytes_follow_the_work_counters():
    s = {"photon_items": 1000, "grid_cells": 7500, "candidates": 23800, "merges": 3700, "photon_continued": 0}
    # per photon: state (48) + U (4) + hit (8); per cell two bounds; one
    # packed position per candidate; 52 record bytes + a 3-float image
    # atomic (read and write) per accepted merge
    want = 1000 * 60 + 7500 * 8 + 23800 * 16 + 3700 * (52 + 24)
    assert bench.algorithmic_bytes(s, "photon_merge", 0, 0) == want


def test_roofline_is_bytes_per_launch_over_launch_time(monkeypatch):
    monkeypatch.setattr(bench, "committed_traffic", lambda name: 3.0e9)
    kernels = {"photon_merge": {"launches": 4, "ms": 2.0, "algorithmic_bytes": 4_000_000_000}}
    r = bench.roofline_of(kernels, "photon_merge")
    # 1e9 bytes per launch in 0.5 ms: 2000 GB/s of the 8000 GB/s peak
    assert r["achieved"] == pytest.approx(2000.0)
    assert r["frac"] == pytest.approx(0.25)
    assert r["avg_launch_us"] == pytest.approx(500.0)
    assert r["traffic"] == 3_000_000_000
    assert bench.roofline_of(kernels, "missing") is None


def test_committed_traffic_needs_the_profiled_sources(monkeypatch):
    path = os.path.join(ROOT, "profiles", "photon_merge_room_counters.txt")
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    monkeypatch.setattr(bench, "source_digest", lambda: kv["source_digest"])
    assert bench.committed_traffic("photon_merge") == float(kv["hbm_bytes_per_launch"])
    # fetch (calibrated) plus write bytes make the total
    assert int(kv["hbm_bytes_per_launch"]) == int(kv["hbm_fetch_bytes_per_launch"]) + int(
        kv["hbm_write_bytes_per_launch"])
    monkeypatch.setattr(bench, "source_digest", lambda: "0" * 16)
    assert bench.committed_traffic("photon_merge") is None
    assert bench.committed_traffic("no_such_kernel") is None


def test_committed_traffic_matches_the_current_sources():
    """The committed merge-kernel counters were taken from the sources in
    the tree (a kernel edit must come with new counters)."""
    assert bench.committed_traffic("photon_merge") is not None


def test_several_gpus_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
