"""CPU tests of bench.py's host logic: the HBM traffic guard, the small-level
threshold it shares with the library, and the one-GPU refusal.

Nothing here touches a device.
"""
from __future__ import annotations

import os
import re
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _tuned(slots, tiles):
    return {"slots_per_lane": slots, "tiles_per_wave": tiles}


def test_traffic_only_for_the_measured_build_workload_and_tiling(monkeypatch):
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda: bench.ENUM_TRAFFIC["sources_sha256_16"])
    for (slots, tiles), (fetch, write) in bench.ENUM_TRAFFIC["kib_per_launch"].items():
        # FETCH_SIZE counts half of what a plain copy moves (x2), WRITE_SIZE all of it
        assert bench.enum_traffic_bytes("plain192", _tuned(slots, tiles)) == (fetch * 2 + write) * 1024
    assert bench.enum_traffic_bytes("plain128", _tuned(16, 4)) is None
    assert bench.enum_traffic_bytes("plain192", _tuned(4, 4)) is None
    assert bench.enum_traffic_bytes("plain192", None) is None


def test_traffic_is_refused_for_another_build(monkeypatch):
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda: "0000000000000000")
    assert bench.enum_traffic_bytes("plain192", _tuned(16, 4)) is None


def test_small_level_threshold_matches_the_library():
    # bench counts the dominant kernel's launches with the library's rule for
    # the levels that run with fewer lane sums
    text = open(os.path.join(ROOT, "paper_1911_08963_amd", "csrc", "bz_internal.h")).read()
    m = re.search(r"kSmallLevelComb\s*=\s*([0-9.]+)", text)
    assert m and float(m.group(1)) == bench.SMALL_LEVEL_COMB


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""
