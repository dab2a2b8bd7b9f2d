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


def test_group_rule_matches_the_library():
    # bench counts the dominant kernel's launches with the library's rule for
    # the levels whose full-rank Gamma_j share a launch
    api = open(os.path.join(ROOT, "paper_1911_08963_amd", "csrc", "bz_api.cpp")).read()
    m = re.search(r"kGroupMaxComb\s*=\s*([0-9.]+)", api)
    assert m and float(m.group(1)) == bench.GROUP_LEVEL_COMB
    kh = open(os.path.join(ROOT, "paper_1911_08963_amd", "csrc", "bz_kernels.h")).read()
    m = re.search(r"kMaxGroup\s*=\s*([0-9]+)", kh)
    assert m and int(m.group(1)) == bench.GROUP_MAX
    m = re.search(r"kMaxLevelTasks\s*=\s*([0-9]+)", kh)
    assert m and int(m.group(1)) == bench.LEVEL_GROUP_MAX
    m = re.search(r"kSpanMaxComb\s*=\s*([0-9.]+)", api)
    assert m and float(m.group(1)) == bench.SPAN_MAX_COMB
    # [192,64], 3 full-rank sets: levels 5 (7.6e6 sums, small variant), 6 (7.5e7, one
    # grouped launch), 7 and 8 (one launch per task)
    stats = [(j, g, 0, 0, 0) for g in (5, 6, 7, 8) for j in range(3)]
    assert bench.dominant_launches(stats, 64, 3) == 1 + 3 + 3
    # a partial Gamma_m runs alone
    assert bench.dominant_launches([(j, 6, 0, 0, 0) for j in range(3)], 64, 2) == 2
    # k = 40: levels 7 (1.9e7 sums) and 8 (7.7e7) share launches within each level
    # only (a later level's task is past the speculation cap), 9 (2.7e8) not at all
    stats = [(j, g, 0, 0, 0) for g in (6, 7, 8, 9) for j in range(2)]
    assert bench.dominant_launches(stats, 40, 2) == 1 + 1 + 2
    # a partial task in between ends a group
    assert bench.dominant_launches(stats, 40, 1) == 4 + 2
    # six full-rank sets: one level runs four tasks, then two, per launch
    assert bench.dominant_launches([(j, 6, 0, 0, 0) for j in range(6)], 64, 6) == 2
    stats = [(j, g, 0, 0, 0) for g in (7, 8, 9) for j in range(6)]
    assert bench.dominant_launches(stats, 40, 6) == 2 + 2 + 6
    # below the cap a group spans level ends (the rule itself, on small levels)
    old = bench.SMALL_LEVEL_COMB
    try:
        bench.SMALL_LEVEL_COMB = 1
        # k = 20, two sets: levels 2-4 (190, 1140, 4845 sums) in one launch of six tasks
        stats = [(j, g, 0, 0, 0) for g in (2, 3, 4) for j in range(2)]
        assert bench.dominant_launches(stats, 20, 2) == 1
    finally:
        bench.SMALL_LEVEL_COMB = old


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_paper_context_figures():
    # Table 2 (Sec. 4.6): mat023 with GAP/Guava on one core against the paper's D-Lex on 288 cores
    m23 = bench.PAPER_CONTEXT["mat023 [232,51,61]"]
    assert m23["Guava 3.12, 1 core"] == 456413.2 and m23["paper's D-Lex, 288 cores"] == 282.6
    assert bench.PAPER_CONTEXT["mat015 [150,77,17]"]["paper's D-Lex, 288 cores"] == 38.9


def test_serving_level_budget():
    import math

    from paper_1911_08963_amd import workloads
    for n, k, m_f, k_m in ((192, 96, 1, 40), (128, 64, 2, 0), (100, 45, 2, 10), (64, 32, 1, 0)):
        nsets = m_f + (1 if k_m else 0)
        for budget in (1e6, 1e9, 1e10):
            g = workloads.level_within(n, k, m_f, k_m, budget)
            cost = lambda lv: sum(nsets * math.comb(k, x) for x in range(1, lv + 1))
            assert g >= 1
            assert g == 1 or cost(g) <= budget
            assert g == k or cost(g + 1) > budget
