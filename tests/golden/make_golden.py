"""Writes tests/golden/plain_oracle.json from the CPU oracle only.

    python tests/golden/make_golden.py

For each plain workload: its generator draw count, (m_f, k_m), and the oracle's
result: d (when the run converges), the final bounds and the per-(Gamma_j, g)
statistics (min weight, count at min, combinations), in both the per-Gamma
and the per-level stop modes. The [192, 64] workload is run up to level 6.
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1911_08963_amd import inputs  # noqa: E402

RUNS = [("plain40", 0), ("plain128", 0), ("plain192", 6)]


def main():
    out = {}
    for name, max_level in RUNS:
        c = inputs.plain_code(name)
        entry = {"n": c.n, "k": c.k, "seed": c.seed, "draws": c.draws, "max_level": max_level}
        for mode, level_stop in (("per_gamma", False), ("per_level", True)):
            t0 = time.time()
            r = oracle.min_distance(c.G, c.n, level_stop=level_stop, max_level=max_level)
            entry[mode] = {
                "status": r.status, "d": r.d, "lower_bound": r.lower_bound,
                "upper_bound": r.upper_bound, "last_level": r.last_level,
                "num_full": r.num_full, "partial_rank": r.partial_rank,
                "combinations": r.combinations, "stats": [list(s) for s in r.stats],
                "oracle_seconds": round(time.time() - t0, 2),
            }
            print(name, mode, r.status, r.d, r.upper_bound, r.lower_bound, flush=True)
        out[name] = entry
    with open(os.path.join(HERE, "plain_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
