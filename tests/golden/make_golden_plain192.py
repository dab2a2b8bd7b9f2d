"""Writes tests/golden/plain192_oracle.json: the full Brouwer-Zimmermann run of
the [192, 64] workload by the multi-process CPU oracle (Alg. 3's prefix split,
cyclic over processes), calling only oracle/.

    python tests/golden/make_golden_plain192.py [nprocs]

About 2e12 combinations: roughly an hour on 8 cores.
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import parallel  # noqa: E402
from paper_1911_08963_amd import inputs  # noqa: E402


def main():
    nprocs = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    c = inputs.plain_code("plain192")
    t0 = time.time()

    def progress(j, g, mn, cnt, U, L):
        print(f"{time.time() - t0:8.1f}s task (j={j}, g={g}) min={mn} count={cnt} U={U} L={L}", flush=True)

    r = parallel.min_distance_parallel(c.G, c.n, nprocs=nprocs, prefix=3, progress=progress)
    out = {"n": c.n, "k": c.k, "seed": c.seed, "draws": c.draws, "d": r["d"],
           "lower_bound": r["lower_bound"], "upper_bound": r["upper_bound"],
           "combinations": r["combinations"], "stats": [list(s) for s in r["stats"]],
           "witness": [int(x) for x in r["witness"]], "oracle_seconds": round(r["seconds"], 1),
           "nprocs": r["nprocs"]}
    with open(os.path.join(HERE, "plain192_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("done d =", r["d"], flush=True)


if __name__ == "__main__":
    main()
