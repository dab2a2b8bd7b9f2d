"""Serving driver: a Poisson stream of minimum-distance requests into a bz.Server.

Request i arrives at the i-th time of inputs.serve_arrivals (exponential gaps)
and carries the code inputs.serve_code(i). On arrival it is prepared on the
host (bz_prepare, host-only Gamma_j) and admitted unless its estimated cost
(workloads.estimated_cost) exceeds cost_cap: those are rejected, the status a
caller would see being BZ_ELIMIT. An admitted request is submitted at once, or,
when the server has no free slot or HBM budget, as soon as one frees up.

Latency of a request = its wait from arrival to submission (host preparation
and any admission wait) + the library's submission-to-completion time.
Every search runs in libbz; this module only paces arrivals and keeps score.
"""
from __future__ import annotations

import time
from collections import deque

import numpy as np

from . import bz, inputs, workloads


def run(rate_hz: float = 200.0, duration_s: float = 60.0, seed: int = 7, cost_cap: float = 1e11,
        slots: int = 1024, stats: bool = False, keep_results: bool = False, progress=None) -> dict:
    arrivals = inputs.serve_arrivals(rate_hz, duration_s, seed)
    requests = [inputs.serve_code(i) for i in range(len(arrivals))]   # drawn before the clock starts
    srv = bz.Server(slots=slots, stats=stats)
    lat, results = [], {}
    admitted = rejected = deferred = errors = 0
    combos = 0
    queue = deque()                  # (index, code, arrival time) waiting for admission
    live = {}                        # ticket -> (index, arrival time, submit time)
    i = 0
    t0 = time.perf_counter()
    last_report = t0
    t_last_done = t0
    try:
        while i < len(arrivals) or queue or live:
            now = time.perf_counter()
            while i < len(arrivals) and t0 + arrivals[i] <= now:
                c = requests[i]
                code = bz.Code(c.G, c.n, host_only=True)
                est = workloads.estimated_cost(c.n, c.k, code.num_full, code.partial_rank)
                if est > cost_cap:
                    rejected += 1
                    code.close()
                else:
                    admitted += 1
                    queue.append((i, code, t0 + arrivals[i]))
                i += 1
            while queue:
                idx, code, t_arr = queue[0]
                t = srv.submit(code)
                if t is None:
                    deferred += 1
                    break
                live[t] = (idx, t_arr, time.perf_counter())
                queue.popleft()
                code.close()
            for t, res in srv.poll():
                idx, t_arr, t_sub = live.pop(t)
                if res.status != bz.BZ_OK:
                    errors += 1
                    continue
                lat.append((t_sub - t_arr) + res.search_s)
                combos += res.combinations
                t_last_done = time.perf_counter()
                if keep_results:
                    results[idx] = res
            if progress and now - last_report > 5.0:
                last_report = now
                progress(f"serving t={now - t0:6.1f}s arrived={i} admitted={admitted} rejected={rejected} "
                         f"in_flight={len(live)} queued={len(queue)} done={len(lat)}")
            if i < len(arrivals):
                wait = t0 + arrivals[i] - time.perf_counter()
                time.sleep(min(max(wait, 0.0), 200e-6))
            else:
                time.sleep(100e-6)
    finally:
        srv.close()
    wall = t_last_done - t0
    lat_ms = np.asarray(lat) * 1e3
    out = {
        "arrivals": int(len(arrivals)), "admitted": admitted, "rejected": rejected,
        "deferred_submits": deferred, "completed": len(lat), "errors": errors,
        "cost_cap": cost_cap, "slots": slots, "rate_hz": rate_hz, "duration_s": duration_s,
        "p50_ms": float(np.percentile(lat_ms, 50)) if len(lat) else None,
        "p99_ms": float(np.percentile(lat_ms, 99)) if len(lat) else None,
        "mean_ms": float(lat_ms.mean()) if len(lat) else None,
        "max_ms": float(lat_ms.max()) if len(lat) else None,
        "codes_per_s": len(lat) / wall if wall > 0 else None,
        "combinations": int(combos),
        "comb_per_s": combos / wall if wall > 0 else None,
        "wall_s": wall,
    }
    if keep_results:
        out["results"] = results
    return out


if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--duration", type=float, default=60.0)
    ap.add_argument("--cost-cap", type=float, default=1e11)
    ap.add_argument("--slots", type=int, default=1024)
    a = ap.parse_args()
    r = run(a.rate, a.duration, cost_cap=a.cost_cap, slots=a.slots, progress=lambda m: print(m, flush=True))
    print(json.dumps(r))
