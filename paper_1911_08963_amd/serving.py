"""Serving driver: a Poisson stream of minimum-distance requests into a bz.Server.

Request i arrives at the i-th time of inputs.serve_arrivals (exponential gaps)
and carries the code inputs.serve_code(i). On arrival it is prepared on the
host (bz_prepare, host-only Gamma_j) and submitted at once, or, when the
server has no free slot or HBM budget, as soon as one frees up.

Random codes of the stream's shapes have very uneven costs (a few need 1e15
row combinations or more, far beyond what any device finishes while the
stream runs). A request whose estimated cost (workloads.estimated_cost)
exceeds cost_cap is therefore handled in one of two ways:
- over_cap="bound" (default): it is still served, with a per-request
  max_level: the deepest level whose estimated cumulative cost stays within
  bound_budget. It ends with status BZ_ELIMIT and the certified bounds
  L <= d <= U of the levels it completed, a partial answer the caller gets
  back like any other.
- over_cap="reject": it is refused on arrival (the status a caller would see
  is BZ_ELIMIT), and counted as a miss in the latency figures.

Latency of a request = its wait from arrival to submission (host preparation
and any admission wait) + the library's submission-to-completion time.
Every search runs in libbz; this module only paces arrivals and keeps score.
"""
from __future__ import annotations

import math
import time
from collections import deque

import numpy as np

from . import bz, inputs, workloads

N_BANDS = ((64, 96), (96, 128), (128, 160), (160, 193))


def _band(n: int) -> str:
    for lo, hi in N_BANDS:
        if lo <= n < hi:
            return f"n {lo}-{hi - 1}"
    return "other"


def _ops(res, W_full: int, W_partial: int, num_full: int) -> int:
    """int32 lane operations of the enumeration (2W + 1 per combination, W of each task's matrix)."""
    if res.stats:
        return sum(s[4] * (2 * (W_full if s[0] < num_full else W_partial) + 1) for s in res.stats)
    return res.combinations * (2 * W_full + 1)


def run(rate_hz: float = 200.0, duration_s: float = 60.0, seed: int = 7, cost_cap: float = 1e11,
        slots: int = 1024, stats: bool = False, keep_results: bool = False, progress=None,
        over_cap: str = "bound", bound_budget: float = 1e10, hbm_budget: int = 0,
        codes_per_launch: int = 0) -> dict:
    if over_cap not in ("bound", "reject"):
        raise ValueError("over_cap must be 'bound' or 'reject'")
    arrivals = inputs.serve_arrivals(rate_hz, duration_s, seed)
    requests = [inputs.serve_code(i) for i in range(len(arrivals))]   # drawn before the clock starts
    srv = bz.Server(slots=slots, stats=stats, hbm_budget=hbm_budget, codes_per_launch=codes_per_launch)
    lat_exact, lat_bound, results = [], [], {}
    submitted = rejected = deferred = errors = bounded = 0
    combos = ops = 0
    gaps = []                        # U - L of the bounded answers
    bands = {}                       # n band -> [arrivals, over the cap]
    queue = deque()                  # (index, code, arrival time, max_level, shape) waiting for admission
    live = {}                        # ticket -> (index, arrival time, submit time, shape)
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
                b = bands.setdefault(_band(c.n), [0, 0])
                b[0] += 1
                max_level = 0
                if est > cost_cap:
                    b[1] += 1
                    if over_cap == "reject":
                        rejected += 1
                        code.close()
                        i += 1
                        continue
                    max_level = workloads.level_within(c.n, c.k, code.num_full, code.partial_rank, bound_budget)
                shape = (code.W_full, code.W_partial, code.num_full)
                queue.append((i, code, t0 + arrivals[i], max_level, shape))
                i += 1
            while queue:
                idx, code, t_arr, max_level, shape = queue[0]
                t = srv.submit(code, max_level=max_level)
                if t is None:
                    deferred += 1
                    break
                submitted += 1
                live[t] = (idx, t_arr, time.perf_counter(), shape)
                queue.popleft()
                code.close()
            for t, res in srv.poll():
                idx, t_arr, t_sub, shape = live.pop(t)
                latency = (t_sub - t_arr) + res.search_s
                if res.status == bz.BZ_OK:
                    lat_exact.append(latency)
                elif res.status == bz.BZ_ELIMIT:
                    bounded += 1
                    lat_bound.append(latency)
                    gaps.append(res.upper_bound - res.lower_bound)
                else:
                    errors += 1
                    continue
                combos += res.combinations
                ops += _ops(res, *shape)
                t_last_done = time.perf_counter()
                if keep_results:
                    results[idx] = res
            if progress and now - last_report > 5.0:
                last_report = now
                progress(f"serving t={now - t0:6.1f}s arrived={i} submitted={submitted} rejected={rejected} "
                         f"in_flight={len(live)} queued={len(queue)} exact={len(lat_exact)} bounded={bounded}")
            if i < len(arrivals):
                wait = t0 + arrivals[i] - time.perf_counter()
                time.sleep(min(max(wait, 0.0), 200e-6))
            else:
                time.sleep(100e-6)
    finally:
        srv.close()
    wall = t_last_done - t0
    def pct(x, q):
        if not len(x):
            return None
        v = float(np.percentile(np.asarray(x) * 1e3, q))
        return v if math.isfinite(v) else None          # None: that percentile is a refused request
    served = lat_exact + lat_bound
    # every arrival counts: a refused request is a miss, its latency taken as infinite
    everyone = served + [math.inf] * rejected
    out = {
        "arrivals": int(len(arrivals)), "submitted": submitted, "rejected": rejected,
        "over_cap": over_cap, "cost_cap": cost_cap,
        "bound_budget": bound_budget if over_cap == "bound" else None,
        "exact": len(lat_exact), "bounded": bounded, "errors": errors,
        "deferred_submits": deferred, "slots": slots, "hbm_budget": hbm_budget,
        "codes_per_launch": codes_per_launch or None, "rate_hz": rate_hz, "duration_s": duration_s,
        "p50_ms": pct(everyone, 50) if everyone else None,
        "p99_ms": pct(everyone, 99) if everyone else None,
        "p50_ms_exact": pct(lat_exact, 50), "p99_ms_exact": pct(lat_exact, 99),
        "p50_ms_bounded": pct(lat_bound, 50), "p99_ms_bounded": pct(lat_bound, 99),
        "max_ms": pct(served, 100),
        "bounded_gap_mean": float(np.mean(gaps)) if gaps else None,
        "over_cap_by_band": {k: {"arrivals": v[0], "over_cap": v[1], "fraction": v[1] / v[0]}
                             for k, v in sorted(bands.items())},
        "codes_per_s": len(served) / wall if wall > 0 else None,
        "exact_codes_per_s": len(lat_exact) / wall if wall > 0 else None,
        "combinations": int(combos),
        "comb_per_s": combos / wall if wall > 0 else None,
        "lane_ops": int(ops),
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
    ap.add_argument("--over-cap", default="bound", choices=("bound", "reject"))
    ap.add_argument("--bound-budget", type=float, default=1e10)
    ap.add_argument("--slots", type=int, default=1024)
    ap.add_argument("--hbm-budget", type=int, default=0)
    ap.add_argument("--codes-per-launch", type=int, default=0)
    a = ap.parse_args()
    r = run(a.rate, a.duration, cost_cap=a.cost_cap, slots=a.slots, over_cap=a.over_cap,
            bound_budget=a.bound_budget, hbm_budget=a.hbm_budget, codes_per_launch=a.codes_per_launch,
            progress=lambda m: print(m, flush=True))
    print(json.dumps(r))
