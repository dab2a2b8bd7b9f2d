"""Benchmark: row-combinations/s and time-to-d of the Brouwer-Zimmermann search on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload plain192] [--no-cpu]
                    [--batch 4096] [--serve-seconds 60]

One step is one complete minimum-distance computation of the workload's code:
bz_prepare (information sets, Gamma_j, upload), the level loop of Alg. 1 with
every enumeration launch, the reductions, and witness recovery. The code is
resident on the device when a step's search starts; the step also includes
its own prepare.
Printed: one JSON line with value = combinations enumerated per second of
wall time over the timed steps, ms_per_step = time-to-d, the roofline of the
enumeration kernel (int32 VALU: 2W+1 operations per combination, measured
with HIP events on the search stream) and the CPU oracle timed on a bounded
sample of the same code. Beside it: the paper's eight prefix schedules
against the default tiles (time-to-d), the batched workload in one persistent
launch against plain per-code launches (codes/s), and a Poisson serving
stream through the resident server (p50/p99 latency, codes/s).
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math

import numpy as np
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X int32 VALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one op per lane per clock)
PEAK_INT32_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

# HBM bytes per launch of the enumeration kernel on the [192,64] workload from
# rocprofv3 FETCH_SIZE and WRITE_SIZE (each scaled by what the counter reads for
# a plain copy of known size: x2 and x1), valid for the kernel sources whose
# hash is given and the tilings the counters were taken with, keyed by (slots
# per lane, tiles per resident wave); any other build or tiling reports traffic
# as unmeasured. Values: (FETCH_SIZE mean, WRITE_SIZE mean) in KiB per launch
# of the dominant kernel (the 15 working launches of a search on levels of at
# least 2^24 sums). With 16 lane sums per lane they are register spills of the
# lane setup written back, not data: the algorithmic bytes are 0.
ENUM_TRAFFIC = {"sources_sha256_16": "2055a62e14e4fd15", "workload": "plain192",
                "kib_per_launch": {(16, 4): (8899.34, 51262.12), (16, 8): (8922.06, 52215.45),
                                   (16, 16): (8983.04, 55241.33), (8, 8): (171.34, 100.29),
                                   (8, 4): (170.95, 100.33)}}


def enum_traffic_bytes(workload: str, tuned) -> float | None:
    """Scaled HBM bytes per enumeration launch for this build, workload and tiling, else None."""
    if kernel_sources_hash() != ENUM_TRAFFIC["sources_sha256_16"] or workload != ENUM_TRAFFIC["workload"]:
        return None
    key = ((tuned or {}).get("slots_per_lane"), (tuned or {}).get("tiles_per_wave"))
    if key not in ENUM_TRAFFIC["kib_per_launch"]:
        return None
    fetch, write = ENUM_TRAFFIC["kib_per_launch"][key]
    return (fetch * 2 + write) * 1024
# Levels below this many sums use fewer lane sums per lane (the library's rule
# for a single search), hence another variant of the enumeration kernel.
SMALL_LEVEL_COMB = 1 << 24
# Levels below this many sums run up to GROUP_MAX full-rank Gamma_j in one launch
# (the library's rule); above it every task is a launch of its own.
GROUP_LEVEL_COMB = 1 << 27
GROUP_MAX = 4
LEVEL_GROUP_MAX = 8
SPAN_MAX_COMB = 1 << 24


def dominant_launches(stats, k: int, m_f: int) -> int:
    """Launches of the dominant enumeration variant (levels of at least 2^24 sums, 16
    lane sums per lane: W <= 4) that a search with these per-task records (in Alg. 1's
    order) made, by the library's rule: one per task from 2^27 sums up and per partial
    task; below that, consecutive full-rank tasks share a launch, up to LEVEL_GROUP_MAX
    when they span a level's end (while the later levels' tasks hold at most
    SPAN_MAX_COMB sums: never for this variant), else up to GROUP_MAX of one level (the library's
    shared-memory and window limits never bind on the bench's workloads). Launches
    enqueued past the stop return at once and are not counted."""
    recs = list(stats)

    def groupable(s):
        cb = math.comb(k, s[1])
        return SMALL_LEVEL_COMB <= cb < GROUP_LEVEL_COMB and s[0] < m_f

    n = p = 0
    while p < len(recs):
        s = recs[p]
        if math.comb(k, s[1]) < SMALL_LEVEL_COMB:
            p += 1
            continue
        n += 1
        if not groupable(s):
            p += 1
            continue
        span, later = 1, 0
        while span < LEVEL_GROUP_MAX and p + span < len(recs) and groupable(recs[p + span]):
            if recs[p + span][1] != s[1]:
                later += math.comb(k, recs[p + span][1])
                if later > SPAN_MAX_COMB:
                    break
            span += 1
        if recs[p + span - 1][1] != s[1]:
            p += span
            continue
        grp = 1
        while grp < GROUP_MAX and p + grp < len(recs) and groupable(recs[p + grp]) and recs[p + grp][1] == s[1]:
            grp += 1
        p += grp
    return n
KERNEL_SOURCES = ("bz_kernels.hip", "bz_tile.h", "bz_kernels.h", "bz_internal.h", "bz_plan.cpp")


def kernel_sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1911_08963_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]

WORKLOADS = {
    "plain192": "random binary [192,64] rate-1/3 code, G = [I_64 | R1 | R2], R iid Bernoulli(1/2) "
                "from seed 3 (redrawn until R1 and R2 are invertible), 3 disjoint information sets, "
                "full time-to-d",
    "plain128": "random binary [128,64] code, G = [I_64 | R], R iid Bernoulli(1/2) from seed 2 "
                "(redrawn until R is invertible), 2 disjoint information sets, full time-to-d",
}


def _oracle_code(args):
    """One complete oracle search (run in a worker process): (d, combinations, seconds)."""
    import oracle
    G, n = args
    t = time.perf_counter()
    r = oracle.min_distance(G, n)
    return r.d, r.combinations, time.perf_counter() - t


def cpu_codes_rate(pool, nprocs: int, codes, gpu_d, gpu_comb, max_comb: float, seconds: float) -> dict:
    """The oracle on a bounded sample of a workload's codes: complete searches, in the
    workload's order, of the codes whose search enumerates at most max_comb combinations
    (one code per process, nprocs at a time), until `seconds` have passed. Each d is
    checked against the GPU's."""
    import itertools
    sample = [(c.G, c.n, d) for c, d, cb in zip(codes, gpu_d, gpu_comb) if cb <= max_comb]
    it = iter(sample)
    t0 = time.perf_counter()
    done = comb = 0
    while time.perf_counter() - t0 < seconds:
        chunk = list(itertools.islice(it, nprocs * 2))
        if not chunk:
            break
        for (G, n, d), (od, cb, _) in zip(chunk, pool.map(_oracle_code, [(G, n) for G, n, _ in chunk])):
            assert od == d, "oracle and GPU disagree on d"
            done += 1
            comb += cb
    wall = time.perf_counter() - t0
    return {"codes": done, "combinations": comb, "wall_s": wall, "cores": nprocs,
            "comb_per_s": comb / wall, "codes_per_s_on_sample": done / wall,
            "sample": f"complete oracle searches of the first {done} codes, in workload order, whose search "
                      f"enumerates at most {max_comb:.0e} combinations, {nprocs} processes (one code each)"}


def batch_comparison(bz, inputs, count: int, cap: float, autotune: bool = True, pool=None,
                     nprocs: int = 1, cpu_seconds: float = 10.0, plain: bool = True) -> dict:
    """codes/s of one bz_min_distance_batch call against bz_min_distance per code."""
    import torch

    from paper_1911_08963_amd import workloads
    t = time.perf_counter()
    kept, drawn, est = workloads.select(inputs.batch_code, lambda c: bz.prepare_host(c.G, c.n)[1:3],
                                        count, cap)
    objs = [bz.Code(c.G, c.n) for c in kept]
    setup = time.perf_counter() - t
    tiles = None
    if autotune:
        # tiles per task, picked by timing the first 512 codes
        tiles, _ = bz.autotune_batch(objs[: min(512, len(objs))])
        print(f"autotune batch: {tiles} tiles per task", file=sys.stderr, flush=True)
    bz.min_distance_batch(objs[: min(64, len(objs))])            # warm-up: code objects, graph path
    torch.cuda.synchronize()
    t = time.perf_counter()
    outs, sts = bz.min_distance_batch(objs)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t
    assert all(s == 0 for s in sts), "batched search failed"
    tp = float("nan")
    if plain:
        t = time.perf_counter()
        plain_res = [bz.min_distance(o) for o in objs]
        torch.cuda.synchronize()
        tp = time.perf_counter() - t
        mism = sum(1 for a, b in zip(outs, plain_res) if a.d != b.d)
        assert mism == 0, f"{mism} codes differ between batched and plain"
    comb = sum(o.combinations for o in outs)
    # algorithmic work: 2W + 1 int32 operations per combination, W of each task's matrix
    ops = sum(s[4] * (2 * (o_.W_full if s[0] < o_.num_full else o_.W_partial) + 1)
              for o_, r in zip(objs, outs) for s in r.stats)
    assert sum(s[4] for r in outs for s in r.stats) == comb, "per-task records cover every combination"
    kern = outs[0].kernel_s
    print(f"batch: {len(objs)} codes ({drawn} drawn, setup {setup:.1f} s): batched {tb:.3f} s "
          f"(kernel {kern:.3f} s), plain {tp:.3f} s", file=sys.stderr, flush=True)
    for o in objs:
        o.close()
    cpu = None
    if pool is not None:
        cpu = cpu_codes_rate(pool, nprocs, kept, [o.d for o in outs], [o.combinations for o in outs],
                             2e8, cpu_seconds)
        cpu["codes_per_s_at_workload_mean"] = cpu["comb_per_s"] / (comb / len(outs))
        cpu["kind"] = "oracle"
        print(f"batch cpu baseline: {cpu['codes']} codes, {cpu['comb_per_s']:.3e} comb/s on {nprocs} cores",
              file=sys.stderr, flush=True)
    return {
        "workload": "batched: random binary codes, n ~ U{48..160}, rho ~ U[0.33, 0.6], k = round(n rho), "
                    "seeds 1000000+i, kept when the estimated cost is <= cap",
        "codes": len(objs), "drawn": drawn, "cost_cap": cap, "combinations": comb,
        "batched_s": tb, "plain_s": tp if plain else None, "tiles_per_task": tiles if tiles else 64,
        "batched_codes_per_s": len(objs) / tb, "plain_codes_per_s": len(objs) / tp if plain else None,
        "speedup": tp / tb if plain else None, "batched_combinations_per_s": comb / tb,
        "kernel_s": kern,
        "roofline": {"bound": "alu", "kernel": "bz_batch_kernel (one graph launch, with witness recovery)",
                     "ops": ops, "ops_per_combination": ops / comb,
                     "achieved": ops / kern / 1e12, "peak": PEAK_INT32_TOPS,
                     "unit": "TOP/s (int32 lane operations)", "frac": ops / kern / 1e12 / PEAK_INT32_TOPS,
                     "frac_of_wall": ops / tb / 1e12 / PEAK_INT32_TOPS},
        "cpu_baseline": cpu,
        "d_histogram": {str(d): int(n) for d, n in zip(*np.unique([o.d for o in outs], return_counts=True))},
    }


# Prefix sizes for the paper's schedules on this GPU's 5-8k waves: the fastest of
# a sweep on each workload (absolute for D-*, relative to g for S-*).
SCHED_PREFIX = {"plain192": {"D": 4, "S": 6}, "plain128": {"D": 2, "S": 5}}


def schedules_comparison(bz, c, workload: str, d: int) -> dict:
    """The paper's eight distributed schedules (Sec. 3) with the device's waves as workers,
    against the default equal-cost tiles: time-to-d of the same code, one run each."""
    pre = SCHED_PREFIX[workload]
    code = bz.Code(c.G, c.n)
    out = {"workload": workload, "prefix": {"dynamic (absolute)": pre["D"], "static (relative)": pre["S"]},
           "seconds": {}}
    r = bz.min_distance(code)
    out["seconds"]["tiles"] = r.search_s
    for name in ("D-Lex", "D-Lex-2cm", "D-Lle", "D-Lle-2cm", "S-Lex", "S-Lex-Snc", "S-Lle", "S-Lle-Snc"):
        r = bz.min_distance(code, schedule=name, prefix=pre[name[0]])
        assert r.d == d
        out["seconds"][name] = r.search_s
        print(f"schedule {name}: {r.search_s:.3f} s", file=sys.stderr, flush=True)
    code.close()
    best = min((v, k) for k, v in out["seconds"].items() if k != "tiles")
    out["best_schedule"] = best[1]
    out["tiles_speedup_over_best"] = best[0] / out["seconds"]["tiles"]
    return out


def time_to_d_small(bz, inputs, name: str, runs: int) -> dict:
    """Median time-to-d of a small plain workload over many runs (prepare and search split),
    with its int32 VALU roofline figures: (2W+1) x combinations over the median kernel time
    (the search's launches, timed with HIP events) and over the median time-to-d."""
    c = inputs.plain_code(name)
    tot, prep, srch, kern, ds, combs = [], [], [], [], set(), set()
    W = 0
    for _ in range(runs):
        t = time.perf_counter()
        code = bz.Code(c.G, c.n)
        r = bz.min_distance(code)
        tot.append(time.perf_counter() - t)
        W = code.W_full
        prep.append(r.prepare_s)
        srch.append(r.search_s)
        kern.append(r.kernel_s)
        ds.add(r.d)
        combs.add(r.combinations)
        code.close()
    assert len(ds) == 1 and len(combs) == 1
    med = lambda x: float(np.median(x))
    comb = combs.pop()
    ops = comb * (2 * W + 1)
    return {"workload": name, "n": c.n, "k": c.k, "d": ds.pop(), "runs": runs, "median_s": med(tot),
            "prepare_s": med(prep), "search_s": med(srch), "kernel_s": med(kern), "combinations": comb,
            "roofline": {"bound": "alu", "kernel": "bz_enum_kernel", "ops_per_combination": 2 * W + 1,
                         "achieved": ops / med(kern) / 1e12, "peak": PEAK_INT32_TOPS,
                         "unit": "TOP/s (int32 lane operations)",
                         "frac": ops / med(kern) / 1e12 / PEAK_INT32_TOPS,
                         "frac_of_time_to_d": ops / med(tot) / 1e12 / PEAK_INT32_TOPS}}


def cpu_oracle_rate(c, max_level: int, min_seconds: float, pool=None, nprocs: int = 1):
    """Combinations/s of the oracle on levels 1..max_level of the code, repeated for min_seconds."""
    import oracle
    from oracle import parallel
    t = time.perf_counter()
    done = reps = 0
    while reps == 0 or time.perf_counter() - t < min_seconds:
        if pool is None:
            ro = oracle.min_distance(c.G, c.n, max_level=max_level)
            done += ro.combinations
        else:
            ro = parallel.min_distance_parallel(c.G, c.n, nprocs=nprocs, max_level=max_level, pool=pool)
            done += ro["combinations"]
        reps += 1
    dt = time.perf_counter() - t
    return done / dt, done, reps, dt


# The paper's own end-to-end figures (Table 2, Sec. 4.6), for context only: its
# codes are not available, and its hardware is a 2009-era CPU cluster.
PAPER_CONTEXT = {
    "source": "arXiv:1911.08963, Table 2 (Sec. 4.6): time to d, seconds",
    "mat023 [232,51,61]": {"Guava 3.12, 1 core": 456413.2, "Magma 2.22-3, 1 core": 503984.2,
                           "Magma, 6 cores": 85341.1, "paper's D-Lex, 288 cores": 282.6},
    "mat015 [150,77,17]": {"Guava 3.12, 1 core": 40804.3, "Magma 2.22-3, 1 core": 53052.9,
                           "Magma, 6 cores": 9562.8, "paper's D-Lex, 288 cores": 38.9},
    "summary": "about 5 days with GAP/Guava against under 5 minutes on 288 cores (24 nodes of 2 Xeon X5560, "
               "InfiniBand) for mat023; the codes are not public, so this build measures random codes",
}
# Oracle process pools are sized to the CPUs the GPU machine grants one GPU (16), whatever
# os.cpu_count() reports there; a smaller host uses all its cores.
CORES_NOTE = "oracle processes = min(16, os.cpu_count()): the GPU box grants one GPU 16 CPUs"


def serving_runs(args, pool, nprocs) -> dict:
    """The Poisson stream through the resident server (default: every arrival served, requests
    over the cost cap limited to a level budget), then two shorter variants: an HBM budget that
    binds admission, and a small codes_per_launch that forces kernel relaunches."""
    from paper_1911_08963_amd import serving
    say = lambda m: print(m, file=sys.stderr, flush=True)
    sv = serving.run(args.serve_rate, args.serve_seconds, cost_cap=args.serve_cap, progress=say,
                     keep_results=pool is not None)
    sv["workload"] = ("serving: Poisson arrivals (seed 7), request i a random binary code from seed "
                      "2000000+i with n ~ U{64..192}, k ~ U{ceil(n/3)..floor(n/2)}; every arrival is "
                      "served; requests whose estimated cost exceeds cost_cap run only the levels that fit "
                      "bound_budget and return their certified bounds (status ELIMIT)")
    sv["roofline"] = {"bound": "alu", "kernel": "bz_serve_kernel (resident for the whole stream)",
                      "achieved": sv["lane_ops"] / sv["wall_s"] / 1e12, "peak": PEAK_INT32_TOPS,
                      "unit": "TOP/s (int32 lane operations)",
                      "frac": sv["lane_ops"] / sv["wall_s"] / 1e12 / PEAK_INT32_TOPS,
                      "note": "over the stream's wall time: bounded by the offered load, not the kernel"}
    results = sv.pop("results", None)
    if pool is not None and results:
        from paper_1911_08963_amd import inputs
        idx = sorted(i for i, r in results.items() if r.status == 0)
        codes = [inputs.serve_code(i) for i in idx]
        cpu = cpu_codes_rate(pool, nprocs, codes, [results[i].d for i in idx],
                             [results[i].combinations for i in idx], 2e8, args.cpu_min_seconds)
        exact_comb = sum(results[i].combinations for i in idx)
        cpu["codes_per_s_at_workload_mean"] = cpu["comb_per_s"] / (exact_comb / max(1, len(idx)))
        cpu["kind"] = "oracle"
        sv["cpu_baseline"] = cpu
        say(f"serving cpu baseline: {cpu['codes']} codes, {cpu['comb_per_s']:.3e} comb/s on {nprocs} cores")
    if args.serve_variants_seconds > 0:
        sv["variants"] = {}
        # a request of this stream needs at most about 16 KiB of device memory (Gamma_j rows and
        # their prefix XORs, full rows, code state, task records): 32 KiB admits two at a time
        for name, kw in (("hbm_budget_binding", {"hbm_budget": 32 * 1024}),
                         ("codes_per_launch_256", {"codes_per_launch": 256})):
            v = serving.run(args.serve_rate, args.serve_variants_seconds, cost_cap=args.serve_cap,
                            progress=say, **kw)
            sv["variants"][name] = {k: v[k] for k in (
                "arrivals", "exact", "bounded", "errors", "deferred_submits", "hbm_budget", "codes_per_launch",
                "p50_ms", "p99_ms", "p50_ms_exact", "p99_ms_exact", "codes_per_s", "duration_s")}
    return sv


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="plain192", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--cpu-max-level", type=int, default=6)
    ap.add_argument("--cpu-min-seconds", type=float, default=10.0,
                    help="repeat each CPU-oracle sample until this much time has accumulated")
    ap.add_argument("--cpu-procs", type=int, default=0,
                    help="processes of the multi-process oracle (0 = min(16, cpu count))")
    ap.add_argument("--small-runs", type=int, default=100,
                    help="runs of the [40,20] and [128,64] workloads for their median time-to-d (0 skips)")
    ap.add_argument("--batch", type=int, default=4096,
                    help="codes in the batched-vs-plain comparison (0 skips it)")
    ap.add_argument("--no-batch-plain", dest="batch_plain", action="store_false",
                    help="skip the per-code plain searches of the batch comparison (for profiling runs)")
    ap.add_argument("--valu-probe", action="store_true",
                    help="only run the int32 issue-rate probe and print its rate (for profiling runs)")
    ap.add_argument("--batch-cap", type=float, default=1e10,
                    help="keep batched-workload codes whose estimated cost is at most this")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the Poisson serving stream (0 skips it)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-cap", type=float, default=1e11,
                    help="serving: requests whose estimated cost exceeds this run only the levels within "
                         "a 1e10-combination budget and return bounds")
    ap.add_argument("--serve-variants-seconds", type=float, default=15.0,
                    help="length of each of the two serving variants (binding HBM budget, kernel "
                         "relaunch every 256 requests); 0 skips them")
    ap.add_argument("--no-count", dest="count_min_weight", action="store_false",
                    help="skip counting the workload's minimum-weight codewords")
    ap.add_argument("--no-schedules", dest="schedules", action="store_false",
                    help="skip the paper's eight prefix schedules (about 15 s)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="use the fixed rules for slots per lane, tile size and tiles per task")
    ap.add_argument("--tiling", default="", metavar="SLOTS,TILES_PER_WAVE",
                    help="install this tiling of the plain search instead of tuning it")
    ap.add_argument("--copy-ref", type=int, default=0, metavar="BYTES",
                    help="only run a device-to-device copy of BYTES three times (calibrates HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the search shards by "
              "combination rank ranges across GPUs, which this library does not do.", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    pool, nprocs = None, 1
    if not args.no_cpu and not args.copy_ref:
        # the oracle's worker processes are forked before anything touches the GPU
        import multiprocessing as mp
        nprocs = args.cpu_procs or min(16, os.cpu_count() or 1)
        pool = mp.get_context("fork").Pool(nprocs)

    import torch

    from paper_1911_08963_amd import inputs
    if not os.path.exists(os.path.join(ROOT, "paper_1911_08963_amd", "libbz.so")):
        from paper_1911_08963_amd import build as _b
        _b.build()
    from paper_1911_08963_amd import bz

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_ref:
        src = torch.empty(args.copy_ref, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_ref_bytes": args.copy_ref, "launches": 3}), flush=True)
        return
    if args.valu_probe:
        rate, secs = ctypes.c_double(), ctypes.c_double()
        assert bz.lib().bz_debug_valu_rate(0, ctypes.byref(rate), ctypes.byref(secs)) == 0
        print(json.dumps({"valu_probe_lane_ops_per_s": rate.value, "seconds": secs.value}), flush=True)
        return
    c = inputs.plain_code(args.workload)
    tuned = None
    if args.tiling:
        # a fixed (slots per lane, tiles per wave), for profiles that must match a tuned run
        sl, tw = (int(x) for x in args.tiling.split(","))
        probe = bz.Code(c.G, c.n)
        bz.autotune_set(probe.W_full, sl, tw)
        tuned = bz.autotune_get(probe.W_full)
        probe.close()
    elif args.autotune:
        # the chunk size and lane sums per lane of this shape, picked by timing
        probe = bz.Code(c.G, c.n)
        tuned = bz.autotune(probe.W_full, probe.k)
        probe.close()
        print(f"autotune W={tuned['W']} k={tuned['k']}: slots {tuned['slots_per_lane']}, tiles per wave "
              f"{tuned['tiles_per_wave']} ({tuned['comb_per_s']:.3e} comb/s vs {tuned['default_comb_per_s']:.3e} "
              "with the fixed rule)", file=sys.stderr, flush=True)

    probe = bz.Code(c.G, c.n, host_only=True)
    code_mf = probe.num_full                      # full-rank Gamma_j (they share small-level launches)
    probe.close()

    def one_step():
        code = bz.Code(c.G, c.n)
        r = bz.min_distance(code)
        W = code.W_full
        code.close()
        return r, W

    for i in range(args.warmup):
        r, _ = one_step()
        print(f"warmup {i}: d={r.d} combinations={r.combinations} search_s={r.search_s:.3f}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for i in range(args.steps):
        r, W = one_step()
        results.append(r)
        print(f"step {i}: d={r.d} combinations={r.combinations} search_s={r.search_s:.3f} "
              f"kernel_s={r.kernel_s:.3f}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    ds = {r.d for r in results}
    assert len(ds) == 1, f"d differs across steps: {ds}"
    d = ds.pop()
    for r in results:
        assert int(np.bitwise_count(r.witness).sum()) == d
    comb = sum(r.combinations for r in results)
    kern = sum(r.kernel_s for r in results)
    # Levels of fewer than 2^24 sums run a variant with fewer lane sums (a few
    # short launches, under 0.3 % of the kernel time); the per-launch figures
    # are those of the dominant kernel, the launches on the larger levels.
    big = [s for r in results for s in r.stats if math.comb(c.k, s[1]) >= SMALL_LEVEL_COMB]
    launches = sum(dominant_launches(r.stats, c.k, code_mf) for r in results)
    comb_big = sum(s[4] for s in big)
    ops = comb * (2 * W + 1)
    achieved = ops / kern / 1e12
    line = {
        "metric": "row-combinations/s (XOR+popcount), time-to-d",
        "value": comb / wall,
        "unit": "combinations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "n": c.n, "k": c.k, "seed": c.seed,
                   "d": d, "combinations_per_step": comb // args.steps},
        "time_to_d_s": sorted(r.search_s for r in results)[len(results) // 2],
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_INT32_TOPS,
            "unit": "TOP/s (int32 lane operations)",
            "frac": achieved / PEAK_INT32_TOPS,
            "traffic": enum_traffic_bytes(args.workload, tuned),
            "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "algorithmic_bytes_per_launch": 0,
            "kernel": "bz_enum_kernel",
            "ops_per_combination": 2 * W + 1,
            "avg_launch_ms": kern / launches * 1e3,
            "avg_combinations_per_launch": comb_big / launches,
            "launches_per_step": launches / args.steps,
        },
        "autotune": tuned,
    }
    line["paper_context"] = PAPER_CONTEXT
    line["time_to_d_s"] = {"plain192": {
        "workload": args.workload, "n": c.n, "k": c.k, "d": d, "runs": args.steps,
        "median_s": float(np.median([r.prepare_s + r.search_s for r in results])),
        "prepare_s": float(np.median([r.prepare_s for r in results])),
        "search_s": float(np.median([r.search_s for r in results]))}}
    line["roofline_by_config"] = {"plain192": dict(line["roofline"], frac_of_time_to_d=ops / wall / 1e12 /
                                                   PEAK_INT32_TOPS)}
    if args.small_runs:
        for name in ("plain40", "plain128"):
            t = time_to_d_small(bz, inputs, name, args.small_runs)
            line["roofline_by_config"][name] = t.pop("roofline")
            line["time_to_d_s"][name] = t
    if args.count_min_weight:
        # the number of codewords of weight d: the search continued until the
        # certified bound passes d, weight-d sums collected and de-duplicated
        code = bz.Code(c.G, c.n)
        cnt = bz.count_codewords(code, d, cap=1 << 16)
        code.close()
        for x in cnt["codewords"]:
            assert int(np.bitwise_count(x).sum()) == d
        line["min_weight_codewords"] = {"workload": args.workload, "weight": d, "count": cnt["count"],
                                        "hits": cnt["hits"], "combinations": cnt["combinations"],
                                        "last_level": cnt["last_level"], "seconds": cnt["search_s"]}
        print(f"codewords of weight {d}: {cnt['count']} ({cnt['search_s']:.3f} s)", file=sys.stderr, flush=True)
    if args.schedules and args.workload in SCHED_PREFIX:
        line["schedules"] = schedules_comparison(bz, c, args.workload, d)
    if args.batch:
        line["batch"] = batch_comparison(bz, inputs, args.batch, args.batch_cap, args.autotune,
                                         pool, nprocs, args.cpu_min_seconds, args.batch_plain)
        line["roofline_by_config"]["batch"] = line["batch"]["roofline"]
    if args.serve_seconds > 0:
        line["serving"] = serving_runs(args, pool, nprocs)
        line["roofline_by_config"]["serving"] = line["serving"]["roofline"]
    if not args.no_cpu:
        v1, n1, r1, t1 = cpu_oracle_rate(c, args.cpu_max_level, args.cpu_min_seconds)
        vp, np_, rp, tp = cpu_oracle_rate(c, args.cpu_max_level, args.cpu_min_seconds, pool, nprocs)
        # the oracle's own time-to-d: plain40 on one core, plain128 on the pool,
        # plain192's full run as cached with the golden file
        import oracle
        from oracle import parallel
        import statistics
        c40 = inputs.plain_code("plain40")
        t40 = []
        for _ in range(20):
            t0 = time.perf_counter()
            oracle.min_distance(c40.G, c40.n)
            t40.append(time.perf_counter() - t0)
        c128 = inputs.plain_code("plain128")
        t0 = time.perf_counter()
        r128 = parallel.min_distance_parallel(c128.G, c128.n, nprocs=nprocs, pool=pool)
        t128 = time.perf_counter() - t0
        pool.close()
        with open(os.path.join(ROOT, "tests", "golden", "plain192_oracle.json")) as fh:
            g192 = json.load(fh)
        oracle_ttd = {
            "plain40": {"seconds": statistics.median(t40), "cores": 1, "runs": 20},
            "plain128": {"seconds": t128, "cores": nprocs, "d": r128["d"]},
            "plain192": {"seconds": g192["oracle_seconds"], "cores": g192["nprocs"],
                         "note": "the full run cached with tests/golden/plain192_oracle.json, "
                                 "measured once on the build machine, not this host"},
        }
        line["cpu_baseline"] = {
            "value": vp, "unit": "combinations/s", "cores": nprocs, "kind": "oracle",
            "cores_note": CORES_NOTE,
            "sample": f"C oracle on the same code, levels 1-{args.cpu_max_level} of all 3 Gamma_j, "
                      f"in {nprocs} processes splitting each level's lex prefixes cyclically (Alg. 3); "
                      f"{rp} repetitions ({np_} combinations in {tp:.1f} s)",
            "single_core": {"value": v1, "cores": 1,
                            "sample": f"the same levels single-threaded, {r1} repetitions ({n1} combinations "
                                      f"in {t1:.1f} s)"},
            "time_to_d_s": oracle_ttd,
        }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
