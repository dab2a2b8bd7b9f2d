"""Multi-process CPU oracle: the paper's static prefix split -- TEST INFRASTRUCTURE.

Each (Gamma_j, g) task is cut into prefixes (Alg. 3) and the prefixes are dealt
cyclically to worker processes (the static S-Lex distribution of Sec. 3.3).
Every task is completed before the bounds are checked, so merging the workers'
(min, count) gives exactly the single-process per-task statistics, and replaying
the stop rule of Alg. 1 (with the per-Gamma check) on the merged minima gives
the same d. Used to obtain d for workloads too large for one core, and as the
all-cores CPU baseline.
"""
from __future__ import annotations

import ctypes
import multiprocessing as mp
import os
import time

import numpy as np

from . import OR_NW, OR_OK, _load, binomial, certified_bound, level_bound, prepare


class _TaskResult(ctypes.Structure):
    _fields_ = [("min_weight", ctypes.c_uint32), ("_pad", ctypes.c_uint32),
                ("count_at_min", ctypes.c_uint64), ("combinations", ctypes.c_uint64),
                ("witness", ctypes.c_uint64 * OR_NW)]


def _lib():
    lib = _load()
    if not hasattr(lib, "_task_typed"):
        P = ctypes.POINTER
        lib.or_task.argtypes = [P(ctypes.c_uint64), ctypes.c_uint32, ctypes.c_uint32,
                                ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                P(_TaskResult)]
        lib.or_task.restype = ctypes.c_int
        lib.or_prefix_sequence.argtypes = [ctypes.c_uint32, ctypes.c_uint32, P(ctypes.c_int32),
                                           ctypes.c_uint32, P(ctypes.c_int32), ctypes.c_uint64]
        lib.or_prefix_sequence.restype = ctypes.c_int64
        lib.or_prefix_count.argtypes = [ctypes.c_uint32] * 3
        lib.or_prefix_count.restype = ctypes.c_int64
        lib._task_typed = True
    return lib


def task_share(G: np.ndarray, n: int, matrix: int, g: int, p: int, part: int, nparts: int):
    """One worker's share of task (Gamma_matrix, g): (min, count, combinations, witness)."""
    lib = _lib()
    G = np.ascontiguousarray(G, dtype=np.uint64)
    k, ld = G.shape
    tr = _TaskResult()
    st = lib.or_task(G.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), k, n, ld, matrix, g, p,
                     part, nparts, ctypes.byref(tr))
    if st != OR_OK:
        raise ValueError(f"or_task failed with status {st}")
    return int(tr.min_weight), int(tr.count_at_min), int(tr.combinations), \
        np.array(list(tr.witness), dtype=np.uint64)


def prefix_sequence(k: int, g: int, prefix) -> list:
    """The g-tuples that Process_prefix visits for one prefix (Sec. 3.1)."""
    lib = _lib()
    p = len(prefix)
    pre = np.asarray(prefix, dtype=np.int32)
    cap = binomial(k, g)
    out = np.zeros(max(1, cap * g), dtype=np.int32)
    cnt = lib.or_prefix_sequence(k, g, pre.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), p,
                                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), cap)
    return [tuple(int(x) for x in out[i * g:(i + 1) * g]) for i in range(cnt)]


def prefix_count(k: int, g: int, p: int) -> int:
    return int(_lib().or_prefix_count(k, g, p))


def _worker(args):
    G, n, matrix, g, p, part, nparts = args
    return task_share(G, n, matrix, g, p, part, nparts)


def min_distance_parallel(G: np.ndarray, n: int, nprocs: int | None = None, prefix: int = 3,
                          level_stop: bool = False, max_level: int = 0, pool=None,
                          progress=None) -> dict:
    """Brouwer-Zimmermann with every task split over processes; returns
    {d, lower_bound, upper_bound, stats, combinations, witness, seconds, nprocs}."""
    G = np.ascontiguousarray(G, dtype=np.uint64)
    k = G.shape[0]
    nprocs = nprocs or os.cpu_count() or 1
    _, m_f, k_m, gam = prepare(G, n)
    nsets = m_f + (1 if k_m > 0 else 0)
    L, U = 1, n - k + 1
    witness = None
    stats = []
    total = 0
    t0 = time.perf_counter()
    own = pool is None
    if own:
        pool = mp.get_context("fork").Pool(nprocs)
    try:
        if k == n:
            return dict(d=1, lower_bound=1, upper_bound=1, stats=[], combinations=0,
                        witness=gam[0].copy(), seconds=0.0, nprocs=nprocs, status=OR_OK)
        g = 1
        done = False
        status = OR_OK
        while g <= k and L < U and not done:
            if max_level and g > max_level:
                status = -5
                break
            for j in range(nsets):
                parts = pool.map(_worker, [(G, n, j, g, prefix, q, nprocs) for q in range(nprocs)])
                mn = min(r[0] for r in parts)
                cnt = sum(r[1] for r in parts if r[0] == mn)
                comb = sum(r[2] for r in parts)
                assert comb == binomial(k, g)
                total += comb
                stats.append((j, g, mn, cnt, comb))
                if mn < U or (mn == U and witness is None):
                    U = mn
                    witness = next(r[3] for r in parts if r[0] == mn)
                if progress:
                    progress(j, g, mn, cnt, U, L)
                if not level_stop:
                    L = max(L, certified_bound(j, g, m_f, k_m, k))
                    if L >= U:
                        done = True
                        break
            if not done:
                L = max(L, level_bound(g, m_f, k_m, k))
            g += 1
    finally:
        if own:
            pool.close()
            pool.join()
    return dict(d=U if status == OR_OK else 0, lower_bound=L, upper_bound=U, stats=stats,
                combinations=total, witness=witness, seconds=time.perf_counter() - t0,
                nprocs=nprocs, status=status)
