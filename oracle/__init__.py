"""CPU oracle for the Brouwer-Zimmermann minimum distance over F2 -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. It wraps ``bz_oracle.c`` (plain C,
single-threaded) through ctypes; nothing here is used by the GPU library, and
the GPU library's code is never used here.

Every function states the passage of arXiv:1911.08963 that it follows; the C
source carries the step-by-step description.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bz_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OR_LEVEL_STOP = 2
OR_OK, OR_EINVAL, OR_ERANK, OR_ENOMEM, OR_ELIMIT = 0, -1, -2, -3, -5
OR_NW = 4


class _Stat(ctypes.Structure):
    _fields_ = [("matrix", ctypes.c_uint32), ("level", ctypes.c_uint32),
                ("min_weight", ctypes.c_uint32), ("_pad", ctypes.c_uint32),
                ("count_at_min", ctypes.c_uint64), ("combinations", ctypes.c_uint64)]


class _Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("d", ctypes.c_uint32),
                ("lower_bound", ctypes.c_uint32), ("upper_bound", ctypes.c_uint32),
                ("last_level", ctypes.c_uint32), ("num_full", ctypes.c_uint32),
                ("partial_rank", ctypes.c_uint32), ("stats_len", ctypes.c_uint32),
                ("combinations", ctypes.c_uint64), ("witness", ctypes.c_uint64 * OR_NW)]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no tuning)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        lib.or_min_distance.argtypes = [P(ctypes.c_uint64), ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                        P(_Result), P(_Stat), ctypes.c_uint32]
        lib.or_min_distance.restype = ctypes.c_int
        lib.or_prepare.argtypes = [P(ctypes.c_uint64), ctypes.c_uint32, ctypes.c_uint32,
                                   ctypes.c_uint32, P(ctypes.c_int32), P(ctypes.c_uint32),
                                   P(ctypes.c_uint32), P(ctypes.c_uint64), ctypes.c_uint32,
                                   ctypes.c_uint32]
        lib.or_prepare.restype = ctypes.c_int
        lib.or_lex_sequence.argtypes = [ctypes.c_uint32, ctypes.c_uint32, P(ctypes.c_int32),
                                        ctypes.c_uint64]
        lib.or_lex_sequence.restype = ctypes.c_int64
        lib.or_set_permutation_search.argtypes = [ctypes.c_uint32, ctypes.c_uint64]
        lib.or_set_permutation_search.restype = None
        lib.or_splitmix64.argtypes = [P(ctypes.c_uint64)]
        lib.or_splitmix64.restype = ctypes.c_uint64
        lib.or_trial_order.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, P(ctypes.c_int32)]
        lib.or_trial_order.restype = None
        lib.or_count_weight.argtypes = [P(ctypes.c_uint64), ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                        P(ctypes.c_uint64), P(ctypes.c_uint64), ctypes.c_uint64,
                                        P(ctypes.c_uint32)]
        lib.or_count_weight.restype = ctypes.c_int
        lib.or_binomial.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        lib.or_binomial.restype = ctypes.c_uint64
        for f in (lib.or_certified_bound, lib.or_level_bound):
            f.restype = ctypes.c_int
        lib.or_certified_bound.argtypes = [ctypes.c_int] * 5
        lib.or_level_bound.argtypes = [ctypes.c_int] * 4
        _lib = lib
    return _lib


def _as_words(G: np.ndarray) -> np.ndarray:
    G = np.ascontiguousarray(G, dtype=np.uint64)
    if G.ndim != 2:
        raise ValueError("G must be (k, ld) uint64")
    return G


@dataclass
class OracleResult:
    status: int
    d: int
    lower_bound: int
    upper_bound: int
    last_level: int
    num_full: int
    partial_rank: int
    combinations: int
    witness: np.ndarray
    stats: list = field(default_factory=list)   # (matrix, level, min_weight, count_at_min, combinations)


class _Permutations:
    """Sets the permutation search of step 7 for one call (Sec. 2.2's random permutations)."""

    def __init__(self, trials: int, seed: int):
        self.trials, self.seed = trials, seed

    def __enter__(self):
        _load().or_set_permutation_search(self.trials, self.seed)

    def __exit__(self, *exc):
        _load().or_set_permutation_search(0, 0)


def min_distance(G: np.ndarray, n: int, *, level_stop: bool = False, max_level: int = 0,
                 stats_cap: int = 4096, perm_trials: int = 0, perm_seed: int = 0) -> OracleResult:
    """Brouwer-Zimmermann minimum weight (Alg. 1 with the per-Gamma check of Sec. 2.2);
    perm_trials > 1 searches column permutations for the information sets (Sec. 2.2)."""
    lib = _load()
    G = _as_words(G)
    k, ld = G.shape
    res = _Result()
    stats = (_Stat * stats_cap)()
    with _Permutations(perm_trials, perm_seed):
        st = lib.or_min_distance(G.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), k, n, ld,
                                 OR_LEVEL_STOP if level_stop else 0, max_level, ctypes.byref(res),
                                 stats, stats_cap)
    out = OracleResult(int(st), res.d, res.lower_bound, res.upper_bound, res.last_level,
                       res.num_full, res.partial_rank, res.combinations,
                       np.array(list(res.witness), dtype=np.uint64))
    for i in range(min(res.stats_len, stats_cap)):
        s = stats[i]
        out.stats.append((s.matrix, s.level, s.min_weight, s.count_at_min, s.combinations))
    return out


def prepare(G: np.ndarray, n: int, perm_trials: int = 0, perm_seed: int = 0):
    """Information sets and Gamma matrices (Sec. 2.1; Sec. 2.2's permutation search when
    perm_trials > 1). Returns (set_of_column[n], m_f, k_m, gamma[(m_f + [k_m>0]) * k, ld])."""
    lib = _load()
    G = _as_words(G)
    k, ld = G.shape
    soc = np.zeros(n, dtype=np.int32)
    mf = ctypes.c_uint32()
    km = ctypes.c_uint32()
    cap = (n + 1) * k
    out_ld = (n + 63) // 64
    gam = np.zeros((cap, out_ld), dtype=np.uint64)
    with _Permutations(perm_trials, perm_seed):
        st = lib.or_prepare(G.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), k, n, ld,
                            soc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(mf),
                            ctypes.byref(km), gam.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                            out_ld, cap)
    if st != OR_OK:
        raise ValueError(f"oracle prepare failed with status {st}")
    nsets = mf.value + (1 if km.value > 0 else 0)
    return soc, mf.value, km.value, gam[: nsets * k].copy()


def count_weight(G: np.ndarray, n: int, w: int, *, max_hits: int = 1 << 22, cap: int = 0,
                 perm_trials: int = 0, perm_seed: int = 0):
    """Step 8: (number of codewords of weight w, up to cap of them sorted, last level)."""
    lib = _load()
    G = _as_words(G)
    k, ld = G.shape
    cnt = ctypes.c_uint64()
    lvl = ctypes.c_uint32()
    out = np.zeros((max(cap, 1), OR_NW), dtype=np.uint64)
    with _Permutations(perm_trials, perm_seed):
        st = lib.or_count_weight(G.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), k, n, ld, w,
                                 max_hits, ctypes.byref(cnt),
                                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), cap,
                                 ctypes.byref(lvl))
    if st != OR_OK:
        raise ValueError(f"oracle count failed with status {st}")
    return int(cnt.value), out[: min(cap, cnt.value)], int(lvl.value)


def splitmix64(state: int, count: int) -> list:
    """The first outputs of SplitMix64 from a state (the generator of step 7)."""
    st = ctypes.c_uint64(state)
    return [int(_load().or_splitmix64(ctypes.byref(st))) for _ in range(count)]


def trial_order(n: int, t: int, seed: int) -> list:
    """The column scan order p_t of trial t of the permutation search (step 7)."""
    out = np.zeros(n, dtype=np.int32)
    _load().or_trial_order(n, t, seed, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return [int(x) for x in out]


def lex_sequence(k: int, g: int) -> list:
    """The lexicographic order of g-subsets of {0..k-1} the enumeration visits (Sec. 3.1.3)."""
    lib = _load()
    total = lib.or_binomial(k, g)
    out = np.zeros(max(1, total * g), dtype=np.int32)
    cnt = lib.or_lex_sequence(k, g, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), total)
    return [tuple(int(x) for x in out[i * g:(i + 1) * g]) for i in range(cnt)]


def binomial(a: int, b: int) -> int:
    return int(_load().or_binomial(a, b))


def certified_bound(j: int, g: int, m_f: int, k_m: int, k: int) -> int:
    return int(_load().or_certified_bound(j, g, m_f, k_m, k))


def level_bound(g: int, m_f: int, k_m: int, k: int) -> int:
    return int(_load().or_level_bound(g, m_f, k_m, k))
