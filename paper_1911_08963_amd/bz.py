"""Python binding of libbz (include/bz.h): argument marshalling only.

Every step of the search runs in libbz: the host preparation in its C++ part
and the enumeration, reductions and witness recovery in its HIP kernels.
PyTorch provides the device workspace and the stream. Importing this module
loads libbz.so; it raises if the library has not been built
(``python -m paper_1911_08963_amd.build``). There is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libbz.so")

BZ_OK, BZ_EINVAL, BZ_ERANK, BZ_ENOMEM, BZ_EDEVICE, BZ_ELIMIT, BZ_ECANCELED, BZ_EBUSY = \
    0, -1, -2, -3, -4, -5, -6, -7
BZ_F_STATS, BZ_F_LEVEL_STOP, BZ_F_NO_WITNESS, BZ_F_TASK_LAUNCHES = 1, 2, 4, 8
# bz_opts.schedule: the equal-cost tiles (0) or the paper's eight distributed schedules
SCHEDULES = {"tiles": 0, "D-Lex": 1, "D-Lex-2cm": 2, "D-Lle": 3, "D-Lle-2cm": 4,
             "S-Lex": 5, "S-Lex-Snc": 6, "S-Lle": 7, "S-Lle-Snc": 8}
BZ_MAX_N = 256

P = ctypes.POINTER


class PrepareOpts(ctypes.Structure):
    _fields_ = [("perm_trials", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("perm_seed", ctypes.c_uint64)]


BZ_PREPARE_HOST_ONLY = 1


class CodeInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("k", ctypes.c_uint32), ("num_full", ctypes.c_uint32),
                ("partial_rank", ctypes.c_uint32), ("W_full", ctypes.c_uint32),
                ("W_partial", ctypes.c_uint32)]


class Opts(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("max_level", ctypes.c_uint32),
                ("hip_stream", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t), ("cancel", P(ctypes.c_uint32)),
                ("slots_per_lane", ctypes.c_uint32), ("heads_per_tile", ctypes.c_uint32),
                ("tiles_per_task", ctypes.c_uint32), ("schedule", ctypes.c_uint32),
                ("prefix", ctypes.c_uint32), ("_reserved", ctypes.c_uint32)]


class TuneEntry(ctypes.Structure):
    _fields_ = [("W", ctypes.c_uint32), ("k", ctypes.c_uint32), ("g", ctypes.c_uint32),
                ("slots_per_lane", ctypes.c_uint32), ("tiles_per_wave", ctypes.c_uint32),
                ("heads_per_tile", ctypes.c_uint32), ("combinations", ctypes.c_uint64),
                ("comb_per_s", ctypes.c_double), ("default_comb_per_s", ctypes.c_double)]


class LevelStat(ctypes.Structure):
    _fields_ = [("matrix", ctypes.c_uint16), ("level", ctypes.c_uint16),
                ("min_weight", ctypes.c_uint32), ("count_at_min", ctypes.c_uint64),
                ("combinations", ctypes.c_uint64)]


class Result(ctypes.Structure):
    _fields_ = [("d", ctypes.c_uint32), ("lower_bound", ctypes.c_uint32),
                ("upper_bound", ctypes.c_uint32), ("last_level", ctypes.c_uint32),
                ("combinations", ctypes.c_uint64), ("witness", P(ctypes.c_uint64)),
                ("stats", P(LevelStat)), ("stats_cap", ctypes.c_uint32),
                ("stats_len", ctypes.c_uint32), ("launches", ctypes.c_uint32),
                ("_pad", ctypes.c_uint32), ("prepare_s", ctypes.c_double),
                ("search_s", ctypes.c_double), ("kernel_s", ctypes.c_double)]


class DebugRect(ctypes.Structure):
    _fields_ = [("lane_off", ctypes.c_uint32), ("lane_n", ctypes.c_uint32),
                ("lane_t", ctypes.c_uint32), ("head_off", ctypes.c_uint32),
                ("head_n", ctypes.c_uint32), ("head_t", ctypes.c_uint32),
                ("lane_mult", ctypes.c_uint32), ("_reserved1", ctypes.c_uint32),
                ("lane_count", ctypes.c_uint64), ("head_count", ctypes.c_uint64),
                ("tile_begin", ctypes.c_uint64), ("lane_blocks", ctypes.c_uint64),
                ("head_blocks", ctypes.c_uint64), ("_reserved2", ctypes.c_uint64)]


class WeightCount(ctypes.Structure):
    _fields_ = [("weight", ctypes.c_uint32), ("last_level", ctypes.c_uint32),
                ("count", ctypes.c_uint64), ("hits", ctypes.c_uint64),
                ("combinations", ctypes.c_uint64), ("codewords", P(ctypes.c_uint64)),
                ("codewords_cap", ctypes.c_uint64), ("codewords_len", ctypes.c_uint64),
                ("search_s", ctypes.c_double)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("hbm_budget", ctypes.c_size_t), ("stats_cap", ctypes.c_uint32),
                ("target_tiles", ctypes.c_uint32), ("arena_bytes", ctypes.c_size_t),
                ("codes_per_launch", ctypes.c_uint32), ("_reserved", ctypes.c_uint32)]


class BZError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def _signatures(lib):
    vp = ctypes.c_void_p
    u32, u64 = ctypes.c_uint32, ctypes.c_uint64
    sig = {
        "bz_prepare": ([P(u64), u32, u32, u32, P(PrepareOpts), P(vp)], ctypes.c_int),
        "bz_code_get_info": ([vp, P(CodeInfo), P(ctypes.c_int32)], ctypes.c_int),
        "bz_code_get_gamma": ([vp, u32, P(u64), u32], ctypes.c_int),
        "bz_free": ([vp], None),
        "bz_workspace_bytes": ([P(vp), u32, P(Opts), P(ctypes.c_size_t)], ctypes.c_int),
        "bz_min_distance": ([vp, P(Opts), P(Result)], ctypes.c_int),
        "bz_min_distance_noalloc": ([vp, P(Opts), P(Result)], ctypes.c_int),
        "bz_min_distance_batch": ([P(vp), u32, P(Opts), P(Result), P(ctypes.c_int)], ctypes.c_int),
        "bz_status_str": ([ctypes.c_int], ctypes.c_char_p),
        "bz_last_error": ([], ctypes.c_char_p),
        "bz_count_codewords": ([vp, P(Opts), P(WeightCount)], ctypes.c_int),
        "bz_autotune": ([u32, u32, P(TuneEntry)], ctypes.c_int),
        "bz_autotune_get": ([u32, P(TuneEntry)], ctypes.c_int),
        "bz_autotune_set": ([P(TuneEntry)], ctypes.c_int),
        "bz_autotune_clear": ([], None),
        "bz_autotune_batch": ([P(vp), u32, P(Opts), P(u32), P(ctypes.c_double)], ctypes.c_int),
        "bz_debug_valu_rate": ([u32, P(ctypes.c_double), P(ctypes.c_double)], ctypes.c_int),
        "bz_server_create": ([P(ServerOpts), P(vp)], ctypes.c_int),
        "bz_server_submit": ([vp, vp, P(Opts), P(Result), P(u64)], ctypes.c_int),
        "bz_server_poll": ([vp, P(u64), P(ctypes.c_int), u32, P(u32)], ctypes.c_int),
        "bz_server_pending": ([vp, P(u32)], ctypes.c_int),
        "bz_server_destroy": ([vp, ctypes.c_double], ctypes.c_int),
        "bz_debug_prepare_host": ([P(u64), u32, u32, u32, P(u32), P(u32), P(ctypes.c_int32),
                                   P(u64), u32, P(u32), ctypes.c_size_t], ctypes.c_int),
        "bz_debug_plan_level": ([u32, u32, u32, u32, u64, u32, P(DebugRect), u32, P(u32), P(u64),
                                 P(u32)], ctypes.c_int),
        "bz_debug_schedule": ([u32, u32, u32, u32, u32, u32, P(ctypes.c_int32), u64, P(u32), P(u64)],
                              ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res


_lib = None


def lib():
    """The loaded libbz.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libbz.so is not built ({LIB_PATH}); run python -m paper_1911_08963_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        _signatures(L)
        _lib = L
    return _lib


def _check(st: int):
    if st != BZ_OK:
        raise BZError(st, lib().bz_last_error().decode() or lib().bz_status_str(st).decode())


def _words(G) -> np.ndarray:
    G = np.ascontiguousarray(G, dtype=np.uint64)
    if G.ndim != 2:
        raise ValueError("G must be a (k, ld) uint64 array")
    return G


class Code:
    """A prepared code (bz_prepare): information sets and Gamma_j on the current device
    (host_only: on the host only, for a Server)."""

    def __init__(self, G, n: int, perm_trials: int = 0, perm_seed: int = 0, host_only: bool = False):
        G = _words(G)
        k, ld = G.shape
        self.n, self.k = int(n), int(k)
        h = ctypes.c_void_p()
        po = PrepareOpts(perm_trials, BZ_PREPARE_HOST_ONLY if host_only else 0, perm_seed)
        _check(lib().bz_prepare(G.ctypes.data_as(P(ctypes.c_uint64)), k, n, ld, ctypes.byref(po),
                                ctypes.byref(h)))
        self._h = h
        info = CodeInfo()
        soc = np.zeros(n, dtype=np.int32)
        _check(lib().bz_code_get_info(h, ctypes.byref(info), soc.ctypes.data_as(P(ctypes.c_int32))))
        self.num_full, self.partial_rank = info.num_full, info.partial_rank
        self.W_full, self.W_partial = info.W_full, info.W_partial
        self.set_of_column = soc

    @property
    def handle(self):
        return self._h

    @property
    def nsets(self) -> int:
        return self.num_full + (1 if self.partial_rank else 0)

    def gamma(self, j: int) -> np.ndarray:
        ld = (self.n + 63) // 64
        out = np.zeros((self.k, ld), dtype=np.uint64)
        _check(lib().bz_code_get_gamma(self._h, j, out.ctypes.data_as(P(ctypes.c_uint64)), ld))
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().bz_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class SearchResult:
    status: int
    d: int
    lower_bound: int
    upper_bound: int
    last_level: int
    combinations: int
    witness: np.ndarray
    stats: list = field(default_factory=list)   # (matrix, level, min_weight, count_at_min, combinations)
    launches: int = 0
    prepare_s: float = 0.0
    search_s: float = 0.0
    kernel_s: float = 0.0


_ws_cache = {}


_ws_single = []


def workspace_bytes() -> int:
    """bz_workspace_bytes of a single search (the same for every code: asked once)."""
    if not _ws_single:
        b = ctypes.c_size_t()
        _check(lib().bz_workspace_bytes(None, 0, None, ctypes.byref(b)))
        _ws_single.append(b.value)
    return _ws_single[0]


def _workspace(device, nbytes):
    """A cached torch device buffer of at least nbytes (grown on demand)."""
    import torch
    key = str(device)
    t = _ws_cache.get(key)
    if t is None or t.numel() < nbytes:
        t = torch.empty(nbytes, dtype=torch.uint8, device=device)
        _ws_cache[key] = t
    return t


def _opts(flags, max_level, stream, ws, cancel, slots, heads, tiles=0) -> Opts:
    o = Opts()
    o.tiles_per_task = tiles
    o.flags = flags
    o.max_level = max_level
    o.hip_stream = stream
    o.workspace = ws.data_ptr() if ws is not None else None
    o.workspace_bytes = ws.numel() if ws is not None else 0
    o.cancel = cancel
    o.slots_per_lane = slots
    o.heads_per_tile = heads
    return o


def min_distance(code: Code, *, stats: bool = False, level_stop: bool = False,
                 witness: bool = True, max_level: int = 0, slots_per_lane: int = 0,
                 heads_per_tile: int = 0, stats_cap: int = 4096, stream=None,
                 cancel=None, raise_on_error: bool = True, schedule=0, prefix: int = 0,
                 task_launches: bool = False) -> SearchResult:
    """bz_min_distance on the current torch stream, with a torch-allocated workspace.

    schedule: 0 / "tiles", or one of the paper's schedules by number (1..8) or
    name ("D-Lex", ..., "S-Lle-Snc", see SCHEDULES) with its prefix size.
    task_launches: one launch per task on every level (BZ_F_TASK_LAUNCHES)."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    stream = stream if stream is not None else torch.cuda.current_stream(dev)
    ws = _workspace(dev, workspace_bytes())
    return _search(lib().bz_min_distance, code, stats, level_stop, witness, max_level, slots_per_lane,
                   heads_per_tile, stats_cap, stream, ws, cancel, raise_on_error, schedule, prefix,
                   task_launches)


def min_distance_noalloc(code: Code, *, stats: bool = False, level_stop: bool = False,
                         witness: bool = True, max_level: int = 0, slots_per_lane: int = 0,
                         heads_per_tile: int = 0, stats_cap: int = 4096, stream=None,
                         cancel=None, raise_on_error: bool = True) -> SearchResult:
    """bz_min_distance_noalloc on the current torch stream: the library's own device scratch
    array, no workspace and no allocation."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    stream = stream if stream is not None else torch.cuda.current_stream(dev)
    return _search(lib().bz_min_distance_noalloc, code, stats, level_stop, witness, max_level,
                   slots_per_lane, heads_per_tile, stats_cap, stream, None, cancel, raise_on_error, 0, 0)


def _search(fn, code, stats, level_stop, witness, max_level, slots_per_lane, heads_per_tile, stats_cap,
            stream, ws, cancel, raise_on_error, schedule, prefix, task_launches=False) -> SearchResult:
    flags = (BZ_F_STATS if stats else 0) | (BZ_F_LEVEL_STOP if level_stop else 0) | \
        (0 if witness else BZ_F_NO_WITNESS) | (BZ_F_TASK_LAUNCHES if task_launches else 0)
    o = _opts(flags, max_level, stream.cuda_stream, ws, cancel, slots_per_lane, heads_per_tile)
    o.schedule = SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
    o.prefix = prefix
    wit = np.zeros(4, dtype=np.uint64)
    st_buf = np.empty(stats_cap, dtype=_STAT_DTYPE)     # written by the library up to stats_len
    r = Result()
    r.witness = wit.ctypes.data_as(P(ctypes.c_uint64))
    r.stats = st_buf.ctypes.data_as(P(LevelStat)) if stats_cap else None   # 0: no per-task records wanted
    r.stats_cap = stats_cap
    st = fn(code.handle, ctypes.byref(o), ctypes.byref(r))
    if st != BZ_OK and raise_on_error:
        _check(st)
    out = SearchResult(st, r.d, r.lower_bound, r.upper_bound, r.last_level, r.combinations,
                       wit[: (code.n + 63) // 64].copy(), [], r.launches, r.prepare_s, r.search_s,
                       r.kernel_s)
    m = min(r.stats_len, stats_cap)
    if m:
        out.stats = _stat_tuples(st_buf[:m])
    return out


def min_distance_batch(codes, *, stats: bool = False, level_stop: bool = False, witness: bool = True,
                       max_level: int = 0, stream=None, stats_cap: int = 512, slots_per_lane: int = 0,
                       heads_per_tile: int = 0, tiles_per_task: int = 0, cancel=None):
    """bz_min_distance_batch: returns (list of SearchResult, list of status)."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    stream = stream if stream is not None else torch.cuda.current_stream(dev)
    cnt = len(codes)
    handles = (ctypes.c_void_p * cnt)(*[c.handle.value for c in codes])
    flags = (BZ_F_STATS if stats else 0) | (BZ_F_LEVEL_STOP if level_stop else 0) | \
        (0 if witness else BZ_F_NO_WITNESS)
    nbytes = ctypes.c_size_t()
    o = _opts(flags, max_level, stream.cuda_stream, None, cancel, slots_per_lane, heads_per_tile, tiles_per_task)
    _check(lib().bz_workspace_bytes(handles, cnt, ctypes.byref(o), ctypes.byref(nbytes)))
    ws = _workspace(dev, nbytes.value)
    o = _opts(flags, max_level, stream.cuda_stream, ws, cancel, slots_per_lane, heads_per_tile, tiles_per_task)
    res = (Result * cnt)()
    wits = np.zeros((cnt, 4), dtype=np.uint64)
    # one buffer for every code's task records (stats_cap each; none when stats_cap is 0)
    stb = np.zeros(cnt * stats_cap, dtype=_STAT_DTYPE) if stats_cap else None
    wbase = wits.ctypes.data
    sbase = stb.ctypes.data if stats_cap else 0
    for i in range(cnt):
        res[i].witness = ctypes.cast(wbase + 32 * i, P(ctypes.c_uint64))
        res[i].stats = ctypes.cast(sbase + i * stats_cap * _STAT_DTYPE.itemsize, P(LevelStat)) if stats_cap else None
        res[i].stats_cap = stats_cap
    per = (ctypes.c_int * cnt)()
    lib().bz_min_distance_batch(handles, cnt, ctypes.byref(o), res, per)
    outs = []
    for i in range(cnt):
        r = res[i]
        o_ = SearchResult(per[i], r.d, r.lower_bound, r.upper_bound, r.last_level, r.combinations,
                          wits[i][: (codes[i].n + 63) // 64].copy(), [], r.launches, r.prepare_s,
                          r.search_s, r.kernel_s)
        m = min(r.stats_len, stats_cap)
        if m:
            o_.stats = _stat_tuples(stb[i * stats_cap: i * stats_cap + m])
        outs.append(o_)
    return outs, [per[i] for i in range(cnt)]


# the layout of bz_level_stat, for reading many records at once
_STAT_DTYPE = np.dtype([("matrix", "<u2"), ("level", "<u2"), ("min_weight", "<u4"),
                        ("count_at_min", "<u8"), ("combinations", "<u8")])
assert _STAT_DTYPE.itemsize == ctypes.sizeof(LevelStat)


def _stat_tuples(a) -> list:
    """(matrix, level, min_weight, count_at_min, combinations) tuples of Python ints."""
    return list(zip(a["matrix"].tolist(), a["level"].tolist(), a["min_weight"].tolist(),
                    a["count_at_min"].tolist(), a["combinations"].tolist()))


# ---------------------------------------------------------------- codewords of a given weight

def count_codewords(code: Code, weight: int = 0, *, cap: int = 0, max_level: int = 0, stream=None) -> dict:
    """bz_count_codewords: the number of codewords of weight `weight` (0 = d), and up to cap of them."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    stream = stream if stream is not None else torch.cuda.current_stream(dev)
    o = _opts(0, max_level, stream.cuda_stream, None, None, 0, 0)
    nw = (code.n + 63) // 64
    buf = np.zeros((max(cap, 1), nw), dtype=np.uint64)
    r = WeightCount()
    r.weight = weight
    r.codewords = buf.ctypes.data_as(P(ctypes.c_uint64)) if cap else None
    r.codewords_cap = cap
    _check(lib().bz_count_codewords(code.handle, ctypes.byref(o), ctypes.byref(r)))
    return {"weight": r.weight, "count": r.count, "hits": r.hits, "combinations": r.combinations,
            "last_level": r.last_level, "codewords": buf[: r.codewords_len].copy(), "search_s": r.search_s}


# ---------------------------------------------------------------- autotuning

def _entry(e: TuneEntry) -> dict:
    return {f: getattr(e, f) for f, _ in TuneEntry._fields_ if not f.startswith("_")}


def autotune(W: int, k: int) -> dict:
    """bz_autotune: times the (slots, tiles per wave) candidates for row width W and installs the fastest."""
    e = TuneEntry()
    _check(lib().bz_autotune(W, k, ctypes.byref(e)))
    return _entry(e)


def autotune_get(W: int):
    e = TuneEntry()
    return _entry(e) if lib().bz_autotune_get(W, ctypes.byref(e)) == BZ_OK else None


def autotune_set(W: int, slots_per_lane: int, tiles_per_wave: int):
    """bz_autotune_set: installs a (slots per lane, tiles per wave) choice for W without timing."""
    e = TuneEntry()
    e.W, e.slots_per_lane, e.tiles_per_wave = W, slots_per_lane, tiles_per_wave
    _check(lib().bz_autotune_set(ctypes.byref(e)))


def autotune_clear():
    lib().bz_autotune_clear()


def autotune_batch(codes) -> tuple:
    """bz_autotune_batch on these codes: (tiles per task installed, its best wall seconds)."""
    cnt = len(codes)
    handles = (ctypes.c_void_p * cnt)(*[c.handle.value for c in codes])
    o = _opts(0, 0, None, None, None, 0, 0)
    t, sec = ctypes.c_uint32(), ctypes.c_double()
    _check(lib().bz_autotune_batch(handles, cnt, ctypes.byref(o), ctypes.byref(t), ctypes.byref(sec)))
    return t.value, sec.value


def valu_rate(iters: int = 0) -> tuple:
    """bz_debug_valu_rate: (int32 lane operations per second, probe seconds)."""
    r, sec = ctypes.c_double(), ctypes.c_double()
    _check(lib().bz_debug_valu_rate(iters, ctypes.byref(r), ctypes.byref(sec)))
    return r.value, sec.value


# ---------------------------------------------------------------- serving

def _fill(st, r, wit, stb, n, stats_cap) -> SearchResult:
    out = SearchResult(st, r.d, r.lower_bound, r.upper_bound, r.last_level, r.combinations,
                       wit[: (n + 63) // 64].copy(), [], r.launches, r.prepare_s, r.search_s,
                       r.kernel_s)
    for t in range(min(r.stats_len, stats_cap)):
        s = stb[t]
        out.stats.append((s.matrix, s.level, s.min_weight, s.count_at_min, s.combinations))
    return out


class Server:
    """bz_server_*: a resident search on the current device that admits requests as they come.

    submit() returns a ticket, or None when the server is busy (no slot or HBM
    budget; poll and retry). poll() returns finished requests as
    (ticket, SearchResult) pairs; search_s is the time from submission to
    completion seen by the library's watcher thread.
    """

    def __init__(self, *, slots: int = 1024, stats: bool = False, hbm_budget: int = 0,
                 stats_cap: int = 512, target_tiles: int = 0, arena_bytes: int = 0,
                 codes_per_launch: int = 0):
        o = ServerOpts(slots, BZ_F_STATS if stats else 0, hbm_budget, stats_cap, target_tiles,
                       arena_bytes, codes_per_launch, 0)
        h = ctypes.c_void_p()
        _check(lib().bz_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.stats = stats
        self.stats_cap = stats_cap
        self._live = {}                     # ticket -> (Result, witness, stats buffer, n)
        self._done = {}                     # finished, collected by wait() for later

    def submit(self, code: Code, *, level_stop: bool = False, witness: bool = True,
               max_level: int = 0):
        flags = (BZ_F_STATS if self.stats else 0) | (BZ_F_LEVEL_STOP if level_stop else 0) | \
            (0 if witness else BZ_F_NO_WITNESS)
        o = _opts(flags, max_level, None, None, None, 0, 0)
        r = Result()
        wit = np.zeros(4, dtype=np.uint64)
        stb = (LevelStat * self.stats_cap)()
        r.witness = wit.ctypes.data_as(P(ctypes.c_uint64))
        r.stats = stb
        r.stats_cap = self.stats_cap
        t = ctypes.c_uint64()
        st = lib().bz_server_submit(self._h, code.handle, ctypes.byref(o), ctypes.byref(r), ctypes.byref(t))
        if st == BZ_EBUSY:
            return None
        _check(st)
        self._live[t.value] = (r, wit, stb, code.n)
        return t.value

    def poll(self, cap: int = 4096):
        if self._done:
            out = list(self._done.items())
            self._done.clear()
            return out + self._poll(cap)
        return self._poll(cap)

    def _poll(self, cap: int):
        tk = (ctypes.c_uint64 * cap)()
        sts = (ctypes.c_int * cap)()
        nd = ctypes.c_uint32()
        _check(lib().bz_server_poll(self._h, tk, sts, cap, ctypes.byref(nd)))
        out = []
        for i in range(nd.value):
            r, wit, stb, n = self._live.pop(tk[i])
            out.append((tk[i], _fill(sts[i], r, wit, stb, n, self.stats_cap)))
        return out

    def pending(self) -> int:
        p = ctypes.c_uint32()
        _check(lib().bz_server_pending(self._h, ctypes.byref(p)))
        return p.value

    def wait(self, ticket: int, timeout: float = 60.0):
        """Polls until the ticket is done; other finished requests are kept for later polls."""
        import time
        t0 = time.perf_counter()
        while True:
            for t, res in self._poll(4096):
                self._done[t] = res
            if ticket in self._done:
                return self._done.pop(ticket)
            if time.perf_counter() - t0 > timeout:
                raise TimeoutError(f"ticket {ticket} not done after {timeout} s")
            time.sleep(50e-6)

    def close(self, timeout: float = 60.0) -> int:
        st = BZ_OK
        if getattr(self, "_h", None):
            st = lib().bz_server_destroy(self._h, timeout)
            self._h = None
        return st

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- host-only inspection

def prepare_host(G, n: int):
    """bz_debug_prepare_host: (set_of_column, m_f, k_m, gamma rows, packed words)."""
    G = _words(G)
    k, ld = G.shape
    mf, km = ctypes.c_uint32(), ctypes.c_uint32()
    soc = np.zeros(n, dtype=np.int32)
    cap = (n + 1) * k
    gam = np.zeros((cap, ld), dtype=np.uint64)
    packed = np.zeros(cap * (BZ_MAX_N // 32), dtype=np.uint32)
    _check(lib().bz_debug_prepare_host(G.ctypes.data_as(P(ctypes.c_uint64)), k, n, ld,
                                       ctypes.byref(mf), ctypes.byref(km),
                                       soc.ctypes.data_as(P(ctypes.c_int32)),
                                       gam.ctypes.data_as(P(ctypes.c_uint64)), cap,
                                       packed.ctypes.data_as(P(ctypes.c_uint32)), packed.size))
    nsets = mf.value + (1 if km.value else 0)
    return soc, mf.value, km.value, gam[: nsets * k].copy(), packed


def plan_level(k: int, g: int, slots: int = 8, heads_per_tile: int = 0, target_tiles: int = 1 << 17,
               widen: bool = False):
    """bz_debug_plan_level: (list of rect dicts, total_tiles, heads_per_tile)."""
    cap = 16384
    rects = (DebugRect * cap)()
    nr, tt, hu = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint32()
    _check(lib().bz_debug_plan_level(k, g, slots, heads_per_tile, target_tiles, int(widen), rects, cap,
                                     ctypes.byref(nr), ctypes.byref(tt), ctypes.byref(hu)))
    out = []
    for i in range(nr.value):
        r = rects[i]
        out.append({f: getattr(r, f) for f, _ in DebugRect._fields_ if not f.startswith("_")})
    return out, tt.value, hu.value


def debug_schedule(schedule, k: int, g: int, p: int, workers: int, turns: int = 4):
    """bz_debug_schedule: (pre_elems, ntasks, table). Static schedules: table[w][s] is
    the prefix (tuple) worker w takes at turn s, or None. Dynamic: table[c] lists the
    prefixes of claim c (one, two, or none). With pre_elems == 0 a prefix is ()."""
    sched = SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
    pe, nt = ctypes.c_uint32(), ctypes.c_uint64()
    _check(lib().bz_debug_schedule(sched, k, g, p, workers, turns, None, 0, ctypes.byref(pe), ctypes.byref(nt)))
    e = max(pe.value, 1)
    per = 2 if 1 <= sched <= 4 else turns
    out = np.full(workers * per * e, -1, dtype=np.int32)
    _check(lib().bz_debug_schedule(sched, k, g, p, workers, turns, out.ctypes.data_as(P(ctypes.c_int32)),
                                   out.size, ctypes.byref(pe), ctypes.byref(nt)))
    table = []
    for w in range(workers):
        row = []
        for s_ in range(per):
            ent = out[(w * per + s_) * e:(w * per + s_ + 1) * e]
            if ent[0] < 0:
                row.append(None)
            else:
                row.append(tuple(int(x) for x in ent) if pe.value else ())
        if 1 <= sched <= 4:
            row = [x for x in row if x is not None]
        table.append(row)
    return pe.value, nt.value, table
