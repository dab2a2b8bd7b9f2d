"""GPU parity: libbz on gfx950 against the CPU oracle, through the C ABI.

Integer results must agree exactly: d, the last level, the final bounds and
every per-(Gamma_j, g) (min weight, count at min, combinations) in statistics
mode. Several witnesses can be correct, so the witness is checked for validity
(in the code, weight d) rather than compared.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest

import bruteforce as bf
import codes
import oracle
from paper_1911_08963_amd import inputs

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "plain_oracle.json")


@pytest.fixture(scope="module")
def bz():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1911_08963_amd import bz as _bz
    _bz.lib()
    torch.cuda.init()
    return _bz


def _say(*a):
    print(*a, flush=True)


def _weight(w):
    return int(np.bitwise_count(np.asarray(w, dtype=np.uint64)).sum())


def _check_witness(res, G, n):
    assert _weight(res.witness) == res.d
    assert bf.in_code(res.witness, G, n)


def _compare(bz, G, n, *, level_stop=False, slots=0, heads=0, max_level=0, tag=""):
    _say("case", tag, "n", n, "k", G.shape[0], "level_stop", level_stop, "slots", slots, "heads", heads)
    ref = oracle.min_distance(G, n, level_stop=level_stop, max_level=max_level)
    code = bz.Code(G, n)
    assert (code.num_full, code.partial_rank) == (ref.num_full, ref.partial_rank)
    got = bz.min_distance(code, stats=True, level_stop=level_stop, slots_per_lane=slots,
                          heads_per_tile=heads, max_level=max_level, raise_on_error=False)
    assert got.status == ref.status, (got.status, ref.status)
    assert got.d == ref.d
    assert got.last_level == ref.last_level
    assert got.upper_bound == ref.upper_bound and got.lower_bound == ref.lower_bound
    assert [tuple(s) for s in got.stats] == [tuple(s) for s in ref.stats]
    assert got.combinations == ref.combinations
    # tasks run in windows; those enqueued past the stop return at once and
    # are not counted: the search ran exactly the oracle's tasks
    assert got.launches == len(ref.stats)
    if got.status == 0:
        _check_witness(got, G, n)
    # one launch per task on every level (the smallest levels otherwise may run
    # in one single-work-group launch): the same search
    per_task = bz.min_distance(code, stats=True, level_stop=level_stop, slots_per_lane=slots,
                               heads_per_tile=heads, max_level=max_level, raise_on_error=False,
                               task_launches=True)
    assert (per_task.status, per_task.d, per_task.lower_bound, per_task.upper_bound) == \
        (got.status, got.d, got.lower_bound, got.upper_bound)
    assert [tuple(s) for s in per_task.stats] == [tuple(s) for s in got.stats]
    assert per_task.combinations == got.combinations
    if per_task.status == 0:
        _check_witness(per_task, G, n)
    fast = bz.min_distance(code, level_stop=level_stop, slots_per_lane=slots, heads_per_tile=heads,
                           max_level=max_level, raise_on_error=False)
    assert fast.status == ref.status and fast.d == ref.d
    if fast.status == 0:
        _check_witness(fast, G, n)
    code.close()
    return got


def _rand(rng, n, k, systematic=True):
    if systematic:
        return inputs.pack_rows(inputs.random_systematic(rng, n, k))
    while True:
        A = rng.integers(0, 2, size=(k, n), dtype=np.uint8)
        if inputs.gf2_rank_dense(A) == k:
            return inputs.pack_rows(A)


def test_small_random_codes(bz):
    rng = np.random.default_rng(2024)
    for t in range(40):
        n = int(rng.integers(8, 48))
        k = int(rng.integers(2, min(n, 20) + 1))
        G = _rand(rng, n, k, systematic=bool(t % 3))
        _compare(bz, G, n, tag=f"rand{t}")
        if t % 4 == 0:
            _compare(bz, G, n, level_stop=True, tag=f"rand{t}-level")


def test_stops_inside_level_spanning_launches(bz):
    # [2k, k] codes with two full-rank sets and no leftover set, k = 26..40: the
    # levels up to about 5 have below 2^21 sums, so consecutive tasks of several
    # levels share one launch; the search stops after a task in the middle of
    # such a launch (d odd: after Gamma_1 of a level), and the tasks after it,
    # run with the bounds from before the launch, must not count
    rng = np.random.default_rng(1911)
    done = 0
    while done < 12:
        k = int(rng.integers(26, 41))
        n = 2 * k
        G = _rand(rng, n, k)
        h = bz.Code(G, n, host_only=True)
        sets = (h.num_full, h.partial_rank)
        h.close()
        if sets != (2, 0):
            continue
        _compare(bz, G, n, tag=f"span{done}")
        if done % 3 == 0:
            _compare(bz, G, n, level_stop=True, tag=f"span{done}-level")
        done += 1


def test_tilings_agree(bz):
    """Slots 2/4/8 and tiny head blocks (many tiles, many colex carries) give identical results."""
    rng = np.random.default_rng(7)
    for t in range(6):
        n = int(rng.integers(40, 90))
        k = int(rng.integers(14, 26))
        G = _rand(rng, n, k, systematic=bool(t % 2))
        for slots, heads in [(2, 0), (4, 0), (8, 0), (16, 0), (2, 1), (8, 3), (4, 7), (16, 5)]:
            _compare(bz, G, n, slots=slots, heads=heads, tag=f"tiling{t}")


@pytest.mark.parametrize("name,builder", [
    ("hamming7", codes.hamming7), ("golay23", codes.golay23),
    ("golay24", lambda: codes.extend(codes.golay23())),
    ("rm26", lambda: codes.reed_muller(2, 6)), ("rm36", lambda: codes.reed_muller(3, 6)),
    ("rm17", lambda: codes.reed_muller(1, 7)), ("simplex5", lambda: codes.simplex(5)),
    ("repetition9", lambda: codes.repetition(9)), ("even_weight12", lambda: codes.even_weight(12)),
    ("whole_space10", lambda: codes.whole_space(10)),
])
def test_structured_codes(bz, name, builder):
    G, n, k, d = builder()
    got = _compare(bz, G, n, tag=name)
    assert got.d == d


def test_edge_shapes(bz):
    """W = 8 (n - k = 255), n = 256, the partial matrix, zero and repeated columns."""
    rng = np.random.default_rng(31)
    cases = []
    cases.append(("n256k1", _rand(rng, 256, 1), 256))
    cases.append(("n256k2", _rand(rng, 256, 2), 256))
    cases.append(("n256k9", _rand(rng, 256, 9), 256))
    cases.append(("n200k100", _rand(rng, 200, 100, systematic=False), 200))
    A = rng.integers(0, 2, size=(12, 70), dtype=np.uint8)
    A[:, 5] = 0
    A[:, 9] = A[:, 3]
    A[:, :12] = np.eye(12, dtype=np.uint8)
    cases.append(("zero_dup", inputs.pack_rows(A), 70))
    for name, G, n in cases:
        _compare(bz, G, n, max_level=4 if G.shape[0] > 20 else 0, tag=name)


def test_plain_workloads_match_golden(bz):
    gold = json.load(open(GOLDEN))
    for name in ("plain40", "plain128", "plain192"):
        c = inputs.plain_code(name)
        e = gold[name]
        assert c.draws == e["draws"]
        code = bz.Code(c.G, c.n)
        for mode, level_stop in (("per_gamma", False), ("per_level", True)):
            ref = e[mode]
            _say("case", name, mode)
            got = bz.min_distance(code, stats=True, level_stop=level_stop,
                                  max_level=e["max_level"], raise_on_error=False)
            assert got.status == ref["status"]
            assert got.d == ref["d"]
            assert (got.lower_bound, got.upper_bound, got.last_level) == \
                (ref["lower_bound"], ref["upper_bound"], ref["last_level"])
            assert [list(s) for s in got.stats] == ref["stats"]
            if got.status == 0:
                _check_witness(got, c.G, c.n)
        code.close()


def test_plain128_fast_mode(bz):
    gold = json.load(open(GOLDEN))["plain128"]["per_gamma"]
    c = inputs.plain_code("plain128")
    code = bz.Code(c.G, c.n)
    for slots in (0, 2, 4, 8):
        got = bz.min_distance(code, slots_per_lane=slots)
        assert got.d == gold["d"]
        _check_witness(got, c.G, c.n)
    code.close()


def test_max_level_and_cancel(bz):
    import torch
    c = inputs.plain_code("plain128")
    code = bz.Code(c.G, c.n)
    got = bz.min_distance(code, max_level=3, stats=True, raise_on_error=False)
    assert got.status == bz.BZ_ELIMIT and got.d == 0
    assert [s[1] for s in got.stats] == [1, 1, 2, 2, 3, 3]
    flag = torch.ones(1, dtype=torch.int32).pin_memory()
    import ctypes
    ptr = ctypes.cast(flag.data_ptr(), ctypes.POINTER(ctypes.c_uint32))
    got = bz.min_distance(code, cancel=ptr, raise_on_error=False)
    assert got.status == bz.BZ_ECANCELED and got.d == 0
    bad = (ctypes.c_uint32 * 1)(1)           # pageable memory is refused, not dereferenced
    got = bz.min_distance(code, cancel=ctypes.cast(bad, ctypes.POINTER(ctypes.c_uint32)),
                          raise_on_error=False)
    assert got.status == bz.BZ_EINVAL
    code.close()


def test_plain192_full_run_matches_oracle(bz):
    """The whole [192, 64] search in statistics mode against the oracle's full run (d = 35)."""
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "plain192_oracle.json")))
    c = inputs.plain_code("plain192")
    assert c.draws == gold["draws"]
    code = bz.Code(c.G, c.n)
    _say("case plain192 full, statistics mode")
    got = bz.min_distance(code, stats=True)
    assert got.d == gold["d"] == 35
    assert (got.lower_bound, got.upper_bound) == (gold["lower_bound"], gold["upper_bound"])
    assert got.combinations == gold["combinations"]
    assert [list(s) for s in got.stats] == gold["stats"]
    _check_witness(got, c.G, c.n)
    fast = bz.min_distance(code)
    assert fast.d == 35
    _check_witness(fast, c.G, c.n)
    code.close()


def test_permutation_search_parity(bz):
    """Information sets from the column-permutation search: the GPU's statistics equal the
    oracle's with the same trials and seed; d is the natural-order d."""
    rng = np.random.default_rng(404)
    items = []
    for t in range(8):
        n = int(rng.integers(20, 70))
        k = int(rng.integers(6, 18))
        items.append((_rand(rng, n, k, systematic=bool(t % 2)), n))
    for name in ("rm17", "rm26"):
        G, n, k, d = codes.reed_muller(1, 7) if name == "rm17" else codes.reed_muller(2, 6)
        items.append((G, n))
    for i, (G, n) in enumerate(items):
        natural = oracle.min_distance(G, n)
        for trials, seed in ((12, i), (60, 1000 + i)):
            _say("case perm", i, "n", n, "k", G.shape[0], "trials", trials)
            ref = oracle.min_distance(G, n, perm_trials=trials, perm_seed=seed)
            code = bz.Code(G, n, perm_trials=trials, perm_seed=seed)
            assert (code.num_full, code.partial_rank) == (ref.num_full, ref.partial_rank)
            got = bz.min_distance(code, stats=True, raise_on_error=False)
            assert got.status == ref.status == 0
            assert got.d == ref.d == natural.d
            assert [tuple(s) for s in got.stats] == [tuple(s) for s in ref.stats]
            _check_witness(got, G, n)
            code.close()
    # the same permuted codes through the batched search
    objs = [bz.Code(G, n, perm_trials=60, perm_seed=1000 + i) for i, (G, n) in enumerate(items)]
    outs, sts = bz.min_distance_batch(objs, stats=True)
    for i, ((G, n), got, st) in enumerate(zip(items, outs, sts)):
        ref = oracle.min_distance(G, n, perm_trials=60, perm_seed=1000 + i)
        assert st == 0 and got.d == ref.d
        assert [tuple(s) for s in got.stats] == [tuple(s) for s in ref.stats]
        _check_witness(got, G, n)
    for o in objs:
        o.close()
