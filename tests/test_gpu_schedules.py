"""GPU parity of the paper's eight distributed schedules (Sec. 3 of
arXiv:1911.08963) run with the device's waves as workers.

A schedule changes only how a (Gamma_j, g) task is cut into prefix tasks and
dealt out, never what is computed: under every schedule and prefix size the
search must give the oracle's d, bounds and per-(Gamma_j, g) statistics
exactly, and a valid witness. Prefix sizes cover the usual split, prefixes of
one element, and prefixes so long (or so short, for the relative sizes of the
static schedules) that each level is a single task.
"""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

import bruteforce as bf
import codes
import oracle
from paper_1911_08963_amd import inputs

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "plain_oracle.json")
NAMES = ["D-Lex", "D-Lex-2cm", "D-Lle", "D-Lle-2cm", "S-Lex", "S-Lex-Snc", "S-Lle", "S-Lle-Snc"]


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


def _check_witness(res, G, n):
    assert int(np.bitwise_count(np.asarray(res.witness, dtype=np.uint64)).sum()) == res.d
    assert bf.in_code(res.witness, G, n)


def _rand(rng, n, k, systematic=True):
    if systematic:
        return inputs.pack_rows(inputs.random_systematic(rng, n, k))
    while True:
        A = rng.integers(0, 2, size=(k, n), dtype=np.uint8)
        if inputs.gf2_rank_dense(A) == k:
            return inputs.pack_rows(A)


def _same(got, ref):
    assert got.status == ref.status, (got.status, ref.status)
    assert got.d == ref.d
    assert (got.lower_bound, got.upper_bound, got.last_level) == (ref.lower_bound, ref.upper_bound, ref.last_level)
    assert [tuple(s) for s in got.stats] == [tuple(s) for s in ref.stats]


def test_every_schedule_matches_oracle(bz):
    rng = np.random.default_rng(1911)
    items = []
    for t in range(8):
        n = int(rng.integers(16, 64))
        k = int(rng.integers(4, min(n, 22) + 1))
        items.append((f"rand{t}", _rand(rng, n, k, systematic=bool(t % 2)), n))
    for name, builder in [("golay24", lambda: codes.extend(codes.golay23())),
                          ("rm26", lambda: codes.reed_muller(2, 6))]:
        G, n, _, _ = builder()
        items.append((name, G, n))
    for name, G, n in items:
        ref = oracle.min_distance(G, n)
        ref_level = oracle.min_distance(G, n, level_stop=True)
        code = bz.Code(G, n)
        for sched in NAMES:
            for prefix in (1, 3, 40):
                _say("case", name, "n", n, "k", G.shape[0], sched, "prefix", prefix)
                got = bz.min_distance(code, stats=True, schedule=sched, prefix=prefix, raise_on_error=False)
                _same(got, ref)
                assert got.combinations == ref.combinations
                _check_witness(got, G, n)
                fast = bz.min_distance(code, schedule=sched, prefix=prefix)
                assert fast.d == ref.d
                _check_witness(fast, G, n)
            got = bz.min_distance(code, stats=True, level_stop=True, schedule=sched, prefix=2,
                                  raise_on_error=False)
            _same(got, ref_level)
        code.close()


def test_edge_shapes(bz):
    """W = 8 (n - k = 255), the partial matrix at k = 100, zero and repeated columns."""
    rng = np.random.default_rng(77)
    cases = [("n256k9", _rand(rng, 256, 9), 256, 0),
             ("n200k100", _rand(rng, 200, 100, systematic=False), 200, 3)]
    A = rng.integers(0, 2, size=(12, 70), dtype=np.uint8)
    A[:, 5] = 0
    A[:, 9] = A[:, 3]
    A[:, :12] = np.eye(12, dtype=np.uint8)
    cases.append(("zero_dup", inputs.pack_rows(A), 70, 0))
    for name, G, n, max_level in cases:
        ref = oracle.min_distance(G, n, max_level=max_level)
        code = bz.Code(G, n)
        for sched, prefix in (("D-Lex-2cm", 2), ("S-Lle-Snc", 1), ("D-Lle", 1), ("S-Lex", 2)):
            _say("case", name, sched, prefix)
            got = bz.min_distance(code, stats=True, schedule=sched, prefix=prefix, max_level=max_level,
                                  raise_on_error=False)
            _same(got, ref)
            if got.status == 0:
                _check_witness(got, G, n)
        code.close()


def test_plain_workloads_match_golden(bz):
    gold = json.load(open(GOLDEN))
    for name in ("plain40", "plain128"):
        c = inputs.plain_code(name)
        ref = gold[name]["per_gamma"]
        code = bz.Code(c.G, c.n)
        for sched in NAMES:
            prefix = 3
            _say("case", name, sched, prefix)
            got = bz.min_distance(code, stats=True, schedule=sched, prefix=prefix,
                                  max_level=gold[name]["max_level"], raise_on_error=False)
            assert got.status == ref["status"] and got.d == ref["d"]
            assert (got.lower_bound, got.upper_bound, got.last_level) == \
                (ref["lower_bound"], ref["upper_bound"], ref["last_level"])
            assert [list(s) for s in got.stats] == ref["stats"]
            _check_witness(got, c.G, c.n)
            fast = bz.min_distance(code, schedule=sched, prefix=prefix)
            assert fast.d == ref["d"]
            _check_witness(fast, c.G, c.n)
        code.close()


def test_schedule_errors(bz):
    c = inputs.plain_code("plain40")
    code = bz.Code(c.G, c.n)
    assert bz.min_distance(code, schedule=9, prefix=2, raise_on_error=False).status == bz.BZ_EINVAL
    assert bz.min_distance(code, schedule="D-Lex", prefix=0, raise_on_error=False).status == bz.BZ_EINVAL
    with pytest.raises(bz.BZError):
        bz.lib()
        import ctypes
        o = bz.Opts()
        o.schedule = 1
        o.prefix = 2
        res = (bz.Result * 1)()
        per = (ctypes.c_int * 1)()
        arr = (ctypes.c_void_p * 1)(code.handle)
        bz._check(bz.lib().bz_min_distance_batch(arr, 1, ctypes.byref(o), res, per))
    code.close()


def test_plain192_best_schedules(bz):
    """The full [192, 64] search (d = 35) under the fastest dynamic and static schedule."""
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "plain192_oracle.json")))
    c = inputs.plain_code("plain192")
    code = bz.Code(c.G, c.n)
    for sched, prefix in (("D-Lle-2cm", 4), ("S-Lle-Snc", 6)):
        _say("case plain192", sched, prefix)
        got = bz.min_distance(code, schedule=sched, prefix=prefix)
        assert got.d == gold["d"] == 35
        assert (got.lower_bound, got.upper_bound) == (gold["lower_bound"], gold["upper_bound"])
        _check_witness(got, c.G, c.n)
    code.close()
