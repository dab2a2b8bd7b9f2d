"""The paper's eight distributed schedules (Sec. 3 of arXiv:1911.08963) as the
GPU search deals them to waves: the host copy of the device mapping
(bz_debug_schedule), checked on the CPU.

Pins:
* the four distribution tables the paper prints for the static schedules
  (Sec. 3.3), verbatim;
* the paper's orders (Sec. 3.1.3): one static worker walks the prefixes in
  lexicographic or left-lexicographic order exactly (the latter against the
  paper's printed list);
* the number of prefixes C(k - (g - p), p) (Secs. 3.1.1 and 3.4.2) and the
  oracle's own count of valid prefixes;
* every prefix handed out exactly once under every schedule, and the
  completions of all prefixes (the oracle's Process_prefix) covering each
  g-subset exactly once;
* the dynamic pair schedule takes one prefix from each end of the order (Sec. 3.2).
"""
from __future__ import annotations

import itertools
import math
import os

import pytest

from paper_1911_08963_amd import bz

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
STATIC = ["S-Lex", "S-Lex-Snc", "S-Lle", "S-Lle-Snc"]
DYNAMIC = ["D-Lex", "D-Lex-2cm", "D-Lle", "D-Lle-2cm"]


def _prefixes_of(schedule, k, g, p, workers):
    """Every prefix the schedule hands out, in (worker, turn) or claim order."""
    pe, nt, _ = bz.debug_schedule(schedule, k, g, p, 1, 1)
    if schedule in STATIC:
        turns = -(-nt // workers)
        _, _, table = bz.debug_schedule(schedule, k, g, p, workers, turns)
        return pe, nt, [x for row in table for x in row if x is not None]
    _, _, table = bz.debug_schedule(schedule, k, g, p, nt + 1)
    return pe, nt, [x for row in table for x in row]


def test_paper_static_tables():
    rows = []
    with open(os.path.join(GOLDEN, "paper_schedule_tables.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(line.split())
    assert len(rows) == 12
    for name, k, g, p, proc, *pres in rows:
        want = [tuple(int(x) for x in s.split(",")) for s in pres]
        pe, _, table = bz.debug_schedule(name, int(k), int(g), int(p), 3, len(want))
        assert pe == 3
        assert table[int(proc)] == want, (name, proc)


def test_one_worker_walks_the_orders():
    # lexicographic: itertools order; left-lexicographic: colex (the paper's k=6, g=4, p=3 list)
    k, g, p = 9, 5, 2                      # relative p = 2: 3-element prefixes of {0..6}
    _, nt, table = bz.debug_schedule("S-Lex", k, g, p, 1, 200)
    lex = [c for c in table[0] if c is not None]
    assert lex == list(itertools.combinations(range(k - (g - 3)), 3))
    _, _, table = bz.debug_schedule("S-Lle", k, g, p, 1, 200)
    colex = [c for c in table[0] if c is not None]
    assert colex == sorted(itertools.combinations(range(k - (g - 3)), 3), key=lambda c: c[::-1])
    with open(os.path.join(GOLDEN, "paper_subset_orders.txt")) as f:
        paper = {}
        for line in f:
            if line.strip() and not line.startswith("#"):
                o, i, *c = line.split()
                paper.setdefault(o, []).append(tuple(int(x) for x in c))
    # the paper's example: k = 6, g = 4, prefixes of 3 elements (relative p = 1)
    assert bz.debug_schedule("S-Lex", 6, 4, 1, 1, 10)[2][0] == paper["lex"]
    assert bz.debug_schedule("S-Lle", 6, 4, 1, 1, 10)[2][0] == paper["colex"]
    assert bz.debug_schedule("D-Lle", 6, 4, 3, 10)[2] == [[c] for c in paper["colex"]]


@pytest.mark.parametrize("schedule", STATIC + DYNAMIC)
def test_every_prefix_once(schedule):
    from oracle import parallel
    for k, g, p, workers in [(12, 5, 2, 3), (12, 5, 3, 7), (16, 6, 4, 5), (10, 10, 1, 4), (9, 2, 1, 64),
                             (20, 4, 2, 1)]:
        pe, nt, got = _prefixes_of(schedule, k, g, p, workers)
        e = p if schedule in DYNAMIC else g - p
        e = e if 0 < e < g else 0
        assert pe == e
        if e == 0:
            assert nt == 1 and got == [()]
            continue
        assert nt == math.comb(k - (g - e), e) == parallel.prefix_count(k, g, e)
        assert sorted(got) == list(itertools.combinations(range(k - (g - e)), e))


def test_completions_cover_each_subset_once():
    from oracle import parallel
    k, g = 11, 5
    for schedule, p in [("S-Lle-Snc", 2), ("D-Lex-2cm", 2), ("D-Lle", 4)]:
        _, _, pres = _prefixes_of(schedule, k, g, p, 4)
        seen = []
        for pre in pres:
            seen += [tuple(t) for t in parallel.prefix_sequence(k, g, pre)]
        assert sorted(seen) == list(itertools.combinations(range(k), g))
        # each prefix costs C(k - 1 - c_p, g - p) (Sec. 3.1.2)
        assert sum(math.comb(k - 1 - c[-1], g - len(c)) for c in pres) == math.comb(k, g)


def test_pairs_take_both_ends():
    k, g, p = 10, 4, 2
    for name, key in [("D-Lex-2cm", lambda c: c), ("D-Lle-2cm", lambda c: c[::-1])]:
        _, nt, table = bz.debug_schedule(name, k, g, p, 30)
        order = sorted(itertools.combinations(range(k - (g - p)), p), key=key)
        assert nt == len(order) == 28
        for c, row in enumerate(table):
            if c < nt // 2:
                assert row == [order[c], order[nt - 1 - c]]
            else:
                assert row == []
    _, nt, table = bz.debug_schedule("D-Lex-2cm", 9, 4, 2, 12)      # odd count: a lone middle
    assert nt == 21 and table[10] == [list(itertools.combinations(range(7), 2))[10]] and table[11] == []


def test_snake_reverses_odd_turns():
    _, nt, table = bz.debug_schedule("S-Lex-Snc", 12, 5, 2, 4, 5)
    order = list(itertools.combinations(range(12 - 2), 3))
    for w in range(4):
        for s in range(5):
            t = s * 4 + (3 - w if s % 2 else w)
            assert table[w][s] == (order[t] if t < nt else None)


def test_errors():
    lib = bz.lib()
    assert lib.bz_debug_schedule(0, 10, 4, 2, 3, 3, None, 0, None, None) == bz.BZ_EINVAL
    assert lib.bz_debug_schedule(9, 10, 4, 2, 3, 3, None, 0, None, None) == bz.BZ_EINVAL
    assert lib.bz_debug_schedule(1, 10, 4, 0, 3, 3, None, 0, None, None) == bz.BZ_EINVAL
    assert lib.bz_debug_schedule(1, 10, 4, 2, 0, 3, None, 0, None, None) == bz.BZ_EINVAL
    assert lib.bz_debug_schedule(1, 10, 11, 2, 3, 3, None, 0, None, None) == bz.BZ_EINVAL
    import ctypes
    import numpy as np
    out = np.zeros(3, dtype=np.int32)
    assert lib.bz_debug_schedule(5, 10, 4, 2, 3, 3, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 3,
                                 None, None) == bz.BZ_ELIMIT
