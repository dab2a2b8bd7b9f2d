"""GPU: autotuning picks among tilings that all give the same results.

bz_autotune times (slots per lane, tiles per wave) candidates on a synthetic
task and installs the fastest for that row width; bz_autotune_batch does the
same for a batch's tiles per task. Neither may change a result: searches with
the installed choices must equal the searches with the fixed rules, field by
field in statistics mode.
"""
from __future__ import annotations

import numpy as np
import pytest

import bruteforce as bf
from paper_1911_08963_amd import inputs, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bz():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1911_08963_amd import bz as _bz
    _bz.lib()
    _bz.autotune_clear()
    yield _bz
    _bz.autotune_clear()


def _same(a, b):
    assert (a.status, a.d, a.lower_bound, a.upper_bound, a.last_level, a.combinations) == \
        (b.status, b.d, b.lower_bound, b.upper_bound, b.last_level, b.combinations)
    assert [tuple(s) for s in a.stats] == [tuple(s) for s in b.stats]


def test_autotune_plain(bz):
    c = inputs.plain_code("plain128")
    code = bz.Code(c.G, c.n)
    before = bz.min_distance(code, stats=True)
    e = bz.autotune(code.W_full, code.k)
    print("tuned", e, flush=True)
    assert e["W"] == code.W_full and e["k"] == 64
    assert e["slots_per_lane"] in (2, 4, 8, 16) and e["tiles_per_wave"] in (1, 2, 4, 8, 16, 64)
    assert e["comb_per_s"] >= e["default_comb_per_s"] > 0
    assert bz.autotune_get(code.W_full) == e
    after = bz.min_distance(code, stats=True)              # runs with the installed choice
    _same(after, before)
    fast = bz.min_distance(code)
    assert fast.d == before.d and bf.in_code(fast.witness, c.G, c.n)
    code.close()
    for W in (1, 3, 6):
        e = bz.autotune(W, 48)
        assert e["comb_per_s"] >= e["default_comb_per_s"] > 0


def test_autotune_batch(bz):
    info = lambda c: bz.prepare_host(c.G, c.n)[1:3]
    kept, drawn, est = workloads.select(inputs.batch_code, info, 96, 1e9)
    objs = [bz.Code(c.G, c.n) for c in kept]
    before, sts = bz.min_distance_batch(objs, stats=True, tiles_per_task=64)
    t, sec = bz.autotune_batch(objs)
    print("batch tiles per task", t, "best", sec, flush=True)
    assert t in (16, 64, 256, 1024) and sec > 0
    after, sts2 = bz.min_distance_batch(objs, stats=True)   # with the installed tiles per task
    for a, b, c in zip(after, before, kept):
        _same(a, b)
        assert bf.in_code(a.witness, c.G, c.n)
    for o in objs:
        o.close()
