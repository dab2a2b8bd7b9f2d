"""GPU: the batched persistent search equals the single-code search, code by code.

bz_min_distance_batch runs every code's whole level loop inside one captured
graph launch (device-side task advance). Each code's result must equal what
bz_min_distance gives for it alone -- d, bounds, last level, every per-task
(min, count, combinations) in statistics mode -- and match the CPU oracle on the
codes small enough to run it here.
"""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import bruteforce as bf
import codes as textbook
import oracle
from paper_1911_08963_amd import inputs, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bz():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1911_08963_amd import bz as _bz
    _bz.lib()
    return _bz


def _say(*a):
    print(*a, flush=True)


def _mixed_codes(seed=99, count=90):
    rng = np.random.default_rng(seed)
    out = []
    for t in range(count):
        n = int(rng.integers(6, 96))
        k = int(rng.integers(1, min(n, 22) + 1))
        if t % 3 == 0:
            G = inputs.pack_rows(inputs.random_systematic(rng, n, k))
        else:
            while True:
                A = rng.integers(0, 2, size=(k, n), dtype=np.uint8)
                if inputs.gf2_rank_dense(A) == k:
                    break
            G = inputs.pack_rows(A)
        out.append((G, n))
    for builder in (lambda: textbook.whole_space(9), lambda: textbook.repetition(17), textbook.golay23,
                    lambda: textbook.reed_muller(2, 6), lambda: textbook.simplex(5)):
        G, n, k, d = builder()
        out.append((G, n))
    return out


def _check_same(bz, a, b):
    assert a.status == b.status
    assert a.d == b.d
    assert (a.lower_bound, a.upper_bound, a.last_level) == (b.lower_bound, b.upper_bound, b.last_level)
    assert a.combinations == b.combinations
    assert [tuple(s) for s in a.stats] == [tuple(s) for s in b.stats]


@pytest.mark.parametrize("level_stop", [False, True])
def test_batch_equals_plain_statistics(bz, level_stop):
    items = _mixed_codes()
    objs = [bz.Code(G, n) for G, n in items]
    _say("batch", len(objs), "codes, statistics mode, level_stop", level_stop)
    outs, sts = bz.min_distance_batch(objs, stats=True, level_stop=level_stop)
    for i, ((G, n), code, got) in enumerate(zip(items, objs, outs)):
        alone = bz.min_distance(code, stats=True, level_stop=level_stop, raise_on_error=False)
        _check_same(bz, got, alone)
        assert sts[i] == 0
        ref = oracle.min_distance(G, n, level_stop=level_stop)
        assert got.d == ref.d
        assert [tuple(s) for s in got.stats] == [tuple(s) for s in ref.stats]
        assert int(np.bitwise_count(got.witness).sum()) == got.d
        assert bf.in_code(got.witness, G, n)
    for c in objs:
        c.close()


def test_batch_fast_mode_and_witnesses(bz):
    items = _mixed_codes(seed=5, count=60)
    objs = [bz.Code(G, n) for G, n in items]
    outs, sts = bz.min_distance_batch(objs)
    for (G, n), code, got, st in zip(items, objs, outs, sts):
        assert st == 0
        ref = oracle.min_distance(G, n)
        assert got.d == ref.d
        assert int(np.bitwise_count(got.witness).sum()) == got.d
        assert bf.in_code(got.witness, G, n)
    for c in objs:
        c.close()


def test_batch_workload_sample_equals_plain(bz):
    """64 codes of the batched workload (cost-capped) against their single-code runs."""
    info = lambda c: bz.prepare_host(c.G, c.n)[1:3]
    kept, drawn, est = workloads.select(inputs.batch_code, info, 64, 1e9)
    objs = [bz.Code(c.G, c.n) for c in kept]
    _say("workload sample", len(objs), "of", drawn, "drawn; est. combinations", sum(est))
    outs, sts = bz.min_distance_batch(objs, stats=True)
    for c, code, got, st in zip(kept, objs, outs, sts):
        assert st == 0
        alone = bz.min_distance(code, stats=True)
        _check_same(bz, got, alone)
        assert bf.in_code(got.witness, c.G, c.n)
    fast, sts2 = bz.min_distance_batch(objs)
    for c, a, b in zip(kept, outs, fast):
        assert a.d == b.d
        assert bf.in_code(b.witness, c.G, c.n)
    for c in objs:
        c.close()


def test_batch_max_level_and_cancel(bz):
    import torch
    items = _mixed_codes(seed=11, count=20)
    objs = [bz.Code(G, n) for G, n in items]
    outs, sts = bz.min_distance_batch(objs, stats=True, max_level=2)
    for (G, n), got, st in zip(items, outs, sts):
        ref = oracle.min_distance(G, n, max_level=2)
        assert st == ref.status
        assert got.d == ref.d
        assert [tuple(s) for s in got.stats] == [tuple(s) for s in ref.stats]
    flag = torch.ones(1, dtype=torch.int32).pin_memory()
    ptr = ctypes.cast(flag.data_ptr(), ctypes.POINTER(ctypes.c_uint32))
    outs, sts = bz.min_distance_batch(objs, cancel=ptr)
    big = [i for i, c in enumerate(objs) if c.k != c.n]
    assert all(sts[i] == bz.BZ_ECANCELED for i in big)
    for c in objs:
        c.close()
