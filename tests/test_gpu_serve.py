"""GPU: the resident server gives every request the result it gets alone.

bz_server_* keeps one persistent kernel on the device and admits requests
while others run on it (continuous batching). Each request's result must be
what bz_min_distance gives for that code alone: in statistics mode every field
(d, bounds, last level, combinations, each task's min, count and combinations),
whether the request ran alone on the server or in a mix with others. Its witness
must be a codeword of weight d. The plain searches run before the server starts:
a running server holds every compute unit.
"""
from __future__ import annotations

import time

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
    torch.cuda.init()
    return _bz


def _say(*a):
    print(*a, flush=True)


def _mixed_codes(seed, count):
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


def _same(a, b):
    assert a.status == b.status, (a.status, b.status)
    assert a.d == b.d
    assert (a.lower_bound, a.upper_bound, a.last_level) == (b.lower_bound, b.upper_bound, b.last_level)
    assert a.combinations == b.combinations
    assert [tuple(s) for s in a.stats] == [tuple(s) for s in b.stats]


def _plain(bz, items, **kw):
    out = []
    for G, n in items:
        c = bz.Code(G, n)
        out.append(bz.min_distance(c, raise_on_error=False, **kw))
        c.close()
    return out


def _run_mix(srv, hcodes, per_request=None, timeout=120.0):
    """Submits every code as soon as the server admits it; returns results in order."""
    per_request = per_request or [{}] * len(hcodes)
    nxt, tickets, done = 0, {}, {}
    t0 = time.perf_counter()
    while len(done) < len(hcodes):
        while nxt < len(hcodes):
            t = srv.submit(hcodes[nxt], **per_request[nxt])
            if t is None:
                break
            tickets[t] = nxt
            nxt += 1
        for t, res in srv.poll():
            done[tickets[t]] = res
        assert time.perf_counter() - t0 < timeout, "server did not finish the mix"
        time.sleep(100e-6)
    return [done[i] for i in range(len(hcodes))]


def test_alone_equals_mix_statistics(bz):
    items = _mixed_codes(21, 60)
    plain = _plain(bz, items, stats=True)
    hcodes = [bz.Code(G, n, host_only=True) for G, n in items]
    _say("server, statistics mode:", len(items), "codes alone, then mixed")
    with bz.Server(slots=64, stats=True) as srv:
        alone = [srv.wait(srv.submit(c)) for c in hcodes]
        mix = _run_mix(srv, hcodes)
    for (G, n), p, a, m in zip(items, plain, alone, mix):
        _same(a, p)
        _same(m, p)
        assert m.status == 0
        assert int(np.bitwise_count(m.witness).sum()) == m.d and bf.in_code(m.witness, G, n)
        assert int(np.bitwise_count(a.witness).sum()) == a.d and bf.in_code(a.witness, G, n)
        ref = oracle.min_distance(G, n)
        assert m.d == ref.d
        assert [tuple(s) for s in m.stats] == [tuple(s) for s in ref.stats]


def test_fast_mode_mix(bz):
    items = _mixed_codes(5, 60)
    hcodes = [bz.Code(G, n, host_only=True) for G, n in items]
    with bz.Server(slots=16) as srv:
        mix = _run_mix(srv, hcodes)
    for (G, n), m in zip(items, mix):
        ref = oracle.min_distance(G, n)
        assert m.status == 0 and m.d == ref.d
        assert int(np.bitwise_count(m.witness).sum()) == m.d and bf.in_code(m.witness, G, n)


def test_per_request_options_in_one_mix(bz):
    """level_stop and max_level are per request; the mix mixes them."""
    items = _mixed_codes(11, 24)
    opts = [dict(level_stop=bool(i % 2), max_level=(2 if i % 3 == 0 else 0)) for i in range(len(items))]
    plain = []
    for (G, n), o in zip(items, opts):
        plain += _plain(bz, [(G, n)], stats=True, **o)
    hcodes = [bz.Code(G, n, host_only=True) for G, n in items]
    with bz.Server(slots=32, stats=True) as srv:
        mix = _run_mix(srv, hcodes, opts)
    for p, m in zip(plain, mix):
        _same(m, p)


def test_relaunch_after_codes_per_launch(bz):
    """Five codes per kernel launch: the server drains and relaunches; results unchanged."""
    items = _mixed_codes(33, 23)
    plain = _plain(bz, items, stats=True)
    hcodes = [bz.Code(G, n, host_only=True) for G, n in items]
    with bz.Server(slots=4, stats=True, codes_per_launch=5) as srv:
        mix = _run_mix(srv, hcodes)
    for p, m in zip(plain, mix):
        _same(m, p)


def test_admission(bz):
    c = inputs.plain_code("plain128")
    hc = bz.Code(c.G, c.n, host_only=True)
    with bz.Server(slots=2) as srv:
        t1, t2 = srv.submit(hc), srv.submit(hc)
        assert t1 is not None and t2 is not None
        # both slots taken until polled: a third request is refused
        assert srv.submit(hc) is None
        r1, r2 = srv.wait(t1), srv.wait(t2)
        assert r1.d == r2.d == 16
        t3 = srv.submit(hc)
        assert t3 is not None and srv.wait(t3).d == 16
    with bz.Server(slots=8, hbm_budget=1024) as srv:
        assert srv.submit(hc) is None               # one request needs more than the budget
    with pytest.raises(bz.BZError):
        bz.min_distance(hc)                          # host-only codes are for servers


def test_serving_workload_sample(bz):
    """40 requests of the serving stream's code distribution (cost-capped), alone vs in the mix."""
    info = lambda c: bz.prepare_host(c.G, c.n)[1:3]
    kept, drawn, est = workloads.select(inputs.serve_code, info, 40, 1e9)
    _say("serving sample", len(kept), "of", drawn, "drawn; est. combinations", sum(est))
    plain = _plain(bz, [(c.G, c.n) for c in kept], stats=True)
    hcodes = [bz.Code(c.G, c.n, host_only=True) for c in kept]
    with bz.Server(slots=64, stats=True) as srv:
        mix = _run_mix(srv, hcodes)
    for c, p, m in zip(kept, plain, mix):
        _same(m, p)
        assert bf.in_code(m.witness, c.G, c.n)


def _large_serving_codes(bz, count, lo, hi):
    kept, i = [], 0
    while len(kept) < count:
        c = inputs.serve_code(i)
        i += 1
        mf, km = bz.prepare_host(c.G, c.n)[1:3]
        if lo <= workloads.estimated_cost(c.n, c.k, mf, km) <= hi:
            kept.append(c)
    return kept


def test_large_requests(bz):
    """Requests of 2e10-1e11 combinations, whose large tasks have thousands of tiles (claimed
    2, 4 or 8 at a time): statistics equal the plain search's, alone and mixed."""
    kept = _large_serving_codes(bz, 6, 2e10, 1e11)
    _say("large requests:", [(c.n, c.k) for c in kept])
    plain = _plain(bz, [(c.G, c.n) for c in kept], stats=True)
    hcodes = [bz.Code(c.G, c.n, host_only=True) for c in kept]
    with bz.Server(slots=16, stats=True) as srv:
        alone = [srv.wait(srv.submit(h)) for h in hcodes]
        mix = _run_mix(srv, hcodes)
    for c, p, a, m in zip(kept, plain, alone, mix):
        _same(a, p)
        _same(m, p)
        assert bf.in_code(m.witness, c.G, c.n) and bf.in_code(a.witness, c.G, c.n)
    # the batched search with as many tiles per task (multi-tile claims there too)
    objs = [bz.Code(c.G, c.n) for c in kept]
    outs, sts = bz.min_distance_batch(objs, stats=True, tiles_per_task=16384)
    for c, p, o, st in zip(kept, plain, outs, sts):
        assert st == 0
        _same(o, p)
        assert bf.in_code(o.witness, c.G, c.n)
    for o in objs:
        o.close()


def test_burst_of_requests(bz):
    """1000 requests of the serving distribution (estimated cost <= 1e9) submitted as one burst,
    up to 1024 in flight: every statistics-mode result equals the plain search's."""
    info = lambda c: bz.prepare_host(c.G, c.n)[1:3]
    kept, drawn, est = workloads.select(lambda i: inputs.serve_code(i, base_seed=5_000_000), info, 1000, 1e9)
    _say("burst:", len(kept), "requests of", drawn, "drawn; est. combinations", f"{sum(est):.3g}")
    hcodes = [bz.Code(c.G, c.n, host_only=True) for c in kept]
    with bz.Server(slots=1024, stats=True) as srv:
        mix = _run_mix(srv, hcodes, timeout=240.0)
    plain = _plain(bz, [(c.G, c.n) for c in kept], stats=True)
    for c, p, m in zip(kept, plain, mix):
        _same(m, p)
        assert m.status == 0 and bf.in_code(m.witness, c.G, c.n)
