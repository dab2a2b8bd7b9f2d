"""GPU parity on the workloads' own code distributions, against stored oracle runs.

tests/golden/workload_oracle.json holds CPU-oracle results (written by
tests/golden/make_golden_workloads.py, which calls only oracle/) for codes of
the batched and serving distributions, many with a partial Gamma_m (the
[[I_{k_m}, A], [0, B]] block of Sec. 2.1) enumerated on levels of up to 2.2e9
sums, and for the plain workloads at further seeds. Every path of the library
must reproduce them exactly in statistics mode: the single-code search, the
batched persistent launch and the resident server. Compared: status, d, the
final bounds, the last level, the total combinations and every per-(Gamma_j, g)
(min weight, count at min, combinations); the witness must be a codeword of
weight d.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np
import pytest

import bruteforce as bf
from paper_1911_08963_amd import inputs

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "workload_oracle.json")


@pytest.fixture(scope="module")
def bz():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1911_08963_amd import bz as _bz
    _bz.lib()
    torch.cuda.init()
    return _bz


@pytest.fixture(scope="module")
def gold():
    with open(GOLDEN) as f:
        return json.load(f)


def _say(*a):
    print(*a, flush=True)


def _code_of(kind, e):
    if kind == "batch":
        c = inputs.batch_code(e["index"])
    elif kind == "serve":
        c = inputs.serve_code(e["index"])
    else:
        c = inputs.plain_code(e["name"], e["seed"])
    assert (c.n, c.k, c.seed) == (e["n"], e["k"], e["seed"])
    return c


def _match(got, e, c, tag):
    assert got.status == e["status"], (tag, got.status, e["status"])
    assert got.d == e["d"], tag
    assert (got.lower_bound, got.upper_bound, got.last_level) == \
        (e["lower_bound"], e["upper_bound"], e["last_level"]), tag
    assert got.combinations == e["combinations"], tag
    assert [list(s) for s in got.stats] == e["stats"], tag
    if got.d:
        assert int(np.bitwise_count(got.witness).sum()) == got.d, tag
        assert bf.in_code(got.witness, c.G, c.n), tag


def test_plain_seeds(bz, gold):
    """plain40 and plain128 at three more seeds (both stop modes), plain192 to level 6 at two."""
    for e in gold["plain"]:
        c = _code_of("plain", e)
        tag = f"{e['name']} seed {e['seed']} {e['mode']}"
        _say("case", tag)
        code = bz.Code(c.G, c.n)
        assert (code.num_full, code.partial_rank) == (e["num_full"], e["partial_rank"])
        got = bz.min_distance(code, stats=True, level_stop=e["mode"] == "per_level",
                              max_level=e["max_level"], raise_on_error=False)
        _match(got, e, c, tag)
        code.close()


@pytest.mark.parametrize("kind", ["batch", "serve"])
def test_single_search_on_workload_codes(bz, gold, kind):
    for e in gold[kind]:
        c = _code_of(kind, e)
        tag = f"{kind} {e['index']} [{c.n},{c.k}] k_m={e['partial_rank']} ({e['group']})"
        _say("case", tag)
        code = bz.Code(c.G, c.n)
        assert (code.num_full, code.partial_rank) == (e["num_full"], e["partial_rank"])
        got = bz.min_distance(code, stats=True, raise_on_error=False)
        _match(got, e, c, tag)
        code.close()


def test_batched_launch_on_workload_codes(bz, gold):
    """All 48 codes of both distributions in one batched persistent launch."""
    entries = [("batch", e) for e in gold["batch"]] + [("serve", e) for e in gold["serve"]]
    codes = [_code_of(k, e) for k, e in entries]
    objs = [bz.Code(c.G, c.n) for c in codes]
    _say("batched launch of", len(objs), "codes, statistics mode")
    outs, sts = bz.min_distance_batch(objs, stats=True)
    for (k, e), c, got, st in zip(entries, codes, outs, sts):
        tag = f"batched {k} {e['index']} [{c.n},{c.k}]"
        assert st == e["status"], tag
        _match(got, e, c, tag)
    fast, sts = bz.min_distance_batch(objs)
    for (k, e), c, got, st in zip(entries, codes, fast, sts):
        assert st == 0 and got.d == e["d"], (k, e["index"])
        assert bf.in_code(got.witness, c.G, c.n)
    for o in objs:
        o.close()


def test_server_on_workload_codes(bz, gold):
    """All 48 codes submitted to the resident server together (statistics mode)."""
    entries = [("serve", e) for e in gold["serve"]] + [("batch", e) for e in gold["batch"]]
    codes = [_code_of(k, e) for k, e in entries]
    hcodes = [bz.Code(c.G, c.n, host_only=True) for c in codes]
    _say("server mix of", len(hcodes), "codes, statistics mode")
    done, tickets = {}, {}
    with bz.Server(slots=64, stats=True) as srv:
        nxt = 0
        t0 = time.perf_counter()
        while len(done) < len(hcodes):
            while nxt < len(hcodes):
                t = srv.submit(hcodes[nxt])
                if t is None:
                    break
                tickets[t] = nxt
                nxt += 1
            for t, res in srv.poll():
                done[tickets[t]] = res
            assert time.perf_counter() - t0 < 100.0, "server did not finish the mix"
            time.sleep(100e-6)
    for i, ((k, e), c) in enumerate(zip(entries, codes)):
        _match(done[i], e, c, f"served {k} {e['index']} [{c.n},{c.k}]")
