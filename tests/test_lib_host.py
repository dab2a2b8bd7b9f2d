"""CPU tests of libbz: exported symbols, host preparation and the level planner.

The library is loaded, never asked to touch a device here.
"""
from __future__ import annotations

import itertools
import math
import os
import re

import numpy as np
import pytest

import oracle
from paper_1911_08963_amd import bz, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(bz_[a-z_0-9]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_library_exports_every_declared_function():
    lib = bz.lib()
    names = _declared_functions()
    assert "bz_prepare" in names and "bz_min_distance" in names and "bz_min_distance_batch" in names
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings():
    lib = bz.lib()
    for s in range(-7, 1):
        assert lib.bz_status_str(s)


def test_prepare_argument_errors():
    G = inputs.pack_rows(np.array([[1, 0, 1, 1], [1, 0, 1, 1]], dtype=np.uint8))
    with pytest.raises(bz.BZError) as e:
        bz.prepare_host(G, 4)
    assert e.value.status == bz.BZ_ERANK
    with pytest.raises(bz.BZError) as e:
        bz.prepare_host(G[:1], 300)
    assert e.value.status == bz.BZ_EINVAL
    G1 = inputs.pack_rows(np.eye(3, 5, dtype=np.uint8))
    with pytest.raises(bz.BZError) as e:
        bz.prepare_host(G1, 2)          # k > n
    assert e.value.status == bz.BZ_EINVAL


def _rand(rng, n, k, systematic):
    if systematic:
        return inputs.pack_rows(inputs.random_systematic(rng, n, k))
    while True:
        A = rng.integers(0, 2, size=(k, n), dtype=np.uint8)
        if inputs.gf2_rank_dense(A) == k:
            return inputs.pack_rows(A)


def test_prepare_matches_oracle_bit_exact():
    """Gamma_j is the unique reduced echelon form for its column order, so the
    library's Gamma_j must equal the oracle's word for word."""
    rng = np.random.default_rng(77)
    seen_partial = 0
    for t in range(200):
        n = int(rng.integers(2, 200))
        k = int(rng.integers(1, min(n, 100) + 1))
        G = _rand(rng, n, k, bool(t % 2))
        soc, mf, km, gam, packed = bz.prepare_host(G, n)
        soc2, mf2, km2, gam2 = oracle.prepare(G, n)
        assert (mf, km) == (mf2, km2)
        assert np.array_equal(soc, soc2)
        assert np.array_equal(gam, gam2)
        seen_partial += km > 0
        # packed rows are Gamma_j restricted to the columns outside S_j
        bits = inputs.unpack_rows(gam, n)
        off = 0
        for j in range(mf + (km > 0)):
            cols = [c for c in range(n) if soc[c] != j]
            W = (len(cols) + 31) // 32
            for i in range(k):
                words = packed[off:off + W]
                off += W
                want = np.zeros(W * 32, dtype=np.uint8)
                want[:len(cols)] = bits[j * k + i, cols]
                got = np.unpackbits(words.view(np.uint8), bitorder="little")
                assert np.array_equal(got, want)
    assert seen_partial > 30
    # k above 128: the column vectors are built from three or four 64-row blocks
    for t in range(12):
        n = int(rng.integers(150, 257))
        k = int(rng.integers(129, n + 1))
        G = _rand(rng, n, k, bool(t % 2))
        soc, mf, km, gam, _ = bz.prepare_host(G, n)
        soc2, mf2, km2, gam2 = oracle.prepare(G, n)
        assert (mf, km) == (mf2, km2)
        assert np.array_equal(soc, soc2) and np.array_equal(gam, gam2)


def test_prepare_plain_workloads():
    for name, (mf, km) in [("plain40", (2, 0)), ("plain128", (2, 0)), ("plain192", (3, 0))]:
        c = inputs.plain_code(name)
        soc, m, k_m, gam, _ = bz.prepare_host(c.G, c.n)
        assert (m, k_m) == (mf, km)
        # the generator rule makes S_j the j-th block of k columns
        for j in range(m):
            assert [x for x in range(c.n) if soc[x] == j] == list(range(j * c.k, (j + 1) * c.k))


def _rect_subsets(r):
    lane = [tuple(r["lane_off"] + x for x in s) for s in itertools.combinations(range(r["lane_n"]), r["lane_t"])]
    head = [tuple(r["head_off"] + x for x in s) for s in itertools.combinations(range(r["head_n"]), r["head_t"])]
    for a in lane:
        for b in head:
            yield tuple(sorted(a + b))


@pytest.mark.parametrize("slots", [2, 8, 16])
def test_plan_covers_every_subset_once(slots):
    for k in list(range(1, 15)) + [17, 20]:
        for g in range(1, k + 1):
            if math.comb(k, g) > 20000:
                continue
            rects, tiles, ht = bz.plan_level(k, g, slots=slots, target_tiles=64)
            got = sorted(s for r in rects for s in _rect_subsets(r))
            assert got == list(itertools.combinations(range(k), g)), (k, g)


@pytest.mark.parametrize("slots", [2, 16])
def test_widened_tiles_cover_each_pair_once(slots):
    """Walking the tiles as the kernels do (tile -> rectangle, lane block lb of
    lane_mult blocks, head block hb) visits every (lane rank, head rank) pair of
    every rectangle exactly once."""
    widened = False
    for k, g, ht in ((20, 5, 32), (24, 6, 64), (30, 4, 32), (17, 3, 32), (40, 4, 64)):
        rects, tiles, used = bz.plan_level(k, g, slots=slots, heads_per_tile=ht, widen=True)
        assert used == ht
        items = 64 * slots
        seen = {}
        for tile in range(tiles):
            ri = max(i for i, r in enumerate(rects) if r["tile_begin"] <= tile)
            r = rects[ri]
            local = tile - r["tile_begin"]
            lb, hb = divmod(local, r["head_blocks"])
            for sb in range(r["lane_mult"]):
                base = (lb * r["lane_mult"] + sb) * items
                if base >= r["lane_count"]:
                    break
                for q in range(base, min(base + items, r["lane_count"])):
                    for h in range(hb * ht, min(hb * ht + ht, r["head_count"])):
                        seen[(ri, q, h)] = seen.get((ri, q, h), 0) + 1
        assert all(v == 1 for v in seen.values())
        assert len(seen) == math.comb(k, g)
        widened = widened or any(r["lane_mult"] > 1 for r in rects)
    assert widened


@pytest.mark.parametrize("widen", [False, True])
@pytest.mark.parametrize("k,g", [(64, 7), (64, 11), (96, 12), (150, 9), (200, 6), (256, 8), (40, 20)])
def test_plan_invariants(k, g, widen):
    for slots in (2, 4, 8, 16):
        rects, tiles, ht = bz.plan_level(k, g, slots=slots, target_tiles=8192, widen=widen)
        tot = 0
        tb = 0
        for r in rects:
            assert r["head_n"] <= 64 and r["head_t"] <= r["head_n"]
            assert r["lane_t"] >= 1
            assert r["lane_count"] == math.comb(r["lane_n"], r["lane_t"])
            assert r["head_count"] == math.comb(r["head_n"], r["head_t"])
            assert r["lane_t"] + r["head_t"] == g
            # disjoint ranges
            if r["head_t"]:
                a = set(range(r["lane_off"], r["lane_off"] + r["lane_n"]))
                b = set(range(r["head_off"], r["head_off"] + r["head_n"]))
                assert not (a & b)
            assert r["lane_off"] + r["lane_n"] <= k and r["head_off"] + r["head_n"] <= k
            assert r["tile_begin"] == tb
            # a tile: lane_mult blocks of 64 * slots lane subsets by ht heads, and no
            # more lane subsets than ht full heads would give it
            m = r["lane_mult"]
            assert m >= 1 and (widen or m == 1)
            assert m * min(r["head_count"], ht) <= ht or m == 1
            if widen and r["head_count"] < ht:
                # a lane block's setup counts as 12 head steps
                assert m == max(1, min(-(-r["lane_count"] // (64 * slots)), (ht + 12) // (r["head_count"] + 12)))
            assert r["lane_blocks"] == -(-(-(-r["lane_count"] // (64 * slots))) // m)
            assert r["head_blocks"] == -(-r["head_count"] // ht)
            tb += r["lane_blocks"] * r["head_blocks"]
            tot += r["lane_count"] * r["head_count"]
        assert tot == math.comb(k, g)
        assert tb == tiles < 2 ** 40


def test_autotune_table_set_get_clear():
    """bz_autotune_set / _get / _clear manage the per-process tuning table (no device needed)."""
    from paper_1911_08963_amd import bz
    bz.autotune_clear()
    assert bz.autotune_get(4) is None
    bz.autotune_set(4, 16, 2)
    e = bz.autotune_get(4)
    assert (e["W"], e["slots_per_lane"], e["tiles_per_wave"]) == (4, 16, 2)
    for bad in ((0, 8, 4), (9, 8, 4), (4, 3, 4), (5, 16, 4), (4, 8, 0)):
        with pytest.raises(bz.BZError):
            bz.autotune_set(*bad)
    bz.autotune_clear()
    assert bz.autotune_get(4) is None
