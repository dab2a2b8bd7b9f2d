"""Pins of the information-set permutation search (CPU).

Sec. 2.2 finds information sets by trying random column permutations. The
library and the oracle each implement the same published generator (SplitMix64
driving a Fisher-Yates shuffle; trial 0 is the natural order) and keep the
trial with the most full-rank sets, then the largest leftover rank. Here:
- the generator against its published reference outputs;
- the shuffle: a permutation, identity at trial 0, uniform over many trials;
- the selection rule against an independent greedy written with numpy ranks;
- d, the witness and every per-(Gamma_j, g) statistic against brute force
  on the permuted sets;
- the library's host preparation (host-only codes, no device) equal to the
  oracle's, set for set and row for row.
"""
from __future__ import annotations

import math
import os
from collections import Counter

import numpy as np
import pytest

import bruteforce as bf
import codes
import oracle
from paper_1911_08963_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_reference.txt")


def _rand_code(rng, n, k):
    while True:
        A = rng.integers(0, 2, size=(k, n), dtype=np.uint8)
        if inputs.gf2_rank_dense(A) == k:
            return inputs.pack_rows(A)


def test_splitmix64_reference_outputs():
    want = [int(l, 16) for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert oracle.splitmix64(0, len(want)) == want


def test_trial_orders_are_uniform_permutations():
    assert oracle.trial_order(12, 0, 99) == list(range(12))
    for t in range(1, 20):
        assert sorted(oracle.trial_order(40, t, 5)) == list(range(40))
    assert oracle.trial_order(40, 3, 5) == oracle.trial_order(40, 3, 5)
    assert oracle.trial_order(40, 3, 5) != oracle.trial_order(40, 3, 6)
    # all 120 orders of 5 columns, about equally often (a shuffle that never
    # leaves an entry in place, or skips one, fails this by far)
    from scipy.stats import chisquare
    cnt = Counter(tuple(oracle.trial_order(5, t, 7)) for t in range(1, 24001))
    assert len(cnt) == 120
    assert chisquare([cnt[p] for p in cnt]).pvalue > 1e-4


def _greedy_sets(A, k, scan):
    """Independent greedy: numpy ranks over the scan order (Sec. 2.1)."""
    taken, full = set(), []
    while True:
        chosen = []
        for c in scan:
            if c in taken:
                continue
            if inputs.gf2_rank_dense(A[:, chosen + [c]]) > len(chosen):
                chosen.append(c)
                if len(chosen) == k:
                    break
        if len(chosen) == k:
            full.append(sorted(chosen))
            taken |= set(chosen)
            continue
        return full, sorted(chosen)


@pytest.mark.parametrize("trials,seed", [(5, 1), (30, 77)])
def test_selection_rule_matches_independent_greedy(trials, seed):
    rng = np.random.default_rng(100 + trials)
    for t in range(12):
        n = int(rng.integers(8, 36))
        k = int(rng.integers(2, min(n, 12) + 1))
        G = _rand_code(rng, n, k)
        A = inputs.unpack_rows(G, n)
        best = None
        for tr in range(trials):
            full, part = _greedy_sets(A, k, oracle.trial_order(n, tr, seed))
            key = (len(full), len(part))
            if best is None or key > best[0]:
                best = (key, full, part)
        soc, m_f, k_m, gam = oracle.prepare(G, n, perm_trials=trials, perm_seed=seed)
        assert (m_f, k_m) == best[0]
        sets = best[1] + ([best[2]] if best[2] else [])
        assert [[c for c in range(n) if soc[c] == j] for j in range(len(sets))] == sets


def test_rm17_reaches_sixteen_full_sets():
    """RM(1,7) = [128, 8]: 128/8 = 16 disjoint information sets exist; natural order finds 11."""
    G, n, k, d = codes.reed_muller(1, 7)
    assert oracle.prepare(G, n)[1:3] == (11, 7)
    soc, m_f, k_m, _ = oracle.prepare(G, n, perm_trials=200, perm_seed=1)
    assert (m_f, k_m) == (16, 0)
    r = oracle.min_distance(G, n, perm_trials=200, perm_seed=1)
    assert r.d == d == 64 and (r.num_full, r.partial_rank) == (16, 0)


def test_permuted_sets_search_against_bruteforce():
    rng = np.random.default_rng(8)
    for t in range(10):
        n = int(rng.integers(10, 40))
        k = int(rng.integers(3, min(n, 14) + 1))
        G = _rand_code(rng, n, k)
        d = bf.min_distance(G, n, k)
        for level_stop in (False, True):
            r = oracle.min_distance(G, n, perm_trials=20, perm_seed=t, level_stop=level_stop)
            assert r.status == 0 and r.d == d
            assert int(np.bitwise_count(r.witness).sum()) == d and bf.in_code(r.witness, G, n)
        soc, m_f, k_m, gam = oracle.prepare(G, n, perm_trials=20, perm_seed=t)
        assert (r.num_full, r.partial_rank) == (m_f, k_m)
        sets = [[c for c in range(n) if soc[c] == j] for j in range(m_f + (k_m > 0))]
        r = oracle.min_distance(G, n, perm_trials=20, perm_seed=t)
        for j, S in enumerate(sets):
            if j < m_f:
                ref = bf.restricted_stats(G, n, k, S)
                for (jj, g, mn, cnt, comb) in r.stats:
                    if jj == j:
                        assert ref[g] == (mn, cnt) and comb == math.comb(k, g)
            else:
                ref = bf.subset_level_stats(gam[j * k:(j + 1) * k], k)
                for (jj, g, mn, cnt, comb) in r.stats:
                    if jj == j:
                        assert ref[g] == (mn, cnt, comb)


def test_library_host_prepare_equals_oracle_with_permutations():
    from paper_1911_08963_amd import bz
    rng = np.random.default_rng(3)
    for t in range(20):
        n = int(rng.integers(10, 90))
        k = int(rng.integers(2, min(n, 30) + 1))
        G = _rand_code(rng, n, k) if t % 2 else inputs.pack_rows(inputs.random_systematic(rng, n, k))
        for trials, seed in ((0, 0), (8, 11), (40, 12345)):
            c = bz.Code(G, n, perm_trials=trials, perm_seed=seed, host_only=True)
            soc, m_f, k_m, gam = oracle.prepare(G, n, perm_trials=trials, perm_seed=seed)
            assert (c.num_full, c.partial_rank) == (m_f, k_m)
            assert (c.set_of_column == soc).all()
            for j in range(c.nsets):
                assert (c.gamma(j) == gam[j * k:(j + 1) * k]).all()
            c.close()
