"""Pins of the CPU oracle against facts that do not come from the oracle itself.

* the paper's printed lexicographic list (Sec. 3.1.3) and prefix examples (Sec. 3.1);
* brute force over all 2^k codewords (tests/bruteforce.py, numpy, no elimination),
  itself pinned by the MacWilliams identity and by textbook weight distributions;
* textbook codes with known minimum distance;
* Singleton and Griesmer bounds, witness membership, C(k, g) counts;
* the certified lower bounds, checked codeword by codeword.
"""
from __future__ import annotations

import math
import os

import numpy as np
import pytest

import bruteforce as bf
import codes
import oracle
from oracle import parallel
from paper_1911_08963_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_orders():
    out = {"lex": [], "colex": []}
    with open(os.path.join(GOLDEN, "paper_subset_orders.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            out[t[0]].append(tuple(int(x) for x in t[2:]))
    return out


def test_lex_order_matches_paper():
    assert oracle.lex_sequence(5, 3) == _golden_orders()["lex"]


def test_prefix_examples_match_paper():
    rows = {}
    with open(os.path.join(GOLDEN, "paper_prefix_examples.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            rows.setdefault(t[0], []).append([int(x) for x in t[1:]])
    seq = parallel.prefix_sequence(9, 5, (0, 1, 2))
    assert [list(s) for s in seq[:3]] == rows["expand_start"]
    # after (0,1,2,3,x) for x up to k-1 comes (0,1,2,4,5), then (0,1,2,4,6)
    i = seq.index((0, 1, 2, 4, 5))
    assert seq[i + 1] == (0, 1, 2, 4, 6)
    assert all(s[:3] == (0, 1, 2) for s in seq)
    assert len(seq) == math.comb(9 - 3, 2)
    k, g, p, mx = rows["valid_max"][0]
    # the last valid prefix is (k-1-(g-p)-2, ..., k-1-(g-p)); no prefix contains 5 at k=6
    assert parallel.prefix_count(k, g, p) == math.comb(mx + 1, p)
    assert parallel.prefix_sequence(k, g, (0, 1, 5)) == []
    single = rows["single_completion"][0]
    assert parallel.prefix_sequence(single[0], single[1], tuple(single[2:5])) == [tuple(single[2:])]
    for k, g, p in [(6, 4, 3), (11, 4, 3), (20, 7, 3), (30, 9, 4)]:
        assert parallel.prefix_count(k, g, p) == math.comb(k - (g - p), p)


def test_binomial_closed_form():
    for a in range(0, 97):
        for b in range(0, 20):
            if math.comb(a, b) < 2 ** 63:      # the range the enumeration may use
                assert oracle.binomial(a, b) == math.comb(a, b)


# ---------------------------------------------------------------- brute force pins

def _rand_code(rng, n, k, systematic=True):
    if systematic:
        G = inputs.random_systematic(rng, n, k)
    else:
        while True:
            G = rng.integers(0, 2, size=(k, n), dtype=np.uint8)
            if inputs.gf2_rank_dense(G) == k:
                break
    return inputs.pack_rows(G)


def test_bruteforce_known_distributions():
    G, n, k, d = codes.golay23()
    A = bf.weight_distribution(G, n, k)
    want = {0: 1, 7: 253, 8: 506, 11: 1288, 12: 1288, 15: 506, 16: 253, 23: 1}
    assert {i: int(a) for i, a in enumerate(A) if a} == want
    G, n, k, d = codes.hamming7()
    A = bf.weight_distribution(G, n, k)
    assert list(A) == [1, 0, 0, 7, 7, 0, 0, 1]


def test_bruteforce_macwilliams():
    rng = np.random.default_rng(11)
    for _ in range(25):
        n = int(rng.integers(6, 20))
        k = int(rng.integers(1, n))
        G = _rand_code(rng, n, k, systematic=bool(rng.integers(0, 2)))
        A = bf.weight_distribution(G, n, k)
        H = bf.dual_generator(G, n, k)
        assert H.shape[0] == n - k
        B = bf.weight_distribution(H, n, n - k) if n - k > 0 else np.eye(1, n + 1, 0, dtype=np.int64)[0]
        assert list(bf.macwilliams(A, n, k)) == list(B)


# ---------------------------------------------------------------- textbook codes

STRUCTURED = [
    ("repetition9", lambda: codes.repetition(9)),
    ("even_weight12", lambda: codes.even_weight(12)),
    ("whole_space10", lambda: codes.whole_space(10)),
    ("hamming7", codes.hamming7),
    ("ext_hamming8", lambda: codes.extend(codes.hamming7())),
    ("golay23", codes.golay23),
    ("golay24", lambda: codes.extend(codes.golay23())),
    ("simplex3", lambda: codes.simplex(3)),
    ("simplex5", lambda: codes.simplex(5)),
    ("rm13", lambda: codes.reed_muller(1, 3)),
    ("rm24", lambda: codes.reed_muller(2, 4)),
    ("rm15", lambda: codes.reed_muller(1, 5)),
    ("rm25", lambda: codes.reed_muller(2, 5)),
    ("rm26", lambda: codes.reed_muller(2, 6)),
    ("rm36", lambda: codes.reed_muller(3, 6)),
    ("rm17", lambda: codes.reed_muller(1, 7)),
]


@pytest.mark.parametrize("name,builder", STRUCTURED, ids=[s[0] for s in STRUCTURED])
def test_structured_codes_known_distance(name, builder):
    G, n, k, d = builder()
    for level_stop in (False, True):
        r = oracle.min_distance(G, n, level_stop=level_stop)
        assert r.status == 0
        assert r.d == d, (name, r.d, d)
        assert int(np.bitwise_count(r.witness).sum()) == d
        assert bf.in_code(r.witness, G, n)
    if k <= bf.MAX_K:
        assert bf.min_distance(G, n, k) == d


@pytest.mark.slow
def test_rm37_shape_of_plain128():
    """RM(3,7) = [128, 64, 16]: the [128,64] shape with a known distance and many ties."""
    G, n, k, d = codes.reed_muller(3, 7)
    r = oracle.min_distance(G, n)
    assert r.status == 0 and r.d == 16
    assert bf.in_code(r.witness, G, n)


# ---------------------------------------------------------------- random codes vs brute force

def _griesmer(k, d):
    return sum(-(-d // (1 << i)) for i in range(k))


def _pivot_columns(rows, n, order):
    """Pivot (first nonzero in the given column order) of each packed row."""
    A = inputs.unpack_rows(rows, n)
    piv = []
    for r in A:
        nz = [c for c in order if r[c]]
        piv.append(nz[0] if nz else -1)
    return piv


def _check_code(G, n, k, check_bounds_per_codeword=True):
    r = oracle.min_distance(G, n)
    rl = oracle.min_distance(G, n, level_stop=True)
    d = bf.min_distance(G, n, k)
    assert r.status == 0 and rl.status == 0
    assert r.d == d and rl.d == d
    for res in (r, rl):
        assert int(np.bitwise_count(res.witness).sum()) == d
        assert bf.in_code(res.witness, G, n)
        for (j, g, mn, cnt, comb) in res.stats:
            assert comb == math.comb(k, g)
    assert d <= n - k + 1                      # Singleton
    assert n >= _griesmer(k, d)                # Griesmer

    soc, m_f, k_m, gam = oracle.prepare(G, n)
    assert (r.num_full, r.partial_rank) == (m_f, k_m)
    sets = [[c for c in range(n) if soc[c] == j] for j in range(m_f + (k_m > 0))]
    for j, S in enumerate(sets):
        assert len(S) == (k if j < m_f else k_m)
        rows = gam[j * k:(j + 1) * k]
        assert bf.gf2_rank(rows, n) == k
        assert bf.gf2_rank(np.vstack([rows, G]), n) == k        # same code
        A = inputs.unpack_rows(rows, n)
        if j < m_f:
            assert np.array_equal(A[:, S], np.eye(k, dtype=np.uint8))
        else:
            assert np.array_equal(A[:k_m][:, S], np.eye(k_m, dtype=np.uint8))
            assert not A[k_m:][:, S].any()
    # the greedy is canonical: S_1 is the lexicographically first basis
    A = inputs.unpack_rows(G, n)
    chosen = []
    for c in range(n):
        if inputs.gf2_rank_dense(A[:, chosen + [c]]) > len(chosen):
            chosen.append(c)
        if len(chosen) == k:
            break
    assert chosen == sets[0]

    # per-(j, g) statistics: for a full-rank S_j they are the code invariant
    # (min wt(x), count) over x with wt(x|S_j) = g; for the partial matrix they
    # are the brute-force statistics of its rows.
    for j, S in enumerate(sets):
        if j < m_f:
            ref = bf.restricted_stats(G, n, k, S)
            for (jj, g, mn, cnt, comb) in r.stats:
                if jj == j:
                    assert ref[g] == (mn, cnt), (j, g)
        else:
            ref = bf.subset_level_stats(gam[j * k:(j + 1) * k], k)
            for (jj, g, mn, cnt, comb) in r.stats:
                if jj == j:
                    assert ref[g] == (mn, cnt, comb), (j, g)

    if check_bounds_per_codeword:
        # every codeword not yet enumerated after task (j*, g*) has weight >= the certified bound
        cw = bf.all_codewords(G, k)[1:]
        w = bf.weights(cw)
        Ab = inputs.unpack_rows(cw, n)
        lev = []
        for j, S in enumerate(sets):
            if j < m_f:
                lev.append(Ab[:, S].sum(axis=1))
            else:
                rows = gam[j * k:(j + 1) * k]
                order = S + [c for c in range(n) if c not in S]
                piv = _pivot_columns(rows, n, order)
                lev.append(Ab[:, piv].sum(axis=1))
        nsets = len(sets)
        for g in range(1, k + 1):
            for js in range(nsets):
                seen = np.zeros(len(w), dtype=bool)
                for j in range(nsets):
                    done = g if j <= js else g - 1
                    seen |= lev[j] <= done
                Lb = oracle.certified_bound(js, g, m_f, k_m, k)
                if (~seen).any():
                    assert w[~seen].min() >= Lb, (g, js)
            Lg = oracle.level_bound(g, m_f, k_m, k)
            seen = np.zeros(len(w), dtype=bool)
            for j in range(nsets):
                seen |= lev[j] <= g
            if (~seen).any():
                assert w[~seen].min() >= Lg
    return r


def test_random_codes_vs_bruteforce():
    rng = np.random.default_rng(1234)
    npart = 0
    for t in range(160):
        n = int(rng.integers(4, 26))
        k = int(rng.integers(1, min(n, 13) + 1))
        G = _rand_code(rng, n, k, systematic=bool(t % 3))
        r = _check_code(G, n, k, check_bounds_per_codeword=(t % 4 == 0))
        npart += int(r.partial_rank > 0)
    assert npart > 40          # the partial matrix is exercised


def test_codes_with_zero_and_repeated_columns():
    rng = np.random.default_rng(99)
    for t in range(30):
        n = int(rng.integers(8, 22))
        k = int(rng.integers(2, min(n - 2, 10) + 1))
        while True:
            A = rng.integers(0, 2, size=(k, n), dtype=np.uint8)
            A[:, rng.integers(0, n)] = 0
            c = int(rng.integers(0, n))
            A[:, (c + 1) % n] = A[:, c]
            if inputs.gf2_rank_dense(A) == k:
                break
        _check_code(inputs.pack_rows(A), n, k)


def test_plain40_vs_bruteforce():
    c = inputs.plain_code("plain40")
    r = _check_code(c.G, c.n, c.k, check_bounds_per_codeword=False)
    assert r.num_full == 2 and r.partial_rank == 0


def test_rank_deficient_and_invalid():
    G = inputs.pack_rows(np.array([[1, 0, 1, 1], [1, 0, 1, 1]], dtype=np.uint8))
    assert oracle.min_distance(G, 4).status == oracle.OR_ERANK
    assert oracle.min_distance(G[:, :1], 300).status == oracle.OR_EINVAL


def test_max_level_limits_search():
    c = inputs.plain_code("plain40")
    r = oracle.min_distance(c.G, c.n, max_level=1)
    assert r.status in (0, oracle.OR_ELIMIT)
    assert all(s[1] <= 1 for s in r.stats)


def test_parallel_oracle_matches_serial():
    rng = np.random.default_rng(5)
    import multiprocessing as mp
    with mp.get_context("fork").Pool(3) as pool:
        for t in range(12):
            n = int(rng.integers(10, 40))
            k = int(rng.integers(3, min(n, 16) + 1))
            G = _rand_code(rng, n, k)
            a = oracle.min_distance(G, n)
            for p in (1, 2, 3):
                b = parallel.min_distance_parallel(G, n, nprocs=3, prefix=p, pool=pool)
                assert b["d"] == a.d
                assert [s[:4] for s in b["stats"]] == [s[:4] for s in a.stats]
                assert bf.in_code(b["witness"], G, n)


def test_plain192_full_run_golden_is_consistent():
    """The stored full [192, 64] run (multi-process oracle) against what pins it down:
    its first 18 tasks equal the single-process oracle's run to level 6, every task
    enumerated all C(64, g) sums, the witness is a codeword of weight d, and the
    bound certified after the last task (Sec. 2.1, three full Gamma_j) reaches d."""
    import json
    here = os.path.join(os.path.dirname(__file__), "golden")
    full = json.load(open(os.path.join(here, "plain192_oracle.json")))
    to6 = json.load(open(os.path.join(here, "plain_oracle.json")))["plain192"]["per_gamma"]
    c = inputs.plain_code("plain192")
    assert full["draws"] == c.draws
    assert full["stats"][:len(to6["stats"])] == to6["stats"]
    assert all(s[4] == math.comb(64, s[1]) for s in full["stats"])
    assert full["combinations"] == sum(s[4] for s in full["stats"])
    w = np.asarray(full["witness"], dtype=np.uint64)
    assert int(np.bitwise_count(w).sum()) == full["d"] == 35
    assert bf.in_code(w, c.G, c.n)
    j, g = full["stats"][-1][:2]
    m_f = 3
    assert (j + 1) * (g + 1) + (m_f - j - 1) * g >= full["d"]
    # one task earlier the certificate was still short of d
    pj, pg = full["stats"][-2][:2]
    assert (pj + 1) * (pg + 1) + (m_f - pj - 1) * pg < full["d"]
    assert min(s[2] for s in full["stats"]) == full["d"]


# ---------------------------------------------------------------- codewords of a given weight

def _rm_min_weight_count(r, m):
    """A_{2^(m-r)} of RM(r, m) (MacWilliams & Sloane, Ch. 13, Thm. 9)."""
    num = den = 1
    for i in range(m - r):
        num *= (1 << (m - i)) - 1
        den *= (1 << (m - r - i)) - 1
    return (1 << r) * num // den


@pytest.mark.parametrize("name,builder,w,want", [
    ("hamming7", codes.hamming7, 3, 7), ("hamming7", codes.hamming7, 4, 7),
    ("golay23", codes.golay23, 7, 253), ("golay23", codes.golay23, 8, 506),
    ("golay24", lambda: codes.extend(codes.golay23()), 8, 759),
    ("golay24", lambda: codes.extend(codes.golay23()), 12, 2576),
    ("rm26", lambda: codes.reed_muller(2, 6), 16, _rm_min_weight_count(2, 6)),
    ("rm17", lambda: codes.reed_muller(1, 7), 64, 254),
    ("simplex5", lambda: codes.simplex(5), 16, 31),
])
def test_count_weight_textbook(name, builder, w, want):
    G, n, k, d = builder()
    cnt, cws, lvl = oracle.count_weight(G, n, w, cap=4)
    assert cnt == want
    for x in cws:
        assert int(np.bitwise_count(x).sum()) == w and bf.in_code(x, G, n)


def test_count_weight_vs_bruteforce():
    rng = np.random.default_rng(77)
    for t in range(14):
        n = int(rng.integers(8, 40))
        k = int(rng.integers(2, min(n, 14) + 1))
        G = _rand_code(rng, n, k)
        cw = bf.all_codewords(G, k)[1:]
        wts = bf.weights(cw)
        d = int(wts.min())
        for w in (d, d + 1, d + 2):
            want = sorted(tuple(int(v) for v in x) for x, wt in zip(cw, wts) if wt == w)
            cnt, got, _ = oracle.count_weight(G, n, w, cap=len(want) + 1)
            assert cnt == len(want), (t, w)
            keys = sorted(tuple(int(v) for v in x[: cw.shape[1]]) for x in got)
            assert keys == want
        # and with permuted information sets
        assert oracle.count_weight(G, n, d, perm_trials=9, perm_seed=t)[0] == int((wts == d).sum())
