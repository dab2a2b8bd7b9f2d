"""Independent brute force over all 2^k codewords (numpy), used to pin the oracle.

It never eliminates: the codewords are the XORs of subsets of G's rows, built by
doubling (codewords of rows 0..i-1, then those XOR row i). Weights are
popcounts. Nothing here shares code with the oracle or the GPU library.
"""
from __future__ import annotations

import numpy as np

MAX_K = 22


def all_codewords(G: np.ndarray, k: int) -> np.ndarray:
    """(2^k, ld) uint64: entry c (as a k-bit integer, bit i = row i) is c*G."""
    if k > MAX_K:
        raise ValueError("brute force limited to k <= %d" % MAX_K)
    G = np.asarray(G, dtype=np.uint64)
    cw = np.zeros((1, G.shape[1]), dtype=np.uint64)
    for i in range(k):
        cw = np.concatenate([cw, cw ^ G[i][None, :]], axis=0)
    return cw


def weights(words: np.ndarray) -> np.ndarray:
    return np.bitwise_count(words).sum(axis=1).astype(np.int64)


def index_weights(k: int) -> np.ndarray:
    """wt(c) for every c in [0, 2^k), in the same order as all_codewords."""
    w = np.zeros(1, dtype=np.int64)
    for _ in range(k):
        w = np.concatenate([w, w + 1])
    return w


def weight_distribution(G: np.ndarray, n: int, k: int) -> np.ndarray:
    """A_0..A_n."""
    w = weights(all_codewords(G, k))
    return np.bincount(w, minlength=n + 1)[: n + 1]


def min_distance(G: np.ndarray, n: int, k: int) -> int:
    w = weights(all_codewords(G, k))[1:]
    return int(w.min())


def restricted_stats(G: np.ndarray, n: int, k: int, cols) -> dict:
    """For every value a of wt(x|S) (S = cols) over nonzero codewords x:
    (min wt(x), number of x reaching it)."""
    cw = all_codewords(G, k)[1:]
    mask = np.zeros(G.shape[1], dtype=np.uint64)
    for c in cols:
        mask[c // 64] |= np.uint64(1) << np.uint64(c % 64)
    a = weights(cw & mask[None, :])
    w = weights(cw)
    out = {}
    for val in np.unique(a):
        sel = w[a == val]
        m = int(sel.min())
        out[int(val)] = (m, int((sel == m).sum()))
    return out


def subset_level_stats(rows: np.ndarray, k: int) -> dict:
    """For the k given rows (packed): for every g, (min wt(c*rows), count) over wt(c) = g."""
    cw = all_codewords(rows, k)
    w = weights(cw)
    cwt = index_weights(k)
    out = {}
    for g in range(1, k + 1):
        sel = w[cwt == g]
        m = int(sel.min())
        out[g] = (m, int((sel == m).sum()), int(sel.size))
    return out


def gf2_rank(words: np.ndarray, n: int) -> int:
    """Rank over GF(2) of packed rows (a separate elimination from every other one here)."""
    from paper_1911_08963_amd.inputs import unpack_rows
    A = unpack_rows(np.asarray(words, dtype=np.uint64), n).astype(np.uint8)
    r = 0
    rows = A.shape[0]
    for c in range(n):
        piv = None
        for i in range(r, rows):
            if A[i, c]:
                piv = i
                break
        if piv is None:
            continue
        A[[r, piv]] = A[[piv, r]]
        for i in range(rows):
            if i != r and A[i, c]:
                A[i] ^= A[r]
        r += 1
        if r == rows:
            break
    return r


def dual_generator(G: np.ndarray, n: int, k: int) -> np.ndarray:
    """A generator of the dual code, from a dense reduced echelon form."""
    from paper_1911_08963_amd.inputs import pack_rows, unpack_rows
    A = unpack_rows(np.asarray(G, dtype=np.uint64), n).astype(np.uint8)
    piv = []
    r = 0
    for c in range(n):
        p = None
        for i in range(r, k):
            if A[i, c]:
                p = i
                break
        if p is None:
            continue
        A[[r, p]] = A[[p, r]]
        for i in range(k):
            if i != r and A[i, c]:
                A[i] ^= A[r]
        piv.append(c)
        r += 1
    free = [c for c in range(n) if c not in piv]
    H = np.zeros((len(free), n), dtype=np.uint8)
    for t, f in enumerate(free):
        H[t, f] = 1
        for i, p in enumerate(piv):
            H[t, p] = A[i, f]
    return pack_rows(H)


def krawtchouk(n: int, j: int, i: int) -> int:
    from math import comb
    return sum((-1) ** s * comb(i, s) * comb(n - i, j - s) for s in range(0, j + 1))


def macwilliams(A: np.ndarray, n: int, k: int) -> np.ndarray:
    """Weight distribution of the dual from that of the code."""
    B = []
    for j in range(n + 1):
        tot = sum(int(A[i]) * krawtchouk(n, j, i) for i in range(n + 1))
        assert tot % (1 << k) == 0
        B.append(tot >> k)
    return np.asarray(B, dtype=np.int64)


def in_code(x: np.ndarray, G: np.ndarray, n: int) -> bool:
    """x is in the row space of G iff appending it does not raise the rank."""
    G = np.asarray(G, dtype=np.uint64)
    return gf2_rank(np.vstack([G, np.asarray(x, dtype=np.uint64)[None, : G.shape[1]]]), n) == gf2_rank(G, n)
