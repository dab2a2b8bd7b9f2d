"""Workload assembly for the batched and serving runs: a cost estimate per code.

Random codes of the batched and serving shapes ([48..192] bits, rate 1/3 to
0.6) have wildly uneven cost: a few need 10^15 or more row combinations. The
runs therefore keep only codes whose *estimated* cost is under a cap. The
estimate takes the expected weight distribution of a random systematic code
and the code's actual information-set structure (m_f, k_m).

* Expected number of codewords of weight i (c != 0 of the k information bits,
  the n - k redundancy bits uniform): E_i = (C(n, i) - C(n - k, i)) / 2^(n - k).
* d_est = the smallest w with 1 - exp(-(E_1 + ... + E_w)) >= 1/2.
* Cost: the C(k, g) of every (Gamma_j, g) task in search order, until the
  certified lower bound after a task reaches d_est.

The estimate only selects codes; every kept code is solved exactly.
"""
from __future__ import annotations

import math


def d_estimate(n: int, k: int) -> int:
    acc = 0.0
    for w in range(1, n + 1):
        acc += (math.comb(n, w) - math.comb(n - k, w)) / 2.0 ** (n - k)
        if 1.0 - math.exp(-acc) >= 0.5:
            return w
    return n - k + 1


def _certified(j: int, g: int, m_f: int, k_m: int, k: int) -> int:
    if j >= m_f:
        extra = (g + 1 - k + k_m) if k_m else 0
        return m_f * (g + 1) + max(0, extra)
    extra = (g - k + k_m) if k_m else 0
    return (j + 1) * (g + 1) + (m_f - j - 1) * g + max(0, extra)


def estimated_cost(n: int, k: int, m_f: int, k_m: int) -> int:
    """Row combinations the search is expected to enumerate."""
    if k == n:
        return 0
    d = min(d_estimate(n, k), n - k + 1)
    nsets = m_f + (1 if k_m else 0)
    total = 0
    for g in range(1, k + 1):
        for j in range(nsets):
            total += math.comb(k, g)
            if _certified(j, g, m_f, k_m, k) >= d:
                return total
    return total


def select(draw, info, count: int, cap: float, max_draws: int = 1_000_000):
    """Draw codes with draw(i) and keep those with estimated cost <= cap.

    info(code) -> (m_f, k_m). Returns (kept codes, number drawn, estimated costs of the kept)."""
    kept, costs = [], []
    i = 0
    while len(kept) < count and i < max_draws:
        c = draw(i)
        i += 1
        m_f, k_m = info(c)
        est = estimated_cost(c.n, c.k, m_f, k_m)
        if est <= cap:
            kept.append(c)
            costs.append(est)
    return kept, i, costs


def level_within(n: int, k: int, m_f: int, k_m: int, budget: float) -> int:
    """The deepest level g >= 1 whose tasks (every Gamma_j at levels 1..g) enumerate at most
    budget combinations in all: a request limited to it stays within that budget."""
    nsets = m_f + (1 if k_m else 0)
    total, g = 0, 0
    while g < k:
        nxt = total + nsets * math.comb(k, g + 1)
        if nxt > budget:
            break
        total, g = nxt, g + 1
    return max(g, 1)
