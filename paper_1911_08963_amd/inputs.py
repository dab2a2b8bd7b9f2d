"""Seeded synthetic generator matrices for the minimum-distance workloads.

This module only draws random bits and packs them; it contains none of the
minimum-distance arithmetic, so both the GPU path and the CPU oracle may take
their inputs from it.

Packing convention (shared by every consumer): a k x n binary matrix is stored
row-major as ``uint64`` words, ``ld = ceil(n / 64)`` words per row, with
coordinate ``c`` of row ``i`` at bit ``c % 64`` of word ``G[i, c // 64]``
(least significant bit first); bits at positions >= n are zero.

Workloads (all bits iid Bernoulli(1/2) from ``numpy.random.default_rng(seed)``):

* ``plain40``  -- [40, 20] code, G = [I_20 | R], redrawn until R is invertible
  over GF(2), so that the last 20 columns form a second disjoint information set.
* ``plain128`` -- [128, 64] code, G = [I_64 | R], redrawn until R is invertible
  (two disjoint information sets).
* ``plain192`` -- [192, 64] rate-1/3 code, G = [I_64 | R1 | R2], redrawn until
  R1 and R2 are both invertible (three disjoint information sets).
* ``batch_code(i)`` -- n uniform in [48, 160], rho uniform in [0.33, 0.6],
  k = round(n rho), G = [I_k | R]; no redraw.
* ``serve_code(i)`` -- n uniform in [64, 192], k uniform in [ceil(n/3), floor(n/2)],
  G = [I_k | R]; no redraw.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "pack_rows", "unpack_rows", "systematic", "gf2_rank_dense", "random_systematic",
    "plain_code", "batch_code", "serve_code", "serve_arrivals", "PLAIN_WORKLOADS",
    "Code",
]


@dataclass
class Code:
    """A generator matrix with its provenance."""
    G: np.ndarray          # (k, ceil(n/64)) uint64, packed as described above
    n: int
    k: int
    seed: int
    draws: int = 1         # how many matrices were drawn to satisfy the workload's rule
    name: str = ""

    @property
    def ld(self) -> int:
        return int(self.G.shape[1])


def pack_rows(bits: np.ndarray) -> np.ndarray:
    """Pack a (k, n) 0/1 array into (k, ceil(n/64)) uint64 words, LSB first."""
    bits = np.asarray(bits, dtype=np.uint8)
    k, n = bits.shape
    ld = max(1, (n + 63) // 64)
    padded = np.zeros((k, ld * 64), dtype=np.uint8)
    padded[:, :n] = bits
    by = np.packbits(padded.reshape(k, ld * 8, 8), axis=2, bitorder="little").reshape(k, ld * 8)
    return by.view("<u8").reshape(k, ld).astype(np.uint64)


def unpack_rows(G: np.ndarray, n: int) -> np.ndarray:
    """Inverse of :func:`pack_rows`: (k, ld) uint64 -> (k, n) uint8."""
    G = np.ascontiguousarray(G, dtype="<u8")
    k, ld = G.shape
    by = G.view(np.uint8).reshape(k, ld * 8)
    bits = np.unpackbits(by, axis=1, bitorder="little")
    return bits[:, :n].copy()


def gf2_rank_dense(M: np.ndarray) -> int:
    """Rank over GF(2) of a small dense 0/1 matrix (used only by the redraw rules)."""
    A = (np.asarray(M, dtype=np.uint8) & 1).copy()
    rows, cols = A.shape
    r = 0
    for c in range(cols):
        if r == rows:
            break
        nz = np.nonzero(A[r:, c])[0]
        if nz.size == 0:
            continue
        p = r + int(nz[0])
        if p != r:
            A[[r, p]] = A[[p, r]]
        mask = A[:, c].astype(bool)
        mask[r] = False
        A[mask] ^= A[r]
        r += 1
    return r


def systematic(R: np.ndarray) -> np.ndarray:
    """[I_k | R] as a dense (k, k + cols(R)) 0/1 array."""
    k = R.shape[0]
    return np.concatenate([np.eye(k, dtype=np.uint8), R.astype(np.uint8)], axis=1)


def random_systematic(rng: np.random.Generator, n: int, k: int) -> np.ndarray:
    """Draw R (k x (n-k)) iid Bernoulli(1/2) and return dense [I_k | R]."""
    R = rng.integers(0, 2, size=(k, n - k), dtype=np.uint8)
    return systematic(R)


def _plain(name: str, n: int, k: int, seed: int, blocks: int, max_draws: int = 10_000) -> Code:
    rng = np.random.default_rng(seed)
    for draw in range(1, max_draws + 1):
        R = rng.integers(0, 2, size=(k, n - k), dtype=np.uint8)
        if all(gf2_rank_dense(R[:, b * k:(b + 1) * k]) == k for b in range(blocks)):
            return Code(pack_rows(systematic(R)), n, k, seed, draw, name)
    raise RuntimeError(f"{name}: no admissible draw in {max_draws} attempts")


# name -> (n, k, default seed, number of k x k blocks of R that must be invertible)
PLAIN_WORKLOADS = {
    "plain40": (40, 20, 1, 1),
    "plain128": (128, 64, 2, 1),
    "plain192": (192, 64, 3, 2),
}


def plain_code(name: str, seed: int | None = None) -> Code:
    n, k, s0, blocks = PLAIN_WORKLOADS[name]
    return _plain(name, n, k, s0 if seed is None else seed, blocks)


def batch_code(i: int, base_seed: int = 1_000_000) -> Code:
    """Code i of the batched workload: n ~ U{48..160}, rho ~ U[0.33, 0.6], k = round(n rho)."""
    seed = base_seed + i
    rng = np.random.default_rng(seed)
    n = int(rng.integers(48, 161))
    rho = float(rng.uniform(0.33, 0.6))
    k = int(math.floor(n * rho + 0.5))
    return Code(pack_rows(random_systematic(rng, n, k)), n, k, seed, 1, f"batch{i}")


def serve_code(i: int, base_seed: int = 2_000_000) -> Code:
    """Request i of the serving workload: n ~ U{64..192}, k ~ U{ceil(n/3)..floor(n/2)}."""
    seed = base_seed + i
    rng = np.random.default_rng(seed)
    n = int(rng.integers(64, 193))
    k = int(rng.integers(-(-n // 3), n // 2 + 1))
    return Code(pack_rows(random_systematic(rng, n, k)), n, k, seed, 1, f"serve{i}")


def serve_arrivals(rate_hz: float = 200.0, duration_s: float = 60.0, seed: int = 7) -> np.ndarray:
    """Poisson arrival times (seconds) with exponential gaps of mean 1/rate over [0, duration)."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    while True:
        t += float(rng.exponential(1.0 / rate_hz))
        if t >= duration_s:
            break
        out.append(t)
    return np.asarray(out, dtype=np.float64)
