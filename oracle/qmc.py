"""Randomised Richtmyer lattice points (the uniform matrix R of Algorithm 2).

The paper fills R with U(0,1) values and calls the method quasi-Monte Carlo
without naming the point set.  The reading used here: Richtmyer's lattice
w = frac(j * sqrt(p_{i+1}) + Delta_{s,i}) with p_k the k-th prime, points
j = 1..N, and S independent random shifts Delta_s.  Everything is defined in
64-bit integer arithmetic so that two implementations produce identical
points:

  A_i       = floor(frac(sqrt(p_{i+1})) * 2^64)  = isqrt(p_{i+1} * 2^128) mod 2^64
  D_{s,i}   = output number s*n + i (0-based) of SplitMix64 seeded with
              ``seed`` (Steele, Lea & Flood, OOPSLA 2014)
  x         = (j * A_i + D_{s,i}) mod 2^64
  w         = ((x >> 11) + 1/2) * 2^-53          (never 0 or 1)

Sample column c = s*N + (j - 1) holds shift s, point j.
"""
from __future__ import annotations

import math

import numpy as np

MASK64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def first_primes(count: int) -> list[int]:
    """The first ``count`` primes by a sieve of Eratosthenes."""
    if count <= 0:
        return []
    limit = max(16, int(count * (math.log(count + 1) + math.log(math.log(count + 3)) + 3)))
    while True:
        sieve = bytearray([1]) * (limit + 1)
        sieve[0:2] = b"\x00\x00"
        for q in range(2, math.isqrt(limit) + 1):
            if sieve[q]:
                sieve[q * q::q] = bytearray(len(range(q * q, limit + 1, q)))
        primes = [i for i in range(limit + 1) if sieve[i]]
        if len(primes) >= count:
            return primes[:count]
        limit *= 2


def lattice(n: int) -> np.ndarray:
    """Generating vector A_0..A_{n-1} as uint64 (exact integer square roots)."""
    return np.array([math.isqrt(p << 128) & MASK64 for p in first_primes(n)], dtype=np.uint64)


def splitmix64(seed: int, k: int) -> int:
    """Output number k (0-based) of SplitMix64 started from state ``seed``."""
    z = (seed + (k + 1) * _GAMMA) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def shifts(seed: int, n: int, S: int) -> np.ndarray:
    """D[s, i] = SplitMix64 output s*n + i, shape (S, n), uint64."""
    return np.array([[splitmix64(seed, s * n + i) for i in range(n)] for s in range(S)],
                    dtype=np.uint64).reshape(S, n)


def points(i: int, cols: np.ndarray, A: np.ndarray, D: np.ndarray, N: int,
           periodize: bool = False) -> np.ndarray:
    """w for dimension i at the given global sample columns (float64 array)."""
    cols = np.asarray(cols, dtype=np.int64)
    s = cols // N
    j = (cols % N + 1).astype(np.uint64)
    with np.errstate(over="ignore"):
        x = j * A[i] + D[s, i]          # uint64 arithmetic wraps mod 2^64
    w = ((x >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53
    if periodize:
        w = 1.0 - np.abs(2.0 * w - 1.0)  # baker's transform
    return w
