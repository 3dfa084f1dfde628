"""Monte Carlo check of nested-set probabilities (test infrastructure: see
the package header).

Section V-C validates detected confidence regions by plain Monte Carlo:
draw fields from the fitted distribution, X = mu + L Z with Z standard
normal and L the Cholesky factor of Sigma, and take the fraction of fields
that meet the event on every site of the region.  Since the regions of
Algorithm 1 are nested (the first k sites in exceedance order), one set of
draws gives every nested set at once: a field meets the event on the first
k sites exactly when its first failing site comes at or after k.

Normals are drawn from a counter-based generator, so that any column of
draws can be produced on its own:

  U_k     = ((SplitMix64 output k of ``seed``) >> 11) + 1/2) * 2^-53
  Z[i, j] = Phi^-1(U_{j n + i})      (site i, sample j, n sites)

(SplitMix64 as in ``qmc.splitmix64``: Steele, Lea & Flood, OOPSLA 2014.)
"""
from __future__ import annotations

import numpy as np
import scipy.special as sp

from .qmc import splitmix64


def uniforms(seed: int, n: int, cols) -> np.ndarray:
    """U for sites 0..n-1 and the given sample columns, shape (n, len(cols))."""
    cols = np.asarray(cols, dtype=np.int64)
    out = np.empty((n, cols.size))
    for c, j in enumerate(cols):
        for i in range(n):
            out[i, c] = (float(splitmix64(seed, int(j) * n + i) >> 11) + 0.5) * 2.0 ** -53
    return out


def normals(seed: int, n: int, cols) -> np.ndarray:
    """Z[i, c] = Phi^-1(U) for sites 0..n-1 and the given sample columns."""
    return sp.ndtri(uniforms(seed, n, cols))


def fields(L: np.ndarray, mu, seed: int, cols) -> np.ndarray:
    """X = mu + L Z for the given sample columns, shape (n, len(cols))."""
    n = L.shape[0]
    mu = np.zeros(n) if mu is None else np.asarray(mu, dtype=np.float64)
    return mu[:, None] + L @ normals(seed, n, cols)


def first_failure(X: np.ndarray, a, b) -> np.ndarray:
    """Per column of X: the first site i with X_i outside [a_i, b_i]
    (a NaN limit never holds), or n if every site is inside."""
    a = np.asarray(a, dtype=np.float64)[:, None]
    b = np.asarray(b, dtype=np.float64)[:, None]
    inside = (a <= X) & (X <= b)
    n = X.shape[0]
    fail = ~inside
    return np.where(fail.any(axis=0), np.argmax(fail, axis=0), n)


def prefix_counts(first: np.ndarray, n: int) -> np.ndarray:
    """count[k - 1] = number of samples inside the limits on the first k
    sites, k = 1..n: the samples whose first failure is at or after k."""
    first = np.asarray(first)
    return np.array([int(np.sum(first >= k)) for k in range(1, n + 1)], dtype=np.int64)


def mc_prefix(L: np.ndarray, a, b, mu, M: int, seed: int, cols=None) -> dict:
    """First failing site of every sample column (all M, or the given
    columns) and, over all M, the per-prefix counts."""
    n = L.shape[0]
    cols = np.arange(M) if cols is None else np.asarray(cols, dtype=np.int64)
    first = first_failure(fields(L, mu, seed, cols), a, b)
    out = {"first": first}
    if cols.size == M:
        out["count"] = prefix_counts(first, n)
    return out
