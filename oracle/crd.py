"""Nested-set probabilities of confidence-region detection, from one SOV
sweep (test infrastructure: see the package header).

Section III-C with Algorithm 1 of Section IV-A detects the excursion region of a Gaussian field
by ordering the sites by marginal exceedance probability and evaluating
P(X_i in [a_i, b_i] for i in S_k) for the nested sets S_k = {first k sites},
k = 1..n.  With the sites in that order, the SOV recurrence of Eq. (sov1) for
the first k rows involves only the leading k x k block of L, which is the
Cholesky factor of the leading block of Sigma; so the running product
d_1 ... d_k of every sample is a sample of the k-site problem, and one sweep
gives every P(S_k) as the mean over samples of those running products.

(The QMC points of row i are those of the n-site problem; the estimate of
P(S_k) is therefore not the k-site call's estimate on its own points, but an
estimate of the same probability from the same estimator.)
"""
from __future__ import annotations

import numpy as np
import scipy.special as sp

from .qmc import lattice, shifts, points
from .sov import condition, reduce_samples


def sweep_prefix(L: np.ndarray, at: np.ndarray, bt: np.ndarray, N: int, S: int, seed: int,
                 periodize: bool = False, dim: int | None = None) -> np.ndarray:
    """Running log-products: ell[k, c] = sum_{i <= k} log d_i of sample c,
    for every row k (the recurrence of ``sov.sweep``, recorded after each
    row).  ``dim``: the dimension of the problem whose leading rows L, at
    and bt are (default: L's own); it fixes the QMC shifts, which are
    numbered s * dim + i, so the first rows of a large problem can be
    evaluated without the rest."""
    n = L.shape[0]
    dim = n if dim is None else int(dim)
    if dim < n:
        raise ValueError("dim must be at least the number of rows")
    cols = np.arange(N * S, dtype=np.int64)
    A = lattice(n)
    D = shifts(seed, dim, S)
    Y = np.zeros((n, cols.size))
    run = np.zeros(cols.size)
    ell = np.zeros((n, cols.size))
    for i in range(n):
        s = L[i, :i] @ Y[:i] if i > 0 else np.zeros(cols.size)
        lii = L[i, i]
        with np.errstate(all="ignore"):
            alpha = (at[i] - s) / lii
            beta = (bt[i] - s) / lii
        w = points(i, cols, A, D, N, periodize)
        y, logd = condition(alpha, beta, w)
        Y[i] = y
        run = run + logd
        ell[i] = run
    return ell


def prefix_probs(L: np.ndarray, at: np.ndarray, bt: np.ndarray, N: int, S: int, seed: int,
                 periodize: bool = False, dim: int | None = None) -> dict:
    """log P-hat(S_k) for k = 1..n (index k - 1) and its relative standard
    error over the S shifts (NaN for S == 1), each reduced exactly as the
    full estimate (mean over a shift's N points, then over shifts).
    ``dim`` as in ``sweep_prefix``."""
    ell = sweep_prefix(L, at, bt, N, S, seed, periodize, dim)
    n = ell.shape[0]
    logp = np.empty(n)
    rel = np.empty(n)
    for k in range(n):
        r = reduce_samples(ell[k], N, S)
        logp[k] = r["logP"]
        rel[k] = r["rel_stderr"]
    return {"logP": logp, "rel_stderr": rel}


def exceedance_order(mu: np.ndarray, sd: np.ndarray, u: float) -> np.ndarray:
    """Sites in order of decreasing marginal exceedance probability
    P(X_i > u) = 1 - Phi((u - mu_i) / sd_i) (ties in site order)."""
    p = sp.ndtr((np.asarray(mu, dtype=np.float64) - u) / np.asarray(sd, dtype=np.float64))
    return np.argsort(-p, kind="stable")
