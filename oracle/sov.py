"""The SOV estimator of the MVN probability (paper Section III-B, Eq. (sov1)
and Eq. (sov2); organised as in Algorithms 2 and 3), in log space.

For one sample (shift s, point j) and rows i = 0..n-1 in order:

  s_i   = sum_{k<i} L_ik y_k
  a'_i  = (a~_i - s_i) / L_ii ,   b'_i = (b~_i - s_i) / L_ii
  d_i   = Phi(b'_i) - Phi(a'_i)
  y_i   = Phi^{-1}( Phi(a'_i) + w_i d_i )
  l     = sum_i log d_i                       (the sample's log of prod d_i)

and the estimate is the mean of exp(l) over all samples.  Readings of the
paper used here (each is listed with its reason in the design notes):

* Eq. (sov1) gives y_i = Phi^{-1}[Phi(a') + w (Phi(b') - Phi(a'))]; the
  QMC listing drops the Phi(a') term, which is taken as a typo.
* Limits are centred, a~ = a - mu, b~ = b - mu; L is the factor of Sigma
  itself, not of the correlation matrix.
* Products of n factors underflow FP64 at the workload sizes, so every
  sample keeps l = log prod d_i and the mean is a log-sum-exp.
* Evaluation is arranged to avoid cancellation, by exact identities:
  if a' > 0 the interval is reflected, (a', b', w) -> (-b', -a', 1-w) and
  y -> -y, so the lower end is never in the upper tail; y is taken from
  Phi^{-1}(p) if p = Phi(a') + u d <= 1/2, else from -Phi^{-1}(q) with
  q = Phi(-b') + (1-u) d = 1 - p; when b' < -35 (both ends deep in the
  lower tail) d and p are formed from log Phi values.
* A sample whose interval has zero mass gets l = -inf and y = 0.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.special as sp

from .qmc import lattice, shifts, points

DEEP_TAIL = -35.0


def centre(a, b, mu=None):
    """a~ = a - mu, b~ = b - mu (infinite limits stay infinite)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if mu is None:
        return a.copy(), b.copy()
    mu = np.asarray(mu, dtype=np.float64)
    return a - mu, b - mu


def condition(alpha: np.ndarray, beta: np.ndarray, w: np.ndarray):
    """One conditioning step for a row: returns (y, log d) per sample."""
    cw = 1.0 - w
    refl = alpha > 0.0
    lo = np.where(refl, -beta, alpha)
    hi = np.where(refl, -alpha, beta)
    u = np.where(refl, cw, w)
    v = np.where(refl, w, cw)
    with np.errstate(all="ignore"):
        # ordinary range: probabilities in linear scale
        pa = sp.ndtr(lo)
        pb = sp.ndtr(hi)
        qb = sp.ndtr(-hi)
        d = pb - pa
        p = pa + u * d
        q = qb + v * d
        y_lin = np.where(p <= 0.5, sp.ndtri(p), -sp.ndtri(q))
        logd_lin = np.log(d)
        # both ends deep in the lower tail: log scale
        la = sp.log_ndtr(lo)
        lb = sp.log_ndtr(hi)
        logd_log = lb + np.log1p(-np.exp(la - lb))
        lp = np.logaddexp(la, np.log(u) + logd_log)
        y_log = sp.ndtri_exp(lp)
    deep = hi < DEEP_TAIL
    y = np.where(deep, y_log, y_lin)
    logd = np.where(deep, logd_log, logd_lin)
    dead = ~(logd > -np.inf)
    y = np.where(dead, 0.0, y)
    logd = np.where(dead, -np.inf, logd)
    y = np.where(refl, -y, y)
    return y, logd


def sweep(L: np.ndarray, at: np.ndarray, bt: np.ndarray, N: int, S: int, seed: int,
          cols=None, periodize: bool = False, return_y: bool = False):
    """Per-sample log-products l_c for the sample columns ``cols``
    (default: all N*S).  Rows are processed in order, samples in parallel,
    which is the only parallelism the recurrence allows (Section IV-C)."""
    n = L.shape[0]
    if cols is None:
        cols = np.arange(N * S, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    A = lattice(n)
    D = shifts(seed, n, S)
    Y = np.zeros((n, cols.size))
    ell = np.zeros(cols.size)
    for i in range(n):
        s = L[i, :i] @ Y[:i] if i > 0 else np.zeros(cols.size)
        lii = L[i, i]
        with np.errstate(all="ignore"):
            alpha = (at[i] - s) / lii
            beta = (bt[i] - s) / lii
        w = points(i, cols, A, D, N, periodize)
        y, logd = condition(alpha, beta, w)
        Y[i] = y
        ell += logd
    return (ell, Y) if return_y else ell


def reduce_samples(ell: np.ndarray, N: int, S: int) -> dict:
    """Mean over samples in log space (Algorithm 2, final mean), per shift and
    over shifts, with the spread across shifts as the error estimate."""
    ell = np.asarray(ell, dtype=np.float64).reshape(S, N)
    logp_s = sp.logsumexp(ell, axis=1) - math.log(N)
    logp = sp.logsumexp(logp_s) - math.log(S)
    out = {"logP": float(logp), "P": float(math.exp(logp)) if logp > -745 else 0.0,
           "logP_s": logp_s}
    if S > 1 and np.isfinite(logp):
        m = np.max(logp_s)
        r = np.exp(logp_s - m)
        rel = math.sqrt(np.var(r, ddof=1) / S) / np.mean(r)
        out["rel_stderr"] = float(rel)
        out["stderr"] = float(rel * out["P"])
    else:
        out["rel_stderr"] = float("nan")
        out["stderr"] = float("nan")
    return out


def mvn_prob(sigma: np.ndarray, a, b, mu=None, N: int = 1000, S: int = 10,
             seed: int = 1, periodize: bool = False, L: np.ndarray | None = None) -> dict:
    """Full estimator: factor, centre, sweep all N*S samples, reduce."""
    from .cholesky import cholesky
    if L is None:
        L = cholesky(sigma)
    at, bt = centre(a, b, mu)
    ell = sweep(L, at, bt, N, S, seed, periodize=periodize)
    out = reduce_samples(ell, N, S)
    out["ell"] = ell
    return out
