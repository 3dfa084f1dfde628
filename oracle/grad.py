"""Derivatives of log P-hat at fixed QMC points.

The paper does not differentiate the estimator; this is the plain chain rule
applied to the recurrence of Eq. (sov1) (see ``oracle.sov``):

  d(log d_i) = [phi(b'_i) db'_i - phi(a'_i) da'_i] / d_i
  dy_i       = [(1 - w_i) phi(a'_i) da'_i + w_i phi(b'_i) db'_i] / phi(y_i)
  da'_i      = (da~_i - ds_i) / L_ii ,  db'_i = (db~_i - ds_i) / L_ii
  ds_i       = sum_{k<i} L_ik dy_k

evaluated with ratios of densities formed in log scale so deep tails do not
overflow.  log P-hat = logsumexp(l) - log(N S) over all samples, so its
directional derivative is the softmax(l)-weighted mean of dl.  Since
a~ = a - mu and b~ = b - mu, d/dmu = -(d/da + d/db) exactly.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.special as sp

from .qmc import lattice, shifts, points
from .sov import condition, reduce_samples, sweep

_HALF_LOG_2PI = 0.5 * math.log(2.0 * math.pi)


def _log_phi(x):
    with np.errstate(all="ignore"):
        return np.where(np.isfinite(x), -0.5 * x * x - _HALF_LOG_2PI, -np.inf)


def tangent_sweep(L, at, bt, dat, dbt, N, S, seed, cols=None, periodize=False):
    """Forward sweep of (l, dl) for the direction (da~, db~)."""
    n = L.shape[0]
    if cols is None:
        cols = np.arange(N * S, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    A = lattice(n)
    D = shifts(seed, n, S)
    Y = np.zeros((n, cols.size))
    dY = np.zeros((n, cols.size))
    ell = np.zeros(cols.size)
    dell = np.zeros(cols.size)
    for i in range(n):
        s = L[i, :i] @ Y[:i] if i else np.zeros(cols.size)
        ds = L[i, :i] @ dY[:i] if i else np.zeros(cols.size)
        lii = L[i, i]
        with np.errstate(all="ignore"):
            alpha = (at[i] - s) / lii
            beta = (bt[i] - s) / lii
        dalpha = (dat[i] - ds) / lii
        dbeta = (dbt[i] - ds) / lii
        w = points(i, cols, A, D, N, periodize)
        y, logd = condition(alpha, beta, w)
        lpa, lpb, lpy = _log_phi(alpha), _log_phi(beta), _log_phi(y)
        with np.errstate(all="ignore"):
            dlogd = np.exp(lpb - logd) * dbeta - np.exp(lpa - logd) * dalpha
            dy = (1.0 - w) * np.exp(lpa - lpy) * dalpha + w * np.exp(lpb - lpy) * dbeta
        dead = ~(logd > -np.inf)
        dlogd = np.where(dead, 0.0, dlogd)
        dy = np.where(dead, 0.0, dy)
        Y[i] = y
        dY[i] = dy
        ell += logd
        dell += dlogd
    return ell, dell


def logp_directional(L, at, bt, dat, dbt, N, S, seed, periodize=False):
    """(log P-hat, its derivative along (da~, db~))."""
    ell, dell = tangent_sweep(L, at, bt, dat, dbt, N, S, seed, periodize=periodize)
    wts = sp.softmax(ell)
    logp = reduce_samples(ell, N, S)["logP"]
    return logp, float(np.sum(wts * dell))


def logp_fd(L, at, bt, dat, dbt, N, S, seed, h=1e-5, periodize=False):
    """Central finite difference of log P-hat along (da~, db~) with step h."""
    def f(t):
        ell = sweep(L, at + t * dat, bt + t * dbt, N, S, seed, periodize=periodize)
        return reduce_samples(ell, N, S)["logP"]
    return (f(h) - f(-h)) / (2.0 * h)


def gradient_full(L, at, bt, N, S, seed, periodize=False):
    """Full gradient (d/da~, d/db~) by n tangent sweeps per limit vector;
    for small n only."""
    n = L.shape[0]
    ga = np.zeros(n)
    gb = np.zeros(n)
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        ga[k] = logp_directional(L, at, bt, e, np.zeros(n), N, S, seed, periodize)[1]
        gb[k] = logp_directional(L, at, bt, np.zeros(n), e, N, S, seed, periodize)[1]
    return ga, gb
