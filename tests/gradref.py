"""Closed forms for pins of d P / d b_i (test helper; no estimator code).

For X ~ N(mu, Sigma) and the box a <= X <= b,

  d P / d b_i = phi((b_i - mu_i) / sigma_i) / sigma_i
                * P(a_{-i} <= X_{-i} <= b_{-i} | X_i = b_i),

where the conditional law of X_{-i} given X_i = b_i is normal with mean
mu_{-i} + Sigma_{-i,i} (b_i - mu_i) / Sigma_ii and covariance
Sigma_{-i,-i} - Sigma_{-i,i} Sigma_{i,-i} / Sigma_ii (differentiate the
integral over x_i's upper limit; the remaining integral is the conditional
probability times the marginal density).  The conditional probability is
evaluated exactly by one-dimensional adaptive quadrature when it is
bivariate (n = 3), and by SciPy's Genz-Bretz integration otherwise.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.integrate as si
import scipy.special as sp
import scipy.stats as st


def conditional(Sigma, mu, i, x):
    """Mean and covariance of X_{-i} given X_i = x."""
    n = Sigma.shape[0]
    keep = np.array([k for k in range(n) if k != i])
    c = Sigma[keep, i]
    m = mu[keep] + c * (x - mu[i]) / Sigma[i, i]
    C = Sigma[np.ix_(keep, keep)] - np.outer(c, c) / Sigma[i, i]
    return keep, m, C


def box2_quad(m, C, a, b):
    """P(a <= Z <= b) for a bivariate normal Z ~ N(m, C), by quadrature over
    z_0 of its density times the conditional probability of z_1."""
    s0 = math.sqrt(C[0, 0])
    s1 = math.sqrt(C[1, 1] - C[0, 1] ** 2 / C[0, 0])

    def f(z0):
        m1 = m[1] + C[0, 1] / C[0, 0] * (z0 - m[0])
        return (math.exp(-0.5 * ((z0 - m[0]) / s0) ** 2) / (s0 * math.sqrt(2 * math.pi))
                * (sp.ndtr((b[1] - m1) / s1) - sp.ndtr((a[1] - m1) / s1)))

    lo = max(a[0], m[0] - 40 * s0)
    hi = min(b[0], m[0] + 40 * s0)
    if not lo < hi:
        return 0.0
    v, _ = si.quad(f, lo, hi, epsabs=1e-14, epsrel=1e-12, limit=200)
    return v


def box_genz(m, C, a, b):
    """P(a <= Z <= b), Z ~ N(m, C), by SciPy's Genz-Bretz integration."""
    if len(m) == 1:
        s = math.sqrt(C[0, 0])
        return float(sp.ndtr((b[0] - m[0]) / s) - sp.ndtr((a[0] - m[0]) / s))
    return float(st.multivariate_normal.cdf(b, mean=m, cov=C, lower_limit=a, abseps=1e-9, releps=1e-8,
                                            maxpts=2_000_000 * len(m)))


def dP_db(Sigma, mu, a, b, i):
    """d P / d b_i in closed form (exact quadrature for n = 3)."""
    n = Sigma.shape[0]
    s = math.sqrt(Sigma[i, i])
    dens = math.exp(-0.5 * ((b[i] - mu[i]) / s) ** 2) / (s * math.sqrt(2 * math.pi))
    keep, m, C = conditional(Sigma, mu, i, b[i])
    if n == 3:
        return dens * box2_quad(m, C, a[keep], b[keep])
    return dens * box_genz(m, C, a[keep], b[keep])
