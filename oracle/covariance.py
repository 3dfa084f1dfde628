"""Matern covariance (paper Section IV-A, Eq. for C(||h||; theta)).

C(h) = sigma^2 / (2^(nu-1) Gamma(nu)) (h/beta)^nu K_nu(h/beta),  C(0) = sigma^2.

The paper names the range parameter "a"; it is called ``beta`` here because
"a" is the lower integration limit.  The formula is taken exactly as printed
(h/beta, no sqrt(2 nu) rescaling).  For nu = 1/2 and nu = 3/2 the Bessel
form reduces to the closed forms below, which are what the oracle evaluates;
other nu use scipy's K_nu.
"""
from __future__ import annotations

import numpy as np
import scipy.special as sp


def matern(h, sigma2: float, beta: float, nu: float) -> np.ndarray:
    """Matern C(h) for distances ``h`` (any shape)."""
    h = np.asarray(h, dtype=np.float64)
    z = h / beta
    if nu == 0.5:
        # K_{1/2}(z) = sqrt(pi/(2z)) e^{-z}, Gamma(1/2) = sqrt(pi)
        return sigma2 * np.exp(-z)
    if nu == 1.5:
        # K_{3/2}(z) = sqrt(pi/(2z)) e^{-z} (1 + 1/z), Gamma(3/2) = sqrt(pi)/2
        return sigma2 * (1.0 + z) * np.exp(-z)
    out = np.full(z.shape, float(sigma2))
    pos = z > 0
    zp = z[pos]
    out[pos] = sigma2 / (2.0 ** (nu - 1.0) * sp.gamma(nu)) * zp ** nu * sp.kv(nu, zp)
    return out


def covariance(locs: np.ndarray, sigma2: float, beta: float, nu: float,
               nugget: float = 0.0) -> np.ndarray:
    """Sigma_ij = C(||s_i - s_j||) + nugget * delta_ij  (Algorithm 1, first step)."""
    locs = np.asarray(locs, dtype=np.float64)
    diff = locs[:, None, :] - locs[None, :, :]
    h = np.sqrt(np.sum(diff * diff, axis=-1))
    sig = matern(h, sigma2, beta, nu)
    sig[np.diag_indices_from(sig)] += nugget
    return sig
