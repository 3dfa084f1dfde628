"""Posterior of a Gaussian field given noisy observations of some of its
sites (test infrastructure: see the package header).

Section IV-A builds its synthetic confidence-region problems from a field
x ~ N(mu, Sigma) observed at m of its n sites with additive noise
N(0, sigma_eps^2): y = A x + eps, A the m x n indicator matrix of the
observed sites.  The posterior of x given y is Gaussian with (the two
displayed equations of that section)

  Sigma_post = (Sigma^-1 + A^T A / sigma_eps^2)^-1
  mu_post    = mu + Sigma_post A^T (y - A mu) / sigma_eps^2

evaluated here literally, with dense inverses.  Sigma_post and mu_post then
take the place of Sigma and mu in Algorithm 1.
"""
from __future__ import annotations

import numpy as np


def indicator(obs, n: int) -> np.ndarray:
    """A[k, obs[k]] = 1: the m x n matrix that picks the observed sites."""
    obs = np.asarray(obs, dtype=np.int64)
    A = np.zeros((obs.size, n))
    A[np.arange(obs.size), obs] = 1.0
    return A


def posterior(Sigma: np.ndarray, mu, obs, y, noise_var: float) -> tuple[np.ndarray, np.ndarray]:
    """(Sigma_post, mu_post) by the section's two equations."""
    n = Sigma.shape[0]
    mu = np.zeros(n) if mu is None else np.asarray(mu, dtype=np.float64)
    A = indicator(obs, n)
    Sigma_post = np.linalg.inv(np.linalg.inv(Sigma) + A.T @ A / noise_var)
    Sigma_post = 0.5 * (Sigma_post + Sigma_post.T)  # the inverse of a symmetric matrix, rounded
    mu_post = mu + Sigma_post @ A.T @ (np.asarray(y, dtype=np.float64) - A @ mu) / noise_var
    return Sigma_post, mu_post
