"""Posterior of a Gaussian field given noisy observations of some of its
sites (test infrastructure: see the package header).

Section V-B builds its synthetic confidence-region problems from a field
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


def posterior_at(locs: np.ndarray, kern: tuple, mu, obs, y, noise_var: float, sites) -> dict:
    """Posterior mean and variance at the given sites, and Sigma_post among
    them, for a Matern field on ``locs`` (kern = sigma2, beta, nu, nugget):
    the same two equations written in their kriging form,
      Sigma_post = Sigma - Sigma_.o K^-1 Sigma_o.,  K = Sigma_oo + noise_var I,
      mu_post = mu + Sigma_.o K^-1 (y - mu_o),
    which needs only the m observed sites' K (the form is pinned equal to
    the printed one).  For spot checks of large problems."""
    from .covariance import covariance, matern
    locs = np.asarray(locs, dtype=np.float64)
    obs = np.asarray(obs, dtype=np.int64)
    sites = np.asarray(sites, dtype=np.int64)
    n = locs.shape[0]
    mu = np.zeros(n) if mu is None else np.asarray(mu, dtype=np.float64)
    sigma2, beta, nu, nugget = kern
    K = covariance(locs[obs], sigma2, beta, nu, nugget)
    K[np.diag_indices_from(K)] += noise_var
    # repeated sites share the nugget (covariance() puts it on the diagonal only)
    same = obs[:, None] == obs[None, :]
    K[same & ~np.eye(obs.size, dtype=bool)] += nugget
    d = np.sqrt(np.sum((locs[sites][:, None, :] - locs[obs][None, :, :]) ** 2, axis=-1))
    C = matern(d, sigma2, beta, nu) + nugget * (sites[:, None] == obs[None, :])
    Kinv_C = np.linalg.solve(K, C.T)
    r = np.asarray(y, dtype=np.float64) - mu[obs]
    dss = np.sqrt(np.sum((locs[sites][:, None, :] - locs[sites][None, :, :]) ** 2, axis=-1))
    S_ss = matern(dss, sigma2, beta, nu) + nugget * (sites[:, None] == sites[None, :])
    S_post = S_ss - C @ Kinv_C
    return {"mu_post": mu[sites] + C @ np.linalg.solve(K, r), "var_post": np.diag(S_post).copy(),
            "sigma_post": S_post}
