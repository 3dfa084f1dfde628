"""Pins of the oracle's posterior (Section V-B: Sigma_post and mu_post of a
field observed with noise at some sites): the scalar conjugate normal case,
the kriging (Woodbury) form, the noiseless limit (the conditional Gaussian
of the unobserved sites, variance zero at the observed ones), repeated
observations of one site, and the posterior moments of many joint draws."""
import numpy as np

import oracle
from oracle import posterior as op


def _sigma(n, seed, beta=0.2):
    rng = np.random.default_rng(seed)
    locs = rng.uniform(0, 1, (n, 2))
    return oracle.covariance(locs, 1.3, beta, 0.5, 1e-6)


def test_one_site_is_the_conjugate_normal():
    s2, t2, mu, y = 1.7, 0.25, 0.4, 1.9
    S, m = op.posterior(np.array([[s2]]), [mu], [0], [y], t2)
    assert abs(S[0, 0] - s2 * t2 / (s2 + t2)) < 1e-15
    assert abs(m[0] - (mu + s2 / (s2 + t2) * (y - mu))) < 1e-15


def test_equals_the_kriging_form():
    """Sigma - Sigma A^T (A Sigma A^T + t^2 I)^-1 A Sigma and the matching
    mean: the Woodbury identity, computed without inverting Sigma."""
    n, t2 = 60, 0.25
    Sig = _sigma(n, 1)
    rng = np.random.default_rng(2)
    obs = np.sort(rng.choice(n, 17, replace=False))
    mu = rng.normal(0, 1, n)
    y = rng.normal(0, 1, obs.size)
    S, m = op.posterior(Sig, mu, obs, y, t2)
    C = Sig[:, obs]
    K = Sig[np.ix_(obs, obs)] + t2 * np.eye(obs.size)
    S2 = Sig - C @ np.linalg.solve(K, C.T)
    m2 = mu + C @ np.linalg.solve(K, y - mu[obs])
    np.testing.assert_allclose(S, S2, rtol=0, atol=1e-9)
    np.testing.assert_allclose(m, m2, rtol=0, atol=1e-9)


def test_noiseless_limit_is_the_conditional_gaussian():
    n = 40
    Sig = _sigma(n, 3)
    obs = np.arange(0, n, 4)
    rest = np.setdiff1d(np.arange(n), obs)
    rng = np.random.default_rng(4)
    y = rng.normal(0, 1, obs.size)
    S, m = op.posterior(Sig, None, obs, y, 1e-10)
    Soo = Sig[np.ix_(obs, obs)]
    Sro = Sig[np.ix_(rest, obs)]
    cond = Sig[np.ix_(rest, rest)] - Sro @ np.linalg.solve(Soo, Sro.T)
    np.testing.assert_allclose(S[np.ix_(rest, rest)], cond, rtol=0, atol=1e-6)
    np.testing.assert_allclose(m[rest], Sro @ np.linalg.solve(Soo, y), rtol=0, atol=1e-5)
    assert np.max(np.abs(np.diag(S)[obs])) < 1e-6
    np.testing.assert_allclose(m[obs], y, atol=1e-6)


def test_repeated_observations_average():
    """Observing one site twice with noise t^2 equals observing it once
    with noise t^2 / 2 at the mean of the two values."""
    Sig = _sigma(10, 5)
    S1, m1 = op.posterior(Sig, None, [3, 3], [0.2, 1.0], 0.5)
    S2, m2 = op.posterior(Sig, None, [3], [0.6], 0.25)
    np.testing.assert_allclose(S1, S2, atol=1e-12)
    np.testing.assert_allclose(m1, m2, atol=1e-12)


def test_moments_of_joint_draws():
    """Draw (x, y) from the joint model many times; within bins of nearby y
    the spread is not usable, so use the regression form instead: the
    residual x - mu_post(y) is uncorrelated with y and has covariance
    Sigma_post (moments of 200 000 draws, 5 standard errors)."""
    n, t2, R = 6, 0.3, 200_000
    Sig = _sigma(n, 6, beta=0.5)
    obs = np.array([1, 4])
    rng = np.random.default_rng(7)
    X = rng.multivariate_normal(np.zeros(n), Sig, size=R)
    Y = X[:, obs] + rng.normal(0, np.sqrt(t2), (R, obs.size))
    S, _ = op.posterior(Sig, None, obs, np.zeros(obs.size), t2)
    # mu_post is linear in y: mu_post(y) = G y with G from unit observations
    G = np.column_stack([op.posterior(Sig, None, obs, e, t2)[1] for e in np.eye(obs.size)])
    res = X - Y @ G.T
    cov = res.T @ res / R
    se = np.sqrt((np.outer(np.diag(S), np.diag(S)) + S * S) / R)
    assert np.all(np.abs(cov - S) < 5 * se + 1e-12)
    cross = res.T @ Y / R
    assert np.all(np.abs(cross) < 5 * np.sqrt(np.outer(np.diag(S), np.diag(Sig)[obs] + t2) / R))


def test_spot_form_equals_the_full_equations():
    """The spot-check routine (kriging form on the observed sites only)
    against the full equations at every site, with a repeated observation."""
    rng = np.random.default_rng(12)
    n, t2 = 45, 0.3
    locs = rng.uniform(0, 1, (n, 2))
    kern = (1.1, 0.25, 1.5, 1e-4)
    Sig = oracle.covariance(locs, *kern)
    obs = np.array([3, 7, 7, 20, 44, 0])
    y = rng.normal(0, 1, obs.size)
    mu = rng.normal(0, 0.5, n)
    S, m = op.posterior(Sig, mu, obs, y, t2)
    sites = np.array([0, 5, 7, 30, 44])
    spot = op.posterior_at(locs, kern, mu, obs, y, t2, sites)
    np.testing.assert_allclose(spot["mu_post"], m[sites], atol=1e-10)
    np.testing.assert_allclose(spot["var_post"], np.diag(S)[sites], atol=1e-10)
    np.testing.assert_allclose(spot["sigma_post"], S[np.ix_(sites, sites)], atol=1e-10)
