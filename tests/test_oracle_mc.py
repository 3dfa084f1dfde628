"""Pins of the oracle's Monte Carlo check of nested sets (Section V-C: the
fraction of fields X = mu + L Z inside the limits on every site of a set):
the counter layout of the draws against published SplitMix64 outputs, the
distribution of the normals, independent sites, the two- and three-site
orthant closed forms, the first-failure rule on hand-made fields, and
agreement with the QMC nested-set estimates of a correlated field.

The statistical pins use fixed seeds (deterministic) and bounds of five
binomial standard errors."""
import math
import os

import numpy as np
import scipy.special as sp
import scipy.stats as st

import oracle
from oracle import mc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _published(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                out[int(k)] = int(v, 0)
    return out


def _five_sigma(p, M):
    return 5.0 * math.sqrt(max(p * (1.0 - p), 1.0 / M) / M)


def test_counter_layout_matches_published_splitmix_outputs():
    """Draw (site i, sample j) of an n-site field is output j n + i: with
    three sites, sample 0 takes outputs 0, 1, 2; with one site, samples
    0, 1, 2 take them."""
    v = _published("splitmix64_seed0.txt")
    want = np.array([((v[k] >> 11) + 0.5) * 2.0 ** -53 for k in range(3)])
    np.testing.assert_array_equal(mc.uniforms(0, 3, [0])[:, 0], want)
    np.testing.assert_array_equal(mc.uniforms(0, 1, [0, 1, 2])[0], want)
    assert np.all((want > 0) & (want < 1))


def test_normals_are_standard_normal():
    z = mc.normals(11, 50, np.arange(400)).ravel()
    assert abs(z.mean()) < 5.0 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5.0 * math.sqrt(2.0 / z.size)
    assert st.kstest(z, "norm").pvalue > 1e-3
    # sites and samples are not tied: correlation of neighbouring sites
    zz = mc.normals(12, 2, np.arange(5000))
    assert abs(np.corrcoef(zz)[0, 1]) < 5.0 / math.sqrt(5000)


def test_first_failure_rule():
    X = np.array([[0.5, 0.5, 2.0, 0.5, 0.5, 0.0],
                  [0.1, -1.0, 0.0, 0.2, 0.2, 0.0],
                  [0.3, 0.3, 0.3, 5.0, 0.3, 1.0]])
    a = np.array([0.0, 0.0, -np.inf])
    b = np.array([1.0, np.inf, 1.0])
    # the interval is closed: the last field sits on a_1, a_2 and b_3
    np.testing.assert_array_equal(mc.first_failure(X, a, b), [3, 1, 0, 2, 3, 3])
    # a NaN limit never holds; a > b admits nothing
    np.testing.assert_array_equal(mc.first_failure(X, [0.0, np.nan, 0.0], [1.0, 1.0, 1.0]), [1, 1, 0, 1, 1, 1])
    np.testing.assert_array_equal(mc.first_failure(X, [2.0, 0, 0], [1.0, 9, 9]), [0, 0, 0, 0, 0, 0])
    np.testing.assert_array_equal(mc.prefix_counts(np.array([3, 1, 0, 2, 3]), 3), [4, 3, 2])


def test_independent_sites_give_products():
    rng = np.random.default_rng(4)
    n, M = 8, 4000
    sd = rng.uniform(0.5, 2.0, n)
    a = rng.uniform(-2.5, -0.5, n)
    b = a + rng.uniform(1.0, 4.0, n)
    mu = rng.uniform(-0.3, 0.3, n)
    out = mc.mc_prefix(np.diag(sd), a, b, mu, M, seed=21)
    p = np.cumprod(sp.ndtr((b - mu) / sd) - sp.ndtr((a - mu) / sd))
    for k in range(n):
        assert abs(out["count"][k] / M - p[k]) < _five_sigma(p[k], M), k


def test_two_and_three_site_orthants():
    """P(X_1 > 0, X_2 > 0) = 1/4 + asin(rho)/(2 pi) and the three-site
    orthant 1/8 + (asin r12 + asin r13 + asin r23)/(4 pi)."""
    r12, r13, r23 = 0.6, -0.3, 0.45
    C = np.array([[1.0, r12, r13], [r12, 1.0, r23], [r13, r23, 1.0]])
    sd = np.array([1.5, 0.7, 2.0])
    L = np.linalg.cholesky(C * np.outer(sd, sd))
    M = 20000
    out = mc.mc_prefix(L, np.zeros(3), np.full(3, np.inf), None, M, seed=99)
    p2 = 0.25 + math.asin(r12) / (2 * math.pi)
    p3 = 0.125 + (math.asin(r12) + math.asin(r13) + math.asin(r23)) / (4 * math.pi)
    assert abs(out["count"][0] / M - 0.5) < _five_sigma(0.5, M)
    assert abs(out["count"][1] / M - p2) < _five_sigma(p2, M)
    assert abs(out["count"][2] / M - p3) < _five_sigma(p3, M)


def test_agrees_with_qmc_nested_sets():
    """A 30-site exponential-covariance field with an uneven mean: every
    nested-set fraction against the oracle's QMC running-product estimate
    (different draws, different estimator, the same probabilities)."""
    rng = np.random.default_rng(8)
    n, M = 30, 20000
    locs = rng.uniform(0, 1, (n, 2))
    Sigma = oracle.covariance(locs, 1.0, 0.3, 0.5, 1e-8)
    mu = rng.normal(1.0, 0.8, n)
    order = np.argsort(-sp.ndtr(mu))
    L = oracle.cholesky(Sigma[np.ix_(order, order)])
    a, b = np.zeros(n), np.full(n, np.inf)
    out = mc.mc_prefix(L, a, b, mu[order], M, seed=5)
    at, bt = oracle.centre(a, b, mu[order])
    q = oracle.prefix_probs(L, at, bt, N=4000, S=8, seed=6)
    pq = np.exp(q["logP"])
    for k in range(n):
        tol = _five_sigma(pq[k], M) + 5.0 * pq[k] * q["rel_stderr"][k]
        assert abs(out["count"][k] / M - pq[k]) < tol, (k, out["count"][k] / M, pq[k])
    assert np.all(np.diff(out["count"]) <= 0)
