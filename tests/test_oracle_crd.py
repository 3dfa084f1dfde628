"""Pins of the oracle's nested-set probabilities (Section III-C with Algorithm 1 of Section IV-A:
P(S_k) for the first k sites, from the running products of one sweep):
exact first prefix, exact products for independent sites, closed-form
orthant probabilities for the two- and three-site prefixes, monotonicity,
and the last prefix equal to the full estimate."""
import math

import numpy as np
import scipy.special as sp

import oracle


def _ar1(n, rho, s=1.0):
    i = np.arange(n)
    return s * s * rho ** np.abs(i[:, None] - i[None, :])


def test_first_prefix_is_exact():
    """d_1 = Phi(b_1/L_11) - Phi(a_1/L_11) for every sample."""
    sig = _ar1(6, 0.6, 1.3)
    a = np.array([-0.4, -np.inf, -1.0, -2.0, -np.inf, 0.0])
    b = np.array([1.1, 0.5, np.inf, 0.3, 1.0, 2.0])
    L = oracle.cholesky(sig)
    out = oracle.prefix_probs(L, a, b, N=97, S=3, seed=5)
    ref = math.log(sp.ndtr(1.1 / 1.3) - sp.ndtr(-0.4 / 1.3))
    assert abs(out["logP"][0] - ref) < 1e-14


def test_independent_sites_give_products():
    """Diagonal Sigma: every prefix is the product of the univariate terms."""
    rng = np.random.default_rng(3)
    n = 12
    sd = rng.uniform(0.5, 2.0, n)
    a = rng.uniform(-3.0, -0.5, n)
    b = a + rng.uniform(0.3, 4.0, n)
    L = np.diag(sd)
    out = oracle.prefix_probs(L, a, b, N=50, S=2, seed=9)
    ref = np.cumsum(np.log(sp.ndtr(b / sd) - sp.ndtr(a / sd)))
    np.testing.assert_allclose(out["logP"], ref, rtol=0, atol=1e-12)


def test_orthant_prefixes_match_closed_forms():
    """Prefixes 2 and 3 of an orthant problem: 1/4 + asin(r12)/(2 pi) and
    1/8 + (asin r12 + asin r13 + asin r23)/(4 pi), within five standard
    errors of the QMC estimate."""
    sig = np.array([[1.0, 0.5, 0.3, 0.2], [0.5, 1.0, -0.4, 0.1], [0.3, -0.4, 1.0, 0.25],
                    [0.2, 0.1, 0.25, 1.0]])
    L = oracle.cholesky(sig)
    a = np.full(4, -np.inf)
    b = np.zeros(4)
    out = oracle.prefix_probs(L, a, b, N=20000, S=10, seed=21)
    p2 = 0.25 + math.asin(0.5) / (2 * math.pi)
    p3 = 0.125 + (math.asin(0.5) + math.asin(0.3) + math.asin(-0.4)) / (4 * math.pi)
    for k, p in ((1, p2), (2, p3)):
        est = math.exp(out["logP"][k])
        assert abs(est - p) <= 5 * out["rel_stderr"][k] * est + 1e-12, (k, est, p)
    assert abs(out["logP"][0] - math.log(0.5)) < 1e-14


def test_prefixes_decrease_and_the_last_is_the_estimate():
    """Every d_i <= 1, so the running products (and their means) do not
    increase; the last prefix is the full estimate of the same sweep."""
    locs = np.stack(np.meshgrid(np.linspace(0, 1, 6), np.linspace(0, 1, 5)), -1).reshape(-1, 2)
    sig = oracle.covariance(locs, 1.0, 0.3, 0.5, 1e-8)
    rng = np.random.default_rng(7)
    mu = rng.normal(size=len(locs))
    a = np.full(len(locs), -np.inf)
    b = 0.4 - mu
    L = oracle.cholesky(sig)
    N, S, seed = 300, 4, 17
    out = oracle.prefix_probs(L, a, b, N=N, S=S, seed=seed)
    assert np.all(np.diff(out["logP"]) <= 1e-15)
    full = oracle.reduce_samples(oracle.sweep(L, a, b, N, S, seed), N, S)
    assert out["logP"][-1] == full["logP"]
    assert out["rel_stderr"][-1] == full["rel_stderr"]


def test_exceedance_order():
    mu = np.array([0.0, 1.0, -1.0, 1.0])
    sd = np.array([1.0, 2.0, 1.0, 1.0])
    # P(X > 0.5): 1 - Phi((0.5 - mu) / sd) = 0.309, 0.599, 0.067, 0.691
    assert oracle.exceedance_order(mu, sd, 0.5).tolist() == [3, 1, 0, 2]


def test_leading_rows_of_a_larger_problem():
    """The first k nested sets of an n-site problem from its leading k x k
    block alone, with dim = n numbering the shifts: equal, bit for bit, to
    the first k entries of the full n-site computation; without dim the
    shifts (and so the estimates) differ; dim below the row count is an
    error."""
    n, k, N, S, seed = 30, 11, 131, 3, 17
    rng = np.random.default_rng(4)
    sig = _ar1(n, 0.7)
    a = rng.uniform(-2.0, 0.0, n)
    b = rng.uniform(0.2, 2.0, n)
    L = oracle.cholesky(sig)
    full = oracle.prefix_probs(L, a, b, N=N, S=S, seed=seed)["logP"]
    lead = oracle.prefix_probs(L[:k, :k], a[:k], b[:k], N=N, S=S, seed=seed, dim=n)["logP"]
    assert np.array_equal(lead, full[:k])
    own = oracle.prefix_probs(L[:k, :k], a[:k], b[:k], N=N, S=S, seed=seed)["logP"]
    assert not np.array_equal(own, full[:k])
    try:
        oracle.prefix_probs(L[:k, :k], a[:k], b[:k], N=N, S=S, seed=seed, dim=k - 1)
    except ValueError:
        pass
    else:
        raise AssertionError("dim below the row count was accepted")
