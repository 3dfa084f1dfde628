"""Pins of the oracle's SOV estimator (Eq. (sov1)/(sov2), Algorithms 2-3)
against exact per-sample identities, closed-form orthant probabilities,
one-dimensional quadrature, brute-force Monte Carlo, SciPy's independent
MVN CDF, and 500-digit evaluation of the conditioning step."""
import math

import mpmath
import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as sp
import scipy.stats as st

import oracle
from oracle import sov


def _prob(sigma, a, b, N=4000, S=10, seed=11):
    return oracle.mvn_prob(sigma, a, b, N=N, S=S, seed=seed)


def _within(est, exact, k=5.0, floor=1e-14):
    assert abs(est["P"] - exact) <= k * est["stderr"] + floor, (est["P"], exact, est["stderr"])


# ------------------------------------------------ exact, per sample
def test_univariate_every_sample_exact():
    """n = 1: every sample equals Phi(b/sigma) - Phi(a/sigma)."""
    sig = np.array([[2.25]])
    for a, b in [(-np.inf, 0.3), (-1.0, 2.0), (0.5, np.inf), (1.2, 4.0), (-50.0, -48.0)]:
        out = _prob(sig, [a], [b], N=64, S=3)
        ref = math.log(sp.ndtr(b / 1.5) - sp.ndtr(a / 1.5)) if b / 1.5 > -30 else \
            float(mpmath.log(mpmath.ncdf(b / 1.5) - mpmath.ncdf(a / 1.5)))
        np.testing.assert_allclose(out["ell"], ref, rtol=1e-13, atol=1e-13)


def test_diagonal_sigma_product_of_univariates():
    """Diagonal Sigma: d_i does not depend on y, so l = sum log(Phi(b_i/s_i) - Phi(a_i/s_i))."""
    rng = np.random.default_rng(1)
    n = 40
    sd = rng.uniform(0.3, 2.0, n)
    a = rng.uniform(-3, 0, n)
    b = a + rng.uniform(0.2, 4, n)
    a[::3] = -np.inf
    b[::5] = np.inf
    out = _prob(np.diag(sd ** 2), a, b, N=50, S=2)
    ref = np.sum(np.log(sp.ndtr(b / sd) - sp.ndtr(a / sd)))
    np.testing.assert_allclose(out["ell"], ref, rtol=1e-13)


def test_unbounded_limits_give_zero_log():
    rng = np.random.default_rng(2)
    m = rng.standard_normal((12, 12))
    out = _prob(m @ m.T + np.eye(12), np.full(12, -np.inf), np.full(12, np.inf), N=30, S=2)
    assert np.all(out["ell"] == 0.0)
    assert out["logP"] == pytest.approx(0.0, abs=1e-15)


def test_zero_width_interval_gives_minus_infinity():
    sig = np.array([[1.0, 0.3], [0.3, 1.0]])
    out = _prob(sig, [0.2, -np.inf], [0.2, 1.0], N=16, S=2)
    assert np.all(out["ell"] == -np.inf) and out["logP"] == -np.inf


@pytest.mark.parametrize("alpha,beta", [
    (-np.inf, 0.7), (-2.0, 1.5), (0.4, 3.0), (2.5, np.inf), (-0.3, np.inf),
    (-40.0, -36.5), (-np.inf, -39.0), (36.0, 41.0), (7.0, 9.0), (-9.0, -7.5),
    (1e-3, 2e-3), (-1.0, -0.999),
])
def test_conditioning_step_against_high_precision_reference(alpha, beta):
    """The reflected / log-scale evaluation equals the unreflected formula
    y = Phi^-1(Phi(a') + w (Phi(b') - Phi(a'))) evaluated with 500 digits
    (enough to hold 1 - Phi(41) without cancellation); Phi^-1 is a root solve
    of log Phi(t) = log p in that precision."""
    mpmath.mp.dps = 500
    ws = np.array([2.0 ** -54, 1e-9, 0.013, 0.5, 0.77, 1 - 1e-9, 1 - 2.0 ** -53])
    y, logd = sov.condition(np.full(ws.size, alpha), np.full(ws.size, beta), ws)
    A = mpmath.ncdf(alpha) if np.isfinite(alpha) else mpmath.mpf(0)
    B = mpmath.ncdf(beta) if np.isfinite(beta) else mpmath.mpf(1)
    d = B - A
    assert logd[0] == pytest.approx(float(mpmath.log(d)), rel=1e-13, abs=1e-13)
    for k, w in enumerate(ws):
        p = A + mpmath.mpf(w) * d
        if p < 0.5:
            yref = mpmath.findroot(lambda t: mpmath.log(mpmath.ncdf(t)) - mpmath.log(p), float(y[k]))
        else:
            q = 1 - p
            yref = -mpmath.findroot(lambda t: mpmath.log(mpmath.ncdf(t)) - mpmath.log(q), -float(y[k]))
        assert y[k] == pytest.approx(float(yref), rel=2e-12, abs=2e-12), (w, y[k], yref)
    mpmath.mp.dps = 15


# ------------------------------------------------ statistical, vs truth
def test_bivariate_orthant_sheppard():
    for rho in (-0.6, 0.0, 0.45, 0.9):
        sig = np.array([[1.0, rho], [rho, 1.0]])
        exact = 0.25 + math.asin(rho) / (2 * math.pi)
        _within(_prob(sig, [-np.inf] * 2, [0.0, 0.0]), exact)


def test_trivariate_orthant_closed_form():
    r12, r13, r23 = 0.3, -0.2, 0.6
    sig = np.array([[1, r12, r13], [r12, 1, r23], [r13, r23, 1.0]])
    exact = 0.125 + (math.asin(r12) + math.asin(r13) + math.asin(r23)) / (4 * math.pi)
    _within(_prob(sig, [-np.inf] * 3, [0.0] * 3), exact)


@pytest.mark.parametrize("n", [5, 20, 60])
def test_equicorrelated_half_orthant_is_one_over_n_plus_one(n):
    sig = np.full((n, n), 0.5) + 0.5 * np.eye(n)
    _within(_prob(sig, [-np.inf] * n, [0.0] * n), 1.0 / (n + 1))


def test_equicorrelated_general_rho_by_quadrature():
    """P(X <= b 1) = int phi(z) Phi((b + sqrt(rho) z)/sqrt(1-rho))^n dz."""
    n, rho, bb = 80, 0.3, 1.2
    sig = np.full((n, n), rho) + (1 - rho) * np.eye(n)

    def integrand(z):
        return math.exp(sp.log_ndtr((bb + math.sqrt(rho) * z) / math.sqrt(1 - rho)) * n) * \
            math.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)
    exact = si.quad(integrand, -12, 12, epsabs=1e-14, limit=200)[0]
    _within(_prob(sig, [-np.inf] * n, [bb] * n, N=2000), exact)


def test_brute_force_monte_carlo_finite_limits():
    """Finite lower and upper limits at n <= 6 against 4e6 direct draws.
    (Dropping the Phi(a') term of Eq. (sov1) fails this test.)"""
    rng = np.random.default_rng(7)
    n = 5
    m = rng.standard_normal((n, n))
    sig = m @ m.T / n + 0.5 * np.eye(n)
    sd = np.sqrt(np.diag(sig))
    a = -0.4 * sd
    b = 1.1 * sd
    x = rng.multivariate_normal(np.zeros(n), sig, size=4_000_000)
    inside = np.all((x >= a) & (x <= b), axis=1)
    mc = inside.mean()
    mc_se = math.sqrt(mc * (1 - mc) / x.shape[0])
    est = _prob(sig, a, b)
    assert abs(est["P"] - mc) <= 5 * math.hypot(est["stderr"], mc_se)


def test_scipy_mvn_cdf_with_mean_and_lower_limits():
    """SciPy's Genz-Bretz CDF (independent code path) at n = 10 with a mean."""
    rng = np.random.default_rng(8)
    n = 10
    locs = rng.uniform(size=(n, 2))
    sig = oracle.covariance(locs, 1.0, 0.3, 1.5, nugget=1e-6)
    mu = rng.normal(size=n) * 0.3
    a = mu - 1.5
    b = mu + rng.uniform(0.5, 2.0, n)
    ref = st.multivariate_normal.cdf(b, mean=mu, cov=sig, lower_limit=a, abseps=1e-7,
                                     releps=1e-7, maxpts=2_000_000)
    est = oracle.mvn_prob(sig, a, b, mu=mu, N=4000, S=10, seed=3)
    assert abs(est["P"] - ref) <= 5 * est["stderr"] + 2e-6


def test_reflection_symmetry_of_limits():
    """P(a <= X <= b) = P(-b <= X <= -a) for a centred field (different samples)."""
    rng = np.random.default_rng(9)
    n = 15
    sig = oracle.covariance(rng.uniform(size=(n, 2)), 1.0, 0.2, 0.5, 1e-8)
    a = rng.uniform(-2.0, -0.2, n)
    b = a + rng.uniform(0.5, 3.0, n)
    p1 = _prob(sig, a, b)
    p2 = _prob(sig, -b, -a)
    assert abs(p1["P"] - p2["P"]) <= 5 * math.hypot(p1["stderr"], p2["stderr"])


def test_planted_typo_is_detected():
    """Replacing Eq. (sov1)'s y by the listing's Phi^-1[w d] (Phi(a') dropped)
    changes the estimate far beyond its error bar when a is finite."""
    sig = np.array([[1.0, 0.7], [0.7, 1.0]])
    a, b = [0.3, -np.inf], [2.0, 0.5]
    good = _prob(sig, a, b)
    orig = sov.condition

    def typo(alpha, beta, w):
        y, logd = orig(alpha, beta, w)
        d = sp.ndtr(beta) - sp.ndtr(alpha)
        return sp.ndtri(w * d), logd
    sov.condition = typo
    try:
        bad = _prob(sig, a, b)
    finally:
        sov.condition = orig
    exact = st.multivariate_normal(cov=sig).cdf(np.array([2.0, 0.5]), lower_limit=np.array([0.3, -np.inf]))
    _within(good, exact, floor=1e-6)
    assert abs(bad["P"] - exact) > 20 * good["stderr"] + 1e-3


def test_reduction_log_sum_exp_matches_linear_mean():
    rng = np.random.default_rng(4)
    ell = rng.normal(-3, 1, size=(4, 50))
    out = oracle.reduce_samples(ell.ravel(), 50, 4)
    p_s = np.exp(ell).mean(axis=1)
    assert out["P"] == pytest.approx(p_s.mean(), rel=1e-14)
    np.testing.assert_allclose(np.exp(out["logP_s"]), p_s, rtol=1e-14)
    assert out["stderr"] == pytest.approx(p_s.std(ddof=1) / 2.0, rel=1e-12)
