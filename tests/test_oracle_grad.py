"""Pins of the oracle's derivatives of log P-hat at fixed QMC points:
central finite differences, exact per-sample derivatives for diagonal Sigma,
the mu-invariant, and the bivariate closed form of dP/db_i."""
import math

import numpy as np
import pytest
import scipy.special as sp
import scipy.stats as st

import oracle
from oracle import grad


def _setup(n=6, seed=0):
    rng = np.random.default_rng(seed)
    sig = oracle.covariance(rng.uniform(size=(n, 2)), 1.0, 0.25, 1.5, 1e-6)
    L = oracle.cholesky(sig)
    a = rng.uniform(-2.5, -0.5, n)
    b = rng.uniform(0.0, 2.0, n)
    return sig, L, a, b, rng


def test_tangent_matches_central_differences():
    _, L, a, b, rng = _setup(7)
    N, S, seed = 500, 2, 4
    for _ in range(4):
        da = rng.standard_normal(7)
        db = rng.standard_normal(7)
        _, dd = grad.logp_directional(L, a, b, da, db, N, S, seed)
        fd = grad.logp_fd(L, a, b, da, db, N, S, seed, h=1e-5)
        assert dd == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_tangent_with_infinite_lower_limits():
    _, L, a, b, rng = _setup(6, seed=1)
    a[:] = -np.inf
    db = rng.standard_normal(6)
    _, dd = grad.logp_directional(L, a, b, np.zeros(6), db, 300, 2, 9)
    fd = grad.logp_fd(L, a, b, np.zeros(6), db, 300, 2, 9)
    assert dd == pytest.approx(fd, rel=1e-6)


def test_diagonal_sigma_exact_derivative():
    """Diagonal Sigma: dl/db_i = phi(b_i/s_i) / (s_i d_i) for every sample."""
    sd = np.array([0.7, 1.3, 2.0, 0.4])
    a = np.array([-1.0, -np.inf, 0.2, -3.0])
    b = np.array([0.5, 1.0, 2.5, -0.1])
    L = np.diag(sd)
    for i in range(4):
        e = np.zeros(4)
        e[i] = 1.0
        _, dell = grad.tangent_sweep(L, a, b, np.zeros(4), e, 20, 1, 3)
        d = sp.ndtr(b[i] / sd[i]) - sp.ndtr(a[i] / sd[i])
        ref = math.exp(-0.5 * (b[i] / sd[i]) ** 2) / math.sqrt(2 * math.pi) / (sd[i] * d)
        np.testing.assert_allclose(dell, ref, rtol=1e-13)


def test_mu_derivative_is_minus_sum_of_limit_derivatives():
    """a~ = a - mu, b~ = b - mu: shifting mu by t equals shifting both limits by -t."""
    _, L, a, b, rng = _setup(5, seed=2)
    v = rng.standard_normal(5)
    N, S, seed = 400, 2, 6
    _, g_ab = grad.logp_directional(L, a, b, v, v, N, S, seed)

    def f(t):
        at, bt = oracle.centre(a, b, mu=t * v)
        return oracle.reduce_samples(oracle.sweep(L, at, bt, N, S, seed), N, S)["logP"]
    fd_mu = (f(1e-5) - f(-1e-5)) / 2e-5
    assert fd_mu == pytest.approx(-g_ab, rel=1e-6)


def test_bivariate_closed_form_dP_db():
    """dP/db_1 = phi(b_1/s_1)/s_1 * P(a_2 <= X_2 <= b_2 | X_1 = b_1), exact for n = 2."""
    rho, s1, s2 = 0.6, 1.2, 0.8
    sig = np.array([[s1 * s1, rho * s1 * s2], [rho * s1 * s2, s2 * s2]])
    L = oracle.cholesky(sig)
    a = np.array([-1.0, -0.7])
    b = np.array([0.8, 1.1])
    N, S = 20000, 10
    _, g = grad.logp_directional(L, a, b, np.zeros(2), np.array([1.0, 0.0]), N, S, 12)
    est = oracle.reduce_samples(oracle.sweep(L, a, b, N, S, 12), N, S)
    dP = g * est["P"]
    m = rho * s2 / s1 * b[0]
    sc = s2 * math.sqrt(1 - rho * rho)
    cond = sp.ndtr((b[1] - m) / sc) - sp.ndtr((a[1] - m) / sc)
    exact = st.norm.pdf(b[0] / s1) / s1 * cond
    assert dP == pytest.approx(exact, rel=5e-3)


def _box_problem(n, seed):
    rng = np.random.default_rng(seed)
    sig = oracle.covariance(rng.uniform(size=(n, 2)), 1.0, 0.3, 1.5, 1e-6)
    mu = rng.normal(0.0, 0.3, n)
    a = mu - rng.uniform(0.5, 2.5, n)
    b = mu + rng.uniform(0.2, 2.0, n)
    return sig, mu, a, b


def _dP_db_estimate(L, at, bt, i, N, S, seed):
    """dP/db_i from the oracle's tangent sweep, with its standard error over
    the S shifts."""
    n = L.shape[0]
    e = np.zeros(n)
    e[i] = 1.0
    ell, dell = grad.tangent_sweep(L, at, bt, np.zeros(n), e, N, S, seed)
    p = np.exp(ell).reshape(S, N)
    dp = (np.exp(ell) * dell).reshape(S, N).mean(axis=1)
    return dp.mean(), dp.std(ddof=1) / math.sqrt(S), p.mean()


def test_closed_form_box2_quadrature_matches_scipy():
    """The quadrature helper against SciPy's bivariate normal CDF."""
    from gradref import box2_quad
    m = np.array([0.3, -0.2])
    C = np.array([[1.1, 0.5], [0.5, 0.7]])
    a, b = np.array([-0.9, -1.3]), np.array([1.2, 0.4])
    ref = st.multivariate_normal.cdf(b, mean=m, cov=C, lower_limit=a, abseps=1e-12, releps=1e-12)
    assert box2_quad(m, C, a, b) == pytest.approx(ref, abs=1e-9)


def test_closed_form_dP_db_exact_at_n3():
    """n = 3: the oracle's derivative of the estimator (tangent sweep times
    P-hat) equals the closed form phi/sigma * P(bivariate conditional box),
    the latter by exact quadrature, for every coordinate, within the QMC
    error of N S = 200 000 samples."""
    from gradref import dP_db
    sig, mu, a, b = _box_problem(3, seed=11)
    L = oracle.cholesky(sig)
    at, bt = oracle.centre(a, b, mu)
    N, S, seed = 20000, 10, 5
    for i in range(3):
        est, se, _ = _dP_db_estimate(L, at, bt, i, N, S, seed)
        exact = dP_db(sig, mu, a, b, i)
        assert abs(est - exact) <= max(5 * se, 2e-4 * abs(exact)), (i, est, exact, se)
        assert est == pytest.approx(exact, rel=2e-3)


@pytest.mark.parametrize("n", [4, 5, 6, 7, 8])
def test_closed_form_dP_db_statistical_n4_to_8(n):
    """n = 4..8: the oracle's dP/db_i within five standard errors (over the
    shifts) of the closed form with the conditional probability from SciPy's
    Genz-Bretz integration (absolute error 1e-9 requested)."""
    from gradref import dP_db
    sig, mu, a, b = _box_problem(n, seed=20 + n)
    L = oracle.cholesky(sig)
    at, bt = oracle.centre(a, b, mu)
    N, S, seed = 4000, 10, 7 + n
    for i in (0, n // 2, n - 1):
        est, se, _ = _dP_db_estimate(L, at, bt, i, N, S, seed)
        exact = dP_db(sig, mu, a, b, i)
        assert abs(est - exact) <= 5 * se + 1e-6, (n, i, est, exact, se)

