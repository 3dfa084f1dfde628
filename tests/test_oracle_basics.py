"""Pins of the oracle's covariance, Cholesky and QMC points against closed
forms, library routines of different lineage and published values."""
import math
import os

import mpmath
import numpy as np
import pytest
import scipy.special as sp

import oracle
from oracle import qmc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_pairs(name):
    out = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                out.append((int(k), int(v, 0)))
    return out


# ---------------------------------------------------------------- covariance
@pytest.mark.parametrize("nu", [0.5, 1.5])
def test_matern_closed_forms_match_bessel_formula(nu):
    """nu=1/2, 3/2 closed forms equal the printed K_nu formula (Section IV-A)."""
    h = np.linspace(1e-4, 3.0, 500)
    sigma2, beta = 1.7, 0.13
    z = h / beta
    bessel = sigma2 / (2 ** (nu - 1) * sp.gamma(nu)) * z ** nu * sp.kv(nu, z)
    got = oracle.matern(h, sigma2, beta, nu)
    np.testing.assert_allclose(got, bessel, rtol=2e-14, atol=0)
    assert oracle.matern(np.array([0.0]), sigma2, beta, nu)[0] == sigma2


def test_matern_bessel_branch_at_nu_5_2_is_the_closed_form():
    """nu = 5/2 is not special-cased in the oracle, so it takes the K_nu
    branch; the printed formula reduces to sigma^2 (1 + z + z^2/3) e^{-z}
    there (K_{5/2}(z) = sqrt(pi/(2z)) e^{-z} (1 + 3/z + 3/z^2))."""
    h = np.linspace(1e-3, 2.0, 300)
    sigma2, beta = 0.8, 0.21
    z = h / beta
    np.testing.assert_allclose(oracle.matern(h, sigma2, beta, 2.5), sigma2 * (1 + z + z * z / 3) * np.exp(-z),
                               rtol=1e-13, atol=0)


def test_matern_general_nu_against_high_precision():
    """The K_nu branch against 40-digit values (mpmath, independent of
    scipy's Bessel routines) at the smoothness fitted to the paper's wind
    data (1.43391) and at 0.7."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    for nu, beta in ((1.43391, 0.005069), (0.7, 0.1)):
        h = np.array([1e-5, 1e-3, 0.004, 0.02, 0.1, 0.7])
        got = oracle.matern(h, 1.0, beta, nu)
        for hv, g in zip(h, got):
            z = mp.mpf(hv) / mp.mpf(beta)
            ref = z ** nu * mp.besselk(nu, z) / (mp.mpf(2) ** (nu - 1) * mp.gamma(nu))
            assert abs(g / float(ref) - 1) < 1e-12, (nu, hv)


def test_matern_general_nu_limit():
    """General-nu branch: C(0) = sigma^2 and continuity at h -> 0."""
    c = oracle.matern(np.array([0.0, 1e-9]), 2.0, 0.1, 1.2)
    assert c[0] == 2.0 and abs(c[1] - 2.0) < 1e-6


def test_covariance_symmetric_with_nugget():
    rng = np.random.default_rng(0)
    locs = rng.uniform(size=(50, 2))
    s = oracle.covariance(locs, 1.0, 0.1, 1.5, nugget=1e-3)
    assert np.array_equal(s, s.T)
    np.testing.assert_allclose(np.diag(s), 1.0 + 1e-3, rtol=0, atol=0)
    d = math.dist(locs[3], locs[7])
    assert abs(s[3, 7] - (1 + d / 0.1) * math.exp(-d / 0.1)) < 1e-15


# ---------------------------------------------------------------- Cholesky
@pytest.mark.parametrize("n,block", [(1, 4), (37, 8), (300, 64), (257, 128)])
def test_cholesky_matches_lapack(n, block):
    """Blocked factor equals LAPACK dpotrf (numpy.linalg.cholesky)."""
    rng = np.random.default_rng(n)
    locs = rng.uniform(size=(n, 2))
    s = oracle.covariance(locs, 1.0, 0.2, 0.5, nugget=1e-6)
    L = oracle.cholesky(s, block=block)
    ref = np.linalg.cholesky(s)
    np.testing.assert_allclose(L, ref, rtol=0, atol=1e-12)
    assert np.all(np.triu(L, 1) == 0)


def test_cholesky_ar1_closed_form():
    """Exponential kernel on equispaced 1-D points is AR(1):
    L_i0 = rho^i, L_ij = rho^(i-j) sqrt(1 - rho^2) for j >= 1."""
    n, delta, beta = 120, 0.01, 0.05
    x = np.arange(n) * delta
    locs = np.stack([x, np.zeros(n)], axis=1)
    s = oracle.covariance(locs, 1.0, beta, 0.5)
    L = oracle.cholesky(s, block=32)
    rho = math.exp(-delta / beta)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ref = np.where(j == 0, rho ** i, rho ** (i - j) * math.sqrt(1 - rho * rho))
    ref = np.where(j <= i, ref, 0.0)
    np.testing.assert_allclose(L, ref, rtol=0, atol=5e-13)


def test_cholesky_residual_and_not_spd():
    rng = np.random.default_rng(3)
    m = rng.standard_normal((80, 80))
    s = m @ m.T + 80 * np.eye(80)
    L = oracle.cholesky(s, block=16)
    assert np.linalg.norm(L @ L.T - s) / np.linalg.norm(s) < 80 * 2.0 ** -52
    bad = s.copy()
    bad[41, 41] = -1.0
    with pytest.raises(oracle.NotPositiveDefinite) as e:
        oracle.cholesky(bad, block=16)
    assert e.value.index == 42
    # two identical locations without a nugget: singular at the second copy
    locs = rng.uniform(size=(10, 2))
    locs[6] = locs[2]
    with pytest.raises(oracle.NotPositiveDefinite) as e:
        oracle.cholesky(oracle.covariance(locs, 1.0, 0.3, 0.5), block=4)
    assert e.value.index == 7


# ---------------------------------------------------------------- QMC points
def test_splitmix64_published_outputs():
    for k, v in _read_pairs("splitmix64_seed0.txt"):
        assert qmc.splitmix64(0, k) == v


def test_primes_table():
    pairs = _read_pairs("primes.txt")
    ps = qmc.first_primes(max(k for k, _ in pairs))
    for k, v in pairs:
        assert ps[k - 1] == v


def test_lattice_is_fractional_sqrt_of_primes():
    """A_i = floor(frac(sqrt(p_{i+1})) 2^64), checked with 60-digit mpmath."""
    A = qmc.lattice(300)
    ps = qmc.first_primes(300)
    mpmath.mp.dps = 60
    for i in list(range(20)) + [150, 299]:
        r = mpmath.sqrt(ps[i])
        frac = r - mpmath.floor(r)
        assert int(A[i]) == int(mpmath.floor(frac * mpmath.mpf(2) ** 64))


def test_points_dimension0_is_shifted_richtmyer():
    """w_{s,j,0} = frac(j sqrt(2) + Delta) to within the 53-bit truncation."""
    N, S, n, seed = 50, 3, 4, 99
    A = qmc.lattice(n)
    D = qmc.shifts(seed, n, S)
    cols = np.arange(N * S)
    w = qmc.points(0, cols, A, D, N)
    mpmath.mp.dps = 50
    for c in [0, 1, 17, 49, 50, 149]:
        s, j = divmod(c, N)
        j += 1
        ref = j * mpmath.sqrt(2) + mpmath.mpf(int(D[s, 0])) / 2 ** 64
        ref = ref - mpmath.floor(ref)
        assert abs(float(ref) - w[c]) < 2.0 ** -52
    assert np.all((w > 0) & (w < 1))
