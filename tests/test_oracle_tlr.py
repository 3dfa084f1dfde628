"""Pins of the oracle's tile low-rank compression and TLR Cholesky:
Eckart-Young bounds, exact recovery of known ranks, eps -> 0 reproducing the
dense factor, and the residual of the TLR factor scaling with eps."""
import numpy as np
import pytest

import oracle
import workloads


def _morton_cov(k, beta=0.1, nugget=1e-8):
    locs = workloads.grid_locations(k)[workloads.morton_permutation(k)]
    return oracle.covariance(locs, 1.0, beta, 0.5, nugget)


def test_compression_meets_eckart_young_bound():
    sig = _morton_cov(16)  # n = 256, tiles of 64
    a = sig[128:192, 0:64]
    s_all = np.linalg.svd(a, compute_uv=False)
    for eps in (1e-2, 1e-4, 1e-7):
        u, v, s = oracle.compress_tile(a, eps, 64)
        k = u.shape[1]
        assert k == int(np.sum(s_all > eps))
        err2 = np.linalg.norm(a - u @ v.T, 2)
        assert err2 <= eps * (1 + 1e-8) + 1e-14
        # the next singular value is exactly the 2-norm error (Eckart-Young)
        if k < len(s_all):
            assert err2 == pytest.approx(s_all[k], rel=1e-6)


def test_compression_recovers_exact_rank():
    rng = np.random.default_rng(0)
    x, y = rng.standard_normal((50, 5)), rng.standard_normal((40, 5))
    u, v, _ = oracle.compress_tile(x @ y.T, 1e-10, 40)
    assert u.shape[1] == 5
    np.testing.assert_allclose(u @ v.T, x @ y.T, atol=1e-10)


def test_rank_cap_binds():
    sig = _morton_cov(16)
    u, v, _ = oracle.compress_tile(sig[64:128, 0:64], 1e-12, 3)
    assert u.shape[1] == 3


def test_tlr_cholesky_with_zero_eps_is_the_dense_factor():
    sig = _morton_cov(12)  # n = 144, ragged last tile with tile 64
    D, U, V, ranks = oracle.tlr_cholesky(sig, 64, 0.0, 64)
    L = oracle.tlr_dense(D, U, V, 144, 64)
    np.testing.assert_allclose(L, np.linalg.cholesky(sig), atol=1e-10)


def test_tlr_cholesky_residual_scales_with_eps():
    sig = _morton_cov(16)
    prev = None
    for eps in (1e-3, 1e-5, 1e-7):
        D, U, V, ranks = oracle.tlr_cholesky(sig, 64, eps, 64)
        L = oracle.tlr_dense(D, U, V, 256, 64)
        res = np.linalg.norm(L @ L.T - sig, 2)
        assert res < 50 * eps, (eps, res)
        if prev is not None:
            assert ranks.sum() >= prev
        prev = ranks.sum()
