"""Posterior of a field observed with noise (Section V-B) through the C
ABI: Sigma_post, mu_post and the marginal variances from one partial
factorisation of the bordered matrix against the oracle's literal
equations; the factor of Sigma_post in a given site order against the
oracle's; Algorithm 1 on the posterior against the oracle end to end;
rejections."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import posterior as opost
import paper_2405_14892_amd as mvn
import workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _problem(k, n, m, seed, beta=0.1, nugget=1e-4, noise=0.25):
    rng = np.random.default_rng(seed)
    locs = workloads.grid_locations(k)[:n]
    kern = (1.0, beta, 0.5, nugget)
    x = workloads.gp_draw_grid(k, 1.0, beta, 0.5, nugget, rng)[0][:n]
    obs = np.sort(rng.choice(n, m, replace=False))
    y = x[obs] + rng.normal(0, math.sqrt(noise), m)
    mu = rng.normal(0, 0.3, n)
    return locs, kern, obs, y, mu, noise


@pytest.mark.parametrize("n,m,tile", [(300, 45, 64), (257, 128, 128), (100, 1, 16), (130, 70, 100)])
def test_posterior_matches_oracle(n, m, tile):
    print(f"posterior n={n} m={m} tile={tile}", flush=True)
    locs, kern, obs, y, mu, noise = _problem(18, n, m, seed=n + m)
    if m > 3:
        obs[1] = obs[2]  # a site observed twice
    post = mvn.mvn_posterior(locs, kern, obs, y, noise, mu=mu, opts=mvn.options(tile=tile), device=DEV)
    torch.cuda.synchronize()
    assert post["info"] == 0
    S_ref, m_ref = opost.posterior(oracle.covariance(locs, *kern), mu, obs, y, noise)
    S = np.tril(post["sigma_post"].cpu().numpy())
    err_s = np.max(np.abs(S - np.tril(S_ref)))
    err_m = np.max(np.abs(post["mu_post"].cpu().numpy() - m_ref))
    err_v = np.max(np.abs(post["var_post"].cpu().numpy() - np.diag(S_ref)))
    print(f"max error: Sigma_post {err_s:.2e} mu_post {err_m:.2e} var {err_v:.2e}", flush=True)
    assert err_s < 1e-9 and err_m < 1e-9 and err_v < 1e-9


@pytest.mark.parametrize("tlr", [False, True])
def test_permuted_factor_matches_oracle(tlr):
    n, m = 400, 60
    locs, kern, obs, y, mu, noise = _problem(20, n, m, seed=3)
    post = mvn.mvn_posterior(locs, kern, obs, y, noise, mu=mu, opts=mvn.options(tile=128), device=DEV)
    perm = np.random.default_rng(4).permutation(n)
    opts = mvn.options(tile=128, tlr_eps=1e-12, max_rank=128) if tlr else mvn.options(tile=128)
    f = mvn.mvn_cholesky_permuted(post["sigma_post"], perm, opts=opts)
    torch.cuda.synchronize()
    assert f.info() == 0
    S_ref, _ = opost.posterior(oracle.covariance(locs, *kern), mu, obs, y, noise)
    L_ref = oracle.cholesky(S_ref[np.ix_(perm, perm)])
    if tlr:
        D0 = np.tril(f.tiles()[0].cpu().numpy())
        assert np.max(np.abs(D0 - L_ref[:128, :128])) < 1e-9
    else:
        assert np.max(np.abs(f.L().cpu().numpy() - L_ref)) < 1e-9
    # the identity order gives mvn_cholesky's factor of the same matrix
    if not tlr:
        g = mvn.mvn_cholesky_permuted(post["sigma_post"], np.arange(n), opts=opts)
        full = torch.tril(post["sigma_post"]) + torch.tril(post["sigma_post"], -1).T
        h = mvn.mvn_cholesky(n, sigma=full.contiguous(), opts=opts, device=DEV)
        torch.cuda.synchronize()
        assert torch.equal(g.L(), h.L())


def test_posterior_confidence_region_matches_oracle():
    """Algorithm 1 on the posterior: order by posterior marginal exceedance,
    factor of Sigma_post in that order, nested-set sweep; the same steps
    through the oracle give the same order, probabilities and region."""
    k, m, u, alpha = 22, 90, 0.2, 0.1
    n = k * k
    locs, kern, obs, y, mu, noise = _problem(k, n, m, seed=11, beta=0.15)
    N, S, seed = 2000, 6, 21
    res = mvn.posterior_confidence_region(locs, kern, obs, y, noise, u, alpha=alpha, mu=mu, N=N, S=S, seed=seed,
                                          opts=mvn.options(tile=128), device=DEV)
    assert res["info"] == 0
    S_ref, m_ref = opost.posterior(oracle.covariance(locs, *kern), mu, obs, y, noise)
    order = oracle.exceedance_order(m_ref, np.sqrt(np.diag(S_ref)), u)
    assert np.array_equal(res["order"], order)
    L = oracle.cholesky(S_ref[np.ix_(order, order)])
    at, bt = oracle.centre(np.full(n, u), np.full(n, np.inf), m_ref[order])
    ref = oracle.prefix_probs(L, at, bt, N, S, seed)
    np.testing.assert_allclose(res["logP"], ref["logP"], rtol=1e-8, atol=1e-10)
    kref = int(np.sum(np.exp(ref["logP"]) >= 1 - alpha))
    assert np.array_equal(res["region"], np.sort(order[:kref]))
    print(f"posterior region {kref} of {n}", flush=True)
    assert 0 < kref < n


def test_rejections():
    """Host-checked arguments return their position; the device index arrays
    (observed sites, site permutation) are checked on the device: a bad entry
    gives info = -1 and NaN outputs, with nothing read back by the call."""
    n, m = 50, 5
    locs, kern, obs, y, mu, noise = _problem(10, n, m, seed=1)
    o = mvn.options(tile=64)
    for badval in (n, -1):
        bad = obs.copy()
        bad[0] = badval
        post = mvn.mvn_posterior(locs, kern, bad, y, noise, opts=o, device=DEV)
        assert post["info"] == -1
        assert torch.all(torch.isnan(post["mu_post"])) and torch.all(torch.isnan(post["var_post"]))
    with pytest.raises(mvn.MvnError) as e:
        mvn.mvn_posterior(locs, kern, obs, y, 0.0, opts=o, device=DEV)
    assert e.value.code == -8
    with pytest.raises(mvn.MvnError) as e:
        mvn.mvn_posterior(locs, kern, obs, y, noise, opts=mvn.options(tile=64, precision=mvn.MVN_FP32), device=DEV)
    assert e.value.code == -9
    post = mvn.mvn_posterior(locs, kern, obs, y, noise, opts=o, device=DEV)
    assert post["info"] == 0
    for tlr in (False, True):
        oo = mvn.options(tile=128, tlr_eps=1e-6, max_rank=64) if tlr else o
        for broken in ("repeat", "range"):
            perm = np.arange(n)
            perm[3] = 4 if broken == "repeat" else n + 7
            f = mvn.mvn_cholesky_permuted(post["sigma_post"], perm, opts=oo)
            torch.cuda.synchronize()
            assert f.info() == -1, (tlr, broken)
            r = mvn.mvn_prob(f, np.full(n, -np.inf), np.zeros(n), N=64, S=1, seed=1, opts=oo)
            assert torch.isnan(r["logP"])
        f = mvn.mvn_cholesky_permuted(post["sigma_post"], np.arange(n)[::-1].copy(), opts=oo)
        torch.cuda.synchronize()
        assert f.info() == 0


def test_exceedance_order_on_the_device():
    """Algorithm 1's order computed on the device: equal to the oracle's
    (decreasing Phi((mu - u) / sd), ties by index) on 5000 sites with exact
    ties, zero variances (p = 1 above u, else 0) and a non-power-of-two
    size; p to 1e-15 against the oracle's; a NaN variance gives all -1."""
    rng = np.random.default_rng(9)
    n, u = 5000, 0.3
    mu = rng.normal(0.0, 1.0, n)
    var = rng.uniform(0.05, 2.0, n)
    mu[100:120], var[100:120] = 0.7, 0.5        # 20 exact ties
    mu[200:210], var[200:210] = 1.0, 0.0        # known above u: p = 1
    mu[300:310], var[300:310] = -1.0, 0.0       # known below u: p = 0
    perm, p = mvn.mvn_exceedance_order(mu, var, u, device=DEV)
    torch.cuda.synchronize()
    sd = np.sqrt(np.maximum(var, 0.0))
    with np.errstate(divide="ignore", invalid="ignore"):
        ref_order = oracle.exceedance_order(mu, sd, u)
    from scipy.special import ndtr
    with np.errstate(divide="ignore", invalid="ignore"):
        pref = ndtr(np.where(sd > 0, (mu - u) / sd, np.where(mu > u, np.inf, -np.inf)))
    got = perm.cpu().numpy()
    assert np.array_equal(np.sort(got), np.arange(n))
    assert np.array_equal(got, ref_order)
    np.testing.assert_allclose(p.cpu().numpy(), pref, rtol=1e-14, atol=1e-300)
    var[7] = np.nan
    perm, _ = mvn.mvn_exceedance_order(mu, var, u, device=DEV)
    assert np.all(perm.cpu().numpy() == -1)
    perm, p = mvn.mvn_exceedance_order(np.array([2.0]), np.array([1.0]), u, device=DEV)
    assert perm.cpu().numpy().tolist() == [0]
