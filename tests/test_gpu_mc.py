"""Monte Carlo check of nested sets (Section V-C) through the C ABI: every
sample's first failing site against the oracle's draws of the same fields
(counter-based normals, so the same Z on both sides), over ragged sizes,
both block shapes, samples that fail early (the chunk stops) and samples
that never fail (every block, the diagonal ones included); the counts
against the first failures; against the QMC nested-set estimate of the same
field within the Monte Carlo error; edge cases and rejections; and the check
a confidence region carries."""
import math

import numpy as np
import pytest
import scipy.stats as st
import torch

import oracle
from oracle import mc as omc
import paper_2405_14892_amd as mvn
import workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _field(k, n, seed, beta=0.1, nu=0.5, nugget=1e-8):
    rng = np.random.default_rng(seed)
    locs = workloads.grid_locations(k)[:n]
    mu = workloads.gp_draw_grid(k, 1.0, beta, nu, nugget, rng)[0][:n]
    return locs, (1.0, beta, nu, nugget), mu


def _compare_first(first_gpu, X, a, b, first_ref):
    """Equal first failures, except where the deciding value sits within
    1e-9 of a limit (the two sides round the product differently)."""
    bad = np.nonzero(first_gpu != first_ref)[0]
    for j in bad:
        m = min(first_gpu[j], first_ref[j])
        margin = min(abs(X[m, j] - a[m]), abs(X[m, j] - b[m]))
        assert margin < 1e-9, (j, first_gpu[j], first_ref[j], margin)
    assert bad.size <= 2


@pytest.mark.parametrize("n,M,rows,case", [(333, 1000, 64, "region"), (333, 1000, 128, "region"),
                                           (300, 700, 64, "wide"), (300, 700, 128, "wide"),
                                           (1, 65, 64, "wide"), (130, 1, 128, "region")])
def test_first_failure_matches_oracle(n, M, rows, case):
    print(f"mc n={n} M={M} rows={rows} {case}", flush=True)
    locs, kern, mu = _field(20, n, seed=40 + n)
    sd = math.sqrt(kern[0] + kern[3])
    if case == "region":  # exceedance order, level 0: samples fail along the way
        order = oracle.exceedance_order(mu, np.full(n, sd), 0.0)
        locs, mu = locs[order], mu[order]
        a, b = np.zeros(n), np.full(n, np.inf)
    else:  # wide two-sided limits: most samples never fail
        a, b = mu - 4.0 * sd, mu + 4.0 * sd
    opts = mvn.options(tile=64, sweep_rows=rows)
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=opts, device=DEV)
    seed = 777
    r = mvn.mvn_mc_prefix(f, a, b, mu, M=M, seed=seed, opts=opts)
    torch.cuda.synchronize()
    assert f.info() == 0
    first = r["first"].cpu().numpy()
    count = r["count"].cpu().numpy()
    L = oracle.cholesky(oracle.covariance(locs, *kern))
    X = omc.fields(L, mu, seed, np.arange(M))
    ref = omc.first_failure(X, a, b)
    _compare_first(first, X, a, b, ref)
    np.testing.assert_array_equal(count, omc.prefix_counts(first, n))
    if case == "wide" and n > 1:
        assert np.mean(first == n) > 0.5
    print(f"first failures: min {first.min()} median {np.median(first)} none {np.sum(first == n)}", flush=True)


def test_agrees_with_qmc_nested_sets():
    """n = 2000 in exceedance order, M = 50 000: every prefix count against
    the nested-set QMC estimate of the same factor (different estimator,
    same probabilities) by its exact binomial tail probability (> 1e-6 over
    2000 nested, strongly dependent prefixes), and sampled columns against
    the oracle."""
    k, n, M, u = 50, 2000, 50000, 0.3
    locs, kern, mu = _field(k, n, seed=9, beta=0.05)
    order = oracle.exceedance_order(mu, np.full(n, math.sqrt(kern[0] + kern[3])), u)
    locs, mu = locs[order], mu[order]
    a, b = np.full(n, u), np.full(n, np.inf)
    opts = mvn.options(tile=128)
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=opts, device=DEV)
    r = mvn.mvn_mc_prefix(f, a, b, mu, M=M, seed=3, opts=opts)
    q = mvn.mvn_prob_prefix(f, a, b, mu, N=5000, S=10, seed=4, opts=opts)
    torch.cuda.synchronize()
    cnt = r["count"].cpu().numpy()
    pq = np.exp(q["logP"].cpu().numpy())
    rq = q["rel_stderr"].cpu().numpy()
    # exact binomial tails (counts of a few samples are far from Gaussian),
    # with the QMC estimate's own error widening the band
    lo = np.clip(pq * (1 - 5 * rq), 0, 1)
    hi = np.clip(pq * (1 + 5 * rq), 0, 1)
    pval = np.minimum(st.binom.sf(cnt - 1, M, hi), st.binom.cdf(cnt, M, lo))
    worst = int(np.argmin(pval))
    print(f"worst prefix {worst}: mc {cnt[worst]} of {M}, qmc {pq[worst] * M:.2f}, tail {pval[worst]:.2e}",
          flush=True)
    assert pval.min() > 1e-6
    first = r["first"].cpu().numpy()
    cols = np.array([0, 1, 63, 64, M // 2, M - 1])
    L = oracle.cholesky(oracle.covariance(locs, *kern))
    X = omc.fields(L, mu, 3, cols)
    _compare_first(first[cols], X, a, b, omc.first_failure(X, a, b))


def test_limits_edge_cases_and_failed_factor():
    n, M = 70, 200
    locs, kern, mu = _field(10, n, seed=2)
    opts = mvn.options(tile=64)
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=opts, device=DEV)
    a, b = np.full(n, -np.inf), np.full(n, np.inf)
    r = mvn.mvn_mc_prefix(f, a, b, None, M=M, seed=1, opts=opts)
    torch.cuda.synchronize()
    assert torch.all(r["first"] == n) and torch.all(r["count"] == M)
    a2, b2 = a.copy(), b.copy()
    a2[5] = np.nan           # never holds: every sample fails at site 5
    b2[9] = a2[9] = 1.0      # a point interval: probability zero
    r = mvn.mvn_mc_prefix(f, a2, b2, None, M=M, seed=1, opts=opts)
    torch.cuda.synchronize()
    assert torch.all(r["first"] == 5)
    assert r["count"][4].item() == M and r["count"][5].item() == 0
    rng = np.random.default_rng(1)
    m = rng.standard_normal((100, 100))
    s = m @ m.T + 100 * np.eye(100)
    s[17, 17] = -1.0
    g = mvn.mvn_cholesky(100, sigma=s, opts=opts, device=DEV)
    r = mvn.mvn_mc_prefix(g, np.zeros(100), np.full(100, np.inf), None, M=100, seed=1, opts=opts)
    torch.cuda.synchronize()
    assert g.info() == 18
    assert torch.all(r["first"] == -1) and torch.all(r["count"] == -1)


def test_rejections():
    n = 200
    locs, kern, mu = _field(16, n, seed=5)
    t = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=mvn.options(tile=128, tlr_eps=1e-6, max_rank=32),
                         device=DEV)
    a, b = np.zeros(n), np.full(n, np.inf)
    with pytest.raises(mvn.MvnError) as e:
        mvn.mvn_mc_prefix(t, a, b, M=64, seed=1)
    assert e.value.code == -1
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=mvn.options(tile=128), device=DEV)
    with pytest.raises(mvn.MvnError) as e:
        mvn.mvn_mc_prefix(f, a, b, M=0, seed=1)
    assert e.value.code == -2          # from the workspace query
    with pytest.raises(mvn.MvnError) as e:
        mvn.mvn_mc_prefix(f, a, b, M=64, seed=1, opts=mvn.options(tile=128, sweep_rows=32))
    assert e.value.code == -3


def test_confidence_region_carries_its_check():
    """The region's Monte Carlo fraction against its QMC probability (the
    check of Section V-C: near 1 - alpha)."""
    k, u, alpha, M = 30, 0.3, 0.1, 40000
    locs, kern, mu = _field(k, k * k, seed=77, beta=0.08)
    res = mvn.confidence_region(locs, kern, mu, u, alpha=alpha, N=4000, S=10, seed=5,
                                opts=mvn.options(tile=128), device=DEV, mc_samples=M, mc_seed=6)
    kreg = res["region"].size
    assert 0 < kreg < k * k
    p_qmc = math.exp(res["logP"][kreg - 1])
    tol = 5.0 * math.sqrt(p_qmc * (1 - p_qmc) / M) + 5.0 * p_qmc * res["rel_stderr"][kreg - 1]
    print(f"region {kreg}: qmc {p_qmc} mc {res['mc_p_region']} (1 - alpha = {1 - alpha})", flush=True)
    assert abs(res["mc_p_region"] - p_qmc) < tol
    assert p_qmc >= 1 - alpha


def test_confidence_region_from_a_tlr_factor_carries_its_check():
    """Regions from a TLR factor are checked against the fitted
    distribution itself (dense factor of the same ordered Sigma)."""
    k, u, alpha, M = 30, 0.3, 0.1, 40000
    locs, kern, mu = _field(k, k * k, seed=77, beta=0.08)
    res = mvn.confidence_region(locs, kern, mu, u, alpha=alpha, N=4000, S=10, seed=5,
                                opts=mvn.options(tile=128, tlr_eps=1e-6, max_rank=128), device=DEV,
                                mc_samples=M, mc_seed=6)
    kreg = res["region"].size
    assert 0 < kreg < k * k
    p_qmc = math.exp(res["logP"][kreg - 1])
    tol = 5.0 * math.sqrt(p_qmc * (1 - p_qmc) / M) + 5.0 * p_qmc * res["rel_stderr"][kreg - 1] + 1e-4
    print(f"TLR region {kreg}: qmc {p_qmc} mc {res['mc_p_region']}", flush=True)
    assert abs(res["mc_p_region"] - p_qmc) < tol
