"""Nested-set probabilities of confidence-region detection (Section III-C with
Algorithm 1 of Section IV-A) through the C ABI: every prefix log P-hat of one sweep against
the oracle's running products (oracle.prefix_probs) on identical QMC points,
FP64 to 1e-10 relative; the last prefix against the full estimate; mixed
precision against the same call's full estimate; rejections; and the
confidence region of a small field against the one the oracle's prefixes
give.  Nested sets through a TLR factor against the oracle on the dense
factor assembled from the same compressed tiles."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2405_14892_amd as mvn
import workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _field(k, n, seed, beta=0.1, nu=0.5, nugget=1e-8, u=0.0):
    rng = np.random.default_rng(seed)
    locs = workloads.grid_locations(k)[:n]
    mu = workloads.gp_draw_grid(k, 1.0, beta, nu, nugget, rng)[0][:n]
    return locs, (1.0, beta, nu, nugget), mu


@pytest.mark.parametrize("n,tile,N,S,rows", [(400, 100, 10000, 10, 128), (333, 128, 100, 3, 128),
                                              (333, 128, 100, 3, 64), (70, 64, 64, 1, 128)])
def test_prefix_matches_oracle(n, tile, N, S, rows):
    """N = 100: chunks of 64 samples straddle the shift boundaries; S = 1:
    no standard error."""
    print(f"prefix n={n} tile={tile} N={N} S={S} rows={rows}", flush=True)
    locs, kern, mu = _field(20, n, seed=31 + n)
    a, b = np.full(n, -np.inf), -mu
    opts = mvn.options(tile=tile, sweep_rows=rows)
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=opts, device=DEV)
    seed = 1234
    r = mvn.mvn_prob_prefix(f, a, b, None, N=N, S=S, seed=seed, opts=opts)
    full = mvn.mvn_prob(f, a, b, None, N=N, S=S, seed=seed, opts=opts)
    torch.cuda.synchronize()
    logp = r["logP"].cpu().numpy()
    rel = r["rel_stderr"].cpu().numpy()
    L = oracle.cholesky(oracle.covariance(locs, *kern))
    at, bt = oracle.centre(a, b)
    ref = oracle.prefix_probs(L, at, bt, N, S, seed)
    err = np.abs(logp - ref["logP"]) / np.maximum(1.0, np.abs(ref["logP"]))
    print(f"max rel err {err.max():.3e}; last prefix {logp[-1]} full {full['logP'].item()}", flush=True)
    assert err.max() < 1e-10
    if S > 1:
        np.testing.assert_allclose(rel, ref["rel_stderr"], rtol=1e-8, atol=1e-14)
    else:
        assert np.all(np.isnan(rel))
    assert np.all(np.diff(logp) <= 1e-12)
    assert abs(logp[-1] - full["logP"].item()) < 1e-12 * max(1.0, abs(logp[-1]))


@pytest.mark.parametrize("prec", [mvn.MVN_FP32, mvn.MVN_BF16X3])
def test_prefix_mixed_precision_last_equals_full(prec):
    n = 300
    locs, kern, mu = _field(20, n, seed=5)
    a, b = np.full(n, -np.inf), 0.5 - mu
    opts = mvn.options(tile=128, precision=prec)
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=opts, device=DEV)
    r = mvn.mvn_prob_prefix(f, a, b, None, N=500, S=4, seed=7, opts=opts)
    full = mvn.mvn_prob(f, a, b, None, N=500, S=4, seed=7, opts=opts)
    torch.cuda.synchronize()
    logp = r["logP"].cpu().numpy()
    assert abs(logp[-1] - full["logP"].item()) < 1e-12 * max(1.0, abs(logp[-1]))
    # first prefix: d_1 does not depend on the points
    sd = math.sqrt(kern[0] + kern[3])
    assert abs(logp[0] - math.log(0.5 * math.erfc(-b[0] / sd / math.sqrt(2.0)))) < 1e-6


def test_prefix_rejections_and_invalid_limits():
    n = 50
    locs, kern, mu = _field(10, n, seed=3)
    opts = mvn.options(tile=64)
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=opts, device=DEV)
    a, b = np.full(n, -np.inf), -mu
    with pytest.raises(mvn.MvnError) as e:  # from the workspace query (argument 2) or the call (5)
        mvn.mvn_prob_prefix(f, a, b, N=63, S=2, seed=1, opts=opts)
    assert e.value.code in (-2, -5) and "N >= 64" in str(e.value)
    bad = b.copy()
    bad[7] = np.nan
    r = mvn.mvn_prob_prefix(f, a, bad, N=64, S=2, seed=1, opts=opts)
    torch.cuda.synchronize()
    assert torch.all(torch.isnan(r["out"]))
    t = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=mvn.options(tile=128, tlr_eps=1e-6, max_rank=64),
                         device=DEV)
    with pytest.raises(mvn.MvnError) as e:  # the TLR sweep is FP64 only
        mvn.mvn_prob_prefix(t, a, b, N=64, S=2, seed=1, opts=mvn.options(tile=128, precision=mvn.MVN_FP32))
    assert e.value.code == -8


def _dense_from_tlr(f):
    """Dense L assembled on the host from the TLR buffers (tiles, U, Vt)."""
    m, nt, n = f.handle.tile, f.nt, f.n
    tiles = f.tiles().cpu().numpy()
    U, Vt = f.U().cpu().numpy(), f.Vt().cpu().numpy()
    L = np.zeros((nt * m, nt * m))
    for i in range(nt):
        L[i * m:(i + 1) * m, i * m:(i + 1) * m] = np.tril(tiles[i * (i + 1) // 2 + i])
        for k in range(i):
            p = i * (i - 1) // 2 + k
            L[i * m:(i + 1) * m, k * m:(k + 1) * m] = U[p] @ Vt[p]
    return L[:n, :n]


@pytest.mark.parametrize("rows", [64, 128, 256])
def test_prefix_on_tlr_factor_matches_oracle(rows):
    """Nested sets through the tile low-rank sweep (ranks of some tens, a
    partial last tile): every prefix against the oracle's running products
    through the dense L assembled from the same compressed factor, and the
    last prefix against the TLR full estimate."""
    n, tile, N, S, seed = 1100, 128, 300, 3, 919
    print(f"tlr prefix rows={rows}", flush=True)
    rng = np.random.default_rng(44)
    perm = workloads.morton_permutation(40)
    locs = workloads.grid_locations(40)[perm][:n]
    mu = workloads.gp_draw_grid(40, 1.0, 0.05, 0.5, 1e-8, rng)[0][perm][:n]
    kern = (1.0, 0.05, 0.5, 1e-8)
    a, b = np.full(n, -np.inf), -mu
    opts = mvn.options(tile=tile, tlr_eps=1e-5, max_rank=128, sweep_rows=rows)
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=opts, device=DEV)
    r = mvn.mvn_prob_prefix(f, a, b, None, N=N, S=S, seed=seed, opts=opts)
    full = mvn.mvn_prob(f, a, b, None, N=N, S=S, seed=seed, opts=opts)
    torch.cuda.synchronize()
    assert f.info() == 0
    assert f.ranks().cpu().numpy().max() > 16
    logp = r["logP"].cpu().numpy()
    L = _dense_from_tlr(f)
    at, bt = oracle.centre(a, b)
    ref = oracle.prefix_probs(L, at, bt, N, S, seed)
    err = np.abs(logp - ref["logP"]) / np.maximum(1.0, np.abs(ref["logP"]))
    print(f"max rel err {err.max():.3e}; last {logp[-1]} full {full['logP'].item()}", flush=True)
    assert err.max() < 1e-9
    np.testing.assert_allclose(r["rel_stderr"].cpu().numpy(), ref["rel_stderr"], rtol=1e-6, atol=1e-12)
    assert abs(logp[-1] - full["logP"].item()) < 1e-12 * max(1.0, abs(logp[-1]))


def test_confidence_region_matches_oracle_prefixes():
    """Algorithm 1 on a 24 x 24 field: the region is the longest prefix (in
    order of marginal exceedance) whose joint probability >= 1 - alpha; the
    same order, factor and points through the oracle give the same region."""
    k, u, alpha = 24, 0.3, 0.1
    n = k * k
    locs, kern, mu = _field(k, n, seed=77, beta=0.08)
    N, S, seed = 2000, 8, 99
    res = mvn.confidence_region(locs, kern, mu, u, alpha=alpha, N=N, S=S, seed=seed,
                                opts=mvn.options(tile=128), device=DEV)
    assert res["info"] == 0
    order = oracle.exceedance_order(mu, np.full(n, math.sqrt(kern[0] + kern[3])), u)
    assert np.array_equal(res["order"], order)
    L = oracle.cholesky(oracle.covariance(locs[order], *kern))
    at, bt = oracle.centre(np.full(n, u), np.full(n, np.inf), mu[order])
    ref = oracle.prefix_probs(L, at, bt, N, S, seed)
    np.testing.assert_allclose(res["logP"], ref["logP"], rtol=1e-10, atol=1e-12)
    kref = int(np.sum(np.exp(ref["logP"]) >= 1 - alpha))
    assert np.array_equal(res["region"], np.sort(order[:kref]))
    print(f"region size {kref} of {n}", flush=True)
    assert 0 < kref < n


@pytest.mark.parametrize("prec", [mvn.MVN_FP32, mvn.MVN_BF16X3])
def test_prefix_mixed_precision_every_prefix_within_1e4(prec):
    """Reduced-precision nested sets against the FP64 oracle's on the same
    points: |P-hat - P-hat_oracle| <= 1e-4 for every prefix (the mixed
    precision bar, stated where P = O(1); the deep prefixes are smaller)."""
    n, N, S, seed = 400, 2000, 4, 71
    locs, kern, mu = _field(20, n, seed=13)
    order = oracle.exceedance_order(mu, np.full(n, math.sqrt(kern[0] + kern[3])), 0.2)
    locs, mu = locs[order], mu[order]
    a, b = np.full(n, 0.2), np.full(n, np.inf)
    opts = mvn.options(tile=128, precision=prec)
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=opts, device=DEV)
    r = mvn.mvn_prob_prefix(f, a, b, mu, N=N, S=S, seed=seed, opts=opts)
    torch.cuda.synchronize()
    p = np.exp(r["logP"].cpu().numpy())
    L = oracle.cholesky(oracle.covariance(locs, *kern))
    at, bt = oracle.centre(a, b, mu)
    ref = np.exp(oracle.prefix_probs(L, at, bt, N, S, seed)["logP"])
    err = np.abs(p - ref)
    print(f"prec {prec}: max |dP| {err.max():.2e} (P from {ref.max():.3f} down to {ref.min():.2e})", flush=True)
    assert err.max() <= 1e-4
