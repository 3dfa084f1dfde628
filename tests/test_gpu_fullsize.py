"""The benchmark workloads at their full sizes, in the configurations the
benchmark times, checked on outputs the oracle can compute one at a time or
through properties that hold at any size.

* 16384 sites (tile 512, FP64, N = 20000 x S = 10): the whole factor against
  the oracle's Cholesky, and the per-sample log-products l of sampled sample
  columns against the oracle's sweep of those columns (1e-10 relative, the
  FP64 bar).
* Confidence-region detection on the same field (sites in exceedance
  order, one nested-set sweep): the first 200 nested-set probabilities
  against the oracle's from the leading block, 1e-10 relative.
* 65536 sites, tile low rank (tile 1024, eps = 1e-5, max_rank 256): sampled
  panel tiles meet ||A - L_ik L_kk^T||_F <= eps on the tile compressed and
  have at least the SVD eps-rank; log P-hat agrees with the dense FP64 path
  (whose factor and sweep are the ones checked above) to 1e-7 relative.
* 2000 confidence-region problems (FP64, 64-row sweep blocks as tuned):
  sampled problems against the oracle, all samples, 1e-10.
* The Monte Carlo check on the 16384-site factor (50 000 fields, as the
  benchmark draws): sampled samples' first failing sites against the
  oracle's fields through its own factor; the counts against the first
  failures.
* The posterior at 40 000 sites and 6 250 observations (tile 512): mu_post,
  variances and Sigma_post at sampled sites against the oracle's kriging
  form, 1e-9; the factor of Sigma_post in exceedance order reproduces
  sampled entries of the permuted Sigma_post (L L^T at any size).
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import mc as omc
from oracle import posterior as opost
import paper_2405_14892_amd as mvn
import workloads

pytestmark = pytest.mark.gpu


# Per-sample error bars of the reduced-precision modes on the 16384-site
# workload (sampled columns; |l - l_oracle| with the oracle's FP64 factor and
# sweep on identical QMC points; log P is about -458).  They state the
# error, they are not parity: reduced precision has no exact pin.  Measured
# maxima: FP32 1.4e-3, split BF16 4.1e-3, BF16 2.07 (the sweep GEMM's
# operand rounding, amplified by 1 / L_ii = 23 on this field, dominates: the
# adaptive and FP64 factorisations give the same errors).
REDUCED_MODES = [
    (mvn.MVN_FP32, mvn.MVN_CHOL_ADAPTIVE, 1e-2),
    (mvn.MVN_FP32, mvn.MVN_CHOL_FP64, 1e-2),
    (mvn.MVN_BF16X3, mvn.MVN_CHOL_ADAPTIVE, 3e-2),
    (mvn.MVN_BF16X3, mvn.MVN_CHOL_FP64, 3e-2),
    (mvn.MVN_BF16, mvn.MVN_CHOL_ADAPTIVE, 20.0),
    (mvn.MVN_BF16, mvn.MVN_CHOL_FP64, 20.0),
]


@pytest.fixture(scope="module")
def prec16k_oracle():
    w = workloads.make_workload("prec16k")
    kern = (w.sigma2, w.beta, w.nu, w.nugget)
    print("prec16k: oracle Cholesky", flush=True)
    L = oracle.cholesky(oracle.covariance(w.locs, *kern), block=512)
    at, bt = oracle.centre(w.a, w.b, w.mu)
    NS = w.N * w.S
    cols = np.array([0, 1, w.N - 1, w.N, NS // 2, NS // 2 + 63, NS - 64, NS - 1])
    print("prec16k: oracle sweep of sampled columns", flush=True)
    ref = oracle.sweep(L, at, bt, w.N, w.S, w.seed, cols=cols)
    return w, L, cols, ref


@pytest.mark.parametrize("prec,mode,bound", REDUCED_MODES)
def test_prec16k_reduced_precision_error_statement(prec16k_oracle, prec, mode, bound):
    """Each reduced-precision mode on the precision workload (condition
    number about 4e6): the factorisation keeps positive definiteness and the
    per-sample log-products of sampled columns stay within the stated bar of
    the oracle's FP64 values."""
    w, L, cols, ref = prec16k_oracle
    kern = (w.sigma2, w.beta, w.nu, w.nugget)
    o = mvn.options(tile=w.tile, precision=prec, chol_mode=mode)
    print(f"prec16k reduced: precision {prec} chol_mode {mode}", flush=True)
    f = mvn.mvn_cholesky(w.n, locs=w.locs, kern=kern, opts=o)
    r = mvn.mvn_prob(f, w.a, w.b, w.mu, N=w.N, S=w.S, seed=w.seed, opts=o, return_ell=True)
    torch.cuda.synchronize()
    assert f.info() == 0
    err = np.abs(r["ell"].cpu().numpy()[cols] - ref)
    counts = f.update_counts()
    print(f"  info 0, |dl| max {err.max():.3e} median {np.median(err):.3e}, log P {r['logP'].item():.6f}, "
          f"tile updates {counts}", flush=True)
    assert np.all(np.isfinite(err))
    assert err.max() <= bound, (prec, mode, err)
    if mode == mvn.MVN_CHOL_ADAPTIVE:
        assert counts["fp64"] + counts["fp32"] + counts["reduced"] > 0
    else:
        assert counts == {"fp64": 0, "fp32": 0, "reduced": 0}


def test_prec16k_full_size_factor_and_sampled_columns():
    w = workloads.make_workload("prec16k")
    kern = (w.sigma2, w.beta, w.nu, w.nugget)
    opts = mvn.options(tile=w.tile)
    print("prec16k: GPU", flush=True)
    f = mvn.mvn_cholesky(w.n, locs=w.locs, kern=kern, opts=opts)
    r = mvn.mvn_prob(f, w.a, w.b, w.mu, N=w.N, S=w.S, seed=w.seed, opts=opts, return_ell=True)
    torch.cuda.synchronize()
    assert f.info() == 0
    L_gpu = f.L().cpu().numpy()
    ell = r["ell"].cpu().numpy()
    print("prec16k: oracle Cholesky", flush=True)
    L = oracle.cholesky(oracle.covariance(w.locs, *kern), block=512)
    assert np.max(np.abs(L_gpu - L)) < 1e-10
    del L_gpu
    at, bt = oracle.centre(w.a, w.b, w.mu)
    NS = w.N * w.S
    cols = np.array([0, 1, w.N - 1, w.N, NS // 2, NS // 2 + 63, NS - 64, NS - 1])
    ref = oracle.sweep(L, at, bt, w.N, w.S, w.seed, cols=cols)
    rel = np.abs(ell[cols] - ref) / np.maximum(1.0, np.abs(ref))
    print("prec16k: sampled l", ref, "max rel", rel.max(), flush=True)
    assert rel.max() < 1e-10
    # the Monte Carlo check on the same factor, at the benchmark's 50 000 fields
    M = 50000
    m = mvn.mvn_mc_prefix(f, w.a, w.b, w.mu, M=M, seed=w.seed + 1, opts=opts)
    first = m["first"].cpu().numpy()
    count = m["count"].cpu().numpy()
    np.testing.assert_array_equal(count, omc.prefix_counts(first, w.n))
    mc_cols = np.array([0, 63, 64, 777, M // 2, M - 1])
    X = omc.fields(L, w.mu, w.seed + 1, mc_cols)
    ref_first = omc.first_failure(X, w.a, w.b)
    print("prec16k: Monte Carlo first failures", first[mc_cols], ref_first, flush=True)
    bad = np.nonzero(first[mc_cols] != ref_first)[0]
    for j in bad:  # only where the deciding value sits on a limit to rounding
        k = min(first[mc_cols][j], ref_first[j])
        assert min(abs(X[k, j] - w.a[k]), abs(X[k, j] - w.b[k])) < 1e-9


def test_crd16k_full_size_leading_nested_sets():
    """Confidence-region detection on the 16384-site field as the benchmark
    runs it (sites in order of marginal exceedance of u = 0.5, tile 512,
    N = 20000 x S = 10, 128-row blocks): the first 200 nested-set log P-hat
    of the one sweep against the oracle's from the leading 200 x 200 block
    of the ordered covariance, with the shifts of the 16384-site problem
    (1e-10 relative, the FP64 bar); the last nested set is the full
    estimate."""
    import math
    w = workloads.make_workload("prec16k")
    u, K = 0.5, 200
    kern = (w.sigma2, w.beta, w.nu, w.nugget)
    field = w.extra["field"]
    order = oracle.exceedance_order(field, np.full(w.n, math.sqrt(w.sigma2 + w.nugget)), u)
    a, b, mu = np.full(w.n, u), np.full(w.n, np.inf), field[order]
    opts = mvn.options(tile=w.tile)
    print("crd16k: GPU", flush=True)
    f = mvn.mvn_cholesky(w.n, locs=w.locs[order], kern=kern, opts=opts)
    r = mvn.mvn_prob_prefix(f, a, b, mu, N=w.N, S=w.S, seed=w.seed, opts=opts)
    full = mvn.mvn_prob(f, a, b, mu, N=w.N, S=w.S, seed=w.seed, opts=opts)
    torch.cuda.synchronize()
    assert f.info() == 0
    logp = r["logP"].cpu().numpy()
    full_logp = full["logP"].item()
    del f, r, full
    print("crd16k: oracle on the leading block", flush=True)
    Lk = oracle.cholesky(oracle.covariance(w.locs[order][:K], *kern))
    at, bt = oracle.centre(a[:K], b[:K], mu[:K])
    ref = oracle.prefix_probs(Lk, at, bt, w.N, w.S, w.seed, dim=w.n)["logP"]
    rel = np.abs(logp[:K] - ref) / np.maximum(1.0, np.abs(ref))
    print("crd16k: log P of nested sets 1, 10, 200:", logp[[0, 9, K - 1]], "max rel", rel.max(), flush=True)
    assert rel.max() < 1e-10
    assert abs(logp[-1] - full_logp) <= 1e-12 * max(1.0, abs(full_logp))


def test_tlr64k_full_size_properties():
    w = workloads.make_workload("tlr64k")
    kern = (w.sigma2, w.beta, w.nu, w.nugget)
    eps, rcap = 1e-5, 256
    to = mvn.options(tile=w.tile, tlr_eps=eps, max_rank=rcap)
    print("tlr64k: TLR", flush=True)
    f = mvn.mvn_cholesky(w.n, locs=w.locs, kern=kern, opts=to)
    r = mvn.mvn_prob(f, w.a, w.b, None, N=w.N, S=w.S, seed=w.seed, opts=to)
    torch.cuda.synchronize()
    assert f.info() == 0
    logp_tlr = r["logP"].item()
    ranks = f.ranks().cpu().numpy()
    assert np.all(ranks >= 0) and np.all(ranks <= rcap)
    nt = f.nt
    tiles, U, Vt = f.tiles(), f.U(), f.Vt()
    for i, k in ((1, 0), (2, 1), (63, 62), (40, 3), (63, 0), (33, 17)):
        p = i * (i - 1) // 2 + k
        A = tiles[i * (i + 1) // 2 + k].cpu().numpy()
        Dk = np.tril(tiles[k * (k + 1) // 2 + k].cpu().numpy())
        Lik = U[p].cpu().numpy() @ Vt[p].cpu().numpy()
        res = np.linalg.norm(A - Lik @ Dk.T)
        s = np.linalg.svd(A, compute_uv=False)
        tail = np.sqrt(np.cumsum((s ** 2)[::-1]))[::-1]
        kopt = int(np.sum(tail > eps))  # Frobenius eps-rank
        print(f"tile ({i},{k}) rank {ranks[p]} eps-rank {int(np.sum(s > eps))} Frobenius eps-rank {kopt} "
              f"residual {res:.3g}", flush=True)
        assert res <= eps * (1 + 1e-6) + 1e-12
        assert ranks[p] >= kopt
    del f, r, tiles, U, Vt
    torch.cuda.empty_cache()
    print("tlr64k: dense", flush=True)
    do = mvn.options(tile=512)
    fd = mvn.mvn_cholesky(w.n, locs=w.locs, kern=kern, opts=do)
    rd = mvn.mvn_prob(fd, w.a, w.b, None, N=w.N, S=w.S, seed=w.seed, opts=do)
    torch.cuda.synchronize()
    logp_dense = rd["logP"].item()
    print(f"log P TLR {logp_tlr} dense {logp_dense}", flush=True)
    # The compression threshold bounds each tile's error (Section III-E: the
    # truncated SVD of every tile); the shift of log P it causes has no bound
    # of its own.  With ranks at the tiles' eps-ranks each tile's error is
    # close to eps (measured 1.5e-4 in log P, i.e. P x 1.00015), so this is a
    # statement of the observed accuracy with a margin, not a pin.
    assert abs(logp_tlr - logp_dense) < 5e-7 * abs(logp_dense)


def test_batch2000_full_size_sampled_problems():
    bw = workloads.make_batch()
    kern = (bw.sigma2, bw.beta, bw.nu, bw.nugget)
    plan = mvn.mvn_batch_plan(bw.n_p, bw.N, bw.S, opts=mvn.options(tile=128, sweep_rows=64))
    out = mvn.mvn_prob_batch(plan, bw.idx, bw.locs, kern, bw.a, bw.b, seed=bw.seed).cpu().numpy()
    assert torch.all(plan.info == 0)
    order = np.argsort(bw.n_p)
    picks = list(order[:3]) + [int(order[len(order) // 8])]
    for p in picks:
        sl = slice(bw.off[p], bw.off[p + 1])
        L = oracle.cholesky(oracle.covariance(bw.locs[bw.idx[sl]], *kern))
        ref = oracle.reduce_samples(oracle.sweep(L, bw.a[sl], bw.b[sl], bw.N, bw.S, bw.seed), bw.N, bw.S)
        print(f"problem {p} n={bw.n_p[p]} logP {out[p, 0]} oracle {ref['logP']}", flush=True)
        assert abs(out[p, 0] - ref["logP"]) < 1e-10 * max(1.0, abs(ref["logP"]))


def test_post40k_full_size_sampled_sites():
    d = workloads.make_posterior(beta=0.1)
    kern = (d.sigma2, d.beta, d.nu, d.nugget)
    n = d.locs.shape[0]
    opts = mvn.options(tile=512)
    print("post40k: GPU posterior", flush=True)
    post = mvn.mvn_posterior(d.locs, kern, d.obs, d.y, d.noise_sd ** 2, opts=opts)
    torch.cuda.synchronize()
    assert post["info"] == 0
    sites = np.array([0, 1, int(d.obs[0]), int(d.obs[-1]), 12345, 20000, n - 1])
    print("post40k: oracle at sampled sites", flush=True)
    ref = opost.posterior_at(d.locs, kern, None, d.obs, d.y, d.noise_sd ** 2, sites)
    mu_post = post["mu_post"].cpu().numpy()
    var_post = post["var_post"].cpu().numpy()
    err_m = np.max(np.abs(mu_post[sites] - ref["mu_post"]))
    err_v = np.max(np.abs(var_post[sites] - ref["var_post"]))
    S = post["sigma_post"]
    got = np.array([[S[max(i, j), min(i, j)].item() for j in sites] for i in sites])
    err_s = np.max(np.abs(got - ref["sigma_post"]))
    print(f"post40k: max error mu {err_m:.2e} var {err_v:.2e} Sigma {err_s:.2e}", flush=True)
    assert err_m < 1e-9 and err_v < 1e-9 and err_s < 1e-9
    # the factor in exceedance order (u = 0.5) reproduces the permuted entries
    from scipy.special import ndtr
    order = np.argsort(-ndtr((mu_post - 0.5) / np.sqrt(var_post)), kind="stable")
    f = mvn.mvn_cholesky_permuted(S, order, opts=opts)
    torch.cuda.synchronize()
    assert f.info() == 0
    rows = [0, 1, 4095, 20000, n - 1]
    Lr = {i: f.L()[i, : i + 1].cpu().numpy() for i in rows}
    for i in rows:
        for j in rows:
            if j <= i:
                lhs = float(Lr[i][: j + 1] @ Lr[j][: j + 1])
                a, b = int(order[i]), int(order[j])
                rhs = S[max(a, b), min(a, b)].item()
                assert abs(lhs - rhs) < 1e-10, (i, j, lhs, rhs)
