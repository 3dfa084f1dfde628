"""The benchmark workloads at their full sizes, in the configurations the
benchmark times, checked on outputs the oracle can compute one at a time or
through properties that hold at any size.

* 16384 sites (tile 512, FP64, N = 20000 x S = 10): the whole factor against
  the oracle's Cholesky, and the per-sample log-products l of sampled sample
  columns against the oracle's sweep of those columns (1e-10 relative, the
  FP64 bar).
* 65536 sites, tile low rank (tile 1024, eps = 1e-5, max_rank 256): sampled
  panel tiles meet ||A - L_ik L_kk^T||_F <= eps on the tile compressed and
  have at least the SVD eps-rank; log P-hat agrees with the dense FP64 path
  (whose factor and sweep are the ones checked above) to 1e-7 relative.
* 2000 confidence-region problems (FP64, 64-row sweep blocks as tuned):
  sampled problems against the oracle, all samples, 1e-10.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2405_14892_amd as mvn
import workloads

pytestmark = pytest.mark.gpu


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
        print(f"tile ({i},{k}) rank {ranks[p]} eps-rank {int(np.sum(s > eps))} residual {res:.3g}", flush=True)
        assert res <= eps * (1 + 1e-6) + 1e-12
        assert ranks[p] >= int(np.sum(s > eps))
    del f, r, tiles, U, Vt
    torch.cuda.empty_cache()
    print("tlr64k: dense", flush=True)
    do = mvn.options(tile=512)
    fd = mvn.mvn_cholesky(w.n, locs=w.locs, kern=kern, opts=do)
    rd = mvn.mvn_prob(fd, w.a, w.b, None, N=w.N, S=w.S, seed=w.seed, opts=do)
    torch.cuda.synchronize()
    logp_dense = rd["logP"].item()
    print(f"log P TLR {logp_tlr} dense {logp_dense}", flush=True)
    assert abs(logp_tlr - logp_dense) < 1e-7 * abs(logp_dense)


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
