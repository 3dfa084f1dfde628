"""The autotuner on the device: it times every candidate shape through the
library, and the options it returns give the oracle's result (the shapes
change the schedule, not the arithmetic)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2405_14892_amd as mvn
from paper_2405_14892_amd import autotune
import workloads

pytestmark = pytest.mark.gpu


def test_tuned_batch_matches_oracle(tmp_path):
    bw = workloads.make_batch(count=12, n_min=40, n_max=500, seed=11, N=300, S=2)
    kern = (bw.sigma2, bw.beta, bw.nu, bw.nugget)
    res = autotune.tune_batch(bw.n_p, bw.idx, bw.locs, kern, bw.a, bw.b, N=bw.N, S=bw.S, seed=bw.seed,
                              cache_path=str(tmp_path / "t.json"))
    print(res, flush=True)
    assert res["sweep_rows"] in (64, 128) and all(v > 0 for v in res["batch_s"].values())
    plan = mvn.mvn_batch_plan(bw.n_p, bw.N, bw.S, opts=mvn.options(tile=128, sweep_rows=res["sweep_rows"]))
    out = mvn.mvn_prob_batch(plan, bw.idx, bw.locs, kern, bw.a, bw.b, seed=bw.seed).cpu().numpy()
    for p in range(len(bw.n_p)):
        sl = slice(bw.off[p], bw.off[p + 1])
        L = oracle.cholesky(oracle.covariance(bw.locs[bw.idx[sl]], *kern))
        ref = oracle.reduce_samples(oracle.sweep(L, bw.a[sl], bw.b[sl], bw.N, bw.S, bw.seed), bw.N, bw.S)
        assert abs(out[p, 0] - ref["logP"]) < 1e-10


def test_tuned_dense_matches_oracle():
    w = workloads.make_workload("dense400")
    kern = (w.sigma2, w.beta, w.nu, w.nugget)
    res = autotune.tune_dense(w.n, w.locs, kern, w.a, w.b, N=2000, S=2, seed=w.seed, tiles=(64, 128, 256))
    print(res, flush=True)
    assert res["tile"] in (64, 128, 256) and res["sweep_rows"] in (64, 128)
    o = mvn.options(tile=res["tile"], sweep_rows=res["sweep_rows"])
    f = mvn.mvn_cholesky(w.n, locs=w.locs, kern=kern, opts=o)
    r = mvn.mvn_prob(f, w.a, w.b, N=2000, S=2, seed=w.seed, opts=o)
    torch.cuda.synchronize()
    L = oracle.cholesky(oracle.covariance(w.locs, *kern))
    at, bt = oracle.centre(w.a, w.b)
    ref = oracle.reduce_samples(oracle.sweep(L, at, bt, 2000, 2, w.seed), 2000, 2)
    assert abs(r["logP"].item() - ref["logP"]) < 1e-10
