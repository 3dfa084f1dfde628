"""The narrow FP64 sweep (sweep_rows = 32; the automatic choice for N*S <=
20480 with N*S*n <= 9e7, 4.5e7 above 12288 samples): 16 or 32 sample columns per workgroup, 32-row blocks, the next block's
limit-update GEMM overlapped with the recurrence.  Per-sample log-products
against the oracle's sweep on identical QMC points (1e-9 absolute, as for the
other sweeps), nested-set probabilities against the oracle's running
products (1e-10 relative), ragged row blocks and column chunks, several
chunks per workgroup, both column widths, and sampled columns at the
4096-site gradient workload's full size."""
import numpy as np
import pytest
import torch

import oracle
import paper_2405_14892_amd as mvn
import workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _sub(n):
    w = workloads.make_workload("grad4096")
    idx = np.arange(n)
    return w, w.locs[idx], (w.sigma2, w.beta, w.nu, w.nugget), w.a[idx], w.b[idx], w.mu[idx]


@pytest.mark.parametrize("n,N,S,per", [(1, 40, 1, False), (31, 700, 3, False), (32, 1000, 2, True),
                                       (33, 333, 5, False), (257, 5000, 4, False), (400, 1003, 3, True)])
def test_narrow_per_sample_parity(n, N, S, per):
    """16-column chunks: one-row, one-block, exactly one block, a one-row last
    block; N*S = 20000 gives 1250 chunks for 768 workgroups (two passes)."""
    print(f"narrow n={n} N={N} S={S} periodize={per}", flush=True)
    w, locs, kern, a, b, mu = _sub(n)
    opts = mvn.options(tile=64, sweep_rows=32, periodize=per)
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=mvn.options(tile=64), device=DEV)
    r = mvn.mvn_prob(f, a, b, mu, N=N, S=S, seed=w.seed, opts=opts, return_ell=True)
    torch.cuda.synchronize()
    L = oracle.cholesky(oracle.covariance(locs, *kern))
    at, bt = oracle.centre(a, b, mu)
    ell_ref = oracle.sweep(L, at, bt, N, S, w.seed, periodize=per)
    ell = r["ell"].cpu().numpy()
    err = np.max(np.abs(ell - ell_ref))
    print(f"max |dl| {err:.2e}", flush=True)
    assert err < 1e-9
    ref = oracle.reduce_samples(ell_ref, N, S)
    assert abs(r["logP"].item() - ref["logP"]) < 1e-10


def test_narrow_32_columns_sampled():
    """N*S = 24003 > 20480 samples: 32-column chunks (751 for 512 workgroups,
    the last one ragged), n = 300; sampled columns of every chunk."""
    n, N, S = 300, 8001, 3
    print(f"narrow-32 n={n} N={N} S={S}", flush=True)
    w, locs, kern, a, b, mu = _sub(n)
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=mvn.options(tile=64), device=DEV)
    r = mvn.mvn_prob(f, a, b, mu, N=N, S=S, seed=w.seed, opts=mvn.options(tile=64, sweep_rows=32),
                     return_ell=True)
    torch.cuda.synchronize()
    L = oracle.cholesky(oracle.covariance(locs, *kern))
    at, bt = oracle.centre(a, b, mu)
    NS = N * S
    cols = np.unique(np.concatenate([np.arange(0, NS, 11), np.arange(NS - 40, NS)]))
    ell_ref = oracle.sweep(L, at, bt, N, S, w.seed, cols=cols)
    ell = r["ell"].cpu().numpy()
    assert np.max(np.abs(ell[cols] - ell_ref)) < 1e-9
    assert np.all(np.isfinite(ell))


@pytest.mark.parametrize("n,N,S", [(333, 100, 3), (70, 64, 1), (300, 7000, 3)])
def test_narrow_prefix_matches_oracle(n, N, S):
    """Every nested-set probability from the narrow sweep: chunks of 16 (32
    for N*S = 21000) straddle the shift boundaries when N = 100."""
    print(f"narrow prefix n={n} N={N} S={S}", flush=True)
    rng = np.random.default_rng(31 + n)
    locs = workloads.grid_locations(20)[:n]
    kern = (1.0, 0.1, 0.5, 1e-8)
    mu = workloads.gp_draw_grid(20, 1.0, 0.1, 0.5, 1e-8, rng)[0][:n]
    a, b = np.full(n, -np.inf), -mu
    opts = mvn.options(tile=128, sweep_rows=32)
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=mvn.options(tile=128), device=DEV)
    seed = 1234
    r = mvn.mvn_prob_prefix(f, a, b, None, N=N, S=S, seed=seed, opts=opts)
    full = mvn.mvn_prob(f, a, b, None, N=N, S=S, seed=seed, opts=opts)
    torch.cuda.synchronize()
    logp = r["logP"].cpu().numpy()
    L = oracle.cholesky(oracle.covariance(locs, *kern))
    at, bt = oracle.centre(a, b)
    ref = oracle.prefix_probs(L, at, bt, N, S, seed)
    err = np.abs(logp - ref["logP"]) / np.maximum(1.0, np.abs(ref["logP"]))
    print(f"max rel err {err.max():.3e}", flush=True)
    assert err.max() < 1e-10
    if S > 1:
        np.testing.assert_allclose(r["rel_stderr"].cpu().numpy(), ref["rel_stderr"], rtol=1e-8, atol=1e-14)
    assert abs(logp[-1] - full["logP"].item()) < 1e-12 * max(1.0, abs(logp[-1]))


def test_narrow_is_the_automatic_choice_and_full_size_sampled():
    """The 4096-site gradient workload (N*S = 10^4): the automatic choice and
    sweep_rows = 32 give bit-identical per-sample values (the same kernel),
    sampled columns match the oracle, and a 64-column sweep agrees in log P."""
    w = workloads.make_workload("grad4096")
    print(f"narrow full size n={w.n} N={w.N} S={w.S}", flush=True)
    kern = (w.sigma2, w.beta, w.nu, w.nugget)
    f = mvn.mvn_cholesky(w.n, locs=w.locs, kern=kern, opts=mvn.options(tile=w.tile), device=DEV)
    r0 = mvn.mvn_prob(f, w.a, w.b, w.mu, N=w.N, S=w.S, seed=w.seed, opts=mvn.options(tile=w.tile),
                      return_ell=True)
    r32 = mvn.mvn_prob(f, w.a, w.b, w.mu, N=w.N, S=w.S, seed=w.seed,
                       opts=mvn.options(tile=w.tile, sweep_rows=32), return_ell=True)
    r128 = mvn.mvn_prob(f, w.a, w.b, w.mu, N=w.N, S=w.S, seed=w.seed,
                        opts=mvn.options(tile=w.tile, sweep_rows=128), return_ell=True)
    torch.cuda.synchronize()
    assert torch.equal(r0["ell"], r32["ell"])
    ell = r0["ell"].cpu().numpy()
    L = oracle.cholesky(oracle.covariance(w.locs, *kern))
    at, bt = oracle.centre(w.a, w.b, w.mu)
    NS = w.N * w.S
    cols = np.unique(np.concatenate([np.arange(0, NS, 211), np.arange(NS - 20, NS)]))
    ell_ref = oracle.sweep(L, at, bt, w.N, w.S, w.seed, cols=cols)
    assert np.max(np.abs(ell[cols] - ell_ref)) < 1e-9
    assert np.max(np.abs(ell - r128["ell"].cpu().numpy())) < 1e-9
    assert abs(r0["logP"].item() - r128["logP"].item()) < 1e-10


def test_narrow_rejections():
    """sweep_rows = 32 is the FP64 dense sweep only."""
    n = 100
    w, locs, kern, a, b, mu = _sub(n)
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=mvn.options(tile=64, precision=mvn.MVN_FP32), device=DEV)
    with pytest.raises(mvn.MvnError):
        mvn.mvn_prob(f, a, b, mu, N=64, S=1, seed=1, opts=mvn.options(tile=64, precision=mvn.MVN_FP32,
                                                                    sweep_rows=32))
    ft = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=mvn.options(tile=128, tlr_eps=1e-6, max_rank=32),
                          device=DEV)
    with pytest.raises(mvn.MvnError):
        mvn.mvn_prob(ft, a, b, mu, N=64, S=1, seed=1, opts=mvn.options(tile=128, sweep_rows=32))


def test_narrow_graph_capture_replays_match_eager():
    """The narrow sweep and its nested-set form enqueue no allocation, copy
    of device data to the host or fill: captured in a graph, every replay (with
    eager work in between) equals the eager result bit for bit."""
    n, N, S = 300, 700, 3
    w, locs, kern, a, b, mu = _sub(n)
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=mvn.options(tile=64), device=DEV)
    opts = mvn.options(tile=64, sweep_rows=32)
    ta, tb, tm = (torch.as_tensor(x, device=DEV) for x in (a, b, mu))
    wsb = mvn.mvn_prob_workspace_bytes(n, N, S, opts)
    ws = torch.empty(wsb, dtype=torch.uint8, device=DEV)
    r = mvn.mvn_prob(f, ta, tb, tm, N=N, S=S, seed=5, opts=opts, workspace=ws)
    p = mvn.mvn_prob_prefix(f, ta, tb, tm, N=N, S=S, seed=5, opts=opts)
    torch.cuda.synchronize()
    eager, eager_p = r["out"].clone(), p["out"].clone()
    assert torch.isfinite(eager[0])
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            rg = mvn.mvn_prob(f, ta, tb, tm, N=N, S=S, seed=5, opts=opts, workspace=ws)
            pg = mvn.mvn_prob_prefix(f, ta, tb, tm, N=N, S=S, seed=5, opts=opts)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        rg["out"].fill_(0.0)
        pg["out"].fill_(0.0)
        junk = torch.randn(1 << 20, device=DEV).sum()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(rg["out"], eager), rep
        assert torch.equal(pg["out"], eager_p), rep
        del junk


@pytest.mark.parametrize("n,N,S,narrow", [(6144, 1000, 10, True), (9216, 1000, 10, False),
                                          (2048, 2000, 10, True), (4096, 2000, 10, False)])
def test_narrow_automatic_choice_bounds(n, N, S, narrow):
    """The automatic choice takes the narrow sweep up to N*S*n = 9e7 with
    16-column chunks (N*S <= 12 288) and 4.5e7 with 32-column ones: each case
    equals, bit for bit, the sweep it should pick (sweep_rows = 32 for the
    narrow one, 128 for the 64-column one), and the two agree to 1e-9."""
    print(f"narrow auto n={n} N={N} S={S} narrow={narrow}", flush=True)
    k = int(np.ceil(np.sqrt(n)))
    locs = workloads.grid_locations(k)[:n]
    kern = (1.0, 0.1, 0.5, 1e-8)
    rng = np.random.default_rng(5)
    a, b = np.full(n, -np.inf), rng.normal(0.5, 1.0, n)
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=mvn.options(tile=256), device=DEV)
    r = {rows: mvn.mvn_prob(f, a, b, None, N=N, S=S, seed=9, opts=mvn.options(tile=256, sweep_rows=rows),
                            return_ell=True)["ell"] for rows in (0, 32, 128)}
    torch.cuda.synchronize()
    assert torch.equal(r[0], r[32] if narrow else r[128])
    assert torch.max(torch.abs(r[32] - r[128])).item() < 1e-9
