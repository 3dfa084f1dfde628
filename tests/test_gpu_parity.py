"""GPU parity of the FP64 HIP path against the CPU oracle, through the C ABI.

Tolerances: the factor entries are O(1) and agree to 1e-12 absolute (rounding
order only); log P-hat agrees to 1e-10 absolute (= 1e-10 relative in
P-hat); per-sample log-products agree to 1e-9 absolute (they are sums of up
to n terms of size O(1..100), each carrying rounding-order differences)."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2405_14892_amd as mvn
import workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _matern_case(n, seed, nu=0.5, beta=0.2, nugget=1e-8):
    rng = np.random.default_rng(seed)
    locs = rng.uniform(size=(n, 2))
    return locs, (1.0, beta, nu, nugget)


@pytest.mark.parametrize("n,tile", [(1, 16), (37, 16), (300, 64), (400, 100), (520, 128), (1000, 256),
                                    (1100, 512)])
def test_cholesky_from_locations_matches_oracle(n, tile):
    print(f"cholesky n={n} tile={tile}", flush=True)
    locs, kern = _matern_case(n, n, nu=1.5 if n % 2 else 0.5)
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=mvn.options(tile=tile), device=DEV)
    torch.cuda.synchronize()
    assert f.info() == 0
    L = f.L().cpu().numpy()
    ref = oracle.cholesky(oracle.covariance(locs, *kern))
    assert np.max(np.abs(L - ref)) < 1e-12
    assert np.all(np.triu(L, 1) == 0)


def test_cholesky_many_tile_columns_matches_oracle():
    """4500 sites, tile 128: 36 tile columns, so 34 side-stream trailing
    updates (595 tiles in the first) overlap the sub-panel chains."""
    n, tile = 4500, 128
    print(f"cholesky n={n} tile={tile}", flush=True)
    locs, kern = _matern_case(n, 7, nu=0.5, beta=0.1, nugget=1e-4)
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=mvn.options(tile=tile), device=DEV)
    torch.cuda.synchronize()
    assert f.info() == 0
    L = f.L().cpu().numpy()
    ref = oracle.cholesky(oracle.covariance(locs, *kern))
    assert np.max(np.abs(L - ref)) < 1e-12
    assert np.all(np.triu(L, 1) == 0)


def test_cholesky_from_sigma_and_not_spd():
    rng = np.random.default_rng(3)
    m = rng.standard_normal((300, 300))
    s = m @ m.T + 300 * np.eye(300)
    f = mvn.mvn_cholesky(300, sigma=s, opts=mvn.options(tile=64), device=DEV)
    torch.cuda.synchronize()
    assert f.info() == 0
    assert np.max(np.abs(f.L().cpu().numpy() - oracle.cholesky(s))) < 1e-12
    bad = s.copy()
    bad[41, 41] = -1.0
    f = mvn.mvn_cholesky(300, sigma=bad, opts=mvn.options(tile=64), device=DEV)
    torch.cuda.synchronize()
    assert f.info() == 42
    # the probability call propagates the failure as NaN
    r = mvn.mvn_prob(f, np.full(300, -np.inf), np.zeros(300), N=64, S=2, seed=1)
    assert torch.isnan(r["out"]).all()


def _prob_case(w, N, S, tile=None, rows=0):
    f = mvn.mvn_cholesky(w.n, locs=w.locs, kern=(w.sigma2, w.beta, w.nu, w.nugget),
                         opts=mvn.options(tile=tile or w.tile), device=DEV)
    r = mvn.mvn_prob(f, w.a, w.b, w.mu, N=N, S=S, seed=w.seed, return_ell=True,
                     opts=mvn.options(tile=tile or w.tile, sweep_rows=rows))
    torch.cuda.synchronize()
    L = oracle.cholesky(oracle.covariance(w.locs, w.sigma2, w.beta, w.nu, w.nugget))
    at, bt = oracle.centre(w.a, w.b, w.mu)
    return f, r, L, at, bt


def test_prob_per_sample_parity_dense400_ragged():
    """n = 400 (ragged against the 128-row blocks), 3 shifts x 2000 points
    (ragged against the 128-column blocks)."""
    w = workloads.make_workload("dense400")
    print("dense400 N=2000 S=3", flush=True)
    f, r, L, at, bt = _prob_case(w, 2000, 3)
    ell_ref = oracle.sweep(L, at, bt, 2000, 3, w.seed)
    ell = r["ell"].cpu().numpy()
    assert np.max(np.abs(ell - ell_ref)) < 1e-9
    ref = oracle.reduce_samples(ell_ref, 2000, 3)
    assert abs(r["logP"].item() - ref["logP"]) < 1e-10
    np.testing.assert_allclose(r["logP_s"].cpu().numpy(), ref["logP_s"], rtol=0, atol=1e-10)
    assert r["rel_stderr"].item() == pytest.approx(ref["rel_stderr"], rel=1e-8)


@pytest.mark.parametrize("rows", [128, 64])
def test_prob_full_dense400_workload(rows):
    """The full n = 400, N = 10000 x S = 10 workload: log P-hat to 1e-10, with
    both sweep shapes (128- and 64-row blocks)."""
    w = workloads.make_workload("dense400")
    print(f"dense400 full rows={rows}", flush=True)
    f, r, L, at, bt = _prob_case(w, w.N, w.S, rows=rows)
    ell_ref = oracle.sweep(L, at, bt, w.N, w.S, w.seed)
    ref = oracle.reduce_samples(ell_ref, w.N, w.S)
    assert abs(r["logP"].item() - ref["logP"]) < 1e-10
    assert np.max(np.abs(r["ell"].cpu().numpy() - ell_ref)) < 1e-9


@pytest.mark.parametrize("n,N,S", [(257, 57341, 2), (300, 33000, 4), (300, 150, 1), (520, 1000, 7)])
def test_prob_wide_sweep_pass_shapes(n, N, S):
    """The FP64 sweeps' column distributions.  With at least 65536 samples
    the 128-column sweep runs: N*S = 114682 gives every workgroup seven
    32-column slices (a 128-column pass, a 64-column pass and a 32-column
    pass, the last slice ragged), 132000 gives 8 or 9; 150 and 7000 samples
    take the 64-column sweep.  n = 257 leaves a one-row last block.  Sampled
    columns of every workgroup against the oracle, 1e-9."""
    w = workloads.make_workload("grad4096")
    idx = np.arange(n)
    locs = w.locs[idx]
    kern = (w.sigma2, w.beta, w.nu, w.nugget)
    print(f"wide sweep n={n} N={N} S={S}", flush=True)
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=mvn.options(tile=64), device=DEV)
    r = mvn.mvn_prob(f, w.a[idx], w.b[idx], w.mu[idx], N=N, S=S, seed=w.seed, opts=mvn.options(tile=64),
                     return_ell=True)
    torch.cuda.synchronize()
    L = oracle.cholesky(oracle.covariance(locs, *kern))
    at, bt = oracle.centre(w.a[idx], w.b[idx], w.mu[idx])
    NS = N * S
    cols = np.unique(np.concatenate([np.arange(0, NS, 13), np.arange(max(0, NS - 70), NS)]))
    ell_ref = oracle.sweep(L, at, bt, N, S, w.seed, cols=cols)
    ell = r["ell"].cpu().numpy()
    assert np.max(np.abs(ell[cols] - ell_ref)) < 1e-9
    assert np.all(np.isfinite(ell))


def test_prob_finite_limits_with_mean_and_periodize():
    """Finite two-sided limits, a mean vector, nu = 3/2, the baker's transform."""
    w = workloads.make_workload("grad4096")
    idx = np.arange(300)
    locs = w.locs[idx]
    f = mvn.mvn_cholesky(300, locs=locs, kern=(w.sigma2, w.beta, w.nu, w.nugget),
                         opts=mvn.options(tile=64), device=DEV)
    for per in (False, True):
        r = mvn.mvn_prob(f, w.a[idx], w.b[idx], w.mu[idx], N=700, S=2, seed=w.seed,
                         opts=mvn.options(tile=64, periodize=per), return_ell=True)
        torch.cuda.synchronize()
        L = oracle.cholesky(oracle.covariance(locs, w.sigma2, w.beta, w.nu, w.nugget))
        at, bt = oracle.centre(w.a[idx], w.b[idx], w.mu[idx])
        ell_ref = oracle.sweep(L, at, bt, 700, 2, w.seed, periodize=per)
        assert np.max(np.abs(r["ell"].cpu().numpy() - ell_ref)) < 1e-9


def test_prob_univariate_and_unbounded_and_degenerate():
    sig = np.array([[2.25]])
    f = mvn.mvn_cholesky(1, sigma=sig, opts=mvn.options(tile=16), device=DEV)
    r = mvn.mvn_prob(f, [-1.0], [2.0], N=300, S=1, seed=4, return_ell=True)
    torch.cuda.synchronize()
    exact = math.log(0.5 * math.erfc(-2.0 / 1.5 / math.sqrt(2)) - 0.5 * math.erfc(1.0 / 1.5 / math.sqrt(2)))
    np.testing.assert_allclose(r["ell"].cpu().numpy(), exact, rtol=0, atol=1e-14)
    assert math.isnan(r["stderr"].item())  # one shift: no spread estimate
    n = 200
    locs, kern = _matern_case(n, 5)
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=mvn.options(tile=32), device=DEV)
    r = mvn.mvn_prob(f, np.full(n, -np.inf), np.full(n, np.inf), N=130, S=2, seed=2, return_ell=True)
    torch.cuda.synchronize()
    assert torch.all(r["ell"] == 0.0) and r["logP"].item() == 0.0
    a = np.full(n, -np.inf)
    b = np.zeros(n)
    a[17] = b[17] = 0.25
    r = mvn.mvn_prob(f, a, b, N=130, S=2, seed=2, return_ell=True)
    torch.cuda.synchronize()
    assert torch.all(r["ell"] == -math.inf) and r["logP"].item() == -math.inf


def test_prob_invalid_limits_give_nan():
    n = 50
    locs, kern = _matern_case(n, 9)
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=mvn.options(tile=16), device=DEV)
    a = np.full(n, -1.0)
    b = np.full(n, 1.0)
    b[3] = -2.0
    r = mvn.mvn_prob(f, a, b, N=64, S=2, seed=1)
    torch.cuda.synchronize()
    assert torch.isnan(r["out"]).all()
    b[3] = float("nan")
    r = mvn.mvn_prob(f, a, b, N=64, S=2, seed=1)
    torch.cuda.synchronize()
    assert torch.isnan(r["out"]).all()


def test_host_validation_rejects_bad_arguments():
    n = 20
    locs, kern = _matern_case(n, 1)
    for bad_nu in (0.0, -1.0, 25.0, float("nan")):
        with pytest.raises(mvn.MvnError) as e:
            mvn.mvn_cholesky(n, locs=locs, kern=(1.0, 0.1, bad_nu, 0.0), device=DEV)
        assert e.value.code == -5
    with pytest.raises(mvn.MvnError):
        mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=mvn.options(tile=10), device=DEV)
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=mvn.options(tile=16), device=DEV)
    # the C entry point itself: N is argument 5, the workspace argument 10
    import ctypes
    from paper_2405_14892_amd import _lib
    a = torch.zeros(n, dtype=torch.float64, device=DEV)
    b = torch.ones(n, dtype=torch.float64, device=DEV)
    out = torch.empty(8, dtype=torch.float64, device=DEV)
    ws = torch.empty(1024, dtype=torch.uint8, device=DEV)
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    h = _lib.lib()
    o = mvn.options(tile=16)
    code = h.mvn_prob(ctypes.byref(f.handle), P(a), P(b), None, 0, 1, 1, ctypes.byref(o), P(ws), 1024,
                      P(out), None, None)
    assert code == -5
    code = h.mvn_prob(ctypes.byref(f.handle), P(a), P(b), None, 64, 1, 1, ctypes.byref(o), P(ws), 1024,
                      P(out), None, None)
    assert code == -10 and b"workspace too small" in h.mvn_last_error()
