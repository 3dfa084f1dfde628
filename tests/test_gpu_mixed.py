"""Mixed-precision paths (FP32, BF16, split BF16 trailing updates and SOV
GEMMs; FP64 conditioning) against the FP64 oracle on identical QMC points.

Bar: |P-hat - P-hat_oracle| <= 1e-4 absolute where P = O(1) (problems of
the confidence-region batch with the positive-excursion limits).  The
per-sample and log-scale errors are recorded in the assertion messages; they
are statements of error, not parity claims (mixed precision is unpinned
against the exact integral)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2405_14892_amd as mvn
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cases():
    bw = workloads.make_batch(count=12, positive_excursion=True)
    out = []
    for p in (3, 8, 10):
        o0, o1 = bw.off[p], bw.off[p + 1]
        idx = bw.idx[o0:o1]
        locs, a, b = bw.locs[idx], bw.a[o0:o1], bw.b[o0:o1]
        kern = (bw.sigma2, bw.beta, bw.nu, bw.nugget)
        L = oracle.cholesky(oracle.covariance(locs, *kern))
        N, S = 2000, 4
        ell = oracle.sweep(L, a, b, N, S, bw.seed)
        out.append((locs, a, b, kern, L, N, S, bw.seed, ell, oracle.reduce_samples(ell, N, S)))
    return out


MODES = [mvn.MVN_CHOL_ADAPTIVE, mvn.MVN_CHOL_UNIFORM, mvn.MVN_CHOL_FP64]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("prec", [mvn.MVN_FP32, mvn.MVN_BF16, mvn.MVN_BF16X3])
def test_mixed_precision_probability_within_1e4(cases, prec, mode):
    for locs, a, b, kern, L, N, S, seed, ell, ref in cases:
        n = len(a)
        print(f"prec {prec} chol_mode {mode} n={n} P={ref['P']:.4g}", flush=True)
        o = mvn.options(tile=64, precision=prec, chol_mode=mode)
        f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=o)
        r = mvn.mvn_prob(f, a, b, None, N=N, S=S, seed=seed, opts=o, return_ell=True)
        torch.cuda.synchronize()
        assert f.info() == 0
        dP = abs(r["P"].item() - ref["P"])
        dlog = abs(r["logP"].item() - ref["logP"])
        dell = float(np.max(np.abs(r["ell"].cpu().numpy() - ell)))
        assert dP <= 1e-4, (prec, n, dP, dlog, dell)
        assert np.isfinite(r["logP"].item())


def test_mixed_factor_keeps_fp64_factor_accuracy_bounds(cases):
    """The FP64 factor that the mixed paths keep for the diagonal blocks and
    pivots: FP32 trailing updates perturb it at the 1e-6 level, split BF16 at
    1e-5, plain BF16 at 1e-2 (measured on these covariances)."""
    locs, a, b, kern, L, *_ = cases[1]
    n = len(a)
    for prec, bound in ((mvn.MVN_FP32, 5e-6), (mvn.MVN_BF16X3, 1e-4), (mvn.MVN_BF16, 3e-2)):
        for mode in MODES:
            f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=mvn.options(tile=64, precision=prec, chol_mode=mode))
            torch.cuda.synchronize()
            assert f.info() == 0
            err = np.max(np.abs(f.L().cpu().numpy() - L))
            print(f"prec {prec} chol_mode {mode}: max |L - L_oracle| {err:.3e}, {f.update_counts()}", flush=True)
            assert err < (1e-10 if mode == mvn.MVN_CHOL_FP64 else bound), (prec, mode)


def test_adaptive_map_picks_reduced_type_for_far_tiles_only():
    """Two clusters of sites far apart (covariance between them about
    1e-304): an update of a tile whose rows lie in the other cluster than the
    panel's has a panel block of norm about 1e-304 and runs in the reduced
    type, while tiles inside the panel's cluster stay FP64 or FP32; the
    cross-cluster block of the factor stays negligible and the factor is
    within 1e-5 of the oracle's."""
    rng = np.random.default_rng(5)
    m = 320
    locs = np.concatenate([rng.uniform(0, 0.2, (m, 2)), rng.uniform(0, 0.2, (m, 2)) + 50.0])
    kern = (1.0, 0.1, 0.5, 1e-6)
    L = oracle.cholesky(oracle.covariance(locs, *kern))
    f = mvn.mvn_cholesky(2 * m, locs=locs, kern=kern,
                         opts=mvn.options(tile=64, precision=mvn.MVN_BF16, chol_mode=mvn.MVN_CHOL_ADAPTIVE))
    torch.cuda.synchronize()
    assert f.info() == 0
    c = f.update_counts()
    print("update counts", c, flush=True)
    assert c["reduced"] > 0 and c["fp64"] > 0
    Lg = f.L().cpu().numpy()
    assert np.max(np.abs(Lg[m:, :m])) < 1e-250
    assert np.max(np.abs(Lg - L)) < 1e-5


def test_fp64_sweep_on_a_mixed_factor_is_rejected_only_for_other_precisions(cases):
    locs, a, b, kern, *_ = cases[0]
    n = len(a)
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=mvn.options(tile=64, precision=mvn.MVN_FP32))
    # an FP64 sweep is always available
    r = mvn.mvn_prob(f, a, b, None, N=256, S=2, seed=1, opts=mvn.options(tile=64))
    torch.cuda.synchronize()
    assert np.isfinite(r["logP"].item())
    with pytest.raises(mvn.MvnError) as e:
        mvn.mvn_prob(f, a, b, None, N=256, S=2, seed=1, opts=mvn.options(tile=64, precision=mvn.MVN_BF16))
    assert e.value.code == -8


@pytest.fixture(scope="module")
def quad_case():
    """260 sites of a 20 x 20 grid (two full 128-row blocks and a 4-row
    one), exponential kernel, P(X <= 2.5 everywhere) = O(1); N x S = 65600 x
    2 = 131200 samples (512.5 chunks of 256: the reduced-precision sweep with
    four conditioning waves, last chunk ragged)."""
    g = np.linspace(0.0, 1.0, 20)
    locs = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)[:260].copy()
    kern = (1.0, 0.1, 0.5, 1e-8)
    n = len(locs)
    a, b = np.full(n, -np.inf), np.full(n, 2.5)
    N, S, seed = 65600, 2, 23
    L = oracle.cholesky(oracle.covariance(locs, *kern))
    ell = oracle.sweep(L, a, b, N, S, seed)
    pref = oracle.prefix_probs(L, a, b, N, S, seed)
    return locs, kern, a, b, N, S, seed, ell, oracle.reduce_samples(ell, N, S), pref


@pytest.mark.parametrize("prec,bound", [(mvn.MVN_FP32, 1e-4), (mvn.MVN_BF16X3, 1e-4), (mvn.MVN_BF16, 3e-3)])
def test_four_wave_sweep_within_bound_full_and_nested(quad_case, prec, bound):
    """The 256-column sweep (128-row blocks, enough samples to fill every
    workgroup slot) against the oracle on the same points: |P - P_oracle|
    within the mixed-precision bar for FP32 and split BF16 (the plain BF16
    error stated), for the full estimate and for every nested set; the last
    nested set equals the full estimate."""
    locs, kern, a, b, N, S, seed, ell, ref, pref = quad_case
    n = len(a)
    o = mvn.options(tile=128, precision=prec, sweep_rows=128)
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=o)
    r = mvn.mvn_prob(f, a, b, None, N=N, S=S, seed=seed, opts=o, return_ell=True)
    p = mvn.mvn_prob_prefix(f, a, b, None, N=N, S=S, seed=seed, opts=o)
    torch.cuda.synchronize()
    assert f.info() == 0
    dP = abs(r["P"].item() - ref["P"])
    dell = float(np.max(np.abs(r["ell"].cpu().numpy() - ell)))
    lp = p["logP"].cpu().numpy()
    dpre = float(np.max(np.abs(np.exp(lp) - np.exp(pref["logP"]))))
    print(f"prec {prec}: P {ref['P']:.4f}, |dP| {dP:.2e}, max |d ell| {dell:.2e}, nested max |dP| {dpre:.2e}",
          flush=True)
    assert dP <= bound and dpre <= bound
    assert abs(lp[-1] - r["logP"].item()) < 1e-12 * max(1.0, abs(lp[-1]))
