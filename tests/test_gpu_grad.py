"""Adjoint sweep (d log P-hat / d a, b, mu at fixed QMC points) against the
oracle's forward-mode (tangent) sweep on identical points, against central
finite differences of the GPU forward sweep (h = 1e-5, the 1e-5 relative
bar), and its exact invariants."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import grad as ograd
import paper_2405_14892_amd as mvn
import workloads

pytestmark = pytest.mark.gpu


def _case(n, seed=0, nu=1.5, inf_lower=False):
    w = workloads.make_workload("grad4096")
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(w.n, size=n, replace=False))
    a, b, mu = w.a[idx].copy(), w.b[idx].copy(), w.mu[idx].copy()
    if inf_lower:
        a[::3] = -np.inf
    return w.locs[idx], a, b, mu, (w.sigma2, w.beta, nu, w.nugget), w.seed


def test_full_gradient_matches_oracle_tangent_sweeps():
    locs, a, b, mu, kern, seed = _case(12)
    N, S = 400, 2
    f = mvn.mvn_cholesky(12, locs=locs, kern=kern, opts=mvn.options(tile=16))
    r = mvn.mvn_prob_grad(f, a, b, mu, N=N, S=S, seed=seed)
    torch.cuda.synchronize()
    L = oracle.cholesky(oracle.covariance(locs, *kern))
    at, bt = oracle.centre(a, b, mu)
    ga, gb = ograd.gradient_full(L, at, bt, N, S, seed)
    np.testing.assert_allclose(r["da"].cpu().numpy(), ga, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(r["db"].cpu().numpy(), gb, rtol=1e-9, atol=1e-12)
    np.testing.assert_array_equal(r["dmu"].cpu().numpy(), -(r["da"] + r["db"]).cpu().numpy())
    ref_logp = oracle.reduce_samples(oracle.sweep(L, at, bt, N, S, seed), N, S)["logP"]
    assert abs(r["logP"].item() - ref_logp) < 1e-10


@pytest.mark.parametrize("n,inf_lower", [(300, False), (300, True)])
def test_directional_derivatives_match_oracle(n, inf_lower):
    """Ragged n = 300 (3 blocks), ragged sample count (700 x 2)."""
    locs, a, b, mu, kern, seed = _case(n, seed=1, inf_lower=inf_lower)
    N, S = 700, 2
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=mvn.options(tile=64))
    r = mvn.mvn_prob_grad(f, a, b, mu, N=N, S=S, seed=seed)
    torch.cuda.synchronize()
    da, db = r["da"].cpu().numpy(), r["db"].cpu().numpy()
    if inf_lower:
        assert np.all(da[np.isinf(a)] == 0.0)
    L = oracle.cholesky(oracle.covariance(locs, *kern))
    at, bt = oracle.centre(a, b, mu)
    rng = np.random.default_rng(5)
    for _ in range(3):
        va, vb = rng.standard_normal(n), rng.standard_normal(n)
        va[np.isinf(a)] = 0.0
        _, ref = ograd.logp_directional(L, at, bt, va, vb, N, S, seed)
        got = float(da @ va + db @ vb)
        assert got == pytest.approx(ref, rel=1e-8, abs=1e-10)


def test_gradient_workload_against_finite_differences():
    """The n = 4096 differentiation workload (finite a = mu - 3, b = mu + u,
    N = 10000, one shift): adjoint vs central differences of the FP64 GPU
    forward sweep along random directions, h = 1e-5."""
    w = workloads.make_workload("grad4096")
    kern = (w.sigma2, w.beta, w.nu, w.nugget)
    f = mvn.mvn_cholesky(w.n, locs=w.locs, kern=kern, opts=mvn.options(tile=256))
    r = mvn.mvn_prob_grad(f, w.a, w.b, w.mu, N=w.N, S=w.S, seed=w.seed)
    torch.cuda.synchronize()
    g = torch.cat([r["da"], r["db"]]).cpu().numpy()
    rng = np.random.default_rng(11)
    h = 1e-5
    for _ in range(3):
        v = rng.standard_normal(2 * w.n)
        v /= np.linalg.norm(v)
        lp = []
        for sgn in (1, -1):
            rr = mvn.mvn_prob(f, w.a + sgn * h * v[:w.n], w.b + sgn * h * v[w.n:], w.mu, N=w.N, S=w.S,
                              seed=w.seed)
            torch.cuda.synchronize()
            lp.append(rr["logP"].item())
        fd = (lp[0] - lp[1]) / (2 * h)
        assert float(g @ v) == pytest.approx(fd, rel=1e-5), (float(g @ v), fd)
    # the forward value agrees with mvn_prob on the same points
    rr = mvn.mvn_prob(f, w.a, w.b, w.mu, N=w.N, S=w.S, seed=w.seed)
    torch.cuda.synchronize()
    assert abs(rr["logP"].item() - r["logP"].item()) < 1e-12


def test_autograd_function_backward():
    locs, a, b, mu, kern, seed = _case(40, seed=3)
    f = mvn.mvn_cholesky(40, locs=locs, kern=kern, opts=mvn.options(tile=16))
    ta = torch.tensor(a, dtype=torch.float64, device="cuda", requires_grad=True)
    tb = torch.tensor(b, dtype=torch.float64, device="cuda", requires_grad=True)
    tm = torch.tensor(mu, dtype=torch.float64, device="cuda", requires_grad=True)
    lp = mvn.MVNLogProb.apply(ta, tb, tm, f, 300, 2, seed)
    (2.0 * lp).backward()
    r = mvn.mvn_prob_grad(f, a, b, mu, N=300, S=2, seed=seed)
    torch.cuda.synchronize()
    assert torch.allclose(ta.grad, 2.0 * r["da"]) and torch.allclose(tb.grad, 2.0 * r["db"])
    assert torch.allclose(tm.grad, 2.0 * r["dmu"])
    assert abs(lp.item() - r["logP"].item()) == 0.0


@pytest.mark.parametrize("n", [3, 4, 6, 8])
def test_gradient_against_closed_form_dP_db_small_n(n):
    """The differentiation workload's first n sites (a = mu - 3, b = mu + u):
    dP/db_i = P-hat * d log P-hat / d b_i from the adjoint sweep against the
    closed form phi((b_i - mu_i)/sigma_i)/sigma_i * P(conditional box), the
    conditional probability by exact quadrature at n = 3 and SciPy's
    Genz-Bretz integration above, within the QMC error; and every d/db_i
    against a central finite difference of the GPU's own log P-hat
    (h = 1e-5), 1e-5 relative."""
    from gradref import dP_db
    w = workloads.make_workload("grad4096")
    idx = np.arange(n)
    locs, a, b, mu = w.locs[idx], w.a[idx].copy(), w.b[idx].copy(), w.mu[idx].copy()
    kern = (w.sigma2, w.beta, w.nu, w.nugget)
    sig = oracle.covariance(locs, *kern)
    N, S, seed = 20000, 10, w.seed
    print(f"closed form n={n}", flush=True)
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=mvn.options(tile=16))
    r = mvn.mvn_prob_grad(f, a, b, mu, N=N, S=S, seed=seed)
    torch.cuda.synchronize()
    P = r["P"].item()
    gb = r["db"].cpu().numpy()
    for i in range(n):
        exact = dP_db(sig, mu, a, b, i)
        got = P * gb[i]
        print(f"  i={i}: GPU {got:.8e} closed form {exact:.8e}", flush=True)
        # the QMC error of the derivative at N S = 200 000 (from the oracle on
        # the same points: at most 0.7% relative or 5e-5 absolute where the
        # conditional box probability is tiny)
        assert abs(got - exact) <= 1e-2 * abs(exact) + 2e-4, (i, got, exact)

    def logp(bb):
        q = mvn.mvn_prob(f, a, bb, mu, N=N, S=S, seed=seed)
        torch.cuda.synchronize()
        return q["logP"].item()
    h = 1e-5
    for i in range(n):
        e = np.zeros(n)
        e[i] = h
        fd = (logp(b + e) - logp(b - e)) / (2 * h)
        assert gb[i] == pytest.approx(fd, rel=1e-5, abs=1e-9)


@pytest.mark.parametrize("prec,bound", [(mvn.MVN_FP32, 1e-4), (mvn.MVN_BF16X3, 1e-3), (mvn.MVN_BF16, 0.3)])
def test_mixed_precision_adjoint_error_statement(prec, bound):
    """The adjoint with the forward GEMM in a reduced type (factor in FP64,
    the type's operand copy for the sweep; reverse GEMM and conditioning in
    FP64): log P-hat and the directional derivative along random directions
    against the oracle's FP64 tangent sweep on identical points.  The bars
    state the error of each type (relative, measured well below them); they
    are not parity."""
    locs, a, b, mu, kern, seed = _case(300, seed=3)
    n, N, S = 300, 800, 2
    o = mvn.options(tile=64, precision=prec, chol_mode=mvn.MVN_CHOL_FP64)
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=o)
    r = mvn.mvn_prob_grad(f, a, b, mu, N=N, S=S, seed=seed, opts=o)
    torch.cuda.synchronize()
    L = oracle.cholesky(oracle.covariance(locs, *kern))
    at, bt = oracle.centre(a, b, mu)
    rng = np.random.default_rng(8)
    da, db = r["da"].cpu().numpy(), r["db"].cpu().numpy()
    for _ in range(2):
        va, vb = rng.standard_normal(n), rng.standard_normal(n)
        logp, dd = ograd.logp_directional(L, at, bt, va, vb, N, S, seed)
        got = float(da @ va + db @ vb)
        rel = abs(got - dd) / abs(dd)
        print(f"precision {prec}: log P {r['logP'].item():.10f} (oracle {logp:.10f}), directional {got:.8e} "
              f"(oracle {dd:.8e}), rel {rel:.2e}", flush=True)
        assert rel < bound
        assert abs(r["logP"].item() - logp) < bound * abs(logp)
