"""Batched uneven problems (nested confidence-region sets) through
mvn_batch_plan / mvn_prob_batch: every problem of the batch against the
oracle on its own points, mixed precision within 1e-4 where P = O(1), and
replays of a captured graph against the eager result."""
import numpy as np
import pytest
import torch

import oracle
import paper_2405_14892_amd as mvn
import workloads

pytestmark = pytest.mark.gpu


def _oracle(bw, sizes, idx, a, b, off, N, S):
    kern = (bw.sigma2, bw.beta, bw.nu, bw.nugget)
    out = []
    for p in range(len(sizes)):
        sl = slice(off[p], off[p + 1])
        L = oracle.cholesky(oracle.covariance(bw.locs[idx[sl]], *kern))
        out.append(oracle.reduce_samples(oracle.sweep(L, a[sl], b[sl], N, S, bw.seed), N, S))
    return out


SIZES = [1, 7, 300, 50, 129, 257, 5, 64, 200, 130]


@pytest.mark.parametrize("rows", [128, 64])
def test_batch_fp64_matches_oracle_per_problem(rows):
    """Both sweep shapes (128- and 64-row blocks) on ragged sizes."""
    # n_max of the generator must reach the largest requested size
    bw = workloads.make_batch(count=len(SIZES), n_min=300, n_max=301, seed=7, N=400, S=3)
    sizes = np.array(SIZES, dtype=np.int32)
    off = np.zeros(len(SIZES) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    idx = np.concatenate([bw.idx[bw.off[p]:bw.off[p] + n] for p, n in enumerate(SIZES)])
    a = np.concatenate([bw.a[bw.off[p]:bw.off[p] + n] for p, n in enumerate(SIZES)])
    b = np.concatenate([bw.b[bw.off[p]:bw.off[p] + n] for p, n in enumerate(SIZES)])
    N, S = 400, 3
    plan = mvn.mvn_batch_plan(sizes, N, S, opts=mvn.options(tile=128, sweep_rows=rows))
    out = mvn.mvn_prob_batch(plan, idx, bw.locs, (bw.sigma2, bw.beta, bw.nu, bw.nugget), a, b, seed=bw.seed)
    torch.cuda.synchronize()
    assert torch.all(plan.info == 0)
    got = out.cpu().numpy()
    ref = _oracle(bw, sizes, idx, a, b, off, N, S)
    for p in range(len(SIZES)):
        assert abs(got[p, 0] - ref[p]["logP"]) < 1e-10, (p, SIZES[p], got[p, 0], ref[p]["logP"])
        np.testing.assert_allclose(got[p, 4:], ref[p]["logP_s"], rtol=0, atol=1e-10)


@pytest.mark.parametrize("prec,rows", [(mvn.MVN_FP32, 128), (mvn.MVN_BF16X3, 128), (mvn.MVN_FP32, 64),
                                       (mvn.MVN_BF16X3, 64)])
def test_batch_mixed_precision_within_1e4(prec, rows):
    bw = workloads.make_batch(count=8, n_min=100, n_max=600, seed=5, positive_excursion=True, N=800, S=4)
    N, S = 800, 4
    plan = mvn.mvn_batch_plan(bw.n_p, N, S, opts=mvn.options(tile=128, precision=prec, sweep_rows=rows))
    out = mvn.mvn_prob_batch(plan, bw.idx, bw.locs, (bw.sigma2, bw.beta, bw.nu, bw.nugget), bw.a, bw.b,
                             seed=bw.seed)
    torch.cuda.synchronize()
    assert torch.all(plan.info == 0)
    got = out.cpu().numpy()
    ref = _oracle(bw, bw.n_p, bw.idx, bw.a, bw.b, bw.off, N, S)
    for p in range(len(bw.n_p)):
        assert abs(got[p, 1] - ref[p]["P"]) <= 1e-4, (p, got[p, 1], ref[p]["P"])


@pytest.mark.parametrize("rows", [128, 64])
def test_batch_plain_bf16_error_statement(rows):
    """Plain BF16 GEMMs (8 significant bits) do not meet 1e-4 on every
    problem of this batch (|dP| reached 1.5e-4 at P = 0.40); the stated
    error bar for MVN_BF16 is 1e-3 absolute, and the split form MVN_BF16X3
    is the BF16 mode that meets 1e-4."""
    bw = workloads.make_batch(count=8, n_min=100, n_max=600, seed=5, positive_excursion=True, N=800, S=4)
    N, S = 800, 4
    plan = mvn.mvn_batch_plan(bw.n_p, N, S, opts=mvn.options(tile=128, precision=mvn.MVN_BF16, sweep_rows=rows))
    out = mvn.mvn_prob_batch(plan, bw.idx, bw.locs, (bw.sigma2, bw.beta, bw.nu, bw.nugget), bw.a, bw.b,
                             seed=bw.seed)
    torch.cuda.synchronize()
    assert torch.all(plan.info == 0)
    got = out.cpu().numpy()
    ref = _oracle(bw, bw.n_p, bw.idx, bw.a, bw.b, bw.off, N, S)
    err = [abs(got[p, 1] - ref[p]["P"]) for p in range(len(bw.n_p))]
    print(f"rows={rows} BF16 max |dP| = {max(err):.3g}")
    assert max(err) <= 1e-3, err


def test_batch_graph_capture_replays_match_eager():
    bw = workloads.make_batch(count=20, n_min=20, n_max=400, seed=9, N=300, S=2)
    N, S = 300, 2
    kern = (bw.sigma2, bw.beta, bw.nu, bw.nugget)
    plan = mvn.mvn_batch_plan(bw.n_p, N, S)
    idx = torch.as_tensor(bw.idx, device="cuda")
    locs = torch.as_tensor(bw.locs, device="cuda")
    a = torch.as_tensor(bw.a, device="cuda")
    b = torch.as_tensor(bw.b, device="cuda")
    mvn.mvn_prob_batch(plan, idx, locs, kern, a, b, seed=bw.seed)
    torch.cuda.synchronize()
    eager = plan.out.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            mvn.mvn_prob_batch(plan, idx, locs, kern, a, b, seed=bw.seed)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        plan.out.fill_(0.0)
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(plan.out, eager), rep
        del junk


def test_batch_more_size_groups_than_one_launch_holds():
    """34 distinct padded sizes (128 ... 4352): the batched Cholesky steps
    split their compact grids over two launches; the smallest problems (in the
    second launch) and the largest ones match the oracle."""
    sizes = np.array([128 * k - 5 for k in range(1, 35)], dtype=np.int32)
    rng = np.random.default_rng(21)
    k = 70
    locs = workloads.grid_locations(k)
    idx = np.concatenate([rng.choice(k * k, size=n, replace=False) for n in sizes]).astype(np.int64)
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    a = np.full(off[-1], -np.inf)
    b = rng.normal(0.5, 1.0, off[-1])
    kern = (1.0, 0.1, 0.5, 1e-4)
    N, S, seed = 64, 2, 99
    plan = mvn.mvn_batch_plan(sizes, N, S, opts=mvn.options(tile=128, sweep_rows=64))
    out = mvn.mvn_prob_batch(plan, idx, locs, kern, a, b, seed=seed)
    torch.cuda.synchronize()
    assert torch.all(plan.info == 0)
    got = out.cpu().numpy()
    for p in (0, 1, 2, 32, 33):
        sl = slice(off[p], off[p + 1])
        L = oracle.cholesky(oracle.covariance(locs[idx[sl]], *kern))
        ref = oracle.reduce_samples(oracle.sweep(L, a[sl], b[sl], N, S, seed), N, S)
        print(p, sizes[p], got[p, 0], ref["logP"], flush=True)
        assert abs(got[p, 0] - ref["logP"]) < 1e-9 * max(1.0, abs(ref["logP"]))
