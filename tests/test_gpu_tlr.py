"""Tile low-rank (TLR) factorisation and sweep on the GPU, through the C ABI.

Parity: with tlr_eps -> 0 and a rank cap equal to the tile, the TLR factor is
the dense factor up to rounding, so the TLR sweep is checked sample by sample
against the oracle's dense Cholesky + SOV sweep.  At a working accuracy the
result of the compression is not unique (cross approximation and truncated
SVD pick different factors), so the checks are the properties that define
it: every panel tile satisfies ||A_ik - L_ik L_kk^T||_F <= eps on the tile it
was compressed from, its rank is at least the eps-rank of that tile
(Eckart-Young), ||L L^T - Sigma|| stays at the size of the accumulated
truncations, and log P moves by an amount of that order."""
import numpy as np
import pytest
import torch

import oracle
import paper_2405_14892_amd as mvn
import workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _tlr_inputs(k, n, seed=77, beta=0.1, nu=0.5, nugget=1e-8):
    """First n sites of a Morton-ordered k x k grid, a = -inf, b = -(GP draw)."""
    rng = np.random.default_rng(seed)
    perm = workloads.morton_permutation(k)
    locs = workloads.grid_locations(k)[perm][:n]
    field = workloads.gp_draw_grid(k, 1.0, beta, nu, nugget, rng)[0][perm][:n]
    return locs, (1.0, beta, nu, nugget), np.full(n, -np.inf), -field


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


def _factor(n, locs, kern, tile, eps, max_rank):
    f = mvn.mvn_cholesky(n, locs=locs, kern=kern, opts=mvn.options(tile=tile, tlr_eps=eps, max_rank=max_rank),
                         device=DEV)
    torch.cuda.synchronize()
    return f


def _prob(f, a, b, N, S, seed, tile, eps, max_rank, rows=0):
    opts = mvn.options(tile=tile, tlr_eps=eps, max_rank=max_rank, sweep_rows=rows)
    r = mvn.mvn_prob(f, a, b, None, N=N, S=S, seed=seed, opts=opts, return_ell=True)
    torch.cuda.synchronize()
    return r


@pytest.mark.parametrize("n,tile,rows", [(1000, 128, 128), (700, 256, 128), (700, 256, 64), (1000, 128, 256),
                                        (700, 256, 256)])
def test_tlr_exact_limit_matches_dense_oracle(n, tile, rows):
    """eps = 1e-13 with the cap at the tile edge: the factor and every
    sample's log-product agree with the dense oracle (n ragged against the
    tile and the sweep blocks; N*S ragged against the 64-column chunks)."""
    print(f"tlr exact limit n={n} tile={tile} rows={rows}", flush=True)
    locs, kern, a, b = _tlr_inputs(32, n)
    rcap = min(tile, 256)
    f = _factor(n, locs, kern, tile, 1e-13, rcap)
    assert f.info() == 0
    sigma = oracle.covariance(locs, *kern)
    Lref = oracle.cholesky(sigma)
    L = _dense_from_tlr(f)
    assert np.max(np.abs(L - Lref)) < 1e-10
    N, S, seed = 777, 2, 4242
    r = _prob(f, a, b, N, S, seed, tile, 1e-13, rcap, rows)
    at, bt = oracle.centre(a, b)
    ell_ref = oracle.sweep(Lref, at, bt, N, S, seed)
    ell = r["ell"].cpu().numpy()
    assert np.max(np.abs(ell - ell_ref)) < 1e-8
    ref = oracle.reduce_samples(ell_ref, N, S)
    assert abs(r["logP"].item() - ref["logP"]) < 1e-9 * max(1.0, abs(ref["logP"]))


@pytest.mark.parametrize("rows", [128, 64, 256])
def test_tlr_sweep_matches_oracle_on_the_compressed_factor(rows):
    """At a working accuracy (ranks from near zero on far tiles to some tens
    on adjacent ones, a partial last tile of 20 rows), the TLR sweep equals,
    sample by sample, the oracle's sweep through the dense L assembled from
    the same compressed factor: the stacked and packed products change
    nothing but the rounding."""
    n, tile, eps, rcap = 1300, 128, 1e-5, 128
    print(f"tlr sweep on compressed factor rows={rows}", flush=True)
    locs, kern, a, b = _tlr_inputs(40, n, seed=81, beta=0.05)
    f = _factor(n, locs, kern, tile, eps, rcap)
    assert f.info() == 0
    ranks = f.ranks().cpu().numpy()
    assert ranks.max() > 16 and len(set(ranks.tolist())) > 5, ranks
    L = _dense_from_tlr(f)
    N, S, seed = 300, 3, 515
    r = _prob(f, a, b, N, S, seed, tile, eps, rcap, rows)
    at, bt = oracle.centre(a, b)
    ell_ref = oracle.sweep(L, at, bt, N, S, seed)
    ell = r["ell"].cpu().numpy()
    assert np.max(np.abs(ell - ell_ref)) < 1e-8


def test_tlr_tile_accuracy_ranks_and_probability():
    """eps = 1e-6, tile 256, n = 1024: per-tile residual <= eps, ranks >= the
    SVD eps-rank of the compressed tile, ||L L^T - Sigma||_max small, log P
    within 1e-4 of the dense oracle's on the same QMC points."""
    n, tile, eps, rcap = 1024, 256, 1e-6, 128
    print(f"tlr eps={eps} n={n} tile={tile}", flush=True)
    locs, kern, a, b = _tlr_inputs(32, n, seed=78)
    f = _factor(n, locs, kern, tile, eps, rcap)
    assert f.info() == 0
    tiles = f.tiles().cpu().numpy()
    U, Vt, ranks = f.U().cpu().numpy(), f.Vt().cpu().numpy(), f.ranks().cpu().numpy()
    nt = f.nt
    assert np.all(ranks >= 0) and np.all(ranks <= rcap)
    for i in range(nt):
        for k in range(i):
            p = i * (i - 1) // 2 + k
            A = tiles[i * (i + 1) // 2 + k]            # the tile as it was compressed
            Dk = np.tril(tiles[k * (k + 1) // 2 + k])
            r = ranks[p]
            assert np.all(U[p][:, r:] == 0) and np.all(Vt[p][r:] == 0)
            res = np.linalg.norm(A - (U[p] @ Vt[p]) @ Dk.T)
            assert res <= eps * (1 + 1e-6) + 1e-12, (i, k, res)
            s = np.linalg.svd(A, compute_uv=False)
            assert r >= int(np.sum(s > eps)), (i, k, r)
    sigma = oracle.covariance(locs, *kern)
    L = _dense_from_tlr(f)
    assert np.max(np.abs(L @ L.T - sigma)) < 50 * eps
    N, S, seed = 1000, 2, 99
    r = _prob(f, a, b, N, S, seed, tile, eps, rcap)
    at, bt = oracle.centre(a, b)
    ref = oracle.reduce_samples(oracle.sweep(oracle.cholesky(sigma), at, bt, N, S, seed), N, S)
    assert abs(r["logP"].item() - ref["logP"]) < 1e-4 * max(1.0, abs(ref["logP"]))
    print(f"ranks mean={ranks.mean():.1f} max={ranks.max()} dlogP={r['logP'].item() - ref['logP']:.3e}")


def _frob_eps_rank(A, eps):
    """Smallest k with ||A - A_k||_F <= eps (A_k the truncated SVD): the
    optimal rank for the Frobenius criterion (Eckart-Young)."""
    s = np.linalg.svd(A, compute_uv=False)
    tail = np.sqrt(np.cumsum((s ** 2)[::-1]))[::-1]  # tail[k] = ||s[k:]||
    return int(np.sum(tail > eps))


@pytest.mark.parametrize("n,tile,eps", [(2048, 256, 1e-6), (1536, 128, 1e-5)])
def test_tlr_recompressed_ranks_near_svd_eps_rank(n, tile, eps):
    """After the recompression every panel keeps ||A_ik - U V'^T L_kk^T||_F
    <= eps, no rank is below the tile's Frobenius eps-rank (no rank-k matrix
    does better than the truncated SVD), and the ranks sum to within 10% of
    the eps-ranks' sum."""
    print(f"tlr recompression n={n} tile={tile} eps={eps}", flush=True)
    locs, kern, a, b = _tlr_inputs(64, n, seed=91)
    f = _factor(n, locs, kern, tile, eps, 128)
    assert f.info() == 0
    tiles = f.tiles().cpu().numpy()
    U, Vt, ranks = f.U().cpu().numpy(), f.Vt().cpu().numpy(), f.ranks().cpu().numpy()
    tot_r = tot_opt = 0
    for i in range(f.nt):
        for k in range(i):
            p = i * (i - 1) // 2 + k
            A = tiles[i * (i + 1) // 2 + k]
            Dk = np.tril(tiles[k * (k + 1) // 2 + k])
            r = int(ranks[p])
            assert r >= 0
            assert np.all(U[p][:, r:] == 0) and np.all(Vt[p][r:] == 0)
            res = np.linalg.norm(A - (U[p] @ Vt[p]) @ Dk.T)
            assert res <= eps * (1 + 1e-6) + 1e-12, (i, k, res)
            kopt = _frob_eps_rank(A, eps)
            assert r >= kopt, (i, k, r, kopt)
            tot_r += r
            tot_opt += kopt
    print(f"sum of ranks {tot_r}, of Frobenius eps-ranks {tot_opt}: ratio {tot_r / max(tot_opt, 1):.3f}", flush=True)
    assert tot_r <= 1.10 * tot_opt


def test_tlr_rank_cap_is_flagged():
    """A cap below the eps-rank is reported by a negative rank; with a large
    nugget the truncated matrix stays positive definite."""
    n, tile = 512, 128
    locs, _, a, b = _tlr_inputs(32, n, seed=79)
    kern = (1.0, 0.1, 0.5, 0.5)
    f = _factor(n, locs, kern, tile, 1e-12, 4)
    assert f.info() == 0
    ranks = f.ranks().cpu().numpy()
    assert np.all(np.abs(ranks) <= 4)
    assert np.any(ranks < 0)
    r = _prob(f, a, b, 256, 2, 5, tile, 1e-12, 4)
    assert np.isfinite(r["logP"].item())


def test_tlr_truncation_that_breaks_definiteness_is_reported():
    """Rank 4 on the nearly singular exponential covariance (nugget 1e-8):
    a trailing tile loses positive definiteness; info names a pivot past the
    first tile and the probability is NaN."""
    n, tile = 512, 128
    locs, kern, a, b = _tlr_inputs(32, n, seed=79)
    f = _factor(n, locs, kern, tile, 1e-12, 4)
    assert f.info() > tile
    r = _prob(f, a, b, 256, 2, 5, tile, 1e-12, 4)
    assert torch.isnan(r["out"]).all()


@pytest.mark.parametrize("n", [1, 100, 128])
def test_tlr_single_tile_is_the_dense_factor(n):
    locs, kern, a, b = _tlr_inputs(16, n, seed=80)
    f = _factor(n, locs, kern, 128, 1e-8, 32)
    assert f.info() == 0 and f.nt == 1
    sigma = oracle.covariance(locs, *kern)
    Lref = oracle.cholesky(sigma)
    assert np.max(np.abs(_dense_from_tlr(f) - Lref)) < 1e-12
    N, S, seed = 300, 3, 17
    r = _prob(f, a, b, N, S, seed, 128, 1e-8, 32)
    at, bt = oracle.centre(a, b)
    ell_ref = oracle.sweep(Lref, at, bt, N, S, seed)
    assert np.max(np.abs(r["ell"].cpu().numpy() - ell_ref)) < 1e-9
    ref = oracle.reduce_samples(ell_ref, N, S)
    assert abs(r["logP"].item() - ref["logP"]) < 1e-10 * max(1.0, abs(ref["logP"]))


def test_tlr_not_spd_reports_the_global_pivot():
    n = 400
    s = np.eye(n)
    s[300, 300] = -1.0
    opts = mvn.options(tile=128, tlr_eps=1e-8, max_rank=16)
    f = mvn.mvn_cholesky(n, sigma=s, opts=opts, device=DEV)
    torch.cuda.synchronize()
    assert f.info() == 301
    r = mvn.mvn_prob(f, np.full(n, -np.inf), np.zeros(n), N=64, S=2, seed=1, opts=opts)
    torch.cuda.synchronize()
    assert torch.isnan(r["out"]).all()


def test_tlr_factor_rejected_where_unsupported():
    locs, kern, a, b = _tlr_inputs(16, 200, seed=81)
    f = _factor(200, locs, kern, 128, 1e-8, 32)
    with pytest.raises(mvn.MvnError) as e:
        mvn.mvn_prob_grad(f, a, b, N=64, S=1, seed=1)
    assert e.value.code == -1
    with pytest.raises(mvn.MvnError) as e:
        mvn.mvn_prob(f, a, b, N=64, S=1, seed=1, opts=mvn.options(tile=128, precision=mvn.MVN_FP32))
    assert e.value.code == -8
    with pytest.raises(mvn.MvnError):
        f.L()


@pytest.mark.parametrize("rows", [0, 256])
def test_tlr_sweep_graph_capture_replays_match_eager(rows):
    """A TLR probability call reads nothing back (its index tables and the
    layout of its workspace are built on the device from the ranks), so it can
    be captured in a graph: every replay, with eager work in between, equals
    the eager result bit for bit; a workspace too small for one sweep
    workgroup once the ranks are known gives NaN outputs, not a fault.  Both
    the 64-column form (the automatic choice here) and the four-wave form."""
    print(f"tlr graph capture rows={rows}", flush=True)
    locs, kern, a, b = _tlr_inputs(32, 900)
    f = _factor(900, locs, kern, 256, 1e-5, 64)
    opts = mvn.options(tile=256, tlr_eps=1e-5, max_rank=64, sweep_rows=rows)
    N, S = 500, 3
    wsb = mvn.mvn_prob_workspace_bytes_factor(f, N, S, opts)
    ws = torch.empty(wsb, dtype=torch.uint8, device=DEV)
    ta, tb = torch.as_tensor(a, device=DEV), torch.as_tensor(b, device=DEV)
    r = mvn.mvn_prob(f, ta, tb, None, N=N, S=S, seed=5, opts=opts, workspace=ws)
    torch.cuda.synchronize()
    eager = r["out"].clone()
    assert torch.isfinite(eager[0])
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            rg = mvn.mvn_prob(f, ta, tb, None, N=N, S=S, seed=5, opts=opts, workspace=ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        rg["out"].fill_(0.0)
        junk = torch.randn(1 << 20, device=DEV).sum()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(rg["out"], eager), rep
        del junk
    # one 64-sample chunk needs one workgroup: 4 KiB short of its size for
    # these ranks is accepted on the host (the ranks are not read back) and
    # gives NaN on the device; the exact size gives the probability
    need = mvn.mvn_prob_workspace_bytes_factor(f, 64, 1, opts)
    small = torch.empty(need - 4096, dtype=torch.uint8, device=DEV)
    q = mvn.mvn_prob(f, ta, tb, None, N=64, S=1, seed=5, opts=opts, workspace=small)
    torch.cuda.synchronize()
    assert torch.isnan(q["out"][0])
    exact = torch.empty(need, dtype=torch.uint8, device=DEV)
    q = mvn.mvn_prob(f, ta, tb, None, N=64, S=1, seed=5, opts=opts, workspace=exact)
    torch.cuda.synchronize()
    assert torch.isfinite(q["out"][0])


@pytest.mark.parametrize("n,tile", [(1300, 128), (700, 256)])
def test_tlr_dense_form_and_dense_sweep(n, tile):
    """The TLR factor in dense form (the configuration of Section IV-C: TLR
    factorisation, dense SOV sweep): the written factor equals the one
    assembled on the host from the same tiles, U and V'^T; the dense sweep on
    it equals, sample by sample, the oracle's sweep through that factor; and
    with enough samples for the 128-column FP64 sweep it equals the TLR
    sweep of the same factor (the same products in a different order)."""
    eps, rcap = 1e-5, 128
    print(f"tlr dense form n={n} tile={tile}", flush=True)
    locs, kern, a, b = _tlr_inputs(40, n, seed=83, beta=0.05)
    f = _factor(n, locs, kern, tile, eps, rcap)
    assert f.info() == 0
    d = mvn.mvn_tlr_dense(f)
    torch.cuda.synchronize()
    assert not d.is_tlr and d.info() == 0 and d.ld == (n + 127) // 128 * 128
    L = _dense_from_tlr(f)
    Ld = d.L().cpu().numpy()
    assert np.max(np.abs(np.tril(Ld) - L)) < 1e-13
    N, S, seed = 300, 3, 616
    r = mvn.mvn_prob(d, a, b, None, N=N, S=S, seed=seed, opts=mvn.options(tile=tile), return_ell=True)
    torch.cuda.synchronize()
    at, bt = oracle.centre(a, b)
    ell_ref = oracle.sweep(L, at, bt, N, S, seed)
    assert np.max(np.abs(r["ell"].cpu().numpy() - ell_ref)) < 1e-8
    N, S = 33000, 2  # N * S >= 65536: the 128-column sweep
    rd = mvn.mvn_prob(d, a, b, None, N=N, S=S, seed=seed, opts=mvn.options(tile=tile), return_ell=True)
    rt = _prob(f, a, b, N, S, seed, tile, eps, rcap)
    dl = np.max(np.abs(rd["ell"].cpu().numpy() - rt["ell"].cpu().numpy()))
    print(f"  dense-form vs TLR sweep: max |d ell| {dl:.2e}", flush=True)
    assert dl < 1e-8
    assert abs(rd["logP"].item() - rt["logP"].item()) < 1e-9 * max(1.0, abs(rt["logP"].item()))


@pytest.mark.parametrize("n,tile,rows", [(1300, 128, 64), (700, 256, 128), (1300, 128, 256)])
def test_tlr_compact_factor(n, tile, rows):
    """The compact TLR factor (diagonal tiles and U, V'^T at the actual
    ranks): its buffer is what the ranks need, a sweep through it is bit for
    bit the sweep through the full factor (the same packed operands, read
    from the factor instead of packed per call), full and nested, also after
    the full factor is dropped; the dense form refuses it."""
    eps, rcap = 1e-5, 128
    print(f"tlr compact n={n} tile={tile} rows={rows}", flush=True)
    locs, kern, a, b = _tlr_inputs(40, n, seed=85, beta=0.05)
    f = _factor(n, locs, kern, tile, eps, rcap)
    assert f.info() == 0
    ranks = np.abs(f.ranks().cpu().numpy())
    c = mvn.mvn_tlr_compact(f)
    torch.cuda.synchronize()
    assert c.is_tlr and c.is_compact and c.info() == 0
    m, nt, k = tile, f.nt, int(ranks.sum())
    # diagonal tiles, V' rows (+128 zero rows), U columns (each tile-row padded to 16), the Z index table
    bound = 8 * (nt * m * m + (k + 128) * m + m * (k + 16 * nt) + len(ranks) * rcap) + 2**16
    print(f"  full factor {f.nbytes() / 2**20:.1f} MiB, compact {c.nbytes() / 2**20:.1f} MiB "
          f"(bound {bound / 2**20:.1f} MiB)", flush=True)
    assert c.nbytes() <= bound and c.nbytes() < f.nbytes() / 2
    N, S, seed = 300, 3, 717
    opts = mvn.options(tile=tile, tlr_eps=eps, max_rank=rcap, sweep_rows=rows)
    rf = mvn.mvn_prob(f, a, b, None, N=N, S=S, seed=seed, opts=opts, return_ell=True)
    pf = mvn.mvn_prob_prefix(f, a, b, None, N=N, S=S, seed=seed, opts=opts)
    torch.cuda.synchronize()
    ell_f, lp_f = rf["ell"].cpu().numpy(), pf["logP"].cpu().numpy()
    del f, rf, pf
    torch.cuda.empty_cache()
    rc = mvn.mvn_prob(c, a, b, None, N=N, S=S, seed=seed, opts=opts, return_ell=True)
    pc = mvn.mvn_prob_prefix(c, a, b, None, N=N, S=S, seed=seed, opts=opts)
    torch.cuda.synchronize()
    assert np.array_equal(rc["ell"].cpu().numpy(), ell_f)
    assert np.array_equal(pc["logP"].cpu().numpy(), lp_f)
    with pytest.raises(mvn.MvnError):
        mvn.mvn_tlr_dense(c)


def test_tlr_four_wave_sweep_with_many_chunks():
    """The four-wave form (sweep_rows = 256) at N*S = 140 000: 547 chunks of
    256 columns for at most 512 workgroups (some sweep two, reusing their Y
    and Z slices); sampled columns of every chunk match the oracle's sweep
    through the assembled factor, every column the 64-column sweep's (the
    automatic choice, bit for bit sweep_rows = 64) to 1e-9."""
    n, tile, eps, rcap = 300, 128, 1e-6, 128
    N, S, seed = 14000, 10, 333
    print(f"tlr four-wave n={n} N={N} S={S}", flush=True)
    locs, kern, a, b = _tlr_inputs(20, n, seed=87, beta=0.05)
    f = _factor(n, locs, kern, tile, eps, rcap)
    assert f.info() == 0
    r0 = _prob(f, a, b, N, S, seed, tile, eps, rcap, 0)
    r256 = _prob(f, a, b, N, S, seed, tile, eps, rcap, 256)
    r64 = _prob(f, a, b, N, S, seed, tile, eps, rcap, 64)
    assert torch.equal(r0["ell"], r64["ell"])
    ell = r256["ell"].cpu().numpy()
    NS = N * S
    cols = np.unique(np.concatenate([np.arange(0, NS, 97), np.arange(NS - 300, NS)]))
    L = _dense_from_tlr(f)
    at, bt = oracle.centre(a, b)
    ell_ref = oracle.sweep(L, at, bt, N, S, seed, cols=cols)
    assert np.max(np.abs(ell[cols] - ell_ref)) < 1e-8
    assert np.max(np.abs(ell - r64["ell"].cpu().numpy())) < 1e-9
    assert abs(r256["logP"].item() - r64["logP"].item()) < 1e-10 * max(1.0, abs(r64["logP"].item()))
