"""Benchmark of the SOV MVN-probability hot path on one MI355X.

One step = one whole MVN problem of the largest single-GPU workload, the
65536-site field (256 x 256 grid in Morton order, exponential Matern,
nugget 1e-8, b = -mu) in dense FP64: Matern covariance generation, tiled
Cholesky (tile 1024), and the SOV sweep over N = 10000 Richtmyer points x
S = 10 shifts with the final log-sum-exp reduction.  Inputs (locations,
limits) are resident in HBM before the timed region.  Prints one JSON line.

After the timed steps the same line carries measured variants (each run once
after a warm-up, outside the timed region):
  precision   the 16384-site problem (Matern nu = 3/2, condition number about
              4e6) in FP64 and with FP32 / BF16 / split-BF16 arithmetic, with
              the error against the FP64 result
  oracle400   the 400-site problem in every precision against the CPU oracle
              on identical QMC points
  tlr64k      the timed problem as a tile low-rank factor at 1e-5 and 1e-7
              (ranks, times over 3 steps after a warm-up, log P difference
              and speed-up against the timed dense FP64 steps)
  autotune    the autotuner's choice of Cholesky tile and sweep block rows
              for the timed workload, with every candidate's time
  batch2000   2000 confidence-region problems of uneven size in one call
              (sweep block rows chosen by the autotuner)
  grad4096    forward + adjoint sweep for d log P / d(a, b, mu)

    python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--no-cpu-baseline] [--no-variants]
    python bench.py --tlr-eps 1e-5 --no-variants --no-cpu-baseline
    python bench.py --workload prec16k --precision bf16 --no-variants --no-cpu-baseline
    python bench.py --steps 1 --warmup 0 --no-cpu-baseline --variants batch2000
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time
import traceback

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MVN probs/sec + effective TFLOP/s (Cholesky+SOV) at stated error vs FP64 oracle"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "bf16x3": 2500.0}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16x3": 3}

# HBM bytes per sweep launch on the dense FP64 workloads from rocprofv3
# FETCH_SIZE x2 + WRITE_SIZE x1 (factors from a 1 GiB copy; the summaries are
# profiles/sweep_kernel_f64_dense64k.md and sweep_kernel_f64_prec16k.md),
# valid only for the kernel sources they were measured on (checked by hash).
TRAFFIC_SOURCES = ["paper_2405_14892_amd/csrc/kernels_sov_wide.hip", "paper_2405_14892_amd/csrc/mvn_device.h",
                   "paper_2405_14892_amd/csrc/sweep_block.h", "paper_2405_14892_amd/csrc/gemm_f64.h"]
TRAFFIC_MEASURED = {"tlr64k": ("577b5c4ccdc95436", 7.2924e12), "prec16k": ("577b5c4ccdc95436", 9.148e11)}


def _traffic(workload: str):
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    rec = TRAFFIC_MEASURED.get(workload)
    return rec[1] if rec and rec[0] == h.hexdigest()[:16] else None


def _cpu_baseline(w, n_sub: int = 8192, cols: int = 1024) -> dict:
    """The oracle, untuned, on a bounded sample of the same workload: the
    first n_sub sites (covariance + Cholesky + SOV sweep over `cols` sample
    columns), scaled to one full problem by n^3 (factor) and n^2 N S (sweep).
    The figure is an extrapolation, labelled as such."""
    import numpy as np
    import oracle
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        blas_threads = 1
    n_sub = min(n_sub, w.n)
    idx = np.arange(n_sub)
    locs = w.locs[idx]
    t0 = time.perf_counter()
    sig = oracle.covariance(locs, w.sigma2, w.beta, w.nu, w.nugget)
    L = oracle.cholesky(sig)
    t1 = time.perf_counter()
    at, bt = oracle.centre(w.a[idx], w.b[idx], w.mu[idx] if w.mu is not None else None)
    oracle.sweep(L, at, bt, w.N, w.S, w.seed, cols=np.arange(cols))
    t2 = time.perf_counter()
    n, NS = w.n, w.N * w.S
    full = (t1 - t0) * (n / n_sub) ** 3 + (t2 - t1) * (n / n_sub) ** 2 * (NS / cols)
    return {"value": 1.0 / full, "unit": "MVN probs/s", "cores": int(os.cpu_count() or 1),
            "blas_threads": int(blas_threads), "kind": "oracle", "extrapolated": True,
            "sample": (f"EXTRAPOLATED: oracle covariance+Cholesky of the first {n_sub} sites ({t1 - t0:.1f} s) and "
                       f"SOV sweep of {cols} sample columns at n={n_sub} ({t2 - t1:.1f} s), "
                       f"scaled by (n/{n_sub})^3 and (n/{n_sub})^2*(N*S/{cols}) to n={n}, "
                       f"N*S={NS}; {os.cpu_count()} host cores, BLAS threads {blas_threads}"),
            "seconds_full_problem_extrapolated": full}


class Problem:
    """One MVN problem with its device buffers, run through the C ABI on the
    current stream; phase times come from HIP events on that stream."""

    def __init__(self, w, opts, dev):
        import torch
        import paper_2405_14892_amd as mvn
        from paper_2405_14892_amd import _lib
        self.torch, self.mvn, self.lib = torch, mvn, _lib
        self.h = _lib.lib()
        self.w, self.opts, self.dev = w, opts, dev
        n, N, S = w.n, w.N, w.S
        self.kern = _lib.MvnMatern(w.sigma2, w.beta, w.nu, w.nugget)
        f64 = lambda x: torch.as_tensor(x, dtype=torch.float64).to(dev).contiguous()
        self.locs, self.a, self.b = f64(w.locs), f64(w.a), f64(w.b)
        self.mu = f64(w.mu) if w.mu is not None else None
        self.fb = mvn.mvn_factor_bytes(n, opts)
        self.cwb = mvn.mvn_cholesky_workspace_bytes(n, opts)
        self.tlr = opts.tlr_eps > 0
        # a TLR workspace is sized for the factor's ranks, after the first factorisation
        self.wsb = 0 if self.tlr else mvn.mvn_prob_workspace_bytes(n, N, S, opts)
        self.fbuf = torch.empty(self.fb, dtype=torch.uint8, device=dev)
        self.cws = torch.empty(max(self.cwb, 1), dtype=torch.uint8, device=dev)
        self.ws = None if self.tlr else torch.empty(self.wsb, dtype=torch.uint8, device=dev)
        self.out = torch.empty(4 + S, dtype=torch.float64, device=dev)
        self.fac = _lib.MvnFactor()
        self.stream = torch.cuda.current_stream(dev)
        self.sp = ctypes.c_void_p(self.stream.cuda_stream)

    @staticmethod
    def _p(t):
        return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)

    def step(self):
        """Enqueue one problem; returns the (start, factored, done) events."""
        torch, P, w = self.torch, self._p, self.w
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record(self.stream)
        self.lib.check(self.h.mvn_cholesky(w.n, None, 0, P(self.locs), ctypes.byref(self.kern),
                                           ctypes.byref(self.opts), P(self.fbuf), self.fb, P(self.cws), self.cwb,
                                           ctypes.byref(self.fac), self.sp))
        e[1].record(self.stream)
        if self.ws is None:
            out = ctypes.c_size_t(0)
            self.lib.check(self.h.mvn_prob_workspace_bytes_factor(ctypes.byref(self.fac), w.N, w.S,
                                                                  ctypes.byref(self.opts), ctypes.byref(out), self.sp))
            self.wsb = out.value
            self.ws = torch.empty(self.wsb, dtype=torch.uint8, device=self.dev)
        self.lib.check(self.h.mvn_prob(ctypes.byref(self.fac), P(self.a), P(self.b), P(self.mu), w.N, w.S,
                                       ctypes.c_uint64(w.seed), ctypes.byref(self.opts), P(self.ws), self.wsb,
                                       P(self.out), None, self.sp))
        e[2].record(self.stream)
        return e

    def run(self, steps, warmup):
        torch = self.torch
        for _ in range(warmup):
            self.step()
            torch.cuda.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev = [self.step() for _ in range(steps)]
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        chol = [a.elapsed_time(b) for a, b, _ in ev]
        sov = [b.elapsed_time(c) for _, b, c in ev]
        res = self.out.cpu().numpy()
        return {"wall_ms": wall * 1e3, "cholesky_ms": sum(chol) / len(chol), "sov_ms": sum(sov) / len(sov),
                "wall_ms_steps": [a.elapsed_time(c) for a, _, c in ev],
                "logP": float(res[0]), "P": float(res[1]), "rel_stderr": float(res[3]), "info": self.info()}

    def info(self):
        off = self.fac.info - self.fbuf.data_ptr()
        return int(self.fbuf[off: off + 4].view(self.torch.int32).item())

    def update_counts(self):
        if self.tlr or not self.fac.update_counts:
            return None
        off = self.fac.update_counts - self.fbuf.data_ptr()
        c = self.fbuf[off: off + 24].view(self.torch.int64).cpu().tolist()
        return {"fp64": c[0], "fp32": c[1], "reduced": c[2]}

    def ranks(self):
        import numpy as np
        nt = self.fac.ld // self.fac.tile
        cnt = nt * (nt - 1) // 2
        off = self.fac.ranks - self.fbuf.data_ptr()
        return self.fbuf[off: off + 4 * cnt].view(self.torch.int32).cpu().numpy().astype(np.int64)

    def tile(self, i, j):
        """Tile (i, j), j <= i, of a TLR factor's tile store: for j < i the
        tile the panel was compressed from."""
        m = self.fac.tile
        off = self.fac.L - self.fbuf.data_ptr() + 8 * (i * (i + 1) // 2 + j) * m * m
        return self.fbuf[off: off + 8 * m * m].view(self.torch.float64).view(m, m).cpu().numpy()


def _frob_eps_rank(A, eps):
    """Smallest k with ||A - A_k||_F <= eps for the truncated SVD A_k."""
    import numpy as np
    s = np.linalg.svd(A, compute_uv=False)
    tail = np.sqrt(np.cumsum((s ** 2)[::-1]))[::-1]
    return int(np.sum(tail > eps))


def _flops(n, NS):
    return n ** 3 / 3.0, float(n) * (n - 1) * NS


def _free():
    import gc
    import torch
    gc.collect()
    torch.cuda.empty_cache()


def variant_precision(dev) -> dict:
    """The 16384-site problem (Matern 3/2, condition number about 4e6) in
    FP64 and in each reduced precision: with the adaptive tile-wise precision
    map of the trailing updates (the default), with the factorisation in FP64
    and only the sweep's GEMM reduced, and with every trailing update in the
    reduced type.  Errors against the FP64 result on identical QMC points,
    beside the QMC relative standard error."""
    import paper_2405_14892_amd as mvn
    import workloads
    w = workloads.make_workload("prec16k")
    p = Problem(w, mvn.options(tile=w.tile), dev)
    ref = p.run(1, 1)
    del p
    _free()
    out = {"fp64": {k: ref[k] for k in ("wall_ms", "cholesky_ms", "sov_ms", "info", "logP", "P", "rel_stderr")}}
    chol, sov = _flops(w.n, w.N * w.S)
    modes = (("adaptive", mvn.MVN_CHOL_ADAPTIVE), ("fp64_factor", mvn.MVN_CHOL_FP64),
             ("uniform", mvn.MVN_CHOL_UNIFORM))
    for name in ("fp32", "bf16x3", "bf16"):
        for mname, mode in modes:
            p = Problem(w, mvn.options(tile=w.tile, precision=PRECISIONS[name], chol_mode=mode), dev)
            r = p.run(1, 1)
            counts = p.update_counts()
            del p
            _free()
            out[f"{name}_{mname}"] = {
                "wall_ms": r["wall_ms"], "cholesky_ms": r["cholesky_ms"], "sov_ms": r["sov_ms"],
                "info": r["info"], "logP": r["logP"], "abs_dlogP_vs_fp64": abs(r["logP"] - ref["logP"]),
                "abs_dP_vs_fp64": abs(r["P"] - ref["P"]), "rel_stderr": r["rel_stderr"],
                "fp64_rel_stderr": ref["rel_stderr"], "speedup_vs_fp64": ref["wall_ms"] / r["wall_ms"],
                "sweep_tflops": sov / (r["sov_ms"] * 1e-3) / 1e12,
                "cholesky_tflops": chol / (r["cholesky_ms"] * 1e-3) / 1e12,
                "trailing_tile_updates": counts}
    out["note"] = ("error against the FP64 GPU result on identical QMC points (the FP64 path matches the oracle "
                   "to 1e-10); adaptive = tile-wise precision map of the trailing updates (default tolerance "
                   "1e-9 of max diag Sigma per tile update), fp64_factor = FP64 factorisation with the reduced "
                   "type only in the sweep GEMM, uniform = every trailing update in the reduced type.  info > 0: "
                   "the factorisation lost positive definiteness at that pivot (outputs NaN)")
    return out


def variant_oracle400(dev) -> dict:
    import numpy as np
    import oracle
    import paper_2405_14892_amd as mvn
    import workloads
    out = {}
    for excursion in (False, True):
        w = workloads.make_workload("dense400", positive_excursion=excursion)
        t0 = time.perf_counter()
        L = oracle.cholesky(oracle.covariance(w.locs, w.sigma2, w.beta, w.nu, w.nugget))
        at, bt = oracle.centre(w.a, w.b, w.mu)
        ref = oracle.reduce_samples(oracle.sweep(L, at, bt, w.N, w.S, w.seed), w.N, w.S)
        t_or = time.perf_counter() - t0
        key = "b=mu-u" if excursion else "b=u-mu"
        rows = {"oracle_logP": ref["logP"], "oracle_P": ref["P"], "oracle_rel_stderr": ref["rel_stderr"],
                "oracle_seconds": t_or}
        for name, code in PRECISIONS.items():
            p = Problem(w, mvn.options(tile=w.tile, precision=code), dev)
            r = p.run(3, 1)
            rows[name] = {"wall_ms": r["wall_ms"], "abs_dlogP": abs(r["logP"] - ref["logP"]),
                          "abs_dP": abs(r["P"] - ref["P"])}
            del p
        out[key] = rows
        _free()
    return out


def _tlr_dense_sweep(p, w, dev) -> dict:
    """The configuration of Section IV-C on the TLR factor held by Problem p:
    the factor written out dense (mvn_tlr_dense), then the dense FP64 sweep
    (one timed call; its kernels are warm from the dense steps).  Frees p's
    TLR sweep workspace first."""
    import torch
    mvn, lib, h, P = p.mvn, p.lib, p.h, p._p
    p.ws = None
    _free()
    nb = ctypes.c_size_t(0)
    lib.check(h.mvn_tlr_dense_bytes(ctypes.byref(p.fac), ctypes.byref(nb)))
    dbuf = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    dfac = lib.MvnFactor()
    dopts = mvn.options(tile=1024)
    wsb = mvn.mvn_prob_workspace_bytes(w.n, w.N, w.S, dopts)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    out = torch.empty(4 + w.S, dtype=torch.float64, device=dev)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    e[0].record(p.stream)
    lib.check(h.mvn_tlr_dense(ctypes.byref(p.fac), P(dbuf), nb.value, ctypes.byref(dfac), p.sp))
    e[1].record(p.stream)
    lib.check(h.mvn_prob(ctypes.byref(dfac), P(p.a), P(p.b), P(p.mu), w.N, w.S, ctypes.c_uint64(w.seed),
                         ctypes.byref(dopts), P(ws), wsb, P(out), None, p.sp))
    e[2].record(p.stream)
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    del dbuf, ws
    _free()
    return {"expand_ms": e[0].elapsed_time(e[1]), "sov_ms": e[1].elapsed_time(e[2]), "logP": float(res[0])}


def _tlr_compact_sweep(p, w, dev) -> dict:
    """The TLR factor held by Problem p cut to its ranks (mvn_tlr_compact),
    then 3 timed TLR sweeps through it after a warm-up: the factor and
    workspace sizes beside those of the full factor."""
    import torch
    lib, h, P = p.lib, p.h, p._p
    nb = ctypes.c_size_t(0)
    lib.check(h.mvn_tlr_compact_bytes(ctypes.byref(p.fac), ctypes.byref(nb), p.sp))
    cbuf = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    cfac = lib.MvnFactor()
    lib.check(h.mvn_tlr_compact(ctypes.byref(p.fac), P(cbuf), nb.value, ctypes.byref(cfac), p.sp))
    wsb = ctypes.c_size_t(0)
    lib.check(h.mvn_prob_workspace_bytes_factor(ctypes.byref(cfac), w.N, w.S, ctypes.byref(p.opts),
                                                ctypes.byref(wsb), p.sp))
    p.ws = None
    _free()
    ws = torch.empty(wsb.value, dtype=torch.uint8, device=dev)
    out = torch.empty(4 + w.S, dtype=torch.float64, device=dev)
    ms = []
    for it in range(4):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        e[0].record(p.stream)
        lib.check(h.mvn_prob(ctypes.byref(cfac), P(p.a), P(p.b), P(p.mu), w.N, w.S, ctypes.c_uint64(w.seed),
                             ctypes.byref(p.opts), P(ws), wsb.value, P(out), None, p.sp))
        e[1].record(p.stream)
        torch.cuda.synchronize()
        if it > 0:
            ms.append(e[0].elapsed_time(e[1]))
    res = out.cpu().numpy()
    del cbuf, ws
    _free()
    return {"factor_bytes_full": p.fb, "factor_bytes_compact": nb.value, "workspace_bytes": wsb.value,
            "sov_ms": sorted(ms)[len(ms) // 2], "logP": float(res[0])}


def variant_tlr(dev, dense=None) -> dict:
    """The 65536-site problem with a tile low-rank factor at 1e-5 and 1e-7,
    each timed over 3 steps after a warm-up (default sweep block shape),
    against the dense FP64 steps of the same problem: the timed headline
    steps when they are that problem, else 3 dense steps here."""
    import numpy as np
    import paper_2405_14892_amd as mvn
    import workloads
    w = workloads.make_workload("tlr64k")
    chol_f, sov_f = _flops(w.n, w.N * w.S)
    out = {}
    if dense is None:
        p = Problem(w, mvn.options(tile=1024), dev)
        dense = p.run(3, 1)
        del p
        _free()
    out["dense_fp64"] = {"wall_ms": dense["wall_ms"], "cholesky_ms": dense["cholesky_ms"], "sov_ms": dense["sov_ms"],
                         "logP": dense["logP"], "info": dense["info"],
                         "cholesky_tflops": chol_f / (dense["cholesky_ms"] * 1e-3) / 1e12,
                         "sweep_tflops": sov_f / (dense["sov_ms"] * 1e-3) / 1e12}
    for eps in (1e-5, 1e-7):
        p = Problem(w, mvn.options(tile=w.tile, tlr_eps=eps, max_rank=256), dev)
        r = p.run(3, 1)
        ranks, ld = np.abs(p.ranks()), p.fac.ld
        # ranks against the tiles' Frobenius eps-ranks (host SVD) on sampled panels:
        # every 8th adjacent tile and 8 others
        nt_ = ld // w.tile
        rng = np.random.default_rng(5)
        sample = [(i, i - 1) for i in range(1, nt_, 8)]
        for _ in range(8):
            i = int(rng.integers(2, nt_))
            sample.append((i, int(rng.integers(0, i - 1))))
        svd_r = [(int(ranks[i * (i - 1) // 2 + k]), _frob_eps_rank(p.tile(i, k), eps)) for i, k in sample]
        full_ws = p.wsb
        csw = _tlr_compact_sweep(p, w, dev)
        dsw = _tlr_dense_sweep(p, w, dev)
        del p
        _free()
        m = w.tile
        nt = ld // m
        # executed sweep flops per sample: 4 m k_ij over the panels + the dense diagonal tiles
        sweep_exec = (4.0 * m * ranks.sum() + nt * float(m) * m) * w.N * w.S
        out[f"tlr_{eps:g}"] = {
            "wall_ms": r["wall_ms"], "wall_ms_steps": r["wall_ms_steps"], "cholesky_ms": r["cholesky_ms"],
            "sov_ms": r["sov_ms"], "logP": r["logP"],
            "abs_dlogP_vs_dense": abs(r["logP"] - dense["logP"]), "info": r["info"],
            "speedup_vs_dense": dense["wall_ms"] / r["wall_ms"],
            "cholesky_speedup_vs_dense": dense["cholesky_ms"] / r["cholesky_ms"],
            "sweep_speedup_vs_dense": dense["sov_ms"] / r["sov_ms"],
            "effective_tflops": (chol_f + sov_f) / (r["wall_ms"] * 1e-3) / 1e12,
            "sweep_executed_tflops": sweep_exec / (r["sov_ms"] * 1e-3) / 1e12,
            "compact_factor": {
                "factor_bytes_full": csw["factor_bytes_full"], "factor_bytes_compact": csw["factor_bytes_compact"],
                "workspace_bytes_full": full_ws, "workspace_bytes_compact": csw["workspace_bytes"],
                "sov_ms": csw["sov_ms"], "abs_dlogP_vs_full": abs(csw["logP"] - r["logP"]),
                "note": "diagonal tiles and U, V'^T at the actual ranks (mvn_tlr_compact); median of 3 sweeps"},
            "tlr_cholesky_dense_sweep": {
                "expand_ms": dsw["expand_ms"], "sov_ms": dsw["sov_ms"],
                "wall_ms": r["cholesky_ms"] + dsw["expand_ms"] + dsw["sov_ms"],
                "speedup_vs_dense": dense["wall_ms"] / (r["cholesky_ms"] + dsw["expand_ms"] + dsw["sov_ms"]),
                "abs_dlogP_vs_tlr_sweep": abs(dsw["logP"] - r["logP"]),
                "note": "TLR factorisation, factor written out dense, dense FP64 sweep (one timed call)"},
            "ranks": {"mean": float(ranks.mean()), "max": int(ranks.max()),
                      "adjacent_mean": float(np.mean([ranks[i * (i - 1) // 2 + i - 1] for i in range(1, nt)])),
                      "histogram_by_16": np.bincount(np.minimum(ranks // 16, 16)).tolist(),
                      "sampled_vs_svd_eps_rank": {
                          "panels": [list(x) for x in sample], "ranks": [a for a, _ in svd_r],
                          "svd_eps_ranks": [b for _, b in svd_r],
                          "sum_ratio": sum(a for a, _ in svd_r) / max(1, sum(b for _, b in svd_r)),
                          "note": "Frobenius eps-rank: smallest k with ||A - A_k||_F <= eps (host SVD of "
                                  "the tile the panel was compressed from)"}}}
    out["config"] = (f"n={w.n} (256^2 Morton grid), Matern nu={w.nu}, beta={w.beta}, nugget={w.nugget}, "
                     f"N={w.N} x S={w.S}; dense tile 1024, TLR tile {w.tile}, max_rank 256; TLR eps > 0 is "
                     "checked by per-tile residual and rank properties, not entry-wise against the oracle")
    return out


def variant_batch(dev) -> dict:
    """The 2000-problem batch: the autotuner picks the sweep block rows per
    precision (both shapes timed), then the tuned configuration is timed on
    the literal limits b = u - mu (P close to 0 for most problems) and on the
    positive-excursion limits b = mu - u (the confidence function of Section
    III-C, P = O(1)), where the absolute probability error against FP64 is
    meaningful."""
    import numpy as np
    import torch
    import paper_2405_14892_amd as mvn
    from paper_2405_14892_amd import autotune
    import workloads
    out = {}
    Ps = {}
    for conv, excursion in (("b=u-mu", False), ("b=mu-u", True)):
        bw = workloads.make_batch(positive_excursion=excursion)
        sizes = bw.n_p.astype(np.int32)
        idx = torch.as_tensor(bw.idx).to(dev)
        locs = torch.as_tensor(bw.locs).to(dev)
        a, b = torch.as_tensor(bw.a).to(dev), torch.as_tensor(bw.b).to(dev)
        kern = (bw.sigma2, bw.beta, bw.nu, bw.nugget)
        NS = bw.N * bw.S
        sov_f = float(np.sum(bw.n_p.astype(np.float64) * (bw.n_p - 1))) * NS
        res_c = {}
        for name in ("fp32", "bf16", "bf16x3", "fp64"):
            if not excursion and name != "fp64":
                tuned = autotune.tune_batch(sizes, idx, locs, kern, a, b, N=bw.N, S=bw.S, seed=bw.seed,
                                            precision=PRECISIONS[name], device=dev)
                rows, tune_s = tuned["sweep_rows"], tuned["batch_s"]
            elif not excursion:
                rows, tune_s = 64, None  # (FP64 runs the four-wave sweep with 64-row blocks only)
            else:
                rows, tune_s = out["b=u-mu"][name]["sweep_rows"], None
            plan = mvn.mvn_batch_plan(sizes, bw.N, bw.S, mvn.options(tile=128, precision=PRECISIONS[name],
                                                                     sweep_rows=rows), device=dev)
            if not excursion:  # (the excursion runs reuse warm code and buffers of the same size)
                mvn.mvn_prob_batch(plan, idx, locs, kern, a, b, None, seed=bw.seed)
            torch.cuda.synchronize()
            st = torch.cuda.current_stream(dev)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            reps = 1
            for _ in range(reps):
                mvn.mvn_prob_batch(plan, idx, locs, kern, a, b, None, seed=bw.seed)
            e1.record(st)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            res = plan.out.cpu().numpy()
            res_c[name] = {"ms_per_batch": ms, "problems_per_s": len(sizes) / (ms * 1e-3),
                           "sweep_rows": rows, "sweep_tflops_equiv": sov_f / (ms * 1e-3) / 1e12,
                           "conditioning_steps_per_s": float(sizes.sum()) * NS / (ms * 1e-3),
                           "failed": int((plan.info.cpu().numpy() != 0).sum())}
            if tune_s is not None:
                res_c[name]["autotune_s_by_rows"] = tune_s
            Ps[(conv, name)] = res[:, 1].copy()
            del plan
            _free()
        for name in ("fp32", "bf16", "bf16x3"):
            d = np.abs(Ps[(conv, name)] - Ps[(conv, "fp64")])
            res_c[name]["max_abs_dP_vs_fp64"] = float(np.max(d))
            res_c[name]["problems_over_1e-4"] = int(np.sum(d > 1e-4))
        res_c["P_fp64_quantiles_0_50_100"] = [float(q) for q in np.quantile(Ps[(conv, "fp64")], [0, 0.5, 1])]
        out[conv] = res_c
    out["config"] = (f"{len(sizes)} problems, n_p in [{int(sizes.min())}, {int(sizes.max())}], "
                     f"sum n_p = {int(sizes.sum())}, N={bw.N} x S={bw.S}, 256-wide Cholesky steps with every "
                     "trailing update in the stated type; sweep block rows chosen by the autotuner on b = u - mu")
    return out


def variant_autotune_dense(w, dev) -> dict:
    """The autotuner on the timed workload itself: Cholesky tile and sweep
    block rows, every candidate timed once."""
    from paper_2405_14892_amd import autotune
    kern = (w.sigma2, w.beta, w.nu, w.nugget)
    res = autotune.tune_dense(w.n, w.locs, kern, w.a, w.b, w.mu, N=w.N, S=w.S, seed=w.seed,
                              tiles=(256, 512, 1024), device=dev)
    res.pop("key", None)
    return res


def variant_crd(dev) -> dict:
    """Confidence-region detection (Section III-C with Algorithm 1 of Section IV-A) on the
    16384-site field: sites ordered by marginal exceedance of u = 0.5, the
    factor in that order, and one nested-set sweep giving log P-hat of every
    prefix; beside it the full-estimate sweep on the same factor.  The cost
    of one call per nested set is estimated from the sweep's k^2 work."""
    import math
    import numpy as np
    import torch
    import paper_2405_14892_amd as mvn
    import workloads
    from scipy.special import ndtr
    w = workloads.make_workload("prec16k")
    u = 0.5
    field = w.extra["field"]  # the mean field of the workload's GP draw
    kern = (w.sigma2, w.beta, w.nu, w.nugget)
    order = np.argsort(-ndtr((field - u) / math.sqrt(w.sigma2 + w.nugget)), kind="stable")
    opts = mvn.options(tile=w.tile)
    st = torch.cuda.current_stream(dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    a, b, mu = np.full(w.n, u), np.full(w.n, np.inf), field[order]
    mvn.mvn_prob_prefix(mvn.mvn_cholesky(w.n, locs=w.locs[order], kern=kern, opts=opts, device=dev), a, b, mu,
                        N=64, S=2, seed=w.seed, opts=opts)  # warm-up
    torch.cuda.synchronize()
    ev[0].record(st)
    f = mvn.mvn_cholesky(w.n, locs=w.locs[order], kern=kern, opts=opts, device=dev)
    ev[1].record(st)
    r = mvn.mvn_prob_prefix(f, a, b, mu, N=w.N, S=w.S, seed=w.seed, opts=opts)
    ev[2].record(st)
    full = mvn.mvn_prob(f, a, b, mu, N=w.N, S=w.S, seed=w.seed, opts=opts)
    ev[3].record(st)
    torch.cuda.synchronize()
    logp = r["logP"].cpu().numpy()
    p = np.exp(logp)
    prefix_ms, full_ms = ev[1].elapsed_time(ev[2]), ev[2].elapsed_time(ev[3])
    per_set_s = full_ms * 1e-3 * sum((k / w.n) ** 2 for k in range(1, w.n + 1))
    # Monte Carlo check of the regions (Section V-C): M fields on the same factor
    M = 50000
    mc = {}
    for rows in (64, 128):
        mo = mvn.options(tile=w.tile, sweep_rows=rows)
        mvn.mvn_mc_prefix(f, a, b, mu, M=M, seed=w.seed + 1, opts=mo)  # warm-up
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        m = mvn.mvn_mc_prefix(f, a, b, mu, M=M, seed=w.seed + 1, opts=mo)
        e1.record(st)
        torch.cuda.synchronize()
        first = m["first"].cpu().numpy()
        cnt = m["count"].cpu().numpy()
        # GEMM work actually done: each 64-sample chunk runs its blocks up to
        # the one holding its latest first failure
        last = np.maximum.reduce(np.pad(first, (0, -M % 64), constant_values=0).reshape(-1, 64), axis=1)
        blocks = np.minimum(last // rows + 1, -(-w.n // rows))
        flops = float(np.sum(2.0 * rows * rows * 64 * blocks * (blocks + 1) / 2))
        ms = e0.elapsed_time(e1)
        mc[f"rows{rows}"] = {"ms": ms, "gemm_tflops": flops / (ms * 1e-3) / 1e12,
                             "median_first_failure": float(np.median(first)), "max_first_failure": int(first.max())}
    checks = {}
    for al in (0.01, 0.05, 0.1):
        k = int(np.sum(p >= 1 - al))
        pm = float(cnt[k - 1]) / M if k > 0 else 1.0
        checks[str(al)] = {"region": k, "p_qmc": float(p[k - 1]) if k else 1.0, "p_mc": pm,
                           "one_minus_alpha_minus_p_mc": 1 - al - pm}
    return {"cholesky_ms": ev[0].elapsed_time(ev[1]), "prefix_sweep_ms": prefix_ms, "full_sweep_ms": full_ms,
            "mc_check": {"samples": M, **mc, "regions": checks},
            "prefix_overhead": prefix_ms / full_ms - 1.0, "info": f.info(),
            "last_prefix_minus_full_logP": float(logp[-1] - full["logP"].item()),
            "region_size": {str(al): int(np.sum(p >= 1 - al)) for al in (0.01, 0.05, 0.1)},
            "excursion_at_100_1000_4000": [float(p[99]), float(p[999]), float(p[3999])],
            "one_call_per_set_s_estimated": per_set_s,
            "speedup_vs_one_call_per_set_estimated": per_set_s / (prefix_ms * 1e-3),
            "config": (f"prec16k field, u={u}, event X > u, sites by marginal exceedance, N={w.N} x S={w.S}, "
                       f"tile {w.tile}, FP64; one-call-per-set cost = full sweep time x sum_k (k/n)^2; "
                       f"Monte Carlo check: {M} fields X = mu + L Z on the same factor")}


def variant_posterior(dev) -> dict:
    """Confidence regions on the posterior of Section V-B at the paper's
    synthetic size: 40 000 grid sites, 6 250 noisy observations (noise sd
    0.5), exponential kernel with range 0.033 / 0.1 / 0.234; QMC size
    10 000 (N = 1000 x S = 10); threshold u = 0.5.  Per range: the posterior
    (bordered partial factorisation), the factor of Sigma_post in exceedance
    order, the nested-set sweep, and the Monte Carlo check (50 000 fields)."""
    import numpy as np
    import torch
    import paper_2405_14892_amd as mvn
    import workloads
    from scipy.special import ndtr
    u, N, S, M, tile = 0.5, 1000, 10, 50000, 512
    opts = mvn.options(tile=tile)
    st = torch.cuda.current_stream(dev)
    out = {}
    for beta in (0.033, 0.1, 0.234):
        d = workloads.make_posterior(beta=beta)
        kern = (d.sigma2, d.beta, d.nu, d.nugget)
        n = d.locs.shape[0]
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        torch.cuda.synchronize()
        ev[0].record(st)
        post = mvn.mvn_posterior(d.locs, kern, d.obs, d.y, d.noise_sd ** 2, opts=opts, device=dev)
        ev[1].record(st)
        mu_post = post["mu_post"].cpu().numpy()
        sd_post = np.sqrt(np.maximum(post["var_post"].cpu().numpy(), 0))
        order = np.argsort(-ndtr((mu_post - u) / sd_post), kind="stable")
        e2 = torch.cuda.Event(enable_timing=True)
        e2.record(st)
        f = mvn.mvn_cholesky_permuted(post["sigma_post"], order, opts=opts)
        ev[2].record(st)
        a, b, mo = np.full(n, u), np.full(n, np.inf), mu_post[order]
        r = mvn.mvn_prob_prefix(f, a, b, mo, N=N, S=S, seed=7, opts=opts)
        ev[3].record(st)
        m = mvn.mvn_mc_prefix(f, a, b, mo, M=M, seed=8, opts=opts, return_first=False)
        ev[4].record(st)
        torch.cuda.synchronize()
        p = np.exp(r["logP"].cpu().numpy())
        cnt = m["count"].cpu().numpy()
        regions = {}
        for al in (0.01, 0.05, 0.1):
            k = int(np.sum(p >= 1 - al))
            pm = float(cnt[k - 1]) / M if k else 1.0
            regions[str(al)] = {"region": k, "p_qmc": float(p[k - 1]) if k else 1.0, "p_mc": pm,
                                "one_minus_alpha_minus_p_mc": 1 - al - pm}
        out[f"beta{beta}"] = {"posterior_ms": ev[0].elapsed_time(ev[1]), "factor_ms": e2.elapsed_time(ev[2]),
                              "prefix_sweep_ms": ev[2].elapsed_time(ev[3]), "mc_check_ms": ev[3].elapsed_time(ev[4]),
                              "info": [post["info"], f.info()], "marginal_above_0.95": int(np.sum(
                                  ndtr((mu_post - u) / sd_post) >= 0.95)), "regions": regions}
        del post, f, r, m
        torch.cuda.empty_cache()
    out["config"] = (f"40000 grid sites, 6250 observations, noise sd 0.5, exponential kernel sigma2 1, nugget 1e-8; "
                     f"u = {u}, N = {N} x S = {S}, tile {tile}, FP64; Monte Carlo check {M} fields")
    return out


def variant_grad(dev) -> dict:
    """The differentiation workload: forward sweep alone and forward +
    adjoint, in FP64 and with the forward GEMM in FP32 / split BF16 / BF16
    (FP64 factorisation, reverse GEMM and conditioning), each gradient's
    error against the FP64 one."""
    import numpy as np
    import torch
    import paper_2405_14892_amd as mvn
    import workloads
    w = workloads.make_workload("grad4096")
    st = torch.cuda.current_stream(dev)

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            r = fn()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, r

    out = {}
    ref = None
    for name in ("fp64", "fp32", "bf16x3", "bf16"):
        o = mvn.options(tile=w.tile, precision=PRECISIONS[name], chol_mode=mvn.MVN_CHOL_FP64)
        f = mvn.mvn_cholesky(w.n, locs=w.locs, kern=(w.sigma2, w.beta, w.nu, w.nugget), opts=o, device=dev)
        ws = torch.empty(mvn.mvn_prob_workspace_bytes(w.n, w.N, w.S, o), dtype=torch.uint8, device=dev)
        fwd_ms, rf = timed(lambda: mvn.mvn_prob(f, w.a, w.b, w.mu, N=w.N, S=w.S, seed=w.seed, opts=o, workspace=ws))
        grad_ms, rg = timed(lambda: mvn.mvn_prob_grad(f, w.a, w.b, w.mu, N=w.N, S=w.S, seed=w.seed, opts=o))
        g = np.concatenate([rg["da"].cpu().numpy(), rg["db"].cpu().numpy()])
        row = {"forward_ms": fwd_ms, "forward_plus_adjoint_ms": grad_ms, "ratio": grad_ms / fwd_ms,
               "logP": float(rg["logP"].item()),
               "abs_dlogP_vs_forward": abs(float(rg["logP"].item()) - float(rf["logP"].item()))}
        if ref is None:
            ref = (g, float(rg["logP"].item()))
        else:
            row["max_rel_grad_err_vs_fp64"] = float(np.max(np.abs(g - ref[0])) / np.max(np.abs(ref[0])))
            row["abs_dlogP_vs_fp64"] = abs(row["logP"] - ref[1])
        out[name] = row
        del f, ws
        _free()
    out["config"] = (f"n={w.n}, N={w.N} x S={w.S}, finite limits a=mu-3, b=mu+u; FP64 factorisation; the "
                     "reduced types apply to the forward limit-update GEMM (reverse GEMM and conditioning FP64); "
                     "gradient error = max |g - g_fp64| / max |g_fp64| over (d/da, d/db)")
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="tlr64k")
    ap.add_argument("--precision", default="fp64", choices=sorted(PRECISIONS))
    ap.add_argument("--tlr-eps", type=float, default=0.0)
    ap.add_argument("--max-rank", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--variants", default="",
                    help="comma-separated subset of the variants to run (default: all)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 8, "copy_bytes_written": y.numel() * 8,
                          "copies": 3}))
        return 0
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU: the library has no multi-GPU "
                                   "path (it would shard over sample columns, each GPU holding its own "
                                   "factor)", "n_gpus": args.gpus}))
        return 2

    import torch

    import paper_2405_14892_amd as mvn
    import workloads

    w = workloads.make_workload(args.workload)
    n, N, S = w.n, w.N, w.S
    dev = torch.device("cuda:0")
    tlr = args.tlr_eps > 0
    opts = (mvn.options(tile=w.tile, tlr_eps=args.tlr_eps, max_rank=args.max_rank) if tlr
            else mvn.options(tile=w.tile, precision=PRECISIONS[args.precision]))
    prob = Problem(w, opts, dev)
    for i in range(args.warmup):
        prob.step()
        torch.cuda.synchronize()
        print(f"# warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    r = prob.run(args.steps, 0)
    print(f"# {args.steps} timed steps done", file=sys.stderr, flush=True)
    import numpy as np
    tlr_ranks = np.abs(prob.ranks()) if tlr else None
    tlr_ld = prob.fac.ld if tlr else 0
    del prob
    _free()
    ms = r["wall_ms"]
    chol_flops, sov_flops = _flops(n, N * S)
    roof_flops, roof_note = sov_flops, "achieved = n(n-1)*N*S dense-equivalent flops / event time of the mvn_prob call"
    if tlr:
        # the TLR sweep executes 4 m k_ij flops per sample for each low-rank tile (the packed
        # U.Z and stacked V'^T Y products) and m^2 for each dense diagonal tile
        roof_flops = (4.0 * w.tile * float(tlr_ranks.sum()) + (tlr_ld // w.tile) * float(w.tile) ** 2) * N * S
        roof_note = ("achieved = executed flops (4 m sum_ij k_ij + nt m^2) N S of the TLR sweep / event time of "
                     "the mvn_prob call")
    sweep_tf = roof_flops / (r["sov_ms"] * 1e-3) / 1e12
    peak = PEAK_TFLOPS["fp64" if tlr else args.precision]
    wide = not tlr and args.precision == "fp64" and N * S >= 32768
    kernel = ("tlr_sweep_kernel (TLR SOV update + conditioning, 64-row blocks)" if tlr else
              "wide_sweep_kernel (256-row x 128-column FP64 SOV GEMM + conditioning)" if wide else
              "sweep_kernel (SOV GEMM + conditioning)")
    line = {
        "metric": METRIC,
        "value": 1e3 / ms,
        "unit": "MVN probs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if (tlr or args.precision == "fp64") else f"{args.precision}+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: n={n} ({int(math.isqrt(n))}^2 grid"
                               + (", Morton order" if args.workload == "tlr64k" else "") +
                               f"), Matern nu={w.nu}, beta={w.beta}, nugget={w.nugget}, N={N} x S={S} QMC, "
                               + (f"TLR tile {w.tile}, eps={args.tlr_eps:g}, max_rank={args.max_rank}" if tlr
                                  else f"dense {args.precision}, tile {w.tile}"),
                   "n": n, "N": N, "S": S, "tile": w.tile, "precision": "fp64" if tlr else args.precision,
                   "tlr_eps": args.tlr_eps if tlr else None},
        "effective_tflops": (chol_flops + sov_flops) / (ms * 1e-3) / 1e12,
        "conditioning_steps_per_s": n * N * S / (r["sov_ms"] * 1e-3),
        "phase_ms": {"cholesky": r["cholesky_ms"], "sov": r["sov_ms"]},
        "step_ms": {"median": float(sorted(r["wall_ms_steps"])[len(r["wall_ms_steps"]) // 2]),
                    "min": min(r["wall_ms_steps"]), "max": max(r["wall_ms_steps"])},
        "result": {"logP": r["logP"], "P": r["P"], "rel_stderr": r["rel_stderr"], "info": r["info"]},
        "roofline": {"bound": "mfma", "kernel": kernel, "achieved": sweep_tf, "peak": peak, "unit": "TFLOP/s",
                     "frac": sweep_tf / peak,
                     "traffic": _traffic(args.workload) if wide else None,
                     "algorithmic_flops_per_launch": roof_flops,
                     "note": roof_note},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = _cpu_baseline(w)
        print("# cpu baseline done", file=sys.stderr, flush=True)
    if not args.no_variants:
        variants = {}
        headline_dense = args.workload == "tlr64k" and not tlr and args.precision == "fp64"
        jobs = [("precision", lambda: variant_precision(dev)),
                ("autotune", lambda: variant_autotune_dense(workloads.make_workload("prec16k"), dev)),
                ("oracle400", lambda: variant_oracle400(dev)),
                ("tlr64k", lambda: variant_tlr(dev, r if headline_dense else None)),
                ("batch2000", lambda: variant_batch(dev)),
                ("grad4096", lambda: variant_grad(dev)),
                ("crd16k", lambda: variant_crd(dev)),
                ("post40k", lambda: variant_posterior(dev))]
        only = {v for v in args.variants.split(",") if v}
        for job in jobs:
            if job is None or (only and job[0] not in only):
                continue
            name, fn = job
            t0 = time.perf_counter()
            try:
                variants[name] = fn()
            except Exception as e:  # a failed variant is reported, the line is still printed
                variants[name] = {"error": f"{type(e).__name__}: {e}",
                                  "trace": traceback.format_exc(limit=3)}
            variants[name]["bench_seconds"] = time.perf_counter() - t0
            print(f"# variant {name} done ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
            _free()
        line["variants"] = variants
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
