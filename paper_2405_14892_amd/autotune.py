"""Autotuner for the library's tile shapes.

The shapes it chooses among are options of the C ABI (include/mvn.h):

* ``sweep_rows`` - rows per block of the dense and batched SOV sweeps: 128
  (two workgroups per CU, the sample block Y read once per 128 rows) or 64
  (three workgroups per CU, so more sample columns are conditioned at once);
* ``tile`` - the Cholesky tile of a dense factorisation (the panel width of
  Algorithm 1's factorisation step), and the tile edge of a tile low-rank
  factor.

Each candidate runs on the device through the library itself, on the
caller's problem, and is timed with HIP events on the current stream; the
fastest is returned together with every measured time.  The factorisation
and the sweep are tuned separately (the tile does not change the sweep and
``sweep_rows`` does not change the factorisation).  Results can be cached in
a JSON file keyed by the device name and the problem class, so that a later
call with the same key returns without timing anything.

The timer is a parameter: ``timer(fn, reps) -> seconds`` runs ``fn`` and
returns its time per call.  The default is HIP events on the current stream
after one untimed call.
"""
from __future__ import annotations

import json
import os
from typing import Callable, Dict, Iterable, Optional

from ._lib import MVN_FP64, options

Timer = Callable[[Callable[[], object], int], float]


def event_timer(fn: Callable[[], object], reps: int) -> float:
    """Seconds per call of ``fn`` from HIP events on the current stream
    (one untimed call first)."""
    import torch
    fn()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        fn()
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def _device_name() -> str:
    try:
        import torch
        return torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"
    except Exception:  # pragma: no cover
        return "none"


class Cache:
    """A JSON file of tuning results: {key: result}."""

    def __init__(self, path: Optional[str]):
        self.path = path
        self.data: Dict[str, dict] = {}
        if path and os.path.exists(path):
            with open(path) as fh:
                self.data = json.load(fh)

    def get(self, key: str) -> Optional[dict]:
        return self.data.get(key)

    def put(self, key: str, value: dict) -> None:
        self.data[key] = value
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(self.data, fh, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


def _argmin(times: Dict[str, float]) -> str:
    return min(sorted(times), key=lambda k: times[k])


def tune_dense(n: int, locs, kern: tuple, a, b, mu=None, N: int = 1000, S: int = 10, seed: int = 1,
               precision: int = MVN_FP64, tiles: Iterable[int] = (128, 256, 512, 1024),
               rows: Iterable[int] = (128, 64), reps: int = 1, device="cuda",
               cache_path: Optional[str] = None, timer: Optional[Timer] = None) -> dict:
    """Cholesky tile and sweep block rows for one dense problem.

    Returns {"tile", "sweep_rows", "cholesky_s": {tile: s}, "sweep_s": {rows: s}, "key"}."""
    from . import mvn_cholesky, mvn_prob, mvn_prob_workspace_bytes
    timer = timer or event_timer
    pad = (n + 127) // 128 * 128
    tiles = [t for t in tiles if t <= max(pad, 128)]
    rows = list(rows)
    key = f"dense:{_device_name()}:n={n}:N={N}:S={S}:prec={precision}:tiles={tiles}:rows={rows}"
    cache = Cache(cache_path)
    hit = cache.get(key)
    if hit is not None:
        return hit
    chol = {}
    for t in tiles:
        o = options(tile=t, precision=precision)
        chol[str(t)] = timer(lambda o=o: mvn_cholesky(n, locs=locs, kern=kern, opts=o, device=device), reps)
    best_tile = int(_argmin(chol))
    # device buffers are made by the first (untimed) call of each candidate
    state = {}

    def factor():
        if "f" not in state:
            state["f"] = mvn_cholesky(n, locs=locs, kern=kern, opts=options(tile=best_tile, precision=precision),
                                      device=device)
        return state["f"]

    sweep = {}
    for r in rows:
        o = options(tile=best_tile, precision=precision, sweep_rows=r)

        def run(o=o, r=r):
            if r not in state:
                state[r] = _workspace(mvn_prob_workspace_bytes(n, N, S, o), device)
            return mvn_prob(factor(), a, b, mu, N=N, S=S, seed=seed, opts=o, workspace=state[r])

        sweep[str(r)] = timer(run, reps)
        state.pop(r, None)
    res = {"tile": best_tile, "sweep_rows": int(_argmin(sweep)), "cholesky_s": chol, "sweep_s": sweep, "key": key}
    cache.put(key, res)
    return res


def tune_batch(sizes, idx, locs, kern: tuple, a, b, mu=None, N: int = 1000, S: int = 8, seed: int = 1,
               precision: int = MVN_FP64, rows: Iterable[int] = (128, 64), reps: int = 1, device="cuda",
               cache_path: Optional[str] = None, timer: Optional[Timer] = None) -> dict:
    """Sweep block rows for a batch of uneven problems (the whole enqueue
    sequence of mvn_prob_batch is timed).

    Returns {"sweep_rows", "batch_s": {rows: s}, "key"}."""
    import numpy as np
    from . import mvn_batch_plan, mvn_prob_batch
    timer = timer or event_timer
    sizes = np.asarray(sizes, dtype=np.int32)
    rows = list(rows)
    hist = np.bincount(np.minimum(np.log2(np.maximum(sizes, 1)).astype(int), 16), minlength=17)
    key = (f"batch:{_device_name()}:count={sizes.size}:sizes_log2_hist={hist.tolist()}:N={N}:S={S}:"
           f"prec={precision}:rows={rows}")
    cache = Cache(cache_path)
    hit = cache.get(key)
    if hit is not None:
        return hit
    times = {}
    for r in rows:
        state = {}

        def run(r=r, state=state):
            if "plan" not in state:
                state["plan"] = mvn_batch_plan(sizes, N, S, options(tile=128, precision=precision, sweep_rows=r),
                                               device=device)
            return mvn_prob_batch(state["plan"], idx, locs, kern, a, b, mu, seed=seed)

        times[str(r)] = timer(run, reps)
        state.clear()
    res = {"sweep_rows": int(_argmin(times)), "batch_s": times, "key": key}
    cache.put(key, res)
    return res


def tune_tlr(n: int, locs, kern: tuple, a, b, mu=None, N: int = 1000, S: int = 10, seed: int = 1,
             tlr_eps: float = 1e-5, max_rank: int = 256, tiles: Iterable[int] = (512, 1024), reps: int = 1,
             device="cuda", cache_path: Optional[str] = None, timer: Optional[Timer] = None) -> dict:
    """Tile edge of a tile low-rank factor: factorisation + sweep time per
    candidate (the tile changes both).

    Returns {"tile", "total_s": {tile: s}, "key"}."""
    from . import mvn_cholesky, mvn_prob, mvn_prob_workspace_bytes_factor
    timer = timer or event_timer
    tiles = [t for t in tiles if t % 128 == 0 and t <= 1024 and max_rank <= min(256, t)]
    key = f"tlr:{_device_name()}:n={n}:N={N}:S={S}:eps={tlr_eps:g}:rank={max_rank}:tiles={tiles}"
    cache = Cache(cache_path)
    hit = cache.get(key)
    if hit is not None:
        return hit
    times = {}
    for t in tiles:
        o = options(tile=t, tlr_eps=tlr_eps, max_rank=max_rank)
        state = {}

        def run(o=o, state=state):
            f = mvn_cholesky(n, locs=locs, kern=kern, opts=o, device=device)
            if "ws" not in state:  # sized for the ranks of the first (untimed) factorisation
                state["ws"] = _workspace(mvn_prob_workspace_bytes_factor(f, N, S, o), device)
            return mvn_prob(f, a, b, mu, N=N, S=S, seed=seed, opts=o, workspace=state["ws"])

        times[str(t)] = timer(run, reps)
        state.clear()
    res = {"tile": int(_argmin(times)), "total_s": times, "key": key}
    cache.put(key, res)
    return res


def _workspace(nbytes: int, device):
    import torch
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


__all__ = ["tune_dense", "tune_batch", "tune_tlr", "event_timer", "Cache"]
