"""The autotuner's selection and cache logic on the CPU, with an injected
timer (no device): the fastest candidate wins, every candidate's time is
reported, and a cached key returns without timing again.  The GPU run of
the tuner is in tests/test_gpu_autotune.py."""
import json

import numpy as np

from paper_2405_14892_amd import autotune


class FakeTimer:
    def __init__(self, times):
        self.times = list(times)
        self.calls = 0

    def __call__(self, fn, reps):
        self.calls += 1
        return self.times.pop(0)


def test_dense_picks_fastest_tile_and_rows(tmp_path):
    timer = FakeTimer([0.30, 0.20, 0.25, 0.40,   # Cholesky tiles 128, 256, 512, 1024
                       1.00, 0.90])              # sweep rows 128, 64
    path = str(tmp_path / "tune.json")
    res = autotune.tune_dense(2000, None, (1, 0.1, 0.5, 0), None, None, N=100, S=2, cache_path=path, timer=timer)
    assert res["tile"] == 256 and res["sweep_rows"] == 64
    assert set(res["cholesky_s"]) == {"128", "256", "512", "1024"} and set(res["sweep_s"]) == {"128", "64"}
    again = autotune.tune_dense(2000, None, (1, 0.1, 0.5, 0), None, None, N=100, S=2, cache_path=path,
                                timer=FakeTimer([]))
    assert again == res
    assert json.load(open(path))[res["key"]]["tile"] == 256


def test_dense_drops_tiles_larger_than_the_problem():
    timer = FakeTimer([0.1, 0.2, 0.5, 0.3])
    res = autotune.tune_dense(200, None, None, None, None, tiles=(128, 256, 512), rows=(128, 64), timer=timer)
    assert set(res["cholesky_s"]) == {"128", "256"}   # 512 > padded n = 256
    assert res["tile"] == 128 and res["sweep_rows"] == 64


def test_batch_and_tlr_selection(tmp_path):
    sizes = np.array([50, 400, 4000, 70], dtype=np.int32)
    res = autotune.tune_batch(sizes, None, None, None, None, None, timer=FakeTimer([2.0, 1.5]))
    assert res["sweep_rows"] == 64 and res["batch_s"] == {"128": 2.0, "64": 1.5}
    res = autotune.tune_tlr(65536, None, None, None, None, timer=FakeTimer([3.0, 2.5]))
    assert res["tile"] == 1024
    # a rank cap above the smaller tile removes it
    res = autotune.tune_tlr(65536, None, None, None, None, max_rank=256, tiles=(128, 1024),
                            timer=FakeTimer([2.5]))
    assert res["total_s"] == {"1024": 2.5}
