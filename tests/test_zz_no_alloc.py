"""mvn_prob_static (the entry point that allocates nothing: its workspace is
a device array inside the library) against mvn_prob through the C ABI, on
two calls in a row, the second with a smaller problem; the results must be
the same bit for bit (the sweep's per-sample arithmetic does not depend on
how many workgroups run it)."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2405_14892_amd as mvn
from paper_2405_14892_amd import _lib
import workloads

pytestmark = pytest.mark.gpu


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _call_both(f, a, b, mu, N, S, seed, opts):
    h = _lib.lib()
    dev = f.device
    st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    ta, tb = torch.as_tensor(a).to(dev), torch.as_tensor(b).to(dev)
    tm = torch.as_tensor(mu).to(dev) if mu is not None else None
    out_s = torch.full((4 + S,), np.nan, dtype=torch.float64, device=dev)
    ell_s = torch.full((N * S,), np.nan, dtype=torch.float64, device=dev)
    rc = h.mvn_prob_static(ctypes.byref(f.handle), _p(ta), _p(tb), _p(tm), N, S, ctypes.c_uint64(seed),
                           ctypes.byref(opts), _p(out_s), _p(ell_s), st)
    assert rc == 0, h.mvn_last_error().decode()
    wsb = ctypes.c_size_t(0)
    assert h.mvn_prob_workspace_bytes(f.n, N, S, ctypes.byref(opts), ctypes.byref(wsb)) == 0
    ws = torch.empty(wsb.value, dtype=torch.uint8, device=dev)
    out_r = torch.empty(4 + S, dtype=torch.float64, device=dev)
    ell_r = torch.empty(N * S, dtype=torch.float64, device=dev)
    rc = h.mvn_prob(ctypes.byref(f.handle), _p(ta), _p(tb), _p(tm), N, S, ctypes.c_uint64(seed), ctypes.byref(opts),
                    _p(ws), wsb.value, _p(out_r), _p(ell_r), st)
    assert rc == 0, h.mvn_last_error().decode()
    torch.cuda.synchronize()
    return out_s.cpu().numpy(), ell_s.cpu().numpy(), out_r.cpu().numpy(), ell_r.cpu().numpy()


@pytest.mark.parametrize("prec", [mvn.MVN_FP64, mvn.MVN_FP32])
def test_static_entry_point_equals_mvn_prob_twice(prec):
    w = workloads.make_workload("grad4096")
    kern = (w.sigma2, w.beta, w.nu, w.nugget)
    opts = mvn.options(tile=128, precision=prec)
    # three calls in a row, each smaller than the one before: 4096 sites and
    # 66 000 samples (the 128-column FP64 sweep, with fewer workgroups than
    # mvn_prob runs because the scratch holds no more), 1000 sites and 50 000
    # samples (the 64-column sweep), then a small ragged problem
    for n, N, S in ((4096, 33000, 2), (1000, 5000, 10), (700, 333, 3)):
        idx = np.arange(n)
        print(f"static entry point: precision {prec}, n={n}, N={N}, S={S}", flush=True)
        f = mvn.mvn_cholesky(n, locs=w.locs[idx], kern=kern, opts=opts)
        out_s, ell_s, out_r, ell_r = _call_both(f, w.a[idx], w.b[idx], w.mu[idx], N, S, w.seed, opts)
        assert np.all(np.isfinite(ell_r))
        np.testing.assert_array_equal(ell_s, ell_r)
        np.testing.assert_array_equal(out_s, out_r)


def test_static_entry_point_rejects_what_does_not_fit():
    h = _lib.lib()
    w = workloads.make_workload("grad4096")
    f = mvn.mvn_cholesky(64, locs=w.locs[:64], kern=(w.sigma2, w.beta, w.nu, w.nugget), opts=mvn.options(tile=64))
    torch.cuda.synchronize()
    dev = f.device
    st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    a = torch.full((64,), -np.inf, dtype=torch.float64, device=dev)
    b = torch.zeros(64, dtype=torch.float64, device=dev)
    out = torch.empty(4 + 1, dtype=torch.float64, device=dev)
    # 2^28 samples need 2 GiB of per-sample log-products in scratch
    rc = h.mvn_prob_static(ctypes.byref(f.handle), _p(a), _p(b), None, 1 << 28, 1, ctypes.c_uint64(1),
                           ctypes.byref(mvn.options(tile=64)), _p(out), None, st)
    assert rc == -5
    assert "static limit" in h.mvn_last_error().decode()
