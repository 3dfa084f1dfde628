"""MI355X (gfx950) separation-of-variables MVN probabilities.

Python face of libmvn.so: the functions carry the C entry points' names and
only marshal torch tensors (device memory, current HIP stream) into the C
ABI declared in include/mvn.h.  The estimator is Genz's separation of
variables with randomised Richtmyer QMC, as parallelised in arXiv 2405.14892
(Algorithms 1-3).
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

from . import _lib
from ._lib import (MVN_BF16, MVN_BF16X3, MVN_CHOL_ADAPTIVE, MVN_CHOL_FP64, MVN_CHOL_UNIFORM,  # noqa: F401
                   MVN_FACTOR_TLR, MVN_FP32, MVN_FP64, MvnError, MvnFactor, MvnMatern, MvnOptions, options)

__all__ = ["mvn_factor_bytes", "mvn_cholesky_workspace_bytes", "mvn_prob_workspace_bytes",
           "mvn_prob_workspace_bytes_factor", "mvn_cholesky", "mvn_prob", "mvn_prob_static", "Factor",
           "mvn_prob_prefix_workspace_bytes", "mvn_prob_prefix", "confidence_region",
           "mvn_mc_prefix_workspace_bytes", "mvn_mc_prefix", "mvn_cholesky_permuted", "mvn_tlr_dense", "mvn_tlr_compact", "mvn_exceedance_order", "mvn_posterior",
           "posterior_confidence_region",
           "mvn_prob_grad_workspace_bytes", "mvn_prob_grad", "MVNLogProb", "BatchPlan",
           "mvn_batch_plan", "mvn_prob_batch",
           "options", "MvnError", "MVN_FP64", "MVN_FP32", "MVN_BF16", "MVN_BF16X3", "MVN_CHOL_ADAPTIVE",
           "MVN_CHOL_UNIFORM", "MVN_CHOL_FP64", "library_path"]


def library_path() -> str:
    return _lib.LIB_PATH


def _torch():
    import torch
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev_f64(x, device):
    torch = _torch()
    t = torch.as_tensor(x, dtype=torch.float64)
    return t.to(device).contiguous()


def mvn_factor_bytes(n: int, opts: MvnOptions | None = None) -> int:
    out = ctypes.c_size_t(0)
    _lib.check(_lib.lib().mvn_factor_bytes(n, ctypes.byref(opts or options()), ctypes.byref(out)))
    return out.value


def mvn_cholesky_workspace_bytes(n: int, opts: MvnOptions | None = None) -> int:
    out = ctypes.c_size_t(0)
    _lib.check(_lib.lib().mvn_cholesky_workspace_bytes(n, ctypes.byref(opts or options()), ctypes.byref(out)))
    return out.value


def mvn_prob_workspace_bytes(n: int, N: int, S: int, opts: MvnOptions | None = None) -> int:
    out = ctypes.c_size_t(0)
    _lib.check(_lib.lib().mvn_prob_workspace_bytes(n, N, S, ctypes.byref(opts or options()),
                                                   ctypes.byref(out)))
    return out.value


def mvn_prob_workspace_bytes_factor(f: "Factor", N: int, S: int, opts: MvnOptions | None = None) -> int:
    """Workspace of mvn_prob for this factor (for a TLR factor the ranks are
    read back, which synchronises the current stream)."""
    out = ctypes.c_size_t(0)
    _lib.check(_lib.lib().mvn_prob_workspace_bytes_factor(ctypes.byref(f.handle), N, S, ctypes.byref(opts or options()),
                                                          ctypes.byref(out), _stream(f.device)))
    return out.value


@dataclass
class Factor:
    """Handle from mvn_cholesky plus the device buffer that backs it."""
    handle: MvnFactor
    buffer: object  # torch uint8 tensor on the device
    device: object

    @property
    def n(self) -> int:
        return self.handle.n

    @property
    def ld(self) -> int:
        return self.handle.ld

    @property
    def is_tlr(self) -> bool:
        return bool(self.handle.flags & MVN_FACTOR_TLR)

    @property
    def is_compact(self) -> bool:
        return bool(self.handle.flags & _lib.MVN_FACTOR_TLR_COMPACT)

    def nbytes(self) -> int:
        """Bytes of the device buffer that holds the factor."""
        return self.buffer.numel()

    def _view(self, ptr: int, count: int, dtype):
        torch = _torch()
        off = ptr - self.buffer.data_ptr()
        size = torch.empty((), dtype=dtype).element_size()
        return self.buffer[off: off + count * size].view(dtype)

    def L(self):
        """Dense factor as an n x n float64 tensor view (lower triangular)."""
        torch = _torch()
        if self.is_tlr:
            raise MvnError(-1, "a TLR factor has no dense L; use tiles(), U(), Vt(), ranks()")
        ld = self.handle.ld
        return self._view(self.handle.L, ld * ld, torch.float64).view(ld, ld)[: self.n, : self.n]

    def info(self) -> int:
        torch = _torch()
        owner = getattr(self, "_info_owner", None) or self  # a dense form shares its TLR factor's info
        return int(owner._view(self.handle.info, 1, torch.int32).item())

    def update_counts(self) -> dict:
        """Trailing tile updates by arithmetic (dense factors; the adaptive
        precision map's choices, all zero in the other modes)."""
        torch = _torch()
        if self.is_tlr or not self.handle.update_counts:
            return {"fp64": 0, "fp32": 0, "reduced": 0}
        c = self._view(self.handle.update_counts, 3, torch.int64).cpu().tolist()
        return {"fp64": c[0], "fp32": c[1], "reduced": c[2]}

    # ---- tile low-rank buffers (raw device views, layouts as in mvn.h)
    @property
    def nt(self) -> int:
        return self.handle.ld // self.handle.tile if self.is_tlr else 0

    def tiles(self):
        """(nt(nt+1)/2, m, m) float64: tile (i, j), j <= i, at i(i+1)/2 + j."""
        torch = _torch()
        m, nt = self.handle.tile, self.nt
        cnt = nt * (nt + 1) // 2
        return self._view(self.handle.L, cnt * m * m, torch.float64).view(cnt, m, m)

    def U(self):
        """(nt(nt-1)/2, m, rs) float64: panel (i, k), k < i, at i(i-1)/2 + k."""
        torch = _torch()
        m, nt, rs = self.handle.tile, self.nt, self.handle.rank_stride
        cnt = nt * (nt - 1) // 2
        return self._view(self.handle.U, cnt * m * rs, torch.float64).view(cnt, m, rs)

    def Vt(self):
        """(nt(nt-1)/2, rs, m) float64 with L_ik = U_ik Vt_ik."""
        torch = _torch()
        m, nt, rs = self.handle.tile, self.nt, self.handle.rank_stride
        cnt = nt * (nt - 1) // 2
        return self._view(self.handle.Vt, cnt * rs * m, torch.float64).view(cnt, rs, m)

    def ranks(self):
        """(nt(nt-1)/2,) int32 ranks (negative: capped by max_rank)."""
        torch = _torch()
        nt = self.nt
        return self._view(self.handle.ranks, max(nt * (nt - 1) // 2, 1), torch.int32)[: nt * (nt - 1) // 2]


def mvn_cholesky(n: int, sigma=None, locs=None, kern: tuple | None = None,
                 opts: MvnOptions | None = None, device="cuda") -> Factor:
    """Factor Sigma (device n x n) or the Matern covariance of ``locs``
    (n x 2) with ``kern = (sigma2, beta, nu, nugget)``."""
    torch = _torch()
    opts = opts or options()
    fb = mvn_factor_bytes(n, opts)
    wb = mvn_cholesky_workspace_bytes(n, opts)
    buf = torch.empty(fb, dtype=torch.uint8, device=device)
    ws = torch.empty(wb, dtype=torch.uint8, device=device) if wb else None
    s = _dev_f64(sigma, device) if sigma is not None else None
    lc = _dev_f64(locs, device) if locs is not None else None
    km = MvnMatern(*kern) if kern is not None else None
    h = MvnFactor()
    code = _lib.lib().mvn_cholesky(
        n, _ptr(s), n if s is not None else 0, _ptr(lc), ctypes.byref(km) if km else None,
        ctypes.byref(opts), _ptr(buf), fb, _ptr(ws), wb, ctypes.byref(h), _stream(device))
    _lib.check(code)
    f = Factor(h, buf, device)
    f._keep = (s, lc, ws)  # inputs and workspace must outlive the asynchronous launch
    return f


def mvn_tlr_compact(f: Factor) -> Factor:
    """The TLR factor ``f`` with its storage cut to the ranks: the diagonal
    tiles and U, V'^T packed at the actual ranks (reads the ranks back, which
    synchronises the current stream).  The result owns its own buffer; f
    may be dropped afterwards."""
    torch = _torch()
    if not f.is_tlr or f.is_compact:
        raise MvnError(-1, "not a full TLR factor")
    nb = ctypes.c_size_t(0)
    _lib.check(_lib.lib().mvn_tlr_compact_bytes(ctypes.byref(f.handle), ctypes.byref(nb), _stream(f.device)))
    buf = torch.empty(nb.value, dtype=torch.uint8, device=f.device)
    h = MvnFactor()
    _lib.check(_lib.lib().mvn_tlr_compact(ctypes.byref(f.handle), _ptr(buf), nb.value, ctypes.byref(h),
                                          _stream(f.device)))
    return Factor(h, buf, f.device)


def mvn_tlr_dense(f: Factor) -> Factor:
    """The TLR factor ``f`` written out as a dense FP64 factor (diagonal
    tiles copied, L_ij = U_ij V'^T_ij below them), for the dense SOV sweep
    after a TLR factorisation (the configuration of Section IV-C).  The
    result shares f's info and keeps f alive."""
    torch = _torch()
    if not f.is_tlr:
        raise MvnError(-1, "not a TLR factor")
    nb = ctypes.c_size_t(0)
    _lib.check(_lib.lib().mvn_tlr_dense_bytes(ctypes.byref(f.handle), ctypes.byref(nb)))
    buf = torch.empty(nb.value, dtype=torch.uint8, device=f.device)
    h = MvnFactor()
    _lib.check(_lib.lib().mvn_tlr_dense(ctypes.byref(f.handle), _ptr(buf), nb.value, ctypes.byref(h),
                                        _stream(f.device)))
    d = Factor(h, buf, f.device)
    d._keep = (f,)
    d._info_owner = f
    return d


def mvn_cholesky_permuted(sigma, perm, opts: MvnOptions | None = None) -> Factor:
    """Factor of P Sigma P^T (row i = site perm[i]) from the lower triangle
    of ``sigma``: a float64 device tensor n x n with unit column stride (any
    row stride, e.g. the posterior's view into its workspace)."""
    import numpy as np
    torch = _torch()
    opts = opts or options()
    n = sigma.shape[0]
    if sigma.dtype != torch.float64 or sigma.stride(1) != 1 or sigma.shape[1] != n:
        raise MvnError(-2, "sigma must be a float64 n x n tensor with unit column stride")
    dev = sigma.device
    if isinstance(perm, torch.Tensor) and perm.device == dev and perm.dtype == torch.int64:
        dp = perm.contiguous()  # a device order (mvn_exceedance_order) is used as it is, no read-back
    else:
        dp = torch.as_tensor(np.asarray(perm.cpu() if hasattr(perm, "cpu") else perm, dtype=np.int64)).to(dev)
    if dp.shape != (n,):
        raise MvnError(-4, "perm must have n entries")
    fb = mvn_factor_bytes(n, opts)
    wb = ctypes.c_size_t(0)
    _lib.check(_lib.lib().mvn_cholesky_permuted_workspace_bytes(n, ctypes.byref(opts), ctypes.byref(wb)))
    buf = torch.empty(fb, dtype=torch.uint8, device=dev)
    ws = torch.empty(wb.value, dtype=torch.uint8, device=dev)
    h = MvnFactor()
    code = _lib.lib().mvn_cholesky_permuted(n, _ptr(sigma), sigma.stride(0), _ptr(dp),
                                            ctypes.byref(opts), _ptr(buf), fb, _ptr(ws), wb.value, ctypes.byref(h),
                                            _stream(dev))
    _lib.check(code)
    f = Factor(h, buf, dev)
    f._keep = (sigma, ws, dp)
    return f


def mvn_posterior(locs, kern: tuple, obs, y, noise_var: float, mu=None, opts: MvnOptions | None = None,
                  device="cuda") -> dict:
    """Posterior of the field N(mu, Sigma(locs; kern)) given y = x[obs] +
    N(0, noise_var) (Section V-B).  Returns device tensors ``mu_post``,
    ``var_post``, ``sigma_post`` (n x n view of the lower triangle, valid as
    long as the returned dict is kept) and the host int ``info``."""
    import numpy as np
    torch = _torch()
    opts = opts or options()
    lc = _dev_f64(locs, device)
    n = lc.shape[0]
    do = torch.as_tensor(np.ascontiguousarray(np.asarray(obs, dtype=np.int64))).to(device)
    m = do.numel()
    ty = _dev_f64(y, device)
    tm = _dev_f64(mu, device) if mu is not None else None
    wb = ctypes.c_size_t(0)
    _lib.check(_lib.lib().mvn_posterior_workspace_bytes(n, m, ctypes.byref(opts), ctypes.byref(wb)))
    ws = torch.empty((wb.value + 7) // 8 * 8, dtype=torch.uint8, device=device)
    mu_post = torch.empty(n, dtype=torch.float64, device=device)
    var_post = torch.empty(n, dtype=torch.float64, device=device)
    info = torch.empty(1, dtype=torch.int32, device=device)
    sp_ptr, ld = ctypes.c_void_p(0), ctypes.c_int(0)
    km = MvnMatern(*kern)
    code = _lib.lib().mvn_posterior(n, _ptr(lc), _ptr(tm), m, _ptr(do), _ptr(ty),
                                    ctypes.byref(km), float(noise_var), ctypes.byref(opts), _ptr(ws), wb.value,
                                    _ptr(mu_post), _ptr(var_post), _ptr(info), ctypes.byref(sp_ptr),
                                    ctypes.byref(ld), _stream(device))
    _lib.check(code)
    off = sp_ptr.value - ws.data_ptr()
    assert off % 8 == 0
    flat = ws.view(torch.float64)
    sigma_post = flat[off // 8: off // 8 + (n - 1) * ld.value + n].as_strided((n, n), (ld.value, 1))
    return {"mu_post": mu_post, "var_post": var_post, "sigma_post": sigma_post,
            "info": int(info.item()), "_keep": (lc, ty, tm, ws, do)}


def mvn_prob(f: Factor, a, b, mu=None, N: int = 1000, S: int = 10, seed: int = 1,
             opts: MvnOptions | None = None, return_ell: bool = False, workspace=None):
    """SOV estimate of P(a <= X <= b).  Returns a dict of device tensors:
    logP, P, stderr, rel_stderr, logP_s[S] (and ell[N*S] if asked).
    For a TLR factor a given workspace is used as it is (sizing one reads the
    ranks back; the call itself does not, so it can be graph-captured)."""
    torch = _torch()
    opts = opts or options()
    dev = f.device
    ta, tb = _dev_f64(a, dev), _dev_f64(b, dev)
    tm = _dev_f64(mu, dev) if mu is not None else None
    if f.is_tlr and workspace is not None:
        wsb = workspace.numel()
    else:
        wsb = (mvn_prob_workspace_bytes_factor(f, N, S, opts) if f.is_tlr
               else mvn_prob_workspace_bytes(f.n, N, S, opts))
        if workspace is None or workspace.numel() < wsb:
            workspace = torch.empty(wsb, dtype=torch.uint8, device=dev)
    out = torch.empty(4 + S, dtype=torch.float64, device=dev)
    ell = torch.empty(N * S, dtype=torch.float64, device=dev) if return_ell else None
    code = _lib.lib().mvn_prob(ctypes.byref(f.handle), _ptr(ta), _ptr(tb), _ptr(tm), N, S,
                               ctypes.c_uint64(seed), ctypes.byref(opts), _ptr(workspace), wsb,
                               _ptr(out), _ptr(ell), _stream(dev))
    _lib.check(code)
    res = {"logP": out[0], "P": out[1], "stderr": out[2], "rel_stderr": out[3], "logP_s": out[4:],
           "out": out, "_keep": (ta, tb, tm, workspace)}
    if return_ell:
        res["ell"] = ell
    return res


def mvn_prob_static(f: Factor, a, b, mu=None, N: int = 1000, S: int = 10, seed: int = 1,
                    opts: MvnOptions | None = None, return_ell: bool = False):
    """mvn_prob with the workspace inside the library (no device allocation
    by the library; the outputs are still the caller's tensors).  Same
    results as mvn_prob."""
    torch = _torch()
    opts = opts or options()
    dev = f.device
    ta, tb = _dev_f64(a, dev), _dev_f64(b, dev)
    tm = _dev_f64(mu, dev) if mu is not None else None
    out = torch.empty(4 + S, dtype=torch.float64, device=dev)
    ell = torch.empty(N * S, dtype=torch.float64, device=dev) if return_ell else None
    code = _lib.lib().mvn_prob_static(ctypes.byref(f.handle), _ptr(ta), _ptr(tb), _ptr(tm), N, S,
                                      ctypes.c_uint64(seed), ctypes.byref(opts), _ptr(out), _ptr(ell), _stream(dev))
    _lib.check(code)
    res = {"logP": out[0], "P": out[1], "stderr": out[2], "rel_stderr": out[3], "logP_s": out[4:],
           "out": out, "_keep": (ta, tb, tm)}
    if return_ell:
        res["ell"] = ell
    return res


def mvn_prob_prefix_workspace_bytes(f: Factor, N: int, S: int, opts: MvnOptions | None = None) -> int:
    """Workspace of mvn_prob_prefix for this factor (for a TLR factor the
    ranks are read back, which synchronises the current stream)."""
    out = ctypes.c_size_t(0)
    _lib.check(_lib.lib().mvn_prob_prefix_workspace_bytes(ctypes.byref(f.handle), N, S, ctypes.byref(opts or options()),
                                                          ctypes.byref(out), _stream(f.device)))
    return out.value


def mvn_prob_prefix(f: Factor, a, b, mu=None, N: int = 1000, S: int = 10, seed: int = 1,
                    opts: MvnOptions | None = None, workspace=None):
    """log P-hat of the first k sites, k = 1..n, from one sweep (the
    nested sets of confidence-region detection; sites in the factor's order).
    Returns a dict of device tensors: logP[n], rel_stderr[n]."""
    torch = _torch()
    opts = opts or options()
    dev = f.device
    ta, tb = _dev_f64(a, dev), _dev_f64(b, dev)
    tm = _dev_f64(mu, dev) if mu is not None else None
    wsb = mvn_prob_prefix_workspace_bytes(f, N, S, opts)
    if workspace is None or workspace.numel() < wsb:
        workspace = torch.empty(wsb, dtype=torch.uint8, device=dev)
    out = torch.empty(2 * f.n, dtype=torch.float64, device=dev)
    code = _lib.lib().mvn_prob_prefix(ctypes.byref(f.handle), _ptr(ta), _ptr(tb), _ptr(tm), N, S,
                                      ctypes.c_uint64(seed), ctypes.byref(opts), _ptr(workspace), wsb, _ptr(out),
                                      _stream(dev))
    _lib.check(code)
    return {"logP": out[0::2], "rel_stderr": out[1::2], "out": out, "_keep": (ta, tb, tm, workspace)}


def mvn_mc_prefix_workspace_bytes(n: int, M: int, opts: MvnOptions | None = None) -> int:
    out = ctypes.c_size_t(0)
    _lib.check(_lib.lib().mvn_mc_prefix_workspace_bytes(n, M, ctypes.byref(opts or options()), ctypes.byref(out)))
    return out.value


def mvn_mc_prefix(f: Factor, a, b, mu=None, M: int = 50000, seed: int = 1, opts: MvnOptions | None = None,
                  workspace=None, return_first: bool = True):
    """Monte Carlo check of the nested sets: M fields X = mu + L Z, per
    sample the first site outside [a, b] (n if none), per prefix k the
    number of samples inside on the first k sites.  Returns a dict of device
    tensors: count[n] (int64), first[M] (int32, if asked)."""
    torch = _torch()
    opts = opts or options()
    dev = f.device
    ta, tb = _dev_f64(a, dev), _dev_f64(b, dev)
    tm = _dev_f64(mu, dev) if mu is not None else None
    wsb = mvn_mc_prefix_workspace_bytes(f.n, M, opts)
    if workspace is None or workspace.numel() < wsb:
        workspace = torch.empty(wsb, dtype=torch.uint8, device=dev)
    count = torch.empty(f.n, dtype=torch.int64, device=dev)
    first = torch.empty(M, dtype=torch.int32, device=dev) if return_first else None
    code = _lib.lib().mvn_mc_prefix(ctypes.byref(f.handle), _ptr(ta), _ptr(tb), _ptr(tm), M, ctypes.c_uint64(seed),
                                    ctypes.byref(opts), _ptr(workspace), wsb, _ptr(first), _ptr(count),
                                    _stream(dev))
    _lib.check(code)
    return {"count": count, "first": first, "_keep": (ta, tb, tm, workspace)}


def confidence_region(locs, kern: tuple, mu, u: float, alpha: float = 0.05, N: int = 1000, S: int = 10,
                      seed: int = 1, opts: MvnOptions | None = None, device="cuda", mc_samples: int = 0,
                      mc_seed: int = 2):
    """Positive excursion set of a Gaussian field at level u with joint
    probability >= 1 - alpha (Section III-C with Algorithm 1 of Section IV-A): the sites in order
    of decreasing marginal exceedance probability P(X_i > u), the factor of
    Sigma in that order, and one nested-set sweep of the event X_i > u.
    The excursion function of the k-th site in that order is P-hat of the
    first k sites; the region is the longest prefix whose P-hat >= 1 - alpha.
    kern = (sigma2, beta, nu, nugget).  Returns a dict with ``order``,
    ``logP`` (per prefix), ``excursion`` (per site, in the caller's site
    order) and ``region`` (site indices).  With mc_samples > 0 the region
    is checked by direct sampling of the fitted distribution (Section V-C;
    through the dense factor of the same ordered Sigma, also when the
    regions came from a TLR factor): ``mc_p`` is the fraction of sampled fields above u on
    the first k sites, per k, and ``mc_p_region`` that fraction for the
    region, expected near 1 - alpha."""
    import numpy as np
    from scipy.special import ndtr
    sigma2, beta, nu, nugget = kern
    locs = np.asarray(locs, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    n = len(mu)
    sd = math.sqrt(sigma2 + nugget)
    order = np.argsort(-ndtr((mu - u) / sd), kind="stable")
    opts = opts or options()
    f = mvn_cholesky(n, locs=locs[order], kern=kern, opts=opts, device=device)
    r = mvn_prob_prefix(f, np.full(n, float(u)), np.full(n, np.inf), mu[order], N=N, S=S, seed=seed, opts=opts)
    logp = r["logP"].cpu().numpy()
    excursion = np.empty(n)
    excursion[order] = np.exp(logp)
    k = int(np.sum(np.exp(logp) >= 1.0 - alpha))  # the prefixes do not increase
    out = {"order": order, "logP": logp, "rel_stderr": r["rel_stderr"].cpu().numpy(), "excursion": excursion,
           "region": np.sort(order[:k]), "info": f.info()}
    if mc_samples > 0:
        # the check samples the fitted distribution itself: through the dense factor of the same
        # ordered Sigma when the regions came from a TLR factor
        fm = f if not f.is_tlr else mvn_cholesky(n, locs=locs[order], kern=kern, opts=options(tile=opts.tile),
                                                 device=device)
        m = mvn_mc_prefix(fm, np.full(n, float(u)), np.full(n, np.inf), mu[order], M=mc_samples, seed=mc_seed,
                          opts=options(tile=opts.tile), return_first=False)
        p = m["count"].cpu().numpy() / float(mc_samples)
        out["mc_p"] = p
        out["mc_p_region"] = float(p[k - 1]) if k > 0 else 1.0
    return out


def mvn_exceedance_order(mu, var, u: float, device="cuda"):
    """Sites by decreasing marginal exceedance probability Phi((mu - u) /
    sqrt(var)), ties by index (Algorithm 1's order), computed on the device.
    Returns device tensors (perm int64, p float64 in site order)."""
    torch = _torch()
    tm = _dev_f64(mu, device)
    tv = _dev_f64(var, device)
    n = tm.numel()
    if tv.numel() != n:
        raise MvnError(-3, "mu and var must have the same length")
    wb = ctypes.c_size_t(0)
    _lib.check(_lib.lib().mvn_exceedance_order_workspace_bytes(n, ctypes.byref(wb)))
    ws = torch.empty(wb.value, dtype=torch.uint8, device=tm.device)
    perm = torch.empty(n, dtype=torch.int64, device=tm.device)
    p = torch.empty(n, dtype=torch.float64, device=tm.device)
    _lib.check(_lib.lib().mvn_exceedance_order(n, _ptr(tm), _ptr(tv), float(u), _ptr(perm), _ptr(p), _ptr(ws),
                                               wb.value, _stream(tm.device)))
    perm._keep = (tm, tv, ws)
    return perm, p


def posterior_confidence_region(locs, kern: tuple, obs, y, noise_var: float, u: float, alpha: float = 0.05,
                                mu=None, N: int = 1000, S: int = 10, seed: int = 1,
                                opts: MvnOptions | None = None, device="cuda", mc_samples: int = 0,
                                mc_seed: int = 2) -> dict:
    """Algorithm 1 on the posterior of Section V-B: Sigma_post and mu_post
    from the observations, the sites ordered by decreasing posterior
    marginal exceedance probability of u, the factor of Sigma_post in that
    order (dense, or TLR with opts.tlr_eps > 0), one nested-set sweep, and
    optionally the Monte Carlo check (through the dense factor).  Returns the keys of
    confidence_region plus ``mu_post`` and ``sd_post`` (caller's order)."""
    import numpy as np
    torch = _torch()
    opts = opts or options()
    po = options(tile=opts.tile)  # the posterior itself is FP64 and dense
    post = mvn_posterior(locs, kern, obs, y, noise_var, mu=mu, opts=po, device=device)
    if post["info"] != 0:
        raise MvnError(-7, f"observation covariance not positive definite (pivot {post['info']})")
    n = post["mu_post"].numel()
    # the order, the permuted factor and the nested-set sweep stay on the device
    dorder, dpm = mvn_exceedance_order(post["mu_post"], post["var_post"], u, device=device)
    f = mvn_cholesky_permuted(post["sigma_post"], dorder, opts=opts)
    dmo = post["mu_post"][dorder]
    r = mvn_prob_prefix(f, torch.full((n,), float(u), dtype=torch.float64, device=dmo.device),
                        torch.full((n,), float("inf"), dtype=torch.float64, device=dmo.device), dmo, N=N, S=S,
                        seed=seed, opts=opts)
    logp = r["logP"].cpu().numpy()
    order = dorder.cpu().numpy()
    pm = dpm.cpu().numpy()
    mu_post = post["mu_post"].cpu().numpy()
    sd_post = np.sqrt(np.maximum(post["var_post"].cpu().numpy(), 0.0))
    mo = mu_post[order]
    excursion = np.empty(n)
    excursion[order] = np.exp(logp)
    k = int(np.sum(np.exp(logp) >= 1.0 - alpha))
    out = {"order": order, "logP": logp, "rel_stderr": r["rel_stderr"].cpu().numpy(), "excursion": excursion,
           "region": np.sort(order[:k]), "info": f.info(), "mu_post": mu_post, "sd_post": sd_post,
           "marginal": pm}
    if mc_samples > 0:
        fm = f if not f.is_tlr else mvn_cholesky_permuted(post["sigma_post"], order, opts=options(tile=opts.tile))
        m = mvn_mc_prefix(fm, np.full(n, float(u)), np.full(n, np.inf), mo, M=mc_samples, seed=mc_seed,
                          opts=options(tile=opts.tile), return_first=False)
        p = m["count"].cpu().numpy() / float(mc_samples)
        out["mc_p"] = p
        out["mc_p_region"] = float(p[k - 1]) if k > 0 else 1.0
    return out


def mvn_prob_grad_workspace_bytes(n: int, N: int, S: int, opts: MvnOptions | None = None) -> int:
    out = ctypes.c_size_t(0)
    _lib.check(_lib.lib().mvn_prob_grad_workspace_bytes(n, N, S, ctypes.byref(opts or options()),
                                                        ctypes.byref(out)))
    return out.value


def mvn_prob_grad(f: Factor, a, b, mu=None, N: int = 1000, S: int = 1, seed: int = 1,
                  opts: MvnOptions | None = None):
    """log P-hat and its gradient w.r.t. a, b, mu at fixed QMC points.
    Returns a dict of device tensors: logP, P, out[4+S], da, db, dmu."""
    torch = _torch()
    opts = opts or options()
    dev = f.device
    ta, tb = _dev_f64(a, dev), _dev_f64(b, dev)
    tm = _dev_f64(mu, dev) if mu is not None else None
    wsb = mvn_prob_grad_workspace_bytes(f.n, N, S, opts)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    out = torch.empty(4 + S, dtype=torch.float64, device=dev)
    da = torch.empty(f.n, dtype=torch.float64, device=dev)
    db = torch.empty(f.n, dtype=torch.float64, device=dev)
    dmu = torch.empty(f.n, dtype=torch.float64, device=dev)
    code = _lib.lib().mvn_prob_grad(ctypes.byref(f.handle), _ptr(ta), _ptr(tb), _ptr(tm), N, S,
                                    ctypes.c_uint64(seed), ctypes.byref(opts), _ptr(ws), wsb, _ptr(out),
                                    _ptr(da), _ptr(db), _ptr(dmu), _stream(dev))
    _lib.check(code)
    return {"logP": out[0], "P": out[1], "out": out, "da": da, "db": db, "dmu": dmu,
            "_keep": (ta, tb, tm, ws)}


def _make_autograd():
    torch = _torch()

    class MVNLogProb(torch.autograd.Function):
        """log P(a <= X <= b), X ~ N(mu, L L^T), as a differentiable function
        of (a, b, mu) at fixed QMC points.  When a gradient is needed, forward
        calls mvn_prob_grad (the adjoint sweep runs with the forward sweep, on
        the same points) and saves the gradients, which backward scales by
        the incoming gradient; otherwise it runs only the forward sweep
        (mvn_prob).  `opts` selects the arithmetic of the sweep's GEMMs (the
        factor's precision or FP64)."""

        @staticmethod
        def forward(ctx, a, b, mu, factor, N, S, seed, opts=None):
            if not any(ctx.needs_input_grad[:3]):
                r = mvn_prob(factor, a.detach(), b.detach(), mu.detach(), N=N, S=S, seed=seed, opts=opts)
                return r["logP"].clone().to(a.dtype)
            r = mvn_prob_grad(factor, a.detach(), b.detach(), mu.detach(), N=N, S=S, seed=seed, opts=opts)
            ctx.save_for_backward(r["da"], r["db"], r["dmu"])
            return r["logP"].clone().to(a.dtype)

        @staticmethod
        def backward(ctx, g):
            da, db, dmu = ctx.saved_tensors
            return g * da, g * db, g * dmu, None, None, None, None, None

    return MVNLogProb


class _LazyAutograd:
    _cls = None

    def __getattr__(self, name):
        if _LazyAutograd._cls is None:
            _LazyAutograd._cls = _make_autograd()
        return getattr(_LazyAutograd._cls, name)


MVNLogProb = _LazyAutograd()


@dataclass
class BatchPlan:
    """A planned batch: host sizes, the plan on the device, and the buffers
    mvn_prob_batch fills (allocated once, reusable across calls)."""
    n_p: object            # numpy int32 array (host)
    plan: object           # device uint8 tensor
    factor: object         # device uint8 tensor
    workspace: object      # device uint8 tensor
    out: object            # device float64 (count, 4 + S)
    info: object           # device int32 (count,)
    N: int
    S: int
    opts: MvnOptions


def mvn_batch_plan(n_p, N: int, S: int, opts: MvnOptions | None = None, device="cuda") -> BatchPlan:
    import numpy as np
    torch = _torch()
    opts = opts or options()
    sizes = np.ascontiguousarray(np.asarray(n_p, dtype=np.int32))
    count = int(sizes.size)
    pb = ctypes.c_size_t(0)
    _lib.check(_lib.lib().mvn_batch_plan_bytes(count, ctypes.byref(pb)))
    host = np.zeros(pb.value, dtype=np.uint8)
    fb, wb = ctypes.c_size_t(0), ctypes.c_size_t(0)
    _lib.check(_lib.lib().mvn_batch_plan(count, sizes.ctypes.data_as(ctypes.c_void_p), N, S, ctypes.byref(opts),
                                         host.ctypes.data_as(ctypes.c_void_p), pb.value, ctypes.byref(fb),
                                         ctypes.byref(wb)))
    return BatchPlan(sizes, torch.from_numpy(host).to(device), torch.empty(fb.value, dtype=torch.uint8, device=device),
                     torch.empty(wb.value, dtype=torch.uint8, device=device),
                     torch.empty((count, 4 + S), dtype=torch.float64, device=device),
                     torch.empty(count, dtype=torch.int32, device=device), N, S, opts)


def mvn_prob_batch(plan: BatchPlan, idx, locs, kern: tuple, a, b, mu=None, seed: int = 1):
    """Enqueue the whole batch (factorisations, sweep, reductions) on the
    current stream; results land in plan.out and plan.info."""
    torch = _torch()
    dev = plan.out.device
    tidx = torch.as_tensor(idx, dtype=torch.int64).to(dev).contiguous()
    tl = _dev_f64(locs, dev)
    ta, tb = _dev_f64(a, dev), _dev_f64(b, dev)
    tm = _dev_f64(mu, dev) if mu is not None else None
    km = MvnMatern(*kern)
    code = _lib.lib().mvn_prob_batch(
        int(plan.n_p.size), plan.n_p.ctypes.data_as(ctypes.c_void_p), _ptr(plan.plan), _ptr(tidx), _ptr(tl),
        ctypes.byref(km), _ptr(ta), _ptr(tb), _ptr(tm), plan.N, plan.S, ctypes.c_uint64(seed),
        ctypes.byref(plan.opts), _ptr(plan.factor), plan.factor.numel(), _ptr(plan.workspace),
        plan.workspace.numel(), _ptr(plan.out), _ptr(plan.info), _stream(dev))
    _lib.check(code)
    plan._keep = (tidx, tl, ta, tb, tm)
    return plan.out
