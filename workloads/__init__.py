"""Seeded synthetic workloads for the MVN-probability hot path.

This module only builds inputs: spatial locations on regular grids, their
orderings, Gaussian-process draws that serve as the mean field, integration
limits and batches of nested problems.  It holds none of the estimator's
arithmetic (no Cholesky factor, no separation-of-variables sweep, no QMC
points), so both the CPU oracle and the HIP path can consume its arrays
without sharing code.

The recipes follow the paper's synthetic setting (exponential / Matern fields
on a regular grid in the unit square, Section V-B) at the sizes of the five
benchmark workloads:

  dense400   n = 400   (20 x 20), nu = 1/2, beta = 0.1,  nugget 1e-8
  prec16k    n = 16384 (128x128), nu = 3/2, beta = 0.05, nugget 1e-6, u = 0.5
  tlr64k     n = 65536 (256x256, Morton order), nu = 1/2, beta = 0.1
  batch2000  2000 top-k problems on a 64 x 64 field, nu = 1/2, beta = 0.08
  grad4096   n = 4096  (64 x 64), nu = 3/2, beta = 0.1, finite limits

Gaussian-process draws use circulant embedding of the stationary covariance
on the padded torus (Wood & Chan 1994), which needs no factorisation of the
n x n covariance; the covariance values come from the general Matern formula
evaluated with ``scipy.special.kv``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.special as _sp

__all__ = [
    "grid_locations", "morton_permutation", "gp_draw_grid", "Workload",
    "make_workload", "WORKLOAD_NAMES", "BatchWorkload", "make_batch",
]


def grid_locations(k: int) -> np.ndarray:
    """k*k points at linspace(0, 1, k) in each axis, row-major (i = iy*k + ix).

    Returns an (n, 2) float64 array of (x, y)."""
    t = np.linspace(0.0, 1.0, k)
    xx, yy = np.meshgrid(t, t, indexing="xy")
    return np.stack([xx.ravel(), yy.ravel()], axis=1).astype(np.float64)


def morton_permutation(k: int) -> np.ndarray:
    """Permutation that lists the k*k row-major grid points in Z (Morton) order.

    ``locs[perm]`` is the Morton-ordered location set.  Used where tile
    low-rank compression needs spatial locality of consecutive indices."""
    iy, ix = np.divmod(np.arange(k * k, dtype=np.int64), k)

    def spread(v):
        v = v.astype(np.uint64)
        out = np.zeros_like(v)
        for b in range(32):
            out |= ((v >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b)
        return out

    code = spread(ix) | (spread(iy) << np.uint64(1))
    return np.argsort(code, kind="stable").astype(np.int64)


def _matern_general(h, sigma2, beta, nu):
    """sigma2 / (2^(nu-1) Gamma(nu)) (h/beta)^nu K_nu(h/beta), with C(0)=sigma2."""
    h = np.asarray(h, dtype=np.float64)
    z = h / beta
    out = np.full(h.shape, float(sigma2))
    pos = z > 0
    zp = z[pos]
    out[pos] = sigma2 / (2.0 ** (nu - 1.0) * _sp.gamma(nu)) * zp ** nu * _sp.kv(nu, zp)
    return out


def gp_draw_grid(k: int, sigma2: float, beta: float, nu: float, nugget: float,
                 rng: np.random.Generator, count: int = 1) -> np.ndarray:
    """``count`` zero-mean Gaussian field draws on the k x k unit-square grid.

    Covariance C(h) + nugget * delta, C the Matern function.  Circulant
    embedding on a (p*k)^2 torus; p grows until the embedding's spectrum is
    non-negative.  Returns (count, k*k) in row-major grid order."""
    h = 1.0 / (k - 1) if k > 1 else 1.0
    for pad in (2, 3, 4, 6, 8):
        m = pad * k
        ix = np.arange(m)
        dx = np.minimum(ix, m - ix) * h
        dist = np.sqrt(dx[:, None] ** 2 + dx[None, :] ** 2)
        lam = np.fft.fft2(_matern_general(dist, sigma2, beta, nu)).real
        if lam.min() >= -1e-9 * lam.max():
            break
    else:  # pragma: no cover - embeddings above always succeed for the recipes
        raise RuntimeError("circulant embedding is not non-negative definite")
    lam = np.clip(lam, 0.0, None)
    out = np.empty((count, k * k))
    sq = np.sqrt(lam / (m * m))
    for c in range(count):
        z = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
        f = np.fft.fft2(sq * z)
        out[c] = f.real[:k, :k].ravel()
        if nugget > 0:
            out[c] += math.sqrt(nugget) * rng.standard_normal(k * k)
    return out


@dataclass
class Workload:
    """One MVN problem: locations + Matern parameters + limits + QMC sizes.

    Limits ``a``/``b`` are in X-space; ``mu`` is the mean (None means the
    limits are already centred).  ``tile`` is the Cholesky tile size and
    ``N``/``S`` the QMC points per shift and the number of random shifts."""
    name: str
    locs: np.ndarray
    sigma2: float
    beta: float
    nu: float
    nugget: float
    a: np.ndarray
    b: np.ndarray
    mu: np.ndarray | None
    tile: int
    N: int
    S: int
    seed: int
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.locs.shape[0]


WORKLOAD_NAMES = ("dense400", "prec16k", "tlr64k", "grad4096")


def make_workload(name: str, N: int | None = None, S: int | None = None,
                  positive_excursion: bool = False) -> Workload:
    """Build one of the benchmark workloads with its fixed seeds.

    ``positive_excursion`` flips the limit convention from b = u - mu
    (P(X <= u)) to b = mu - u (P(X > u) of the centred field)."""
    if name == "dense400":
        k, s2, beta, nu, nug, u, tile, n_pts, n_sh, seed = 20, 1.0, 0.1, 0.5, 1e-8, 0.0, 100, 10_000, 10, 1001
    elif name == "prec16k":
        k, s2, beta, nu, nug, u, tile, n_pts, n_sh, seed = 128, 1.0, 0.05, 1.5, 1e-6, 0.5, 512, 20_000, 10, 1002
    elif name == "tlr64k":
        k, s2, beta, nu, nug, u, tile, n_pts, n_sh, seed = 256, 1.0, 0.1, 0.5, 1e-8, 0.0, 1024, 10_000, 10, 1003
    elif name == "grad4096":
        k, s2, beta, nu, nug, u, tile, n_pts, n_sh, seed = 64, 1.0, 0.1, 1.5, 1e-6, None, 256, 10_000, 1, 1005
    else:
        raise KeyError(name)
    rng = np.random.default_rng(seed)
    locs = grid_locations(k)
    field_ = gp_draw_grid(k, s2, beta, nu, nug, rng)[0]
    extra = {}
    if name == "tlr64k":
        perm = morton_permutation(k)
        locs = locs[perm]
        field_ = field_[perm]
        extra["perm"] = perm
    n = k * k
    if name == "grad4096":
        uu = rng.uniform(0.0, 2.0, n)
        a = field_ - 3.0
        b = field_ + uu
        mu = field_.copy()
        extra["u"] = uu
    else:
        a = np.full(n, -np.inf)
        b = (field_ - u) if positive_excursion else (u - field_)
        mu = None
        extra["u"] = u
        extra["field"] = field_
    return Workload(name, locs, s2, beta, nu, nug, a, b, mu, tile,
                    N if N is not None else n_pts, S if S is not None else n_sh,
                    seed + 1, extra)


@dataclass
class BatchWorkload:
    """Many MVN problems that index one shared set of locations.

    Problem p uses locations ``idx[off[p]:off[p+1]]`` (in that order) with
    centred limits ``a[off[p]:off[p+1]]``, ``b[...]``."""
    locs: np.ndarray
    sigma2: float
    beta: float
    nu: float
    nugget: float
    n_p: np.ndarray
    off: np.ndarray
    idx: np.ndarray
    a: np.ndarray
    b: np.ndarray
    u: np.ndarray
    N: int
    S: int
    seed: int


def make_batch(count: int = 2000, n_min: int = 50, n_max: int = 4096, k: int = 64,
               N: int = 5000, S: int = 8, seed: int = 1004,
               positive_excursion: bool = False) -> BatchWorkload:
    """Nested confidence-region problems: per problem one GP draw on the k x k
    grid, a threshold u in {0, 0.5, 1}, a log-uniform size n_p, and the n_p
    sites of highest marginal exceedance 1 - Phi((u - mu_i)/sigma_i) in
    descending order (the ordering step of the detection algorithm)."""
    s2, beta, nu, nug = 1.0, 0.08, 0.5, 1e-8
    rng = np.random.default_rng(seed)
    locs = grid_locations(k)
    n_max = min(n_max, k * k)
    n_p = np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), count))).astype(np.int64)
    n_p = np.clip(n_p, n_min, n_max)
    us = rng.choice(np.array([0.0, 0.5, 1.0]), size=count)
    fields = gp_draw_grid(k, s2, beta, nu, nug, rng, count=count)
    sd = math.sqrt(s2 + nug)
    off = np.zeros(count + 1, dtype=np.int64)
    off[1:] = np.cumsum(n_p)
    idx = np.empty(off[-1], dtype=np.int64)
    a = np.full(off[-1], -np.inf)
    b = np.empty(off[-1])
    for p in range(count):
        f, u = fields[p], us[p]
        exceed = _sp.ndtr(-(u - f) / sd)
        order = np.argsort(-exceed, kind="stable")[: n_p[p]]
        idx[off[p]:off[p + 1]] = order
        b[off[p]:off[p + 1]] = (f[order] - u) if positive_excursion else (u - f[order])
    return BatchWorkload(locs, s2, beta, nu, nug, n_p, off, idx, a, b, us, N, S, seed + 1)


@dataclass
class PosteriorData:
    """Synthetic observations of one Gaussian field draw: the k x k grid
    sites, the field x, m observed sites (distinct, random) and y = x[obs] +
    N(0, noise_sd^2).  The shape of the paper's synthetic posterior problems:
    40 000 sites, 6 250 observations, noise sd 0.5, exponential kernel
    (nu = 1/2) with range 0.033, 0.1 or 0.234."""
    locs: np.ndarray
    x: np.ndarray
    obs: np.ndarray
    y: np.ndarray
    sigma2: float
    beta: float
    nu: float
    nugget: float
    noise_sd: float


def make_posterior(k: int = 200, m: int = 6250, beta: float = 0.1, noise_sd: float = 0.5, nu: float = 0.5,
                   sigma2: float = 1.0, nugget: float = 1e-8, seed: int = 2405) -> PosteriorData:
    rng = np.random.default_rng(seed)
    locs = grid_locations(k)
    x = gp_draw_grid(k, sigma2, beta, nu, nugget, rng)[0]
    obs = np.sort(rng.choice(k * k, m, replace=False)).astype(np.int64)
    y = x[obs] + noise_sd * rng.standard_normal(m)
    return PosteriorData(locs, x, obs, y, sigma2, beta, nu, nugget, noise_sd)
