"""Cholesky factor Sigma = L L^T (Algorithm 1, factorisation step; Eq. (sov1)
defines L as the lower Cholesky factor).

Right-looking blocked algorithm, FP64: factor a diagonal block column by
column, solve the block column below it, subtract the block column's outer
product from the trailing matrix.  numpy matmul is the only library step.
"""
from __future__ import annotations

import math

import numpy as np


class NotPositiveDefinite(ValueError):
    """Raised with the 1-based index of the first non-positive pivot."""

    def __init__(self, index: int):
        super().__init__(f"matrix is not positive definite at pivot {index}")
        self.index = index


def cholesky(sigma: np.ndarray, block: int = 128) -> np.ndarray:
    """Lower factor L with L @ L.T == sigma; only the lower triangle is read."""
    a = np.array(sigma, dtype=np.float64, copy=True)
    n = a.shape[0]
    for k0 in range(0, n, block):
        k1 = min(k0 + block, n)
        for j in range(k0, k1):
            piv = a[j, j] - a[j, k0:j] @ a[j, k0:j]
            if not piv > 0.0:
                raise NotPositiveDefinite(j + 1)
            ljj = math.sqrt(piv)
            a[j, j] = ljj
            # column j below the pivot, including the rows under the block
            a[j + 1:, j] = (a[j + 1:, j] - a[j + 1:, k0:j] @ a[j, k0:j]) / ljj
        if k1 < n:
            p = a[k1:, k0:k1]
            a[k1:, k1:] -= p @ p.T
    return np.tril(a)
