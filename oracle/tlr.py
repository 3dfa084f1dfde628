"""Tile low-rank (TLR) compression and TLR Cholesky (paper Section III-E;
Algorithm 1's factorisation step in its TLR form; the rank / accuracy
settings of Section V).

Reading used here (the paper names per-tile SVD truncation to an accuracy
and a maximum rank, but not whether the accuracy is absolute or relative):
an off-diagonal tile A_ij is replaced by U V^T keeping the singular values
above ``eps`` (absolute), at most ``max_rank`` of them, so that
||A_ij - U V^T||_2 <= eps whenever the rank cap does not bind.  Diagonal
tiles stay dense.

TLR Cholesky, right-looking over tile columns k (the dense storage of the
not-yet-factored tiles is kept; the updates use the low-rank factors):
  1. L_kk = chol(A_kk)
  2. A_ik ~ U_ik V_ik^T for i > k (compression of the panel)
  3. V'_ik = L_kk^{-1} V_ik, so that L_ik = U_ik V'_ik^T = A_ik L_kk^{-T}
  4. A_ij -= U_ik (V'_ik^T V'_jk) U_jk^T for i >= j > k
The factor is the dense diagonal tiles and the pairs (U_ik, V'_ik).
"""
from __future__ import annotations

import numpy as np

from .cholesky import cholesky


def compress_tile(a: np.ndarray, eps: float, max_rank: int):
    """Truncated SVD of one tile: (U diag(s), V) with s > eps, rank <= max_rank."""
    u, s, vt = np.linalg.svd(a, full_matrices=False)
    k = int(np.sum(s > eps))
    k = min(k, max_rank)
    return u[:, :k] * s[:k], vt[:k].T.copy(), s


def tlr_cholesky(sigma: np.ndarray, tile: int, eps: float, max_rank: int):
    """Returns (D, U, V, ranks): dense lower factors D[k] of the diagonal tiles
    and, for i > k, U[i][k] (m_i x r), V[i][k] (m_k x r) with
    L_ik = U[i][k] @ V[i][k].T."""
    n = sigma.shape[0]
    starts = list(range(0, n, tile))
    nt = len(starts)
    blk = [slice(s, min(s + tile, n)) for s in starts]
    A = [[sigma[blk[i], blk[j]].copy() if j <= i else None for j in range(nt)] for i in range(nt)]
    D = [None] * nt
    U = [[None] * nt for _ in range(nt)]
    V = [[None] * nt for _ in range(nt)]
    ranks = np.zeros((nt, nt), dtype=np.int64)
    for k in range(nt):
        D[k] = cholesky(A[k][k])
        for i in range(k + 1, nt):
            u, v, _ = compress_tile(A[i][k], eps, max_rank)
            U[i][k] = u
            V[i][k] = np.linalg.solve(D[k], v)  # L_kk^{-1} V
            ranks[i, k] = u.shape[1]
        for i in range(k + 1, nt):
            for j in range(k + 1, i + 1):
                w = V[i][k].T @ V[j][k]
                A[i][j] -= U[i][k] @ w @ U[j][k].T
    return D, U, V, ranks


def tlr_dense(D, U, V, n: int, tile: int) -> np.ndarray:
    """The dense lower-triangular matrix represented by a TLR factor."""
    L = np.zeros((n, n))
    starts = list(range(0, n, tile))
    nt = len(starts)
    blk = [slice(s, min(s + tile, n)) for s in starts]
    for k in range(nt):
        L[blk[k], blk[k]] = D[k]
        for i in range(k + 1, nt):
            L[blk[i], blk[k]] = U[i][k] @ V[i][k].T
    return L
