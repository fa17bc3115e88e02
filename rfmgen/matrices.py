"""Small structured test matrices (seeded) in the CSR layout the solver takes."""

from __future__ import annotations

import numpy as np


def csr_from_dense(M: np.ndarray, keep_zeros: bool = False):
    """(row_ptr int64, col int32, val float64) of a dense matrix; columns ascend."""
    M = np.asarray(M, dtype=np.float64)
    mask = np.ones_like(M, dtype=bool) if keep_zeros else (M != 0.0)
    rows, cols = np.nonzero(mask)
    row_ptr = np.zeros(M.shape[0] + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=M.shape[0]), out=row_ptr[1:])
    return row_ptr, cols.astype(np.int32), M[rows, cols].astype(np.float64)


def dense_from_csr(row_ptr, col, val, m: int, n: int) -> np.ndarray:
    M = np.zeros((m, n), dtype=np.float64)
    rows = np.repeat(np.arange(m), np.diff(row_ptr))
    M[rows, col] = val
    return M


def dense_with_condition(m: int, n: int, kappa: float, seed: int = 0) -> np.ndarray:
    """A = U diag(sigma) V^T, orthonormal U (m x n), V (n x n), with sigma spaced
    geometrically from 1 down to 1/kappa, so cond_2(A) = kappa."""
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    sigma = np.geomspace(1.0, 1.0 / kappa, n)
    return (U * sigma[None, :]) @ V.T


def random_csr(m: int, n: int, density: float, seed: int = 0, empty_rows=()):
    """Random sparse matrix with N(0,1) values; rows listed in empty_rows have no entries.
    Every column receives at least one entry so the matrix can have full column rank."""
    rng = np.random.default_rng(seed)
    M = np.where(rng.random((m, n)) < density, rng.standard_normal((m, n)), 0.0)
    empty = set(int(i) for i in empty_rows)
    live = [i for i in range(m) if i not in empty]
    for j in range(n):
        if not np.any(M[live, j]):
            M[live[j % len(live)], j] = 1.0 + rng.random()
    for i in empty:
        M[i, :] = 0.0
    return csr_from_dense(M)
