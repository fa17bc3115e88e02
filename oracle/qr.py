"""R factor of the sketched matrix (Alg. 1 step 3; Thm 3.1-3.2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Plain definition: for SA of full column rank, R is the unique upper-triangular
matrix with positive diagonal such that R^T R = (SA)^T (SA).  It is computed by
Householder QR (never from the Gram matrix, whose condition number is the
square of SA's).  The QR is unique up to the signs of R's rows, so every row
with a negative diagonal entry is negated.  A rank check follows Sec. 4.4's
"fails in the preconditioning phase", which gives no threshold; the reading used
here is |r_ii| <= 16 u max_j |r_jj|: a pivot within a few rounding errors of
the largest one (an exactly dependent column leaves a pivot of a few u) means
SA, hence A by Thm 3.1, is numerically rank deficient.

Two implementations:
  r_factor           LAPACK's Householder QR (numpy.linalg.qr, a library primitive)
  r_factor_textbook  column-by-column Householder reflections written out
                     (Golub & Van Loan, Alg. 5.2.1), for small matrices; the
                     tests check the two against each other and against the
                     defining identity.
"""

from __future__ import annotations

import numpy as np


class RankDeficient(ValueError):
    pass


class PrecisionInsufficient(ValueError):
    """A float32 factor that cannot precondition the system (see rho_min)."""


def _normalise(R: np.ndarray) -> np.ndarray:
    d = np.sign(np.diag(R)).astype(R.dtype)
    d[d == 0] = 1
    return R * d[:, None]


def rank_ok(R: np.ndarray) -> bool:
    n = R.shape[0]
    if n == 0:
        return True
    dg = np.abs(np.diag(R)).astype(np.float64)
    u = np.finfo(R.dtype).eps / 2
    return bool(dg.min() > 16.0 * u * dg.max())


def rho_min(R: np.ndarray) -> float:
    """min_j |r_jj| / ||R[:, j]||: the distance of column j of SA from the span of
    the columns before it, relative to the column's length (||R[:, j]|| equals
    ||SA[:, j]|| because Q has orthonormal columns).  Householder QR in unit
    roundoff u perturbs each column of SA by a few u times its length, so a
    factor computed or stored in float32 whose rho_min is within 16 u32
    (u32 = 2^-24; the margin of the float64 rank test) carries only rounding
    noise in that direction (the reading used for the float32 preconditioner;
    the paper has no float32 factor)."""
    R = np.asarray(R, dtype=np.float64)
    if R.shape[0] == 0:
        return np.inf
    return float(np.min(np.abs(np.diag(R)) / np.linalg.norm(R, axis=0)))


U32 = 2.0 ** -24
# a factor computed or stored in float32 is refused at or below this rho_min
PRECISION_TOL = 16.0 * U32


def r_factor(SA: np.ndarray, check_rank: bool = True) -> np.ndarray:
    """R (n x n, diag >= 0) of SA (s x n, s >= n), in SA's dtype."""
    s, n = SA.shape
    if s < n:
        raise ValueError("sketch has fewer rows than columns")
    R = np.linalg.qr(SA, mode="r")[:n, :n]
    R = np.triu(_normalise(R))
    if check_rank and not rank_ok(R):
        raise RankDeficient("R has a pivot below 16*u*max|r_jj|")
    return R


def r_factor_textbook(M: np.ndarray) -> np.ndarray:
    """Householder QR written out, one reflector per column; returns R with diag >= 0."""
    A = np.array(M, dtype=np.float64, copy=True)
    s, n = A.shape
    for k in range(n):
        x = A[k:, k]
        normx = np.linalg.norm(x)
        if normx == 0.0:
            continue
        alpha = -normx if x[0] >= 0 else normx
        v = x.copy()
        v[0] -= alpha
        v /= np.linalg.norm(v)
        A[k:, k:] -= 2.0 * np.outer(v, v @ A[k:, k:])
    return np.triu(_normalise(A[:n, :n]))
