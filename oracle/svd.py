"""SVD preconditioner of the CSSVDP-LSQR method (Alg. 2 step 3; Thm 3.4).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Plain definition: the compact SVD of the sketch, SA = U Sigma V^T, truncated at
the numerical rank r = #{i : sigma_i > rcond * sigma_1} (Sec. 3.2 takes the
threshold as LAPACK does, the largest singular value times a constant RCOND;
the paper gives no value for it, and the reading here is rcond = n u with
u = 2^-53 unless the caller passes one), and the preconditioner
P = V_r Sigma_r^{-1} (n x r).  The SVD itself is LAPACK's (numpy.linalg.svd, a
library primitive serving as one step).

Since B = A P has r columns, LSQR (Alg. 2 step 5) works in R^r and the solution
is x = P y (step 6); for a rank-deficient A it is the minimum-norm
least-squares solution of the truncated problem (Thm 3.4).
"""

from __future__ import annotations

import numpy as np


def default_rcond(n: int) -> float:
    return n * 2.0 ** -53


def svd_preconditioner(SA: np.ndarray, rcond: float | None = None):
    """Returns (sigma, V, r, P): all n singular values of SA (descending), the
    n x n right singular vectors, the numerical rank and P = V_r Sigma_r^{-1}."""
    SA = np.asarray(SA, np.float64)
    s, n = SA.shape
    if s < n:
        raise ValueError("sketch has fewer rows than columns")
    if rcond is None:
        rcond = default_rcond(n)
    _, sigma, Vt = np.linalg.svd(SA, full_matrices=False)
    V = Vt.T
    r = int(np.count_nonzero(sigma > rcond * sigma[0])) if n and sigma[0] > 0 else 0
    P = V[:, :r] / sigma[:r]
    return sigma, V, r, P
