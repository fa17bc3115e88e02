"""Gradients of a loss of the least-squares solution (the differentiable solve).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For A of full column rank, x = A^+ b and r = b - A x.  Differentiating the
normal equations A^T A x = A^T b gives

    dx = (A^T A)^{-1} (dA^T r - A^T dA x)

so for a loss L(x) with g = dL/dx, w = (A^T A)^{-1} g and lambda = A w:

    dL/db  = lambda = A (A^T A)^{-1} g
    dL/dA  = r w^T - lambda x^T      (kept on A's sparsity pattern only)

dense_gradients computes this from the definition (Householder QR of A).
iterative_gradients follows the preconditioned route the solver uses: with
B = A R^{-1}, (A^T A)^{-1} = R^{-1} (B^T B)^{-1} R^{-T}.  LSQR on the consistent
under-determined system B^T lambda = c, c = R^{-T} g, started from lambda = 0,
converges to the minimum-norm solution lambda = B (B^T B)^{-1} c = B z; the
iterates are tracked in the coordinates z (every Golub-Kahan vector v_k lies in
range(B), v_k = B vt_k), and w = R^{-1} z.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def dense_gradients(Ad: np.ndarray, b: np.ndarray, g: np.ndarray):
    """(x, r, w, lam) for one right-hand side, from the dense matrix Ad."""
    Q, RA = np.linalg.qr(Ad)
    x = sla.solve_triangular(RA, Q.T @ b)
    r = b - Ad @ x
    w = sla.solve_triangular(RA, sla.solve_triangular(RA, g, trans="T"))
    lam = Ad @ w
    return x, r, w, lam


def pattern_grad(row_ptr, col, r, w, lam, x):
    """dL/dA on the pattern: dA[i, j] = r_i w_j - lam_i x_j for every stored (i, j)."""
    m = len(row_ptr) - 1
    rows = np.repeat(np.arange(m), np.diff(row_ptr))
    return r[rows] * w[col] - lam[rows] * x[col]


def iterative_gradients(A, R, x, r, g, atol=1e-10, btol=1e-10, itmax=None):
    """(w, lam, itn) by LSQR on B^T lambda = R^{-T} g with the z-shadow (see module doc)."""
    m, n = A.shape
    AT = A.T.tocsr()
    itmax = n if itmax is None else itmax

    def Bmul(z):  # B z = A R^{-1} z
        return A @ sla.solve_triangular(R, z)

    def Btmul(l):  # B^T l = R^{-T} A^T l
        return sla.solve_triangular(R, AT @ l, trans="T")

    c = sla.solve_triangular(R, g, trans="T")
    beta = float(np.linalg.norm(c))
    z = np.zeros(n)
    if beta == 0.0:
        return np.zeros(n), np.zeros(m), 0
    u = c / beta                       # u lives in R^n
    vt = u.copy()                      # v = B vt
    v = Bmul(vt)
    alpha = float(np.linalg.norm(v))
    v /= alpha
    vt /= alpha
    wt = vt.copy()
    phibar, rhobar = beta, alpha
    itn = 0
    while itn < itmax:
        itn += 1
        u = Btmul(v) - alpha * u
        beta = float(np.linalg.norm(u))
        if beta > 0.0:
            u /= beta
        vt_new = u - beta * vt
        v_new = Bmul(u) - beta * v
        alpha = float(np.linalg.norm(v_new))
        if alpha > 0.0:
            v_new /= alpha
            vt_new /= alpha
        v, vt = v_new, vt_new
        rho = float(np.hypot(rhobar, beta))
        cs, sn = rhobar / rho, beta / rho
        theta = sn * alpha
        rhobar = -cs * alpha
        phi = cs * phibar
        phibar = sn * phibar
        z = z + (phi / rho) * wt
        wt = vt - (theta / rho) * wt
        if phibar <= btol * np.linalg.norm(c):
            break
    w = sla.solve_triangular(R, z)
    return w, A @ w, itn
