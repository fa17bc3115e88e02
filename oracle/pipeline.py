"""The CSQRP-LSQR solve (Alg. 1), its SVD variant CSSVDP-LSQR (Alg. 2) and
the quantities Sec. 4.1 reports.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Steps, in the paper's order:
  1. s = gamma n sketch rows (chosen by the caller)
  2. SA by the count sketch (countsketch.sketch_dense)
  3. R from the QR of SA (qr.r_factor)
  4. the preconditioned operator B = A R^{-1}, applied implicitly (Remark 3.2)
     or, for comparison only, formed explicitly as a dense matrix
  5. LSQR on min ||B y - b|| from y = 0 (Sec. 4.1)
  6. x = R^{-1} y
Remark 3.3 observes that the implicit operator loses accuracy on ill-conditioned
problems; the reading adopted here recovers it with iterative refinement: after
a sweep, the true residual r = b - A x is recomputed and the same preconditioned
LSQR solves min ||A d - r||, x <- x + d (`refine` extra sweeps, default 1).

CSSVDP-LSQR (Alg. 2) replaces step 3 by the truncated SVD of SA and R^{-1} by
P = V_r Sigma_r^{-1} (svd.svd_preconditioner): LSQR runs on B = A P, applied
implicitly as B v = A (P v), B^T u = P^T (A^T u), and x = P y.

Starting point (Alg. 1 takes y^(0) as an input).  Sec. 4.1 starts from zero;
Remark 3.1 offers y^(0) = Q^T (S b), obtained by carrying S b through the
Householder QR as an extra column of [SA | Sb]: the top n entries of that
column of the triangular factor are Q^T (S b), and x^(0) = R^{-1} y^(0) is the
minimiser of ||S (A x - b)|| (`sketched_start`).  A sweep from a non-zero x
solves for the correction from the residual b - A x, as the refinement sweeps do.

Reported: iterations, the true residual ||b - A x|| / ||b|| recomputed from x,
the normal-equation residual ||A^T r|| / (||A||_F ||r||), and ||r||^2/||b||^2
(the paper's squared "relative least squares error", Sec. 4.1).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import countsketch, qr, svd
from .lsqr import lsqr


def csr(row_ptr, col, val, m, n):
    return sp.csr_matrix((np.asarray(val, np.float64), np.asarray(col, np.int64),
                          np.asarray(row_ptr, np.int64)), shape=(m, n))


def precondition(row_ptr, col, val, m, n, s, seed, qr_dtype="f64", r_store="f64", b=None,
                 hash_in=None, check_precision=True):
    """Steps 1-3: returns dict(h, sign, SA, Sb, R) with R as a float64 array holding the
    stored preconditioner (rounded to float32 first when r_store == 'f32').  A factor
    computed or stored in float32 with rho_min <= 16 u32 raises qr.PrecisionInsufficient
    (check_precision)."""
    if hash_in is None:
        h, sign = countsketch.hash_sign(m, s, seed)
    else:
        h, sign = hash_in
    SA, Sb = countsketch.sketch_dense(row_ptr, col, val, h, sign, s, n, b=b)
    if qr_dtype == "f32":
        R = qr.r_factor(SA.astype(np.float32), check_rank=False).astype(np.float64)
    else:
        R = qr.r_factor(SA)
    if check_precision and "f32" in (qr_dtype, r_store) and qr.rho_min(R) <= qr.PRECISION_TOL:
        raise qr.PrecisionInsufficient("float32 factor: min |r_jj| / ||SA[:, j]|| <= 16 u32")
    if r_store == "f32":
        R = R.astype(np.float32).astype(np.float64)
    return dict(h=h, sign=sign, SA=SA, Sb=Sb, R=R)


def lsqr_on_preconditioned(A, R, b, atol=1e-10, btol=1e-10, conlim=1e8, itmax=None,
                           operator="implicit", keep_history=False):
    """Steps 4-6 for one right-hand side; returns (x, LSQRResult)."""
    m, n = A.shape
    if operator == "implicit":
        AT = A.T.tocsr()

        def apply_B(v):
            return A @ sla.solve_triangular(R, v, lower=False)

        def apply_Bt(u):
            return sla.solve_triangular(R, AT @ u, lower=False, trans="T")
    elif operator == "explicit":
        # B = A R^{-1}: solve B R = A row-wise, i.e. R^T B^T = A^T.
        Bd = sla.solve_triangular(R, A.toarray().T, lower=False, trans="T").T

        def apply_B(v):
            return Bd @ v

        def apply_Bt(u):
            return Bd.T @ u
    else:
        raise ValueError(operator)
    res = lsqr(apply_B, apply_Bt, b, n, atol=atol, btol=btol, conlim=conlim, itmax=itmax,
               keep_history=keep_history)
    x = sla.solve_triangular(R, res.y, lower=False)
    return x, res


def lsqr_on_svd_preconditioned(A, P, b, atol=1e-10, btol=1e-10, conlim=1e8, itmax=None,
                               keep_history=False):
    """Alg. 2 steps 4-6 for one right-hand side with B = A P applied implicitly;
    returns (x, LSQRResult)."""
    AT = A.T.tocsr()
    r = P.shape[1]
    res = lsqr(lambda v: A @ (P @ v), lambda u: P.T @ (AT @ u), b, r, atol=atol, btol=btol,
               conlim=conlim, itmax=A.shape[1] if itmax is None else itmax, keep_history=keep_history)
    return P @ res.y, res


def residual_metrics(A, x, b):
    r = b - A @ x
    nb = float(np.linalg.norm(b))
    nr = float(np.linalg.norm(r))
    afro = float(sp.linalg.norm(A)) if sp.issparse(A) else float(np.linalg.norm(A))
    nar = float(np.linalg.norm(A.T @ r))
    return dict(normr=nr, relres=nr / nb if nb else 0.0,
                normal_relres=nar / (afro * nr) if nr else 0.0,
                rel_ls_error_sq=(nr / nb) ** 2 if nb else 0.0)


def l2_error(E, x, u_exact):
    uh = E @ x
    return float(np.linalg.norm(uh - u_exact) / np.linalg.norm(u_exact))


def sketched_start(SA, SB, check_rank=True):
    """Remark 3.1: Householder QR of [SA | SB] (SB: s x k sketched right-hand
    sides, in SA's dtype).  Returns (R, Y0, X0): R the n x n factor of SA (diag
    > 0), Y0 = Q^T SB (its top n x k block of the extended factor, with R's row
    signs) and X0 = R^{-1} Y0, the minimisers of ||SA x - SB[:, k]||."""
    SA = np.asarray(SA)
    SB = np.asarray(SB, SA.dtype).reshape(SA.shape[0], -1)
    n = SA.shape[1]
    Rx = qr.r_factor(np.hstack([SA, SB]), check_rank=False)
    R = Rx[:n, :n].astype(np.float64)
    if check_rank and not qr.rank_ok(Rx[:n, :n]):
        raise qr.RankDeficient("R has a pivot below 16*u*max|r_jj|")
    Y0 = Rx[:n, n:].astype(np.float64)
    X0 = sla.solve_triangular(R, Y0, lower=False)
    return R, Y0, X0


def refined_lsqr(A, R, b, refine=1, x0=None, P=None, on_sweep=None, **kw):
    """LSQR sweeps with iterative refinement on the true residual, from x = 0
    or from x0; returns (x, [results]).  With P given (CSSVDP-LSQR) the
    preconditioner is P instead of R^{-1}.  on_sweep(k, result), if given, is
    called after each sweep (progress reporting; no effect on the result)."""
    b = np.asarray(b, np.float64)
    x = np.zeros(A.shape[1]) if x0 is None else np.array(x0, np.float64)
    r = b.copy() if x0 is None else b - A @ x
    results = []
    for sweep in range(1 + refine):
        if P is None:
            dx, res = lsqr_on_preconditioned(A, R, r, **kw)
        else:
            kw.pop("operator", None)
            dx, res = lsqr_on_svd_preconditioned(A, P, r, **kw)
        results.append(res)
        if on_sweep is not None:
            on_sweep(sweep, res)
        x = x + dx
        r = b - A @ x
        if res.itn == 0:
            break
    return x, results


def solve_svd(row_ptr, col, val, b, m, n, s, seed, rcond=None, atol=1e-10, btol=1e-10,
              conlim=1e8, itmax=None, refine=1, hash_in=None):
    """Full CSSVDP-LSQR (Alg. 2) for one right-hand side from y^(0) = 0, float64;
    returns a dict of results (sigma, V, rank r, P, x and the residual metrics)."""
    if hash_in is None:
        h, sign = countsketch.hash_sign(m, s, seed)
    else:
        h, sign = hash_in
    SA, _ = countsketch.sketch_dense(row_ptr, col, val, h, sign, s, n)
    sigma, V, r, P = svd.svd_preconditioner(SA, rcond)
    A = csr(row_ptr, col, val, m, n)
    x, results = refined_lsqr(A, None, b, refine=refine, P=P, atol=atol, btol=btol,
                              conlim=conlim, itmax=itmax)
    res = results[0]
    out = dict(x=x, itn=sum(q.itn for q in results), itn_sweeps=[q.itn for q in results],
               istop=res.istop, acond=res.acond, sigma=sigma, V=V, rank=r, P=P, SA=SA, h=h,
               sign=sign)
    out.update(residual_metrics(A, x, np.asarray(b, np.float64)))
    return out


def solve(row_ptr, col, val, b, m, n, s, seed, atol=1e-10, btol=1e-10, conlim=1e8, itmax=None,
          qr_dtype="f64", r_store="f64", operator="implicit", refine=1, keep_history=False,
          start="zero"):
    """Full CSQRP-LSQR for one right-hand side (start "zero": y^(0) = 0, Sec. 4.1;
    "sketch": y^(0) = Q^T (S b), Remark 3.1); returns a dict of results."""
    pre = precondition(row_ptr, col, val, m, n, s, seed, qr_dtype=qr_dtype, r_store=r_store,
                       b=np.asarray(b, np.float64) if start == "sketch" else None)
    A = csr(row_ptr, col, val, m, n)
    x0 = None
    if start == "sketch":
        SA = pre["SA"].astype(np.float32) if qr_dtype == "f32" else pre["SA"]
        R, _, X0 = sketched_start(SA, pre["Sb"], check_rank=qr_dtype == "f64")
        if r_store == "f32":
            R = R.astype(np.float32).astype(np.float64)
        pre["R"] = R
        x0 = X0[:, 0]
    elif start != "zero":
        raise ValueError(start)
    x, results = refined_lsqr(A, pre["R"], b, refine=refine, x0=x0, atol=atol, btol=btol,
                              conlim=conlim, itmax=itmax, operator=operator,
                              keep_history=keep_history)
    res = results[0]
    out = dict(x=x, itn=sum(r.itn for r in results), itn_sweeps=[r.itn for r in results],
               istop=res.istop, est_normr=res.normr, est_normar=res.normar, anorm=res.anorm,
               acond=res.acond, R=pre["R"], h=pre["h"], sign=pre["sign"],
               history=[r.history for r in results], x0=x0)
    out.update(residual_metrics(A, x, np.asarray(b, np.float64)))
    return out
