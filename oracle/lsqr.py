"""Textbook LSQR (Paige & Saunders, ACM TOMS 8(1), 1982) for min ||B y - b||.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Alg. 1 step 5 runs LSQR on the preconditioned matrix B = A R^{-1}; with the
preconditioner applied inside the iteration (Remark 3.2) B is never formed:
B v = A (R^{-1} v) and B^T u = R^{-T} (A^T u).  The iteration is the
Golub-Kahan bidiagonalisation followed by the plane-rotation update of the
solution, written out in the order of Paige & Saunders:

  beta_1 u_1 = b,   alpha_1 v_1 = B^T u_1,   w_1 = v_1,   phibar_1 = beta_1,
  rhobar_1 = alpha_1, and for i = 1, 2, ...
    beta_{i+1} u_{i+1}   = B v_i - alpha_i u_i
    alpha_{i+1} v_{i+1}  = B^T u_{i+1} - beta_{i+1} v_i
    rho_i   = sqrt(rhobar_i^2 + beta_{i+1}^2)
    c_i     = rhobar_i / rho_i,     s_i = beta_{i+1} / rho_i
    theta_{i+1} = s_i alpha_{i+1},  rhobar_{i+1} = -c_i alpha_{i+1}
    phi_i   = c_i phibar_i,         phibar_{i+1} = s_i phibar_i
    y_i     = y_{i-1} + (phi_i / rho_i) w_i
    w_{i+1} = v_{i+1} - (theta_{i+1} / rho_i) w_i

Stopping rules (Paige & Saunders Sec. 6), with the estimates
||r_i|| = phibar_{i+1}, ||B^T r_i|| = phibar_{i+1} alpha_{i+1} |c_i|,
||B||_F^2 ~ sum(alpha^2 + beta^2), cond(B) ~ ||B||_F sqrt(sum ||w_i/rho_i||^2):
  istop 1 (S1): ||r|| <= btol ||b|| + atol ||B|| ||y||
  istop 2 (S2): ||B^T r|| <= atol ||B|| ||r||
  istop 3 (S3): cond(B) >= conlim (conlim <= 0 disables this test)
  istop 7     : itmax iterations done
Sec. 4.1 starts from y = 0 and uses at most n iterations.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class LSQRResult:
    y: np.ndarray
    istop: int
    itn: int
    normr: float
    normar: float
    anorm: float
    acond: float
    ynorm: float
    history: list = field(default_factory=list)


def lsqr(apply_B, apply_Bt, b: np.ndarray, n: int, atol: float = 1e-10, btol: float = 1e-10,
         conlim: float = 1e8, itmax: int | None = None, keep_history: bool = False) -> LSQRResult:
    itmax = n if itmax is None else itmax
    y = np.zeros(n)
    beta = float(np.linalg.norm(b))
    if beta == 0.0:
        return LSQRResult(y, 0, 0, 0.0, 0.0, 0.0, 0.0, 0.0)
    u = b / beta
    v = apply_Bt(u)
    alpha = float(np.linalg.norm(v))
    if alpha == 0.0:
        return LSQRResult(y, 0, 0, beta, 0.0, 0.0, 0.0, 0.0)
    v = v / alpha
    w = v.copy()
    phibar, rhobar = beta, alpha
    bnorm = beta
    anorm2 = 0.0
    ddnorm = 0.0
    istop, itn = 7, 0
    normr, normar, acond, ynorm = beta, alpha * beta, 0.0, 0.0
    hist = []
    while itn < itmax:
        itn += 1
        # bidiagonalisation
        u = apply_B(v) - alpha * u
        beta = float(np.linalg.norm(u))
        if beta > 0.0:
            u = u / beta
        anorm2 += alpha * alpha + beta * beta
        vnew = apply_Bt(u) - beta * v
        alpha = float(np.linalg.norm(vnew))
        if alpha > 0.0:
            vnew = vnew / alpha
        v = vnew
        # plane rotation
        rho = float(np.hypot(rhobar, beta))
        c = rhobar / rho
        s = beta / rho
        theta = s * alpha
        rhobar = -c * alpha
        phi = c * phibar
        phibar = s * phibar
        # update of the solution and the search direction
        ddnorm += float(np.linalg.norm(w / rho)) ** 2
        y = y + (phi / rho) * w
        w = v - (theta / rho) * w
        # estimates and stopping tests
        anorm = np.sqrt(anorm2)
        acond = anorm * np.sqrt(ddnorm)
        ynorm = float(np.linalg.norm(y))
        normr = phibar
        normar = phibar * alpha * abs(c)
        if keep_history:
            hist.append((itn, normr, normar / (anorm * normr) if normr > 0 else 0.0))
        if normr <= btol * bnorm + atol * anorm * ynorm:
            istop = 1
        elif normr == 0.0 or normar <= atol * anorm * normr:
            istop = 2
        elif conlim > 0 and acond >= conlim:
            istop = 3
        if istop != 7:
            break
    return LSQRResult(y, istop, itn, normr, normar, float(np.sqrt(anorm2)), acond, ynorm, hist)
