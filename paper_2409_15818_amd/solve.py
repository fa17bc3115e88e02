"""The CSQRP-LSQR pipeline (Alg. 1) over the C-ABI, its SVD variant
CSSVDP-LSQR (Alg. 2), and the differentiable form.

csqrp_lsqr      sketch -> QR preconditioner -> LSQR for one or many right-hand sides
cssvdp_lsqr     sketch -> truncated SVD preconditioner -> LSQR
LstsqFunction   torch.autograd.Function: x = A^+ b with gradients w.r.t. b and the
                stored values of A (restricted to A's pattern), the backward running
                the preconditioned LSQR on the transposed operator.
"""

from __future__ import annotations

import warnings
from dataclasses import dataclass, field

import torch

from .api import (CSR, Handle, Precond, default_opts, rfmls_form_B, rfmls_precond, rfmls_precond_svd,
                  rfmls_precond_x0, rfmls_sketch, rfmls_solve, rfmls_solve_backward, rfmls_solve_explicit,
                  rfmls_transpose, sketch_buffer)


@dataclass
class Result:
    x: torch.Tensor
    residual: torch.Tensor | None
    info: list
    status: int
    precond: Precond
    AT: CSR
    timings: dict = field(default_factory=dict)


def csqrp_lsqr(h: Handle, A: CSR, b: torch.Tensor, s: int, seed: int = 2, qr_dtype: str = "f64",
               r_store: str = "f64", opts=None, AT: CSR | None = None,
               start: str = "zero", operator: str = "implicit") -> Result:
    """Alg. 1 on the GPU: s = gamma n sketch rows, seed of the count sketch.
    start "zero": y^(0) = 0 (Sec. 4.1); "sketch": y^(0) = Q^T (S b) (Remark 3.1).
    operator "implicit": A (R^{-1} v) and R^{-T} (A^T u) (Remark 3.2); "explicit":
    the dense B = A R^{-1} formed first (Alg. 1 step 4)."""
    if AT is None:
        AT = rfmls_transpose(h, A)
    if start == "zero":
        SA, _, _, _ = rfmls_sketch(h, A, s, seed, dtype=qr_dtype)
        P = rfmls_precond(h, SA, qr_dtype, r_store)
        x0 = None
    elif start == "sketch":
        nrhs = 1 if b.dim() == 1 else b.shape[0]
        SA = sketch_buffer(s, A.n + nrhs, qr_dtype, b.device)
        SA, _, _, Sb = rfmls_sketch(h, A, s, seed, b=b, dtype=qr_dtype, SA=SA)
        P, x0 = rfmls_precond_x0(h, SA, A.n, Sb if b.dim() == 2 else Sb[0], qr_dtype, r_store)
    else:
        raise ValueError(f"unknown start {start!r}")
    del SA
    if operator == "explicit":
        Bm = rfmls_form_B(h, A, P)
        X, R, info, rc = rfmls_solve_explicit(h, A, AT, P, Bm, b, opts, x0=x0)
        del Bm
    elif operator == "implicit":
        X, R, info, rc = rfmls_solve(h, A, AT, P, b, opts, x0=x0)
    else:
        raise ValueError(f"unknown operator {operator!r}")
    return Result(X, R, info, rc, P, AT)


def cssvdp_lsqr(h: Handle, A: CSR, b: torch.Tensor, s: int, seed: int = 2, rcond: float = 0.0,
                p_store: str = "f64", opts=None, AT: CSR | None = None,
                operator: str = "implicit") -> Result:
    """Alg. 2 on the GPU: the count sketch, the truncated SVD preconditioner
    P = V_r Sigma_r^{-1} (rcond <= 0: n u) and LSQR on A P from y^(0) = 0,
    x = P y.  operator "explicit" forms the dense B = A P first."""
    if AT is None:
        AT = rfmls_transpose(h, A)
    SA, _, _, _ = rfmls_sketch(h, A, s, seed, dtype="f64")
    P = rfmls_precond_svd(h, SA, A.n, rcond=rcond, p_store=p_store)
    del SA
    if operator == "explicit":
        Bm = rfmls_form_B(h, A, P)
        X, R, info, rc = rfmls_solve_explicit(h, A, AT, P, Bm, b, opts)
        del Bm
    elif operator == "implicit":
        X, R, info, rc = rfmls_solve(h, A, AT, P, b, opts)
    else:
        raise ValueError(f"unknown operator {operator!r}")
    return Result(X, R, info, max(rc, P.status), P, AT)


class LstsqFunction(torch.autograd.Function):
    """x = argmin ||A x - b|| with A given by its CSR pattern and differentiable values.

    forward(val, b, solver) -> x;  backward gives dL/dval (on the pattern) and dL/db."""

    @staticmethod
    def forward(ctx, val, b, solver):
        A = CSR(solver.m, solver.n, solver.row_ptr, solver.col, val.detach().contiguous())
        res = csqrp_lsqr(solver.handle, A, b.detach(), solver.s, solver.seed, solver.qr_dtype,
                         solver.r_store, solver.opts)
        solver.last = res
        if res.status != 0:
            # RFMLS_W_NOCONV: a right-hand side stopped at the iteration limit; x
            # (and the gradients taken through it) are not at the tolerance
            warnings.warn(f"LstsqFunction: the solve returned status {res.status} "
                          f"(iteration limit reached); x is not converged", RuntimeWarning)
        ctx.solver = solver
        ctx.A = A
        ctx.res = res
        ctx.single = b.dim() == 1
        return res.x

    @staticmethod
    def backward(ctx, gx):
        solver, A, res = ctx.solver, ctx.A, ctx.res
        G = gx.contiguous()
        dB, dA, info, _ = rfmls_solve_backward(solver.handle, A, res.AT, res.precond, res.x,
                                               res.residual, G, solver.opts)
        solver.last_backward_info = info
        if any(i["istop"] == 7 for i in info):
            warnings.warn("LstsqFunction.backward: the adjoint solve reached its iteration limit; "
                          "the gradients are not converged", RuntimeWarning)
        return dA, dB, None


@dataclass
class LstsqSolver:
    """Configuration holder for LstsqFunction (pattern of A, sketch size, precisions)."""
    handle: Handle
    m: int
    n: int
    row_ptr: torch.Tensor
    col: torch.Tensor
    s: int
    seed: int = 2
    qr_dtype: str = "f64"
    r_store: str = "f64"
    opts: object = None
    last: Result | None = None
    last_backward_info: list | None = None

    def __post_init__(self):
        if self.opts is None:
            self.opts = default_opts()

    def __call__(self, val: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
        return LstsqFunction.apply(val, b, self)
