"""More pins of the CPU oracle, each against an independent computation.

* LSQR's stopping rules (Paige & Saunders Sec. 6: S1, S2, S3 at
  atol = btol = 1e-10, conlim = 1e8, the values every solve here uses) against
  scipy's LSQR on problems built to stop by each rule: same rule, same
  iteration, same iterate.
* The spot-check sketch (`sketch_rows`) against the dense sketch and the
  explicit product S A, bitwise.
* The Householder QR written out (`r_factor_textbook`) against LAPACK at a few
  hundred columns, and against R's defining identity.
* The least-squares solution x* = A^+ b of the whole pipeline (sketch, QR,
  LSQR, refinement) against the normal equations solved by brute force in
  extended precision (numpy's longdouble: the x87 80-bit format, unit roundoff
  5.4e-20) on tiny systems with kappa <= 1e4, where kappa^2 u_ld is far below
  the gate.
* The gradients of the loss at the 10^4 sample points on the 2x2-box RFM
  system against a Householder least-squares solve carried out entirely in
  extended precision.
"""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import backward, countsketch, pipeline, qr
from oracle.lsqr import lsqr
from rfmgen import (build_config, csr_from_dense, dense_from_csr, dense_with_condition,
                    feature_eval, random_csr, sample_points)

LD = np.longdouble


def _with_spectrum(m, n, sigma, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (U * np.asarray(sigma)[None, :]) @ V.T


def _clustered(seed):
    # six tight clusters of singular values: the Krylov space is (nearly)
    # exhausted after a handful of steps, so the stopping ratios fall by orders
    # of magnitude per iteration and the stopping point is not a near tie
    rng = np.random.default_rng(seed + 100)
    sig = np.repeat([1.0, 0.8, 0.6, 0.4, 0.3, 0.2], 10) * (1 + 1e-4 * rng.standard_normal(60))
    return _with_spectrum(300, 60, sig, seed)


def _stop_cases():
    for seed in (50, 51):
        A = _clustered(seed)
        b = A @ np.random.default_rng(seed).standard_normal(60)  # consistent: S1
        yield "S1", 1, A, b, 1e-12
    for seed in (52, 53):
        A = _clustered(seed)
        b = np.random.default_rng(seed).standard_normal(300)  # inconsistent: S2
        yield "S2", 2, A, b, 1e-12
    for seed, scale in ((70, 1.0), (71, 1.0), (72, 1e3)):
        # three singular values near 1e-9: cond(B) passes conlim = 1e8 before
        # the normal-equation test is met (the scaled copy makes cond(B)'s
        # factor ||B|| matter)
        sig = scale * np.r_[np.linspace(1.0, 0.5, 27), 1e-8, 3e-9, 1e-9]
        A = _with_spectrum(200, 30, sig, seed)
        b = np.random.default_rng(seed).standard_normal(200)
        yield "S3", 3, A, b, 1e-6


@pytest.mark.parametrize("case", list(_stop_cases()), ids=lambda c: c[0])
def test_lsqr_stopping_rules_match_scipy(case):
    rule, istop, A, b, ytol = case
    n = A.shape[1]
    ours = lsqr(lambda v: A @ v, lambda u: A.T @ u, b, n, atol=1e-10, btol=1e-10, conlim=1e8,
                itmax=10 * n)
    ref = spla.lsqr(A, b, atol=1e-10, btol=1e-10, conlim=1e8, iter_lim=10 * n)
    y_ref, istop_ref, itn_ref, normr_ref = ref[0], ref[1], ref[2], ref[3]
    assert istop_ref == istop, f"scipy stopped by rule {istop_ref}, the case is built for {rule}"
    assert ours.istop == istop
    assert ours.itn == itn_ref
    assert np.linalg.norm(ours.y - y_ref) <= ytol * np.linalg.norm(y_ref)
    assert abs(ours.normr - normr_ref) <= 1e-9 * normr_ref + 1e-14 * np.linalg.norm(b)


# ---------------------------------------------------------------- sketch rows
def test_sketch_rows_equals_dense_sketch_and_explicit_product():
    m, n, s = 700, 37, 90
    rp, col, val = random_csr(m, n, 0.3, seed=12, empty_rows=(3, 400))
    h, sign = countsketch.hash_sign(m, s, 77)
    SA, _ = countsketch.sketch_dense(rp, col, val, h, sign, s, n)
    rows = np.r_[0, 5, np.random.default_rng(1).choice(s, 20, replace=False), s - 1]
    got = countsketch.sketch_rows(rp, col, val, h, sign, n, rows)
    assert np.array_equal(got, SA[rows])
    # and S A formed from the explicit s x m matrix, summed in ascending row order
    S = countsketch.explicit_S(h, sign, s)
    Ad = dense_from_csr(rp, col, val, m, n)
    for k, j in enumerate(rows):
        acc = np.zeros(n)
        for i in np.nonzero(S[j])[0]:
            acc = acc + S[j, i] * Ad[i]
        assert np.array_equal(got[k], acc)
    # a bucket that no row maps to is a zero row
    empty = np.setdiff1d(np.arange(s), h)
    if empty.size:
        assert not countsketch.sketch_rows(rp, col, val, h, sign, n, empty[:1]).any()


# ---------------------------------------------------------------- R factor
@pytest.mark.parametrize("kappa", [1e3, 1e8])
def test_textbook_qr_at_a_few_hundred_columns(kappa):
    M = dense_with_condition(2000, 400, kappa, seed=9)
    Rt = qr.r_factor_textbook(M)
    Rl = qr.r_factor(M, check_rank=False)
    assert np.all(np.diag(Rt) > 0) and not np.tril(Rt, -1).any()
    # backward error of either factor: R^T R = M^T M to a few n u ||M||^2
    for R in (Rt, Rl):
        err = np.linalg.norm(R.T @ R - M.T @ M) / np.linalg.norm(M) ** 2
        assert err < 400 * 1.2e-16
    # elementwise agreement, relative to the row scale, to kappa u
    scale = np.abs(np.diag(Rl))[:, None] + np.abs(Rl).max(axis=1, keepdims=True)
    assert (np.abs(Rt - Rl) / scale).max() <= 50 * kappa * 1.1e-16


# ---------------------------------------------------------------- brute force in long double
def _householder_ld(M, rhs):
    """Householder QR of M carried out in longdouble, the same reflections applied
    to rhs; returns (R, Q^T rhs) with R's diagonal made positive."""
    A = np.array(M, dtype=LD)
    B = np.array(rhs, dtype=LD).reshape(A.shape[0], -1)
    s, n = A.shape
    for k in range(n):
        x = A[k:, k]
        nx = np.sqrt(np.sum(x * x))
        alpha = -nx if x[0] >= 0 else nx
        v = x.copy()
        v[0] -= alpha
        v /= np.sqrt(np.sum(v * v))
        A[k:, k:] -= LD(2) * np.outer(v, v @ A[k:, k:])
        B[k:] -= LD(2) * np.outer(v, v @ B[k:])
    R, QtB = A[:n, :n], B[:n]
    d = np.where(np.diag(R) < 0, LD(-1), LD(1))
    return np.triu(R * d[:, None]), QtB * d[:, None]


def _back_ld(R, y):
    x = np.zeros(R.shape[0], dtype=LD)
    for i in range(R.shape[0] - 1, -1, -1):
        x[i] = (y[i] - R[i, i + 1:] @ x[i + 1:]) / R[i, i]
    return x


def _fwd_t_ld(R, g):  # R^T z = g
    z = np.zeros(R.shape[0], dtype=LD)
    for i in range(R.shape[0]):
        z[i] = (g[i] - R[:i, i] @ z[:i]) / R[i, i]
    return z


def _cholesky_solve_ld(G, c):
    """G x = c for symmetric positive definite G, Cholesky in longdouble."""
    n = G.shape[0]
    L = np.zeros((n, n), dtype=LD)
    for j in range(n):
        L[j, j] = np.sqrt(G[j, j] - L[j, :j] @ L[j, :j])
        for i in range(j + 1, n):
            L[i, j] = (G[i, j] - L[i, :j] @ L[j, :j]) / L[j, j]
    z = np.zeros(n, dtype=LD)
    for i in range(n):
        z[i] = (c[i] - L[i, :i] @ z[:i]) / L[i, i]
    x = np.zeros(n, dtype=LD)
    for i in range(n - 1, -1, -1):
        x[i] = (z[i] - L[i + 1:, i] @ x[i + 1:]) / L[i, i]
    return x


@pytest.mark.parametrize("kappa,seed", [(1e1, 1), (1e3, 2), (1e4, 3)])
def test_pipeline_matches_long_double_normal_equations(kappa, seed):
    assert np.finfo(LD).eps < 1e-18, "needs an extended-precision longdouble"
    m, n = 90, 12
    Ad = dense_with_condition(m, n, kappa, seed=seed)
    b = np.random.default_rng(seed).standard_normal(m)
    AL = Ad.astype(LD)
    xs = _cholesky_solve_ld(AL.T @ AL, AL.T @ b.astype(LD))  # error ~ kappa^2 u_ld <= 5e-12
    rp, col, val = csr_from_dense(Ad, keep_zeros=True)
    out = pipeline.solve(rp, col, val, b, m, n, 4 * n, seed=3, refine=1)
    x = out["x"]
    assert np.linalg.norm(x - xs.astype(np.float64)) <= 1e-9 * float(np.linalg.norm(xs))
    rstar = float(np.linalg.norm(b.astype(LD) - AL @ xs))
    assert abs(out["normr"] - rstar) <= 1e-12 * rstar


def test_dense_and_iterative_gradients_match_long_double_on_rfm_2x2():
    # L = 1/2 ||E x - u||^2 at the 10^4 sample points, g = E^T (E x - u);
    # dL/db = lambda = A (A^T A)^{-1} g and w = (A^T A)^{-1} g.  kappa(A) = 7e5
    # bounds the float64 error of lambda near kappa u and of w near kappa^2 u.
    S, s = build_config("poisson2d_2x2")
    Ad = dense_from_csr(S.row_ptr, S.col, S.val, S.m, S.n)
    b = S.b[0]
    pts = sample_points(2)
    E = pipeline.csr(*feature_eval(S, pts), len(pts), S.n)
    R_ld, Qtb = _householder_ld(Ad, b)
    x_ld = _back_ld(R_ld, Qtb[:, 0])
    g = E.T @ (E @ x_ld.astype(np.float64) - S.exact(pts))
    w_ld = _back_ld(R_ld, _fwd_t_ld(R_ld, g.astype(LD)))
    lam_ld = Ad.astype(LD) @ w_ld
    r_ld = b.astype(LD) - Ad.astype(LD) @ x_ld

    def rel(a, ref):
        return float(np.linalg.norm(a.astype(LD) - ref) / np.linalg.norm(ref))

    x, r, w, lam = backward.dense_gradients(Ad, b, g)
    assert rel(x, x_ld) < 1e-10 and rel(r, r_ld) < 1e-9
    assert rel(w, w_ld) < 1e-9 and rel(lam, lam_ld) < 1e-9
    R = pipeline.precondition(S.row_ptr, S.col, S.val, S.m, S.n, s, 2)["R"]
    w2, lam2, itn = backward.iterative_gradients(sp.csr_matrix(Ad), R, x, r, g)
    assert rel(lam2, lam_ld) < 1e-8 and rel(w2, w_ld) < 1e-8
    dA_ld = backward.pattern_grad(S.row_ptr, S.col, r_ld, w_ld, lam_ld, x_ld)
    dA = backward.pattern_grad(S.row_ptr, S.col, r, w2, lam2, x)
    assert float(np.linalg.norm(dA - dA_ld) / np.linalg.norm(dA_ld)) < 1e-8


# ---------------------------------------------------------------- float32 factor check
def _near_dependent(delta, seed=3):
    A = dense_with_condition(600, 40, 1e2, seed=seed)
    rng = np.random.default_rng(seed + 1)
    A[:, 7] = A[:, 3] + delta * np.linalg.norm(A[:, 3]) * rng.standard_normal(600) / np.sqrt(600)
    return A, rng.standard_normal(600)


def test_rho_min_is_the_distance_of_a_column_from_the_span_before_it():
    # rho_j = |r_jj| / ||SA[:, j]|| is the sine of the angle between column j
    # and the span of the columns before it: check it against a least-squares
    # projection computed independently
    A, _ = _near_dependent(1e-6)
    R = qr.r_factor(A)
    for j in (3, 7, 20):
        coef = np.linalg.lstsq(A[:, :j], A[:, j], rcond=None)[0]
        dist = np.linalg.norm(A[:, j] - A[:, :j] @ coef) / np.linalg.norm(A[:, j])
        assert abs(abs(R[j, j]) / np.linalg.norm(R[:, j]) - dist) <= 1e-9 * dist
    assert abs(qr.rho_min(R) - 1e-6) <= 0.2e-6


def test_float32_factor_refused_where_it_cannot_precondition():
    # a column within 1e-11 of an earlier one: the float32 QR leaves only
    # rounding noise in that direction (its rho_min falls to the noise floor),
    # the check refuses it, and without the check LSQR on A R32^{-1} ends far
    # from the optimum that the float64 factor reaches
    A, b = _near_dependent(1e-11)
    m, n = A.shape
    rp, col, val = csr_from_dense(A, keep_zeros=True)
    with pytest.raises(qr.PrecisionInsufficient):
        pipeline.precondition(rp, col, val, m, n, 4 * n, 5, qr_dtype="f32")
    with pytest.raises(qr.PrecisionInsufficient):
        pipeline.precondition(rp, col, val, m, n, 4 * n, 5, qr_dtype="f64", r_store="f32")
    R64 = pipeline.precondition(rp, col, val, m, n, 4 * n, 5)["R"]
    R32 = pipeline.precondition(rp, col, val, m, n, 4 * n, 5, qr_dtype="f32", check_precision=False)["R"]
    # float64 resolves the true distance; float32's value is noise, far from it
    assert abs(qr.rho_min(R64) - 1e-11) <= 0.2e-11
    r32 = qr.rho_min(R32)
    assert r32 <= qr.PRECISION_TOL and not 0.1 < r32 / 1e-11 < 10.0
    rstar = np.linalg.norm(b - A @ np.linalg.lstsq(A, b, rcond=None)[0])
    errs = {}
    for name, R in (("f64", R64), ("f32", R32)):
        x, _ = pipeline.lsqr_on_preconditioned(sp.csr_matrix(A), R, b, itmax=200)
        errs[name] = abs(np.linalg.norm(b - A @ x) - rstar) / rstar
    assert errs["f64"] <= 1e-7 and errs["f32"] >= 1e-6


def test_float32_factor_on_rfm_3x3_accepted_and_4x4_refused():
    # 3x3-box RFM system: the float32 factor's rho_min (4.3e-6) clears 16 u32
    # and the float32 form reaches the float64 optimum.  4x4-box system: its
    # rho_min (1.0e-7 in float32, 9.7e-8 in float64) is within 16 u32, so it is
    # refused; the float32 form there still converges, but needs about three
    # times the iterations of the float64 one (measured on the GPU: 187 vs 56)
    S, s = build_config("poisson2d_3x3")
    o64 = pipeline.solve(S.row_ptr, S.col, S.val, S.b[0], S.m, S.n, s, 2, refine=1)
    o32 = pipeline.solve(S.row_ptr, S.col, S.val, S.b[0], S.m, S.n, s, 2, refine=1, qr_dtype="f32",
                         r_store="f32")
    assert qr.rho_min(o32["R"]) > qr.PRECISION_TOL
    assert o32["istop"] in (1, 2)
    assert abs(o32["normr"] - o64["normr"]) <= 1e-10 * o64["normr"]
    S, s = build_config("poisson2d_4x4")
    with pytest.raises(qr.PrecisionInsufficient):
        pipeline.precondition(S.row_ptr, S.col, S.val, S.m, S.n, s, 2, qr_dtype="f32", r_store="f32")
