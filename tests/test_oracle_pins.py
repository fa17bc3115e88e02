"""Pins of the CPU oracle to facts fixed by the paper and by mathematics.

Every check here is independent of the oracle's own formulas: published
generator vectors, the paper's worked example, closed forms, invariants of the
factorisation, an independent LSQR implementation (scipy), dense least-squares
solutions, Thm 3.2's conditioning bound, eq. (3.5)-(3.6)'s convergence bound,
finite differences for the gradients and the manufactured-solution trend of
the RFM (Sec. 4, Ex. 4.4)."""

import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import backward, countsketch, pipeline, qr, svd
from oracle.lsqr import lsqr
from rfmgen import (build_config, csr_from_dense, dense_from_csr, dense_with_condition,
                    exact_solution, feature_eval, poisson_system, random_csr, sample_points)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- count sketch
def test_splitmix64_reference_vectors():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64_vectors.txt"))
            if l.strip() and not l.startswith("#")]
    by_seed = {}
    for seed, idx, val in rows:
        by_seed.setdefault(int(seed), []).append((int(idx), int(val, 16)))
    for seed, items in by_seed.items():
        out = countsketch.splitmix64_stream(seed, max(i for i, _ in items) + 1)
        for i, v in items:
            assert int(out[i]) == v, (seed, i)


def test_hash_uniform_and_signs_balanced():
    m, s = 400_000, 1000
    h, sign = countsketch.hash_sign(m, s, seed=12345)
    assert h.min() >= 0 and h.max() < s
    counts = np.bincount(h, minlength=s)
    e = m / s
    chi2 = ((counts - e) ** 2 / e).sum()
    assert abs(chi2 - (s - 1)) < 6 * np.sqrt(2 * (s - 1))  # Def. 2.3: h(i) = j w.p. 1/s
    assert abs(int(sign.astype(np.int64).sum())) < 6 * np.sqrt(m)  # D: +-1 equiprobable
    assert set(np.unique(sign)) == {-1, 1}


def test_hash_power_of_two_range_is_top_bits():
    # multiply-shift with s = 2^k keeps the top k bits of the 64-bit output
    m, k = 1000, 10
    h, _ = countsketch.hash_sign(m, 1 << k, seed=7)
    x = countsketch.splitmix64_stream(7, m)
    assert np.array_equal(h.astype(np.uint64), x >> np.uint64(64 - k))


def test_worked_example_matrix():
    S_paper = np.loadtxt(os.path.join(GOLDEN, "worked_example_S.txt"))
    h = np.array([1, 3, 0, 0, 2], dtype=np.int32)
    sign = np.array([1, -1, -1, 1, 1], dtype=np.int8)
    assert np.array_equal(countsketch.explicit_S(h, sign, 4), S_paper)
    rng = np.random.default_rng(0)
    A = rng.integers(-9, 10, size=(5, 7)).astype(np.float64)
    rp, col, val = csr_from_dense(A)
    SA, _ = countsketch.sketch_dense(rp, col, val, h, sign, 4, 7)
    assert np.array_equal(SA, S_paper @ A)  # integer data: every summation order is exact


def test_sketch_equals_explicit_product():
    rp, col, val = random_csr(300, 40, 0.2, seed=3, empty_rows=(5, 17))
    h, sign = countsketch.hash_sign(300, 90, seed=9)
    SA, Sb = countsketch.sketch_dense(rp, col, val, h, sign, 90, 40, b=np.arange(300.0))
    S = countsketch.explicit_S(h, sign, 90)
    A = dense_from_csr(rp, col, val, 300, 40)
    assert np.allclose(SA, S @ A, rtol=1e-14, atol=1e-14)
    assert np.allclose(Sb, S @ np.arange(300.0), rtol=0, atol=1e-10)
    # one nonzero per column of S: sum of bucket sizes is m
    ptr, perm = countsketch.bucket_rows(h, 90)
    assert ptr[-1] == 300 and np.array_equal(np.sort(perm), np.arange(300))


def test_sketch_sums_in_ascending_row_order():
    # three rows in one bucket whose float sum depends on the order
    A = np.array([[1e16], [1.0], [-1e16]])
    rp, col, val = csr_from_dense(A)
    h = np.zeros(3, dtype=np.int32)
    sign = np.ones(3, dtype=np.int8)
    SA, _ = countsketch.sketch_dense(rp, col, val, h, sign, 1, 1)
    assert SA[0, 0] == ((0.0 + 1e16) + 1.0) + (-1e16)  # = 0.0 in float64
    h2 = np.array([0, 0, 0], dtype=np.int32)
    A2 = np.array([[1.0], [1e16], [-1e16]])
    SA2, _ = countsketch.sketch_dense(*csr_from_dense(A2), h2, sign, 1, 1)
    assert SA2[0, 0] == 1.0 + 1e16 - 1e16


# ---------------------------------------------------------------- R factor
def test_r_factor_defining_identity():
    rng = np.random.default_rng(1)
    SA = rng.standard_normal((400, 60))
    R = qr.r_factor(SA)
    assert np.allclose(np.tril(R, -1), 0) and np.all(np.diag(R) > 0)
    err = np.linalg.norm(R.T @ R - SA.T @ SA) / np.linalg.norm(SA) ** 2
    assert err < 60 * 1.2e-16 * 10
    Q = sla.solve_triangular(R, SA.T, trans="T").T  # Q = SA R^{-1}
    assert np.abs(Q.T @ Q - np.eye(60)).max() < 1e-13


def test_r_textbook_equals_lapack():
    rng = np.random.default_rng(2)
    M = rng.standard_normal((50, 12))
    assert np.allclose(qr.r_factor(M), qr.r_factor_textbook(M), rtol=1e-12, atol=1e-12)


def test_r_closed_form_2x2():
    a, b, c, d = 3.0, -1.0, 4.0, 2.0
    R = qr.r_factor(np.array([[a, b], [c, d]]))
    r11 = np.hypot(a, c)
    assert np.allclose(R, [[r11, (a * b + c * d) / r11], [0.0, abs(a * d - b * c) / r11]], rtol=1e-15)


def test_rank_deficient_sketch_is_rejected():
    rng = np.random.default_rng(4)
    M = rng.standard_normal((100, 8))
    M[:, 5] = M[:, 2]
    with pytest.raises(qr.RankDeficient):
        qr.r_factor(M)


# ---------------------------------------------------------------- LSQR
def _small_problem(m=120, n=15, kappa=1e3, seed=5):
    A = dense_with_condition(m, n, kappa, seed=seed)
    b = np.random.default_rng(seed + 1).standard_normal(m)
    return A, b


def test_lsqr_iterates_match_scipy():
    # an independent implementation of the same recurrences; kappa = 10 keeps the
    # iterates' own sensitivity to rounding near 1e-15 for these k
    A, b = _small_problem(kappa=10.0)
    for k in range(1, 9):
        ours = lsqr(lambda v: A @ v, lambda u: A.T @ u, b, A.shape[1], atol=0, btol=0, conlim=0,
                    itmax=k)
        ref = spla.lsqr(A, b, atol=0, btol=0, conlim=0, iter_lim=k)
        assert np.allclose(ours.y, ref[0], rtol=1e-12, atol=1e-13), k
        assert abs(ours.normr - ref[3]) <= 1e-12 * abs(ref[3])


def test_lsqr_reaches_dense_solution():
    A, b = _small_problem(kappa=1e2)
    res = lsqr(lambda v: A @ v, lambda u: A.T @ u, b, A.shape[1], itmax=500)
    xs = np.linalg.lstsq(A, b, rcond=None)[0]
    assert res.istop in (1, 2)
    assert np.linalg.norm(res.y - xs) <= 1e-8 * np.linalg.norm(xs)


def test_lsqr_degenerate_cases():
    A, b = _small_problem()
    r0 = lsqr(lambda v: A @ v, lambda u: A.T @ u, np.zeros(A.shape[0]), A.shape[1])
    assert r0.itn == 0 and r0.istop == 0 and not r0.y.any()
    A0 = A.copy()
    A0[-10:] = 0.0
    bperp = np.zeros(A.shape[0])
    bperp[-3:] = [1.0, -2.0, 0.5]  # exactly orthogonal to range(A0): A0^T b = 0
    r1 = lsqr(lambda v: A0 @ v, lambda u: A0.T @ u, bperp, A.shape[1])
    assert r1.itn == 0 and np.linalg.norm(r1.y) == 0.0
    r2 = lsqr(lambda v: A @ v, lambda u: A.T @ u, b, A.shape[1], itmax=1)
    assert r2.itn == 1 and r2.istop == 7


def test_injective_sketch_gives_one_iteration():
    # s >= m with distinct buckets: SA = P D A, so R is A's own factor, A R^{-1}
    # has orthonormal columns and LSQR converges in one step (Thm 3.2, eps = 0).
    A, b = _small_problem(m=80, n=10, kappa=1e6)
    rp, col, val = csr_from_dense(A)
    m, n = A.shape
    h = np.random.default_rng(3).permutation(m).astype(np.int32)
    sign = np.where(np.arange(m) % 3 == 0, -1, 1).astype(np.int8)
    SA, _ = countsketch.sketch_dense(rp, col, val, h, sign, m, n)
    R = qr.r_factor(SA)
    x, res = pipeline.lsqr_on_preconditioned(sp.csr_matrix(A), R, b)
    assert res.itn == 1
    xs = np.linalg.lstsq(A, b, rcond=None)[0]
    assert np.linalg.norm(A @ (x - xs)) <= 1e-10 * np.linalg.norm(b)


@pytest.mark.parametrize("kappa", [1e2, 1e6, 1e10, 1e14])
def test_preconditioned_condition_independent_of_kappa(kappa):
    # Thm 3.2: kappa(A R^{-1}) <= sqrt((1+eps)/(1-eps)), not depending on kappa(A)
    m, n = 3000, 50
    A = dense_with_condition(m, n, kappa, seed=11)
    rp, col, val = csr_from_dense(A, keep_zeros=True)
    pre = pipeline.precondition(rp, col, val, m, n, 4 * n, seed=2)
    B = sla.solve_triangular(pre["R"], A.T, trans="T").T
    sv = np.linalg.svd(B, compute_uv=False)
    assert sv[0] / sv[-1] < 10.0


def test_energy_norm_bound_eq_3_5():
    # ||y_k - y*||_{B^T B} <= 2 rho^k ||y_0 - y*||_{B^T B}, rho = (kappa(B)-1)/(kappa(B)+1)
    m, n = 2000, 40
    A = dense_with_condition(m, n, 1e8, seed=21)
    b = np.random.default_rng(0).standard_normal(m)
    rp, col, val = csr_from_dense(A, keep_zeros=True)
    R = pipeline.precondition(rp, col, val, m, n, 3 * n, seed=5)["R"]
    B = sla.solve_triangular(R, A.T, trans="T").T
    sv = np.linalg.svd(B, compute_uv=False)
    rho = (sv[0] / sv[-1] - 1) / (sv[0] / sv[-1] + 1)
    ystar = np.linalg.lstsq(B, b, rcond=None)[0]
    e0 = np.linalg.norm(B @ ystar)
    for k in range(1, 12):
        yk = lsqr(lambda v: B @ v, lambda u: B.T @ u, b, n, atol=0, btol=0, conlim=0, itmax=k).y
        assert np.linalg.norm(B @ (yk - ystar)) <= 2 * rho ** k * e0 * (1 + 1e-6) + 1e-12


def test_explicit_and_implicit_operators_agree():
    # Remark 3.3: identical in exact arithmetic; on a mildly conditioned system
    # the two final residual norms agree closely.
    S, s = build_config("poisson2d_2x2")
    A = pipeline.csr(S.row_ptr, S.col, S.val, S.m, S.n)
    R = pipeline.precondition(S.row_ptr, S.col, S.val, S.m, S.n, s, 2)["R"]
    xi, ri = pipeline.lsqr_on_preconditioned(A, R, S.b[0], operator="implicit")
    xe, re = pipeline.lsqr_on_preconditioned(A, R, S.b[0], operator="explicit")
    ni = np.linalg.norm(S.b[0] - A @ xi)
    ne = np.linalg.norm(S.b[0] - A @ xe)
    assert abs(ni - ne) <= 1e-10 * ne
    assert abs(ri.itn - re.itn) <= 2


def test_refined_solve_reaches_dense_optimum():
    S, s = build_config("poisson2d_3x3")
    Ad = dense_from_csr(S.row_ptr, S.col, S.val, S.m, S.n)
    Q, RA = np.linalg.qr(Ad)
    xs = sla.solve_triangular(RA, Q.T @ S.b[0])
    rstar = np.linalg.norm(S.b[0] - Ad @ xs)
    out = pipeline.solve(S.row_ptr, S.col, S.val, S.b[0], S.m, S.n, s, 2, refine=1)
    assert abs(out["normr"] - rstar) <= 1e-10 * rstar
    assert out["istop"] in (1, 2)


# --------------------------------------------- SVD preconditioner (Alg. 2)
def test_svd_2x2_closed_form():
    # singular values of [[a, b], [c, d]]: (sqrt((a+d)^2+(b-c)^2) +- sqrt((a-d)^2+(b+c)^2)) / 2
    rng = np.random.default_rng(7)
    for _ in range(20):
        a, b, c, d = rng.standard_normal(4)
        p, q = np.hypot(a + d, b - c), np.hypot(a - d, b + c)
        sigma, V, r, P = svd.svd_preconditioner(np.array([[a, b], [c, d]]))
        assert np.allclose(sigma, [(p + q) / 2, abs(p - q) / 2], rtol=1e-13, atol=1e-15)
        assert r == 2 and P.shape == (2, 2)


def _constructed(s, sig, seed):
    # U (s x n) and V (n x n) with orthonormal columns from Householder QR of
    # random matrices; SA = U diag(sig) V^T has exactly the singular values sig
    rng = np.random.default_rng(seed)
    n = len(sig)
    U, _ = np.linalg.qr(rng.standard_normal((s, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (U * np.asarray(sig)) @ V.T, U, V


def test_svd_recovers_constructed_factors():
    sig = np.geomspace(1.0, 1e-6, 8)
    SA, U, V = _constructed(60, sig, 3)
    sigma, Vo, r, P = svd.svd_preconditioner(SA)
    assert r == 8
    assert np.max(np.abs(sigma - sig)) <= 1e-14
    # right singular vectors equal the construction's up to sign (distinct sigma)
    assert np.allclose(np.abs(np.sum(Vo * V, axis=0)), 1.0, atol=1e-9)
    # P = V Sigma^{-1}: SA P = U up to column signs, i.e. orthonormal columns
    SP = SA @ P
    assert np.max(np.abs(SP.T @ SP - np.eye(8))) <= 1e-9
    assert np.allclose(np.abs(np.sum(SP * U, axis=0)), 1.0, atol=1e-9)


def test_svd_rank_truncation():
    sig = np.array([1.0, 0.3, 1e-9, 1e-17, 0.0])
    SA, U, V = _constructed(40, sig, 5)
    sigma, Vo, r, P = svd.svd_preconditioner(SA)  # rcond = n u = 5.6e-16
    assert r == 3 and P.shape == (5, 3)
    SP = SA @ P
    assert np.max(np.abs(SP.T @ SP - np.eye(3))) <= 1e-6  # sigma_3 = 1e-9 amplifies u by 1e9
    assert svd.svd_preconditioner(SA, rcond=1e-6)[2] == 2
    # the threshold is relative to sigma_1: scaling SA keeps the rank
    assert svd.svd_preconditioner(1e3 * SA)[2] == 3
    assert svd.svd_preconditioner(1e-3 * SA)[2] == 3
    assert svd.svd_preconditioner(np.zeros((6, 3)))[2] == 0


def test_cssvdp_injective_sketch_gives_one_iteration():
    A, b = _small_problem(m=80, n=10, kappa=1e6)
    rp, col, val = csr_from_dense(A)
    m, n = A.shape
    h = np.random.default_rng(3).permutation(m).astype(np.int32)
    sign = np.where(np.arange(m) % 3 == 0, -1, 1).astype(np.int8)
    SA, _ = countsketch.sketch_dense(rp, col, val, h, sign, m, n)
    _, _, r, P = svd.svd_preconditioner(SA)
    x, res = pipeline.lsqr_on_svd_preconditioned(sp.csr_matrix(A), P, b)
    assert r == n and res.itn == 1
    Q, RA = np.linalg.qr(A)
    xs = sla.solve_triangular(RA, Q.T @ b)
    assert np.linalg.norm(A @ (x - xs)) <= 1e-10 * np.linalg.norm(b)


@pytest.mark.parametrize("kappa", [1e2, 1e8, 1e14])
def test_svd_preconditioned_condition_independent_of_kappa(kappa):
    m, n = 3000, 50
    A = dense_with_condition(m, n, kappa, seed=11)
    rp, col, val = csr_from_dense(A, keep_zeros=True)
    h, sign = countsketch.hash_sign(m, 4 * n, 2)
    SA, _ = countsketch.sketch_dense(rp, col, val, h, sign, 4 * n, n)
    _, _, r, P = svd.svd_preconditioner(SA)
    sv = np.linalg.svd(A @ P, compute_uv=False)
    assert r == n and sv[0] / sv[-1] < 10.0


def test_cssvdp_minimum_norm_with_a_duplicated_column():
    # Sec. 3.2 / Thm 3.4: a rank-deficient A; duplicating column j of a full-rank
    # A0 leaves the residual unchanged and the minimum-norm solution splits
    # A0's coefficient x0_j equally between the two copies.
    A0, b = _small_problem(m=300, n=12, kappa=1e3)
    j = 4
    A = np.hstack([A0, A0[:, [j]]])
    m, n = A.shape
    rp, col, val = csr_from_dense(A)
    out = pipeline.solve_svd(rp, col, val, b, m, n, 4 * n, seed=9, rcond=1e-12)
    assert out["rank"] == n - 1
    Q, R0 = np.linalg.qr(A0)
    x0 = sla.solve_triangular(R0, Q.T @ b)
    x = out["x"]
    assert abs(x[j] - x[n - 1]) <= 1e-9 * np.abs(x0).max()
    expect = x0.copy()
    expect[j] = x0[j] / 2
    assert np.max(np.abs(x[:n - 1] - expect)) <= 1e-9 * np.abs(x0).max()
    # the QR preconditioner cannot be formed for this A
    with pytest.raises(qr.RankDeficient):
        pipeline.precondition(rp, col, val, m, n, 4 * n, seed=9)


def test_cssvdp_and_csqrp_reach_the_same_optimum():
    S, s = build_config("poisson2d_2x2")
    qo = pipeline.solve(S.row_ptr, S.col, S.val, S.b[0], S.m, S.n, s, 2, refine=1)
    so = pipeline.solve_svd(S.row_ptr, S.col, S.val, S.b[0], S.m, S.n, s, 2, refine=1)
    assert so["rank"] == S.n
    assert abs(so["normr"] - qo["normr"]) <= 1e-10 * qo["normr"]
    assert so["istop"] in (1, 2)


# ------------------------------------------------- starting point (Remark 3.1)
def _sketch_case(m=300, n=12, s=60, kappa=1e3, seed=4, k=1):
    A = dense_with_condition(m, n, kappa, seed=seed)
    B = np.random.default_rng(seed + 1).standard_normal((k, m))
    rp, col, val = csr_from_dense(A, keep_zeros=True)
    h, sign = countsketch.hash_sign(m, s, seed + 2)
    SA, SB = countsketch.sketch_dense(rp, col, val, h, sign, s, n, b=B)
    return A, B, SA, SB.T  # SB: s x k


def test_sketched_start_minimises_the_sketched_residual():
    A, B, SA, SB = _sketch_case()
    R, Y0, X0 = pipeline.sketched_start(SA, SB)
    xs = np.linalg.lstsq(SA, SB[:, 0], rcond=None)[0]
    assert np.linalg.norm(X0[:, 0] - xs) <= 1e-10 * np.linalg.norm(xs)
    # the extended factor's last pivot is the sketched residual norm
    Rx = qr.r_factor(np.hstack([SA, SB]), check_rank=False)
    assert abs(Rx[-1, -1] - np.linalg.norm(SA @ xs - SB[:, 0])) <= 1e-10 * np.linalg.norm(SB)
    # R is the sketch's own factor and Y0 = Q^T S b with Q = SA R^{-1}
    assert np.linalg.norm(R.T @ R - SA.T @ SA) <= 1e-12 * np.linalg.norm(SA) ** 2
    Q = sla.solve_triangular(R, SA.T, trans="T").T
    assert np.linalg.norm(Y0[:, 0] - Q.T @ SB[:, 0]) <= 1e-10 * np.linalg.norm(SB)


def test_sketched_start_columns_are_independent():
    A, B, SA, SB = _sketch_case(k=3)
    _, _, X0 = pipeline.sketched_start(SA, SB)
    for k in range(3):
        _, _, xk = pipeline.sketched_start(SA, SB[:, k])
        assert np.linalg.norm(X0[:, k] - xk[:, 0]) <= 1e-12 * np.linalg.norm(xk)


def test_sketched_start_with_injective_sketch_is_the_solution():
    # s >= m with distinct buckets: ||S (A x - b)|| = ||A x - b||, so x0 is already
    # the least-squares solution and a sweep from it has nothing left to do
    A, b = _small_problem(m=80, n=10, kappa=1e6)
    rp, col, val = csr_from_dense(A)
    m, n = A.shape
    h = np.random.default_rng(3).permutation(m).astype(np.int32)
    sign = np.where(np.arange(m) % 3 == 0, -1, 1).astype(np.int8)
    SA, Sb = countsketch.sketch_dense(rp, col, val, h, sign, m, n, b=b)
    R, _, X0 = pipeline.sketched_start(SA, Sb)
    xs = np.linalg.lstsq(A, b, rcond=None)[0]
    assert np.linalg.norm(A @ (X0[:, 0] - xs)) <= 1e-10 * np.linalg.norm(b)
    _, res = pipeline.refined_lsqr(sp.csr_matrix(A), R, b, refine=0, x0=X0[:, 0])
    assert res[0].itn <= 1


def test_sketched_start_recovers_a_consistent_solution():
    m, n = 400, 15
    A = dense_with_condition(m, n, 1e4, seed=9)
    xt = np.random.default_rng(10).standard_normal(n)
    b = A @ xt
    rp, col, val = csr_from_dense(A, keep_zeros=True)
    h, sign = countsketch.hash_sign(m, 4 * n, 7)
    SA, Sb = countsketch.sketch_dense(rp, col, val, h, sign, 4 * n, n, b=b)
    _, _, X0 = pipeline.sketched_start(SA, Sb)
    assert np.linalg.norm(X0[:, 0] - xt) <= 1e-9 * np.linalg.norm(xt)


def test_solve_from_sketched_start_reaches_dense_optimum_sooner():
    S, s = build_config("poisson2d_3x3")
    Ad = dense_from_csr(S.row_ptr, S.col, S.val, S.m, S.n)
    Q, RA = np.linalg.qr(Ad)
    xs = sla.solve_triangular(RA, Q.T @ S.b[0])
    rstar = np.linalg.norm(S.b[0] - Ad @ xs)
    cold = pipeline.solve(S.row_ptr, S.col, S.val, S.b[0], S.m, S.n, s, 2, refine=1)
    warm = pipeline.solve(S.row_ptr, S.col, S.val, S.b[0], S.m, S.n, s, 2, refine=1,
                          start="sketch")
    assert abs(warm["normr"] - rstar) <= 1e-10 * rstar
    assert warm["istop"] in (1, 2)
    assert warm["itn"] < cold["itn"]


# ---------------------------------------------------------------- gradients
def test_dense_gradients_match_finite_differences():
    rng = np.random.default_rng(8)
    m, n = 30, 6
    Ad = rng.standard_normal((m, n))
    b = rng.standard_normal(m)
    E = rng.standard_normal((5, n))
    t = rng.standard_normal(5)

    def loss(Ax, bx):
        x = np.linalg.lstsq(Ax, bx, rcond=None)[0]
        return 0.5 * np.sum((E @ x - t) ** 2)

    x, r, w, lam = backward.dense_gradients(Ad, b, E.T @ (E @ np.linalg.lstsq(Ad, b, rcond=None)[0] - t))
    rp, col, _ = csr_from_dense(Ad, keep_zeros=True)
    dA = backward.pattern_grad(rp, col, r, w, lam, x).reshape(m, n)
    eps = 1e-6
    for i in range(0, m, 7):
        db = np.zeros(m)
        db[i] = eps
        fd = (loss(Ad, b + db) - loss(Ad, b - db)) / (2 * eps)
        assert abs(fd - lam[i]) <= 1e-6 * (1 + abs(fd))
        for j in range(n):
            dAe = np.zeros((m, n))
            dAe[i, j] = eps
            fd = (loss(Ad + dAe, b) - loss(Ad - dAe, b)) / (2 * eps)
            assert abs(fd - dA[i, j]) <= 1e-6 * (1 + abs(fd))


def test_iterative_gradients_match_dense():
    m, n = 400, 30
    Ad = dense_with_condition(m, n, 1e4, seed=31)
    rng = np.random.default_rng(32)
    b = rng.standard_normal(m)
    g = rng.standard_normal(n)
    x, r, w, lam = backward.dense_gradients(Ad, b, g)
    rp, col, val = csr_from_dense(Ad, keep_zeros=True)
    R = pipeline.precondition(rp, col, val, m, n, 4 * n, seed=1)["R"]
    w2, lam2, itn = backward.iterative_gradients(sp.csr_matrix(Ad), R, x, r, g)
    assert np.linalg.norm(lam2 - lam) <= 1e-8 * np.linalg.norm(lam)
    assert np.linalg.norm(w2 - w) <= 1e-6 * np.linalg.norm(w)
    assert itn < 60


# ---------------------------------------------------------------- RFM inputs
def test_workload_sizes():
    for name, (m, n, nnz, s) in {"poisson2d_2x2": (1920, 200, 104000, 800),
                                 "poisson2d_8x8": (112640, 12800, 24320000, 51200)}.items():
        S, sk = build_config(name)
        assert (S.m, S.n, S.nnz, sk) == (m, n, nnz, s)
        assert np.all(np.diff(S.row_ptr) > 0)
        for i in (0, S.m // 2, S.m - 1):
            c = S.col[S.row_ptr[i]:S.row_ptr[i + 1]]
            assert np.all(np.diff(c) > 0)


def test_manufactured_solution_error_decreases_with_features():
    # RFM converges as the number of features grows (Sec. 4, Ex. 4.4 trend)
    pts = sample_points(2, 2000)
    errs = []
    for J in (10, 20, 35, 50):
        S = poisson_system(2, 2, J, 20)
        out = pipeline.solve(S.row_ptr, S.col, S.val, S.b[0], S.m, S.n, 4 * S.n, 2)
        E = pipeline.csr(*feature_eval(S, pts), len(pts), S.n)
        errs.append(pipeline.l2_error(E, out["x"], exact_solution(pts)))
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-2


# ------------------------------------------- Helmholtz inputs (Example 4.5)
def _fd_laplacian(fun, p, h=1e-3):
    lap = np.zeros(p.shape[0])
    for a in range(p.shape[1]):
        e = np.zeros(p.shape[1])
        e[a] = h
        lap += (fun(p + e) - 2.0 * fun(p) + fun(p - e)) / (h * h)
    return lap


def test_helmholtz_rhs_and_rows_match_finite_differences():
    S, _ = build_config("helmholtz3d_2x2x2_small", modes=(1, 2, 3))
    pts = np.random.default_rng(5).uniform(0.1, 0.9, (40, 3))
    for k in (1, 2, 3):
        # f = Laplace(u) + kappa^2 u (second-order differences, h = 1e-3)
        f_fd = _fd_laplacian(lambda q: S.exact(q, k), pts) + S.kwave ** 2 * S.exact(pts, k)
        f_gen = build_config.__globals__["_rhs_f"](pts, k, "helmholtz", S.kwave)
        assert np.abs(f_fd - f_gen).max() <= 1e-4 * np.abs(f_gen).max()
    # an interior row holds Laplace(phi_j) + kappa^2 phi_j of box 0's features at its point
    row = 5
    c0 = S.centres[0]
    Q = S.Q
    ijk = np.unravel_index(row, (Q, Q, Q))
    p = (c0 - S.radius + (np.array(ijk) + 0.5) * 2 * S.radius / Q)[None, :]
    vals = S.val[S.row_ptr[row]:S.row_ptr[row + 1]]
    for j in (0, 7, S.J - 1):
        phi = lambda q: np.tanh(((q - c0) / S.radius) @ S.W[0][j] + S.B0[0][j])
        want = _fd_laplacian(phi, p)[0] + S.kwave ** 2 * phi(p)[0]
        assert abs(vals[j] - want) <= 1e-4 * max(1.0, abs(want))
    # Dirichlet data is the exact solution
    assert S.counts == {"interior": 4096, "dirichlet": 1536, "interface": 1536}


def test_helmholtz_manufactured_error_decreases_with_features():
    pts = sample_points(3, 2000)
    errs = []
    for J in (50, 100, 200):  # measured 0.50, 0.10, 0.014 (12 points per axis)
        S = poisson_system(3, 2, J, 12, pde="helmholtz", kwave=0.5)
        out = pipeline.solve(S.row_ptr, S.col, S.val, S.b[0], S.m, S.n, 4 * S.n, 2)
        E = pipeline.csr(*feature_eval(S, pts), len(pts), S.n)
        errs.append(pipeline.l2_error(E, out["x"], S.exact(pts)))
    assert all(e2 < 0.5 * e1 for e1, e2 in zip(errs, errs[1:])), errs
    assert errs[-1] < 0.05
