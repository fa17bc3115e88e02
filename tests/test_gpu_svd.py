"""GPU parity of the CSSVDP-LSQR path (Alg. 2) against the CPU oracle.

The singular values from the GPU's Jacobi SVD of R are compared with LAPACK's
SVD of the oracle's sketch (to a few units of rounding relative to sigma_1;
singular vectors are not unique, so they are checked through the property the
preconditioner needs: the columns of SA P kept by the truncation are
orthonormal to the rounding that kappa(SA) amplifies).  The solve is gated as
CSQRP-LSQR's: true residual within 1e-10 of the oracle's, PDE error within
1.1x.  Inputs are the oracle's seeded generators; nothing here feeds a GPU
result to the oracle."""

import numpy as np
import pytest

from oracle import backward, countsketch, pipeline, svd as osvd
from rfmgen import (build_config, csr_from_dense, dense_from_csr, dense_with_condition,
                    feature_eval, sample_points)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2409_15818_amd")

SEED = 2
SMALL = ["poisson2d_2x2", "poisson2d_3x3", "poisson3d_2x2x2", "helmholtz3d_2x2x2_small"]
U64 = 2.0 ** -53


def gpu_csr(rp, col, val, m, n):
    return R.CSR.from_numpy(rp, col, val, m, n)


def oracle_sketch(rp, col, val, m, n, s, seed=SEED):
    h, sign = countsketch.hash_sign(m, s, seed)
    return countsketch.sketch_dense(rp, col, val, h, sign, s, n)[0]


def l2(S, x):
    pts = sample_points(S.d)
    E = pipeline.csr(*feature_eval(S, pts), len(pts), S.n)
    return pipeline.l2_error(E, x, S.exact(pts))


def check_svd(handle, rp, col, val, m, n, s, rcond=0.0, sigma_tol=2e-12):
    """Sketch and SVD preconditioner on the GPU, checked against the oracle."""
    A = gpu_csr(rp, col, val, m, n)
    SA = R.rfmls_sketch(handle, A, s, SEED)[0]
    P = R.rfmls_precond_svd(handle, SA, n, rcond=rcond)
    sig = R.rfmls_precond_export_sigma(handle, P).cpu().numpy()
    Pg = R.rfmls_precond_export_P(handle, P).cpu().numpy()
    SAo = oracle_sketch(rp, col, val, m, n, s)
    so, _, ro, _ = osvd.svd_preconditioner(SAo, rcond if rcond > 0 else None)
    assert P.status == 0 and P.sweeps >= 1, (P.status, P.sweeps, P.off)
    assert P.rank == ro
    assert np.max(np.abs(np.sort(sig)[::-1] - so)) <= sigma_tol * so[0]
    keep = sig > (rcond if rcond > 0 else n * U64) * sig.max()
    assert int(keep.sum()) == P.rank
    assert not Pg[:, ~keep].any()  # dropped directions are zero columns
    # SA P_r has orthonormal columns up to the rounding kappa(SA_r) amplifies
    U = SAo @ Pg[:, keep]
    kap = so[0] / so[ro - 1]
    dev = np.max(np.abs(U.T @ U - np.eye(P.rank)))
    assert dev <= n * U64 * kap + 1e-12, (dev, kap)
    return P, sig, Pg, so


@pytest.mark.parametrize("name", SMALL)
def test_svd_preconditioner_matches_oracle(handle, name):
    S, s = build_config(name)
    check_svd(handle, S.row_ptr, S.col, S.val, S.m, S.n, s)


@pytest.mark.parametrize("n", [1, 2, 3, 63, 65, 257, 600, 1100])
def test_svd_ragged_sizes(handle, n):
    # odd n (a padding column in the round-robin), sizes around the 64-tiles and
    # the rows-per-thread steps of the Jacobi kernel
    m = 4 * n + 40
    Ad = dense_with_condition(m, n, 1e5, seed=n)
    rp, col, val = csr_from_dense(Ad, keep_zeros=True)
    check_svd(handle, rp, col, val, m, n, 2 * n + 5)


def test_svd_truncates_a_rank_deficient_sketch(handle):
    m, n = 300, 13
    A0 = dense_with_condition(m, n - 1, 1e3, seed=41)
    Ad = np.hstack([A0, A0[:, [4]]])
    rp, col, val = csr_from_dense(Ad)
    P, sig, Pg, so = check_svd(handle, rp, col, val, m, n, 4 * n, rcond=1e-12)
    assert P.rank == n - 1


@pytest.mark.parametrize("name", SMALL)
@pytest.mark.parametrize("store", ["f64", "f32"])
def test_cssvdp_pipeline_parity(handle, name, store):
    S, s = build_config(name)
    A = gpu_csr(S.row_ptr, S.col, S.val, S.m, S.n)
    b = torch.tensor(S.b[0], device="cuda")
    res = R.cssvdp_lsqr(handle, A, b, s, SEED, p_store=store)
    info = res.info[0]
    orc = pipeline.solve_svd(S.row_ptr, S.col, S.val, S.b[0], S.m, S.n, s, SEED)
    assert res.status == 0 and info["istop"] in (1, 2)
    assert abs(info["normr"] - orc["normr"]) <= 1e-10 * orc["normr"], (info["normr"], orc["normr"])
    x = res.x.cpu().numpy()
    assert l2(S, x) <= 1.1 * l2(S, orc["x"])
    if store == "f64":
        assert abs(info["itn_first"] - orc["itn_sweeps"][0]) <= 2
    # the same least-squares optimum as CSQRP-LSQR
    qo = pipeline.solve(S.row_ptr, S.col, S.val, S.b[0], S.m, S.n, s, SEED)
    assert abs(info["normr"] - qo["normr"]) <= 1e-10 * qo["normr"]


def test_cssvdp_minimum_norm_solution(handle):
    # Thm 3.4: with a duplicated column the truncated problem's minimum-norm
    # solution splits the original coefficient equally between the copies
    m, n, j = 300, 13, 4
    A0 = dense_with_condition(m, n - 1, 1e3, seed=41)
    b = np.random.default_rng(42).standard_normal(m)
    Ad = np.hstack([A0, A0[:, [j]]])
    rp, col, val = csr_from_dense(Ad)
    A = gpu_csr(rp, col, val, m, n)
    res = R.cssvdp_lsqr(handle, A, torch.tensor(b, device="cuda"), 4 * n, SEED, rcond=1e-12)
    assert res.precond.rank == n - 1
    Q, R0 = np.linalg.qr(A0)
    x0 = np.linalg.solve(R0, Q.T @ b)
    x = res.x.cpu().numpy()
    scale = np.abs(x0).max()
    assert abs(x[j] - x[n - 1]) <= 1e-9 * scale
    expect = x0.copy()
    expect[j] /= 2
    assert np.max(np.abs(x[:n - 1] - expect)) <= 1e-9 * scale


def test_cssvdp_lockstep_explicit_and_form_B(handle):
    S, s = build_config("poisson2d_3x3")
    A = gpu_csr(S.row_ptr, S.col, S.val, S.m, S.n)
    Ah = pipeline.csr(S.row_ptr, S.col, S.val, S.m, S.n)
    AT = R.rfmls_transpose(handle, A)
    P = R.rfmls_precond_svd(handle, R.rfmls_sketch(handle, A, s, SEED)[0], S.n)
    rng = np.random.default_rng(5)
    Bn = np.stack([S.b[0], rng.standard_normal(S.m), Ah @ rng.standard_normal(S.n)])
    Bt = torch.tensor(Bn, device="cuda")
    X, _, info, _ = R.rfmls_solve(handle, A, AT, P, Bt)
    Xs, _, info_s, _ = R.rfmls_solve(handle, A, AT, P, Bt, R.default_opts(lockstep=0))
    Po = osvd.svd_preconditioner(oracle_sketch(S.row_ptr, S.col, S.val, S.m, S.n, s))[3]
    for k in range(3):
        nb = np.linalg.norm(Bn[k])
        if k == 2:  # consistent right-hand side: both reach the S1 floor
            assert info[k]["normr"] <= 1e-9 * nb and info_s[k]["normr"] <= 1e-9 * nb
            continue
        xo, _ = pipeline.refined_lsqr(Ah, None, Bn[k], refine=1, P=Po)
        ro = pipeline.residual_metrics(Ah, xo, Bn[k])["normr"]
        assert abs(info[k]["normr"] - ro) <= 1e-10 * ro, k
        assert abs(info_s[k]["normr"] - ro) <= 1e-10 * ro, k
    # explicit B = A P: each entry a dot product of a row of A with a column of P
    Pg = R.rfmls_precond_export_P(handle, P).cpu().numpy()
    Ad = dense_from_csr(S.row_ptr, S.col, S.val, S.m, S.n)
    Bg = R.rfmls_form_B(handle, A, P).cpu().numpy()
    nnz_row = int(np.max(np.count_nonzero(Ad, axis=1)))
    assert np.all(np.abs(Bg - Ad @ Pg) <= 2 * nnz_row * 1.1e-16 * (np.abs(Ad) @ np.abs(Pg)) + 1e-300)
    x, _, info_e, _ = R.rfmls_solve_explicit(handle, A, AT, P, torch.tensor(Bg, device="cuda"),
                                             torch.tensor(S.b[0], device="cuda"))
    xo, _ = pipeline.refined_lsqr(Ah, None, S.b[0], refine=1, P=Po)
    ro = pipeline.residual_metrics(Ah, xo, S.b[0])["normr"]
    assert abs(info_e[0]["normr"] - ro) <= 1e-10 * ro


def test_cssvdp_backward_matches_dense_gradients(handle):
    m, n = 400, 30
    Ad = dense_with_condition(m, n, 1e4, seed=31)
    rng = np.random.default_rng(32)
    b = rng.standard_normal(m)
    g = rng.standard_normal(n)
    rp, col, val = csr_from_dense(Ad, keep_zeros=True)
    A = gpu_csr(rp, col, val, m, n)
    AT = R.rfmls_transpose(handle, A)
    P = R.rfmls_precond_svd(handle, R.rfmls_sketch(handle, A, 4 * n, 1)[0], n)
    assert P.rank == n
    xg, rg, info, _ = R.rfmls_solve(handle, A, AT, P, torch.tensor(b, device="cuda"))
    dB, dA, binfo, rc = R.rfmls_solve_backward(handle, A, AT, P, xg, rg, torch.tensor(g, device="cuda"))
    x, r, w, lam = backward.dense_gradients(Ad, b, g)
    assert np.linalg.norm(dB.cpu().numpy() - lam) <= 1e-8 * np.linalg.norm(lam)
    dAo = backward.pattern_grad(rp, col, r, w, lam, x)
    assert np.linalg.norm(dA.cpu().numpy() - dAo) <= 1e-7 * np.linalg.norm(dAo)


def test_svd_invalid_arguments(handle):
    m, n = 60, 5
    rp, col, val = csr_from_dense(dense_with_condition(m, n, 10.0, seed=1))
    A = gpu_csr(rp, col, val, m, n)
    SA = R.rfmls_sketch(handle, A, 20, SEED)[0]
    with pytest.raises(R.RfmlsError) as e:
        R.rfmls_precond_svd(handle, SA, n, rcond=1.0)
    assert e.value.status == -1
    P = R.rfmls_precond_svd(handle, SA, n)
    with pytest.raises(R.RfmlsError) as e:
        R.rfmls_precond_export_Rinv(handle, P)
    assert e.value.status == -1
    # a truncated SVD preconditioner has no backward
    Ad = dense_from_csr(rp, col, val, m, n)
    rp2, col2, val2 = csr_from_dense(np.hstack([Ad, Ad[:, [0]]]))
    A2 = gpu_csr(rp2, col2, val2, m, n + 1)
    AT2 = R.rfmls_transpose(handle, A2)
    P2 = R.rfmls_precond_svd(handle, R.rfmls_sketch(handle, A2, 24, SEED)[0], n + 1, rcond=1e-12)
    assert P2.rank == n
    b = torch.ones(m, dtype=torch.float64, device="cuda")
    x, r, _, _ = R.rfmls_solve(handle, A2, AT2, P2, b)
    with pytest.raises(R.RfmlsError) as e:
        R.rfmls_solve_backward(handle, A2, AT2, P2, x, r, torch.ones(n + 1, dtype=torch.float64, device="cuda"))
    assert e.value.status == -1
