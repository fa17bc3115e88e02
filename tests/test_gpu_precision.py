"""The float32 factor check of rfmls_precond (RFMLS_E_PRECISION) against the
oracle's reading of it: a factor computed or stored in float32 is refused when
min_j |r_jj| / ||SA[:, j]|| <= u32, where the float32 factor carries only
rounding noise in some direction; accepted otherwise, and then the float32 form
reaches the float64 form's optimum."""

import numpy as np
import pytest

from oracle import pipeline, qr as oqr
from rfmgen import build_config, csr_from_dense, dense_with_condition

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2409_15818_amd")

SEED = 2


def _near_dependent(delta, seed=3):
    A = dense_with_condition(600, 40, 1e2, seed=seed)
    rng = np.random.default_rng(seed + 1)
    A[:, 7] = A[:, 3] + delta * np.linalg.norm(A[:, 3]) * rng.standard_normal(600) / np.sqrt(600)
    return A


def _sketch(handle, rp, col, val, m, n, s, dtype):
    A = R.CSR.from_numpy(rp, col, val, m, n)
    SA, _, _, _ = R.rfmls_sketch(handle, A, s, 5, dtype=dtype)
    return A, SA


@pytest.mark.parametrize("qd,rd", [("f32", "f32"), ("f64", "f32"), ("f32", "f64")])
def test_float32_factor_refused_for_a_column_dependent_in_float32(handle, qd, rd):
    A = _near_dependent(1e-11)
    m, n = A.shape
    rp, col, val = csr_from_dense(A, keep_zeros=True)
    with pytest.raises(oqr.PrecisionInsufficient):
        pipeline.precondition(rp, col, val, m, n, 4 * n, 5, qr_dtype=qd, r_store=rd)
    _, SA = _sketch(handle, rp, col, val, m, n, 4 * n, qd)
    with pytest.raises(R.RfmlsError) as e:
        R.rfmls_precond(handle, SA, qd, rd)
    if qd == "f32":
        # rounded to float32 the two columns of SA can coincide exactly: then
        # the float32 QR leaves an exact zero pivot, which is refused as rank
        # deficient before the precision test
        assert e.value.status in (-6, -2)
    else:
        assert e.value.status == -6 and "float32" in str(e.value)


def test_float64_factor_of_the_same_system_accepted_with_its_statistics(handle):
    A = _near_dependent(1e-11)
    m, n = A.shape
    rp, col, val = csr_from_dense(A, keep_zeros=True)
    _, SA = _sketch(handle, rp, col, val, m, n, 4 * n, "f64")
    P = R.rfmls_precond(handle, SA, "f64", "f64")
    st = R.rfmls_precond_stats(P)
    Ro = pipeline.precondition(rp, col, val, m, n, 4 * n, 5)["R"]
    d = np.abs(np.diag(Ro))
    # both factors resolve the 1e-11 distance (to about u / rho relative)
    assert abs(st["rho_min"] - oqr.rho_min(Ro)) <= 1e-3 * oqr.rho_min(Ro)
    assert abs(st["pivot_ratio"] - d.min() / d.max()) <= 1e-3 * d.min() / d.max()


def test_float32_form_accepted_on_rfm_3x3_and_refused_on_4x4(handle):
    S, s = build_config("poisson2d_3x3")
    A = R.CSR.from_numpy(S.row_ptr, S.col, S.val, S.m, S.n)
    res = R.csqrp_lsqr(handle, A, torch.tensor(S.b[0], device="cuda"), s, SEED, qr_dtype="f32",
                       r_store="f32", opts=R.default_opts(refine=1))
    st = R.rfmls_precond_stats(res.precond)
    assert st["rho_min"] > oqr.PRECISION_TOL
    o64 = pipeline.solve(S.row_ptr, S.col, S.val, S.b[0], S.m, S.n, s, SEED, refine=1)
    assert res.status == 0 and res.info[0]["istop"] in (1, 2)
    assert abs(res.info[0]["normr"] - o64["normr"]) <= 1e-10 * o64["normr"]
    # the 4x4-box system's float32 factor: refused by the oracle's reading and the library
    S, s = build_config("poisson2d_4x4")
    with pytest.raises(oqr.PrecisionInsufficient):
        pipeline.precondition(S.row_ptr, S.col, S.val, S.m, S.n, s, SEED, qr_dtype="f32")
    A = R.CSR.from_numpy(S.row_ptr, S.col, S.val, S.m, S.n)
    SA, _, _, _ = R.rfmls_sketch(handle, A, s, SEED, dtype="f32")
    with pytest.raises(R.RfmlsError) as e:
        R.rfmls_precond(handle, SA, "f32", "f32")
    assert e.value.status == -6
