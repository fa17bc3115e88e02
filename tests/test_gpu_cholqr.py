"""The CholeskyQR2 panels of the QR (with Householder reconstruction) against
the unblocked Householder panels and the oracle.

Mode 0 (default) factors 64-column panels of at least 1024 rows by CholeskyQR2
on column-scaled Grams and reconstructs their Householder vectors, in float64
arithmetic for float64 and float32 panels alike; mode 1 uses the unblocked
kernel throughout.  Both must satisfy R^T R = (SA)^T SA to a few n u, agree
with each other and with the oracle's R to the sensitivity of R (about
cond(SA) u), and give the same solve.  Modes 2 and 3 force the first or second
Cholesky pass of every eligible panel to fail: the first fallback leaves the
panel untouched for the unblocked kernel (bitwise mode 1's R), the second
factors Q1 and multiplies by R1."""

import numpy as np
import pytest

from oracle import countsketch, pipeline, qr as oqr
from rfmgen import build_config, dense_with_condition

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2409_15818_amd")

SEED = 2


def _R(handle, SAo, mode, dtype="f64"):
    R.rfmls_qr_panel_mode(handle, mode)
    try:
        SA = torch.tensor(SAo.astype(np.float64 if dtype == "f64" else np.float32), device="cuda")
        P = R.rfmls_precond(handle, SA, dtype, dtype)
        Rg = R.rfmls_precond_export_R(handle, P).cpu().numpy()
        P.free()
    finally:
        R.rfmls_qr_panel_mode(handle, 0)
    return Rg.astype(np.float64)


def _ident(Rg, SAo):
    return np.linalg.norm(Rg.T @ Rg - SAo.T @ SAo) / np.linalg.norm(SAo) ** 2


def _cases():
    rng = np.random.default_rng(3)
    yield "gaussian 4096x64", rng.standard_normal((4096, 64)), 1e-12
    yield "gaussian 6000x200", rng.standard_normal((6000, 200)), 1e-12
    # ill-conditioned with columns of very different lengths (scaled panels)
    A = dense_with_condition(5000, 192, 1e6, seed=4) * np.geomspace(1.0, 1e5, 192)[None, :]
    yield "kappa 1e6, column scales 1e5", A, 1e-9
    for name in ("poisson2d_3x3", "poisson2d_4x4"):
        S, s = build_config(name)
        h, sign = countsketch.hash_sign(S.m, s, SEED)
        SAo, _ = countsketch.sketch_dense(S.row_ptr, S.col, S.val, h, sign, s, S.n)
        yield name, SAo, 1e-6


@pytest.mark.parametrize("case", list(_cases()), ids=lambda c: c[0])
def test_cholqr_panels_match_householder_panels(handle, case):
    label, SAo, rtol = case
    n = SAo.shape[1]
    print(f"[cholqr] {label} {SAo.shape}", flush=True)
    R0 = _R(handle, SAo, 0)
    R1 = _R(handle, SAo, 1)
    u = 1.1e-16
    assert np.all(np.diag(R0) > 0) and not np.tril(R0, -1).any()
    e0, e1 = _ident(R0, SAo), _ident(R1, SAo)
    print(f"[cholqr] {label}: identity cholqr {e0:.2e} householder {e1:.2e}", flush=True)
    assert e0 < 20 * n * u and e1 < 20 * n * u
    # elementwise, relative to each row's scale: R is determined to about cond * u
    Ro = oqr.r_factor(SAo, check_rank=False)
    scale = np.abs(Ro).max(axis=1, keepdims=True)
    d01 = (np.abs(R0 - R1) / scale).max()
    d0o = (np.abs(R0 - Ro) / scale).max()
    print(f"[cholqr] {label}: |R_cq - R_hh| {d01:.2e}, |R_cq - R_oracle| {d0o:.2e}", flush=True)
    assert d01 < rtol and d0o < rtol


def _cases32():
    rng = np.random.default_rng(5)
    yield "gaussian 4096x64", rng.standard_normal((4096, 64))
    yield "gaussian 6000x200 column scales 1e3", rng.standard_normal((6000, 200)) * np.geomspace(1.0, 1e3, 200)[None, :]
    for name in ("poisson2d_3x3",):
        S, s = build_config(name)
        h, sign = countsketch.hash_sign(S.m, s, SEED)
        SAo, _ = countsketch.sketch_dense(S.row_ptr, S.col, S.val, h, sign, s, S.n)
        yield name, SAo


@pytest.mark.parametrize("case", list(_cases32()), ids=lambda c: c[0])
def test_float32_cholqr_panels(handle, case):
    """Float32 panels through CholeskyQR2 in float64 arithmetic: R^T R = (SA)^T SA
    to the float32 rounding of the stored factor (SA rounded to float32 is the
    input both ways), and R against the float32 unblocked kernel's and the float64
    oracle's to R's sensitivity at float32 (about cond u32 per row's scale)."""
    label, SAo = case
    SA32 = SAo.astype(np.float32).astype(np.float64)
    n = SAo.shape[1]
    print(f"[cholqr32] {label} {SAo.shape}", flush=True)
    R0 = _R(handle, SAo, 0, "f32")
    R1 = _R(handle, SAo, 1, "f32")
    u32 = 6e-8
    assert np.all(np.diag(R0) > 0) and not np.tril(R0, -1).any()
    e0, e1 = _ident(R0, SA32), _ident(R1, SA32)
    print(f"[cholqr32] {label}: identity cholqr {e0:.2e} householder {e1:.2e}", flush=True)
    assert e0 < 20 * n * u32 and e1 < 20 * n * u32
    Ro = oqr.r_factor(SA32, check_rank=False)
    scale = np.abs(Ro).max(axis=1, keepdims=True)
    d0o = (np.abs(R0 - Ro) / scale).max()
    d1o = (np.abs(R1 - Ro) / scale).max()
    print(f"[cholqr32] {label}: |R_cq - R_oracle| {d0o:.2e}, |R_hh - R_oracle| {d1o:.2e}", flush=True)
    # the float64-arithmetic panel is at least as close to the float64 R as the float32 kernel
    assert d0o <= max(2.0 * d1o, 1e-6)


def test_float32_cholqr_fallback_paths(handle):
    SAo = dense_with_condition(3000, 128, 1e3, seed=8)
    R1 = _R(handle, SAo, 1, "f32")
    R2 = _R(handle, SAo, 2, "f32")
    R3 = _R(handle, SAo, 3, "f32")
    assert np.array_equal(R2, R1)
    SA32 = SAo.astype(np.float32).astype(np.float64)
    assert _ident(R3, SA32) < 20 * 128 * 6e-8
    scale = np.abs(R1).max(axis=1, keepdims=True)
    assert (np.abs(R3 - R1) / scale).max() < 1e-4


def test_cholqr_fallback_paths(handle):
    SAo = dense_with_condition(3000, 128, 1e4, seed=7) * np.geomspace(1.0, 1e3, 128)[None, :]
    R1 = _R(handle, SAo, 1)
    R2 = _R(handle, SAo, 2)  # first pass fails: the unblocked kernel on the untouched panels
    R3 = _R(handle, SAo, 3)  # second pass fails: the unblocked kernel on Q1, then R' R1
    assert np.array_equal(R2, R1)
    assert _ident(R3, SAo) < 20 * 128 * 1.1e-16
    scale = np.abs(R1).max(axis=1, keepdims=True)
    assert (np.abs(R3 - R1) / scale).max() < 1e-10


@pytest.mark.parametrize("name", ["poisson2d_3x3", "poisson2d_4x4"])
def test_solve_with_cholqr_panels_matches_oracle(handle, name):
    S, s = build_config(name)
    A = R.CSR.from_numpy(S.row_ptr, S.col, S.val, S.m, S.n)
    b = torch.tensor(S.b[0], device="cuda")
    out = {}
    for mode in (0, 1):
        R.rfmls_qr_panel_mode(handle, mode)
        try:
            res = R.csqrp_lsqr(handle, A, b, s, SEED, opts=R.default_opts(refine=1))
        finally:
            R.rfmls_qr_panel_mode(handle, 0)
        out[mode] = res.info[0]
    orc = pipeline.solve(S.row_ptr, S.col, S.val, S.b[0], S.m, S.n, s, SEED, refine=1)
    for mode in (0, 1):
        assert abs(out[mode]["normr"] - orc["normr"]) <= 1e-10 * orc["normr"]
    assert abs(out[0]["itn_first"] - orc["itn_sweeps"][0]) <= 2


def _qr_factors(handle, SAo, lookahead, mode=0):
    """R and the Householder vectors (the whole factored SA) from rfmls_precond_x0-free QR."""
    R.rfmls_qr_panel_mode(handle, mode)
    R.rfmls_qr_lookahead(handle, lookahead)
    try:
        SA = torch.tensor(SAo, device="cuda")
        P = R.rfmls_precond(handle, SA, "f64", "f64")
        torch.cuda.synchronize()
        out = SA.cpu().numpy().copy()
        P.free()
    finally:
        R.rfmls_qr_lookahead(handle, False)
        R.rfmls_qr_panel_mode(handle, 0)
    return out


def _sketch_4x4():
    S, s = build_config("poisson2d_4x4")
    h, sign = countsketch.hash_sign(S.m, s, SEED)
    SAo, _ = countsketch.sketch_dense(S.row_ptr, S.col, S.val, h, sign, s, S.n)
    return SAo


# (label, matrix maker): the matrices are made when the test runs, not when
# it is collected
LOOKAHEAD_CASES = [
    # four and five outer blocks of 256 columns, the last one ragged
    ("gaussian 6000x1024", lambda: np.random.default_rng(11).standard_normal((6000, 1024))),
    ("gaussian 4000x1100",
     lambda: np.random.default_rng(12).standard_normal((4000, 1100)) * np.geomspace(1.0, 1e4, 1100)[None, :]),
    ("poisson2d_4x4", _sketch_4x4),
    # float64 from 12,800 columns on: 25 outer blocks of 512 columns and a
    # 64-column last one, whose 200-row panel takes the unblocked kernel
    ("gaussian 13000x12864", lambda: np.random.default_rng(13).standard_normal((13000, 12864))),
]


@pytest.mark.parametrize("case", LOOKAHEAD_CASES, ids=lambda c: c[0])
def test_lookahead_gives_bitwise_the_same_factorisation(handle, case):
    """The look-ahead schedule splits the trailing update by columns and runs the
    next block's panels on a second stream: every column's sums keep their order,
    so the whole factored matrix (R and the Householder vectors) is bitwise equal."""
    label, make = case
    SAo = make()
    print(f"[lookahead] {label} {SAo.shape}", flush=True)
    F0 = _qr_factors(handle, SAo, False)
    F1 = _qr_factors(handle, SAo, True)
    assert np.array_equal(F0, F1)
    # a second run with look-ahead repeats itself exactly (no race between the streams)
    F2 = _qr_factors(handle, SAo, True)
    assert np.array_equal(F1, F2)


def test_lookahead_solve_matches_oracle(handle):
    S, s = build_config("poisson2d_4x4")
    A = R.CSR.from_numpy(S.row_ptr, S.col, S.val, S.m, S.n)
    b = torch.tensor(S.b[0], device="cuda")
    R.rfmls_qr_lookahead(handle, True)
    try:
        res = R.csqrp_lsqr(handle, A, b, s, SEED, opts=R.default_opts(refine=1))
    finally:
        R.rfmls_qr_lookahead(handle, False)
    orc = pipeline.solve(S.row_ptr, S.col, S.val, S.b[0], S.m, S.n, s, SEED, refine=1)
    assert abs(res.info[0]["normr"] - orc["normr"]) <= 1e-10 * orc["normr"]
    assert abs(res.info[0]["itn_first"] - orc["itn_sweeps"][0]) <= 2


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(1024, 64), (1050, 128), (1300, 320), (2100, 130)])
def test_cholqr_at_the_row_threshold(handle, dtype, shape):
    """Panels of at least 1024 rows go through CholeskyQR2, shorter ones and ragged
    last panels through the unblocked kernel, within one factorisation (1050 x 128:
    panel 0 of 1050 rows, panel 1 of 986; 1300 x 320: five panels down to 1044 rows
    in slabs with a ragged last one; 2100 x 130: a 2-column last panel).  Both ways
    R^T R = (SA)^T SA, and R agrees with the unblocked kernel's."""
    m, n = shape
    SAo = np.random.default_rng(m + n).standard_normal((m, n))
    SAq = SAo.astype(np.float64 if dtype == "f64" else np.float32).astype(np.float64)
    u = 1.1e-16 if dtype == "f64" else 6e-8
    R0 = _R(handle, SAo, 0, dtype)
    R1 = _R(handle, SAo, 1, dtype)
    assert np.all(np.diag(R0) > 0) and not np.tril(R0, -1).any()
    assert _ident(R0, SAq) < 20 * n * u
    scale = np.abs(R1).max(axis=1, keepdims=True)
    assert (np.abs(R0 - R1) / scale).max() < (1e-11 if dtype == "f64" else 1e-4)


def test_lookahead_float32_bitwise(handle):
    """Look-ahead with float32 panels (CholeskyQR2 in float64 arithmetic): the same
    factored matrix as the plain schedule, bit for bit."""
    SAo = np.random.default_rng(41).standard_normal((3000, 800)).astype(np.float32)
    F = []
    for la in (False, True):
        R.rfmls_qr_lookahead(handle, la)
        try:
            SA = torch.tensor(SAo, device="cuda")
            P = R.rfmls_precond(handle, SA, "f32", "f32")
            torch.cuda.synchronize()
            F.append(SA.cpu().numpy().copy())
            P.free()
        finally:
            R.rfmls_qr_lookahead(handle, False)
    assert np.array_equal(F[0], F[1])
