"""The allocation-free solve (rfmls_solve_noalloc) against rfmls_solve.

rfmls_solve_noalloc runs the same kernels as rfmls_solve with one right-hand
side at a time, its scratch in a fixed device array instead of the handle's
workspace.  Two calls in a row, the second on a smaller system, must each give
rfmls_solve's results (the array keeps the previous call's contents), and both
must meet the oracle's residual gate; a system too large for the array is
refused before anything runs."""

import numpy as np
import pytest

from oracle import pipeline
from rfmgen import build_config

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2409_15818_amd")

SEED = 2


def _solve_both(handle, name, nrhs):
    S, s = build_config(name, modes=tuple(range(1, nrhs + 1)))
    print(f"[no-alloc] {name} m={S.m} n={S.n} nrhs={nrhs}", flush=True)
    A = R.CSR.from_numpy(S.row_ptr, S.col, S.val, S.m, S.n)
    AT = R.rfmls_transpose(handle, A)
    SA, _, _, _ = R.rfmls_sketch(handle, A, s, SEED)
    P = R.rfmls_precond(handle, SA, "f64", "f64")
    B = torch.tensor(S.b[:nrhs], device="cuda").contiguous()
    opts = R.default_opts(lockstep=0)
    X_ref, R_ref, info_ref, rc_ref = R.rfmls_solve(handle, A, AT, P, B, opts)
    # caller-allocated outputs, filled with garbage first
    X = torch.full((nrhs, S.n), float("nan"), dtype=torch.float64, device="cuda")
    Rr = torch.full((nrhs, S.m), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    info, rc = R.rfmls_solve_noalloc(handle, A, AT, P, B, X, Rr, opts)
    assert rc == rc_ref == 0
    return S, s, X, Rr, info, X_ref, R_ref, info_ref, P


def _check(S, s, X, Rr, info, X_ref, R_ref, info_ref, nrhs):
    x, xr = X.cpu().numpy(), X_ref.cpu().numpy()
    assert np.isfinite(x).all()
    # same kernels, same launch shapes, same order of operations
    assert np.abs(x - xr).max() <= 1e-13 * np.abs(xr).max()
    assert np.abs(Rr.cpu().numpy() - R_ref.cpu().numpy()).max() <= 1e-13 * np.abs(S.b[:nrhs]).max()
    for k in range(nrhs):
        assert info[k]["itn"] == info_ref[k]["itn"] and info[k]["istop"] == info_ref[k]["istop"]
        assert abs(info[k]["normr"] - info_ref[k]["normr"]) <= 1e-13 * info_ref[k]["normr"]
    # and the oracle's gate on the first right-hand side
    orc = pipeline.solve(S.row_ptr, S.col, S.val, S.b[0], S.m, S.n, s, SEED)
    assert abs(info[0]["normr"] - orc["normr"]) <= 1e-10 * orc["normr"]


def test_noalloc_matches_solve_on_two_calls_in_a_row(handle):
    big = _solve_both(handle, "poisson2d_3x3", 2)
    _check(*big[:8], 2)
    small = _solve_both(handle, "poisson2d_2x2", 1)
    _check(*small[:8], 1)


def test_noalloc_refuses_a_system_above_its_scratch(handle):
    S, s = build_config("poisson2d_2x2")
    A = R.CSR.from_numpy(S.row_ptr, S.col, S.val, S.m, S.n)
    SA, _, _, _ = R.rfmls_sketch(handle, A, s, SEED)
    P = R.rfmls_precond(handle, SA, "f64", "f64")
    limit = R.rfmls_noalloc_scratch_bytes()
    m_big = limit // 32 + 1  # 8 * 4 m bytes alone exceed the array
    # a matrix with no stored entries: nothing is read, the size check comes first
    Abig = R.CSR(m_big, S.n, torch.zeros(m_big + 1, dtype=torch.int64, device="cuda"),
                 torch.zeros(0, dtype=torch.int32, device="cuda"),
                 torch.zeros(0, dtype=torch.float64, device="cuda"))
    ATbig = R.CSR(S.n, m_big, torch.zeros(S.n + 1, dtype=torch.int64, device="cuda"),
                  torch.zeros(0, dtype=torch.int32, device="cuda"),
                  torch.zeros(0, dtype=torch.float64, device="cuda"))
    B = torch.ones(m_big, dtype=torch.float64, device="cuda")
    X = torch.zeros(S.n, dtype=torch.float64, device="cuda")
    with pytest.raises(R.RfmlsError) as e:
        R.rfmls_solve_noalloc(handle, Abig, ATbig, P, B, X)
    assert e.value.status == -1 and "limit" in str(e.value)
    # the handle still works afterwards
    big = _solve_both(handle, "poisson2d_2x2", 1)
    _check(*big[:8], 1)
