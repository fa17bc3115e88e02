"""Degenerate right-hand sides and non-finite inputs through the C-ABI.

* b orthogonal to range(A): the least-squares solution is x = 0 and the
  residual is b itself.  A gets empty rows (no entries) and b lives on them
  only, so A^T b = 0 exactly.  From y0 = 0 LSQR meets alpha_1 = 0 and stops at
  once with x = 0 (Paige and Saunders' istop 0); from the sketched start the
  refinement must bring x back to (numerically) zero.
* A NaN in b is a breakdown (RFMLS_E_BREAKDOWN), not "x = 0 is exact": the
  start of a sweep tests beta_1 and alpha_1 for finiteness.
* A NaN in A's values reaches R's diagonal, which the rank test refuses
  (RFMLS_E_RANK).
"""
import numpy as np
import pytest

from rfmgen import build_config

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2409_15818_amd")

SEED = 2
E_BREAKDOWN = -3
E_RANK = -2


def _with_empty_rows(S, extra):
    rp = np.concatenate([S.row_ptr, np.full(extra, S.row_ptr[-1], dtype=S.row_ptr.dtype)])
    return R.CSR.from_numpy(rp, S.col, S.val, S.m + extra, S.n)


@pytest.mark.parametrize("start", ["zero", "sketch"])
def test_b_orthogonal_to_the_range(handle, start):
    S, s = build_config("poisson2d_2x2")
    extra = 64
    A = _with_empty_rows(S, extra)
    rng = np.random.default_rng(5)
    bn = np.zeros(S.m + extra)
    bn[S.m:] = rng.standard_normal(extra)
    b = torch.tensor(bn, device="cuda")
    print(f"[edge] b orthogonal to range(A), start {start}", flush=True)
    res = R.csqrp_lsqr(handle, A, b, s, SEED, opts=R.default_opts(refine=1), start=start)
    assert res.status == 0
    x = res.x.detach().cpu().numpy().reshape(-1)
    r = res.residual.detach().cpu().numpy().reshape(-1)
    nb = np.linalg.norm(bn)
    # A x from the oracle-free definition: the CSR product on the CPU
    Ax = np.zeros(S.m + extra)
    for i in range(S.m):
        lo, hi = S.row_ptr[i], S.row_ptr[i + 1]
        Ax[i] = S.val[lo:hi] @ x[S.col[lo:hi]]
    if start == "zero":
        assert not x.any()
        assert res.info[0]["istop"] == 0
        assert np.array_equal(r, bn)
    else:
        assert np.linalg.norm(Ax) <= 1e-6 * nb
    assert abs(res.info[0]["normr"] - nb) <= 1e-10 * nb
    assert np.all(np.isfinite(x))


@pytest.mark.parametrize("start", ["zero", "sketch"])
def test_nan_in_b_is_a_breakdown(handle, start):
    S, s = build_config("poisson2d_2x2")
    A = R.CSR.from_numpy(S.row_ptr, S.col, S.val, S.m, S.n)
    bn = S.b[0].copy()
    bn[17] = np.nan
    b = torch.tensor(bn, device="cuda")
    print(f"[edge] NaN in b, start {start}", flush=True)
    with pytest.raises(R.RfmlsError) as e:
        R.csqrp_lsqr(handle, A, b, s, SEED, opts=R.default_opts(refine=1), start=start)
    assert e.value.status == E_BREAKDOWN


def test_nan_in_one_lockstep_column_is_a_breakdown(handle):
    S, s = build_config("poisson2d_2x2", modes=(1, 2, 3))
    A = R.CSR.from_numpy(S.row_ptr, S.col, S.val, S.m, S.n)
    bn = np.array(S.b, dtype=np.float64)
    bn[1, 5] = np.nan
    b = torch.tensor(bn, device="cuda")
    print("[edge] NaN in one of three lockstep columns", flush=True)
    with pytest.raises(R.RfmlsError) as e:
        R.csqrp_lsqr(handle, A, b, s, SEED, opts=R.default_opts(refine=1, lockstep=1), start="zero")
    assert e.value.status == E_BREAKDOWN


def test_nan_in_A_is_refused_by_the_rank_test(handle):
    S, s = build_config("poisson2d_2x2")
    val = S.val.copy()
    val[123] = np.nan
    A = R.CSR.from_numpy(S.row_ptr, S.col, val, S.m, S.n)
    b = torch.tensor(S.b[0], device="cuda")
    print("[edge] NaN in A", flush=True)
    with pytest.raises(R.RfmlsError) as e:
        R.csqrp_lsqr(handle, A, b, s, SEED, opts=R.default_opts(refine=1), start="zero")
    assert e.value.status == E_RANK
