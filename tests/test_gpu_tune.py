"""The launch-shape autotuner of the 32-column sparse products.

Tuning times every candidate shape on the matrix itself the first time the
matrix is used on a handle and keeps the fastest; the candidates differ only in
window width and grid size, which change no sum's order, so the lockstep solve
and its backward must be bitwise the same with tuning on and off, and whatever
the tuner picked."""

import numpy as np
import pytest

from oracle import pipeline
from rfmgen import build_config

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2409_15818_amd")

SEED = 2


@pytest.mark.parametrize("name", ["poisson2d_3x3", "helmholtz3d_2x2x2_small"])
def test_tuned_shapes_give_identical_results(name):
    S, s = build_config(name, modes=(1, 2, 3))
    print(f"[tune] {name}", flush=True)
    results = []
    for tune in (False, True):
        h = R.Handle()
        try:
            R.rfmls_tune_enable(h, tune)
            A = R.CSR.from_numpy(S.row_ptr, S.col, S.val, S.m, S.n)
            AT = R.rfmls_transpose(h, A)
            SA, _, _, _ = R.rfmls_sketch(h, A, s, SEED)
            P = R.rfmls_precond(h, SA, "f64", "f64")
            B = torch.tensor(S.b, device="cuda")
            X, Rr, info, rc = R.rfmls_solve(h, A, AT, P, B, R.default_opts())
            G = torch.ones((3, S.n), dtype=torch.float64, device="cuda") * 1e-3
            dB, dA, binfo, _ = R.rfmls_solve_backward(h, A, AT, P, X, Rr, G, R.default_opts())
            recs = R.rfmls_tune_read(h)
            # a second solve on the same matrices tunes nothing new
            R.rfmls_solve(h, A, AT, P, B, R.default_opts())
            assert len(R.rfmls_tune_read(h)) == len(recs)
            torch.cuda.synchronize()
            results.append((X.clone(), dB.clone(), dA.clone(), [i["itn"] for i in info], recs))
            P.free()
        finally:
            h.close()
    (X0, dB0, dA0, it0, rec0), (X1, dB1, dA1, it1, rec1) = results
    assert rec0 == []
    kinds = sorted((r["rows"], r["cols"]) for r in rec1)
    assert kinds == sorted([(S.m, S.n), (S.n, S.m)])
    for r in rec1:
        assert r["kernel"] == "spmm" and r["candidates"] >= 2
        assert 0.0 < r["ms_best"] <= r["ms_default"]
        print(f"[tune] {r}", flush=True)
    assert torch.equal(X0, X1) and torch.equal(dB0, dB1) and torch.equal(dA0, dA1) and it0 == it1
    # and the tuned solve still meets the oracle's gate
    orc = pipeline.solve(S.row_ptr, S.col, S.val, S.b[0], S.m, S.n, s, SEED)
    x = X1[0].cpu().numpy()
    Ah = pipeline.csr(S.row_ptr, S.col, S.val, S.m, S.n)
    assert abs(np.linalg.norm(S.b[0] - Ah @ x) - orc["normr"]) <= 1e-10 * orc["normr"]
