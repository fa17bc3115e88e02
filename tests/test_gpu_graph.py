"""Graph-captured LSQR iterations against the same iterations launched eagerly.

With opts.graph set (the default) the launches between two polls of the
device stop flag are captured once per call and replayed; every replay runs
the same kernels on the same buffers, with the host's polls and the sweeps'
own eager launches between replays.  The results must be bitwise those of the
eager loop (opts.graph = 0) for the single-right-hand-side solve, the lockstep
solve, the explicit-B solve and both backward passes, on repeated calls."""

import numpy as np
import pytest

from oracle import pipeline
from rfmgen import build_config, feature_eval, sample_points

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2409_15818_amd")

SEED = 2


def _setup(handle, name, nrhs):
    S, s = build_config(name, modes=tuple(range(1, nrhs + 1)))
    print(f"[graph] {name} nrhs={nrhs}", flush=True)
    A = R.CSR.from_numpy(S.row_ptr, S.col, S.val, S.m, S.n)
    AT = R.rfmls_transpose(handle, A)
    SA, _, _, _ = R.rfmls_sketch(handle, A, s, SEED)
    P = R.rfmls_precond(handle, SA, "f64", "f64")
    B = torch.tensor(S.b[0] if nrhs == 1 else S.b[:nrhs], device="cuda")
    return S, s, A, AT, P, B


def _same(a, b):
    return torch.equal(a, b)


@pytest.mark.parametrize("name,nrhs,lockstep", [("poisson2d_3x3", 1, 0), ("poisson3d_2x2x2", 3, 0),
                                                 ("poisson2d_3x3", 3, 1), ("poisson2d_2x2", 35, 1)])
def test_graph_solve_equals_eager(handle, name, nrhs, lockstep):
    S, s, A, AT, P, B = _setup(handle, name, nrhs)
    eager = R.default_opts(graph=0, lockstep=lockstep, refine=2)
    graph = R.default_opts(graph=1, lockstep=lockstep, refine=2)
    Xe, Re, ie, rce = R.rfmls_solve(handle, A, AT, P, B, eager)
    for _ in range(2):  # a fresh capture per call; each call replays it many times
        Xg, Rg, ig, rcg = R.rfmls_solve(handle, A, AT, P, B, graph)
        assert rcg == rce
        assert _same(Xg, Xe) and _same(Rg, Re)
        assert [i["itn"] for i in ig] == [i["itn"] for i in ie]
        assert [i["istop"] for i in ig] == [i["istop"] for i in ie]
    # and the oracle's gate on the first right-hand side
    orc = pipeline.solve(S.row_ptr, S.col, S.val, S.b[0], S.m, S.n, s, SEED, refine=2)
    assert abs(ig[0]["normr"] - orc["normr"]) <= 1e-10 * orc["normr"]


def test_graph_explicit_solve_equals_eager(handle):
    S, s, A, AT, P, B = _setup(handle, "poisson2d_2x2", 1)
    Bm = R.rfmls_form_B(handle, A, P)
    Xe, _, ie, _ = R.rfmls_solve_explicit(handle, A, AT, P, Bm, B, R.default_opts(graph=0))
    Xg, _, ig, _ = R.rfmls_solve_explicit(handle, A, AT, P, Bm, B, R.default_opts(graph=1))
    assert _same(Xg, Xe) and ig[0]["itn"] == ie[0]["itn"]


@pytest.mark.parametrize("nrhs,lockstep", [(1, 0), (3, 1)])
def test_graph_backward_equals_eager(handle, nrhs, lockstep):
    S, s, A, AT, P, B = _setup(handle, "poisson2d_2x2", nrhs)
    X, Rr, _, _ = R.rfmls_solve(handle, A, AT, P, B, R.default_opts(lockstep=lockstep))
    pts = sample_points(S.d)
    E = pipeline.csr(*feature_eval(S, pts), len(pts), S.n)
    Xn = X.reshape(nrhs, S.n).cpu().numpy()
    G = np.stack([E.T @ (E @ Xn[k] - S.exact(pts, S.modes[k])) for k in range(nrhs)])
    Gt = torch.tensor(G[0] if nrhs == 1 else G, device="cuda")
    dBe, dAe, ie, _ = R.rfmls_solve_backward(handle, A, AT, P, X, Rr, Gt,
                                             R.default_opts(graph=0, lockstep=lockstep))
    dBg, dAg, ig, _ = R.rfmls_solve_backward(handle, A, AT, P, X, Rr, Gt,
                                             R.default_opts(graph=1, lockstep=lockstep))
    assert _same(dBg, dBe) and _same(dAg, dAe)
    assert [i["itn"] for i in ig] == [i["itn"] for i in ie]


def test_graph_not_used_while_tracing(handle):
    # with kernel tracing on, the loop is launched eagerly so that every launch
    # is bracketed by its own events; the result is the same
    S, s, A, AT, P, B = _setup(handle, "poisson2d_2x2", 1)
    Xg, _, ig, _ = R.rfmls_solve(handle, A, AT, P, B, R.default_opts(graph=1))
    R.rfmls_trace_enable(handle, True)
    try:
        Xt, _, it, _ = R.rfmls_solve(handle, A, AT, P, B, R.default_opts(graph=1))
        kern = {k["name"]: k for k in R.rfmls_trace_read(handle)}
    finally:
        R.rfmls_trace_enable(handle, False)
    assert _same(Xt, Xg)
    # one traced launch of the triangular product per iteration and per x = X y
    assert kern["trmv_X"]["launches"] >= it[0]["itn"]
