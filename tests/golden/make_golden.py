"""Write the oracle's reference values for the full-size workloads.

Calls only the CPU oracle (oracle/) on inputs from the seeded generator
(rfmgen/); the GPU path is never involved.  Usage:
    python tests/golden/make_golden.py poisson2d_8x8 [poisson3d_4x4x4 ...]
writes tests/golden/<name>.json;
    python tests/golden/make_golden.py --svd helmholtz3d_2x2x2
adds the CSSVDP-LSQR (Alg. 2) results under the key "svd" of that file;
    python tests/golden/make_golden.py --multi poisson2d_8x8
adds per-mode solves of the batched right-hand sides and one column's
gradients under the key "multi".
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import backward, countsketch, pipeline, qr, svd  # noqa: E402
from rfmgen import build_config, feature_eval, sample_points  # noqa: E402

SKETCH_SEED = 2


def main(name: str, refine: int = 2):
    t0 = time.time()
    S, s = build_config(name)
    h, sign = countsketch.hash_sign(S.m, s, SKETCH_SEED)
    SA, _ = countsketch.sketch_dense(S.row_ptr, S.col, S.val, h, sign, s, S.n)
    t1 = time.time()
    R = qr.r_factor(SA, check_rank=False)
    del SA
    t2 = time.time()
    A = pipeline.csr(S.row_ptr, S.col, S.val, S.m, S.n)
    x, results = pipeline.refined_lsqr(A, R, S.b[0], refine=refine)
    t3 = time.time()
    met = pipeline.residual_metrics(A, x, S.b[0])
    pts = sample_points(S.d)
    E = pipeline.csr(*feature_eval(S, pts), len(pts), S.n)
    out = dict(
        workload=name, m=S.m, n=S.n, nnz=S.nnz, s=s, sketch_seed=SKETCH_SEED, refine=refine,
        itn_sweeps=[r.itn for r in results], istop_sweeps=[r.istop for r in results],
        normb=float(np.linalg.norm(S.b[0])), normr=met["normr"], relres=met["relres"],
        normal_relres=met["normal_relres"], l2_error=pipeline.l2_error(E, x, S.exact(pts)),
        rdiag_min=float(np.abs(np.diag(R)).min()), rdiag_max=float(np.abs(np.diag(R)).max()),
        seconds=dict(sketch=t1 - t0, qr=t2 - t1, lsqr=t3 - t2),
    )
    path = os.path.join(HERE, f"{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def main_multi(name: str, modes=(1, 2, 17, 32), grad_mode: int = 1, refine: int = 2, nsample: int = 48):
    """Per-mode oracle solves of the batched workload (right-hand sides
    u_k = sin(k pi x) sin(pi y), k in modes, each solved on its own from y = 0
    with the same refinement sweeps), and the gradients of
    L = 1/2 ||E x_k - u_k||^2 at the 10^4 sample points for k = grad_mode
    (dL/db = lambda and dL/dA on A's pattern, by the preconditioned LSQR on
    B^T lambda = R^{-T} g): their norms, A^T lambda = g's relative residual and
    seeded samples of lambda and dA.  Stored under the key "multi"."""
    t0 = time.time()
    S, s = build_config(name, modes=tuple(modes))
    h, sign = countsketch.hash_sign(S.m, s, SKETCH_SEED)
    SA, _ = countsketch.sketch_dense(S.row_ptr, S.col, S.val, h, sign, s, S.n)
    R = qr.r_factor(SA, check_rank=False)
    del SA
    A = pipeline.csr(S.row_ptr, S.col, S.val, S.m, S.n)
    pts = sample_points(S.d)
    E = pipeline.csr(*feature_eval(S, pts), len(pts), S.n)
    per_mode = {}
    xg = None
    for k, mode in enumerate(modes):
        x, results = pipeline.refined_lsqr(A, R, S.b[k], refine=refine)
        met = pipeline.residual_metrics(A, x, S.b[k])
        per_mode[str(mode)] = dict(itn_sweeps=[r.itn for r in results], istop_sweeps=[r.istop for r in results],
                                   normb=float(np.linalg.norm(S.b[k])), normr=met["normr"], relres=met["relres"],
                                   normal_relres=met["normal_relres"],
                                   l2_error=pipeline.l2_error(E, x, S.exact(pts, mode)))
        print(mode, json.dumps(per_mode[str(mode)]), flush=True)
        if mode == grad_mode:
            xg, kg = x, k
    r = S.b[kg] - A @ xg
    g = E.T @ (E @ xg - S.exact(pts, grad_mode))
    w, lam, itn = backward.iterative_gradients(A, R, xg, r, g)
    dA = backward.pattern_grad(S.row_ptr, S.col, r, w, lam, xg)
    rng = np.random.default_rng(11)
    rows = np.sort(rng.choice(S.m, nsample, replace=False))
    ents = np.sort(rng.choice(S.nnz, nsample, replace=False))
    grad = dict(mode=grad_mode, itn=int(itn), normg=float(np.linalg.norm(g)),
                norm_lambda=float(np.linalg.norm(lam)), norm_dA=float(np.linalg.norm(dA)),
                at_lambda_relres=float(np.linalg.norm(A.T @ lam - g) / np.linalg.norm(g)),
                lambda_rows=[int(i) for i in rows], lambda_sample=[float(v) for v in lam[rows]],
                dA_entries=[int(e) for e in ents], dA_sample=[float(v) for v in dA[ents]],
                lambda_max=float(np.abs(lam).max()), dA_max=float(np.abs(dA).max()))
    rec = dict(modes=list(modes), refine=refine, per_mode=per_mode, gradient=grad,
               seconds=time.time() - t0)
    path = os.path.join(HERE, f"{name}.json")
    data = json.load(open(path))
    data["multi"] = rec
    with open(path, "w") as f:
        json.dump(data, f, indent=1)
    print(json.dumps(grad)[:400])


def main_svd(name: str, refine: int = 2):
    t0 = time.time()
    S, s = build_config(name)
    out = pipeline.solve_svd(S.row_ptr, S.col, S.val, S.b[0], S.m, S.n, s, SKETCH_SEED, refine=refine)
    pts = sample_points(S.d)
    E = pipeline.csr(*feature_eval(S, pts), len(pts), S.n)
    sig = out["sigma"]
    rec = dict(rcond=svd.default_rcond(S.n), rank=out["rank"], sigma_max=float(sig[0]),
               sigma_min=float(sig[-1]), sigma_quantiles=[float(v) for v in np.quantile(sig, [0.1, 0.5, 0.9])],
               itn_sweeps=out["itn_sweeps"], normr=out["normr"], relres=out["relres"],
               normal_relres=out["normal_relres"], l2_error=pipeline.l2_error(E, out["x"], S.exact(pts)),
               seconds=time.time() - t0)
    path = os.path.join(HERE, f"{name}.json")
    data = json.load(open(path))
    data["svd"] = rec
    with open(path, "w") as f:
        json.dump(data, f, indent=1)
    print(json.dumps(rec))


if __name__ == "__main__":
    args = sys.argv[1:]
    if args and args[0] == "--svd":
        for nm in args[1:]:
            main_svd(nm)
    elif args and args[0] == "--multi":
        for nm in args[1:]:
            main_multi(nm)
    else:
        for nm in args:
            main(nm)
