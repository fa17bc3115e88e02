#!/usr/bin/env python3
"""Time-to-tolerance benchmark of the CSQRP-LSQR pipeline on one MI355X.

One step = the whole path on one synthetic RFM system already resident in HBM:
A^T build, count sketch (with S b), Householder QR of [SA | Sb] + R^{-1}, LSQR
from the sketched starting point y0 = Q^T (S b) (Remark 3.1; --start zero for
y0 = 0) to the 1e-10 stopping rule with refinement sweeps, final true
residual.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload poisson2d_8x8] [--precision f64|f32]
                  [--start sketch|zero] [--nrhs K] [--backward]
"""

from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time to rel. residual 1e-10 (FP64 vs FP32-precond); SpMV/trsv HBM GB/s"
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}
COMPUTE_KERNELS = ("qr_gemm_update", "qr_gemm_VtC", "inv_gemm", "qr_inner_update", "qr_inner_VtC")
# everything else in the kernel list (SpMV / SpMM, triangular and dense products
# with the preconditioner, sketch) is priced against HBM bandwidth
# vector-ALU kernels (no matrix cores), priced against the vector peak
ALU_KERNELS = ("qr_panel", "inv_blockrow")
ALU_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}
SKETCH_SEED = 2


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic(kernel, workload, precision):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    (profiles/pmc_hbm_bytes_<workload>_<precision>.md, FETCH_SIZE + WRITE_SIZE scaled by a
    copy of known size), or None when there is none or the kernel's sources changed since."""
    import hashlib
    import re

    path = os.path.join(ROOT, "profiles", f"pmc_hbm_bytes_{workload}_{precision}.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    k = rec.get("kernels", {}).get(kernel)
    if k is None:
        return None
    hsh = hashlib.sha256()
    for f in rec["source_files"]:
        hsh.update(open(os.path.join(ROOT, f), "rb").read())
    if hsh.hexdigest() != rec["source_sha256"]:
        return None
    return k["traffic_bytes_per_launch"]


def cpu_model():
    """The host CPU's model name and the number of cores this process may use."""
    name = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return name


def cpu_full_run(S, s, refine, threads):
    """The whole oracle solve of the workload, timed phase by phase (Sec. 4.1's
    PCPU / CPU split): sketch, Householder QR, LSQR with the same refinement
    sweeps.  Minutes of CPU time; only with --cpu-baseline full."""
    from oracle import countsketch, pipeline, qr

    t0 = time.perf_counter()
    h, sign = countsketch.hash_sign(S.m, s, SKETCH_SEED)
    SA, _ = countsketch.sketch_dense(S.row_ptr, S.col, S.val, h, sign, s, S.n)
    t1 = time.perf_counter()
    log(f"[cpu-full] sketch {t1 - t0:.1f} s")
    R = qr.r_factor(SA, check_rank=False)
    del SA
    t2 = time.perf_counter()
    log(f"[cpu-full] QR {t2 - t1:.1f} s")
    A = pipeline.csr(S.row_ptr, S.col, S.val, S.m, S.n)
    x, results = pipeline.refined_lsqr(
        A, R, S.b[0], refine=refine,
        on_sweep=lambda k, r: log(f"[cpu-full] LSQR sweep {k}: {r.itn} iterations, {time.perf_counter() - t2:.1f} s"))
    t3 = time.perf_counter()
    met = pipeline.residual_metrics(A, x, S.b[0])
    return {"value": t3 - t0, "unit": "s", "cores": threads, "kind": "oracle", "cpu": cpu_model(),
            "sample": f"the whole oracle solve of the {S.m}x{S.n} system, measured (not extrapolated)",
            "phases_s": {"sketch": t1 - t0, "qr": t2 - t1, "lsqr": t3 - t2},
            "itn_sweeps": [r.itn for r in results], "relres": met["relres"]}


def stored_full_run(workload):
    """A measured whole-oracle run of this workload on the GPU machine's host
    (profiles/oracle_full_<workload>.md, written from --cpu-baseline full), or None."""
    import re

    path = os.path.join(ROOT, "profiles", f"oracle_full_{workload}.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    return json.loads(m.group(1)) if m else None


def cpu_baseline(S, s, itn_total, threads):
    """The oracle, as it stands, on a bounded sample of the workload, extrapolated
    to a full time-to-tolerance estimate: the full sketch, the QR of the first n/4
    columns of SA (scaled by the Householder flop ratio), and two LSQR
    iterations of the full-size implicit operator (scaled by the iteration count)."""
    import numpy as np
    import scipy.linalg as sla

    from oracle import countsketch, pipeline, qr
    from oracle.lsqr import lsqr

    t0 = time.perf_counter()
    h, sign = countsketch.hash_sign(S.m, s, SKETCH_SEED)
    SA, _ = countsketch.sketch_dense(S.row_ptr, S.col, S.val, h, sign, s, S.n)
    t_sketch = time.perf_counter() - t0
    ns = max(64, S.n // 4)
    t0 = time.perf_counter()
    qr.r_factor(SA[:, :ns], check_rank=False)
    t_qr_sample = time.perf_counter() - t0
    del SA
    ratio = (ns * ns * (s - ns / 3.0)) / (S.n * S.n * (s - S.n / 3.0))
    A = pipeline.csr(S.row_ptr, S.col, S.val, S.m, S.n)
    AT = A.T.tocsr()
    Rt = np.triu(np.ones((S.n, S.n))) + np.eye(S.n) * S.n
    t0 = time.perf_counter()
    lsqr(lambda v: A @ sla.solve_triangular(Rt, v),
         lambda u: sla.solve_triangular(Rt, AT @ u, trans="T"), S.b[0], S.n, atol=0, btol=0,
         conlim=0, itmax=2)
    t_it = (time.perf_counter() - t0) / 2.0
    est = t_sketch + t_qr_sample / ratio + t_it * itn_total
    return {"value": est, "unit": "s", "cores": threads, "kind": "oracle", "cpu": cpu_model(),
            "estimate": "extrapolated from the bounded sample below, not a whole run",
            "sample": (f"oracle on the {S.m}x{S.n} system: full count sketch ({t_sketch:.1f} s), "
                       f"Householder QR of SA[:, :{ns}] ({t_qr_sample:.1f} s, scaled by the flop "
                       f"ratio {ratio:.4f}), 2 LSQR iterations ({t_it:.2f} s each, scaled to "
                       f"{itn_total} iterations)")}


def pipeline_ideal(S, s, qd, rd, itn, nrhs):
    """The method's phase times at the nominal peaks (sketch and LSQR at HBM
    bandwidth, the QR at the matrix-core peak of its precision), in ms:
      sketch  12 B/nnz + row pointers + hash/sign + the dense SA written once
      qr      2 n^2 (s - n/3) Householder flops (R only)
      lsqr    per iteration two passes over R's n(n+1)/2 stored entries and two
              over A's CSR (12 B/nnz + row pointers); with several right-hand
              sides in lockstep, per block iteration the same passes plus the
              m x p blocks read and written (2 m p 8 B per product)
    itn is the total iteration count (the largest over the right-hand sides)."""
    esz_sa = 8.0 if qd == "f64" else 4.0
    esz_r = 8.0 if rd == "f64" else 4.0
    n, m, nnz = S.n, S.m, S.nnz
    sketch_b = 12.0 * nnz + 8.0 * (m + 1) + 5.0 * m + 8.0 * (s + 1) + esz_sa * s * n
    qr_f = 2.0 * n * n * (s - n / 3.0)
    csr_b = 12.0 * nnz + 8.0 * (m + 1)
    it_b = 2.0 * esz_r * n * (n + 1) / 2.0 + 2.0 * csr_b
    if nrhs > 1:
        it_b += 2.0 * 2.0 * m * min(nrhs, 32) * 8.0 * ((nrhs + 31) // 32)
    parts = {"sketch": sketch_b / (HBM_PEAK_GBS * 1e9) * 1e3,
             "qr": qr_f / (MFMA_PEAK_TFLOPS[qd] * 1e12) * 1e3,
             "lsqr": itn * it_b / (HBM_PEAK_GBS * 1e9) * 1e3}
    return parts


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="poisson2d_8x8")
    ap.add_argument("--precision", default="f64", choices=["f64", "f32", "f64f32"],
                    help="f64: float64 QR and R^-1; f32: float32 QR on matrix cores, float32-stored "
                         "R^-1; f64f32: float64 QR, float32-stored R^-1")
    ap.add_argument("--itmax", type=int, default=0, help="LSQR iteration limit per sweep (0: n)")
    ap.add_argument("--refine", type=int, default=2)
    ap.add_argument("--nrhs", type=int, default=1,
                    help="right-hand sides u_k = sin(k pi x) sin(pi y)..., k = 1..nrhs, solved together")
    ap.add_argument("--lockstep", type=int, default=1, help="1: lockstep blocks of 32; 0: one at a time")
    ap.add_argument("--operator", default="implicit", choices=["implicit", "explicit"],
                    help="implicit: A (R^-1 v), R^-T (A^T u) (Remark 3.2); explicit: dense B = A R^-1 "
                         "formed once, then dense products (Alg. 1 step 4; one right-hand side at a time)")
    ap.add_argument("--start", default="sketch", choices=["sketch", "zero"],
                    help="LSQR starting point: sketch = y0 = Q^T (S b) from the QR of [SA | Sb] "
                         "(Remark 3.1); zero = y0 = 0 (Sec. 4.1)")
    ap.add_argument("--precond", default="qr", choices=["qr", "svd"],
                    help="qr: CSQRP-LSQR (Alg. 1); svd: CSSVDP-LSQR (Alg. 2), the truncated SVD "
                         "preconditioner P = V_r Sigma_r^-1 (float64 QR and SVD; --precision f64f32 "
                         "stores P in float32; starts from y0 = 0)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline", default="sample", choices=["sample", "full"],
                    help="sample: the oracle on a bounded sample (about 10-30 s), extrapolated; "
                         "full: the whole oracle solve, measured (minutes)")
    ap.add_argument("--no-trace", action="store_true")
    ap.add_argument("--qr-lookahead", type=int, default=0, choices=[0, 1],
                    help="1: next outer block's QR panels beside the trailing update")
    ap.add_argument("--backward", action="store_true",
                    help="also time the backward pass (gradients w.r.t. b and A's values) of "
                         "L = 1/2 sum_k ||E x_k - u_k||^2 at 10^4 sample points")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 1 GiB device-to-device copy first (reference kernel of "
                         "known traffic for hardware byte counters)")
    args = ap.parse_args()
    if args.precond == "svd":
        if args.precision == "f32":
            ap.error("--precond svd factors in float64 (use --precision f64 or f64f32)")
        args.start = "zero"  # the sketched start of Remark 3.1 comes from the QR's own factor
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2409_15818_amd as R
    from oracle import pipeline  # only for the L2 error / residual check of the output
    from rfmgen import build_config, feature_eval, sample_points

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {src.numel() * 8} bytes read, {dst.numel() * 8} bytes written")
        del src, dst
    log(f"[bench] building {args.workload}")
    S, s = build_config(args.workload, modes=tuple(range(1, args.nrhs + 1)))
    A = R.CSR.from_numpy(S.row_ptr, S.col, S.val, S.m, S.n)
    b = torch.tensor(S.b[0] if args.nrhs == 1 else S.b, device="cuda")
    h = R.Handle()
    R.rfmls_qr_lookahead(h, bool(args.qr_lookahead))
    opts = R.default_opts(refine=args.refine, lockstep=args.lockstep, itmax=args.itmax)
    qd, rd = {"f64": ("f64", "f64"), "f32": ("f32", "f32"), "f64f32": ("f64", "f32")}[args.precision]

    def step(ev=None):
        if ev is not None:
            ev[0].record()
        AT = R.rfmls_transpose(h, A)
        if ev is not None:
            ev[1].record()
        if args.start == "sketch":
            # S b rides along as extra columns of SA through the QR (Remark 3.1)
            SA = R.sketch_buffer(s, S.n + args.nrhs, qd)
            SA, _, _, Sb = R.rfmls_sketch(h, A, s, SKETCH_SEED, b=b, dtype=qd, SA=SA)
        else:
            SA, _, _, _ = R.rfmls_sketch(h, A, s, SKETCH_SEED, dtype=qd)
        if ev is not None:
            ev[2].record()
        if args.precond == "svd":
            P, X0 = R.rfmls_precond_svd(h, SA, S.n, p_store=rd), None
        elif args.start == "sketch":
            P, X0 = R.rfmls_precond_x0(h, SA, S.n, Sb if args.nrhs > 1 else Sb[0], qd, rd)
        else:
            P, X0 = R.rfmls_precond(h, SA, qd, rd), None
        del SA
        if ev is not None:
            ev[3].record()
        if args.operator == "explicit":
            Bm = R.rfmls_form_B(h, A, P)
            X, Rres, info, rc = R.rfmls_solve_explicit(h, A, AT, P, Bm, b, opts, x0=X0)
            del Bm
        else:
            X, Rres, info, rc = R.rfmls_solve(h, A, AT, P, b, opts, x0=X0)
        if ev is not None:
            ev[4].record()
        return X, info, P, AT, Rres

    for w in range(args.warmup):
        log(f"[bench] warmup {w + 1}/{args.warmup}")
        try:
            out = step()
        except R.RfmlsError as e:
            if e.status != -6:
                raise
            # the float32 factor cannot precondition this system (RFMLS_E_PRECISION):
            # nothing to time; report the library's refusal
            print(json.dumps({
                "metric": METRIC, "value": None, "unit": "s", "n_gpus": 1, "steps": 0, "warmup": args.warmup,
                "ms_per_step": None, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
                "dtype": qd, "data": "synthetic",
                "config": {"workload": args.workload, "m": S.m, "n": S.n, "nnz": S.nnz, "s": s,
                           "precision": args.precision, "refine": args.refine, "nrhs": args.nrhs,
                           "start": args.start, "operator": args.operator, "precond": args.precond},
                "refused": str(e)}), flush=True)
            h.close()
            return
        del out
    torch.cuda.synchronize()
    times, phases = [], []
    X = info = None
    for k in range(args.steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X, info, P, AT, Rres = step(ev)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        times.append(dt)
        phases.append({"transpose": ev[0].elapsed_time(ev[1]), "sketch": ev[1].elapsed_time(ev[2]),
                       ("qr_and_svd" if args.precond == "svd" else "qr_and_inverse"): ev[2].elapsed_time(ev[3]),
                       "lsqr": ev[3].elapsed_time(ev[4])})
        log(f"[bench] step {k + 1}/{args.steps}: {dt * 1e3:.1f} ms  itn={[i['itn'] for i in info]}")
        if k + 1 < args.steps:
            del P, AT, Rres
    med = statistics.median(times)
    ph = {key: statistics.median(p[key] for p in phases) for key in phases[0]}

    kernels, roof = [], None
    if not args.no_trace:
        R.rfmls_trace_enable(h, True)
        _ = step()
        torch.cuda.synchronize()
        kernels = R.rfmls_trace_read(h)
        R.rfmls_trace_enable(h, False)
        _[2].free()
        del _
        for k in kernels:
            k["avg_ms"] = k["ms"] / max(k["launches"], 1)
            k["gbs"] = k["bytes"] / (k["ms"] * 1e-3) / 1e9 if k["ms"] > 0 else 0.0
            k["tflops"] = k["flops"] / (k["ms"] * 1e-3) / 1e12 if k["ms"] > 0 else 0.0
        kernels.sort(key=lambda k: -k["ms"])
        dom = kernels[0]
        traffic = measured_traffic(dom["name"], args.workload, args.precision)
        if dom["name"] in ALU_KERNELS:
            roof = {"kernel": dom["name"], "bound": "alu", "achieved": round(dom["tflops"], 3),
                    "peak": ALU_PEAK_TFLOPS[qd], "unit": "TFLOP/s",
                    "frac": round(dom["tflops"] / ALU_PEAK_TFLOPS[qd], 4), "traffic": traffic}
        elif dom["name"] in COMPUTE_KERNELS:
            roof = {"kernel": dom["name"], "bound": "mfma", "achieved": round(dom["tflops"], 3),
                    "peak": MFMA_PEAK_TFLOPS[qd], "unit": "TFLOP/s",
                    "frac": round(dom["tflops"] / MFMA_PEAK_TFLOPS[qd], 4), "traffic": traffic}
        else:
            roof = {"kernel": dom["name"], "bound": "hbm", "achieved": round(dom["gbs"], 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(dom["gbs"] / HBM_PEAK_GBS, 4),
                    "traffic": traffic}
        roof["algorithmic_bytes_per_launch"] = dom["bytes"] / max(dom["launches"], 1)
        roof["flops_per_launch"] = dom["flops"] / max(dom["launches"], 1)

    # accuracy of the measured solve (every right-hand side)
    Xn = X.detach().cpu().numpy().reshape(args.nrhs, S.n)
    Ah = pipeline.csr(S.row_ptr, S.col, S.val, S.m, S.n)
    pts = sample_points(S.d)
    E = pipeline.csr(*feature_eval(S, pts), len(pts), S.n)
    mets = [pipeline.residual_metrics(Ah, Xn[k], S.b[k]) for k in range(args.nrhs)]
    l2s = [pipeline.l2_error(E, Xn[k], S.exact(pts, S.modes[k])) for k in range(args.nrhs)]
    met, l2, x = mets[0], l2s[0], Xn[0]
    gold_path = os.path.join(ROOT, "tests", "golden", f"{args.workload}.json")
    vs_oracle = None
    if os.path.exists(gold_path):
        gold = json.load(open(gold_path))
        if args.precond == "svd":
            gold = gold.get("svd")
    if os.path.exists(gold_path) and gold:
        vs_oracle = {"oracle_normr": gold["normr"], "rel_diff_normr": abs(met["normr"] - gold["normr"]) / gold["normr"],
                     "oracle_l2_error": gold["l2_error"], "l2_ratio": l2 / gold["l2_error"]}

    bwd = None
    if args.backward:
        # dL/dx_k = E^T (E x_k - u_k) (the loss's own gradient, host side, untimed)
        Gn = np.stack([E.T @ (E @ Xn[k] - S.exact(pts, S.modes[k])) for k in range(args.nrhs)])
        G = torch.tensor(Gn[0] if args.nrhs == 1 else Gn, device="cuda")
        Xd = X.reshape(args.nrhs, S.n) if args.nrhs > 1 else X
        bt = []
        for k in range(args.steps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            dB, dAv, binfo, brc = R.rfmls_solve_backward(h, A, AT, P, Xd, Rres, G, opts)
            torch.cuda.synchronize()
            if k > 0:
                bt.append(time.perf_counter() - t0)
        # adjoint identity for the first right-hand side: <dL/db, db> = g . (A^+ db)
        db = torch.tensor(np.random.default_rng(9).standard_normal(S.m), device="cuda")
        xd, _, _, _ = R.rfmls_solve(h, A, AT, P, db, opts)
        lhs = float((dB if dB.dim() == 1 else dB[0]) @ db)
        rhs = float(np.dot(Gn[0], xd.cpu().numpy()))
        bwd = {"ms": round(1e3 * statistics.median(bt), 3), "nrhs": args.nrhs,
               "iterations_max": int(max(i["itn"] for i in binfo)),
               "adjoint_identity_rel_err": abs(lhs - rhs) / abs(rhs)}
        log(f"[bench] backward {bwd}")

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle sample)")
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
        if args.cpu_baseline == "full":
            cpu = cpu_full_run(S, s, args.refine, threads)
        else:
            cpu = cpu_baseline(S, s, int(sum(i["itn"] for i in info)), threads)
            full = stored_full_run(args.workload)
            if full is not None:
                # the extrapolation checked against a measured whole run on the same host
                cpu["measured_full_run"] = {k: full[k] for k in ("value", "cores", "cpu", "phases_s")
                                            if k in full}

    pipe = None
    if args.operator == "implicit" and args.precond == "qr":
        parts = pipeline_ideal(S, s, qd, rd, int(max(i["itn"] for i in info)), args.nrhs)
        ideal = sum(parts.values())
        pipe = {"ideal_ms": round(ideal, 3), "measured_ms": round(1e3 * med, 3),
                "frac": round(ideal / (1e3 * med), 4),
                "ideal_parts_ms": {k: round(v, 3) for k, v in parts.items()}}

    out = {
        "metric": METRIC, "value": round(med, 6), "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * sum(times) / len(times), 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": qd,
        "data": "synthetic",
        "config": {"workload": args.workload, "m": S.m, "n": S.n, "nnz": S.nnz, "s": s,
                   "precision": args.precision, "refine": args.refine, "itmax": args.itmax, "atol": opts.atol, "btol": opts.btol,
                   "nrhs": args.nrhs, "lockstep": bool(args.lockstep and args.nrhs > 1),
                   "start": args.start, "operator": args.operator, "precond": args.precond,
                   "qr_lookahead": bool(args.qr_lookahead)},
        "svd": None if args.precond != "svd" else {"rank": P.rank, "sweeps": P.sweeps, "last_off": P.off},
        "phases_ms": {k: round(v, 3) for k, v in ph.items()},
        "iterations": {"total": int(info[0]["itn"]), "first_sweep": int(info[0]["itn_first"]),
                       "istop": int(info[0]["istop"]),
                       "max_over_rhs": int(max(i["itn"] for i in info))},
        "relres": met["relres"], "normal_relres": met["normal_relres"], "l2_error": l2,
        "per_rhs": None if args.nrhs == 1 else {
            "relres_max": max(mm["relres"] for mm in mets),
            "normal_relres_max": max(mm["normal_relres"] for mm in mets),
            "l2_error": [float(f"{v:.3e}") for v in l2s]},
        "vs_oracle": vs_oracle,
        "backward": bwd,
        "roofline": roof,
        "pipeline_roofline": pipe,
        "tuned_shapes": [{k: (round(v, 4) if isinstance(v, float) else v) for k, v in t.items()}
                         for t in R.rfmls_tune_read(h)],
        "kernels": [{k2: (round(v, 4) if isinstance(v, float) else v) for k2, v in k.items()}
                    for k in kernels[:12]],
        "cpu_baseline": cpu,
    }
    # release the library's objects while the runtime is fully up (not from
    # finalisers at interpreter exit)
    torch.cuda.synchronize()
    P.free()
    h.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
