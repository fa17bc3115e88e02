"""Python binding of the rfmls C-ABI: the same entry points, taking torch
tensors that live on the GPU (torch provides device memory and the current
stream).  Every function only marshals arguments; all computation happens in
librfmls.so."""

from __future__ import annotations

import ctypes as C
import sys
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import RFMLS_F32, RFMLS_F64, rfmls_csr, rfmls_info, rfmls_opts

DTYPES = {"f64": RFMLS_F64, "f32": RFMLS_F32}


class RfmlsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_lib.STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


@dataclass
class CSR:
    """CSR matrix on the GPU: row_ptr int64[m+1], col int32[nnz], val float64[nnz]."""
    m: int
    n: int
    row_ptr: torch.Tensor
    col: torch.Tensor
    val: torch.Tensor

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    def c(self) -> rfmls_csr:
        for t, dt in ((self.row_ptr, torch.int64), (self.col, torch.int32), (self.val, torch.float64)):
            if t.dtype != dt or not t.is_contiguous() or t.device.type != "cuda":
                raise ValueError("CSR arrays must be contiguous CUDA tensors (int64, int32, float64)")
        return rfmls_csr(self.m, self.n, self.nnz, self.row_ptr.data_ptr(),
                         self.col.data_ptr() if self.nnz else None,
                         self.val.data_ptr() if self.nnz else None)

    @staticmethod
    def from_numpy(row_ptr, col, val, m, n, device="cuda"):
        return CSR(int(m), int(n), torch.as_tensor(row_ptr, dtype=torch.int64).to(device).contiguous(),
                   torch.as_tensor(col, dtype=torch.int32).to(device).contiguous(),
                   torch.as_tensor(val, dtype=torch.float64).to(device).contiguous())


def default_opts(**kw) -> rfmls_opts:
    o = rfmls_opts()
    _lib.load().rfmls_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


class Handle:
    """rfmls_create / rfmls_destroy bound to a device and its current torch stream."""

    def __init__(self, device=None, stream=None):
        lib = _lib.load()
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else
                           torch.device(device).index or 0)
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        self.device = dev
        self.stream = st
        h = C.c_void_p()
        rc = lib.rfmls_create(C.byref(h), dev.index, C.c_void_p(st.cuda_stream))
        if rc != 0:
            raise RfmlsError(rc, "rfmls_create failed")
        self._h = h
        self._lib = lib

    def check(self, rc: int, allow_warn: bool = True) -> int:
        if rc < 0 or (rc > 0 and not allow_warn):
            msg = self._lib.rfmls_last_error(self._h).decode()
            raise RfmlsError(rc, msg)
        return rc

    def close(self):
        if getattr(self, "_h", None):
            self._lib.rfmls_destroy(self._h)
            self._h = None

    def __del__(self):
        # at interpreter exit the HIP runtime may already be torn down: leave the
        # release to process exit then (call close() to release earlier)
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Precond:
    """Library-owned preconditioner (R and X = R^{-1}, or the SVD preconditioner
    P = V_r Sigma_r^{-1}); freed with rfmls_precond_free.  For the SVD kind,
    `rank`, `sweeps`, `off` and `status` (0, or RFMLS_W_NOCONV when the Jacobi
    sweeps hit their limit) are filled in."""

    def __init__(self, handle: Handle, ptr: C.c_void_p, n: int, kind: str = "qr"):
        self.handle = handle
        self._p = ptr
        self.n = n
        self.kind = kind
        self.rank = n
        self.sweeps = 0
        self.off = 0.0
        self.status = 0

    def free(self):
        if getattr(self, "_p", None):
            _lib.load().rfmls_precond_free(self._p)
            self._p = None

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.free()
        except Exception:
            pass


def rfmls_qr_panel_mode(h: Handle, mode: int):
    """0: CholeskyQR2 panels where eligible (default); 1: unblocked Householder panels;
    2 / 3: CholeskyQR2 with its first / second pass forced to fail (fallback tests)."""
    h.check(h._lib.rfmls_qr_panel_mode(h._h, int(mode)))


def rfmls_qr_lookahead(h: Handle, enable: bool):
    """Run the next outer block's QR panels beside the trailing update (CholeskyQR2 panels)."""
    h.check(h._lib.rfmls_qr_lookahead(h._h, int(bool(enable))))


def rfmls_tune_enable(h: Handle, enable: bool = True):
    h.check(h._lib.rfmls_tune_enable(h._h, int(bool(enable))))


def rfmls_tune_read(h: Handle) -> list:
    """The launch shapes the autotuner kept on this handle, one dict per tuned matrix."""
    cap = 64
    buf = (_lib.rfmls_tune_entry * cap)()
    cnt = C.c_int(0)
    h.check(h._lib.rfmls_tune_read(h._h, buf, cap, C.byref(cnt)))
    return [dict(kernel=buf[k].kernel.decode(), rows=buf[k].rows, cols=buf[k].cols, nnz=buf[k].nnz,
                 choice=buf[k].choice.decode(), ms_best=buf[k].ms_best, ms_default=buf[k].ms_default,
                 candidates=buf[k].candidates) for k in range(cnt.value)]


def rfmls_trace_enable(h: Handle, enable: bool = True):
    h.check(h._lib.rfmls_trace_enable(h._h, int(bool(enable))))


def rfmls_trace_read(h: Handle) -> list:
    """Per-kernel aggregates since the last read: name, launches, ms, bytes, flops."""
    cap = 64
    buf = (_lib.rfmls_trace_entry * cap)()
    cnt = C.c_int(0)
    h.check(h._lib.rfmls_trace_read(h._h, buf, cap, C.byref(cnt)))
    return [dict(name=buf[k].name.decode(), launches=buf[k].launches, ms=buf[k].ms,
                 bytes=buf[k].bytes, flops=buf[k].flops) for k in range(cnt.value)]


def rfmls_transpose(h: Handle, A: CSR) -> CSR:
    dev = A.row_ptr.device
    rp = torch.empty(A.n + 1, dtype=torch.int64, device=dev)
    col = torch.empty(max(A.nnz, 1), dtype=torch.int32, device=dev)
    val = torch.empty(max(A.nnz, 1), dtype=torch.float64, device=dev)
    h.check(h._lib.rfmls_transpose(h._h, C.byref(A.c()), _ptr(rp), _ptr(col), _ptr(val)))
    return CSR(A.n, A.m, rp, col[:A.nnz], val[:A.nnz])


def sketch_buffer(s: int, cols: int, dtype: str = "f64", device="cuda") -> torch.Tensor:
    """Row-major s x ld buffer for SA, ld = cols rounded up to 128 elements:
    aligned rows, and room for the QR's widest tile (rfmls_precond_x0 uses
    the columns beyond n as scratch)."""
    ld = (cols + 127) // 128 * 128
    return torch.empty((s, ld), dtype=torch.float64 if dtype == "f64" else torch.float32,
                       device=device)


def rfmls_sketch(h: Handle, A: CSR, s: int, seed: int, hash_in=None, sign_in=None, b=None,
                 dtype: str = "f64", want_maps: bool = False, SA=None):
    """Returns (SA [s x n row-major view, rows ld >= n apart], hash or None, sign
    or None, Sb or None).  SA may be given (any row stride >= n)."""
    dev = A.row_ptr.device
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if SA is None:
        SA = sketch_buffer(s, A.n, dtype, dev)[:, :A.n]
    hout = torch.empty(A.m, dtype=torch.int32, device=dev) if want_maps else None
    sout = torch.empty(A.m, dtype=torch.int8, device=dev) if want_maps else None
    Sb = None
    nrhs = ldb = 0
    if b is not None:
        bb = b if b.dim() == 2 else b.reshape(1, -1)  # [nrhs, m]: rhs k contiguous
        bb = bb.contiguous()
        nrhs, ldb = bb.shape[0], bb.shape[1]
        Sb = torch.empty((nrhs, s), dtype=torch.float64, device=dev)
        b = bb
    h.check(h._lib.rfmls_sketch(h._h, C.byref(A.c()), s, C.c_uint64(seed & (2**64 - 1)),
                                _ptr(hash_in), _ptr(sign_in), _ptr(hout), _ptr(sout), _ptr(b),
                                nrhs, ldb, _ptr(Sb), DTYPES[dtype], _ptr(SA), SA.stride(0)))
    return SA, hout, sout, Sb


def rfmls_precond(h: Handle, SA: torch.Tensor, qr_dtype: str = "f64", r_store: str = "f64") -> Precond:
    s, n = SA.shape
    p = C.c_void_p()
    h.check(h._lib.rfmls_precond(h._h, s, n, DTYPES[qr_dtype], DTYPES[r_store], _ptr(SA),
                                 SA.stride(0), C.byref(p)))
    return Precond(h, p, n)


def rfmls_precond_x0(h: Handle, SA: torch.Tensor, n: int, Sb: torch.Tensor, qr_dtype: str = "f64",
                     r_store: str = "f64"):
    """Preconditioner and sketched starting points (Remark 3.1).  SA: [s, ld]
    with ld >= n + nrhs (its columns n.. are scratch); Sb: [nrhs, s] (or [s])
    from rfmls_sketch.  Returns (Precond, X0 [nrhs, n] or [n])."""
    s = SA.shape[0]
    single = Sb.dim() == 1
    SB = (Sb.reshape(1, -1) if single else Sb).contiguous()
    nrhs = SB.shape[0]
    X0 = torch.empty((nrhs, n), dtype=torch.float64, device=SA.device)
    p = C.c_void_p()
    h.check(h._lib.rfmls_precond_x0(h._h, s, n, DTYPES[qr_dtype], DTYPES[r_store], _ptr(SA),
                                    SA.stride(0), _ptr(SB), nrhs, _ptr(X0), n, C.byref(p)))
    return Precond(h, p, n), (X0[0] if single else X0)


def rfmls_precond_svd(h: Handle, SA: torch.Tensor, n: int | None = None, rcond: float = 0.0,
                      p_store: str = "f64", max_sweeps: int = 0) -> Precond:
    """CSSVDP preconditioner (Alg. 2 step 3) of the float64 sketch SA [s, ld]
    (its first n columns; consumed).  rcond <= 0 selects n u."""
    s = SA.shape[0]
    n = SA.shape[1] if n is None else n
    p = C.c_void_p()
    st = h.check(h._lib.rfmls_precond_svd(h._h, s, n, DTYPES[p_store], _ptr(SA), SA.stride(0),
                                          float(rcond), int(max_sweeps), C.byref(p)))
    P = Precond(h, p, n, kind="svd")
    rank, sweeps, off = C.c_int64(), C.c_int(), C.c_double()
    h.check(h._lib.rfmls_precond_svd_stats(p, C.byref(rank), C.byref(sweeps), C.byref(off)))
    P.rank, P.sweeps, P.off, P.status = rank.value, sweeps.value, off.value, st
    return P


def rfmls_precond_export_P(h: Handle, P: Precond) -> torch.Tensor:
    """The stored preconditioner as a dense n x n float64 matrix."""
    X = torch.empty((P.n, P.n), dtype=torch.float64, device=h.device)
    h.check(h._lib.rfmls_precond_export_P(h._h, P._p, _ptr(X)))
    return X


def rfmls_precond_export_sigma(h: Handle, P: Precond) -> torch.Tensor:
    """Singular values of an SVD preconditioner, in the order of P's columns."""
    sig = torch.empty(P.n, dtype=torch.float64, device=h.device)
    h.check(h._lib.rfmls_precond_export_sigma(h._h, P._p, _ptr(sig)))
    return sig


def rfmls_precond_import_R(h: Handle, R: torch.Tensor, r_store: str = "f64") -> Precond:
    n = R.shape[0]
    R = R.contiguous()
    p = C.c_void_p()
    h.check(h._lib.rfmls_precond_import_R(h._h, n, _ptr(R), DTYPES[r_store], C.byref(p)))
    return Precond(h, p, n)


def rfmls_precond_export_R(h: Handle, P: Precond) -> torch.Tensor:
    R = torch.empty((P.n, P.n), dtype=torch.float64, device=h.device)
    h.check(h._lib.rfmls_precond_export_R(h._h, P._p, _ptr(R)))
    return R


def rfmls_precond_export_Rinv(h: Handle, P: Precond) -> torch.Tensor:
    X = torch.empty((P.n, P.n), dtype=torch.float64, device=h.device)
    h.check(h._lib.rfmls_precond_export_Rinv(h._h, P._p, _ptr(X)))
    return X


def rfmls_solve(h: Handle, A: CSR, AT: CSR, P: Precond, B: torch.Tensor, opts: rfmls_opts | None = None,
                want_residual: bool = True, x0: torch.Tensor | None = None):
    """B: [nrhs, m] (or [m]) float64; x0: optional starting points shaped like
    the result (sets opts.x_init).  Returns (X [nrhs, n], Rres [nrhs, m] or
    None, [info dicts], status)."""
    single = B.dim() == 1
    Bm = (B.reshape(1, -1) if single else B).contiguous()
    nrhs = Bm.shape[0]
    if x0 is None:
        X = torch.empty((nrhs, A.n), dtype=torch.float64, device=B.device)
    else:
        X = x0.reshape(nrhs, A.n).to(dtype=torch.float64, device=B.device).clone()
    R = torch.empty((nrhs, A.m), dtype=torch.float64, device=B.device) if want_residual else None
    infos = (rfmls_info * nrhs)()
    o = opts if opts is not None else default_opts()
    if x0 is not None:
        o = rfmls_opts.from_buffer_copy(o)
        o.x_init = 1
    rc = h.check(h._lib.rfmls_solve(h._h, C.byref(A.c()), C.byref(AT.c()), P._p, _ptr(Bm), A.m, nrhs,
                                    _ptr(X), A.n, _ptr(R), A.m, C.byref(o), infos))
    info = [infos[k].as_dict() for k in range(nrhs)]
    if single:
        return X[0], (R[0] if R is not None else None), info, rc
    return X, R, info, rc


def rfmls_solve_noalloc(h: Handle, A: CSR, AT: CSR, P: Precond, B: torch.Tensor, X: torch.Tensor,
                        Rres: torch.Tensor | None = None, opts: rfmls_opts | None = None):
    """rfmls_solve with nothing allocated: B [nrhs, m] (or [m]), X [nrhs, n] (or [n])
    and Rres (same shape as B, or None) are caller-allocated contiguous float64
    tensors; X is read as the starting point when opts.x_init is set.  Returns
    ([info dicts], status)."""
    for t in (B, X) + (() if Rres is None else (Rres,)):
        if t.dtype != torch.float64 or not t.is_contiguous():
            raise ValueError("B, X and Rres must be contiguous float64 tensors")
    nrhs = 1 if B.dim() == 1 else B.shape[0]
    infos = (rfmls_info * nrhs)()
    o = opts if opts is not None else default_opts()
    rc = h.check(h._lib.rfmls_solve_noalloc(h._h, C.byref(A.c()), C.byref(AT.c()), P._p, _ptr(B), A.m, nrhs,
                                            _ptr(X), A.n, _ptr(Rres), A.m, C.byref(o), infos))
    return [infos[k].as_dict() for k in range(nrhs)], rc


def rfmls_precond_stats(P: Precond) -> dict:
    """min|r_ii| / max|r_jj| and min_j |r_jj| / ||R[:, j]|| of a QR preconditioner."""
    pr, rho = C.c_double(0.0), C.c_double(0.0)
    rc = _lib.load().rfmls_precond_stats(P._p, C.byref(pr), C.byref(rho))
    if rc != 0:
        raise RfmlsError(rc, "rfmls_precond_stats failed")
    return {"pivot_ratio": pr.value, "rho_min": rho.value}


def rfmls_noalloc_scratch_bytes() -> int:
    return int(_lib.load().rfmls_noalloc_scratch_bytes())


def rfmls_form_B(h: Handle, A: CSR, P: Precond) -> torch.Tensor:
    """The explicit B = A R^{-1} ([m, n] row-major float64)."""
    Bm = torch.empty((A.m, A.n), dtype=torch.float64, device=A.row_ptr.device)
    h.check(h._lib.rfmls_form_B(h._h, C.byref(A.c()), P._p, _ptr(Bm), A.n))
    return Bm


def rfmls_solve_explicit(h: Handle, A: CSR, AT: CSR, P: Precond, Bm: torch.Tensor, B: torch.Tensor,
                         opts: rfmls_opts | None = None, want_residual: bool = True,
                         x0: torch.Tensor | None = None):
    """rfmls_solve with the products taken with the explicit Bm (rfmls_form_B)."""
    single = B.dim() == 1
    Bb = (B.reshape(1, -1) if single else B).contiguous()
    nrhs = Bb.shape[0]
    if x0 is None:
        X = torch.empty((nrhs, A.n), dtype=torch.float64, device=B.device)
    else:
        X = x0.reshape(nrhs, A.n).to(dtype=torch.float64, device=B.device).clone()
    R = torch.empty((nrhs, A.m), dtype=torch.float64, device=B.device) if want_residual else None
    infos = (rfmls_info * nrhs)()
    o = opts if opts is not None else default_opts()
    if x0 is not None:
        o = rfmls_opts.from_buffer_copy(o)
        o.x_init = 1
    rc = h.check(h._lib.rfmls_solve_explicit(h._h, C.byref(A.c()), C.byref(AT.c()), P._p, _ptr(Bm),
                                             Bm.stride(0), _ptr(Bb), A.m, nrhs, _ptr(X), A.n, _ptr(R),
                                             A.m, C.byref(o), infos))
    info = [infos[k].as_dict() for k in range(nrhs)]
    if single:
        return X[0], (R[0] if R is not None else None), info, rc
    return X, R, info, rc


def rfmls_solve_backward(h: Handle, A: CSR, AT: CSR, P: Precond, X: torch.Tensor, Rres: torch.Tensor,
                         G: torch.Tensor, opts: rfmls_opts | None = None, want_db=True, want_dA=True):
    """X [nrhs, n], Rres [nrhs, m], G [nrhs, n].  Returns (dB [nrhs, m], dAval [nnz], [info], status)."""
    single = G.dim() == 1
    Xm = (X.reshape(1, -1) if single else X).contiguous()
    Rm = (Rres.reshape(1, -1) if single else Rres).contiguous()
    Gm = (G.reshape(1, -1) if single else G).contiguous()
    nrhs = Gm.shape[0]
    dB = torch.empty((nrhs, A.m), dtype=torch.float64, device=G.device) if want_db else None
    dA = torch.empty(max(A.nnz, 1), dtype=torch.float64, device=G.device) if want_dA else None
    infos = (rfmls_info * nrhs)()
    o = opts if opts is not None else default_opts()
    rc = h.check(h._lib.rfmls_solve_backward(h._h, C.byref(A.c()), C.byref(AT.c()), P._p, _ptr(Xm),
                                             A.n, _ptr(Rm), A.m, _ptr(Gm), A.n, nrhs, _ptr(dB), A.m,
                                             _ptr(dA), C.byref(o), infos))
    info = [infos[k].as_dict() for k in range(nrhs)]
    dA = dA[:A.nnz] if dA is not None else None
    if single and dB is not None:
        dB = dB[0]
    return dB, dA, info, rc
