"""ctypes declarations of librfmls (include/rfmls.h).  Loading fails loudly when
the library has not been built; there is no fallback implementation."""

from __future__ import annotations

import ctypes as C
from pathlib import Path

LIB_PATH = Path(__file__).resolve().parent / "librfmls.so"

RFMLS_OK = 0
RFMLS_W_NOCONV = 1
RFMLS_E_ARG = -1
RFMLS_E_RANK = -2
RFMLS_E_BREAKDOWN = -3
RFMLS_E_HIP = -4
RFMLS_E_NOMEM = -5
RFMLS_E_PRECISION = -6
RFMLS_F64 = 0
RFMLS_F32 = 1

STATUS_NAMES = {0: "RFMLS_OK", 1: "RFMLS_W_NOCONV", -1: "RFMLS_E_ARG", -2: "RFMLS_E_RANK",
                -3: "RFMLS_E_BREAKDOWN", -4: "RFMLS_E_HIP", -5: "RFMLS_E_NOMEM",
                -6: "RFMLS_E_PRECISION"}

EXPORTED = [
    "rfmls_default_opts", "rfmls_create", "rfmls_destroy", "rfmls_last_error", "rfmls_transpose",
    "rfmls_sketch", "rfmls_precond", "rfmls_precond_x0", "rfmls_precond_free", "rfmls_precond_n",
    "rfmls_precond_export_R", "rfmls_precond_export_Rinv", "rfmls_precond_import_R",
    "rfmls_precond_svd", "rfmls_precond_svd_stats", "rfmls_precond_export_P", "rfmls_precond_export_sigma",
    "rfmls_solve", "rfmls_form_B", "rfmls_solve_explicit", "rfmls_solve_backward",
    "rfmls_trace_enable", "rfmls_trace_read", "rfmls_solve_noalloc", "rfmls_noalloc_scratch_bytes", "rfmls_precond_stats",
    "rfmls_tune_enable", "rfmls_tune_read", "rfmls_qr_panel_mode", "rfmls_qr_lookahead",
]


class rfmls_csr(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p)]


class rfmls_opts(C.Structure):
    _fields_ = [("atol", C.c_double), ("btol", C.c_double), ("conlim", C.c_double),
                ("itmax", C.c_int64), ("refine", C.c_int32), ("check_every", C.c_int32),
                ("lockstep", C.c_int32), ("x_init", C.c_int32), ("graph", C.c_int32),
                ("reserved", C.c_int32)]


class rfmls_info(C.Structure):
    _fields_ = [("itn", C.c_int64), ("itn_first", C.c_int64), ("istop", C.c_int32),
                ("istop_last", C.c_int32), ("normr_est", C.c_double), ("normar_est", C.c_double),
                ("anorm_est", C.c_double), ("acond_est", C.c_double), ("normb", C.c_double),
                ("normr", C.c_double), ("normar", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class rfmls_tune_entry(C.Structure):
    _fields_ = [("kernel", C.c_char * 16), ("rows", C.c_int64), ("cols", C.c_int64), ("nnz", C.c_int64),
                ("choice", C.c_char * 48), ("ms_best", C.c_double), ("ms_default", C.c_double),
                ("candidates", C.c_int32)]


class rfmls_trace_entry(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("ms", C.c_double),
                ("bytes", C.c_double), ("flops", C.c_double)]


_lib = None


class LibraryMissing(RuntimeError):
    pass


def load():
    """Load librfmls.so (built in-tree by build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        raise LibraryMissing(f"{LIB_PATH} is not built; run `python -m paper_2409_15818_amd.build`")
    lib = C.CDLL(str(LIB_PATH))
    vp, i64, i32, u64, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_uint64, C.c_double
    P = C.POINTER
    lib.rfmls_default_opts.argtypes = [P(rfmls_opts)]
    lib.rfmls_default_opts.restype = None
    lib.rfmls_create.argtypes = [P(vp), C.c_int, vp]
    lib.rfmls_destroy.argtypes = [vp]
    lib.rfmls_last_error.argtypes = [vp]
    lib.rfmls_last_error.restype = C.c_char_p
    lib.rfmls_transpose.argtypes = [vp, P(rfmls_csr), vp, vp, vp]
    lib.rfmls_sketch.argtypes = [vp, P(rfmls_csr), i64, u64, vp, vp, vp, vp, vp, i64, i64, vp,
                                 C.c_int, vp, i64]
    lib.rfmls_precond.argtypes = [vp, i64, i64, C.c_int, C.c_int, vp, i64, P(vp)]
    lib.rfmls_precond_x0.argtypes = [vp, i64, i64, C.c_int, C.c_int, vp, i64, vp, i64, vp, i64, P(vp)]
    lib.rfmls_precond_free.argtypes = [vp]
    lib.rfmls_precond_free.restype = None
    lib.rfmls_precond_n.argtypes = [vp]
    lib.rfmls_precond_n.restype = i64
    lib.rfmls_precond_export_R.argtypes = [vp, vp, vp]
    lib.rfmls_precond_export_Rinv.argtypes = [vp, vp, vp]
    lib.rfmls_precond_import_R.argtypes = [vp, i64, vp, C.c_int, P(vp)]
    lib.rfmls_precond_svd.argtypes = [vp, i64, i64, C.c_int, vp, i64, C.c_double, C.c_int, P(vp)]
    lib.rfmls_precond_svd_stats.argtypes = [vp, P(i64), P(C.c_int), P(C.c_double)]
    lib.rfmls_precond_export_P.argtypes = [vp, vp, vp]
    lib.rfmls_precond_export_sigma.argtypes = [vp, vp, vp]
    lib.rfmls_solve.argtypes = [vp, P(rfmls_csr), P(rfmls_csr), vp, vp, i64, i64, vp, i64, vp, i64,
                                P(rfmls_opts), P(rfmls_info)]
    lib.rfmls_solve_noalloc.argtypes = [vp, P(rfmls_csr), P(rfmls_csr), vp, vp, i64, i64, vp, i64, vp, i64,
                                        P(rfmls_opts), P(rfmls_info)]
    lib.rfmls_precond_stats.argtypes = [vp, P(C.c_double), P(C.c_double)]
    lib.rfmls_noalloc_scratch_bytes.argtypes = []
    lib.rfmls_noalloc_scratch_bytes.restype = i64
    lib.rfmls_form_B.argtypes = [vp, P(rfmls_csr), vp, vp, i64]
    lib.rfmls_solve_explicit.argtypes = [vp, P(rfmls_csr), P(rfmls_csr), vp, vp, i64, vp, i64, i64, vp,
                                         i64, vp, i64, P(rfmls_opts), P(rfmls_info)]
    lib.rfmls_solve_backward.argtypes = [vp, P(rfmls_csr), P(rfmls_csr), vp, vp, i64, vp, i64, vp,
                                         i64, i64, vp, i64, vp, P(rfmls_opts), P(rfmls_info)]
    lib.rfmls_qr_panel_mode.argtypes = [vp, C.c_int]
    lib.rfmls_qr_lookahead.argtypes = [vp, C.c_int]
    lib.rfmls_tune_enable.argtypes = [vp, C.c_int]
    lib.rfmls_tune_read.argtypes = [vp, P(rfmls_tune_entry), C.c_int, P(C.c_int)]
    lib.rfmls_trace_enable.argtypes = [vp, C.c_int]
    lib.rfmls_trace_read.argtypes = [vp, P(rfmls_trace_entry), C.c_int, P(C.c_int)]
    for name in EXPORTED:
        if name not in ("rfmls_default_opts", "rfmls_precond_free", "rfmls_last_error",
                        "rfmls_precond_n", "rfmls_noalloc_scratch_bytes"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib
