"""rfmls: sketch-preconditioned least squares (CSQRP-LSQR and CSSVDP-LSQR,
Chen & Tan, arXiv:2409.15818) on AMD MI355X.  The numerical path is the HIP library
librfmls.so behind the C-ABI of include/rfmls.h; this package is its binding."""

from ._lib import LibraryMissing, load  # noqa: F401
from .api import (CSR, Handle, Precond, RfmlsError, default_opts, rfmls_precond,  # noqa: F401
                  rfmls_precond_x0, rfmls_precond_export_R, rfmls_precond_export_Rinv, rfmls_precond_import_R,
                  rfmls_precond_svd, rfmls_precond_export_P, rfmls_precond_export_sigma,
                  rfmls_form_B, rfmls_noalloc_scratch_bytes, rfmls_precond_stats, rfmls_qr_panel_mode, rfmls_qr_lookahead, rfmls_sketch, rfmls_solve, rfmls_solve_backward,
                  rfmls_solve_explicit, rfmls_solve_noalloc, rfmls_trace_enable, rfmls_tune_enable,
                  rfmls_tune_read,
                  rfmls_trace_read, rfmls_transpose, sketch_buffer)
from .solve import LstsqFunction, LstsqSolver, Result, cssvdp_lsqr, csqrp_lsqr  # noqa: F401
