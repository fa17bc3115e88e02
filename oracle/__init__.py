"""CPU FP64 oracle for the CSQRP-LSQR path (count sketch -> QR preconditioner -> LSQR).

TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the
benchmark's CPU-baseline leg may import this package.  The GPU product path
never calls, links or falls back to it, and the two share no code: the oracle
is written from the paper (Def. 2.3, Alg. 1, Alg. 2, Remarks 3.1-3.3, Sec. 4.1) and
textbook LSQR (Paige & Saunders 1982) in plain numpy/scipy, slowly and
obviously, in float64.

Modules
  countsketch  hash/sign generator and the dense sketch SA = Phi D A  (Def. 2.3)
  qr           R factor of SA with a non-negative diagonal           (Alg. 1 step 3)
  svd          truncated SVD preconditioner P = V_r Sigma_r^{-1}     (Alg. 2 step 3)
  lsqr         textbook LSQR on the implicit operator A R^{-1}       (Alg. 1 steps 4-6)
  pipeline     the whole CSQRP-LSQR solve plus its reported metrics  (Sec. 4.1)
  backward     gradients of a loss of the solution w.r.t. b and A    (dense and iterative)
"""

from . import countsketch, qr, svd, lsqr, pipeline, backward  # noqa: F401
