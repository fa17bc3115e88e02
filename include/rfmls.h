/*
 * rfmls — sketch-preconditioned least squares for random-feature-method systems
 * on AMD Instinct MI355X (gfx950).
 *
 * Solves min_x ||A x - b||_2 for a sparse, ill-conditioned, overdetermined
 * A (m x n, m >> n; problem (1.1) of Chen & Tan, "High-precision randomized
 * iterative methods for the random feature method", arXiv:2409.15818) by the
 * paper's CSQRP-LSQR pipeline (Algorithm 1):
 *
 *   rfmls_sketch   count sketch SA = Phi D A, s = gamma n rows   (Def. 2.3; Alg. 1 step 2)
 *   rfmls_precond  Householder QR of SA -> R; the library keeps  (Alg. 1 step 3)
 *                  R^{-1} (upper triangular) as the preconditioner
 *                  (rfmls_precond_x0 also returns the sketched     (Remark 3.1)
 *                  solution x^(0) = R^{-1} Q^T S b as a starting point)
 *   rfmls_precond_svd  CSSVDP-LSQR's preconditioner instead:     (Alg. 2 step 3)
 *                  the truncated SVD of SA through R, P = V_r Sigma_r^{-1}
 *   rfmls_solve    LSQR on A R^{-1} (applied implicitly,          (Alg. 1 steps 4-6,
 *                  Remark 3.2) from y = 0 or a given x, x = R^{-1} y, Remarks 3.2-3.3, Sec. 4.1)
 *                  iterative refinement on the true residual
 *   rfmls_form_B / rfmls_solve_explicit  the same with the dense B = A R^{-1}
 *                  formed explicitly (Alg. 1 step 4 taken literally)
 *   rfmls_solve_backward  gradients of a loss of x w.r.t. b and A's stored values
 *
 * Conventions for every entry point
 *   - Pointers are DEVICE pointers unless marked [host].  All device buffers are
 *     owned and allocated by the caller, except the library-owned handle
 *     workspace and rfmls_precond_t.
 *   - Work is enqueued on the stream given to rfmls_create.  rfmls_transpose,
 *     rfmls_sketch and rfmls_precond are asynchronous with respect to the host
 *     (they may still block for internal workspace growth); rfmls_solve and
 *     rfmls_solve_backward synchronise the stream before returning because
 *     they report per-right-hand-side info on the host.
 *   - Return value: RFMLS_OK (0), a positive warning, or a negative error.
 *     Nothing is thrown across the ABI; rfmls_last_error() describes the last
 *     failure on a handle.  Arguments are validated before any work is
 *     enqueued; an invalid argument enqueues nothing.
 *   - Sparse matrices are CSR: row_ptr int64[rows+1] (row_ptr[0] = 0), col
 *     int32[nnz] ascending and unique within each row, val float64[nnz].
 *   - Dense row-major: element (i, j) of a matrix with leading dimension ld
 *     is at p[i * ld + j].  Blocks of right-hand sides are column-major:
 *     right-hand side k of B (m x nrhs, ldb >= m) is B + k * ldb.
 */
#ifndef RFMLS_H
#define RFMLS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RFMLS_OK = 0,
  RFMLS_W_NOCONV = 1,     /* iteration limit reached; X is still written */
  RFMLS_E_ARG = -1,       /* invalid argument (sizes, null pointers, layout) */
  RFMLS_E_RANK = -2,      /* R numerically singular: |r_ii| <= 16 u max|r_jj| */
  RFMLS_E_BREAKDOWN = -3, /* non-finite value met inside the iteration */
  RFMLS_E_HIP = -4,       /* HIP runtime error (message in rfmls_last_error) */
  RFMLS_E_NOMEM = -5,     /* device allocation of library workspace failed */
  RFMLS_E_PRECISION = -6  /* float32 factor too coarse for this system: some
                             |r_jj| / ||SA[:, j]|| <= 16 u32 (rfmls_precond) */
} rfmls_status;

typedef enum { RFMLS_F64 = 0, RFMLS_F32 = 1 } rfmls_dtype;

typedef struct rfmls_handle rfmls_handle;
typedef struct rfmls_precond rfmls_precond_t;

/* CSR matrix, device pointers.  m rows, n columns, nnz stored entries. */
typedef struct {
  int64_t m, n, nnz;
  const int64_t *row_ptr;
  const int32_t *col;
  const double *val;
} rfmls_csr;

/* [host] LSQR options (Paige & Saunders stopping rules; Sec. 4.1 uses
 * tau = 1e-8 and at most n iterations from y = 0). */
typedef struct {
  double atol;    /* S2: ||B^T r|| <= atol ||B|| ||r||; also in S1      */
  double btol;    /* S1: ||r|| <= btol ||b|| + atol ||B|| ||y||         */
  double conlim;  /* S3: cond(B) estimate >= conlim                     */
  int64_t itmax;  /* iteration limit per sweep; <= 0 means n            */
  int32_t refine; /* extra refinement sweeps on the true residual (>= 0) */
  int32_t check_every; /* host polls the device stop flag every this many
                          iterations (>= 1); iterations past the stop are
                          no-ops on the device                           */
  int32_t lockstep; /* nonzero (default): with nrhs > 1, iterate the
                       right-hand sides in lockstep blocks of 32 that share
                       every pass over A, A^T and R^{-1}; 0: one at a time */
  int32_t x_init;   /* nonzero: X holds a starting point on entry (for example
                       from rfmls_precond_x0) and the first sweep solves for
                       the correction from b - A X; 0 (default): start from
                       x = 0 (y^(0) = 0, Sec. 4.1)                        */
  int32_t graph;    /* nonzero (default): the check_every iterations between
                       two polls of the stop flag are captured once per call
                       as a HIP graph and replayed (not while kernel tracing
                       is enabled); 0: launched one kernel at a time.  The
                       iterates are the same either way                   */
  int32_t reserved; /* set to 0                                           */
} rfmls_opts;

/* [host] per right-hand side results */
typedef struct {
  int64_t itn;          /* total LSQR iterations over all sweeps           */
  int64_t itn_first;    /* iterations of the first sweep                   */
  int32_t istop;        /* stopping rule of the first sweep: 0 x=0 exact,
                           1 S1, 2 S2, 3 S3, 7 itmax                        */
  int32_t istop_last;   /* stopping rule of the last sweep                 */
  double normr_est;     /* LSQR estimate of ||r|| at the end of sweep 1    */
  double normar_est;    /* LSQR estimate of ||B^T r|| at the end of sweep 1 */
  double anorm_est;     /* Frobenius estimate of ||B||                     */
  double acond_est;     /* estimate of cond(B)                             */
  double normb;         /* ||b||                                           */
  double normr;         /* true ||b - A x|| recomputed in float64          */
  double normar;        /* true ||A^T (b - A x)||                          */
} rfmls_info;

void rfmls_default_opts(rfmls_opts *opts /* [host] */);

/* Create a handle bound to HIP device `device` and stream `stream`
 * (a hipStream_t; NULL = the null stream).  The handle owns a growable
 * device workspace freed by rfmls_destroy. */
rfmls_status rfmls_create(rfmls_handle **handle /* [host] out */, int device, void *stream);
rfmls_status rfmls_destroy(rfmls_handle *handle);
const char *rfmls_last_error(const rfmls_handle *handle);

/* A^T in CSR (n x m): at_row_ptr int64[n+1], at_col int32[nnz],
 * at_val float64[nnz], caller-allocated.  Entries of each row of A^T are in
 * ascending column (= row of A) order, so the result is deterministic.
 * Needed by rfmls_solve for the products A^T u (Alg. 1 step 5). */
rfmls_status rfmls_transpose(rfmls_handle *h, const rfmls_csr *A, int64_t *at_row_ptr,
                             int32_t *at_col, double *at_val);

/* Count sketch (Def. 2.3, Alg. 1 step 2): SA = Phi D A with Phi[h(i), i] = 1
 * and D = diag(sign).  Row j of SA is the sum, over rows i of A with h(i) = j
 * taken in ascending i, of sign(i) * A[i, :], accumulated in float64 from +0.
 *
 *   s        number of sketch rows, 1 <= s < 2^31 (the paper takes s = gamma n)
 *   seed     generator seed.  h(i) = ((x >> 32) * s) >> 32 with
 *            x = mix64(seed + (i+1) * 0x9E3779B97F4A7C15) and sign(i) = +1 iff the
 *            top bit of mix64((seed ^ 0x5555555555555555) + (i+1) * 0x9E37...15)
 *            is 0; mix64 is the SplitMix64 finaliser (all arithmetic mod 2^64).
 *   hash_in, sign_in   optional int32[m] / int8[m] maps used instead of the
 *            generator (both or neither; h in [0, s), sign in {-1, +1}).
 *   hash_out, sign_out optional int32[m] / int8[m] copies of the maps used.
 *   b, nrhs, ldb, Sb   optional: Sb (s x nrhs column-major, ld = s) = S b.
 *   sa_dtype RFMLS_F64: SA is float64; RFMLS_F32: SA is float32, each element
 *            rounded to nearest-even from its float64 sum.
 *   SA, ld_sa  dense row-major s x n output, ld_sa >= n; fully overwritten
 *            (zeros included).  SA is consumed by rfmls_precond.
 */
rfmls_status rfmls_sketch(rfmls_handle *h, const rfmls_csr *A, int64_t s, uint64_t seed,
                          const int32_t *hash_in, const int8_t *sign_in, int32_t *hash_out,
                          int8_t *sign_out, const double *b, int64_t nrhs, int64_t ldb,
                          double *Sb, rfmls_dtype sa_dtype, void *SA, int64_t ld_sa);

/* Preconditioner (Alg. 1 step 3; Thm 3.1-3.2): Householder QR of SA (s x n,
 * s >= n, row-major, ld_sa >= n; overwritten) in qr_dtype arithmetic
 * (RFMLS_F64, or RFMLS_F32 on matrix cores; must equal the sketch's sa_dtype),
 * rows of R scaled so diag(R) > 0.  The library forms and keeps X = R^{-1}
 * (upper triangular) stored in r_store precision.  Returns RFMLS_E_RANK if
 * some |r_ii| <= 16 u max_j |r_jj| (u = unit roundoff of qr_dtype; for
 * RFMLS_F32 only a zero or non-finite pivot is rejected).  With qr_dtype or
 * r_store RFMLS_F32 it returns RFMLS_E_PRECISION when
 * min_j |r_jj| / ||SA[:, j]|| <= 16 u32 (u32 = 2^-24; the margin of the
 * float64 rank test): some column of SA lies within float32 rounding of the
 * span of the columns before it, so a factor computed or stored in float32
 * carries no information in that direction and LSQR on A R^{-1} would stall
 * or slow down severalfold; such a system must be factored and stored in
 * float64 (the 8 x 8-box 2D Poisson RFM system is one).  *P_out is library-owned; free with rfmls_precond_free.  Asynchronous
 * except for these checks, which synchronise the stream.  On an error nothing
 * is returned in *P_out. */
rfmls_status rfmls_precond(rfmls_handle *h, int64_t s, int64_t n, rfmls_dtype qr_dtype,
                           rfmls_dtype r_store, void *SA, int64_t ld_sa,
                           rfmls_precond_t **P_out /* [host] out */);
/* Preconditioner plus the sketched starting point (Alg. 1 step 3 with the
 * initial guess y^(0) = Q^T (S b) of Remark 3.1).  The sketched right-hand
 * sides SB = S B (rfmls_sketch's Sb) are written into SA as columns
 * n .. n+nrhs-1 and carried through the same Householder QR, so the top n
 * entries of those columns of the triangular factor are y0_k = Q^T (S b_k)
 * (with R's row signs).  The library returns X0[:, k] = R^{-1} y0_k, the
 * minimiser of ||S (A x - b_k)||, for rfmls_solve with opts->x_init = 1.
 * Otherwise as rfmls_precond: R, its rank check (first n pivots only) and the
 * stored X = R^{-1} are those of SA alone.
 *   SA, ld_sa  s x n sketch (row-major, qr_dtype), ld_sa >= n + nrhs, s >= n + nrhs;
 *              columns n .. ld_sa-1 of every row are overwritten (scratch: the
 *              right-hand sides, then room that lets the QR's products run on
 *              whole tiles; ld_sa a multiple of 128 is fastest)
 *   SB         s x nrhs column-major float64 (ld = s), nrhs >= 1
 *   X0, ldx0   n x nrhs column-major float64 output, ldx0 >= n
 * Synchronises the stream (rank check); on error nothing is returned in *P_out. */
rfmls_status rfmls_precond_x0(rfmls_handle *h, int64_t s, int64_t n, rfmls_dtype qr_dtype,
                              rfmls_dtype r_store, void *SA, int64_t ld_sa, const double *SB,
                              int64_t nrhs, double *X0, int64_t ldx0,
                              rfmls_precond_t **P_out /* [host] out */);
/* SVD preconditioner of CSSVDP-LSQR (Alg. 2 step 3; Sec. 3.2, Thm 3.4).
 * Householder QR of SA (s x n, s >= n, row-major float64, ld_sa >= n;
 * overwritten) as rfmls_precond, then the SVD of R (SA = Q R, so SA and R share
 * Sigma and V) by one-sided Jacobi on the GPU, and the preconditioner
 * P = V_r Sigma_r^{-1}: the columns whose singular value is at most
 * rcond * sigma_1 are dropped (stored as zero columns, so LSQR never moves
 * along them), r = the number kept.  rcond <= 0 selects n u (u = 2^-53);
 * rcond >= 1 is rejected.  P is stored n x n in p_store precision and used by
 * rfmls_solve, rfmls_solve_explicit and rfmls_form_B in place of R^{-1}, and
 * by rfmls_solve_backward when r = n.  No rank check: a rank-deficient A gives
 * the minimum-norm solution of the truncated problem.  n <= 16384.
 *   max_sweeps  limit on Jacobi sweeps (<= 0: 60); if the columns are still
 *               not orthogonal to the tolerance, *P_out is returned anyway
 *               with the warning RFMLS_W_NOCONV.
 * Synchronises the stream once per sweep.  RFMLS_E_RANK if every singular
 * value is below the threshold; on an error nothing is returned in *P_out. */
rfmls_status rfmls_precond_svd(rfmls_handle *h, int64_t s, int64_t n, rfmls_dtype p_store, void *SA,
                               int64_t ld_sa, double rcond, int max_sweeps,
                               rfmls_precond_t **P_out /* [host] out */);
/* [host] Numerical rank r, Jacobi sweeps taken and the last sweep's largest
 * |cos| between two columns of R V; any pointer may be null.  RFMLS_E_ARG for a
 * QR preconditioner. */
rfmls_status rfmls_precond_svd_stats(const rfmls_precond_t *P, int64_t *rank, int *sweeps,
                                     double *off);
/* [host] Statistics of the factor R of a QR preconditioner: min|r_ii| / max|r_jj|
 * and min_j |r_jj| / ||R[:, j]|| (the column-relative pivot the float32 check
 * of rfmls_precond uses); either pointer may be null. */
rfmls_status rfmls_precond_stats(const rfmls_precond_t *P, double *pivot_ratio, double *rho_min);
void rfmls_precond_free(rfmls_precond_t *P);
int64_t rfmls_precond_n(const rfmls_precond_t *P);

/* Copies of the factor for tests: R (with positive diagonal) and X = R^{-1},
 * each n x n row-major float64 (ld = n) with zeros below the diagonal
 * (export_Rinv: RFMLS_E_ARG for an SVD preconditioner). */
rfmls_status rfmls_precond_export_R(rfmls_handle *h, const rfmls_precond_t *P, double *R);
rfmls_status rfmls_precond_export_Rinv(rfmls_handle *h, const rfmls_precond_t *P, double *X);
/* The stored preconditioner as n x n row-major float64 (ld = n): X = R^{-1}
 * for rfmls_precond, P = V_r Sigma_r^{-1} for rfmls_precond_svd (columns in the
 * Jacobi order, zero for the dropped ones). */
rfmls_status rfmls_precond_export_P(rfmls_handle *h, const rfmls_precond_t *P, double *X);
/* The n singular values of an SVD preconditioner (float64, device), in the
 * order of P's columns (not sorted). */
rfmls_status rfmls_precond_export_sigma(rfmls_handle *h, const rfmls_precond_t *P, double *sigma);
/* Build a preconditioner from a given upper-triangular R (n x n row-major
 * float64, ld = n, positive diagonal); only the upper triangle is read. */
rfmls_status rfmls_precond_import_R(rfmls_handle *h, int64_t n, const double *R,
                                    rfmls_dtype r_store, rfmls_precond_t **P_out);

/* LSQR on the preconditioned problem min ||A R^{-1} y - b|| (Alg. 1 steps 4-6,
 * operator applied implicitly as A (R^{-1} v) and R^{-T} (A^T u)), from y = 0,
 * x = R^{-1} y (or, with opts->x_init, on min ||A R^{-1} y - (b - A x_in)||,
 * x = x_in + R^{-1} y), followed by opts->refine refinement sweeps on the true
 * residual.  Each of the nrhs right-hand sides is solved independently (the
 * same iterates as a single solve) in lockstep.
 *   A, AT    the matrix and its transpose (rfmls_transpose)
 *   B, ldb   m x nrhs column-major right-hand sides (ldb >= m)
 *   X, ldx   n x nrhs column-major solutions (ldx >= n), overwritten; read
 *            first as the starting point when opts->x_init is set
 *   Rout, ldr  optional m x nrhs column-major true residuals b - A x (ldr >= m)
 *   info     [host] array of nrhs results, may be NULL
 * Returns RFMLS_W_NOCONV if some right-hand side hit itmax in its first sweep. */
rfmls_status rfmls_solve(rfmls_handle *h, const rfmls_csr *A, const rfmls_csr *AT,
                         const rfmls_precond_t *P, const double *B, int64_t ldb, int64_t nrhs,
                         double *X, int64_t ldx, double *Rout, int64_t ldr,
                         const rfmls_opts *opts, rfmls_info *info);

/* For callers that cannot allocate device memory during a call (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * rfmls_solve with nothing allocated.  Arguments, results and status codes are
 * those of rfmls_solve, with the right-hand sides solved one at a time
 * (opts->lockstep is ignored; the iterates are those of rfmls_solve with
 * lockstep = 0).  The solve's device scratch (work vectors, partial sums,
 * LSQR state and the column-run descriptors of A and A^T: 8 (4m + 8n + 8256)
 * + 512 + 68 (m + n) bytes) is a fixed array of
 * rfmls_noalloc_scratch_bytes() bytes (32 MiB) that each device the library
 * runs on holds until the process ends; a problem that needs more is rejected
 * with RFMLS_E_ARG before anything is enqueued.  The preconditioner's buffers
 * (allocated by rfmls_precond*) and the handle's pinned staging buffer
 * (allocated by rfmls_create) are used as rfmls_solve uses them.  Every call on
 * one device shares that device's array, which keeps the last call's
 * contents (the solve initialises all it reads): calls that overlap in time on
 * one device, from any handle or thread, race and give wrong results, so
 * serialise them.  Synchronises the stream before returning. */
rfmls_status rfmls_solve_noalloc(rfmls_handle *h, const rfmls_csr *A, const rfmls_csr *AT,
                                 const rfmls_precond_t *P, const double *B, int64_t ldb,
                                 int64_t nrhs, double *X, int64_t ldx, double *Rout, int64_t ldr,
                                 const rfmls_opts *opts, rfmls_info *info);
/* Size in bytes of rfmls_solve_noalloc's fixed device scratch. */
int64_t rfmls_noalloc_scratch_bytes(void);

/* Alg. 1 step 4 in its literal form: the dense preconditioned matrix
 * B = A R^{-1} (m x n, row-major float64, ld_bmat >= n; caller-allocated,
 * 8 m n bytes), formed as A times the stored X = R^{-1}, 32 columns at a time
 * (each slab of X gathered from the stored tiles, one sparse-times-dense
 * product with A, the slab written into B).  Asynchronous. */
rfmls_status rfmls_form_B(rfmls_handle *h, const rfmls_csr *A, const rfmls_precond_t *P, double *Bmat,
                          int64_t ld_bmat);
/* rfmls_solve with LSQR's products taken with the explicit Bmat from
 * rfmls_form_B (B v and B^T u as dense matrix-vector products) instead of
 * the implicit A (R^{-1} v) and R^{-T} (A^T u) (Alg. 1 step 4 vs Remark 3.2);
 * x = R^{-1} y, the refinement sweeps and the reported residuals use A (and
 * AT for ||A^T r||).  One right-hand side at a time (opts->lockstep is not
 * used); other arguments and results as rfmls_solve. */
rfmls_status rfmls_solve_explicit(rfmls_handle *h, const rfmls_csr *A, const rfmls_csr *AT,
                                  const rfmls_precond_t *P, const double *Bmat, int64_t ld_bmat,
                                  const double *B, int64_t ldb, int64_t nrhs, double *X, int64_t ldx,
                                  double *Rout, int64_t ldr, const rfmls_opts *opts,
                                  rfmls_info *info);
/* Backward of x = A^+ b for a loss L with G = dL/dX (n x nrhs, ldg >= n).
 * With r = b - A x, w = (A^T A)^{-1} g and lambda = A w:
 *   dB[:, k] = lambda_k                        (m x nrhs column-major, lddb >= m)
 *   dAval[e] = sum_k r_k[i] w_k[j] - lambda_k[i] x_k[j]   for each stored (i, j)
 * w is obtained by LSQR on the consistent system (A R^{-1})^T lambda = R^{-T} g
 * from lambda = 0 (its minimum-norm solution lambda = A w), using the same
 * preconditioned products as rfmls_solve.
 *   X, ldx  solutions from rfmls_solve; Rres, ldr residuals b - A x (m x nrhs)
 *   dB may be NULL; dAval (float64[nnz]) may be NULL. */
rfmls_status rfmls_solve_backward(rfmls_handle *h, const rfmls_csr *A, const rfmls_csr *AT,
                                  const rfmls_precond_t *P, const double *X, int64_t ldx,
                                  const double *Rres, int64_t ldr, const double *G, int64_t ldg,
                                  int64_t nrhs, double *dB, int64_t lddb, double *dAval,
                                  const rfmls_opts *opts, rfmls_info *info);

/* ---- Panel factorisation of the QR (Alg. 1 step 3) ----
 * mode 0 (default): 64-column panels of at least 1024 rows are factored by
 * CholeskyQR2 on column-scaled Gram matrices followed by the reconstruction of
 * their Householder vectors (a fixed number of passes over the panel instead
 * of one grid-wide exchange per column), in float64 arithmetic for float64 and
 * float32 panels alike (a float32 panel is rounded where it is stored); a panel
 * whose first Cholesky pivot ratio falls below 1e-7 is factored by the
 * unblocked Householder kernel.  mode 1: the unblocked Householder kernel for
 * every panel.  Modes 2 and 3 force the first, respectively second, Cholesky
 * pass of every eligible panel to fail, so that the fallback paths can be
 * tested.  Every way R satisfies R^T R = (SA)^T SA to the rounding of its
 * dtype.  Errors: RFMLS_E_ARG for a null handle or a mode outside 0..3. */
rfmls_status rfmls_qr_panel_mode(rfmls_handle *h, int mode);

/* ---- Look-ahead in the blocked QR (Alg. 1 step 3) ----
 * enable != 0: once an outer block's panels are factored, the trailing update
 * first covers only the next outer block's columns; that block's panels then
 * run on a second stream of the handle (default priority, created on first
 * use) while the handle's stream updates the remaining columns.  The factors
 * are bitwise those of the plain schedule.  Only QRs in panel mode 0 use it,
 * and only for outer blocks whose panels are all CholeskyQR2-eligible;
 * everything else keeps the plain schedule.  A panel that CholeskyQR2 declines
 * is then factored by the unblocked kernel beside the trailing update, whose
 * grid-wide exchange needs all of its workgroups resident: a bounded wait turns
 * a failure to co-schedule into an error status (RFMLS_E_HIP), never a hang.
 * Default off.  Errors: RFMLS_E_ARG for a null handle. */
rfmls_status rfmls_qr_lookahead(rfmls_handle *h, int enable);

/* ---- Autotuning of launch shapes ----
 * With tuning on (the default), the first lockstep solve, backward pass or
 * rfmls_form_B that uses a matrix of a given shape (rows, columns, stored
 * entries) on a handle times every candidate launch shape of its 32-column
 * sparse products (the width of the input window staged in LDS) on that
 * matrix, and keeps the fastest for later calls on the handle.  The candidates
 * change neither the order of any sum nor the rows each block handles, so
 * results do not depend on the choice.  Tuning synchronises the stream once
 * per matrix shape; off, the hand-picked shape is used. */
typedef struct {
  char kernel[16];        /* kernel family ("spmm")                         */
  int64_t rows, cols, nnz; /* the matrix it was tuned on                     */
  char choice[48];        /* the launch shape kept                           */
  double ms_best;         /* median time of the kept shape (ms)              */
  double ms_default;      /* median time of the hand-picked shape (ms)       */
  int32_t candidates;     /* shapes timed                                    */
} rfmls_tune_entry;

rfmls_status rfmls_tune_enable(rfmls_handle *h, int enable);
/* Writes up to cap records [host] of the shapes tuned on this handle; *count
 * [host] receives the number written. */
rfmls_status rfmls_tune_read(const rfmls_handle *h, rfmls_tune_entry *out, int cap, int *count);

/* ---- Kernel tracing (measurement support; not part of the numerical path) ----
 * While enabled, every launch of the library's kernels is bracketed by HIP
 * events on the handle's stream and tagged with the algorithmic bytes moved and
 * flops performed by that launch (what the method must read/write/compute, not
 * what the hardware happened to fetch).  rfmls_trace_read synchronises the
 * stream and returns one aggregate per kernel name, then clears the records. */
typedef struct {
  char name[32];
  int64_t launches;
  double ms;     /* summed event time of all launches        */
  double bytes;  /* summed algorithmic bytes                 */
  double flops;  /* summed algorithmic floating-point ops    */
} rfmls_trace_entry;

rfmls_status rfmls_trace_enable(rfmls_handle *h, int enable);
/* Writes up to cap entries to out [host]; *count [host] receives the number written. */
rfmls_status rfmls_trace_read(rfmls_handle *h, rfmls_trace_entry *out, int cap, int *count);

#ifdef __cplusplus
}
#endif
#endif /* RFMLS_H */
