// C-ABI entry points of librfmls (declared in include/rfmls.h).  Argument
// checking happens here, before anything is enqueued; the numerical work is in
// sketch.hip, csr.hip, qr.hip, precond.hip and lsqr.hip.
#include <cstdarg>
#include <cstring>
#include <new>

#include "common.h"

namespace rfmls {

rfmls_status fail(rfmls_handle* h, rfmls_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (h) h->last_error = buf;
  return st;
}

rfmls_status workspace(rfmls_handle* h, int slot, size_t bytes, void** out) {
  if ((int)h->ws.size() <= slot) h->ws.resize(WS_NUM_SLOTS);
  Workspace& w = h->ws[slot];
  if (w.bytes < bytes) {
    if (w.ptr) {
      hipError_t e = hipStreamSynchronize(h->stream);
      if (e != hipSuccess) return fail(h, RFMLS_E_HIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
      hipFree(w.ptr);
      w.ptr = nullptr;
      w.bytes = 0;
    }
    size_t nb = bytes < 256 ? 256 : bytes;
    hipError_t e = hipMalloc(&w.ptr, nb);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(h, RFMLS_E_NOMEM, "workspace allocation of %zu bytes failed: %s", nb,
                  hipGetErrorString(e));
    }
    w.bytes = nb;
  }
  *out = w.ptr;
  return RFMLS_OK;
}

hipEvent_t trace_event(rfmls_handle* h) {
  hipEvent_t e = nullptr;
  if (!h->event_pool.empty()) {
    e = h->event_pool.back();
    h->event_pool.pop_back();
  } else {
    hipEventCreate(&e);
  }
  return e;
}

static bool csr_ok(const rfmls_csr* A) {
  return A && A->m >= 0 && A->n >= 1 && A->nnz >= 0 && A->row_ptr && (A->nnz == 0 || (A->col && A->val)) &&
         A->nnz < ((int64_t)1 << 31) && A->m < ((int64_t)1 << 31) && A->n < ((int64_t)1 << 31);
}

static rfmls_status set_device(rfmls_handle* h) {
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return fail(h, RFMLS_E_HIP, "hipSetDevice(%d): %s", h->device, hipGetErrorString(e));
  return RFMLS_OK;
}

}  // namespace rfmls

using namespace rfmls;

extern "C" {

void rfmls_default_opts(rfmls_opts* o) {
  if (!o) return;
  o->atol = 1e-10;
  o->btol = 1e-10;
  o->conlim = 1e8;
  o->itmax = 0;
  o->refine = 1;
  o->check_every = 8;
  o->lockstep = 1;
  o->x_init = 0;
  o->graph = 1;
  o->reserved = 0;
}

rfmls_status rfmls_create(rfmls_handle** out, int device, void* stream) {
  if (!out) return RFMLS_E_ARG;
  *out = nullptr;
  rfmls_handle* h = new (std::nothrow) rfmls_handle();
  if (!h) return RFMLS_E_NOMEM;
  h->device = device;
  h->stream = (hipStream_t)stream;
  h->ws.resize(WS_NUM_SLOTS);
  if (hipSetDevice(device) != hipSuccess) {
    delete h;
    return RFMLS_E_HIP;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    delete h;
    return RFMLS_E_HIP;
  }
  h->num_cus = prop.multiProcessorCount;
  if (hipMalloc(&h->barrier, kBarrierWords * sizeof(unsigned)) != hipSuccess ||
      hipMalloc(&h->dev_flags, 64 * sizeof(int)) != hipSuccess ||
      hipHostMalloc(&h->pinned, 4096, hipHostMallocDefault) != hipSuccess) {
    rfmls_destroy(h);
    return RFMLS_E_NOMEM;
  }
  h->pinned_bytes = 4096;
  hipMemset(h->barrier, 0, kBarrierWords * sizeof(unsigned));
  hipMemset(h->dev_flags, 0, 64 * sizeof(int));
  if (noalloc_scratch_init(h) != RFMLS_OK) {
    rfmls_destroy(h);
    return RFMLS_E_HIP;
  }
  *out = h;
  return RFMLS_OK;
}

rfmls_status rfmls_destroy(rfmls_handle* h) {
  if (!h) return RFMLS_OK;
  hipSetDevice(h->device);
  hipStreamSynchronize(h->stream);
  for (auto& r : h->trace_recs) {
    hipEventDestroy(r.beg);
    hipEventDestroy(r.end);
  }
  for (auto e : h->event_pool) hipEventDestroy(e);
  if (h->cap_stream) hipStreamDestroy(h->cap_stream);
  if (h->la_stream) hipStreamDestroy(h->la_stream);
  for (hipEvent_t e : h->la_event)
    if (e) hipEventDestroy(e);
  for (auto& w : h->ws)
    if (w.ptr) hipFree(w.ptr);
  if (h->barrier) hipFree(h->barrier);
  if (h->dev_flags) hipFree(h->dev_flags);
  if (h->pinned) hipHostFree(h->pinned);
  delete h;
  return RFMLS_OK;
}

const char* rfmls_last_error(const rfmls_handle* h) { return h ? h->last_error.c_str() : "null handle"; }

rfmls_status rfmls_transpose(rfmls_handle* h, const rfmls_csr* A, int64_t* rp, int32_t* col,
                             double* val) {
  if (!h) return RFMLS_E_ARG;
  if (!csr_ok(A) || !rp || (A->nnz > 0 && (!col || !val)))
    return fail(h, RFMLS_E_ARG, "rfmls_transpose: invalid matrix or output pointers");
  RFMLS_CHECK(set_device(h));
  return run_transpose(h, A, rp, col, val);
}

rfmls_status rfmls_sketch(rfmls_handle* h, const rfmls_csr* A, int64_t s, uint64_t seed,
                          const int32_t* hash_in, const int8_t* sign_in, int32_t* hash_out,
                          int8_t* sign_out, const double* b, int64_t nrhs, int64_t ldb,
                          double* Sb, rfmls_dtype sa_dtype, void* SA, int64_t ld_sa) {
  if (!h) return RFMLS_E_ARG;
  if (!csr_ok(A)) return fail(h, RFMLS_E_ARG, "rfmls_sketch: invalid CSR matrix");
  if (s < 1 || s >= ((int64_t)1 << 31)) return fail(h, RFMLS_E_ARG, "rfmls_sketch: s must be in [1, 2^31)");
  if (!SA || ld_sa < A->n) return fail(h, RFMLS_E_ARG, "rfmls_sketch: SA null or ld_sa < n");
  if ((hash_in == nullptr) != (sign_in == nullptr))
    return fail(h, RFMLS_E_ARG, "rfmls_sketch: hash_in and sign_in must be given together");
  if (sa_dtype != RFMLS_F64 && sa_dtype != RFMLS_F32)
    return fail(h, RFMLS_E_ARG, "rfmls_sketch: unknown dtype");
  if (Sb && (!b || nrhs < 1 || ldb < A->m))
    return fail(h, RFMLS_E_ARG, "rfmls_sketch: Sb requested with invalid b / nrhs / ldb");
  RFMLS_CHECK(set_device(h));
  const int32_t* hash = hash_in;
  const int8_t* sign = sign_in;
  if (!hash) {
    int32_t* ph = hash_out;
    int8_t* ps = sign_out;
    void* p;
    if (!ph) {
      RFMLS_CHECK(workspace(h, WS_SKETCH_HASH, sizeof(int32_t) * (size_t)(A->m + 1), &p));
      ph = (int32_t*)p;
    }
    if (!ps) {
      RFMLS_CHECK(workspace(h, WS_SKETCH_SIGN, (size_t)(A->m + 1), &p));
      ps = (int8_t*)p;
    }
    RFMLS_CHECK(launch_hash_sign(h, A->m, s, seed, ph, ps));
    hash = ph;
    sign = ps;
  } else {
    if (hash_out && A->m > 0)
      RFMLS_HIP(h, hipMemcpyAsync(hash_out, hash_in, sizeof(int32_t) * A->m, hipMemcpyDeviceToDevice, h->stream));
    if (sign_out && A->m > 0)
      RFMLS_HIP(h, hipMemcpyAsync(sign_out, sign_in, (size_t)A->m, hipMemcpyDeviceToDevice, h->stream));
  }
  return run_sketch(h, A, s, hash, sign, b, nrhs, ldb, Sb, sa_dtype, SA, ld_sa);
}

// Householder QR of the s x ncols matrix SA, then a check of the panel kernel's
// cross-block hand-over (its bounded waits set the device flag on time-out).
static rfmls_status qr_checked(rfmls_handle* h, int64_t s, int64_t ncols, int64_t n_room,
                               rfmls_dtype dt, void* SA, int64_t ld) {
  RFMLS_CHECK(run_qr(h, s, ncols, n_room, dt, SA, ld));
  int flag = 0;
  RFMLS_HIP(h, hipMemcpyAsync(&flag, h->dev_flags, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  RFMLS_HIP(h, hipStreamSynchronize(h->stream));
  if (flag) {
    hipMemset(h->dev_flags, 0, sizeof(int));
    return fail(h, RFMLS_E_HIP, "QR panel: a workgroup did not receive its partner's sums in time");
  }
  return RFMLS_OK;
}

rfmls_status rfmls_precond(rfmls_handle* h, int64_t s, int64_t n, rfmls_dtype qr_dtype,
                           rfmls_dtype r_store, void* SA, int64_t ld_sa, rfmls_precond_t** P_out) {
  if (!h) return RFMLS_E_ARG;
  if (!P_out) return fail(h, RFMLS_E_ARG, "rfmls_precond: P_out is null");
  *P_out = nullptr;
  if (n < 1 || s < n || !SA || ld_sa < n)
    return fail(h, RFMLS_E_ARG, "rfmls_precond: need s >= n >= 1, SA non-null and ld_sa >= n");
  if ((qr_dtype != RFMLS_F64 && qr_dtype != RFMLS_F32) || (r_store != RFMLS_F64 && r_store != RFMLS_F32))
    return fail(h, RFMLS_E_ARG, "rfmls_precond: unknown dtype");
  RFMLS_CHECK(set_device(h));
  RFMLS_CHECK(qr_checked(h, s, n, n, qr_dtype, SA, ld_sa));
  rfmls_precond_t* P = new (std::nothrow) rfmls_precond_t();
  if (!P) return fail(h, RFMLS_E_NOMEM, "rfmls_precond: out of host memory");
  P->device = h->device;
  rfmls_status st = run_build_precond(h, n, qr_dtype, SA, ld_sa, r_store, P, qr_dtype == RFMLS_F64);
  if (st < 0) {
    rfmls_precond_free(P);
    return st;
  }
  *P_out = P;
  return RFMLS_OK;
}

rfmls_status rfmls_precond_x0(rfmls_handle* h, int64_t s, int64_t n, rfmls_dtype qr_dtype,
                              rfmls_dtype r_store, void* SA, int64_t ld_sa, const double* SB,
                              int64_t nrhs, double* X0, int64_t ldx0, rfmls_precond_t** P_out) {
  if (!h) return RFMLS_E_ARG;
  if (!P_out) return fail(h, RFMLS_E_ARG, "rfmls_precond_x0: P_out is null");
  *P_out = nullptr;
  if (n < 1 || nrhs < 1 || s < n + nrhs || !SA || ld_sa < n + nrhs || !SB || !X0 || ldx0 < n)
    return fail(h, RFMLS_E_ARG,
                "rfmls_precond_x0: need nrhs >= 1, s >= n + nrhs, ld_sa >= n + nrhs, ldx0 >= n "
                "and non-null SA, SB, X0");
  if ((qr_dtype != RFMLS_F64 && qr_dtype != RFMLS_F32) || (r_store != RFMLS_F64 && r_store != RFMLS_F32))
    return fail(h, RFMLS_E_ARG, "rfmls_precond_x0: unknown dtype");
  RFMLS_CHECK(set_device(h));
  RFMLS_CHECK(put_sketched_rhs(h, s, n, nrhs, qr_dtype, SA, ld_sa, SB));
  RFMLS_CHECK(qr_checked(h, s, n + nrhs, ld_sa, qr_dtype, SA, ld_sa));
  rfmls_precond_t* P = new (std::nothrow) rfmls_precond_t();
  if (!P) return fail(h, RFMLS_E_NOMEM, "rfmls_precond_x0: out of host memory");
  P->device = h->device;
  rfmls_status st = run_build_precond(h, n, qr_dtype, SA, ld_sa, r_store, P, qr_dtype == RFMLS_F64);
  if (st >= 0) st = sketched_solution(h, P, nrhs, qr_dtype, SA, ld_sa, X0, ldx0);
  if (st < 0) {
    rfmls_precond_free(P);
    return st;
  }
  *P_out = P;
  return RFMLS_OK;
}

rfmls_status rfmls_precond_svd(rfmls_handle* h, int64_t s, int64_t n, rfmls_dtype p_store, void* SA,
                               int64_t ld_sa, double rcond, int max_sweeps, rfmls_precond_t** P_out) {
  if (!h) return RFMLS_E_ARG;
  if (!P_out) return fail(h, RFMLS_E_ARG, "rfmls_precond_svd: P_out is null");
  *P_out = nullptr;
  if (n < 1 || s < n || !SA || ld_sa < n)
    return fail(h, RFMLS_E_ARG, "rfmls_precond_svd: need s >= n >= 1, SA non-null and ld_sa >= n");
  if (n > svd_max_n())
    return fail(h, RFMLS_E_ARG, "rfmls_precond_svd: n = %lld exceeds %lld", (long long)n,
                (long long)svd_max_n());
  if (p_store != RFMLS_F64 && p_store != RFMLS_F32)
    return fail(h, RFMLS_E_ARG, "rfmls_precond_svd: unknown dtype");
  if (!(rcond < 1.0)) return fail(h, RFMLS_E_ARG, "rfmls_precond_svd: rcond must be below 1");
  if (max_sweeps <= 0) max_sweeps = 60;
  RFMLS_CHECK(set_device(h));
  RFMLS_CHECK(qr_checked(h, s, n, n, RFMLS_F64, SA, ld_sa));
  rfmls_precond_t* P = new (std::nothrow) rfmls_precond_t();
  if (!P) return fail(h, RFMLS_E_NOMEM, "rfmls_precond_svd: out of host memory");
  P->device = h->device;
  rfmls_status st = run_build_svd_precond(h, n, (const double*)SA, ld_sa, p_store, rcond, max_sweeps, P);
  if (st < 0) {
    rfmls_precond_free(P);
    return st;
  }
  *P_out = P;
  return st;
}

rfmls_status rfmls_precond_svd_stats(const rfmls_precond_t* P, int64_t* rank, int* sweeps, double* off) {
  if (!P || !P->full) return RFMLS_E_ARG;
  if (rank) *rank = P->rank;
  if (sweeps) *sweeps = P->sweeps;
  if (off) *off = P->off;
  return RFMLS_OK;
}

rfmls_status rfmls_precond_export_P(rfmls_handle* h, const rfmls_precond_t* P, double* X) {
  if (!h) return RFMLS_E_ARG;
  if (!P || !X) return fail(h, RFMLS_E_ARG, "rfmls_precond_export_P: null argument");
  RFMLS_CHECK(set_device(h));
  return unpack_precond(h, P, X);
}

rfmls_status rfmls_precond_export_sigma(rfmls_handle* h, const rfmls_precond_t* P, double* sigma) {
  if (!h) return RFMLS_E_ARG;
  if (!P || !sigma) return fail(h, RFMLS_E_ARG, "rfmls_precond_export_sigma: null argument");
  if (!P->full) return fail(h, RFMLS_E_ARG, "rfmls_precond_export_sigma: not an SVD preconditioner");
  RFMLS_CHECK(set_device(h));
  RFMLS_HIP(h, hipMemcpyAsync(sigma, P->sigma, sizeof(double) * (size_t)P->n, hipMemcpyDeviceToDevice,
                              h->stream));
  return RFMLS_OK;
}

void rfmls_precond_free(rfmls_precond_t* P) {
  if (!P) return;
  hipSetDevice(P->device);
  hipDeviceSynchronize();
  if (P->Xpk) hipFree(P->Xpk);
  if (P->Rdense) hipFree(P->Rdense);
  if (P->tab_row) hipFree(P->tab_row);
  if (P->tab_col) hipFree(P->tab_col);
  if (P->part) hipFree(P->part);
  if (P->sigma) hipFree(P->sigma);
  delete P;
}

int64_t rfmls_precond_n(const rfmls_precond_t* P) { return P ? P->n : -1; }

rfmls_status rfmls_precond_export_R(rfmls_handle* h, const rfmls_precond_t* P, double* R) {
  if (!h) return RFMLS_E_ARG;
  if (!P || !R) return fail(h, RFMLS_E_ARG, "rfmls_precond_export_R: null argument");
  RFMLS_CHECK(set_device(h));
  RFMLS_HIP(h, hipMemcpyAsync(R, P->Rdense, sizeof(double) * (size_t)P->n * (size_t)P->n,
                              hipMemcpyDeviceToDevice, h->stream));
  return RFMLS_OK;
}

rfmls_status rfmls_precond_export_Rinv(rfmls_handle* h, const rfmls_precond_t* P, double* X) {
  if (!h) return RFMLS_E_ARG;
  if (!P || !X) return fail(h, RFMLS_E_ARG, "rfmls_precond_export_Rinv: null argument");
  if (P->full) return fail(h, RFMLS_E_ARG, "rfmls_precond_export_Rinv: an SVD preconditioner holds P, not R^{-1}");
  RFMLS_CHECK(set_device(h));
  return unpack_precond(h, P, X);
}

rfmls_status rfmls_precond_import_R(rfmls_handle* h, int64_t n, const double* R, rfmls_dtype r_store,
                                    rfmls_precond_t** P_out) {
  if (!h) return RFMLS_E_ARG;
  if (!P_out || !R || n < 1 || (r_store != RFMLS_F64 && r_store != RFMLS_F32))
    return fail(h, RFMLS_E_ARG, "rfmls_precond_import_R: invalid argument");
  *P_out = nullptr;
  RFMLS_CHECK(set_device(h));
  rfmls_precond_t* P = new (std::nothrow) rfmls_precond_t();
  if (!P) return fail(h, RFMLS_E_NOMEM, "out of host memory");
  P->device = h->device;
  rfmls_status st = run_build_precond(h, n, RFMLS_F64, R, n, r_store, P, 1);
  if (st < 0) {
    rfmls_precond_free(P);
    return st;
  }
  *P_out = P;
  return RFMLS_OK;
}

static rfmls_status check_solve_args(rfmls_handle* h, const rfmls_csr* A, const rfmls_csr* AT,
                                     const rfmls_precond_t* P, const rfmls_opts* o) {
  if (!csr_ok(A) || !csr_ok(AT)) return fail(h, RFMLS_E_ARG, "invalid CSR matrix A or A^T");
  if (AT->m != A->n || AT->n != A->m || AT->nnz != A->nnz)
    return fail(h, RFMLS_E_ARG, "A^T does not match A (%lld x %lld vs %lld x %lld)", (long long)A->m,
                (long long)A->n, (long long)AT->m, (long long)AT->n);
  if (A->m < 1) return fail(h, RFMLS_E_ARG, "A has no rows");
  if (!P || P->n != A->n) return fail(h, RFMLS_E_ARG, "preconditioner size does not match A");
  if (!o) return fail(h, RFMLS_E_ARG, "options are null");
  if (!(o->atol >= 0) || !(o->btol >= 0) || o->refine < 0 || o->refine > 16)
    return fail(h, RFMLS_E_ARG, "invalid LSQR options");
  return RFMLS_OK;
}

rfmls_status rfmls_solve(rfmls_handle* h, const rfmls_csr* A, const rfmls_csr* AT,
                         const rfmls_precond_t* P, const double* B, int64_t ldb, int64_t nrhs,
                         double* X, int64_t ldx, double* Rout, int64_t ldr, const rfmls_opts* opts,
                         rfmls_info* info) {
  if (!h) return RFMLS_E_ARG;
  rfmls_opts def;
  rfmls_default_opts(&def);
  const rfmls_opts* o = opts ? opts : &def;
  RFMLS_CHECK(check_solve_args(h, A, AT, P, o));
  if (nrhs < 0 || (nrhs > 0 && (!B || !X)) || ldb < A->m || ldx < A->n || (Rout && ldr < A->m))
    return fail(h, RFMLS_E_ARG, "rfmls_solve: invalid B / X / leading dimensions");
  if (nrhs == 0) return RFMLS_OK;
  RFMLS_CHECK(set_device(h));
  if (o->lockstep && nrhs > 1)
    return run_solve_block(h, A, AT, P, B, ldb, nrhs, X, ldx, Rout, ldr, o, info);
  return run_solve(h, A, AT, P, B, ldb, nrhs, X, ldx, Rout, ldr, o, info);
}

rfmls_status rfmls_solve_noalloc(rfmls_handle* h, const rfmls_csr* A, const rfmls_csr* AT,
                                 const rfmls_precond_t* P, const double* B, int64_t ldb, int64_t nrhs,
                                 double* X, int64_t ldx, double* Rout, int64_t ldr,
                                 const rfmls_opts* opts, rfmls_info* info) {
  if (!h) return RFMLS_E_ARG;
  rfmls_opts def;
  rfmls_default_opts(&def);
  const rfmls_opts* o = opts ? opts : &def;
  RFMLS_CHECK(check_solve_args(h, A, AT, P, o));
  if (nrhs < 0 || (nrhs > 0 && (!B || !X)) || ldb < A->m || ldx < A->n || (Rout && ldr < A->m))
    return fail(h, RFMLS_E_ARG, "rfmls_solve_noalloc: invalid B / X / leading dimensions");
  if (noalloc_needed_bytes(A->m, A->n) > noalloc_scratch_bytes())
    return fail(h, RFMLS_E_ARG, "rfmls_solve_noalloc: m = %lld, n = %lld need %lld bytes of scratch, above "
                "the %lld-byte limit", (long long)A->m, (long long)A->n,
                (long long)noalloc_needed_bytes(A->m, A->n), (long long)noalloc_scratch_bytes());
  if (nrhs == 0) return RFMLS_OK;
  RFMLS_CHECK(set_device(h));
  return run_solve_noalloc(h, A, AT, P, B, ldb, nrhs, X, ldx, Rout, ldr, o, info);
}

int64_t rfmls_noalloc_scratch_bytes(void) { return noalloc_scratch_bytes(); }

rfmls_status rfmls_precond_stats(const rfmls_precond_t* P, double* pivot_ratio, double* rho_min) {
  if (!P) return RFMLS_E_ARG;
  if (pivot_ratio) *pivot_ratio = P->pivot_ratio;
  if (rho_min) *rho_min = P->rho_min;
  return RFMLS_OK;
}

rfmls_status rfmls_form_B(rfmls_handle* h, const rfmls_csr* A, const rfmls_precond_t* P, double* Bmat,
                          int64_t ld_bmat) {
  if (!h) return RFMLS_E_ARG;
  if (!csr_ok(A) || A->m < 1) return fail(h, RFMLS_E_ARG, "rfmls_form_B: invalid CSR matrix");
  if (!P || P->n != A->n) return fail(h, RFMLS_E_ARG, "rfmls_form_B: preconditioner size does not match A");
  if (!Bmat || ld_bmat < A->n) return fail(h, RFMLS_E_ARG, "rfmls_form_B: Bmat null or ld_bmat < n");
  RFMLS_CHECK(set_device(h));
  return run_form_B(h, A, P, Bmat, ld_bmat);
}

rfmls_status rfmls_solve_explicit(rfmls_handle* h, const rfmls_csr* A, const rfmls_csr* AT,
                                  const rfmls_precond_t* P, const double* Bmat, int64_t ld_bmat,
                                  const double* B, int64_t ldb, int64_t nrhs, double* X, int64_t ldx,
                                  double* Rout, int64_t ldr, const rfmls_opts* opts, rfmls_info* info) {
  if (!h) return RFMLS_E_ARG;
  rfmls_opts def;
  rfmls_default_opts(&def);
  const rfmls_opts* o = opts ? opts : &def;
  RFMLS_CHECK(check_solve_args(h, A, AT, P, o));
  if (!Bmat || ld_bmat < A->n) return fail(h, RFMLS_E_ARG, "rfmls_solve_explicit: Bmat null or ld_bmat < n");
  if (nrhs < 0 || (nrhs > 0 && (!B || !X)) || ldb < A->m || ldx < A->n || (Rout && ldr < A->m))
    return fail(h, RFMLS_E_ARG, "rfmls_solve_explicit: invalid B / X / leading dimensions");
  if (nrhs == 0) return RFMLS_OK;
  RFMLS_CHECK(set_device(h));
  return run_solve_explicit(h, A, AT, P, Bmat, ld_bmat, B, ldb, nrhs, X, ldx, Rout, ldr, o, info);
}

rfmls_status rfmls_solve_backward(rfmls_handle* h, const rfmls_csr* A, const rfmls_csr* AT,
                                  const rfmls_precond_t* P, const double* X, int64_t ldx,
                                  const double* Rres, int64_t ldr, const double* G, int64_t ldg,
                                  int64_t nrhs, double* dB, int64_t lddb, double* dAval,
                                  const rfmls_opts* opts, rfmls_info* info) {
  if (!h) return RFMLS_E_ARG;
  rfmls_opts def;
  rfmls_default_opts(&def);
  const rfmls_opts* o = opts ? opts : &def;
  RFMLS_CHECK(check_solve_args(h, A, AT, P, o));
  if (nrhs < 0 || (nrhs > 0 && !G) || ldg < A->n || (dB && lddb < A->m) ||
      (dAval && (!X || !Rres || ldx < A->n || ldr < A->m)))
    return fail(h, RFMLS_E_ARG, "rfmls_solve_backward: invalid arguments");
  if (P->full && P->rank < P->n)
    return fail(h, RFMLS_E_ARG, "rfmls_solve_backward: the SVD preconditioner is truncated (rank %lld < n = %lld)",
                (long long)P->rank, (long long)P->n);
  if (nrhs == 0) return RFMLS_OK;
  RFMLS_CHECK(set_device(h));
  if (o->lockstep && nrhs > 1)
    return run_backward_block(h, A, AT, P, X, ldx, Rres, ldr, G, ldg, nrhs, dB, lddb, dAval, o, info);
  return run_backward(h, A, AT, P, X, ldx, Rres, ldr, G, ldg, nrhs, dB, lddb, dAval, o, info);
}

rfmls_status rfmls_qr_panel_mode(rfmls_handle* h, int mode) {
  if (!h || mode < 0 || mode > 3) return RFMLS_E_ARG;
  h->qr_panel = mode;
  return RFMLS_OK;
}

rfmls_status rfmls_qr_lookahead(rfmls_handle* h, int enable) {
  if (!h) return RFMLS_E_ARG;
  h->qr_lookahead = enable != 0;
  return RFMLS_OK;
}

rfmls_status rfmls_tune_enable(rfmls_handle* h, int enable) {
  if (!h) return RFMLS_E_ARG;
  h->tune = enable != 0;
  return RFMLS_OK;
}

rfmls_status rfmls_tune_read(const rfmls_handle* h, rfmls_tune_entry* out, int cap, int* count) {
  if (!h || (!out && cap > 0) || !count) return RFMLS_E_ARG;
  int k = 0;
  for (const TuneRec& t : h->tuned) {
    if (k >= cap) break;
    rfmls_tune_entry& e = out[k++];
    memset(&e, 0, sizeof(e));
    strncpy(e.kernel, t.kernel, sizeof(e.kernel) - 1);
    e.rows = t.rows;
    e.cols = t.cols;
    e.nnz = t.nnz;
    strncpy(e.choice, t.desc, sizeof(e.choice) - 1);
    e.ms_best = t.ms_best;
    e.ms_default = t.ms_default;
    e.candidates = t.candidates;
  }
  *count = k;
  return RFMLS_OK;
}

rfmls_status rfmls_trace_enable(rfmls_handle* h, int enable) {
  if (!h) return RFMLS_E_ARG;
  h->trace = enable != 0;
  return RFMLS_OK;
}

rfmls_status rfmls_trace_read(rfmls_handle* h, rfmls_trace_entry* out, int cap, int* count) {
  if (!h || (!out && cap > 0) || !count) return RFMLS_E_ARG;
  RFMLS_CHECK(set_device(h));
  RFMLS_HIP(h, hipStreamSynchronize(h->stream));
  std::vector<rfmls_trace_entry> agg;
  for (auto& r : h->trace_recs) {
    float ms = 0.f;
    hipEventElapsedTime(&ms, r.beg, r.end);
    size_t k = 0;
    for (; k < agg.size(); ++k)
      if (strncmp(agg[k].name, r.name, sizeof(agg[k].name)) == 0) break;
    if (k == agg.size()) {
      rfmls_trace_entry e{};
      strncpy(e.name, r.name, sizeof(e.name) - 1);
      agg.push_back(e);
    }
    agg[k].launches += 1;
    agg[k].ms += ms;
    agg[k].bytes += r.bytes;
    agg[k].flops += r.flops;
    h->event_pool.push_back(r.beg);
    h->event_pool.push_back(r.end);
  }
  h->trace_recs.clear();
  int n = 0;
  for (size_t k = 0; k < agg.size() && n < cap; ++k) out[n++] = agg[k];
  *count = n;
  return RFMLS_OK;
}

}  // extern "C"
