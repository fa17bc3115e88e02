// Deterministic transpose of a CSR matrix (A^T as CSR, used for the products
// A^T u of Alg. 1 step 5).  A stable counting sort by column: rows are cut
// into chunks; per chunk and column the entries are counted, the counts are
// scanned over chunks (giving every (chunk, column) pair its first slot), and
// each chunk then walks its rows in order, so every row of A^T lists its
// entries in ascending row-of-A order.  No floating-point arithmetic.
#include "common.h"

namespace rfmls {
namespace {

constexpr int kColPass = 16384;  // columns handled per LDS pass

__global__ void __launch_bounds__(256)
    k_tr_hist(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col, int64_t m,
              int64_t n, int64_t rc, int32_t* __restrict__ hist) {
  __shared__ int32_t cnt[kColPass];
  const int64_t k = blockIdx.x;
  const int64_t rlo = k * rc, rhi = rlo + rc < m ? rlo + rc : m;
  const int64_t elo = row_ptr[rlo], ehi = row_ptr[rhi];
  for (int64_t c0 = 0; c0 < n; c0 += kColPass) {
    const int64_t cw = n - c0 < kColPass ? n - c0 : kColPass;
    for (int t = threadIdx.x; t < cw; t += 256) cnt[t] = 0;
    __syncthreads();
    for (int64_t e = elo + threadIdx.x; e < ehi; e += 256) {
      const int64_t c = (int64_t)col[e] - c0;
      if (c >= 0 && c < cw) atomicAdd(&cnt[c], 1);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < cw; t += 256) hist[k * n + c0 + t] = cnt[t];
    __syncthreads();
  }
}

// hist[k][c] <- exclusive prefix over k; count[c] <- total
__global__ void k_tr_colscan(int32_t* __restrict__ hist, int64_t nchunk, int64_t n,
                             int32_t* __restrict__ count) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  int32_t run = 0;
  for (int64_t k = 0; k < nchunk; ++k) {
    const int32_t v = hist[k * n + c];
    hist[k * n + c] = run;
    run += v;
  }
  count[c] = run;
}

__global__ void __launch_bounds__(256)
    k_tr_fill(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
              const double* __restrict__ val, int64_t m, int64_t n, int64_t rc,
              const int32_t* __restrict__ hist, const int64_t* __restrict__ at_ptr,
              int32_t* __restrict__ at_col, double* __restrict__ at_val) {
  __shared__ int32_t cur[kColPass];
  const int64_t k = blockIdx.x;
  const int64_t rlo = k * rc, rhi = rlo + rc < m ? rlo + rc : m;
  for (int64_t c0 = 0; c0 < n; c0 += kColPass) {
    const int64_t cw = n - c0 < kColPass ? n - c0 : kColPass;
    for (int t = threadIdx.x; t < cw; t += 256) cur[t] = hist[k * n + c0 + t];
    __syncthreads();
    for (int64_t i = rlo; i < rhi; ++i) {
      const int64_t lo = row_ptr[i], hi = row_ptr[i + 1];
      for (int64_t e = lo + threadIdx.x; e < hi; e += 256) {
        const int64_t c = (int64_t)col[e] - c0;
        if (c >= 0 && c < cw) {
          const int64_t pos = at_ptr[c0 + c] + cur[c];
          cur[c] += 1;  // columns are unique within a row: no two threads share c
          at_col[pos] = (int32_t)i;
          at_val[pos] = val[e];
        }
      }
      __syncthreads();
    }
  }
}

}  // namespace

rfmls_status run_transpose(rfmls_handle* h, const rfmls_csr* A, int64_t* rp, int32_t* at_col,
                           double* at_val) {
  const int64_t m = A->m, n = A->n;
  int64_t rc = (m + 1023) / 1024;
  if (rc < 32) rc = 32;
  const int64_t nchunk = m > 0 ? (m + rc - 1) / rc : 0;
  void *p_hist, *p_count;
  RFMLS_CHECK(workspace(h, WS_TRANSPOSE, sizeof(int32_t) * (size_t)(nchunk > 0 ? nchunk : 1) * (size_t)n, &p_hist));
  RFMLS_CHECK(workspace(h, WS_SKETCH_COUNT, sizeof(int32_t) * (size_t)(n + 1), &p_count));
  int32_t* hist = (int32_t*)p_hist;
  int32_t* count = (int32_t*)p_count;
  Trace tr(h, "transpose", 2.0 * (12.0 * (double)A->nnz) + 8.0 * (double)(m + n + 2), 0.0);
  if (nchunk > 0) {
    hipLaunchKernelGGL(k_tr_hist, dim3((unsigned)nchunk), dim3(256), 0, h->stream, A->row_ptr,
                       A->col, m, n, rc, hist);
    hipLaunchKernelGGL(k_tr_colscan, dim3(ceil_div(n, 256)), dim3(256), 0, h->stream, hist, nchunk,
                       n, count);
  } else {
    RFMLS_HIP(h, hipMemsetAsync(count, 0, sizeof(int32_t) * (size_t)n, h->stream));
  }
  RFMLS_HIP(h, hipGetLastError());
  RFMLS_CHECK(scan_counts(h, count, n, rp));
  if (nchunk > 0) {
    hipLaunchKernelGGL(k_tr_fill, dim3((unsigned)nchunk), dim3(256), 0, h->stream, A->row_ptr,
                       A->col, A->val, m, n, rc, hist, rp, at_col, at_val);
    RFMLS_HIP(h, hipGetLastError());
  }
  return RFMLS_OK;
}

}  // namespace rfmls
