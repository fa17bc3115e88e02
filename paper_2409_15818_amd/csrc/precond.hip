// Preconditioner construction (Alg. 1 step 3 and the R^{-1} of steps 4-6).
//
// R is read from the upper triangle of the factored sketch, its rows scaled so
// that diag(R) > 0 (QR is unique up to these signs), and checked for numerical
// rank.  The preconditioner is then applied as X = R^{-1}: X is formed once by
// blocked back substitution on the identity, R X = I, block row by block row
// from the bottom:
//     X_I = R_II^{-1} (E_I - R_{I,>I} X_{>I})
// The product R_{I,>I} X_{>I} runs on the matrix cores (split over K, X's zero
// triangle skipped); the 64 x 64 diagonal block is then applied by plain back
// substitution (one thread per column), so every column of X is a backward-
// stable triangular solve and the residual R X - I stays as small as for
// column-by-column substitution.  Every later application of R^{-1} or R^{-T}
// is a triangular matrix-vector product with X, with no sequential dependency
// chain.  X is finally packed into 64 x 64 tiles (upper triangle only) in
// float64 or float32.
#include "common.h"
#include "gemm.h"

namespace rfmls {
namespace {

template <typename T>
__global__ void k_extract_R(const T* __restrict__ SA, int64_t ld, int64_t n,
                            double* __restrict__ R) {
  const int64_t i = blockIdx.x;
  const double sg = (double)SA[i * ld + i] < 0.0 ? -1.0 : 1.0;
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x)
    R[i * n + j] = j >= i ? sg * (double)SA[i * ld + j] : 0.0;
}

// stats[0] = min |r_ii|, stats[1] = max |r_ii|, stats[2] = count of non-finite
__global__ void __launch_bounds__(256) k_diag_stats(const double* __restrict__ R, int64_t n,
                                                    double* __restrict__ stats) {
  __shared__ double smin[256], smax[256], sbad[256];
  double mn = INFINITY, mx = 0.0, bad = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double d = fabs(R[i * n + i]);
    if (!isfinite(d)) bad += 1.0;
    else {
      mn = fmin(mn, d);
      mx = fmax(mx, d);
    }
  }
  smin[threadIdx.x] = mn;
  smax[threadIdx.x] = mx;
  sbad[threadIdx.x] = bad;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + off]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + off]);
      sbad[threadIdx.x] += sbad[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    stats[0] = smin[0];
    stats[1] = smax[0];
    stats[2] = sbad[0];
  }
}

// Block row I of X = R^{-1}: for the 64 columns j = blockIdx.x*64 + t of the
// range [o, n) (o = 64 I), the right-hand side is e_j restricted to block I
// minus sum_z P[z][:, j - o - 64] (the split-K partials of R_{I,>I} X_{>I});
// then R_II x = rhs is solved by back substitution.
__global__ void __launch_bounds__(64) k_inv_blockrow(const double* __restrict__ R, int64_t n,
                                                     int64_t I, const double* __restrict__ P,
                                                     int nz, int64_t ldp, int64_t zstride,
                                                     double* __restrict__ X) {
  __shared__ double Rs[kTile][kTile + 1];
  __shared__ double Xs[kTile][kTile + 1];
  const int64_t o = I * kTile;
  const int b = (int)(n - o < kTile ? n - o : kTile);
  const int t = threadIdx.x;
  for (int i = 0; i < b; ++i) Rs[i][t] = t < b ? R[(o + i) * n + o + t] : 0.0;
  const int64_t j = o + (int64_t)blockIdx.x * kTile + t;
  const bool live = j < n;
  for (int i = 0; i < b; ++i) {
    double v = (live && j == o + i) ? 1.0 : 0.0;
    if (live && j >= o + kTile && nz > 0) {
      const int64_t jc = j - o - kTile;
      double acc = 0.0;
      for (int z = 0; z < nz; ++z) acc += P[(int64_t)z * zstride + (int64_t)i * ldp + jc];
      v -= acc;
    }
    Xs[i][t] = v;
  }
  __syncthreads();
  if (live) {
    for (int i = b - 1; i >= 0; --i) {
      double acc = Xs[i][t];
      for (int k = i + 1; k < b; ++k) acc -= Rs[i][k] * Xs[k][t];
      Xs[i][t] = acc / Rs[i][i];
    }
    for (int i = 0; i < b; ++i) X[(o + i) * n + j] = Xs[i][t];
  }
}

template <typename TS>
__global__ void k_pack_tiles(const double* __restrict__ X, int64_t n, int64_t nt,
                             TS* __restrict__ pk) {
  // blockIdx.x = tile index in packed order; decode (I, J)
  const int64_t t = blockIdx.x;
  int64_t I = 0;
  // rows: tile_index(I, I) <= t < tile_index(I+1, I+1)
  {
    int64_t lo = 0, hi = nt - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) / 2;
      if (tile_index(mid, mid, nt) <= t) lo = mid;
      else hi = mid - 1;
    }
    I = lo;
  }
  const int64_t J = I + (t - tile_index(I, I, nt));
  TS* out = pk + t * (int64_t)(kTile * kTile);
  for (int e = threadIdx.x; e < kTile * kTile; e += blockDim.x) {
    const int r = e / kTile, c = e % kTile;
    const int64_t gi = I * kTile + r, gj = J * kTile + c;
    double v = 0.0;
    if (gi < n && gj < n && gj >= gi) v = X[gi * n + gj];
    out[e] = (TS)v;
  }
}

__global__ void k_unpack_tiles_f64(const double* __restrict__ pk, int64_t n, int64_t nt,
                                   double* __restrict__ X) {
  const int64_t i = blockIdx.x;
  const int64_t I = i / kTile;
  const int r = (int)(i % kTile);
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
    const int64_t J = j / kTile;
    X[i * n + j] = J < I ? 0.0 : (j < i ? 0.0 : pk[tile_index(I, J, nt) * (kTile * kTile) + r * kTile + (j % kTile)]);
  }
}

__global__ void k_unpack_tiles_f32(const float* __restrict__ pk, int64_t n, int64_t nt,
                                   double* __restrict__ X) {
  const int64_t i = blockIdx.x;
  const int64_t I = i / kTile;
  const int r = (int)(i % kTile);
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
    const int64_t J = j / kTile;
    X[i * n + j] = J < I ? 0.0 : (j < i ? 0.0 : (double)pk[tile_index(I, J, nt) * (kTile * kTile) + r * kTile + (j % kTile)]);
  }
}

// X = R^{-1} by blocked back substitution (see the file comment).  P is the
// split-K workspace (nz slices of kTile x (n - 64) doubles).
rfmls_status invert_upper(rfmls_handle* h, const double* R, double* X, double* P, int64_t n,
                          int64_t nt, int64_t kslice) {
  for (int64_t I = nt - 1; I >= 0; --I) {
    const int64_t o = I * kTile;
    const int64_t rest = n - o - kTile;  // columns / rows beyond block I
    int nz = 0;
    const int64_t ldp = rest > 0 ? rest : 1;
    const int64_t zstride = (int64_t)kTile * ldp;
    if (rest > 0) {
      // K slices: only as many as it takes for about two blocks per compute
      // unit (the 64 x rest output has rest / 64 tiles); every slice writes a
      // 64 x rest partial that the block-row kernel reads back
      const int64_t ntn = (rest + kTile - 1) / kTile;
      int64_t nzt = (2 * (int64_t)h->num_cus + ntn - 1) / ntn;
      int64_t ks = (rest + nzt - 1) / nzt;
      if (ks < kslice) ks = kslice;
      ks = (ks + 15) / 16 * 16;
      nz = (int)((rest + ks - 1) / ks);
      GemmArgs<double> g;
      g.M = n - o < kTile ? n - o : kTile;
      g.N = rest;
      g.K = rest;
      g.A = R + o * n + o + kTile;
      g.lda = n;
      g.B = X + (o + kTile) * n + o + kTile;
      g.ldb = n;
      g.C = P;
      g.ldc = ldp;
      g.alpha = 1.0;
      g.beta = 0.0;
      g.b_upper = 1;
      g.ksplit = ks;
      g.c_zstride = zstride;
      // R_{I,>I} (64 x rest) times the upper-triangular X_{>I}: 64 rest^2 flops
      Trace tr(h, "inv_gemm", 8.0 * ((double)kTile * rest + 0.5 * (double)rest * rest + (double)nz * kTile * rest),
               (double)kTile * (double)rest * (double)rest);
      RFMLS_HIP(h, (gemm<double, GemmRole::Inverse>(g, h->stream)));
    }
    {
      Trace tr(h, "inv_blockrow", 8.0 * ((double)nz * kTile * ldp + (double)kTile * (n - o)),
               (double)kTile * kTile * (double)(n - o));
      hipLaunchKernelGGL(k_inv_blockrow, dim3(ceil_div(n - o, kTile)), dim3(kTile), 0, h->stream, R,
                         n, I, (const double*)P, nz, ldp, zstride, X);
    }
    RFMLS_HIP(h, hipGetLastError());
  }
  return RFMLS_OK;
}

}  // namespace

// Shared tail of rfmls_precond / rfmls_precond_import_R: R (normalised,
// float64 row-major n x n) is in P->Rdense.
rfmls_status finish_precond(rfmls_handle* h, rfmls_precond_t* P, int check_rank, double unit) {
  const int64_t n = P->n;
  void* p_stats;
  RFMLS_CHECK(workspace(h, WS_MISC, 64, &p_stats));
  hipLaunchKernelGGL(k_diag_stats, dim3(1), dim3(256), 0, h->stream, P->Rdense, n,
                     (double*)p_stats);
  double stats[3] = {0, 0, 0};
  RFMLS_HIP(h, hipMemcpyAsync(stats, p_stats, sizeof(stats), hipMemcpyDeviceToHost, h->stream));
  RFMLS_HIP(h, hipStreamSynchronize(h->stream));
  if (stats[2] > 0 || stats[0] == 0.0)
    return fail(h, RFMLS_E_RANK, "R has a zero or non-finite diagonal entry");
  if (check_rank && stats[0] <= 16.0 * unit * stats[1])
    return fail(h, RFMLS_E_RANK, "R numerically singular: min|r_ii| = %.3e <= 16 u max|r_ii| = %.3e",
                stats[0], 16.0 * unit * stats[1]);
  void* p_x;
  void* p_w;
  RFMLS_CHECK(workspace(h, WS_TRSM, sizeof(double) * (size_t)n * (size_t)n, &p_x));
  const int64_t kslice = 512;
  const int64_t nzmax = (n + kslice - 1) / kslice;
  RFMLS_CHECK(workspace(h, WS_QR_W, sizeof(double) * (size_t)nzmax * kTile * (size_t)n, &p_w));
  double* X = (double*)p_x;
  RFMLS_CHECK(invert_upper(h, P->Rdense, X, (double*)p_w, n, P->nt, kslice));
  const int64_t ntiles = P->nt * (P->nt + 1) / 2;
  const size_t esz = P->store == RFMLS_F64 ? sizeof(double) : sizeof(float);
  // work tables of the triangular products
  {
    const int C = P->chunk;
    const int64_t nt = P->nt;
    const int64_t maxk = (nt + C - 1) / C;
    std::vector<int2> tr, tc;
    for (int64_t I = 0; I < nt; ++I)
      for (int64_t k = 0; k < (nt - I + C - 1) / C; ++k) tr.push_back(make_int2((int)I, (int)k));
    for (int64_t J = 0; J < nt; ++J)
      for (int64_t k = 0; k < (J + 1 + C - 1) / C; ++k) tc.push_back(make_int2((int)J, (int)k));
    P->ntab = (int64_t)tr.size();
    RFMLS_HIP(h, hipMalloc(&P->tab_row, sizeof(int2) * tr.size()));
    RFMLS_HIP(h, hipMalloc(&P->tab_col, sizeof(int2) * tc.size()));
    RFMLS_HIP(h, hipMemcpy(P->tab_row, tr.data(), sizeof(int2) * tr.size(), hipMemcpyHostToDevice));
    RFMLS_HIP(h, hipMemcpy(P->tab_col, tc.data(), sizeof(int2) * tc.size(), hipMemcpyHostToDevice));
    RFMLS_HIP(h, hipMalloc(&P->part, sizeof(double) * (size_t)(nt * maxk * kTile)));
  }
  RFMLS_HIP(h, hipMalloc(&P->Xpk, esz * (size_t)ntiles * kTile * kTile));
  if (P->store == RFMLS_F64)
    hipLaunchKernelGGL(k_pack_tiles<double>, dim3((unsigned)ntiles), dim3(256), 0, h->stream, X, n,
                       P->nt, (double*)P->Xpk);
  else
    hipLaunchKernelGGL(k_pack_tiles<float>, dim3((unsigned)ntiles), dim3(256), 0, h->stream, X, n,
                       P->nt, (float*)P->Xpk);
  RFMLS_HIP(h, hipGetLastError());
  return RFMLS_OK;
}

rfmls_status unpack_precond(rfmls_handle* h, const rfmls_precond_t* P, double* Xdense) {
  if (P->store == RFMLS_F64)
    hipLaunchKernelGGL(k_unpack_tiles_f64, dim3((unsigned)P->n), dim3(256), 0, h->stream,
                       (const double*)P->Xpk, P->n, P->nt, Xdense);
  else
    hipLaunchKernelGGL(k_unpack_tiles_f32, dim3((unsigned)P->n), dim3(256), 0, h->stream,
                       (const float*)P->Xpk, P->n, P->nt, Xdense);
  RFMLS_HIP(h, hipGetLastError());
  return RFMLS_OK;
}

rfmls_status run_build_precond(rfmls_handle* h, int64_t n, rfmls_dtype qr_dt, const void* SA,
                               int64_t ld, rfmls_dtype store, rfmls_precond_t* P, int check_rank) {
  P->n = n;
  P->nt = (n + kTile - 1) / kTile;
  P->store = store;
  RFMLS_HIP(h, hipMalloc(&P->Rdense, sizeof(double) * (size_t)n * (size_t)n));
  dim3 grid((unsigned)n);
  if (qr_dt == RFMLS_F64)
    hipLaunchKernelGGL(k_extract_R<double>, grid, dim3(256), 0, h->stream, (const double*)SA, ld, n,
                       P->Rdense);
  else
    hipLaunchKernelGGL(k_extract_R<float>, grid, dim3(256), 0, h->stream, (const float*)SA, ld, n,
                       P->Rdense);
  RFMLS_HIP(h, hipGetLastError());
  const double unit = qr_dt == RFMLS_F64 ? 1.1102230246251565e-16 : 5.960464477539063e-08;
  return finish_precond(h, P, check_rank, unit);
}

}  // namespace rfmls
