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

// Remark 3.1: the sketched right-hand sides become extra columns of the
// factored matrix, element (i, n + k) = SB[k s + i] in the QR's precision.
template <typename T>
__global__ void k_put_rhs(T* __restrict__ SA, int64_t ld, int64_t s, int64_t n, int64_t nrhs,
                          const double* __restrict__ SB) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < s * nrhs;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = e / s, i = e % s;
    SA[i * ld + n + k] = (T)SB[k * s + i];
  }
}

// y0_k = Q^T (S b_k): the top n entries of the extra columns after the QR,
// with the row signs that make diag(R) > 0 (as in k_extract_R).
template <typename T>
__global__ void k_take_y0(const T* __restrict__ SA, int64_t ld, int64_t n, int64_t nrhs,
                          double* __restrict__ Y0) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * nrhs;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = e / n, i = e % n;
    const double sg = (double)SA[i * ld + i] < 0.0 ? -1.0 : 1.0;
    Y0[k * n + i] = sg * (double)SA[i * ld + n + k];
  }
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

// Column-relative pivots rho_j = |r_jj| / ||R[:, j]|| (||R[:, j]|| = ||SA[:, j]||):
// the distance of column j of SA from the span of the columns before it,
// relative to its length.  k_col_sumsq: block (x, z) takes 64 columns and the
// z-th chunk of kRhoRows rows; its four wavefronts sum every fourth row (a
// row's 64 loads are coalesced, four rows in flight per wavefront) and the
// four partial sums are added in a fixed order into ss[z][j].  k_col_rho then
// adds the chunks in order and writes per-block minima into part[blockIdx.x].
constexpr int64_t kRhoRows = 512;
__global__ void __launch_bounds__(256) k_col_sumsq(const double* __restrict__ R, int64_t n,
                                                   double* __restrict__ ss) {
  __shared__ double psum[4][64];
  const int c = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * 64 + c;
  const int64_t i0 = (int64_t)blockIdx.y * kRhoRows;
  double acc = 0.0;
  if (j < n) {
    // rows i0 + q, i0 + q + 4, ... up to min(j, i0 + kRhoRows - 1)
    const int64_t iend = j + 1 < i0 + kRhoRows ? j + 1 : i0 + kRhoRows;
    int64_t i = i0 + q;
    for (; i + 12 < iend; i += 16) {
      const double v0 = R[i * n + j], v1 = R[(i + 4) * n + j], v2 = R[(i + 8) * n + j], v3 = R[(i + 12) * n + j];
      acc = fma(v0, v0, acc);
      acc = fma(v1, v1, acc);
      acc = fma(v2, v2, acc);
      acc = fma(v3, v3, acc);
    }
    for (; i < iend; i += 4) {
      const double v = R[i * n + j];
      acc = fma(v, v, acc);
    }
  }
  psum[q][c] = acc;
  __syncthreads();
  if (q == 0 && j < n) ss[(int64_t)blockIdx.y * n + j] = (psum[0][c] + psum[1][c]) + (psum[2][c] + psum[3][c]);
}

__global__ void __launch_bounds__(64) k_col_rho(const double* __restrict__ R, int64_t n,
                                                const double* __restrict__ ss, double* __restrict__ part) {
  const int c = threadIdx.x;
  const int64_t j = (int64_t)blockIdx.x * 64 + c;
  double rho = INFINITY;
  if (j < n) {
    double t = 0.0;
    const int64_t nz = j / kRhoRows + 1;  // the chunks holding rows 0 .. j
    for (int64_t z = 0; z < nz; ++z) t += ss[z * n + j];
    rho = t > 0.0 ? fabs(R[j * n + j]) / sqrt(t) : 0.0;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) rho = fmin(rho, __shfl_xor(rho, off, 64));
  if (c == 0) part[blockIdx.x] = rho;
}

__global__ void __launch_bounds__(256) k_min_partials(const double* __restrict__ part, int np,
                                                      double* __restrict__ out) {
  __shared__ double smin[256];
  double mn = INFINITY;
  for (int i = threadIdx.x; i < np; i += 256) mn = fmin(mn, part[i]);
  smin[threadIdx.x] = mn;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = smin[0];
}

// Block row I of X = R^{-1} (rows [o, o + b), o = 64 I), columns j in [o, n).
// Every column j >= o of the block row is written, so the diagonal block's
// lower triangle gets the exact zeros back substitution leaves there (0 / r_ii
// below a unit right-hand side); the GEMMs above read those as stored.
// Right-hand side: e_j restricted to the block row, minus R_{I,>I} X_{>I}, which
// arrives in two parts (see invert_upper): nzn split-K slices of Pn (each
// b x (n - o - 64), stride zsn) from the rows of X solved earlier inside the
// same outer block, summed in slice order, and nzf split-K
// slices of Pf (rows roff .. roff + b of a (rows of the outer block) x (n - e2)
// partial) from the rows beyond the outer block, for columns j >= e2.  Then
// R_II x = rhs by back substitution, column-oriented (x_i = rhs_i * (1 / r_ii),
// the 64 reciprocals formed once, then every rhs_k, k < i, is updated at once).  Four neighbouring lanes share a
// column, each holding 16 of its 64 rows in registers; x_i is passed from the
// lane holding row i to the other three by a DPP quad broadcast.  Every element
// sees the same operations in the same order as a one-lane-per-column
// substitution, at a quarter of the registers (more wavefronts in flight).
constexpr int kInvCols = 64;               // columns per block
constexpr int kInvLanes = 4;               // lanes per column
constexpr int kInvRows = kTile / kInvLanes;  // rows per lane

// value of lane (lane & ~3) + Q of each quad, for every lane of the quad
template <int Q>
__device__ __forceinline__ double quad_bcast(double v) {
  constexpr int kCtrl = Q | (Q << 2) | (Q << 4) | (Q << 6);  // DPP quad_perm(Q, Q, Q, Q)
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, kCtrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), kCtrl, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// T: storage of R, the partials and X (float64, or float32 for a factor
// computed and stored in float32); the substitution runs in float64.
template <typename T>
__global__ void __launch_bounds__(kInvCols * kInvLanes)
    k_inv_blockrow(const T* __restrict__ R, int64_t n, int64_t I, const T* __restrict__ Pn,
                   int64_t ldn, int nzn, int64_t zsn, const T* __restrict__ Pf, int nzf, int64_t ldf, int64_t zsf,
                   int64_t roff, int64_t e2, T* __restrict__ X) {
  __shared__ double Rs[kTile][kTile + 1];
  __shared__ double rinv[kTile];  // 1 / r_ii, formed once so no division sits on the chain
  const int64_t o = I * kTile;
  const int b = (int)(n - o < kTile ? n - o : kTile);
  const int t = threadIdx.x;
  // Every load below reads a clamped, in-range address unconditionally and the
  // unused values are dropped by a select, so all of a thread's loads are in
  // flight together (a conditional load per element made the compiler wait for
  // each one before the next: 16 serial memory round trips).
  constexpr int kLoads = kTile * kTile / (kInvCols * kInvLanes);
  double rt[kLoads];
#pragma unroll
  for (int s = 0; s < kLoads; ++s) {
    const int e = t + s * kInvCols * kInvLanes;
    const int i = e / kTile, k = e % kTile;
    rt[s] = (double)R[(o + min(i, b - 1)) * n + o + min(k, b - 1)];
  }
  const double rdiag = (double)R[(o + min(t % kTile, b - 1)) * (n + 1)];
  const int q = t % kInvLanes;  // this lane holds rows q*16 .. q*16 + 15
  const int r0 = q * kInvRows;
  const int64_t j = o + (int64_t)blockIdx.x * kInvCols + t / kInvLanes;
  const bool live = j < n;
  double v[kInvRows];
#pragma unroll
  for (int l = 0; l < kInvRows; ++l) v[l] = (live && j == o + r0 + l) ? 1.0 : 0.0;
  if (live && j >= o + kTile && Pn) {
    const int64_t jc = j - o - kTile;
    double pn[kInvRows];
#pragma unroll
    for (int l = 0; l < kInvRows; ++l) pn[l] = (double)Pn[(int64_t)min(r0 + l, b - 1) * ldn + jc];
    for (int z = 1; z < nzn; ++z) {
      double pz[kInvRows];
#pragma unroll
      for (int l = 0; l < kInvRows; ++l) pz[l] = (double)Pn[(int64_t)z * zsn + (int64_t)min(r0 + l, b - 1) * ldn + jc];
#pragma unroll
      for (int l = 0; l < kInvRows; ++l) pn[l] += pz[l];
    }
#pragma unroll
    for (int l = 0; l < kInvRows; ++l) v[l] = r0 + l < b ? -pn[l] : 0.0;
  }
  // far partials exist only for outer blocks that end before n, whose block
  // rows are all full (b == kTile), so no row test is needed here
  if (live && j >= e2 && b == kTile) {
    const int64_t jf = j - e2;
    for (int z = 0; z < nzf; ++z) {
      const T* Pz = Pf + (int64_t)z * zsf + roff * ldf + jf;
      double pz[kInvRows];
#pragma unroll
      for (int l = 0; l < kInvRows; ++l) pz[l] = (double)Pz[(int64_t)(r0 + l) * ldf];
#pragma unroll
      for (int l = 0; l < kInvRows; ++l) v[l] -= pz[l];
    }
  }
#pragma unroll
  for (int s = 0; s < kLoads; ++s) {
    const int e = t + s * kInvCols * kInvLanes;
    const int i = e / kTile, k = e % kTile;
    // zeros below the diagonal: the update loop below then needs no per-row test
    Rs[i][k] = (i < b && k < b && k >= i) ? rt[s] : (i == k ? 1.0 : 0.0);
  }
  if (t < kTile) rinv[t] = t < b ? 1.0 / rdiag : 1.0;
  __syncthreads();
  // Rows >= b are the identity with v = 0 and stay 0.  The 64 rows go in four
  // groups of 16 from the bottom.  Group qi: the lanes holding it (q == qi)
  // solve its 16 rows among themselves, x_i = v_i / r_ii and v_k -= r_ki x_i for
  // the rows k < i of the group, a chain of 16 steps inside one lane (every
  // lane runs it on a copy; only the owners keep the result); the 16 x_i then
  // go to the whole quad by DPP, and the lanes holding rows above the group
  // (q < qi) apply them, i from high to low.  Every element sees the same
  // updates in the same order as a one-lane-per-column substitution.
#pragma unroll
  for (int qi = kInvLanes - 1; qi >= 0; --qi) {
    const int g0 = qi * kInvRows;
    double w[kInvRows];
#pragma unroll
    for (int l = 0; l < kInvRows; ++l) w[l] = v[l];
#pragma unroll
    for (int li = kInvRows - 1; li >= 0; --li) {
      const double xi = w[li] * rinv[g0 + li];
#pragma unroll
      for (int l = 0; l < li; ++l) w[l] -= Rs[g0 + l][g0 + li] * xi;
      w[li] = xi;
    }
    double xb[kInvRows];
#pragma unroll
    for (int li = 0; li < kInvRows; ++li)
      xb[li] = qi == 0 ? quad_bcast<0>(w[li]) : qi == 1 ? quad_bcast<1>(w[li]) : qi == 2 ? quad_bcast<2>(w[li])
                                                                                          : quad_bcast<3>(w[li]);
    if (q == qi) {
#pragma unroll
      for (int l = 0; l < kInvRows; ++l) v[l] = w[l];
    } else if (q < qi) {
#pragma unroll
      for (int li = kInvRows - 1; li >= 0; --li)
#pragma unroll
        for (int l = 0; l < kInvRows; ++l) v[l] -= Rs[r0 + l][g0 + li] * xb[li];
    }
  }
  if (live) {
#pragma unroll
    for (int l = 0; l < kInvRows; ++l)
      if (r0 + l < b) X[(o + r0 + l) * n + j] = (T)v[l];
  }
}

template <typename TS, typename TX = double>
__global__ void k_pack_tiles(const TX* __restrict__ X, int64_t n, int64_t nt, int full,
                             TS* __restrict__ pk) {
  // blockIdx.x = tile index in packed order; decode (I, J)
  const int64_t t = blockIdx.x;
  int64_t I = 0, J = 0;
  if (full) {
    I = t / nt;
    J = t % nt;
  } else {
    // rows: tile_index(I, I) <= t < tile_index(I+1, I+1)
    int64_t lo = 0, hi = nt - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) / 2;
      if (tile_index(mid, mid, nt) <= t) lo = mid;
      else hi = mid - 1;
    }
    I = lo;
    J = I + (t - tile_index(I, I, nt));
  }
  TS* out = pk + t * (int64_t)(kTile * kTile);
  for (int e = threadIdx.x; e < kTile * kTile; e += blockDim.x) {
    const int r = e / kTile, c = e % kTile;
    const int64_t gi = I * kTile + r, gj = J * kTile + c;
    double v = 0.0;
    if (gi < n && gj < n && (full || gj >= gi)) v = (double)X[gi * n + gj];
    out[e] = (TS)v;
  }
}

template <typename TS>
__global__ void k_unpack_tiles(const TS* __restrict__ pk, int64_t n, int64_t nt, int full,
                               double* __restrict__ X) {
  const int64_t i = blockIdx.x;
  const int64_t I = i / kTile;
  const int r = (int)(i % kTile);
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
    const int64_t J = j / kTile;
    X[i * n + j] = (!full && j < i) ? 0.0 : (double)pk[ptile(I, J, nt, full) * (kTile * kTile) + r * kTile + (j % kTile)];
  }
}

// X = R^{-1} by blocked back substitution, two levels: outer blocks of
// kInvOuter rows (kInvTiles tiles), inner block rows of 64.  For block row I
// inside the outer block [o2, e2):
//   R_{I,>I} X_{>I} = R_{I,(I,e2)} X_{(I,e2)}  (near: K < kInvOuter, one GEMM
//                                                 per block row)
//                   + R_{I,>=e2} X_{>=e2}        (far: computed once per outer
//                                                 block for all its rows)
// so the dominant n^3/3 flops run as kInvOuter-row GEMMs, each panel of X read
// by kInvTiles tile rows.  Measured (total of the three kernels, 12,800 /
// 25,600 columns): 40 / 188 ms at 4 tiles, 39 / 180 ms at 16, 42 / 180 ms at 32
// (the near products grow as fast as the far one shrinks).  Pf holds up to 4
// split-K slices of (e2 - o2) x (n - e2); Pn up to 2 split-K slices of 64 x n
// (the near product has one tile row, so its K range is split in two where
// its output tiles alone give fewer than about two blocks per compute unit;
// measured against 1 and 4 slices: 340 vs 342 / 342 ms for QR + inverse on
// the 8x8-box system, 696 vs 699 / 695 ms on the 4^3-box float32 one, since
// every slice is one more memory round trip for the block-row kernel).
constexpr int64_t kInvTiles = 16;
constexpr int64_t kInvOuter = kInvTiles * kTile;

template <typename T>
rfmls_status invert_upper(rfmls_handle* h, const T* R, T* X, T* Pf, T* Pn, int64_t n, int64_t nt,
                          int64_t kslice) {
  const int64_t nt2 = (nt + kInvTiles - 1) / kInvTiles;
  for (int64_t I2 = nt2 - 1; I2 >= 0; --I2) {
    const int64_t o2 = I2 * kInvOuter;
    const int64_t e2 = o2 + kInvOuter < n ? o2 + kInvOuter : n;
    const int64_t far = n - e2;
    int nzf = 0;
    const int64_t ldf = far > 0 ? far : 1;
    const int64_t zsf = (e2 - o2) * ldf;
    if (far > 0) {
      // K slices only where the (e2 - o2) x far output has too few tiles for
      // about two blocks per compute unit (at most 4 slices, each >= kslice)
      const int64_t tiles = ((e2 - o2 + kTile - 1) / kTile) * ((far + kTile - 1) / kTile);
      int64_t nzt = (2 * (int64_t)h->num_cus + tiles - 1) / tiles;
      int64_t ks = (far + nzt - 1) / nzt;
      if (ks < kslice) ks = kslice;
      if ((far + ks - 1) / ks > 4) ks = (far + 3) / 4;
      ks = (ks + 15) / 16 * 16;
      nzf = (int)((far + ks - 1) / ks);
      GemmArgs<T> g;
      g.M = e2 - o2;
      g.N = far;
      g.K = far;
      g.A = R + o2 * n + e2;
      g.lda = n;
      g.B = X + e2 * n + e2;
      g.ldb = n;
      g.C = Pf;
      g.ldc = ldf;
      g.b_upper = 1;
      g.b_lower_zero = 1;  // k_inv_blockrow wrote the diagonal blocks' lower triangles as zeros
      g.ksplit = ks;
      // the kInvTiles row tiles that read one column strip of X run together,
      // so the strip comes from HBM once: 46 -> 60 TFLOP/s at 24,576 columns
      g.tile_order = 1;
      g.c_zstride = zsf;
      Trace tr(h, "inv_gemm", (double)sizeof(T) * ((double)(e2 - o2) * far + 0.5 * (double)far * far + (double)nzf * (e2 - o2) * far),
               (double)(e2 - o2) * (double)far * (double)far);
      RFMLS_HIP(h, (gemm_clean<T, GemmRole::Inverse>(g, h->stream)));
    }
    for (int64_t I = (e2 - 1) / kTile; I >= I2 * kInvTiles; --I) {
      const int64_t o = I * kTile;
      const int64_t b = n - o < kTile ? n - o : kTile;
      const int64_t kn = e2 - o - b;  // solved rows of this outer block below row block I
      const int64_t ldn = n - o - kTile > 0 ? n - o - kTile : 1;
      int nzn = 0;
      const int64_t zsn = kTile * ldn;
      if (kn > 0) {
        GemmArgs<T> g;
        g.M = b;
        g.N = n - o - kTile;
        g.K = kn;
        g.A = R + o * n + o + kTile;
        g.lda = n;
        g.B = X + (o + kTile) * n + o + kTile;
        g.ldb = n;
        g.C = Pn;
        g.ldc = ldn;
        g.b_upper = 1;
        g.b_lower_zero = 1;
        // one tile row: split K (slices of at least 64 rows, at most 2) until
        // the tiles times the slices give about two blocks per compute unit
        const int64_t tiles = (g.N + kTile - 1) / kTile;
        int64_t want = (2 * (int64_t)h->num_cus + tiles - 1) / tiles;
        if (want > 2) want = 2;
        int64_t ksn = (kn + want - 1) / want;
        ksn = (ksn + kTile - 1) / kTile * kTile;
        nzn = (int)((kn + ksn - 1) / ksn);
        if (nzn > 1) {
          g.ksplit = ksn;
          g.c_zstride = zsn;
        }
        if (nzn < 1) nzn = 1;
        Trace tr(h, "inv_gemm_near", (double)sizeof(T) * ((double)b * kn + (double)kn * g.N + (double)nzn * b * g.N),
                 2.0 * (double)b * kn * (double)g.N);
        RFMLS_HIP(h, (gemm_clean<T, GemmRole::Inverse>(g, h->stream)));
      }
      {
        Trace tr(h, "inv_blockrow",
                 (double)sizeof(T) * ((double)(nzf + nzn + 1) * kTile * (double)(n - o) + (double)kTile * (n - o)),
                 (double)kTile * kTile * (double)(n - o));
        hipLaunchKernelGGL(k_inv_blockrow<T>, dim3(ceil_div(n - o, kInvCols)), dim3(kInvCols * kInvLanes), 0, h->stream, R,
                           n, I, kn > 0 ? (const T*)Pn : (const T*)nullptr, ldn, nzn, zsn,
                           (const T*)Pf, nzf, ldf, zsf, o - o2, e2, X);
      }
      RFMLS_HIP(h, hipGetLastError());
    }
  }
  return RFMLS_OK;
}

}  // namespace

__global__ void k_to_float(const double* __restrict__ src, float* __restrict__ dst, int64_t count) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = (float)src[e];
}

template <typename TX>
static rfmls_status pack_precond_t(rfmls_handle* h, rfmls_precond_t* P, const TX* X);

// Shared tail of rfmls_precond / rfmls_precond_import_R: R (normalised,
// float64 row-major n x n) is in P->Rdense.  invert_f32 (a factor computed
// and stored in float32): X = R^{-1} is formed from R rounded to float32, its
// products on the float32 matrix cores, the block-row substitutions in
// float64 arithmetic on float32 operands.
rfmls_status finish_precond(rfmls_handle* h, rfmls_precond_t* P, int check_rank, double unit,
                            int check_precision, int invert_f32) {
  const int64_t n = P->n;
  const unsigned ncb = ceil_div(n, 64);
  const unsigned nzr = ceil_div(n, kRhoRows);
  void* p_stats;
  RFMLS_CHECK(workspace(h, WS_MISC, sizeof(double) * (8 + (size_t)ncb + (size_t)nzr * (size_t)n), &p_stats));
  double* dstats = (double*)p_stats;
  double* dss = dstats + 8 + ncb;
  hipLaunchKernelGGL(k_diag_stats, dim3(1), dim3(256), 0, h->stream, P->Rdense, n, dstats);
  hipLaunchKernelGGL(k_col_sumsq, dim3(ncb, nzr), dim3(256), 0, h->stream, (const double*)P->Rdense, n, dss);
  hipLaunchKernelGGL(k_col_rho, dim3(ncb), dim3(64), 0, h->stream, (const double*)P->Rdense, n, (const double*)dss,
                     dstats + 8);
  hipLaunchKernelGGL(k_min_partials, dim3(1), dim3(256), 0, h->stream, (const double*)(dstats + 8), (int)ncb,
                     dstats + 3);
  double stats[4] = {0, 0, 0, 0};
  RFMLS_HIP(h, hipMemcpyAsync(stats, p_stats, sizeof(stats), hipMemcpyDeviceToHost, h->stream));
  RFMLS_HIP(h, hipStreamSynchronize(h->stream));
  if (stats[2] > 0 || stats[0] == 0.0)
    return fail(h, RFMLS_E_RANK, "R has a zero or non-finite diagonal entry");
  P->pivot_ratio = stats[0] / stats[1];
  P->rho_min = stats[3];
  if (check_rank && stats[0] <= 16.0 * unit * stats[1])
    return fail(h, RFMLS_E_RANK, "R numerically singular: min|r_ii| = %.3e <= 16 u max|r_ii| = %.3e",
                stats[0], 16.0 * unit * stats[1]);
  // A factor computed or stored in float32 whose column-relative pivot is
  // within 16 u32 (the margin of the float64 rank test above) carries only
  // rounding noise in that direction: the float32 QR's backward error, or the
  // rounding of R or R^{-1} to float32, is a few u32 relative per column.  It
  // then does not precondition that direction, and LSQR on A R^{-1} stalls or
  // slows down severalfold.
  const double tol32 = 16.0 * 5.960464477539063e-08;
  if (check_precision && stats[3] <= tol32)
    return fail(h, RFMLS_E_PRECISION,
                "a float32 factor cannot precondition this system: min_j |r_jj| / ||SA[:, j]|| = %.3e is within "
                "16 u32 = %.3e (columns numerically dependent in float32); factor and store in float64",
                stats[3], tol32);
  void* p_x;
  void* p_w;
  RFMLS_CHECK(workspace(h, WS_TRSM, sizeof(double) * (size_t)n * (size_t)n, &p_x));
  const int64_t kslice = 512;
  // 4 far slices of kInvOuter x n and 2 near slices of 64 x n
  RFMLS_CHECK(workspace(h, WS_QR_W, sizeof(double) * (size_t)(4 * kInvOuter + 2 * kTile) * (size_t)n, &p_w));
  if (invert_f32) {
    // X and R in float32 share the float64 n x n slot
    float* X32 = (float*)p_x;
    float* R32 = X32 + (size_t)n * (size_t)n;
    float* W32 = (float*)p_w;
    const unsigned g = ceil_div(n * n, 256) < 8192 ? ceil_div(n * n, 256) : 8192;
    hipLaunchKernelGGL(k_to_float, dim3(g), dim3(256), 0, h->stream, (const double*)P->Rdense, R32, n * n);
    RFMLS_HIP(h, hipGetLastError());
    // X starts as zeros: the float32 products use 128-column tiles, whose K
    // range for a tile column reaches the 64 x 64 block below the diagonal
    // block, so X's lower triangle must hold zeros everywhere, not only inside
    // the diagonal blocks
    RFMLS_HIP(h, hipMemsetAsync(X32, 0, sizeof(float) * (size_t)n * (size_t)n, h->stream));
    RFMLS_CHECK(invert_upper<float>(h, R32, X32, W32, W32 + (size_t)4 * kInvOuter * n, n, P->nt, kslice));
    return pack_precond_t<float>(h, P, X32);
  }
  double* X = (double*)p_x;
  RFMLS_CHECK(invert_upper<double>(h, P->Rdense, X, (double*)p_w, (double*)p_w + (size_t)4 * kInvOuter * n, n,
                                   P->nt, kslice));
  return pack_precond(h, P, X);
}

rfmls_status pack_precond(rfmls_handle* h, rfmls_precond_t* P, const double* X) {
  return pack_precond_t<double>(h, P, X);
}

template <typename TX>
static rfmls_status pack_precond_t(rfmls_handle* h, rfmls_precond_t* P, const TX* X) {
  const int64_t n = P->n;
  const int full = P->full;
  const int64_t ntiles = stored_tiles(P->nt, full);
  const size_t esz = P->store == RFMLS_F64 ? sizeof(double) : sizeof(float);
  // work tables of the tiled products: (tile row, chunk) and (tile column, chunk)
  {
    const int C = P->chunk;
    const int64_t nt = P->nt;
    const int64_t maxk = (nt + C - 1) / C;
    std::vector<int2> tr, tc;
    for (int64_t I = 0; I < nt; ++I)
      for (int64_t k = 0; k < (nt - row_first(I, full) + C - 1) / C; ++k) tr.push_back(make_int2((int)I, (int)k));
    for (int64_t J = 0; J < nt; ++J)
      for (int64_t k = 0; k < (col_end(J, nt, full) + C - 1) / C; ++k) tc.push_back(make_int2((int)J, (int)k));
    if (tr.size() != tc.size()) return fail(h, RFMLS_E_ARG, "preconditioner work tables disagree");
    P->ntab = (int64_t)tr.size();
    RFMLS_HIP(h, hipMalloc(&P->tab_row, sizeof(int2) * tr.size()));
    RFMLS_HIP(h, hipMalloc(&P->tab_col, sizeof(int2) * tc.size()));
    RFMLS_HIP(h, hipMemcpy(P->tab_row, tr.data(), sizeof(int2) * tr.size(), hipMemcpyHostToDevice));
    RFMLS_HIP(h, hipMemcpy(P->tab_col, tc.data(), sizeof(int2) * tc.size(), hipMemcpyHostToDevice));
    RFMLS_HIP(h, hipMalloc(&P->part, sizeof(double) * (size_t)(nt * maxk * kTile)));
  }
  RFMLS_HIP(h, hipMalloc(&P->Xpk, esz * (size_t)ntiles * kTile * kTile));
  if (P->store == RFMLS_F64)
    hipLaunchKernelGGL((k_pack_tiles<double, TX>), dim3((unsigned)ntiles), dim3(256), 0, h->stream, X, n,
                       P->nt, full, (double*)P->Xpk);
  else
    hipLaunchKernelGGL((k_pack_tiles<float, TX>), dim3((unsigned)ntiles), dim3(256), 0, h->stream, X, n,
                       P->nt, full, (float*)P->Xpk);
  RFMLS_HIP(h, hipGetLastError());
  return RFMLS_OK;
}

rfmls_status unpack_precond(rfmls_handle* h, const rfmls_precond_t* P, double* Xdense) {
  if (P->store == RFMLS_F64)
    hipLaunchKernelGGL(k_unpack_tiles<double>, dim3((unsigned)P->n), dim3(256), 0, h->stream,
                       (const double*)P->Xpk, P->n, P->nt, P->full, Xdense);
  else
    hipLaunchKernelGGL(k_unpack_tiles<float>, dim3((unsigned)P->n), dim3(256), 0, h->stream,
                       (const float*)P->Xpk, P->n, P->nt, P->full, Xdense);
  RFMLS_HIP(h, hipGetLastError());
  return RFMLS_OK;
}

rfmls_status put_sketched_rhs(rfmls_handle* h, int64_t s, int64_t n, int64_t nrhs, rfmls_dtype dt,
                              void* SA, int64_t ld, const double* SB) {
  const unsigned g = ceil_div(s * nrhs, 256) < 4096 ? ceil_div(s * nrhs, 256) : 4096;
  if (dt == RFMLS_F64)
    hipLaunchKernelGGL(k_put_rhs<double>, dim3(g), dim3(256), 0, h->stream, (double*)SA, ld, s, n,
                       nrhs, SB);
  else
    hipLaunchKernelGGL(k_put_rhs<float>, dim3(g), dim3(256), 0, h->stream, (float*)SA, ld, s, n,
                       nrhs, SB);
  RFMLS_HIP(h, hipGetLastError());
  return RFMLS_OK;
}

rfmls_status sketched_solution(rfmls_handle* h, const rfmls_precond_t* P, int64_t nrhs,
                               rfmls_dtype dt, const void* SA, int64_t ld, double* X0,
                               int64_t ldx0) {
  const int64_t n = P->n;
  void* p_y;
  RFMLS_CHECK(workspace(h, WS_X0, sizeof(double) * (size_t)n * (size_t)nrhs, &p_y));
  double* Y0 = (double*)p_y;
  const unsigned g = ceil_div(n * nrhs, 256) < 4096 ? ceil_div(n * nrhs, 256) : 4096;
  if (dt == RFMLS_F64)
    hipLaunchKernelGGL(k_take_y0<double>, dim3(g), dim3(256), 0, h->stream, (const double*)SA, ld,
                       n, nrhs, Y0);
  else
    hipLaunchKernelGGL(k_take_y0<float>, dim3(g), dim3(256), 0, h->stream, (const float*)SA, ld, n,
                       nrhs, Y0);
  RFMLS_HIP(h, hipGetLastError());
  // x0_k = R^{-1} y0_k with the stored X
  for (int64_t k = 0; k < nrhs; ++k)
    RFMLS_CHECK(tri_apply(h, P, 0, Y0 + k * n, X0 + k * ldx0, 0.0, nullptr, nullptr, nullptr, nullptr));
  return RFMLS_OK;
}

rfmls_status run_extract_R(rfmls_handle* h, int64_t n, const double* SA, int64_t ld, rfmls_precond_t* P) {
  RFMLS_HIP(h, hipMalloc(&P->Rdense, sizeof(double) * (size_t)n * (size_t)n));
  hipLaunchKernelGGL(k_extract_R<double>, dim3((unsigned)n), dim3(256), 0, h->stream, SA, ld, n, P->Rdense);
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
  // A float32 factor of at least 16,384 columns is also inverted in float32:
  // its n^3/3 products then run at the float32 rate.  The float32 inverse
  // preconditions slightly worse (4^3-box system, n = 25,600: 102 instead of 90
  // iterations, inverse 81 -> 48 ms, solve 0.785 -> 0.760 s; on the 2^3-box
  // Helmholtz system, n = 3,200, the extra iterations cost more than the
  // smaller inverse saves: 36.6 -> 37.2 ms).
  const bool inv32 = qr_dt == RFMLS_F32 && store == RFMLS_F32 && n >= 16384;
  return finish_precond(h, P, check_rank, unit, qr_dt == RFMLS_F32 || store == RFMLS_F32, inv32);
}

}  // namespace rfmls
