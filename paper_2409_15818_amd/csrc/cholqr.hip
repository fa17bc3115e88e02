// Panel factorisation of the blocked Householder QR (Alg. 1 step 3) by
// CholeskyQR2 with Householder reconstruction: panels stored in float64 or
// float32, every sum, factorisation and product in float64 (a float32 panel's
// rows are rounded to float32 where they are stored, and the second pass's
// Gram is of the stored rows).
//
// The unblocked panel (k_qr_panel) needs one grid-wide exchange per column.
// Here a 64-column panel P (M x 64, row-major, in place) takes three passes
// over its rows and two single-block factorisations:
//   1. k_cq_gram + k_cq_reduce: G = P^T P (partial Grams of 256-row slabs on
//      the matrix cores, then a fixed-order sum);
//   2. k_cq_factor (pass 1): column scaling D = diag(sqrt(G_jj)), Cholesky
//      D^{-1} G D^{-1} = U1^T U1, R1 = U1 D and W1 = R1^{-1};
//   3. k_cq_apply_gram + k_cq_reduce: P <- Q1 = P W1 fused with the Gram of Q1;
//   4. k_cq_factor (pass 2): Cholesky of Q1's Gram = U2^T U2 (Q = Q1 U2^{-1},
//      R = U2 R1), then the Householder reconstruction (Ballard, Demmel,
//      Grigori, Jacquelin, Knight and Nguyen, "Reconstructing Householder
//      vectors from tall-skinny QR", 2015) of Q's top 64 x 64 block: with
//      S = diag(s_j), Q S - [I; 0] = Y (-T Y_1^T) is an LU factorisation
//      without pivoting whose unit lower factor Y holds the Householder vectors
//      of a QR of P and whose pivots give tau_j = -U_jj = 1 + |c_j|, s_j =
//      -sign(c_j) chosen column by column from the current pivot c_j (so
//      |U_jj| >= 1 and the elimination is stable); the QR's triangular factor
//      is S R.  The panel's top block gets S R and Y_1;
//   5. k_cq_apply: the rows below become Y_2 = Q1 (U2^{-1} S U^{-1}).
// The panel is left exactly as the unblocked kernel leaves it: S R on and
// above the diagonal, the vectors below it (unit diagonal implied), tau.
//
// CholeskyQR2 is accurate while the scaled panel's condition number stays
// well below u^{-1/2} (its first pass squares it).  The sketches of the RFM
// systems here have scaled panel conditions up to 3.2e6 (8x8-box system, all
// 200 panels; unscaled up to 2e13).  A panel whose first Cholesky meets a
// non-positive pivot or a pivot ratio below the caller's threshold is flagged
// (status 1) and factored by the unblocked kernel instead, on the untouched
// panel; a second Cholesky failure (status 2) leaves Q1 in the panel, which the
// unblocked kernel then factors, its R multiplied by R1 afterwards
// (k_cq_fix).  Every sum runs in a fixed order.
#include "common.h"

namespace rfmls {
namespace {

constexpr int kNb = 64;      // panel width
constexpr int kSlab = 256;   // rows per partial Gram (tall panels)
// Panels under this many rows take 128-row slabs (two 16-row groups per
// wavefront): twice the workgroups, so a short panel's Gram and apply passes
// use more of the GPU, their partial Grams still few enough to sum (Helmholtz
// sketch, 12,800 rows: 0.155 -> 0.146 ms per panel; 64-row slabs 0.147).
constexpr int64_t kShortPanelRows = 32768;
inline int64_t slab_rows(int64_t M) { return M >= kShortPanelRows ? kSlab : 128; }

typedef double v4d __attribute__((ext_vector_type(4)));

// status: 0 CholeskyQR2 used; 1 first Cholesky failed (panel untouched);
// 2 second Cholesky failed (panel holds Q1, R1 in Rc)

// Operand layout of v_mfma_f64_16x16x4f64 (D += A B, A 16 x 4, B 4 x 16): lane
// l = 16 lk + lr holds A[lr][lk] and B[lk][lr]; accumulator register r holds
// D[lk + 4 r][lr].

// Partial Gram of rows [z S, (z + 1) S) of P (S = 64 NG) on the matrix cores.
// Wave w takes the 16 NG rows from z S + 16 NG w and accumulates the ten upper
// 16 x 16 tiles of their Gram; each lane loads its operands straight from P
// (lane (lr, lk) reads row 4 s + lk, columns 16 q + lr: every 16 lanes read
// 128 contiguous bytes), no LDS staging.  The four waves' tiles are then added
// in wave order through LDS and the full symmetric 64 x 64 partial written.
template <typename TS, int NG>
__global__ void __launch_bounds__(256) k_cq_gram(const TS* __restrict__ P, int64_t ld, int64_t M,
                                                 double* __restrict__ Gpart, const int* __restrict__ status) {
  if (status && *status) return;
  __shared__ double S[kNb][kNb + 1];
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  v4d acc[10];
#pragma unroll
  for (int q = 0; q < 10; ++q) acc[q] = v4d{0.0, 0.0, 0.0, 0.0};
  const int64_t r0 = (int64_t)blockIdx.x * (64 * NG) + 16 * NG * w;
  // all the wavefront's rows' operands loaded first (rows past M read row
  // M - 1 and are replaced by zeros, so the loads carry no branch)
  double x[4 * NG][4];
#pragma unroll
  for (int s = 0; s < 4 * NG; ++s) {
    const int64_t row = r0 + 4 * s + lk;
    const int64_t rr = row < M ? row : M - 1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double v = (double)P[rr * ld + 16 * q + lr];
      x[s][q] = row < M ? v : 0.0;
    }
  }
#pragma unroll
  for (int s = 0; s < 4 * NG; ++s) {
    int tile = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = a; b < 4; ++b, ++tile)
        acc[tile] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[s][a], x[s][b], acc[tile], 0, 0, 0);
  }
  // tile (a, b): D[lk + 4 r][lr] = G[16 a + lk + 4 r][16 b + lr]
  for (int ww = 0; ww < 4; ++ww) {
    if (w == ww) {
      int tile = 0;
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a; b < 4; ++b, ++tile)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            double& g = S[16 * a + lk + 4 * r][16 * b + lr];
            g = ww == 0 ? acc[tile][r] : g + acc[tile][r];
          }
    }
    __syncthreads();
  }
  double* gp = Gpart + (int64_t)blockIdx.x * kNb * kNb;
  for (int e = t; e < kNb * kNb; e += 256) {
    const int i = e / kNb, j = e % kNb;
    // upper tiles hold G[i][j] for tile(i) <= tile(j); the rest by symmetry
    gp[e] = (i >> 4) <= (j >> 4) ? S[i][j] : S[j][i];
  }
}

// G = sum of the nslab partials in slab order.  Block b takes entries
// 16 b .. 16 b + 15; its 16 slices of threads sum every 16th partial, then the
// 16 slice sums are added in order.  With reset, the panel's status is set to 0
// (first pass: a new panel).
__global__ void __launch_bounds__(256) k_cq_reduce(const double* __restrict__ Gpart, int nslab,
                                                   double* __restrict__ G, int* __restrict__ status, int reset) {
  if (!reset && *status) return;
  __shared__ double red[16][17];
  const int t = threadIdx.x;
  const int el = t & 15, zq = t >> 4;
  const int e = blockIdx.x * 16 + el;
  double s = 0.0;
  for (int z = zq; z < nslab; z += 16) s += Gpart[(int64_t)z * kNb * kNb + e];
  red[zq][el] = s;
  __syncthreads();
  if (t < 16) {
    double tot = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) tot += red[q][t];
    G[blockIdx.x * 16 + t] = tot;
  }
  if (reset && blockIdx.x == 0 && t == 0) *status = 0;
}

// ---------------------------------------------------------------------------
// 64 x 64 factorisations in LDS by one block of 256 threads, blocked by 16:
// the eliminations of a 16-row (or 16-column) block on one wavefront in
// registers (values passed by v_readlane), every product of blocks on the
// matrix cores (lds_mm).
// ---------------------------------------------------------------------------
constexpr int kB = 16;
constexpr int kLd = kNb + 1;  // LDS row stride of a 64 x 64 matrix
typedef double Mat[kNb][kLd];
typedef double Blk[kB][kB + 1];

__device__ __forceinline__ double lane_bcast(double v, int lane) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// D = alpha op(A) B + beta D for LDS operands (row strides lda, ldb, ldd), D
// m x n, K the inner dimension, all multiples of 16 (K of 4); op(A) = A (m x K)
// or, with ta, A^T (A stored K x m).  Wave w computes 16 x 16 tiles w, w + 4,
// ... (at most 16 tiles) into registers; after a barrier they are written, so
// D may overlap A or B.  Every thread of the block calls it.
__device__ void lds_mm(double* D, int ldd, const double* A, int lda, bool ta, const double* B, int ldb, int m, int n,
                       int K, double alpha, double beta) {
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int tn = n / 16, nt = (m / 16) * tn;
  const int astep = ta ? 4 * lda : 4;
  v4d acc[4];
  const double* ap[4];
  const double* bp[4];
#pragma unroll
  for (int sl = 0; sl < 4; ++sl) {
    acc[sl] = v4d{0.0, 0.0, 0.0, 0.0};
    const int tile = w + 4 * sl;
    const int ti = tile / tn, tj = tile % tn;
    ap[sl] = ta ? A + lk * lda + 16 * ti + lr : A + (16 * ti + lr) * lda + lk;
    bp[sl] = B + lk * ldb + 16 * tj + lr;
  }
  // the four tiles' chains interleaved: their operand loads issue together
#pragma unroll 2
  for (int k4 = 0; k4 < K / 4; ++k4) {
    double a[4], b[4];
#pragma unroll
    for (int sl = 0; sl < 4; ++sl)
      if (w + 4 * sl < nt) {
        a[sl] = ap[sl][k4 * astep];
        b[sl] = bp[sl][k4 * 4 * ldb];
      }
#pragma unroll
    for (int sl = 0; sl < 4; ++sl)
      if (w + 4 * sl < nt) acc[sl] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[sl], b[sl], acc[sl], 0, 0, 0);
  }
  __syncthreads();
#pragma unroll
  for (int sl = 0; sl < 4; ++sl) {
    const int tile = w + 4 * sl;
    if (tile < nt) {
      const int ti = tile / tn, tj = tile % tn;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double* d = D + (16 * ti + lk + 4 * r) * ldd + 16 * tj + lr;
        *d = beta == 0.0 ? alpha * acc[sl][r] : fma(alpha, acc[sl][r], beta * *d);
      }
    }
  }
  __syncthreads();
}

// Orders a wavefront's LDS writes before its later LDS reads (no block barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Z[w] = inverse of diagonal block w of the upper triangular U, wavefront w
// taking block w, lane l < 16 column l, by a column sweep with U's entries read
// uniformly from LDS.
__device__ void blk_diag_inverses(const Mat& U, Blk* Z) {
  const int t = threadIdx.x;
  const int w = t >> 6, l = t & 63;
  const int k0 = w * kB;
  double rd[kB], acc[kB];
#pragma unroll
  for (int i = 0; i < kB; ++i) {
    rd[i] = 1.0 / U[k0 + i][k0 + i];
    acc[i] = (i == l) ? 1.0 : 0.0;
  }
#pragma unroll
  for (int m2 = kB - 1; m2 >= 0; --m2) {
    const double zm = (m2 <= l) ? acc[m2] * rd[m2] : 0.0;
    acc[m2] = zm;
#pragma unroll
    for (int i = 0; i < m2; ++i) acc[i] = fma(-U[k0 + i][k0 + m2], zm, acc[i]);
  }
  if (l < kB)
#pragma unroll
    for (int i = 0; i < kB; ++i) Z[w][i][l] = acc[i];
  __syncthreads();
}

// Cholesky A = U^T U of the symmetric positive definite A (both triangles
// read: A is kept whole), U written over A with its lower triangle set to
// zero; Z[kb] receives the inverse of diagonal block kb.  Returns false
// (every thread) on a non-positive or non-finite pivot; pmin / pmax: the
// extreme pivots u_kk.  Block row kb (16 rows, columns k0 = 16 kb .. 63) is
// factored by wavefront 0 alone, lane l holding column k0 + l: step s takes
// the pivot from lane s (v_readlane), scales the lanes' row s entries to U's
// row s and subtracts u_s,i u_s,l from the rows i > s below it, u_s,i read
// from lane i; the whole block row of U comes out of the one elimination (no
// product with the diagonal block's inverse) and no LDS round trip sits on the
// chain.  The trailing block then takes A22 -= U12^T U12 on the matrix cores.
__device__ bool blk_cholesky(Mat& A, Blk* Z, double* pmin, double* pmax) {
  __shared__ int bad;
  __shared__ double ext[2];
  const int t = threadIdx.x;
  if (t == 0) bad = 0;
  __syncthreads();
  double mn = 1e300, mx = 0.0;  // uniform on wavefront 0 (pivots by readlane)
  for (int kb = 0; kb < kNb / kB; ++kb) {
    const int k0 = kb * kB;
    if (t < 64) {
      const int l = t;
      const bool act = l < kNb - k0;
      double d[kB];
#pragma unroll
      for (int i = 0; i < kB; ++i) d[i] = act ? A[k0 + i][k0 + l] : 0.0;
      bool badl = false;
#pragma unroll
      for (int s2 = 0; s2 < kB; ++s2) {
        const double piv = lane_bcast(d[s2], s2);
        if (!(piv > 0.0) || !isfinite(piv)) badl = true;
        const double r = rsqrt(piv > 0.0 ? piv : 1.0);
        const double ukk = piv * r;
        mn = fmin(mn, ukk);
        mx = fmax(mx, ukk);
        const double us = l == s2 ? ukk : d[s2] * r;  // u_{s,l} for l >= s
        d[s2] = l >= s2 ? us : 0.0;
#pragma unroll
        for (int i = s2 + 1; i < kB; ++i) d[i] = fma(-lane_bcast(us, i), us, d[i]);
      }
      if (act)
#pragma unroll
        for (int i = 0; i < kB; ++i) A[k0 + i][k0 + l] = d[i];
      if (t == 0) {
        if (badl) bad = 1;
        ext[0] = mn;
        ext[1] = mx;
      }
    }
    __syncthreads();
    if (bad) break;  // uniform: read after the barrier
    const int nc = kNb - k0 - kB;
    if (nc > 0)  // A22 -= U12^T U12
      lds_mm(&A[k0 + kB][k0 + kB], kLd, &A[k0][k0 + kB], kLd, true, &A[k0][k0 + kB], kLd, nc, nc, kB, -1.0, 1.0);
  }
  // lower triangle outside the diagonal blocks
  for (int e = t; e < kNb * kNb; e += 256) {
    const int i = e / kNb, j = e % kNb;
    if ((i >> 4) > (j >> 4)) A[i][j] = 0.0;
  }
  __syncthreads();
  const bool good = !bad;
  if (good) blk_diag_inverses(A, Z);
  *pmin = ext[0];
  *pmax = ext[1];
  return good;
}

// W = U^{-1} for the upper triangular U (zero below the diagonal; Z the
// inverses of its diagonal blocks) by block back substitution from the bottom
// block row up: W[k, >k] = -Z_k (U[k, >k] W[>k, >k]).  T is scratch.
__device__ void blk_upper_inverse(const Mat& U, const Blk* Z, Mat& W, Mat& T) {
  const int t = threadIdx.x;
  for (int e = t; e < kNb * kNb; e += 256) {
    const int i = e / kNb, j = e % kNb;
    W[i][j] = (i >> 4) == (j >> 4) ? Z[i >> 4][i & 15][j & 15] : 0.0;
  }
  __syncthreads();
  for (int kb = kNb / kB - 2; kb >= 0; --kb) {
    const int k0 = kb * kB, nc = kNb - k0 - kB;
    lds_mm(&T[0][0], kLd, &U[k0][k0 + kB], kLd, false, &W[k0 + kB][k0 + kB], kLd, kB, nc, nc, 1.0, 0.0);
    lds_mm(&W[k0][k0 + kB], kLd, &Z[kb][0][0], kB + 1, false, &T[0][0], kLd, kB, nc, kB, -1.0, 0.0);
  }
}

// LU without pivoting of Q1 S - I (Q1 the top 64 x 64 block of Q, in A) with
// s_j = -sign(c_j) taken from the current pivot c_j: the identity and the
// column signs only touch the pivots (u_jj = -|c_j| - 1) and the multipliers
// (l_ij = s_j a_ij / u_jj), so the elimination runs on Q1 itself, blocked by 16
// columns: the 64 x 16 panel on wavefront 0 (lane i holding row i), the block
// row by forward substitution, the trailing block on the matrix cores.  On
// return A holds the multipliers below the diagonal and U = (eliminated Q1
// entries times s_c) above it, u_jj on it; sg holds s.
__device__ void blk_recon_lu(Mat& A, double* sg) {
  __shared__ double prow[kB];
  const int t = threadIdx.x;
  for (int kb = 0; kb < kNb / kB; ++kb) {
    const int k0 = kb * kB;
    if (t < 64) {
      // lane i holds row i of the 64 x 16 panel; step j: the pivot by
      // readlane, the pivot row's next entry by readlane, the rest of it through
      // LDS (written by the pivot row's lane, read uniformly)
      const int i = t;
      double p[kB];
#pragma unroll
      for (int m = 0; m < kB; ++m) p[m] = A[i][k0 + m];
#pragma unroll
      for (int j = 0; j < kB; ++j) {
        const int pr = k0 + j;
        const double cj = lane_bcast(p[j], pr);
        const double sj = cj >= 0.0 ? -1.0 : 1.0;
        const double ujj = -fabs(cj) - 1.0;
        const double fj = sj * (1.0 / ujj);
        if (i == pr) {
          sg[pr] = sj;
          p[j] = ujj;
#pragma unroll
          for (int m = j + 2; m < kB; ++m) prow[m] = p[m];
        }
        const double lij = p[j] * fj;
        if (i > pr) p[j] = lij;
        if (j + 1 < kB) {
          const double un = lane_bcast(p[j + 1], pr);
          if (i > pr) p[j + 1] = fma(-lij, un, p[j + 1]);
          wave_sync();
#pragma unroll
          for (int m = j + 2; m < kB; ++m)
            if (i > pr) p[m] = fma(-lij, prow[m], p[m]);
        }
      }
#pragma unroll
      for (int m = 0; m < kB; ++m) A[i][k0 + m] = p[m];
    }
    __syncthreads();
    const int nc = kNb - k0 - kB;
    if (nc > 0) {
      if (t < nc) {  // block row: unit lower forward substitution, a column per thread
        const int c = k0 + kB + t;
        double x[kB];
#pragma unroll
        for (int i = 0; i < kB; ++i) {
          double acc = A[k0 + i][c];
#pragma unroll
          for (int m = 0; m < i; ++m) acc = fma(-A[k0 + i][k0 + m], x[m], acc);
          x[i] = acc;
        }
#pragma unroll
        for (int i = 0; i < kB; ++i) A[k0 + i][c] = x[i];
      }
      __syncthreads();
      lds_mm(&A[k0 + kB][k0 + kB], kLd, &A[k0 + kB][k0], kLd, false, &A[k0][k0 + kB], kLd, nc, nc, kB, -1.0, 1.0);
    }
  }
  // the column signs on U's off-diagonal entries (the diagonal holds u_jj)
  for (int e = t; e < kNb * kNb; e += 256) {
    const int i = e / kNb, c = e % kNb;
    if (i < c) A[i][c] *= sg[c];
  }
  __syncthreads();
}

// One Cholesky step of CholeskyQR2 on the reduced Gram G.
// pass 1 (column-scaled Gram D^{-1} G D^{-1} = U^T U): R1 = U D into Rc and
//   Wk = R1^{-1} = D^{-1} U^{-1} (the operand of the fused apply + Gram).
// pass 2 (Gram of Q1 = U2^T U2): R = U2 R1 into the panel's top block as S R,
//   and the Householder reconstruction of Q = Q1 U2^{-1}: its top block
//   Q1top U2^{-1} is factored by blk_recon_lu, the multipliers go below the
//   diagonal of the panel's top block, tau_j = -u_jj, and
//   Wk = U2^{-1} S U^{-1}, with which the rows below become the Householder
//   vectors L2 = Q1bot U2^{-1} S U^{-1}.
// A pivot ratio u_min / u_max below min_pivot_ratio (or a non-positive pivot)
// sets *status = pass and leaves everything else untouched.
template <typename TS>
__global__ void __launch_bounds__(256) k_cq_factor(const double* __restrict__ G, double* __restrict__ Wk,
                                                   double* __restrict__ Rc, TS* __restrict__ P, int64_t ld,
                                                   TS* __restrict__ tau, int* __restrict__ status, int pass,
                                                   double min_pivot_ratio) {
  if (pass == 2 && *status) return;
  __shared__ Mat M0, M1, M2, M3;
  __shared__ Blk Z[kNb / kB];
  __shared__ double dsc[kNb];
  __shared__ double sg[kNb];
  __shared__ int bad0;
  const int t = threadIdx.x;
  // thread t takes element (t / 64 + 4 q, t % 64), q < 16, of every 64 x 64
  // operand; each operand's 16 loads are issued together
  const int er = t >> 6, ec = t & 63;
  double gv[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) gv[q] = G[(er + 4 * q) * kNb + ec];
  if (pass == 2) {
    // the panel's top block (Q1's) into M3, read after the Cholesky
    double pv[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) pv[q] = (double)P[(int64_t)(er + 4 * q) * ld + ec];
#pragma unroll
    for (int q = 0; q < 16; ++q) M3[er + 4 * q][ec] = pv[q];
  }
  if (t < kNb) {
    const double gjj = G[t * kNb + t];
    dsc[t] = pass == 1 ? sqrt(gjj > 0.0 ? gjj : 0.0) : 1.0;
  }
  if (t == 0) bad0 = 0;
  __syncthreads();
  if (t < kNb && !(dsc[t] > 0.0)) bad0 = 1;
  {
    const double dj = dsc[ec];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const double di = dsc[er + 4 * q];
      M0[er + 4 * q][ec] = (di > 0.0 && dj > 0.0) ? gv[q] * (1.0 / di) * (1.0 / dj) : 0.0;
    }
  }
  __syncthreads();
  double pmin = 0.0, pmax = 0.0;
  const bool ok = !bad0 && blk_cholesky(M0, Z, &pmin, &pmax);
  if (!ok || !(pmin >= min_pivot_ratio * pmax)) {
    if (t == 0) *status = pass;
    return;
  }
  blk_upper_inverse(M0, Z, M1, M2);  // M1 = U^{-1}
  if (pass == 1) {
    for (int e = t; e < kNb * kNb; e += 256) {
      const int i = e / kNb, j = e % kNb;
      Wk[e] = M1[i][j] * (1.0 / dsc[i]);
      Rc[e] = M0[i][j] * dsc[j];
    }
    return;
  }
  // pass 2: M2 = R = U2 R1 (written over R1); M0 = Q1top U2^{-1}
  {
    double rv[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) rv[q] = Rc[(er + 4 * q) * kNb + ec];
#pragma unroll
    for (int q = 0; q < 16; ++q) M2[er + 4 * q][ec] = rv[q];
  }
  __syncthreads();
  lds_mm(&M2[0][0], kLd, &M0[0][0], kLd, false, &M2[0][0], kLd, kNb, kNb, kNb, 1.0, 0.0);
  lds_mm(&M0[0][0], kLd, &M3[0][0], kLd, false, &M1[0][0], kLd, kNb, kNb, kNb, 1.0, 0.0);
  blk_recon_lu(M0, sg);
  for (int e = t; e < kNb * kNb; e += 256) {
    const int i = e / kNb, c = e % kNb;
    P[(int64_t)i * ld + c] = (TS)(i <= c ? sg[i] * M2[i][c] : M0[i][c]);
  }
  if (t < kNb) tau[t] = (TS)(-M0[t][t]);
  __syncthreads();
  for (int e = t; e < kNb * kNb; e += 256) {  // U alone (zero below the diagonal)
    const int i = e / kNb, c = e % kNb;
    if (i > c) M0[i][c] = 0.0;
  }
  __syncthreads();
  blk_diag_inverses(M0, Z);
  blk_upper_inverse(M0, Z, M2, M3);  // M2 = U^{-1}
  for (int e = t; e < kNb * kNb; e += 256) {
    const int i = e / kNb, c = e % kNb;
    M2[i][c] *= sg[i];
  }
  __syncthreads();
  lds_mm(&M3[0][0], kLd, &M1[0][0], kLd, false, &M2[0][0], kLd, kNb, kNb, kNb, 1.0, 0.0);
  for (int e = t; e < kNb * kNb; e += 256) Wk[e] = M3[e / kNb][e % kNb];
}

// A operands of P W for one row: lane (lr, lk) of a wavefront takes row lr of
// a 16-row group, and step t of the product's K range one of its columns,
// kcol(t, lk).  With 16-byte loads (V16: the row start and ld allow them)
// the lane reads E = 16 / sizeof(TS) adjacent columns at a time, so step t
// takes column 4E (t / E) + E lk + t % E; otherwise column 4 t + lk.  Either
// way the four lanes of a step hold four distinct columns inside the 4E-column
// (or 4-column) chunk of the step, all 64 columns are covered once, and the
// steps t < 4 (q + 1) hold every column <= 16 q + 15.
template <typename TS, bool V16>
__device__ __forceinline__ int kcol(int t, int lk) {
  constexpr int E = 16 / (int)sizeof(TS);
  return V16 ? 4 * E * (t / E) + E * lk + t % E : 4 * t + lk;
}
template <typename TS, bool V16>
__device__ __forceinline__ void load_arow(double (&a)[16], const TS* __restrict__ row, int lk, bool in) {
  if constexpr (V16 && sizeof(TS) == 8) {
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const double2 v = *(const double2*)(row + 8 * m + 2 * lk);
      a[2 * m] = in ? v.x : 0.0;
      a[2 * m + 1] = in ? v.y : 0.0;
    }
  } else if constexpr (V16) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const float4 v = *(const float4*)(row + 16 * m + 4 * lk);
      a[4 * m] = in ? (double)v.x : 0.0;
      a[4 * m + 1] = in ? (double)v.y : 0.0;
      a[4 * m + 2] = in ? (double)v.z : 0.0;
      a[4 * m + 3] = in ? (double)v.w : 0.0;
    }
  } else {
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const double v = (double)row[4 * t + lk];
      a[t] = in ? v : 0.0;
    }
  }
}
// D = A W for a 16-row group, W upper triangular (zeros below its diagonal
// are skipped: tile q's K range stops at column 16 q + 15).  Accumulator
// register r of tile q holds D[lk + 4 r][16 q + lr].
template <typename TS, bool V16>
__device__ __forceinline__ void group_times_upper(const double (&a)[16], const double (*Ws)[kNb + 1], int lr, int lk,
                                                  v4d (&acc)[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int kk = kcol<TS, V16>(t, lk);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (t < 4 * (q + 1)) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], Ws[kk][16 * q + lr], acc[q], 0, 0, 0);
  }
}

// Rows [r_begin, M) of P <- P W (W 64 x 64 upper triangular) on the matrix
// cores, in place: wave w of a block takes 16 rows, reads all 64 of their
// columns (A operands, in registers) before it writes them.  Runs when
// *status == 0.
template <typename TS, bool V16>
__global__ void __launch_bounds__(256) k_cq_apply(TS* __restrict__ P, int64_t ld, int64_t r_begin, int64_t M,
                                                  const double* __restrict__ W, const int* __restrict__ status) {
  if (*status) return;
  __shared__ double Ws[kNb][kNb + 1];
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t rbase = r_begin + (int64_t)blockIdx.x * 64 + 16 * w;
  const int64_t ra = rbase + lr;
  const int64_t rc = ra < M ? ra : M - 1;  // rows past M: row M - 1, replaced by zeros
  double a[16];
  load_arow<TS, V16>(a, P + rc * ld, lk, ra < M);
  for (int e = t; e < kNb * kNb; e += 256) Ws[e / kNb][e % kNb] = W[e];
  __syncthreads();
  v4d acc[4];
  group_times_upper<TS, V16>(a, Ws, lr, lk, acc);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t row = rbase + lk + 4 * r;
    if (row < M)
#pragma unroll
      for (int q = 0; q < 4; ++q) P[row * ld + 16 * q + lr] = (TS)acc[q][r];
  }
}

// First pass's apply fused with the second pass's Gram: rows
// [z S, (z + 1) S) of P (S = 64 NG) <- P W (W upper triangular; matrix cores,
// in place) and the partial Gram of the new rows.  Wave w takes NG groups of 16
// rows from z S + 16 NG w; a group's product tiles (D[lk + 4 r][16 q + lr] in
// register r of tile q) are already the Gram's operands for K-step r.  The
// waves' Gram tiles are added in wave order through LDS.  Runs when
// *status == 0.
template <typename TS, bool V16, int NG>
__global__ void __launch_bounds__(256) k_cq_apply_gram(TS* __restrict__ P, int64_t ld, int64_t M,
                                                       const double* __restrict__ W, double* __restrict__ Gpart,
                                                       const int* __restrict__ status) {
  if (*status) return;
  __shared__ double Ws[kNb][kNb + 1];
  __shared__ double S[kNb][kNb + 1];
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  // the four groups' operands loaded first (rows past M read row M - 1 and
  // are replaced by zeros, so the loads carry no branch)
  double ag[NG][16];
#pragma unroll
  for (int grp = 0; grp < NG; ++grp) {
    const int64_t ra = (int64_t)blockIdx.x * (64 * NG) + 16 * NG * w + 16 * grp + lr;
    const int64_t rc = ra < M ? ra : M - 1;
    load_arow<TS, V16>(ag[grp], P + rc * ld, lk, ra < M);
  }
  for (int e = t; e < kNb * kNb; e += 256) Ws[e / kNb][e % kNb] = W[e];
  __syncthreads();
  v4d gacc[10];
#pragma unroll
  for (int q = 0; q < 10; ++q) gacc[q] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int grp = 0; grp < NG; ++grp) {
    const int64_t rbase = (int64_t)blockIdx.x * (64 * NG) + 16 * NG * w + 16 * grp;
    v4d acc[4];
    group_times_upper<TS, V16>(ag[grp], Ws, lr, lk, acc);
    if constexpr (sizeof(TS) < sizeof(double)) {
      // the Gram below is of the rows as stored
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[q][r] = (double)(TS)acc[q][r];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = rbase + lk + 4 * r;
      if (row < M)
#pragma unroll
        for (int q = 0; q < 4; ++q) P[row * ld + 16 * q + lr] = (TS)acc[q][r];
    }
    // rows past M hold exact zeros (zero operands) and add nothing
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int tile = 0;
#pragma unroll
      for (int a2 = 0; a2 < 4; ++a2)
#pragma unroll
        for (int b = a2; b < 4; ++b, ++tile)
          gacc[tile] = __builtin_amdgcn_mfma_f64_16x16x4f64(acc[a2][r], acc[b][r], gacc[tile], 0, 0, 0);
    }
  }
  for (int ww = 0; ww < 4; ++ww) {
    if (w == ww) {
      int tile = 0;
#pragma unroll
      for (int a2 = 0; a2 < 4; ++a2)
#pragma unroll
        for (int b = a2; b < 4; ++b, ++tile)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            double& g = S[16 * a2 + lk + 4 * r][16 * b + lr];
            g = ww == 0 ? gacc[tile][r] : g + gacc[tile][r];
          }
    }
    __syncthreads();
  }
  double* gp = Gpart + (int64_t)blockIdx.x * kNb * kNb;
  for (int e = t; e < kNb * kNb; e += 256) {
    const int i = e / kNb, j = e % kNb;
    gp[e] = (i >> 4) <= (j >> 4) ? S[i][j] : S[j][i];
  }
}

// After the unblocked kernel factored Q1 (status 2): its R' times R1 (upper
// triangular products, terms in order), written back into the panel's top rows.
template <typename TS>
__global__ void __launch_bounds__(256) k_cq_fix(TS* __restrict__ P, int64_t ld, const double* __restrict__ Rc,
                                                const int* __restrict__ status) {
  if (*status != 2) return;
  __shared__ double A[kNb][kNb + 1];
  __shared__ double B[kNb][kNb + 1];
  const int t = threadIdx.x;
  for (int e = t; e < kNb * kNb; e += 256) {
    const int r = e / kNb, c = e % kNb;
    A[r][c] = c >= r ? (double)P[(int64_t)r * ld + c] : 0.0;
    B[r][c] = Rc[e];
  }
  __syncthreads();
  for (int e = t; e < kNb * kNb; e += 256) {
    const int r = e / kNb, c = e % kNb;
    if (c < r) continue;
    double sacc = 0.0;
    for (int k = r; k <= c; ++k) sacc = fma(A[r][k], B[k][c], sacc);
    P[(int64_t)r * ld + c] = (TS)sacc;
  }
}

}  // namespace

// Partial Grams of an M-row panel.
static int64_t cq_nslab(int64_t M) { return (M + slab_rows(M) - 1) / slab_rows(M); }

int64_t cholqr_workspace_doubles(int64_t M) {
  // room for the most partials of any panel of at most M rows
  const int64_t ms = M < kShortPanelRows - 1 ? M : kShortPanelRows - 1;
  const int64_t a = cq_nslab(M), b = cq_nslab(ms);
  return (a > b ? a : b) * kNb * kNb + 3 * kNb * kNb + 64;
}

// Enqueues CholeskyQR2 and the reconstruction on the 64-column panel P
// (M >= 64 rows, stored as TS, all arithmetic in float64); ws holds
// cholqr_workspace_doubles(M) doubles.  A pass whose Cholesky pivot ratio falls
// below min_ratio1 (first pass) or min_ratio2 (second) sets the status.  The
// caller then launches the unblocked kernel gated on *status != 0, and
// cholqr_fix.
template <typename TS>
static rfmls_status cholqr_panel(rfmls_handle* h, TS* P, int64_t ld, int64_t M, TS* tau, double* ws, int* status,
                                 double min_ratio1, double min_ratio2) {
  hipStream_t st = h->stream;
  const int64_t nslab = cq_nslab(M);
  const bool tall = slab_rows(M) == kSlab;
  // G, Wk and Rc sit after the most partials any panel of this QR writes
  double* Gpart = ws;
  double* G = ws + (cholqr_workspace_doubles(M) - 3 * kNb * kNb - 64);
  double* Wk = G + kNb * kNb;
  double* Rc = Wk + kNb * kNb;
  if (tall)
    hipLaunchKernelGGL((k_cq_gram<TS, 4>), dim3((unsigned)nslab), dim3(256), 0, st, (const TS*)P, ld, M, Gpart,
                       (const int*)nullptr);
  else
    hipLaunchKernelGGL((k_cq_gram<TS, 2>), dim3((unsigned)nslab), dim3(256), 0, st, (const TS*)P, ld, M, Gpart,
                       (const int*)nullptr);
  hipLaunchKernelGGL(k_cq_reduce, dim3(kNb * kNb / 16), dim3(256), 0, st, (const double*)Gpart, (int)nslab, G, status,
                     1);
  hipLaunchKernelGGL(k_cq_factor<TS>, dim3(1), dim3(256), 0, st, (const double*)G, Wk, Rc, P, ld, tau, status, 1,
                     min_ratio1);
  // 16-byte operand loads when every row start allows them
  const bool v16 = ld % (16 / (int64_t)sizeof(TS)) == 0 && reinterpret_cast<uintptr_t>(P) % 16 == 0;
  if (v16 && tall)
    hipLaunchKernelGGL((k_cq_apply_gram<TS, true, 4>), dim3((unsigned)nslab), dim3(256), 0, st, P, ld, M,
                       (const double*)Wk, Gpart, (const int*)status);
  else if (v16)
    hipLaunchKernelGGL((k_cq_apply_gram<TS, true, 2>), dim3((unsigned)nslab), dim3(256), 0, st, P, ld, M,
                       (const double*)Wk, Gpart, (const int*)status);
  else if (tall)
    hipLaunchKernelGGL((k_cq_apply_gram<TS, false, 4>), dim3((unsigned)nslab), dim3(256), 0, st, P, ld, M,
                       (const double*)Wk, Gpart, (const int*)status);
  else
    hipLaunchKernelGGL((k_cq_apply_gram<TS, false, 2>), dim3((unsigned)nslab), dim3(256), 0, st, P, ld, M,
                       (const double*)Wk, Gpart, (const int*)status);
  hipLaunchKernelGGL(k_cq_reduce, dim3(kNb * kNb / 16), dim3(256), 0, st, (const double*)Gpart, (int)nslab, G, status,
                     0);
  hipLaunchKernelGGL(k_cq_factor<TS>, dim3(1), dim3(256), 0, st, (const double*)G, Wk, Rc, P, ld, tau, status, 2,
                     min_ratio2);
  if (M > kNb) {
    const dim3 grid((unsigned)((M - kNb + 63) / 64));
    if (v16)
      hipLaunchKernelGGL((k_cq_apply<TS, true>), grid, dim3(256), 0, st, P, ld, (int64_t)kNb, M, (const double*)Wk,
                         (const int*)status);
    else
      hipLaunchKernelGGL((k_cq_apply<TS, false>), grid, dim3(256), 0, st, P, ld, (int64_t)kNb, M, (const double*)Wk,
                         (const int*)status);
  }
  RFMLS_HIP(h, hipGetLastError());
  return RFMLS_OK;
}

rfmls_status run_cholqr_panel(rfmls_handle* h, double* P, int64_t ld, int64_t M, double* tau, double* ws,
                              int* status, double min_ratio1, double min_ratio2) {
  return cholqr_panel<double>(h, P, ld, M, tau, ws, status, min_ratio1, min_ratio2);
}
rfmls_status run_cholqr_panel(rfmls_handle* h, float* P, int64_t ld, int64_t M, float* tau, double* ws, int* status,
                              double min_ratio1, double min_ratio2) {
  return cholqr_panel<float>(h, P, ld, M, tau, ws, status, min_ratio1, min_ratio2);
}

// Status 2 only: the panel's R (from the unblocked kernel, on Q1) times R1.
template <typename TS>
static rfmls_status cholqr_fix_t(rfmls_handle* h, TS* P, int64_t ld, int64_t M, const double* ws, const int* status) {
  const double* Rc = ws + (cholqr_workspace_doubles(M) - 3 * kNb * kNb - 64) + 2 * kNb * kNb;
  hipLaunchKernelGGL(k_cq_fix<TS>, dim3(1), dim3(256), 0, h->stream, P, ld, Rc, status);
  RFMLS_HIP(h, hipGetLastError());
  return RFMLS_OK;
}
rfmls_status cholqr_fix(rfmls_handle* h, double* P, int64_t ld, int64_t M, const double* ws, const int* status) {
  return cholqr_fix_t<double>(h, P, ld, M, ws, status);
}
rfmls_status cholqr_fix(rfmls_handle* h, float* P, int64_t ld, int64_t M, const double* ws, const int* status) {
  return cholqr_fix_t<float>(h, P, ld, M, ws, status);
}

}  // namespace rfmls
