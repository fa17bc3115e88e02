// CSSVDP-LSQR preconditioner (Alg. 2 step 3): the truncated SVD of the sketch
// SA through its R factor (SA = Q R, so SA and R share Sigma and V), and
// P = V_r Sigma_r^{-1} with r = #{sigma_i > rcond sigma_1} (Sec. 3.2: the
// LAPACK-style threshold, rcond times the largest singular value).
//
// SVD of R by one-sided (Hestenes) Jacobi on its columns: plane rotations J
// applied on the right make the columns of M = R J mutually orthogonal, so
// M = U Sigma with sigma_k = ||M_k||, and V = J.  The rotations are
// accumulated, and P = J Sigma^{-1} is formed from them rather than from the
// normalised columns: R P = M Sigma^{-1} then has orthonormal columns to the
// stopping tolerance however wide the spread of sigma, so SA P = Q U keeps the
// conditioning Thm 3.4 relies on.
//
// Ordering: the round-robin (circle) schedule over N = n rounded up to even
// columns; in each of the N - 1 steps of a sweep the N / 2 pairs are disjoint,
// one block per pair, and every pair meets once per sweep.  A pair (p, q) is
// rotated when |m_p . m_q| > tol ||m_p|| ||m_q||; the sweeps stop when none is.
//
// Layout: M and J column-major (column k contiguous, ld = ldm), so a block
// reads and writes two contiguous columns of each; float64 throughout.
#include <cmath>
#include <cstring>

#include "common.h"

namespace rfmls {
namespace {

// out[c * ldo + r] = in[r * ldi + c] * (rowscale ? rowscale[r] : 1), an LDS-tiled
// transpose of a rows x cols matrix
constexpr int kTr = 32;
__global__ void __launch_bounds__(kTr * 8)
    k_transpose_scale(const double* __restrict__ in, int64_t ldi, int64_t rows, int64_t cols,
                      const double* __restrict__ rowscale, double* __restrict__ out, int64_t ldo) {
  __shared__ double t[kTr][kTr + 1];
  const int64_t r0 = (int64_t)blockIdx.y * kTr, c0 = (int64_t)blockIdx.x * kTr;
  const int tx = threadIdx.x % kTr, ty = threadIdx.x / kTr;
  for (int k = ty; k < kTr; k += 8) {
    const int64_t r = r0 + k, c = c0 + tx;
    double v = 0.0;
    if (r < rows && c < cols) v = in[r * ldi + c] * (rowscale ? rowscale[r] : 1.0);
    t[k][tx] = v;
  }
  __syncthreads();
  for (int k = ty; k < kTr; k += 8) {
    const int64_t c = c0 + k, r = r0 + tx;
    if (r < rows && c < cols) out[c * ldo + r] = t[tx][k];
  }
}

__global__ void k_eye_cols(double* __restrict__ J, int64_t n, int64_t ldm) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * ldm;
       e += (int64_t)gridDim.x * blockDim.x)
    J[e] = (e / ldm == e % ldm) ? 1.0 : 0.0;
}

// counters of one sweep: [0] = bits of the largest |cos| met, [1] = rotations
__global__ void k_zero_counters(unsigned long long* ctr) {
  if (threadIdx.x < 2) ctr[threadIdx.x] = 0ull;
}

// column p of step t in the circle schedule: slot 0 stays, the others turn
__device__ __forceinline__ int64_t circle(int64_t slot, int64_t t, int64_t N) {
  return slot == 0 ? 0 : (slot - 1 + t) % (N - 1) + 1;
}

// One step of a sweep: block k rotates the pair (circle(k), circle(N-1-k)).
// Each of the NT threads holds E rows of both columns in registers.
template <int NT, int E>
__global__ void __launch_bounds__(NT)
    k_jacobi_step(double* __restrict__ M, double* __restrict__ J, int64_t n, int64_t ldm, int64_t N,
                  int64_t t, double tol, unsigned long long* __restrict__ ctr) {
  __shared__ double red[3][NT / 64];
  const int64_t p = circle(blockIdx.x, t, N), q = circle(N - 1 - blockIdx.x, t, N);
  if (p >= n || q >= n) return;  // the padding column of an odd n
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double* mp = M + p * ldm;
  double* mq = M + q * ldm;
  double a[E], b[E];
  double aa = 0.0, bb = 0.0, ab = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int64_t i = tid + (int64_t)e * NT;
    a[e] = i < n ? mp[i] : 0.0;
    b[e] = i < n ? mq[i] : 0.0;
    aa += a[e] * a[e];
    bb += b[e] * b[e];
    ab += a[e] * b[e];
  }
  aa = wave_sum(aa);
  bb = wave_sum(bb);
  ab = wave_sum(ab);
  if (lane == 0) {
    red[0][w] = aa;
    red[1][w] = bb;
    red[2][w] = ab;
  }
  __syncthreads();
  aa = bb = ab = 0.0;
#pragma unroll
  for (int k = 0; k < NT / 64; ++k) {
    aa += red[0][k];
    bb += red[1][k];
    ab += red[2][k];
  }
  // |cos| of the angle between the columns (uniform over the block)
  const double den = sqrt(aa) * sqrt(bb);
  const double rel = den > 0.0 ? fabs(ab) / den : 0.0;
  if (tid == 0 && rel > 0.0) atomicMax(&ctr[0], (unsigned long long)__double_as_longlong(rel));
  if (!(rel > tol)) return;
  if (tid == 0) atomicAdd(&ctr[1], 1ull);
  // rotation [c s; -s c] on (m_p, m_q) that zeroes m_p . m_q:
  // zeta = (||m_q||^2 - ||m_p||^2) / (2 m_p . m_q), t the root of smaller
  // magnitude of t^2 + 2 zeta t - 1 = 0
  const double zeta = (bb - aa) / (2.0 * ab);
  const double az = fabs(zeta);
  const double dz = az > 1.0 ? az * (1.0 + sqrt(1.0 + 1.0 / (az * az))) : az + sqrt(1.0 + az * az);
  const double tn = (zeta >= 0.0 ? 1.0 : -1.0) / dz;
  const double cs = 1.0 / sqrt(1.0 + tn * tn), sn = cs * tn;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int64_t i = tid + (int64_t)e * NT;
    if (i < n) {
      mp[i] = cs * a[e] - sn * b[e];
      mq[i] = sn * a[e] + cs * b[e];
    }
  }
  double* jp = J + p * ldm;
  double* jq = J + q * ldm;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int64_t i = tid + (int64_t)e * NT;
    a[e] = i < n ? jp[i] : 0.0;
    b[e] = i < n ? jq[i] : 0.0;
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int64_t i = tid + (int64_t)e * NT;
    if (i < n) {
      jp[i] = cs * a[e] - sn * b[e];
      jq[i] = sn * a[e] + cs * b[e];
    }
  }
}

// sigma[k] = ||M_k|| (fixed-order block sum), one block per column
__global__ void __launch_bounds__(256)
    k_col_norms(const double* __restrict__ M, int64_t n, int64_t ldm, double* __restrict__ sigma) {
  __shared__ double scratch[256 / 64];
  const int64_t k = blockIdx.x;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += M[k * ldm + i] * M[k * ldm + i];
  s = block_sum(s, scratch);
  if (threadIdx.x == 0) sigma[k] = sqrt(s);
}

typedef void (*StepFn)(double*, double*, int64_t, int64_t, int64_t, int64_t, double,
                       unsigned long long*);

// (threads, rows per thread) for columns of length n: every row in a register
struct StepShape {
  int nt;
  StepFn fn;
};
bool pick_step(int64_t n, StepShape* out) {
  if (n <= 256) *out = {256, k_jacobi_step<256, 1>};
  else if (n <= 512) *out = {256, k_jacobi_step<256, 2>};
  else if (n <= 1024) *out = {256, k_jacobi_step<256, 4>};
  else if (n <= 2048) *out = {256, k_jacobi_step<256, 8>};
  else if (n <= 4096) *out = {256, k_jacobi_step<256, 16>};
  else if (n <= 8192) *out = {1024, k_jacobi_step<1024, 8>};
  else if (n <= 16384) *out = {1024, k_jacobi_step<1024, 16>};
  else return false;
  return true;
}

}  // namespace

int64_t svd_max_n() { return 16384; }

rfmls_status run_build_svd_precond(rfmls_handle* h, int64_t n, const double* SA, int64_t ld,
                                   rfmls_dtype store, double rcond, int max_sweeps,
                                   rfmls_precond_t* P) {
  StepShape sh;
  if (!pick_step(n, &sh))
    return fail(h, RFMLS_E_ARG, "SVD preconditioner: n = %lld exceeds %lld", (long long)n,
                (long long)svd_max_n());
  hipStream_t st = h->stream;
  P->n = n;
  P->nt = (n + kTile - 1) / kTile;
  P->store = store;
  P->full = 1;
  // R (normalised, row-major) kept for export, as for the QR preconditioner
  RFMLS_CHECK(run_extract_R(h, n, SA, ld, P));
  const int64_t ldm = (n + 31) / 32 * 32;  // 256-byte aligned columns
  const int64_t N = n + (n & 1);
  void* pw;
  RFMLS_CHECK(workspace(h, WS_SVD, sizeof(double) * (2 * (size_t)n * ldm + (size_t)n) + 64, &pw));
  double* Mc = (double*)pw;
  double* Jc = Mc + (size_t)n * ldm;
  double* d = Jc + (size_t)n * ldm;
  unsigned long long* ctr = (unsigned long long*)(d + n);
  RFMLS_HIP(h, hipMalloc(&P->sigma, sizeof(double) * (size_t)n));
  {
    dim3 g(ceil_div(n, kTr), ceil_div(n, kTr));
    hipLaunchKernelGGL(k_transpose_scale, g, dim3(kTr * 8), 0, st, (const double*)P->Rdense, n, n, n,
                       (const double*)nullptr, Mc, ldm);
    hipLaunchKernelGGL(k_eye_cols, dim3(ceil_div(n * ldm, 256) < 4096 ? ceil_div(n * ldm, 256) : 4096),
                       dim3(256), 0, st, Jc, n, ldm);
    RFMLS_HIP(h, hipGetLastError());
  }
  // stopping tolerance on |cos(m_p, m_q)|: a few units of the rounding of the
  // blocked dot products (LAPACK's one-sided Jacobi takes sqrt(n) eps)
  const double eps = 2.220446049250313e-16;
  const double tol = (sqrt((double)n) > 8.0 ? sqrt((double)n) : 8.0) * eps;
  unsigned long long* pin = (unsigned long long*)((char*)h->pinned + 3072);
  P->sweeps = 0;
  P->off = 0.0;
  bool converged = false;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, st, ctr);
    {
      // algorithmic bytes of a sweep: both columns of M read for every pair,
      // and for each pair that rotates M's two written and J's two read and
      // written (set below from the sweep's rotation count)
      Trace tr(h, "svd_jacobi_sweep", 0.0, 0.0);
      for (int64_t t = 0; t < N - 1; ++t)
        hipLaunchKernelGGL(sh.fn, dim3((unsigned)(N / 2)), dim3(sh.nt), 0, st, Mc, Jc, n, ldm, N, t, tol,
                           ctr);
    }
    RFMLS_HIP(h, hipGetLastError());
    RFMLS_HIP(h, hipMemcpyAsync(pin, ctr, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    RFMLS_HIP(h, hipStreamSynchronize(st));
    double off;
    const unsigned long long bits = pin[0];
    memcpy(&off, &bits, sizeof(off));
    if (h->trace && !h->trace_recs.empty()) {
      const double pairs = (double)(N / 2) * (double)(N - 1), rot = (double)pin[1];
      h->trace_recs.back().bytes = 8.0 * (double)n * (2.0 * pairs + 6.0 * rot);
      h->trace_recs.back().flops = (double)n * (6.0 * pairs + 12.0 * rot);
    }
    P->sweeps = sweep + 1;
    P->off = off;
    if (!(off == off)) return fail(h, RFMLS_E_BREAKDOWN, "SVD preconditioner: non-finite column products");
    if (pin[1] == 0ull) {
      converged = true;
      break;
    }
  }
  // singular values, rank and P = J diag(d), d_k = 1 / sigma_k above the threshold, else 0
  hipLaunchKernelGGL(k_col_norms, dim3((unsigned)n), dim3(256), 0, st, (const double*)Mc, n, ldm, P->sigma);
  std::vector<double> sig(n), dh(n);
  RFMLS_HIP(h, hipMemcpyAsync(sig.data(), P->sigma, sizeof(double) * n, hipMemcpyDeviceToHost, st));
  RFMLS_HIP(h, hipStreamSynchronize(st));
  double smax = 0.0;
  for (double v : sig) {
    if (!(v == v)) return fail(h, RFMLS_E_BREAKDOWN, "SVD preconditioner: non-finite singular value");
    smax = v > smax ? v : smax;
  }
  if (rcond <= 0.0) rcond = (double)n * 1.1102230246251565e-16;
  const double thr = rcond * smax;
  int64_t r = 0;
  for (int64_t k = 0; k < n; ++k) {
    const bool keep = smax > 0.0 && sig[k] > thr;
    dh[k] = keep ? 1.0 / sig[k] : 0.0;
    r += keep ? 1 : 0;
  }
  P->rank = r;
  if (r == 0) return fail(h, RFMLS_E_RANK, "SVD preconditioner: every singular value is below rcond * sigma_1");
  RFMLS_HIP(h, hipMemcpyAsync(d, dh.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
  void* px;
  RFMLS_CHECK(workspace(h, WS_TRSM, sizeof(double) * (size_t)n * (size_t)n, &px));
  double* Pd = (double*)px;
  {
    // Pd[i][k] = J[i][k] d[k]: J is stored as columns, so row k of Jc is column k of J
    dim3 g(ceil_div(n, kTr), ceil_div(n, kTr));
    hipLaunchKernelGGL(k_transpose_scale, g, dim3(kTr * 8), 0, st, (const double*)Jc, ldm, n, n,
                       (const double*)d, Pd, n);
    RFMLS_HIP(h, hipGetLastError());
  }
  // dh must stay alive until the upload above has been consumed
  RFMLS_HIP(h, hipStreamSynchronize(st));
  RFMLS_CHECK(pack_precond(h, P, Pd));
  if (!converged)
    return fail(h, RFMLS_W_NOCONV, "SVD preconditioner: %d Jacobi sweeps left |cos| = %.3e > %.3e",
                P->sweeps, P->off, tol);
  return RFMLS_OK;
}

}  // namespace rfmls
