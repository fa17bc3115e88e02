// CSSVDP-LSQR preconditioner (Alg. 2 step 3): the truncated SVD of the sketch
// SA through its R factor (SA = Q R, so SA and R share Sigma and V), and
// P = V_r Sigma_r^{-1} with r = #{sigma_i > rcond sigma_1} (Sec. 3.2: the
// LAPACK-style threshold, rcond times the largest singular value).
//
// SVD of R by one-sided (Hestenes) Jacobi, preconditioned by a second QR
// (Drmac and Veselic): R^T = Q2 R2, and plane rotations J applied on the right
// make the columns of M = R2^T J mutually orthogonal, so M = U Sigma with
// sigma_k = ||M_k||, and R = U Sigma (Q2 J)^T: V = Q2 J.  The rotations are
// accumulated, and P = Q2 J Sigma^{-1} is formed from them rather than from the
// normalised columns: R P = M Sigma^{-1} then has orthonormal columns to the
// stopping tolerance however wide the spread of sigma, so SA P = Q U keeps the
// conditioning Thm 3.4 relies on.
//
// Ordering: columns in groups of b (4 for n <= 4096); the round-robin (circle)
// schedule pairs the groups, Gp = the group count rounded up to even, so each
// of the Gp - 1 steps of a sweep gives Gp / 2 disjoint group pairs, one block
// each, and every pair of columns from two groups meets once per sweep.  A
// block rotates all pairs of its 2b columns in registers before it writes
// them back, so a step passes over M and J once for (2b)(2b-1)/2 rotations per
// block instead of one; inside the block the pairs go in 2b - 1 rounds of b
// disjoint pairs, one block reduction per round.  A pair (p, q) is rotated when
// |m_p . m_q| > tol ||m_p|| ||m_q||; the sweeps stop when none is.
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

// M[k ldm + i] = R2[k][i] for i >= k, else 0: column k of L = R2^T is row k of
// the upper-triangular R2 (row-major, ld2)
__global__ void k_upper_rows_to_cols(const double* __restrict__ R2, int64_t ld2, int64_t n,
                                     double* __restrict__ M, int64_t ldm) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = e / n, i = e % n;
    M[k * ldm + i] = i >= k ? R2[k * ld2 + i] : 0.0;
  }
}

__global__ void k_eye_cols(double* __restrict__ J, int64_t n, int64_t ldm) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * ldm;
       e += (int64_t)gridDim.x * blockDim.x)
    J[e] = (e / ldm == e % ldm) ? 1.0 : 0.0;
}

// counters of one sweep: [0] = bits of the largest |cos| met, [1] = rotations,
// [2] = blocks that rotated (and so wrote their columns of M and J)
__global__ void k_zero_counters(unsigned long long* ctr) {
  if (threadIdx.x < 3) ctr[threadIdx.x] = 0ull;
}

// group of step t at slot `slot` in the circle schedule over Gp groups: slot 0
// stays, the others turn
__device__ __forceinline__ int64_t circle(int64_t slot, int64_t t, int64_t Gp) {
  return slot == 0 ? 0 : (slot - 1 + t) % (Gp - 1) + 1;
}

// Wavefront sum of a double on the DPP path (no LDS traffic): rotations by 1, 2,
// 4 and 8 lanes inside each 16-lane row leave every lane with its row's sum,
// and the four row sums (lanes 0, 16, 32, 48) are added in a fixed order, so
// the result is the same on every lane and run to run.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_read(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
  constexpr int kRowRor = 0x120;  // DPP row_ror:n = 0x120 + n
  v += dpp_move<kRowRor + 1>(v);
  v += dpp_move<kRowRor + 2>(v);
  v += dpp_move<kRowRor + 4>(v);
  v += dpp_move<kRowRor + 8>(v);
  return (lane_read(v, 0) + lane_read(v, 16)) + (lane_read(v, 32) + lane_read(v, 48));
}

// local column of slot i in round r of the circle schedule over B2 columns
__host__ __device__ constexpr int lcol(int i, int r, int B2) { return i == 0 ? 0 : (i - 1 + r) % (B2 - 1) + 1; }

// One step of a sweep over column groups of b = B2 / 2: block k takes the
// groups (circle(k), circle(Gp-1-k)) and rotates every pair of its B2 columns,
// all held in registers (thread tid has rows tid + e NT, e < E).  The pairs are
// taken in B2 - 1 rounds of B2 / 2 disjoint pairs (the circle schedule again),
// so the products of a round's pairs share one block reduction; the rotations
// are then replayed, round by round, on the same columns of J.  Over a sweep
// every pair of columns from different groups meets once, pairs inside a
// group at every step.  A column index past n (the ragged last group, the
// padding group of an odd group count) is a zero column and never rotates.
template <int NT, int E, int B2>
__global__ void __launch_bounds__(NT)
    k_jacobi_step(double* __restrict__ M, double* __restrict__ J, int64_t n, int64_t ldm, int64_t Gp,
                  int64_t t, double tol, unsigned long long* __restrict__ ctr) {
  constexpr int b = B2 / 2;
  constexpr int H = B2 / 2;       // pairs per round
  constexpr int NR = B2 - 1;      // rounds
  constexpr int NW = NT / 64;     // wavefronts
  __shared__ double red[3 * H][NW];
  __shared__ double rot[NR][H][2];
  const int64_t g1 = circle(blockIdx.x, t, Gp), g2 = circle(Gp - 1 - blockIdx.x, t, Gp);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int64_t col[B2];
#pragma unroll
  for (int c = 0; c < B2; ++c) {
    const int64_t k = c < b ? g1 * b + c : g2 * b + (c - b);
    col[c] = k < n ? k : -1;
  }
  // column k of M starts at the block-uniform M + k ldm; a thread's rows are
  // 32-bit offsets tid + e NT from it (n < 2^31), so every access is a scalar
  // base plus a small per-thread offset and no 64-bit per-element address
  // has to stay live across the rotations
  double x[B2][E];
#pragma unroll
  for (int c = 0; c < B2; ++c) {
    const double* mc = M + (col[c] >= 0 ? col[c] : 0) * ldm;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const unsigned i = (unsigned)tid + (unsigned)(e * NT);
      x[c][e] = (col[c] >= 0 && i < n) ? mc[i] : 0.0;
    }
  }
  double offmax = 0.0;
  int nrot = 0;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    __syncthreads();  // the previous round's reads of red are done
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const int p = lcol(k, r, B2), q = lcol(B2 - 1 - k, r, B2);
      double aa = 0.0, bb = 0.0, ab = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        aa += x[p][e] * x[p][e];
        bb += x[q][e] * x[q][e];
        ab += x[p][e] * x[q][e];
      }
      aa = wave_sum_dpp(aa);
      bb = wave_sum_dpp(bb);
      ab = wave_sum_dpp(ab);
      if (lane == 0) {
        red[3 * k][w] = aa;
        red[3 * k + 1][w] = bb;
        red[3 * k + 2][w] = ab;
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const int p = lcol(k, r, B2), q = lcol(B2 - 1 - k, r, B2);
      double aa = 0.0, bb = 0.0, ab = 0.0;
#pragma unroll
      for (int u = 0; u < NW; ++u) {
        aa += red[3 * k][u];
        bb += red[3 * k + 1][u];
        ab += red[3 * k + 2][u];
      }
      // |cos| of the angle between the columns (uniform over the block)
      const double den = sqrt(aa) * sqrt(bb);
      const double rel = den > 0.0 ? fabs(ab) / den : 0.0;
      offmax = rel > offmax ? rel : offmax;
      double cs = 1.0, sn = 0.0;
      if (rel > tol) {
        // rotation [c s; -s c] on (x_p, x_q) that zeroes x_p . x_q:
        // zeta = (||x_q||^2 - ||x_p||^2) / (2 x_p . x_q), t the root of smaller
        // magnitude of t^2 + 2 zeta t - 1 = 0
        const double zeta = (bb - aa) / (2.0 * ab);
        const double az = fabs(zeta);
        const double dz = az > 1.0 ? az * (1.0 + sqrt(1.0 + 1.0 / (az * az))) : az + sqrt(1.0 + az * az);
        const double tn = (zeta >= 0.0 ? 1.0 : -1.0) / dz;
        cs = 1.0 / sqrt(1.0 + tn * tn);
        sn = cs * tn;
        ++nrot;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const double xp = x[p][e], xq = x[q][e];
          x[p][e] = cs * xp - sn * xq;
          x[q][e] = sn * xp + cs * xq;
        }
      }
      if (tid == 0) {
        rot[r][k][0] = cs;
        rot[r][k][1] = sn;
      }
    }
  }
  if (tid == 0) {
    if (offmax > 0.0) atomicMax(&ctr[0], (unsigned long long)__double_as_longlong(offmax));
    if (nrot) {
      atomicAdd(&ctr[1], (unsigned long long)nrot);
      atomicAdd(&ctr[2], 1ull);
    }
  }
  if (nrot == 0) return;  // uniform: nothing moved in this block
#pragma unroll
  for (int c = 0; c < B2; ++c) {
    double* mc = M + (col[c] >= 0 ? col[c] : 0) * ldm;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const unsigned i = (unsigned)tid + (unsigned)(e * NT);
      if (col[c] >= 0 && i < n) mc[i] = x[c][e];
    }
  }
  // the same rotations, in the same order, on J's columns
#pragma unroll
  for (int c = 0; c < B2; ++c) {
    const double* jc = J + (col[c] >= 0 ? col[c] : 0) * ldm;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const unsigned i = (unsigned)tid + (unsigned)(e * NT);
      x[c][e] = (col[c] >= 0 && i < n) ? jc[i] : 0.0;
    }
  }
  __syncthreads();  // rot[] complete
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const int p = lcol(k, r, B2), q = lcol(B2 - 1 - k, r, B2);
      const double cs = rot[r][k][0], sn = rot[r][k][1];
      if (sn != 0.0) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const double xp = x[p][e], xq = x[q][e];
          x[p][e] = cs * xp - sn * xq;
          x[q][e] = sn * xp + cs * xq;
        }
      }
    }
#pragma unroll
  for (int c = 0; c < B2; ++c) {
    double* jc = J + (col[c] >= 0 ? col[c] : 0) * ldm;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const unsigned i = (unsigned)tid + (unsigned)(e * NT);
      if (col[c] >= 0 && i < n) jc[i] = x[c][e];
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

// (threads, columns per block) for columns of length n: every row of the
// block's columns in a register (at most 32 doubles per thread at 1024
// threads and 64 at 512, beside the round's partial sums; more spills)
struct StepShape {
  int nt, b2;
  StepFn fn;
};
bool pick_step(int64_t n, StepShape* out) {
  if (n <= 256) *out = {256, 8, k_jacobi_step<256, 1, 8>};
  else if (n <= 512) *out = {256, 8, k_jacobi_step<256, 2, 8>};
  else if (n <= 1024) *out = {256, 8, k_jacobi_step<256, 4, 8>};
  else if (n <= 2048) *out = {512, 8, k_jacobi_step<512, 4, 8>};
  else if (n <= 4096) *out = {512, 8, k_jacobi_step<512, 8, 8>};
  else if (n <= 8192) *out = {1024, 4, k_jacobi_step<1024, 8, 4>};
  else if (n <= 16384) *out = {1024, 2, k_jacobi_step<1024, 16, 2>};
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
  // column groups of b = sh.b2 / 2, rounded up to an even count
  const int64_t gb = sh.b2 / 2;
  const int64_t Gn = (n + gb - 1) / gb;
  const int64_t Gp = Gn + (Gn & 1);
  void* pw;
  RFMLS_CHECK(workspace(h, WS_SVD, sizeof(double) * (2 * (size_t)n * ldm + (size_t)n) + 64, &pw));
  double* Mc = (double*)pw;
  double* Jc = Mc + (size_t)n * ldm;
  double* d = Jc + (size_t)n * ldm;
  unsigned long long* ctr = (unsigned long long*)(d + n);
  RFMLS_HIP(h, hipMalloc(&P->sigma, sizeof(double) * (size_t)n));
  // Preconditioning of the sweeps (Drmac and Veselic): the QR of R^T,
  // R^T = Q2 R2, gives R = R2^T Q2^T; Jacobi then runs on the columns of
  // L = R2^T (the rows of R2): L J = U Sigma, so R's right singular vectors are
  // V = Q2 J.  The QR's rotation towards triangular form leaves L closer to
  // orthogonal columns, and the cyclic sweeps need about a third fewer passes.
  const int64_t ld2 = (n + 127) / 128 * 128;
  void* p2;
  RFMLS_CHECK(workspace(h, WS_SVD2, sizeof(double) * ((size_t)n * ld2 + (size_t)n), &p2));
  double* Rt = (double*)p2;
  double* tau2 = Rt + (size_t)n * ld2;
  {
    dim3 g(ceil_div(n, kTr), ceil_div(n, kTr));
    hipLaunchKernelGGL(k_transpose_scale, g, dim3(kTr * 8), 0, st, (const double*)P->Rdense, n, n, n,
                       (const double*)nullptr, Rt, ld2);
    RFMLS_HIP(h, hipGetLastError());
  }
  RFMLS_CHECK(run_qr(h, n, n, ld2, RFMLS_F64, Rt, ld2, tau2));
  {
    int flag = 0;
    RFMLS_HIP(h, hipMemcpyAsync(&flag, h->dev_flags, sizeof(int), hipMemcpyDeviceToHost, st));
    RFMLS_HIP(h, hipStreamSynchronize(st));
    if (flag) {
      (void)hipMemset(h->dev_flags, 0, sizeof(int));
      return fail(h, RFMLS_E_HIP, "SVD preconditioner: QR panel hand-over timed out");
    }
  }
  {
    const unsigned g = ceil_div(n * n, 256) < 4096 ? ceil_div(n * n, 256) : 4096;
    hipLaunchKernelGGL(k_upper_rows_to_cols, dim3(g), dim3(256), 0, st, (const double*)Rt, ld2, n, Mc, ldm);
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
      for (int64_t t = 0; t < Gp - 1; ++t)
        hipLaunchKernelGGL(sh.fn, dim3((unsigned)(Gp / 2)), dim3(sh.nt), 0, st, Mc, Jc, n, ldm, Gp, t, tol,
                           ctr);
    }
    RFMLS_HIP(h, hipGetLastError());
    RFMLS_HIP(h, hipMemcpyAsync(pin, ctr, 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    RFMLS_HIP(h, hipStreamSynchronize(st));
    double off;
    const unsigned long long bits = pin[0];
    memcpy(&off, &bits, sizeof(off));
    if (h->trace && !h->trace_recs.empty()) {
      // algorithmic bytes of the sweep: every step reads all n columns of M;
      // each block that rotated writes its 2b columns of M back and reads and
      // writes those of J.  Flops: 6 per row for a pair's three products, 12
      // for a rotation of M's and J's two columns.
      const double steps = (double)(Gp - 1), pairs = steps * (double)(Gp / 2) * (sh.b2 * (sh.b2 - 1) / 2);
      const double rot = (double)pin[1], rblocks = (double)pin[2];
      h->trace_recs.back().bytes = 8.0 * (double)n * ((double)n * steps + 3.0 * sh.b2 * rblocks);
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
  // P = V diag(d) = Q2 (J diag(d))
  RFMLS_CHECK(apply_householder(h, Rt, ld2, n, n, tau2, Pd, n, n));
  // dh must stay alive until the upload above has been consumed
  RFMLS_HIP(h, hipStreamSynchronize(st));
  RFMLS_CHECK(pack_precond(h, P, Pd));
  if (!converged)
    return fail(h, RFMLS_W_NOCONV, "SVD preconditioner: %d Jacobi sweeps left |cos| = %.3e > %.3e",
                P->sweeps, P->off, tol);
  return RFMLS_OK;
}

}  // namespace rfmls
