// Blocked Householder QR of the sketch SA (s x n, row-major, in place):
// Alg. 1 step 3.  Only R is needed; Q is never formed.
//
// Two levels of blocking.  Outer blocks of kOuter = 256 columns are factored
// panel by panel (kMaxNb = 64 columns each); the trailing matrix right of an
// outer block is then updated once, with K = 256, which keeps that update --
// most of the flops -- on the matrix cores instead of bound by HBM traffic.
//
// Inner panel at column p0 (M = s - p0 rows):
//   k_qr_panel   unblocked Householder on the M x 64 panel, spread over G
//                co-resident workgroups (rows held in LDS); each column needs one
//                grid-wide reduction of sigma = sum_{i>j} a_ij^2, d_c = sum_{i>j}
//                a_ij a_ic and the pivot row, after which every workgroup forms
//                the same reflector (LAPACK dlarfg convention: beta = -sign(alpha)
//                ||(alpha, x)||, tau = (beta - alpha)/beta, v = [1; x/(alpha-beta)])
//                and applies it to its rows;
//   inside the outer block: W = V^T [V | C] (split-K GEMM), T from V^T V
//                (dlarft, forward, columnwise), C <- C - V (T^T W).
// Outer block at column k0 (M0 = s - k0 rows, V_o = its 256 Householder vectors):
//   W = V_o^T [V_o | C] (split-K GEMM; the first 256 columns are the Gram V_o^T V_o),
//   T_o from the Gram: diagonal 64-blocks by dlarft, off-diagonal blocks by
//   T_o[:q, q] = -T_o[:q, :q] (V_:q^T V_q) T_qq,  then C <- C - V_o (T_o^T W_C).
// All reductions run in a fixed order, so the factorisation is deterministic.
#include "common.h"
#include "gemm.h"

namespace rfmls {
namespace {

constexpr int kMaxNb = 64;

// Grid-wide sum of one payload vector per block, returned to every block.
// Two levels keep both the serialised atomics and the reads short: blocks are
// grouped in clusters of kCluster; the last block to arrive in a cluster sums
// its cluster's payloads (in block order) and arrives at the global counter;
// the last cluster leader sums the cluster sums (in cluster order), publishes
// the result and bumps a generation word that every block waits for.  All
// sums run in a fixed order, so every block receives bit-identical values.
//   pw   [G][kPayload]      block payloads (written by the caller before the call)
//   cw   [nclus][kPayload]  cluster sums
//   out  [2][kPayload]      published result, double-buffered by epoch parity
//   cnt  [(nclus + 2) * kBarrierStride]  cluster counters, global counter and
//                           generation word, each on its own cache line
// Counters only grow; epoch e (0, 1, ...) numbers the calls within one launch.
//
// Memory ordering: every word that crosses blocks (payloads, cluster sums, the
// result, counters) is written and read with relaxed agent-scope atomics,
// which are coherent across the XCDs' separate L2 caches; each writer waits
// for its stores to complete (s_waitcnt) before the counter update or flag
// store that publishes them.  Release/acquire fences would do the same but
// also write back and invalidate the whole L2 of the XCD at every step, which
// made the reduction cost grow linearly with the number of blocks.
constexpr int kCluster = 16;
constexpr int kPayload = 2 * kMaxNb;

__device__ __forceinline__ void st_coh(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_coh(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// wait until every memory operation this thread issued has completed
__device__ __forceinline__ void wait_stores() { __builtin_amdgcn_s_waitcnt(0); }

__device__ bool grid_allreduce(const double* pw, double* cw, double* out, unsigned* cnt, int lo,
                               int hi, unsigned epoch, double* red, int* err) {
  const int G = gridDim.x;
  const int g = blockIdx.x;
  const int nclus = (G + kCluster - 1) / kCluster;
  const int cl = g / kCluster;
  const int csize = (cl == nclus - 1) ? G - cl * kCluster : kCluster;
  unsigned* gcount = cnt + (int64_t)nclus * kBarrierStride;
  unsigned* gen = cnt + (int64_t)(nclus + 1) * kBarrierStride;
  __shared__ int role;  // 0: wait, 1: cluster leader, 2: global leader
  __shared__ int ok;
  wait_stores();  // this block's payload stores (st_coh by the caller) are complete
  __syncthreads();
  if (threadIdx.x == 0) {
    ok = 1;
    const unsigned old = __hip_atomic_fetch_add(&cnt[(int64_t)cl * kBarrierStride], 1u,
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    role = (old == (epoch + 1) * (unsigned)csize - 1u) ? 1 : 0;
  }
  __syncthreads();
  if (role == 1) {
    for (int k = lo + (int)threadIdx.x; k < hi; k += blockDim.x) {
      // issue all loads before summing (one memory round trip, not kCluster)
      double v[kCluster];
#pragma unroll
      for (int q = 0; q < kCluster; ++q)
        v[q] = q < csize ? ld_coh(&pw[(int64_t)(cl * kCluster + q) * kPayload + k]) : 0.0;
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < kCluster; ++q) s += v[q];
      st_coh(&cw[(int64_t)cl * kPayload + k], s);
    }
    wait_stores();
    __syncthreads();
    if (threadIdx.x == 0) {
      const unsigned old =
          __hip_atomic_fetch_add(gcount, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (old == (epoch + 1) * (unsigned)nclus - 1u) role = 2;
    }
    __syncthreads();
    if (role == 2) {
      double* o = out + (int64_t)(epoch & 1u) * kPayload;
      for (int k = lo + (int)threadIdx.x; k < hi; k += blockDim.x) {
        double s = 0.0;
        for (int c0 = 0; c0 < nclus; c0 += kCluster) {
          double v[kCluster];
#pragma unroll
          for (int q = 0; q < kCluster; ++q)
            v[q] = c0 + q < nclus ? ld_coh(&cw[(int64_t)(c0 + q) * kPayload + k]) : 0.0;
#pragma unroll
          for (int q = 0; q < kCluster; ++q) s += v[q];
        }
        st_coh(&o[k], s);
      }
      wait_stores();
      __syncthreads();
      if (threadIdx.x == 0)
        __hip_atomic_store(gen, epoch + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (threadIdx.x == 0) {
    int spins = 0;
    while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch + 1u) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1 << 26)) {
        ok = 0;
        atomicExch(err, 1);
        break;
      }
    }
  }
  __syncthreads();
  if (!ok) return false;
  const double* o = out + (int64_t)(epoch & 1u) * kPayload;
  for (int k = lo + (int)threadIdx.x; k < hi; k += blockDim.x) red[k] = ld_coh(&o[k]);
  __syncthreads();
  return true;
}

// Payload of column j (length 2 (nb - j)): entry c - j for c in [j, nb) holds
// sigma (c == j) or d_c (c > j); entry (nb - j) + (c - j) holds the pivot row
// value a_jc (only the block owning row j contributes, the others add 0).
//
// Each block (NT threads, NG = NT / 64 wavefronts) owns rpw <= NG Q consecutive
// panel rows and keeps them in registers: thread (c = lane, rg = wavefront)
// holds a[q] = P[r0 + rg + NG q][c].
// All threads of a wavefront hold the same rows, so column j reaches every
// lane of the wavefront by v_readlane from lane j (scalar registers, no LDS).
// Few, large blocks keep the per-column grid reduction short (its cost grows
// with the number of blocks).

__device__ __forceinline__ double lane_value(double v, int lane) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double lane_value(float v, int lane) {
  return (double)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

template <typename T, int Q, int NT>
__global__ void __launch_bounds__(NT)
    k_qr_panel(T* __restrict__ P, int64_t ld, int64_t M, int nb, int rpw, T* __restrict__ tau,
               double* __restrict__ ws, unsigned* __restrict__ cnt, int* __restrict__ err) {
  constexpr int kPanelGroups = NT / 64;
  __shared__ double red[kPayload];              // reduced payload
  __shared__ double grp[kPanelGroups][kMaxNb];  // per row-group partials
  __shared__ double piv[kMaxNb];                // pivot row (owner block)
  const int G = gridDim.x;
  const int g = blockIdx.x;
  const int tid = threadIdx.x;
  const int c = tid & 63;
  const int rg = tid >> 6;  // wavefront index: uniform within a wavefront
  const int64_t r0 = (int64_t)g * rpw;
  const int nr = (int)(M - r0 < rpw ? (M - r0 > 0 ? M - r0 : 0) : rpw);
  const int nclus = (G + kCluster - 1) / kCluster;
  double* pw = ws;                               // [G][kPayload]
  double* cw = ws + (int64_t)G * kPayload;       // [nclus][kPayload]
  double* out = cw + (int64_t)nclus * kPayload;  // [2][kPayload]

  // rows beyond the panel are held as zeros and contribute nothing
  T a[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int li = rg + kPanelGroups * q;
    a[q] = (li < nr && c < nb) ? P[(r0 + li) * ld + c] : T(0);
  }

  for (int j = 0; j < nb; ++j) {
    // Only block 0 (rows 0 .. rpw-1, rpw >= 128 >= nb) holds rows i <= j; in
    // every other block all rows take part.  li > j is uniform per wavefront.
    const bool top = (g == 0);
    if (top && rg == (j % kPanelGroups)) {  // pivot row j lives in this wavefront
      const int qj = j / kPanelGroups;
      double pv = 0.0;
#pragma unroll
      for (int q = 0; q < Q; ++q) pv = (q == qj) ? (double)a[q] : pv;
      piv[c] = pv;
    }
    // ---- local partials over rows i > j: sum_i a_ij a_ic ----
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int li = rg + kPanelGroups * q;
      if (!top || li > j) s += lane_value(a[q], j) * (double)a[q];
    }
    grp[rg][c] = s;
    __syncthreads();
    const int L = nb - j;
    if (tid < 64 && c >= j && c < nb) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < kPanelGroups; ++q) t += grp[q][c];
      double* my = pw + (int64_t)g * kPayload;
      st_coh(&my[c - j], t);
      st_coh(&my[L + c - j], top ? piv[c] : 0.0);
    }
    if (!grid_allreduce(pw, cw, out, cnt, 0, 2 * L, (unsigned)j, red, err)) return;
    // ---- reflector (identical in every block) ----
    const double alpha = red[L];
    const double sigma = red[0];
    double beta, tj, scal;
    if (sigma == 0.0) {
      beta = alpha;
      tj = 0.0;
      scal = 0.0;
    } else {
      const double nrm = sqrt(alpha * alpha + sigma);
      beta = alpha >= 0.0 ? -nrm : nrm;
      tj = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    if (g == 0 && tid == 0) tau[j] = (T)tj;
    // ---- apply H_j to rows i >= j of columns c > j; column j becomes v ----
    const bool upd = (c > j && c < nb && tj != 0.0);
    const double f = upd ? tj * (red[L + c - j] + scal * red[c - j]) : 0.0;
    const double sf = scal * f;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int li = rg + kPanelGroups * q;
      const double vj = lane_value(a[q], j);  // read before lane j rewrites it
      if (!top || li > j) {
        if (upd) a[q] = (T)((double)a[q] - sf * vj);
        else if (c == j) a[q] = (T)(scal * vj);
      } else if (li == j) {
        if (upd) a[q] = (T)((double)a[q] - f);
        else if (c == j) a[q] = (T)beta;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int li = rg + kPanelGroups * q;
    if (li < nr && c < nb) P[(r0 + li) * ld + c] = a[q];
  }
}

// Build T (nb x nb upper triangular, row-major) of the compact-WY form
// H_1 ... H_nb = I - V T V^T from tau and the Gram V^T V = sum of nsplit
// partial slices Wz (each nb x ldw; its leading nb columns hold V^T V).
// T is assembled by doubling: starting from T_jj = tau_j, neighbouring
// diagonal blocks T_1, T_2 (b columns each) are joined by
//   T_12 = -T_1 (V_1^T V_2) T_2,
// the block form of the column recursion T[:j, j] = -tau_j T[:j, :j] V_:j^T v_j
// (Schreiber and Van Loan), with all threads working on each level.
template <typename T>
__global__ void __launch_bounds__(256)
    k_qr_buildT(const T* __restrict__ Wz, int64_t zstride, int nsplit, int64_t ldw, int nb,
                const T* __restrict__ tau, T* __restrict__ Tout, int64_t ldt) {
  __shared__ double Gm[kMaxNb][kMaxNb + 1];
  __shared__ double Tm[kMaxNb][kMaxNb + 1];
  __shared__ double Ym[kMaxNb][kMaxNb + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * nb; e += 256) {
    const int i = e / nb, k = e % nb;
    double sacc = 0.0;
    for (int z = 0; z < nsplit; ++z) sacc += (double)Wz[(int64_t)z * zstride + (int64_t)i * ldw + k];
    Gm[i][k] = sacc;
    Tm[i][k] = (i == k) ? (double)tau[i] : 0.0;
  }
  __syncthreads();
  for (int b = 1; b < nb; b *= 2) {
    const int npair = (nb + 2 * b - 1) / (2 * b);
    // Y = T_1 G_12 for every pair (rows of the first block, columns of the second)
    for (int e = tid; e < npair * b * b; e += 256) {
      const int pr = e / (b * b), r = e % (b * b);
      const int f0 = pr * 2 * b, s0 = f0 + b;
      const int i = f0 + r / b, j = s0 + r % b;
      if (j >= nb) continue;
      double acc = 0.0;
      for (int k = i; k < s0; ++k) acc += Tm[i][k] * Gm[k][j];
      Ym[i][j] = acc;
    }
    __syncthreads();
    // T_12 = -Y T_2
    for (int e = tid; e < npair * b * b; e += 256) {
      const int pr = e / (b * b), r = e % (b * b);
      const int f0 = pr * 2 * b, s0 = f0 + b;
      const int i = f0 + r / b, j = s0 + r % b;
      if (j >= nb) continue;
      double acc = 0.0;
      for (int k = s0; k <= j; ++k) acc += Ym[i][k] * Tm[k][j];
      Tm[i][j] = -acc;
    }
    __syncthreads();
  }
  for (int e = tid; e < nb * nb; e += 256) Tout[(int64_t)(e / nb) * ldt + e % nb] = (T)Tm[e / nb][e % nb];
}

// W[e] = sum_z Wz[z * zstride + e] over a contiguous range of len elements
template <typename T>
__global__ void k_sum_slices(const T* __restrict__ Wz, int64_t zstride, int nsplit, int64_t len,
                             T* __restrict__ W) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int z = 0; z < nsplit; ++z) acc += (double)Wz[(int64_t)z * zstride + e];
    W[e] = (T)acc;
  }
}

// W'[:, cols] = T^T * sum_z Wz[:, nb + cols], one block per 64 columns.
template <typename T>
__global__ void __launch_bounds__(256)
    k_qr_wp(const T* __restrict__ Wz, int64_t zstride, int nsplit, int64_t ldw, int nb, int64_t N,
            const T* __restrict__ Tm, int64_t ldt, T* __restrict__ Wp, int64_t ldwp) {
  __shared__ double Ws[kMaxNb][64 + 1];
  __shared__ double Ts[kMaxNb][kMaxNb + 1];
  const int tid = threadIdx.x;
  const int64_t c0 = (int64_t)blockIdx.x * 64;
  for (int e = tid; e < nb * nb; e += 256) Ts[e / nb][e % nb] = (double)Tm[(int64_t)(e / nb) * ldt + e % nb];
  for (int e = tid; e < nb * 64; e += 256) {
    const int i = e / 64, cc = e % 64;
    double sacc = 0.0;
    if (c0 + cc < N)
      for (int z = 0; z < nsplit; ++z)
        sacc += (double)Wz[(int64_t)z * zstride + (int64_t)i * ldw + nb + c0 + cc];
    Ws[i][cc] = sacc;
  }
  __syncthreads();
  for (int e = tid; e < nb * 64; e += 256) {
    const int i = e / 64, cc = e % 64;
    if (c0 + cc >= N) continue;
    double a = 0.0;
    for (int k = 0; k <= i; ++k) a += Ts[k][i] * Ws[k][cc];
    Wp[(int64_t)i * ldwp + c0 + cc] = (T)a;
  }
}

__global__ void k_zero_u32(unsigned* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

constexpr int64_t kOuter = 256;

// Panel launch shapes in increasing rows per block; a float64 row entry takes
// two VGPRs.  The largest shapes are the largest that compile without spills
// (NT / 256 wavefronts per SIMD).
struct PanelShape {
  int nt, q;
  const void* fn;
  int64_t rpw() const { return (int64_t)(nt / 64) * q; }
};
template <typename T>
const PanelShape* panel_shapes();
template <>
const PanelShape* panel_shapes<double>() {
  static const PanelShape s[] = {{512, 16, (const void*)k_qr_panel<double, 16, 512>},
                                 {512, 32, (const void*)k_qr_panel<double, 32, 512>},
                                 {0, 0, nullptr}};
  return s;
}
template <>
const PanelShape* panel_shapes<float>() {
  static const PanelShape s[] = {{512, 16, (const void*)k_qr_panel<float, 16, 512>},
                                 {512, 32, (const void*)k_qr_panel<float, 32, 512>},
                                 {512, 64, (const void*)k_qr_panel<float, 64, 512>},
                                 {0, 0, nullptr}};
  return s;
}

template <typename T>
GemmArgs<T> vt_gemm(T* P, int64_t ld, int64_t M, int64_t vcols, int64_t ncols, T* out,
                    int64_t ksplit) {
  // out_z = V^T [V | C] over row slices: V = the vcols Householder vectors
  // stored below the diagonal of P, C the next ncols - vcols columns
  GemmArgs<T> g;
  g.M = vcols;
  g.N = ncols;
  g.K = M;
  g.A = P;
  g.lda = ld;
  g.transA = 1;
  g.a_vmask = 1;
  g.B = P;
  g.ldb = ld;
  g.b_vcols = vcols;
  g.C = out;
  g.ldc = ncols;
  g.alpha = T(1);
  g.beta = T(0);
  g.ksplit = ksplit;
  g.c_zstride = vcols * ncols;
  return g;
}

template <typename T>
GemmArgs<T> v_update(T* P, int64_t ld, int64_t M, int64_t vcols, int64_t ncols, const T* Wp) {
  // C <- C - V Wp, C = the ncols columns right of the vcols Householder vectors
  GemmArgs<T> g;
  g.M = M;
  g.N = ncols;
  g.K = vcols;
  g.A = P;
  g.lda = ld;
  g.a_vmask = 1;
  g.B = Wp;
  g.ldb = ncols;
  g.C = P + vcols;
  g.ldc = ld;
  g.alpha = T(-1);
  g.beta = T(1);
  return g;
}

template <typename T>
rfmls_status qr_impl(rfmls_handle* h, int64_t s, int64_t n, T* SA, int64_t ld) {
  hipStream_t st = h->stream;
  const int64_t split_in = 512, split_out = 8192;
  const int64_t nsp_in_max = (s + split_in - 1) / split_in;
  const int64_t nsp_out_max = (s + split_out - 1) / split_out;
  void *p_tau, *p_part, *p_wz, *p_w, *p_wp, *p_to, *p_y;
  RFMLS_CHECK(workspace(h, WS_QR_TAU, sizeof(T) * kOuter, &p_tau));
  RFMLS_CHECK(workspace(h, WS_QR_PART, sizeof(double) * kPayload * (1024 + 1024 / kCluster + 2 + 8),
                        &p_part));
  const size_t wz_in = (size_t)nsp_in_max * kMaxNb * kOuter;
  const size_t wz_out = (size_t)nsp_out_max * kOuter * (size_t)n;
  RFMLS_CHECK(workspace(h, WS_QR_W, sizeof(T) * (wz_in > wz_out ? wz_in : wz_out), &p_wz));
  RFMLS_CHECK(workspace(h, WS_QR_WR, sizeof(T) * kOuter * (size_t)n, &p_w));
  RFMLS_CHECK(workspace(h, WS_QR_WP, sizeof(T) * kOuter * (size_t)n, &p_wp));
  RFMLS_CHECK(workspace(h, WS_QR_T, sizeof(T) * kOuter * kOuter, &p_to));
  RFMLS_CHECK(workspace(h, WS_QR_Y, sizeof(T) * kOuter * kOuter, &p_y));
  T* tau = (T*)p_tau;
  T* Wz = (T*)p_wz;
  T* W = (T*)p_w;
  T* Wp = (T*)p_wp;
  T* To = (T*)p_to;
  T* Y = (T*)p_y;
  for (int64_t k0 = 0; k0 < n; k0 += kOuter) {
    const int64_t bw = n - k0 < kOuter ? n - k0 : kOuter;
    // ---------------- inner panels of the outer block ----------------
    for (int64_t p0 = k0; p0 < k0 + bw; p0 += kMaxNb) {
      const int jb = (int)(k0 + bw - p0 < kMaxNb ? k0 + bw - p0 : kMaxNb);
      const int64_t M = s - p0;
      // rows per block rpw = (NT / 64) Q: the smallest shape whose grid is
      // co-resident (fewer rows per thread = less arithmetic per column; the
      // grid reduction costs about the same for any G), else the largest one
      const PanelShape* shapes = panel_shapes<T>();
      int si = 0;
      for (;; ++si) {
        if (shapes[si + 1].q == 0) break;
        int per_cu = 0;
        RFMLS_HIP(h, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, shapes[si].fn, shapes[si].nt, 0));
        const int64_t gmax = (int64_t)per_cu * h->num_cus < 1024 ? (int64_t)per_cu * h->num_cus : 1024;
        if ((M + shapes[si].rpw() - 1) / shapes[si].rpw() <= gmax) break;
      }
      const PanelShape sh = shapes[si];
      const int64_t rpw = sh.rpw();
      const int64_t G = (M + rpw - 1) / rpw;
      if (G > 1024)
        return fail(h, RFMLS_E_ARG, "QR panel of %lld rows needs more than 1024 blocks", (long long)M);
      T* P = SA + p0 * ld + p0;
      T* tau_p = tau + (p0 - k0);
      hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(256), 0, st, h->barrier, kBarrierWords);
      int rpw_i = (int)rpw;
      void* args[] = {(void*)&P, (void*)&ld, (void*)&M, (void*)&jb, (void*)&rpw_i, (void*)&tau_p,
                      (void*)&p_part, (void*)&h->barrier, (void*)&h->dev_flags};
      const void* fn = sh.fn;
      {
        // Householder on an M x jb panel: sum_j 4 (M - j)(jb - j) flops; panel read and written once
        const double pf = 4.0 * (double)M * jb * (jb + 1) / 2.0;
        Trace tr(h, "qr_panel", 2.0 * sizeof(T) * (double)M * jb, pf);
        RFMLS_HIP(h, hipLaunchCooperativeKernel(fn, dim3((unsigned)G), dim3(sh.nt), args, 0, st));
      }
      const int64_t rem = k0 + bw - (p0 + jb);
      if (rem <= 0) continue;
      const int64_t ncols = jb + rem;
      const int64_t nsp = (M + split_in - 1) / split_in;
      {
        Trace tr(h, "qr_inner_VtC", sizeof(T) * ((double)M * ncols + (double)nsp * jb * ncols),
                 2.0 * (double)jb * ncols * M);
        RFMLS_HIP(h, (gemm<T, GemmRole::QrInnerVtC>(vt_gemm<T>(P, ld, M, jb, ncols, Wz, split_in), st)));
        hipLaunchKernelGGL(k_sum_slices<T>, dim3(ceil_div(jb * ncols, 256)), dim3(256), 0, st,
                           (const T*)Wz, (int64_t)jb * ncols, (int)nsp, (int64_t)jb * ncols, W);
      }
      {
        Trace tr(h, "qr_inner_T", sizeof(T) * 2.0 * jb * ncols, 2.0 * (double)jb * jb * rem);
        // this panel's T is also the diagonal block of the outer block's T_o
        T* Tq = To + (p0 - k0) * kOuter + (p0 - k0);
        hipLaunchKernelGGL(k_qr_buildT<T>, dim3(1), dim3(256), 0, st, (const T*)W, (int64_t)0, 1,
                           ncols, jb, (const T*)tau_p, Tq, (int64_t)kOuter);
        hipLaunchKernelGGL(k_qr_wp<T>, dim3(ceil_div(rem, 64)), dim3(256), 0, st, (const T*)W,
                           (int64_t)0, 1, ncols, jb, rem, (const T*)Tq, (int64_t)kOuter, Wp, rem);
      }
      {
        Trace tr(h, "qr_inner_update", sizeof(T) * (2.0 * (double)M * rem + (double)M * jb),
                 2.0 * (double)M * rem * jb);
        RFMLS_HIP(h, (gemm<T, GemmRole::QrInnerUpdate>(v_update<T>(P, ld, M, jb, rem, Wp), st)));
      }
      RFMLS_HIP(h, hipGetLastError());
    }
    // ---------------- trailing update with the whole outer block ----------------
    const int64_t ntr = n - k0 - bw;
    if (ntr <= 0) continue;
    const int64_t M0 = s - k0;
    T* P0 = SA + k0 * ld + k0;
    const int64_t ncols = bw + ntr;
    const int64_t nsp = (M0 + split_out - 1) / split_out;
    {
      Trace tr(h, "qr_gemm_VtC", sizeof(T) * ((double)M0 * ncols + 2.0 * (double)nsp * bw * ncols),
               2.0 * (double)bw * ncols * M0);
      RFMLS_HIP(h, (gemm<T, GemmRole::QrVtC>(vt_gemm<T>(P0, ld, M0, bw, ncols, Wz, split_out), st)));
      hipLaunchKernelGGL(k_sum_slices<T>, dim3(ceil_div(bw * ncols, 256) < 4096 ? ceil_div(bw * ncols, 256) : 4096),
                         dim3(256), 0, st, (const T*)Wz, bw * ncols, (int)nsp, bw * ncols, W);
    }
    {
      // T_o: its diagonal 64-blocks are the inner panels' T, written above,
      // except the last panel's (no inner update follows it), built here from
      // the Gram's diagonal block; then the block columns
      Trace tr(h, "qr_outer_T", sizeof(T) * 4.0 * (double)bw * bw, 2.0 * (double)bw * bw * bw);
      {
        const int64_t q0 = (bw - 1) / kMaxNb * kMaxNb;
        const int jq = (int)(bw - q0);
        hipLaunchKernelGGL(k_qr_buildT<T>, dim3(1), dim3(256), 0, st, (const T*)(W + q0 * ncols + q0),
                           (int64_t)0, 1, ncols, jq, (const T*)(tau + q0), To + q0 * kOuter + q0,
                           (int64_t)kOuter);
      }
      for (int64_t q0 = kMaxNb; q0 < bw; q0 += kMaxNb) {
        const int64_t jq = bw - q0 < kMaxNb ? bw - q0 : kMaxNb;
        GemmArgs<T> ga;  // Y = T_o[:q0, :q0] * Gram[:q0, q0:q0+jq]
        ga.M = q0;
        ga.N = jq;
        ga.K = q0;
        ga.A = To;
        ga.lda = kOuter;
        ga.a_upper = 1;
        ga.B = W + q0;
        ga.ldb = ncols;
        ga.C = Y;
        ga.ldc = jq;
        RFMLS_HIP(h, (gemm<T, GemmRole::QrOuterT>(ga, st)));
        GemmArgs<T> gb;  // T_o[:q0, q0:q0+jq] = -Y * T_qq
        gb.M = q0;
        gb.N = jq;
        gb.K = jq;
        gb.A = Y;
        gb.lda = jq;
        gb.B = To + q0 * kOuter + q0;
        gb.ldb = kOuter;
        gb.b_upper = 1;
        gb.C = To + q0;
        gb.ldc = kOuter;
        gb.alpha = T(-1);
        RFMLS_HIP(h, (gemm<T, GemmRole::QrOuterT>(gb, st)));
      }
    }
    {
      // W' = T_o^T W[:, bw:]  (T_o^T lower triangular)
      Trace tr(h, "qr_outer_TtW", sizeof(T) * 2.0 * (double)bw * ntr, (double)bw * bw * ntr);
      GemmArgs<T> gt;
      gt.M = bw;
      gt.N = ntr;
      gt.K = bw;
      gt.A = To;
      gt.lda = kOuter;
      gt.transA = 1;
      gt.a_lower = 1;
      gt.B = W + bw;
      gt.ldb = ncols;
      gt.C = Wp;
      gt.ldc = ntr;
      RFMLS_HIP(h, (gemm<T, GemmRole::QrOuterT>(gt, st)));
    }
    {
      Trace tr(h, "qr_gemm_update", sizeof(T) * (2.0 * (double)M0 * ntr + (double)M0 * bw + (double)bw * ntr),
               2.0 * (double)M0 * ntr * bw);
      RFMLS_HIP(h, (gemm<T, GemmRole::QrTrailingUpdate>(v_update<T>(P0, ld, M0, bw, ntr, Wp), st)));
    }
    RFMLS_HIP(h, hipGetLastError());
  }
  return RFMLS_OK;
}

}  // namespace

rfmls_status run_qr(rfmls_handle* h, int64_t s, int64_t n, rfmls_dtype dt, void* SA, int64_t ld) {
  if (dt == RFMLS_F64) return qr_impl<double>(h, s, n, (double*)SA, ld);
  return qr_impl<float>(h, s, n, (float*)SA, ld);
}

}  // namespace rfmls
