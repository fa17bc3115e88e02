// Blocked Householder QR of the sketch SA (s x n, row-major, in place):
// Alg. 1 step 3.  Only R is needed; Q is never formed.
//
// Two levels of blocking.  Outer blocks of kOuter = 256 or 512 columns
// are factored panel by panel (kMaxNb = 64 columns each); the trailing matrix
// right of an outer block is then updated once, with K = kOuter, which keeps
// that update -- most of the flops -- on the matrix cores instead of bound by
// HBM traffic.
//
// Inner panel at column p0 (M = s - p0 rows):
//   k_qr_panel   unblocked Householder on the M x 64 panel, spread over G
//                co-resident workgroups (rows held in registers); each column
//                needs one grid-wide sum of sigma = sum_{i>j} a_ij^2, d_c =
//                sum_{i>j} a_ij a_ic and the pivot row, after which every
//                workgroup forms the same reflector and applies it to its rows;
//   inside the outer block: W = V^T [V | C] (split-K GEMM), T from V^T V
//                (the inverse of its strict upper part plus diag(1/tau), by
//                back substitution), C <- C - V (T^T W).
// Outer block at column k0 (M0 = s - k0 rows, V_o = its kOuter Householder vectors):
//   W = V_o^T [V_o | C] (split-K GEMM; the first kOuter columns are the Gram V_o^T V_o),
//   W' = T_o^T W_C without forming T_o's off-diagonal blocks: T_o's block
//   recurrence T_o[:q, q] = -T_o[:q, :q] (V_:q^T V_q) T_qq turns the product
//   into a forward substitution by blocks with the Gram's blocks and the
//   panels' T (k_qr_outer_wp),  then C <- C - V_o W'.
// All reductions run in a fixed order, so the factorisation is deterministic.
#include "common.h"
#include "gemm.h"

namespace rfmls {
namespace {

constexpr int kMaxNb = 64;
// CholeskyQR2 panels: at least this many rows (shorter panels are cheap for
// the unblocked kernel), and the first Cholesky's pivot ratio below which a
// panel falls back to it (scaled panel condition near u^{-1/2})
constexpr int64_t kCholqrMinRows = 1024;
constexpr double kCholqrMinPivot = 1e-7;

// Cross-block exchange of the panel kernel.  Every value crosses blocks in a
// "low-latency" slot: the float64 travels as two 64-bit words (its low or high
// 32 bits, and a tag in the upper 32 bits), each written and read with one
// relaxed agent-scope atomic, which is coherent across the XCDs' separate L2
// caches.  A reader accepts the value once both words carry the tag it
// expects, so no flag, counter or store-completion wait sits on the critical
// path: a hand-over costs one store propagation plus one load round trip.
// Tags are the column's index in the matrix + 1, unique within one QR; the
// slots are zeroed once per QR (a stale value from an earlier panel carries
// another tag).
__device__ __forceinline__ void ll_put(uint64_t* slot, double v, unsigned tag) {
  const uint64_t x = (uint64_t)__double_as_longlong(v);
  const uint64_t t = (uint64_t)tag << 32;
  __hip_atomic_store(&slot[0], (x & 0xffffffffull) | t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&slot[1], (x >> 32) | t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Wait (bounded) for the value tagged `tag`; on time-out flag the error, clear
// the block's `ok` and return 0.
__device__ __forceinline__ bool ll_try(uint64_t* p, unsigned tag, double* v) {
  const uint64_t a = __hip_atomic_load(&p[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint64_t b = __hip_atomic_load(&p[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if ((unsigned)(a >> 32) != tag || (unsigned)(b >> 32) != tag) return false;
  *v = __longlong_as_double((long long)((a & 0xffffffffull) | (b << 32)));
  return true;
}
constexpr int kSpinLimit = 1 << 20;
__device__ __forceinline__ double ll_wait(const uint64_t* slot, unsigned tag, int* err, int* ok) {
  uint64_t* p = const_cast<uint64_t*>(slot);
  double v = 0.0;
  for (int spins = 0; !ll_try(p, tag, &v); ++spins) {
    if (spins > kSpinLimit) {
      atomicExch(err, 1);
      *ok = 0;
      return 0.0;
    }
    __builtin_amdgcn_s_sleep(4);
  }
  return v;
}
// Two values polled together (one round trip per attempt for both).  Every
// workgroup polls the same few slots here (the totals and the pivot row), so
// the attempts are spaced out: 24 x 64 clocks between them measured about 1%
// faster on the whole panel than back-to-back polls (fewer reads queue at
// those cache lines), and two polls kept in flight 8% slower.
__device__ __forceinline__ void ll_wait2(const uint64_t* s0, const uint64_t* s1, unsigned tag,
                                         double* v0, double* v1, int* err, int* ok) {
  uint64_t* p0 = const_cast<uint64_t*>(s0);
  uint64_t* p1 = const_cast<uint64_t*>(s1);
  bool d0 = false, d1 = false;
  for (int spins = 0;; ++spins) {
    if (!d0) d0 = ll_try(p0, tag, v0);
    if (!d1) d1 = ll_try(p1, tag, v1);
    if (d0 && d1) return;
    if (spins > kSpinLimit) {
      atomicExch(err, 1);
      *ok = 0;
      *v0 = *v1 = 0.0;
      return;
    }
    __builtin_amdgcn_s_sleep(24);
  }
}

// Unblocked Householder QR of an M x nb panel (nb <= 64) spread over G
// co-resident workgroups of NT = 1024 threads (16 wavefronts), one per CU.
// Thread (c = lane, rg = wavefront) of block g holds rows
// r0 + rg + 16 q (q < Q, r0 = g rpw, rpw = 16 Q) of column c in registers;
// all lanes of a wavefront hold the same rows, so column j reaches every lane
// by v_readlane from lane j (no LDS).  Block 0 holds rows 0 .. rpw-1 >= nb-1.
//
// Column j needs one grid-wide sum: sigma = sum_{i>j} a_ij^2 and
// d_c = sum_{i>j} a_ij a_ic (c > j), plus the pivot row a_jc from block 0.
// Each block publishes its partial sums (slots r1[j&1][c][g]) and block 0 the
// pivot row (rp[j&1][c]).  With G >= 64 blocks, block c sums the G partials of
// column c (each of its first G threads waits for one, then a fixed-order
// wavefront tree and an ordered sum of the wavefront results) and publishes
// the total (r2[j&1][c]); every block then reads the nb - j totals.  With
// fewer blocks every block sums all G partials itself (16 threads per column,
// each over blocks p, p + 16, ..., then those 16 partial sums in order).  Every
// block thus receives bit-identical totals and forms the same reflector (LAPACK
// dlarfg convention: beta = -sign(alpha) ||(alpha, x)||, tau = (beta -
// alpha)/beta, v = [1; x/(alpha-beta)]), computed once per block by the thread
// of column j, and applies it to its rows.  Slots of column j are reused by
// column j + 2 only: a block can publish column j + 2 only after every block
// has published column j + 1, which each does after reading column j.
//   ll  slots, 16 bytes each: r1 [2][64][G], rp [2][64], r2 [2][64]

__device__ __forceinline__ double lane_value(double v, int lane) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double lane_value(float v, int lane) {
  return (double)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

constexpr int kPanelThreads = 1024;
constexpr int kPanelGroups = kPanelThreads / 64;  // wavefronts per block
constexpr int kPanelMaxBlocks = kPanelThreads;    // a reducer thread per block
__host__ __device__ constexpr int64_t ll_words(int64_t G) { return 2 * (2 * kMaxNb * G + 4 * kMaxNb); }

template <typename T, int Q>
__global__ void __launch_bounds__(kPanelThreads)
    k_qr_panel(T* __restrict__ P, int64_t ld, int64_t M, int nb, int rpw, T* __restrict__ tau,
               uint64_t* __restrict__ ll, int* __restrict__ err, unsigned tag0, const int* __restrict__ run_if) {
  static_assert(kPanelGroups * Q >= kMaxNb, "block 0 must hold the panel's top rows");
  // gated launch (after a CholeskyQR2 attempt): every block reads the same
  // flag and leaves before any exchange when the panel is already factored
  if (run_if && *run_if == 0) return;
  __shared__ double red[2 * kMaxNb];               // totals, then the pivot row
  __shared__ double grp[kPanelGroups][kMaxNb];     // per-wavefront partials
  __shared__ double part[kPanelGroups][kMaxNb];    // partial sums of the totals
  __shared__ double piv[kMaxNb];                   // pivot row (block 0)
  __shared__ double refl[3];                       // beta, tau, 1/(alpha - beta)
  __shared__ int ok;
  const int G = gridDim.x;
  const int g = blockIdx.x;
  const int tid = threadIdx.x;
  const int c = tid & 63;
  const int rg = tid >> 6;  // wavefront index: uniform within a wavefront
  const int64_t r0 = (int64_t)g * rpw;
  const int nr = (int)(M - r0 < rpw ? (M - r0 > 0 ? M - r0 : 0) : rpw);
  uint64_t* r1 = ll;                                // [2][kMaxNb][G] slots
  uint64_t* rp = ll + 2 * (2 * kMaxNb * (int64_t)G);  // [2][kMaxNb]
  uint64_t* r2 = rp + 2 * (2 * kMaxNb);               // [2][kMaxNb]
  if (tid == 0) ok = 1;

  // rows beyond the panel are held as zeros and contribute nothing
  T a[Q];
  const int64_t rstep = (int64_t)kPanelGroups * ld;  // between a thread's rows
  {
    const T* pr = P + (r0 + rg) * ld + c;
#pragma unroll
    for (int q = 0; q < Q; ++q, pr += rstep) {
      const int li = rg + kPanelGroups * q;
      a[q] = (li < nr && c < nb) ? *pr : T(0);
    }
  }

  const bool top = (g == 0);
  for (int j = 0; j < nb; ++j) {
    const unsigned tag = tag0 + (unsigned)j + 1u;
    const int par = j & 1;
    const int L = nb - j;
    // Only block 0 holds rows i <= j (li > j is uniform per wavefront).
    if (top && rg == (j % kPanelGroups)) {  // pivot row j lives in this wavefront
      const int qj = j / kPanelGroups;
      double pv = 0.0;
#pragma unroll
      for (int q = 0; q < Q; ++q) pv = (q == qj) ? (double)a[q] : pv;
      piv[c] = pv;
    }
    // ---- local partials over rows i > j: sum_i a_ij a_ic ----
    // (up to 16 rows per thread, a_ij of the wavefront's rows is kept for the
    // update below, column j not changing in between; more rows would spill)
    constexpr bool kKeep = Q <= 16;
    double s = 0.0;
    T aj[kKeep ? Q : 1];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int li = rg + kPanelGroups * q;
      // rows li >= kMaxNb > j always take part (compile-time for large q)
      if (kPanelGroups * q >= kMaxNb || !top || li > j) {
        const T v = (T)lane_value(a[q], j);
        if constexpr (kKeep) aj[q] = v;
        s += (double)v * (double)a[q];
      } else if constexpr (kKeep) {
        aj[q] = T(0);
      }
    }
    grp[rg][c] = s;
    __syncthreads();
    if (tid < 64 && c >= j && c < nb) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < kPanelGroups; ++q) t += grp[q][c];
      ll_put(&r1[2 * (((int64_t)par * kMaxNb + c) * G + g)], t, tag);
      if (top) ll_put(&rp[2 * (par * kMaxNb + c)], piv[c], tag);
    }
    // ---- totals ----
    double tot = 0.0;  // thread c (< 64): total of column c
    if (G >= kMaxNb) {
      if (g >= j && g < nb) {  // this block sums column g (block-uniform branch)
        double v = 0.0;
        if (tid < G) v = ll_wait(&r1[2 * (((int64_t)par * kMaxNb + g) * G + tid)], tag, err, &ok);
        v = wave_sum(v);
        if (c == 0) part[rg][0] = v;
        __syncthreads();
        if (tid == 0) {
          double t = 0.0;
#pragma unroll
          for (int q = 0; q < kPanelGroups; ++q) t += part[q][0];
          ll_put(&r2[2 * (par * kMaxNb + g)], t, tag);
        }
      }
    } else {
      if (c >= j && c < nb) {
        double t = 0.0;
        for (int gg = rg; gg < G; gg += kPanelGroups)
          t += ll_wait(&r1[2 * (((int64_t)par * kMaxNb + c) * G + gg)], tag, err, &ok);
        part[rg][c] = t;
      }
      __syncthreads();
      if (tid < 64 && c >= j && c < nb) {
#pragma unroll
        for (int q = 0; q < kPanelGroups; ++q) tot += part[q][c];
      }
    }
    if (tid < 64 && c >= j && c < nb) {
      double pc;
      if (G >= kMaxNb)
        ll_wait2(&r2[2 * (par * kMaxNb + c)], &rp[2 * (par * kMaxNb + c)], tag, &tot, &pc, err, &ok);
      else
        pc = ll_wait(&rp[2 * (par * kMaxNb + c)], tag, err, &ok);
      red[c - j] = tot;
      red[L + c - j] = pc;
      if (c == j) {  // the reflector, once per block
        const double alpha = pc, sigma = tot;
        double beta = alpha, tj = 0.0, scal = 0.0;
        if (sigma != 0.0) {
          const double nrm = sqrt(alpha * alpha + sigma);
          beta = alpha >= 0.0 ? -nrm : nrm;
          tj = (beta - alpha) / beta;
          scal = 1.0 / (alpha - beta);
        }
        refl[0] = beta;
        refl[1] = tj;
        refl[2] = scal;
        if (top) tau[j] = (T)tj;
      }
    }
    __syncthreads();
    if (!ok) return;  // a partner block did not answer (error flag set)
    // ---- apply H_j to rows i >= j of columns c > j; column j becomes v ----
    const double beta = refl[0], tj = refl[1], scal = refl[2];
    const bool upd = (c > j && c < nb && tj != 0.0);
    const double f = upd ? tj * (red[L + c - j] + scal * red[c - j]) : 0.0;
    const double sf = scal * f;
    // one multiply-add per row below the diagonal, with no per-lane branch:
    // a - sf v_j on the columns updated, scal v_j on column j (it becomes v),
    // a + 0 v_j (exactly a) on the columns left alone
    const double kv = upd ? -sf : (c == j ? scal : 0.0);
    const bool keep = (c != j);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int li = rg + kPanelGroups * q;
      if (kPanelGroups * q >= kMaxNb || !top || li > j) {
        double vj;
        if constexpr (kKeep) vj = (double)aj[q];
        else vj = lane_value(a[q], j);  // read before lane j rewrites it
        a[q] = (T)fma(kv, vj, keep ? (double)a[q] : 0.0);
      } else if (li == j) {
        a[q] = (T)(upd ? (double)a[q] - f : (c == j ? beta : (double)a[q]));
      }
    }
    // no barrier here: the next writes of red, refl and part follow the next
    // column's first __syncthreads, and piv / grp are not read after this point
  }
  T* pw_row = P + (r0 + rg) * ld + c;
  // an opaque copy: otherwise the compiler reuses the Q row addresses of the
  // initial loads here and keeps them alive (spilled) across the whole kernel
  asm volatile("" : "+v"(pw_row));
#pragma unroll
  for (int q = 0; q < Q; ++q, pw_row += rstep) {
    const int li = rg + kPanelGroups * q;
    if (li < nr && c < nb) *pw_row = a[q];
  }
}

// Build T (nb x nb upper triangular, row-major) of the compact-WY form
// H_1 ... H_nb = I - V T V^T from tau and the Gram V^T V (the sum of nsplit
// partial slices Wz, each nb x ldw, whose leading nb columns hold V^T V).
// T is the inverse of U = (strictly upper part of V^T V) + diag(1/tau): that
// is the matrix form of the column recursion T[:j, j] = -tau_j T[:j, :j]
// V_:j^T v_j (Schreiber and Van Loan).  Column k of T solves U t = e_k by
// back substitution on one wavefront (lane i holds row i), t_l = tau_l x_l
// from the bottom up, so 1/tau is never formed and a reflector with tau_j = 0
// (H_j = I) leaves row and column j zero, as the recursion does.  One
// wavefront per column: ceil(nb / 16) workgroups of 16, each staging the Gram.
template <typename T>
__global__ void __launch_bounds__(1024)
    k_qr_buildT(const T* __restrict__ Wz, int64_t zstride, int nsplit, int64_t ldw, int nb,
                const T* __restrict__ tau, T* __restrict__ Tout, int64_t ldt) {
  // Us[i][l] = (V^T V)_il for i < l < nb, zero elsewhere, so the update below
  // needs no per-row test (rows i >= l subtract exactly 0)
  __shared__ double Us[kMaxNb][kMaxNb + 1];
  __shared__ double ts[kMaxNb + 3];  // three zero entries below index 0 (steps past l = 0)
  const int tid = threadIdx.x;
  for (int e = tid; e < kMaxNb * kMaxNb; e += 1024) {
    const int i = e / kMaxNb, l = e % kMaxNb;
    double sacc = 0.0;
    if (i < l && l < nb)
      for (int z = 0; z < nsplit; ++z) sacc += (double)Wz[(int64_t)z * zstride + (int64_t)i * ldw + l];
    Us[i][l] = sacc;
  }
  if (tid < kMaxNb + 3) ts[tid] = (tid >= 3 && tid - 3 < nb) ? (double)tau[tid - 3] : 0.0;
  __syncthreads();
  const int lane = tid & 63, w = tid >> 6;
  {
    const int k = (int)blockIdx.x * 16 + w;
    if (k >= nb) return;  // uniform within the wavefront (no barrier follows)
    double x = lane == k ? 1.0 : 0.0, t = 0.0;
    // four steps per group, their LDS reads issued together; steps past l = 0
    // read tau = 0 and column 0 of Us (zeros) and change nothing
    for (int l0 = k; l0 >= 0; l0 -= 4) {
      double u[4], tt[4];
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        const int l = l0 - d;
        u[d] = Us[lane][l > 0 ? l : 0];
        tt[d] = ts[l + 3];
      }
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        const int l = l0 - d;
        const double tl = tt[d] * lane_value(x, l > 0 ? l : 0);  // x_l is final once rows > l are done
        if (lane == l) t = tl;
        x -= u[d] * tl;
      }
    }
    if (lane < nb) Tout[(int64_t)lane * ldt + k] = (T)(lane <= k ? t : 0.0);
  }
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

// The same sum for one panel's V^T [V | C] (a short range over many slices):
// a workgroup per 64 elements, its four wavefronts summing every fourth slice,
// the four partial sums then added in a fixed order.
template <typename T>
__global__ void __launch_bounds__(256)
    k_sum_slices_narrow(const T* __restrict__ Wz, int64_t zstride, int nsplit, int64_t len,
                        T* __restrict__ W) {
  __shared__ double part[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * 64 + lane;
  double acc = 0.0;
  if (e < len) {
#pragma unroll 4
    for (int z = w; z < nsplit; z += 4) acc += (double)Wz[(int64_t)z * zstride + e];
  }
  part[w][lane] = acc;
  __syncthreads();
  if (w == 0 && e < len) W[e] = (T)((part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]));
}

__global__ void k_zero_u64(uint64_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// Outer block width: 512 columns for float32, whose trailing update then
// reads and writes the trailing matrix half as often (4^3-box sketch: 2.5% less
// QR time than 256), and for float64 from 12,800 columns on (4^3-box, 25,600
// columns: 1.3% less solve time; 8x8-box, 12,800 columns: QR phase 327.8 ->
// 325.1 ms, the trailing products' 9 ms saved less the inner 64-column
// products, which grow with the width); narrower float64 systems keep 256.
constexpr int64_t kOuterMax = 512;
template <typename T>
int64_t outer_width(int64_t n) { return sizeof(T) == 4 || n >= 12800 ? 512 : 256; }
inline int64_t pad32(int64_t x) { return (x + 31) / 32 * 32; }

// Row slices of an inner panel's split-K product V^T [V | C]: its output is
// only 64 rows by at most kOuter columns, so the slices are what fills the
// GPU.  256-row slices from 32,768 rows on, 128 below (8x8-box sketch, QR
// phase 325.4 -> 323.6 ms against 512-row slices; Helmholtz sketch, 12,800
// rows, 20.35 -> 19.74 ms; 128-row slices on the 8x8-box sketch 325-327 ms,
// the slice sums' extra reads outweighing the fuller grid).
inline int64_t inner_split(int64_t M) { return M >= 32768 ? 256 : 128; }
// most slices any panel of an s-row sketch takes
inline int64_t inner_slices_max(int64_t s) {
  const int64_t a = (s + inner_split(s) - 1) / inner_split(s);
  const int64_t ms = s < 32767 ? s : 32767;
  const int64_t b = (ms + 127) / 128;
  return a > b ? a : b;
}
// Row slices of an outer block's V^T [V | C] below its masked top rows:
// 4096 rows from 32,768 rows on (2% faster than 8192 on the 8x8-box sketch,
// net of the longer slice sum; 2048 there measured even), kOuterSplitShort
// below, where the grid is thinner (Helmholtz sketch, 12,800 rows: V^T C
// 4.07 -> 3.15 ms per solve against 4096-row slices; 2048 rows 3.45 ms,
// 8192 rows 6.6 ms).
constexpr int64_t kOuterSplitShort = 1024;
inline int64_t outer_split(int64_t M0) { return M0 >= 32768 ? 4096 : kOuterSplitShort; }
// most slices any outer block of an s-row sketch takes (the masked top rows
// and a ragged tail included)
inline int64_t outer_slices_max(int64_t s) {
  const int64_t a = (s + outer_split(s) - 1) / outer_split(s);
  const int64_t ms = s < 32767 ? s : 32767;
  const int64_t b = (ms + kOuterSplitShort - 1) / kOuterSplitShort;
  return (a > b ? a : b) + 2;
}

// W' = T^T W_C for one panel: W = V^T [V | C] (nb x ldw, its leading nb
// columns the Gram, W_C the ncol columns after them) and the panel's T (nb x
// nb upper triangular, rows ldt apart).  One workgroup per 32 columns; thread
// (ty, tx) forms rows ty + 32 a and columns tx + 8 b of its strip, summing in
// float64 over LDS copies of T and of the strip.
template <typename T>
__global__ void __launch_bounds__(256)
    k_qr_wp(const T* __restrict__ W, int64_t ldw, int nb, const T* __restrict__ Tm, int64_t ldt,
            int64_t ncol, T* __restrict__ Wp, int64_t ldwp) {
  constexpr int SW = 32;
  __shared__ double Ts[kMaxNb][kMaxNb + 1];  // [k][i] = T_ki (zero below the diagonal)
  __shared__ double Ws[kMaxNb][SW + 1];      // [k][c]
  const int tid = threadIdx.x;
  const int ty = tid >> 3, tx = tid & 7;
  const int64_t c0 = (int64_t)blockIdx.x * SW;
  for (int e = tid; e < kMaxNb * kMaxNb; e += 256) {
    const int k = e / kMaxNb, i = e % kMaxNb;
    Ts[k][i] = (k <= i && i < nb) ? (double)Tm[(int64_t)k * ldt + i] : 0.0;
  }
  for (int e = tid; e < kMaxNb * SW; e += 256) {
    const int k = e / SW, c = e % SW;
    Ws[k][c] = (k < nb && c0 + c < ncol) ? (double)W[(int64_t)k * ldw + nb + c0 + c] : 0.0;
  }
  __syncthreads();
  double o[2][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
#pragma unroll 4
  for (int k = 0; k < kMaxNb; ++k) {
    const double m0 = Ts[k][ty], m1 = Ts[k][ty + 32];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const double r = Ws[k][tx + 8 * b];
      o[0][b] += m0 * r;
      o[1][b] += m1 * r;
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = ty + 32 * a;
      const int64_t c = c0 + tx + 8 * b;
      if (i < nb && c < ncol) Wp[(int64_t)i * ldwp + c] = (T)o[a][b];
    }
}

// W' = T_o^T W_C for an outer block of NQ 64-column panels, without forming
// T_o's blocks above the diagonal.  Since T_o[:q0, q] = -T_o[:q0, :q0]
// G[:q0, q] T_q (G = V_o^T V_o, q the panel at column q0, T_q its T), block
// row q of T_o^T W_C is
//   W'_q = T_q^T (W_q - G[:q0, q]^T W'[:q0]),
// a forward substitution by blocks that every column runs on its own.  G's
// blocks above the diagonal are read from G (rows ldg apart), each T_q (upper
// triangular, zeros stored below the diagonal) from the diagonal 64-blocks of
// Td (rows ldt apart), W_C from W (NQ * 64 rows, ldw apart).  One workgroup
// per 16 columns; wavefront w forms rows 16 w .. 16 w + 15 of each 64-row
// block on the matrix cores, in float64 for either storage type, and the rows
// of W' formed so far stay in LDS.
template <typename T, int NQ>
__global__ void __launch_bounds__(256)
    k_qr_outer_wp(const T* __restrict__ W, int64_t ldw, const T* __restrict__ G, int64_t ldg,
                  const T* __restrict__ Td, int64_t ldt, int64_t ncol, T* __restrict__ Wp, int64_t ldwp) {
  typedef double v4d __attribute__((ext_vector_type(4)));
  constexpr int SW = 16;
  __shared__ double Xs[NQ * kMaxNb][SW + 1];  // W' rows formed so far
  __shared__ double Ys[kMaxNb][SW + 1];       // W_q - G[:q0, q]^T W'[:q0]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int i0 = 16 * w;
  const int64_t col = (int64_t)blockIdx.x * SW + lr;
  const bool cin = col < ncol;
  // operand layout of v_mfma_f64_16x16x4f64: lane (lr, lk) holds A[lr][lk] and
  // B[lk][lr]; accumulator register r holds D[lk + 4 r][lr]
  for (int q = 0; q < NQ; ++q) {
    const int q0 = kMaxNb * q;
    // G[:q0, q]^T W'[:q0]: A[i][k] = G[k][q0 + i], B[k][c] = W'[k][c], K in
    // chunks of 64 (the next chunk's operands loaded during this one's
    // products), two accumulators (even and odd steps)
    v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    const T* ga = G + q0 + i0 + lr;
    double a[16];
    if (q0 > 0)
#pragma unroll
      for (int j = 0; j < 16; ++j) a[j] = (double)ga[(int64_t)(4 * j + lk) * ldg];
    for (int kc = 0; kc < q0; kc += 64) {
      double an[16];
      const bool more = kc + 64 < q0;
      if (more)
#pragma unroll
        for (int j = 0; j < 16; ++j) an[j] = (double)ga[(int64_t)(kc + 64 + 4 * j + lk) * ldg];
#pragma unroll
      for (int j = 0; j < 16; j += 2) {
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[j], Xs[kc + 4 * j + lk][lr], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[j + 1], Xs[kc + 4 * j + 4 + lk][lr], acc1, 0, 0, 0);
      }
      if (more)
#pragma unroll
        for (int j = 0; j < 16; ++j) a[j] = an[j];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + lk + 4 * r;
      const double wv = cin ? (double)W[(int64_t)(q0 + i) * ldw + col] : 0.0;
      Ys[i][lr] = wv - (acc0[r] + acc1[r]);
    }
    __syncthreads();
    // W'_q = T_q^T Y: A[i][k] = T_q[k][i], zero for k > i, so the K range of
    // rows i0 .. i0 + 15 ends at i0 + 16
    const T* ta = Td + (int64_t)q0 * ldt + q0 + i0 + lr;
    const int nk = 4 * (w + 1);
    double tv[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) tv[j] = (double)ta[(int64_t)(4 * j + lk) * ldt];  // inside the block
    v4d o0 = {0.0, 0.0, 0.0, 0.0}, o1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < 16; j += 2) {
      if (j < nk) {
        o0 = __builtin_amdgcn_mfma_f64_16x16x4f64(tv[j], Ys[4 * j + lk][lr], o0, 0, 0, 0);
        o1 = __builtin_amdgcn_mfma_f64_16x16x4f64(tv[j + 1], Ys[4 * j + 4 + lk][lr], o1, 0, 0, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + lk + 4 * r;
      const double v = o0[r] + o1[r];
      Xs[q0 + i][lr] = v;
      if (cin) Wp[(int64_t)(q0 + i) * ldwp + col] = (T)v;
    }
    __syncthreads();
  }
}

// The Gram's 64-blocks above the diagonal (rows ldw apart in W) into the same
// places of To (rows ldt apart), whose diagonal blocks hold the panels' T:
// what k_qr_outer_wp needs when a later product reuses the outer block.
template <typename T>
__global__ void k_qr_keep_gram(const T* __restrict__ W, int64_t ldw, int bw, T* __restrict__ To, int64_t ldt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)bw * bw) return;
  const int r = (int)(e / bw), c = (int)(e % bw);
  if (r / kMaxNb < c / kMaxNb) To[(int64_t)r * ldt + c] = W[(int64_t)r * ldw + c];
}

// Panel launch shapes (rows per thread Q, rows per block 16 Q), increasing.
// The largest are the largest that compile without spills at 1024 threads.
struct PanelShape {
  int q;
  const void* fn;
  int64_t rpw() const { return (int64_t)kPanelGroups * q; }
};
template <typename T>
const PanelShape* panel_shapes() {
  static const PanelShape s[] = {{4, (const void*)k_qr_panel<T, 4>},
                                 {8, (const void*)k_qr_panel<T, 8>},
                                 {16, (const void*)k_qr_panel<T, 16>},
                                 {32, (const void*)k_qr_panel<T, 32>},
                                 {0, nullptr}};
  return s;
}

// The smallest shape whose grid (G = ceil(M / rows per block)) fits one block
// per CU: fewer rows per thread means less arithmetic per column on the
// critical path, and one block per CU keeps the SIMDs' shares equal (two
// blocks on some CUs would double their work per column).
template <typename T>
rfmls_status pick_panel_shape(rfmls_handle* h, int64_t M, PanelShape* out, int64_t* G_out) {
  for (const PanelShape* sh = panel_shapes<T>(); sh->q != 0; ++sh) {
    int per_cu = 0;
    RFMLS_HIP(h, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sh->fn, kPanelThreads, 0));
    int64_t gmax = per_cu >= 1 ? (int64_t)h->num_cus : 0;
    if (gmax > kPanelMaxBlocks) gmax = kPanelMaxBlocks;
    const int64_t G = (M + sh->rpw() - 1) / sh->rpw();
    if (G <= gmax) {
      *out = *sh;
      *G_out = G;
      return RFMLS_OK;
    }
  }
  return fail(h, RFMLS_E_ARG, "QR panel of %lld rows does not fit one co-resident grid",
              (long long)M);
}

template <typename T>
GemmArgs<T> vt_gemm(T* P, int64_t ld, int64_t M, int64_t vcols, int64_t ncols, T* out,
                    int64_t ldo, int64_t ksplit) {
  // out_z = V^T [V | C] over row slices: V = the vcols Householder vectors
  // stored below the diagonal of P, C the next ncols - vcols columns; rows of
  // out are ldo apart, slices vcols ldo apart
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
  g.ldc = ldo;
  g.alpha = T(1);
  g.beta = T(0);
  g.ksplit = ksplit;
  g.c_zstride = vcols * ldo;
  return g;
}

template <typename T>
GemmArgs<T> v_update(T* P, int64_t ld, int64_t M, int64_t vcols, int64_t ncols, const T* Wp,
                     int64_t ldwp) {
  // C <- C - V Wp, C = the ncols columns right of the vcols Householder vectors
  // (rows of Wp ldwp apart)
  GemmArgs<T> g;
  g.M = M;
  g.N = ncols;
  g.K = vcols;
  g.A = P;
  g.lda = ld;
  g.a_vmask = 1;
  g.B = Wp;
  g.ldb = ldwp;
  g.C = P + vcols;
  g.ldc = ld;
  g.alpha = T(-1);
  g.beta = T(1);
  return g;
}

// Buffers of one outer block's panels: tau and the diagonal 64-blocks of T_o
// (written by the panels), and the inner products' slices, Gram and T^T W.
template <typename T>
struct PanelBufs {
  T* tau;
  T* To;
  T* Wz;
  T* W;
  T* Wp;
};

// The inner panels of the outer block [k0, k0 + bw) of SA, each factored and
// applied to the rest of the block, on h->stream; tau_out (if given) receives
// the block's tau.
template <typename T>
rfmls_status qr_block_panels(rfmls_handle* h, int64_t s, int64_t k0, int64_t bw, int64_t kOuter, T* SA, int64_t ld,
                             const PanelBufs<T>& pb, uint64_t* ll, double* cq_ws, int* cq_status, T* tau_out) {
  hipStream_t st = h->stream;
  for (int64_t p0 = k0; p0 < k0 + bw; p0 += kMaxNb) {
    const int jb = (int)(k0 + bw - p0 < kMaxNb ? k0 + bw - p0 : kMaxNb);
    const int64_t M = s - p0;
    const int64_t split_in = inner_split(M);
    PanelShape sh;
    int64_t G = 0;
    RFMLS_CHECK(pick_panel_shape<T>(h, M, &sh, &G));
    const int64_t rpw = sh.rpw();
    T* P = SA + p0 * ld + p0;
    T* tau_p = pb.tau + (p0 - k0);
    int rpw_i = (int)rpw;
    unsigned tag0 = (unsigned)p0;
    const int* run_if = nullptr;
    // Householder on an M x jb panel: sum_j 4 (M - j)(jb - j) flops; panel
    // read and written once (the method's work, whichever way it is factored)
    const double pf = 4.0 * (double)M * jb * (jb + 1) / 2.0;
    if (cq_ws && jb == kMaxNb && M >= kCholqrMinRows) {
      // 64-column panels: CholeskyQR2 + reconstruction in float64 arithmetic;
      // the unblocked kernel below then runs only for a panel it flagged
      Trace tr(h, "qr_panel_cq", 2.0 * sizeof(T) * (double)M * jb, pf);
      const double thr1 = h->qr_panel == 2 ? 2.0 : kCholqrMinPivot;
      const double thr2 = h->qr_panel == 3 ? 2.0 : kCholqrMinPivot;
      RFMLS_CHECK(run_cholqr_panel(h, P, ld, M, tau_p, cq_ws, cq_status, thr1, thr2));
      run_if = cq_status;
    }
    void* args[] = {(void*)&P,     (void*)&ld, (void*)&M,            (void*)&jb,   (void*)&rpw_i,
                    (void*)&tau_p, (void*)&ll, (void*)&h->dev_flags, (void*)&tag0, (void*)&run_if};
    const void* fn = sh.fn;
    {
      Trace tr(h, run_if ? "qr_panel_fallback" : "qr_panel", run_if ? 0.0 : 2.0 * sizeof(T) * (double)M * jb,
               run_if ? 0.0 : pf);
      // The gated launch after CholeskyQR2 on the main stream is an ordinary
      // launch: nothing else runs beside it, so its G <= one-per-CU workgroups
      // are all resident when it does run (its waits are bounded either way),
      // and the cooperative launch's own overhead (about 15 us per panel,
      // 200 panels on the 8x8-box sketch) is not paid when it does nothing.
      if (run_if && !h->qr_lookahead)
        RFMLS_HIP(h, hipLaunchKernel(fn, dim3((unsigned)G), dim3(kPanelThreads), args, 0, st));
      else
        RFMLS_HIP(h, hipLaunchCooperativeKernel(fn, dim3((unsigned)G), dim3(kPanelThreads), args, 0, st));
    }
    if (run_if) RFMLS_CHECK(cholqr_fix(h, P, ld, M, cq_ws, cq_status));
    const int64_t rem = k0 + bw - (p0 + jb);
    if (rem <= 0) continue;
    const int64_t ncols = jb + rem;
    const int64_t ldw = pad32(ncols), ldwp = pad32(rem);
    const int64_t nsp = (M + split_in - 1) / split_in;
    {
      Trace tr(h, "qr_inner_VtC", sizeof(T) * ((double)M * ncols + (double)nsp * jb * ncols),
               2.0 * (double)jb * ncols * M);
      RFMLS_HIP(h, (gemm<T, GemmRole::QrInnerVtC>(vt_gemm<T>(P, ld, M, jb, ncols, pb.Wz, ldw, split_in), st)));
      hipLaunchKernelGGL(k_sum_slices_narrow<T>, dim3(ceil_div(jb * ldw, 64)), dim3(256), 0, st, (const T*)pb.Wz,
                         (int64_t)jb * ldw, (int)nsp, (int64_t)jb * ldw, pb.W);
    }
    {
      Trace tr(h, "qr_inner_T", sizeof(T) * 2.0 * jb * ncols, 2.0 * (double)jb * jb * rem);
      // this panel's T is also a diagonal block of the outer block's T_o
      T* Tq = pb.To + (p0 - k0) * kOuter + (p0 - k0);
      hipLaunchKernelGGL(k_qr_buildT<T>, dim3((jb + 15) / 16), dim3(1024), 0, st, (const T*)pb.W, (int64_t)0, 1, ldw,
                         jb, (const T*)tau_p, Tq, (int64_t)kOuter);
      hipLaunchKernelGGL(k_qr_wp<T>, dim3(ceil_div(rem, 32)), dim3(256), 0, st, (const T*)pb.W, ldw, jb,
                         (const T*)Tq, (int64_t)kOuter, rem, pb.Wp, ldwp);
    }
    {
      Trace tr(h, "qr_inner_update", sizeof(T) * (2.0 * (double)M * rem + (double)M * jb),
               2.0 * (double)M * rem * jb);
      RFMLS_HIP(h, (gemm<T, GemmRole::QrInnerUpdate>(v_update<T>(P, ld, M, jb, rem, pb.Wp, ldwp), st)));
    }
    RFMLS_HIP(h, hipGetLastError());
  }
  // every reflector's tau, for a caller that applies Q afterwards
  if (tau_out)
    RFMLS_HIP(h, hipMemcpyAsync(tau_out + k0, pb.tau, sizeof(T) * (size_t)bw, hipMemcpyDeviceToDevice, st));
  return RFMLS_OK;
}

// Buffers of the trailing update: the outer products' slices, W = V^T [.],
// and W' = T_o^T W.
template <typename T>
struct TrailBufs {
  T* Wz;
  T* W;
  T* Wp;
};

// Trailing update C <- C - V T_o^T (V^T C) with the outer block [k0, k0 + bw)
// (V below its diagonal in SA) for the nc columns starting off columns right
// of the block (nc_m of them the method's own, the rest tile padding within
// the room).  With gram, off must be 0: the product then also covers V itself,
// and T_o is built from that Gram (its diagonal 64-blocks from the panels,
// except the last panel's); without, T_o must already hold the block's T.
template <typename T>
rfmls_status qr_block_trailing(rfmls_handle* h, int64_t s, int64_t k0, int64_t bw, int64_t kOuter, T* SA, int64_t ld,
                               int64_t off, int64_t nc, int64_t nc_m, bool gram, const T* tau, T* To,
                               const TrailBufs<T>& tb, bool keep_gram = false) {
  hipStream_t st = h->stream;
  const int64_t M0 = s - k0;
  const int64_t split_out = outer_split(M0);
  T* P0 = SA + k0 * ld + k0;
  const int64_t vc = gram ? bw : 0;  // V's own columns in the product
  const int64_t ncols = vc + nc, ncols_m = vc + nc_m;
  const int64_t ldw = pad32(ncols), ldwp = pad32(nc);
  T* Bc = P0 + bw + off;  // first product column when V is not included
  // V^T [V | C] (or V^T C) in row slices summed in order: rows [0, bw) hold the
  // triangle of V (masked, general kernel); the rows below are clear of every
  // mask, so a whole number of 16-row chunks of them goes to the clean-only
  // kernel in split_out-row slices, and a tail of fewer than 16 rows (if any) to the
  // general kernel without masks
  const int64_t Kc = (M0 - bw) / 16 * 16, Kt = M0 - bw - Kc;
  const int64_t nsc = (Kc + split_out - 1) / split_out;
  const int64_t nsp = 1 + nsc + (Kt > 0 ? 1 : 0);
  const int64_t zs = bw * ldw;
  auto product = [&](int64_t r0, int64_t rows, T* out, int64_t ksplit) {
    GemmArgs<T> g = vt_gemm<T>(P0 + r0 * ld, ld, rows, bw, ncols, out, ldw, ksplit);
    if (!gram) {
      g.B = Bc + r0 * ld;
      g.b_vcols = 0;
    }
    return g;
  };
  {
    Trace tr(h, gram ? "qr_gemm_VtC" : "qr_gemm_VtC_rest",
             sizeof(T) * ((double)M0 * ncols_m + 2.0 * (double)nsp * bw * ncols_m), 2.0 * (double)bw * ncols_m * M0);
    {
      // op(A) = V^T of the top rows is upper triangular (the mask zeroes the
      // rest): each row tile starts its K range at its own first row
      GemmArgs<T> gt = product(0, bw, tb.Wz, 0);
      gt.a_upper = 1;
      RFMLS_HIP(h, (gemm<T, GemmRole::QrVtC>(gt, st)));
    }
    if (Kc > 0) {
      GemmArgs<T> gc = product(bw, Kc, tb.Wz + zs, split_out);
      gc.a_vmask = 0;
      gc.b_vcols = 0;
      // the kOuter / 64 row tiles of a B strip run together (56 -> 59 TFLOP/s,
      // float64, 256-column blocks) on one XCD (then 481 -> 469 ms on the
      // 4^3-box float64 solve's 512-column blocks, equal at 256)
      gc.tile_order = 3;
      RFMLS_HIP(h, (gemm_clean<T, GemmRole::QrVtC>(gc, st)));
    }
    if (Kt > 0) {
      GemmArgs<T> gr = product(bw + Kc, Kt, tb.Wz + (1 + nsc) * zs, 0);
      gr.a_vmask = 0;
      gr.b_vcols = 0;
      RFMLS_HIP(h, (gemm<T, GemmRole::QrVtC>(gr, st)));
    }
    hipLaunchKernelGGL(k_sum_slices<T>, dim3(ceil_div(bw * ldw, 256) < 4096 ? ceil_div(bw * ldw, 256) : 4096),
                       dim3(256), 0, st, (const T*)tb.Wz, bw * ldw, (int)nsp, zs, tb.W);
  }
  if (gram) {
    // the last panel's T (no inner update followed it) from the Gram's
    // diagonal block; the other panels wrote theirs into To's diagonal
    Trace tr(h, "qr_outer_T", sizeof(T) * 2.0 * kMaxNb * kMaxNb, 2.0 * (double)kMaxNb * kMaxNb * kMaxNb / 3.0);
    const int64_t q0 = (bw - 1) / kMaxNb * kMaxNb;
    const int jq = (int)(bw - q0);
    hipLaunchKernelGGL(k_qr_buildT<T>, dim3((jq + 15) / 16), dim3(1024), 0, st, (const T*)(tb.W + q0 * ldw + q0),
                       (int64_t)0, 1, ldw, jq, (const T*)(tau + q0), To + q0 * kOuter + q0, (int64_t)kOuter);
    if (keep_gram)
      hipLaunchKernelGGL(k_qr_keep_gram<T>, dim3((unsigned)ceil_div(bw * bw, 256)), dim3(256), 0, st,
                         (const T*)tb.W, ldw, (int)bw, To, kOuter);
  }
  {
    // W' = T_o^T W[:, C's columns] by forward substitution with the Gram's
    // blocks (from this product, or kept in To by an earlier one) and the
    // panels' T
    Trace tr(h, "qr_outer_Wp", sizeof(T) * 2.0 * (double)bw * nc_m, (double)bw * bw * nc_m);
    const T* Gp = gram ? tb.W : To;
    const int64_t ldg = gram ? ldw : kOuter;
    const unsigned nb = (unsigned)ceil_div(nc, 16);
    if (bw == 4 * kMaxNb)
      hipLaunchKernelGGL((k_qr_outer_wp<T, 4>), dim3(nb), dim3(256), 0, st, (const T*)(tb.W + vc), ldw, Gp, ldg,
                         (const T*)To, kOuter, nc, tb.Wp, ldwp);
    else if (bw == 8 * kMaxNb)
      hipLaunchKernelGGL((k_qr_outer_wp<T, 8>), dim3(nb), dim3(256), 0, st, (const T*)(tb.W + vc), ldw, Gp, ldg,
                         (const T*)To, kOuter, nc, tb.Wp, ldwp);
    else
      return fail(h, RFMLS_E_ARG, "outer block of %lld columns", (long long)bw);
  }
  {
    Trace tr(h, gram ? "qr_gemm_update" : "qr_gemm_update_rest",
             sizeof(T) * (2.0 * (double)M0 * nc_m + (double)M0 * bw + (double)bw * nc_m), 2.0 * (double)M0 * nc_m * bw);
    // rows [0, bw) meet the triangle of V (masked, general kernel); the rows
    // below are clear of it and take the clean-only kernel
    {
      // V's top rows are lower triangular (the mask zeroes the rest): each
      // row tile ends its K range at its own last row
      GemmArgs<T> gt = v_update<T>(P0, ld, bw, bw, nc, tb.Wp, ldwp);
      gt.C = P0 + bw + off;
      gt.a_lower = 1;
      RFMLS_HIP(h, (gemm<T, GemmRole::QrTrailingUpdate>(gt, st)));
    }
    if (M0 > bw) {
      GemmArgs<T> gu = v_update<T>(P0 + bw * ld, ld, M0 - bw, bw, nc, tb.Wp, ldwp);
      gu.C = P0 + bw * ld + bw + off;
      gu.a_vmask = 0;
      gu.tile_order = 2;  // bands of 32 tile rows: 53.8 -> 56.5 TFLOP/s (float64, 51200 x 12800)
      RFMLS_HIP(h, (gemm_clean<T, GemmRole::QrTrailingUpdate>(gu, st)));
    }
  }
  RFMLS_HIP(h, hipGetLastError());
  return RFMLS_OK;
}

// Second stream and its two events for the look-ahead (created on first use).
rfmls_status lookahead_stream(rfmls_handle* h) {
  if (h->la_stream) return RFMLS_OK;
  if (hipStreamCreateWithFlags(&h->la_stream, hipStreamNonBlocking) != hipSuccess) {
    h->la_stream = nullptr;
    return fail(h, RFMLS_E_HIP, "QR look-ahead: could not create its stream");
  }
  for (int i = 0; i < 2; ++i)
    if (hipEventCreateWithFlags(&h->la_event[i], hipEventDisableTiming) != hipSuccess)
      return fail(h, RFMLS_E_HIP, "QR look-ahead: could not create its events");
  return RFMLS_OK;
}

// n_room >= n columns of SA may be written: the big trailing products round
// their column count up to the tile width inside that room (full tiles, no
// ragged edge); the extra columns only ever hold values nothing reads.
//
// Look-ahead (rfmls_qr_lookahead, float64 CholeskyQR2 panels only): after the
// panels of outer block k, the trailing update first covers only block k + 1's
// columns; block k + 1's panels then run on a second stream while the main
// stream updates the remaining columns, and the main stream waits for them
// before block k + 1's own trailing update.  The split is by columns, every
// column's sums run in the same order, and the two streams touch disjoint
// columns and buffers (T_o and tau alternate between two copies, the panels
// have their own product buffers), so the factors are bitwise the same.
template <typename T>
rfmls_status qr_impl(rfmls_handle* h, int64_t s, int64_t n, int64_t n_room, T* SA, int64_t ld, T* tau_out) {
  const int64_t kOuter = outer_width<T>(n);
  const int64_t nsp_in_max = inner_slices_max(s);
  const int64_t nsp_out_max = outer_slices_max(s);
  void *p_tau, *p_part, *p_wz, *p_w, *p_wp, *p_to, *p_in;
  RFMLS_CHECK(workspace(h, WS_QR_TAU, sizeof(T) * 2 * kOuterMax, &p_tau));
  RFMLS_CHECK(workspace(h, WS_QR_PART, sizeof(uint64_t) * ll_words(kPanelMaxBlocks), &p_part));
  // rows of the products W, W' are padded to 32 elements (128-byte aligned
  // rows for every column count)
  const int64_t npad = pad32(n_room);
  const size_t wz_out = (size_t)nsp_out_max * kOuter * (size_t)npad;
  RFMLS_CHECK(workspace(h, WS_QR_W, sizeof(T) * wz_out, &p_wz));
  RFMLS_CHECK(workspace(h, WS_QR_WR, sizeof(T) * kOuter * (size_t)npad, &p_w));
  RFMLS_CHECK(workspace(h, WS_QR_WP, sizeof(T) * kOuter * (size_t)npad, &p_wp));
  RFMLS_CHECK(workspace(h, WS_QR_T, sizeof(T) * 2 * kOuter * kOuter, &p_to));
  // the panels' own product buffers: slices, Gram and T^T W of at most
  // 64 x kOuter each
  const int64_t kop = pad32(kOuter);
  const size_t in_wz = (size_t)nsp_in_max * kMaxNb * kop, in_w = (size_t)kMaxNb * kop;
  RFMLS_CHECK(workspace(h, WS_QR_INNER, sizeof(T) * (in_wz + 2 * in_w), &p_in));
  // CholeskyQR2 panels (rfmls_qr_panel_mode): workspace for the largest
  // panel and one status word after it
  double* cq_ws = nullptr;
  int* cq_status = nullptr;
  if (h->qr_panel != 1 && s >= kCholqrMinRows) {
    const int64_t nd = cholqr_workspace_doubles(s);
    void* p_cq;
    RFMLS_CHECK(workspace(h, WS_CHOLQR, sizeof(double) * (size_t)(nd + 8), &p_cq));
    cq_ws = (double*)p_cq;
    cq_status = (int*)(cq_ws + nd);
  }
  // only panels that never wait on each other's workgroups may run beside the
  // trailing products: CholeskyQR2 in its normal mode
  const bool lookahead = h->qr_lookahead && cq_ws && h->qr_panel == 0;
  if (lookahead) RFMLS_CHECK(lookahead_stream(h));
  hipStream_t st = h->stream;
  T* tau2[2] = {(T*)p_tau, (T*)p_tau + kOuterMax};
  T* To2[2] = {(T*)p_to, (T*)p_to + kOuter * kOuter};
  const TrailBufs<T> tb = {(T*)p_wz, (T*)p_w, (T*)p_wp};
  T* in = (T*)p_in;
  uint64_t* ll = (uint64_t*)p_part;
  {
    // the panels' exchange slots, zeroed once: their tags are column indices
    const int64_t nll = ll_words(kPanelMaxBlocks);
    hipLaunchKernelGGL(k_zero_u64, dim3(ceil_div(nll, 256) < 512 ? ceil_div(nll, 256) : 512), dim3(256), 0, st, ll,
                       nll);
  }
  auto bufs = [&](int64_t blk) {
    PanelBufs<T> pb = {tau2[blk & 1], To2[blk & 1], in, in + in_wz, in + in_wz + in_w};
    return pb;
  };
  // block k + 1's panels all CholeskyQR2-eligible (64 columns, enough rows)
  auto cq_block = [&](int64_t k1, int64_t bw1) { return bw1 % kMaxNb == 0 && s - (k1 + bw1 - kMaxNb) >= kCholqrMinRows; };
  RFMLS_CHECK(qr_block_panels<T>(h, s, 0, n < kOuter ? n : kOuter, kOuter, SA, ld, bufs(0), ll, cq_ws, cq_status,
                                 tau_out));
  int64_t blk = 0;
  for (int64_t k0 = 0; k0 < n; k0 += kOuter, ++blk) {
    const int64_t bw = n - k0 < kOuter ? n - k0 : kOuter;
    if (n - k0 - bw <= 0) break;
    const int64_t k1 = k0 + bw, bw1 = n - k1 < kOuter ? n - k1 : kOuter;
    // columns right of the block, rounded up to the widest tile (128) within
    // the room; the method's own are the traced work
    const int64_t ntr = (n_room < (n + 127) / 128 * 128 ? n_room : (n + 127) / 128 * 128) - k0 - bw;
    const int64_t ntr_m = n - k0 - bw;
    const PanelBufs<T> pb = bufs(blk), pb1 = bufs(blk + 1);
    if (lookahead && ntr_m > kOuter && cq_block(k1, bw1)) {
      // block k + 1's columns first, its panels on the second stream, the rest here
      RFMLS_CHECK(qr_block_trailing<T>(h, s, k0, bw, kOuter, SA, ld, 0, kOuter, kOuter, true, pb.tau, pb.To, tb,
                                       true));
      RFMLS_HIP(h, hipEventRecord(h->la_event[0], st));
      RFMLS_HIP(h, hipStreamWaitEvent(h->la_stream, h->la_event[0], 0));
      h->stream = h->la_stream;
      const rfmls_status ps =
          qr_block_panels<T>(h, s, k1, bw1, kOuter, SA, ld, pb1, ll, cq_ws, cq_status, tau_out);
      const hipError_t er = hipEventRecord(h->la_event[1], h->la_stream);
      h->stream = st;
      RFMLS_CHECK(ps);
      RFMLS_HIP(h, er);
      const rfmls_status ts = qr_block_trailing<T>(h, s, k0, bw, kOuter, SA, ld, kOuter, ntr - kOuter,
                                                   ntr_m - kOuter, false, pb.tau, pb.To, tb);
      RFMLS_HIP(h, hipStreamWaitEvent(st, h->la_event[1], 0));
      RFMLS_CHECK(ts);
    } else {
      RFMLS_CHECK(qr_block_trailing<T>(h, s, k0, bw, kOuter, SA, ld, 0, ntr, ntr_m, true, pb.tau, pb.To, tb));
      RFMLS_CHECK(qr_block_panels<T>(h, s, k1, bw1, kOuter, SA, ld, pb1, ll, cq_ws, cq_status, tau_out));
    }
  }
  return RFMLS_OK;
}

}  // namespace

rfmls_status run_qr(rfmls_handle* h, int64_t s, int64_t n, int64_t n_room, rfmls_dtype dt, void* SA,
                    int64_t ld, void* tau_out) {
  if (n_room < n || n_room > ld) n_room = n;
  if (dt == RFMLS_F64) return qr_impl<double>(h, s, n, n_room, (double*)SA, ld, (double*)tau_out);
  return qr_impl<float>(h, s, n, n_room, (float*)SA, ld, (float*)tau_out);
}

// Y <- Q Y with Q = H_0 H_1 ... H_{n-1} of a float64 Householder QR left by
// run_qr in P (s x n, vectors below the diagonal, tau from its tau_out): the
// 64-column panels from last to first, each as Y <- (I - V T V^T) Y with
// T from the panel's Gram V^T V and tau, i.e. W = V^T Y, W' = T W, Y -= V W'.
rfmls_status apply_householder(rfmls_handle* h, const double* P, int64_t ld, int64_t s, int64_t n,
                               const double* tau, double* Y, int64_t ldy, int64_t ny) {
  hipStream_t st = h->stream;
  const int64_t ldw = (ny + 31) / 32 * 32;
  void* pw;
  RFMLS_CHECK(workspace(h, WS_APPLYQ, sizeof(double) * (size_t)(2 * kMaxNb * kMaxNb + 2 * kMaxNb * ldw), &pw));
  double* G = (double*)pw;
  double* Tq = G + kMaxNb * kMaxNb;
  double* W = Tq + kMaxNb * kMaxNb;
  double* Wp = W + kMaxNb * ldw;
  for (int64_t p0 = (n - 1) / kMaxNb * kMaxNb; p0 >= 0; p0 -= kMaxNb) {
    const int jb = (int)(n - p0 < kMaxNb ? n - p0 : kMaxNb);
    const int64_t M = s - p0;
    double* V = const_cast<double*>(P) + p0 * ld + p0;
    RFMLS_HIP(h, (gemm<double, GemmRole::Generic>(vt_gemm<double>(V, ld, M, jb, jb, G, kMaxNb, 0), st)));
    hipLaunchKernelGGL(k_qr_buildT<double>, dim3((jb + 15) / 16), dim3(1024), 0, st, (const double*)G, (int64_t)0, 1,
                       (int64_t)kMaxNb, jb, tau + p0, Tq, (int64_t)kMaxNb);
    GemmArgs<double> gw;  // W = V^T Y[p0:, :]
    gw.M = jb;
    gw.N = ny;
    gw.K = M;
    gw.A = V;
    gw.lda = ld;
    gw.transA = 1;
    gw.a_vmask = 1;
    gw.B = Y + p0 * ldy;
    gw.ldb = ldy;
    gw.C = W;
    gw.ldc = ldw;
    RFMLS_HIP(h, (gemm<double, GemmRole::Generic>(gw, st)));
    GemmArgs<double> gt;  // W' = T W (T upper triangular)
    gt.M = jb;
    gt.N = ny;
    gt.K = jb;
    gt.A = Tq;
    gt.lda = kMaxNb;
    gt.a_upper = 1;
    gt.B = W;
    gt.ldb = ldw;
    gt.C = Wp;
    gt.ldc = ldw;
    RFMLS_HIP(h, (gemm<double, GemmRole::Generic>(gt, st)));
    GemmArgs<double> gu;  // Y[p0:, :] -= V W'
    gu.M = M;
    gu.N = ny;
    gu.K = jb;
    gu.A = V;
    gu.lda = ld;
    gu.a_vmask = 1;
    gu.B = Wp;
    gu.ldb = ldw;
    gu.C = Y + p0 * ldy;
    gu.ldc = ldy;
    gu.alpha = -1.0;
    gu.beta = 1.0;
    RFMLS_HIP(h, (gemm<double, GemmRole::Generic>(gu, st)));
  }
  RFMLS_HIP(h, hipGetLastError());
  return RFMLS_OK;
}

}  // namespace rfmls
