// Tiled GEMM on CDNA matrix cores (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32)
// used by the blocked Householder QR (compact-WY trailing updates) and the
// blocked triangular inversion.
//
//   C[M x N] = alpha * op(A)[M x K] * B[K x N] + beta * C      (row-major)
//
// op(A) = A (A[i*lda + k]) or A^T (A[k*lda + i]).  Optional operand masks:
//   - "Householder" mask: the operand is the matrix V of Householder vectors
//     stored below the diagonal of a QR panel; element (r, c) of V in panel
//     coordinates reads 0 for r < c, 1 for r == c and the stored value for
//     r > c.  For A the panel coordinates are (r, c) = (i, k) (no transpose) or
//     (k, i) (transpose); for B they are (k, j) for the first b_vcols columns.
//   - triangular operands: op(A) upper (k >= i only) or lower (k <= i only)
//     triangular and/or B upper triangular (k <= j only); zero K-tiles are
//     skipped and the zero triangle is never read (it may hold anything),
//     unless b_lower_zero says that B's entries below the diagonal inside the
//     K range of each 64-column tile are stored zeros: then they are read as
//     they are and a diagonal chunk needs no mask.
// Split-K: blockIdx.z selects the K range [z*ksplit, (z+1)*ksplit) and output
// C + z*c_zstride (each slice writes its own partial result, no atomics).
//
// Block: 256 threads = 4 waves in a 2 x 2 grid computing a 64 x 64 (float64)
// or up to 128 x 128 (float32) tile of C, each wave a quarter of it as 16 x 16
// MFMA tiles.  K is staged through LDS in steps of 16, the next step
// prefetched into registers.
#pragma once

#include "common.h"

namespace rfmls {

template <typename T>
struct GemmArgs {
  int64_t M = 0, N = 0, K = 0;
  const T* A = nullptr;
  int64_t lda = 0;
  int transA = 0;
  const T* B = nullptr;
  int64_t ldb = 0;
  T* C = nullptr;
  int64_t ldc = 0;
  T alpha = 1, beta = 0;
  int a_vmask = 0;      // A is V (Householder mask)
  int64_t b_vcols = 0;  // first b_vcols columns of B are V (Householder mask)
  int a_upper = 0;      // op(A) upper triangular
  int a_lower = 0;      // op(A) lower triangular
  int b_upper = 0;      // B upper triangular
  int b_lower_zero = 0; // with b_upper: B's lower triangle holds zeros where read
  int64_t ksplit = 0;   // 0 = no split
  int64_t c_zstride = 0;
  int tile_order = 0;   // order the tiles are issued in (see k_gemm)
};

// What a GEMM launch is for.  The role only names the kernel symbol (so that
// profiles separate the uses); the code is the same for every role.
enum class GemmRole : int {
  Generic = 0,
  QrTrailingUpdate = 1,  // C <- C - V (T^T W) after an outer block
  QrVtC = 2,             // W = V^T [V | C] of an outer block
  QrInnerUpdate = 3,     // the same two products inside an outer block
  QrInnerVtC = 4,
  Inverse = 6,           // blocked inversion of R
};

namespace gemm_detail {

constexpr int PAD = 4;

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
// Operand layouts (both instructions): lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16].  Accumulator register r of lane l holds D[row][l % 16] with
//   f64 16x16x4:  row = l / 16 + 4 r      (rows interleaved)
//   f32 16x16x4:  row = 4 (l / 16) + r    (rows blocked)
template <>
struct Mfma<double> {
  typedef v4d acc_t;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct Mfma<float> {
  typedef v4f acc_t;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) * 4 + r; }
};

template <typename T>
__device__ __forceinline__ T vmask(int64_t r, int64_t c, T v) {
  return r < c ? T(0) : (r == c ? T(1) : v);
}

// Tile load helpers: element (i, k) of op(A) and (k, j) of B with masks and bounds.
template <typename T>
__device__ __forceinline__ T load_a(const GemmArgs<T>& g, int64_t gi, int64_t gk, int64_t kend) {
  T v = T(0);
  if (gi < g.M && gk < kend && !(g.a_upper && gk < gi) && !(g.a_lower && gk > gi)) {
    if (!g.transA) {
      v = g.A[gi * g.lda + gk];
      if (g.a_vmask) v = vmask<T>(gi, gk, v);
    } else {
      v = g.A[gk * g.lda + gi];
      if (g.a_vmask) v = vmask<T>(gk, gi, v);
    }
  }
  return v;
}
template <typename T>
__device__ __forceinline__ T load_b(const GemmArgs<T>& g, int64_t gk, int64_t gj, int64_t kend) {
  T v = T(0);
  if (gj < g.N && gk < kend && !(g.b_upper && gk > gj)) {
    v = g.B[gk * g.ldb + gj];
    if (gj < g.b_vcols) v = vmask<T>(gk, gj, v);
  }
  return v;
}

// Block tile BMt x BNt (each 64 or 128) with K chunks of BKt; 4 waves in a
// 2 x 2 grid, each wave (BMt/2) x (BNt/2) made of 16 x 16 MFMA tiles.  The
// next K chunk is fetched from global memory into registers while the current
// one is consumed from LDS, so the loads overlap the matrix-core work.
// A chunk clear of every mask and triangle and inside the K range ("clean",
// decided per block, so the branch is uniform) is read through precomputed
// pointers with no per-element tests, or with one bound test per element on
// a tile over the matrix's last rows or columns; only chunks on a diagonal, a
// mask border or the end of the K range take the element-wise path.
// CleanOnly: the instantiation for launches whose every chunk is clean (no
// mask, no triangle, every block's K range a whole number of chunks; checked by
// gemm_clean on the host): the element-wise path is not compiled in, which
// leaves 74 instead of 109 VGPRs for the float64 64 x 64 tile (6 instead of 4
// wavefronts per SIMD).
template <typename T, int BMt, int BNt, int BKt, int WM, int WN, GemmRole Role, bool CleanOnly = false>
__global__ void __launch_bounds__(64 * WM * WN) k_gemm(GemmArgs<T> g) {
  constexpr int NT = 64 * WM * WN;               // threads: WM x WN wavefronts
  constexpr int WTM = BMt / WM, WTN = BNt / WN;  // wave tile
  constexpr int TM = WTM / 16, TN = WTN / 16;    // MFMA tiles per wave per dim
  constexpr int EA = BMt * BKt / NT;             // A elements per thread per chunk
  constexpr int EB = BNt * BKt / NT;             // B elements per thread per chunk
  static_assert(EA >= 1 && EB >= 1 && BKt % EA == 0 && TM >= 1 && TN >= 1, "tile shape");
  __shared__ T As[BKt][BMt + PAD];
  __shared__ T Bs[BKt][BNt + PAD];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wy = wave / WN, wx = wave % WN;
  // Tile order: 0 row by row (grid x = tile column); 1 column by column
  // (grid x = tile row), which runs the tiles that share a B column strip
  // together; 3 the same with each column's tiles on one XCD; 2 in bands of
  // 32 tile rows, each band column by column, so a band's A strips stay in L2
  // while its B strips are each read for 32 tiles in a row.  Triangular operands make the K range grow with the tile column
  // (B upper: k <= j) or row (op(A) lower: k <= i); those tiles are issued
  // first (reversed order) so the longest blocks do not form a tail at the
  // end of the grid.
  unsigned gx = g.tile_order == 1 ? blockIdx.y : blockIdx.x, nx = g.tile_order == 1 ? gridDim.y : gridDim.x;
  unsigned gy = g.tile_order == 1 ? blockIdx.x : blockIdx.y, ny = g.tile_order == 1 ? gridDim.x : gridDim.y;
  if (g.tile_order == 3) {
    // column by column, XCD-aware: workgroups are dealt to the 8 XCDs in
    // turn, so XCD x runs linear ids x, x + 8, ...; its k-th workgroup takes
    // row k % ny of column x + 8 (k / ny), so a column's row tiles share one
    // L2.  The columns past the last whole group of 8 follow in plain column
    // order.
    const unsigned L = blockIdx.x + blockIdx.y * gridDim.x;
    const unsigned nc8 = nx & ~7u, full = ny * nc8;
    if (L < full) {
      const unsigned k = L >> 3;
      gx = (L & 7u) + 8u * (k / ny);
      gy = k % ny;
    } else {
      gx = nc8 + (L - full) / ny;
      gy = (L - full) % ny;
    }
  }
  if (g.tile_order == 2) {
    constexpr unsigned kBand = 32;
    const unsigned L = blockIdx.x + blockIdx.y * gridDim.x;
    const unsigned r0 = L / (kBand * nx) * kBand, idx = L % (kBand * nx);
    const unsigned gm = ny - r0 < kBand ? ny - r0 : kBand;
    gx = idx / gm;
    gy = r0 + idx % gm;
  }
  const unsigned bx = g.b_upper ? nx - 1 - gx : gx;
  const unsigned by = g.a_lower ? ny - 1 - gy : gy;
  const int64_t i0 = (int64_t)by * BMt;
  const int64_t j0 = (int64_t)bx * BNt;
  int64_t kbeg = 0, kend = g.K;
  if (g.ksplit > 0) {
    kbeg = (int64_t)blockIdx.z * g.ksplit;
    kend = kbeg + g.ksplit < g.K ? kbeg + g.ksplit : g.K;
  }
  if (g.a_upper && i0 > kbeg) kbeg = i0;
  if (g.a_lower) {
    const int64_t lim = i0 + BMt;
    if (lim < kend) kend = lim;
  }
  if (g.b_upper) {
    const int64_t lim = j0 + BNt;
    if (lim < kend) kend = lim;
  }
  T* C = g.C + (int64_t)blockIdx.z * g.c_zstride;

  typename Mfma<T>::acc_t acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = typename Mfma<T>::acc_t{0, 0, 0, 0};

  // thread -> element mapping of the staging loads (contiguous runs in memory)
  // op(A) not transposed: row ra_i = tid / (BKt/EA), k run of EA starting at ra_k
  // op(A) transposed:     k = ra_k, run of EA along i starting at ra_i
  // B:                    k = rb_k, run of EB along j starting at rb_j
  const int ra_i = g.transA ? (tid % (BMt / EA)) * EA : tid / (BKt / EA);
  const int ra_k = g.transA ? tid / (BMt / EA) : (tid % (BKt / EA)) * EA;
  const int rb_k = tid / (BNt / EB);
  const int rb_j = (tid % (BNt / EB)) * EB;
  // pointers for the clean path (only dereferenced for clean chunks)
  const T* pa = g.transA ? g.A + (int64_t)ra_k * g.lda + (i0 + ra_i) : g.A + (i0 + ra_i) * g.lda + ra_k;
  const T* pb = g.B + (int64_t)rb_k * g.ldb + (j0 + rb_j);
  // block-uniform parts of the clean test
  const bool a_rows_in = i0 + BMt <= g.M;
  const bool b_cols_in = j0 + BNt <= g.N;
  // a chunk inside the K range and clear of every mask and triangle (the
  // bounds of the tile's block of rows or columns aside)
  auto clean = [&](int64_t k0) {
    if (k0 + BKt > kend) return false;
    const int64_t klast = k0 + BKt - 1, ilast = i0 + BMt - 1, jlast = j0 + BNt - 1;
    if (g.a_upper && k0 < ilast) return false;
    if (g.a_lower && klast > i0) return false;
    if (g.a_vmask && (g.transA ? !(k0 > ilast) : !(i0 > klast))) return false;
    if (g.b_upper && !g.b_lower_zero && klast > j0) return false;
    if (j0 < g.b_vcols && !(k0 > jlast)) return false;
    return true;
  };
  T ra[EA], rb[EB];
  auto fetch = [&](int64_t k0) {
    if (CleanOnly || clean(k0)) {
      const T* a = g.transA ? pa + k0 * g.lda : pa + k0;
      const T* b = pb + k0 * g.ldb;
      if (a_rows_in && b_cols_in) {
#pragma unroll
        for (int q = 0; q < EA; ++q) ra[q] = a[q];
#pragma unroll
        for (int q = 0; q < EB; ++q) rb[q] = b[q];
      } else {
        // a tile over the last rows or columns: a thread's run of EA (EB)
        // elements inside the matrix is loaded as one run, as on the interior
        // path (vector loads); a run outside reads zeros, and only a run
        // across the edge goes element by element
        const int64_t ia = i0 + ra_i, jb = j0 + rb_j;
        const int64_t a_in = g.transA ? g.M - ia : (ia < g.M ? EA : 0);  // run elements inside
        if (a_in >= EA) {
#pragma unroll
          for (int q = 0; q < EA; ++q) ra[q] = a[q];
        } else {
#pragma unroll
          for (int q = 0; q < EA; ++q) ra[q] = q < a_in ? a[q] : T(0);
        }
        const int64_t b_in = g.N - jb;
        if (b_in >= EB) {
#pragma unroll
          for (int q = 0; q < EB; ++q) rb[q] = b[q];
        } else {
#pragma unroll
          for (int q = 0; q < EB; ++q) rb[q] = q < b_in ? b[q] : T(0);
        }
      }
      return;
    }
    if (CleanOnly) return;
    if (!g.transA) {
#pragma unroll
      for (int q = 0; q < EA; ++q) ra[q] = load_a(g, i0 + ra_i, k0 + ra_k + q, kend);
    } else {
#pragma unroll
      for (int q = 0; q < EA; ++q) ra[q] = load_a(g, i0 + ra_i + q, k0 + ra_k, kend);
    }
#pragma unroll
    for (int q = 0; q < EB; ++q) rb[q] = load_b(g, k0 + rb_k, j0 + rb_j + q, kend);
  };
  auto stash = [&]() {
    if (!g.transA) {
#pragma unroll
      for (int q = 0; q < EA; ++q) As[ra_k + q][ra_i] = ra[q];
    } else {
#pragma unroll
      for (int q = 0; q < EA; ++q) As[ra_k][ra_i + q] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < EB; ++q) Bs[rb_k][rb_j + q] = rb[q];
  };

  if (kbeg < kend) fetch(kbeg);
  for (int64_t k0 = kbeg; k0 < kend; k0 += BKt) {
    __syncthreads();
    stash();
    __syncthreads();
    if (k0 + BKt < kend) fetch(k0 + BKt);
#pragma unroll
    for (int ks = 0; ks < BKt; ks += 4) {
      const int kr = ks + (lane >> 4);
      T av[TM], bv[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) av[a] = As[kr][wy * WTM + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < TN; ++b) bv[b] = Bs[kr][wx * WTN + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = Mfma<T>::op(av[a], bv[b], acc[a][b]);
    }
  }
  // ---- epilogue: register r of each 16x16 tile is element (Mfma::row(lane, r), lane % 16) ----
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = i0 + wy * WTM + a * 16 + Mfma<T>::row(lane, r);
        const int64_t gj = j0 + wx * WTN + b * 16 + (lane & 15);
        if (gi < g.M && gj < g.N) {
          T v = g.alpha * acc[a][b][r];
          if (g.beta != T(0)) v += g.beta * C[gi * g.ldc + gj];
          C[gi * g.ldc + gj] = v;
        }
      }
}

}  // namespace gemm_detail

namespace gemm_detail {
template <typename T, GemmRole Role, bool CleanOnly>
inline hipError_t launch(const GemmArgs<T>& g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  unsigned gz = 1;
  if (g.ksplit > 0) gz = (unsigned)((g.K + g.ksplit - 1) / g.ksplit);
  if (gz == 0) gz = 1;
  // Tiles measured fastest at the QR's shapes on gfx950: 64 x 64 (higher
  // occupancy beats larger register tiles), except float32 products with a
  // long K range (W = V^T [V | C] over 8192-row slices) and, on the clean-only
  // instance, float32 products with K >= 256 (the trailing update: 112 -> 123
  // TFLOP/s in isolation), which prefer 128 x 128.
  const int64_t kspan = g.ksplit > 0 ? g.ksplit : g.K;
  if (sizeof(T) == 4 && g.M > 64 && g.N > 64 && (kspan >= 1024 || (CleanOnly && kspan >= 256))) {
    const unsigned tn = (unsigned)((g.N + 127) / 128), tm = (unsigned)((g.M + 127) / 128);
    dim3 grid(g.tile_order == 1 ? tm : tn, g.tile_order == 1 ? tn : tm, gz);
    hipLaunchKernelGGL((k_gemm<T, 128, 128, 16, 2, 2, Role, CleanOnly>), grid, dim3(256), 0, st, g);
  } else {
    const unsigned tn = (unsigned)((g.N + 63) / 64), tm = (unsigned)((g.M + 63) / 64);
    dim3 grid(g.tile_order == 1 ? tm : tn, g.tile_order == 1 ? tn : tm, gz);
    if constexpr (sizeof(T) == 8 && CleanOnly && (Role == GemmRole::QrVtC || Role == GemmRole::Inverse)) {
      // float64 W = V^T [V | C] over 4096-row slices: K chunks of 8 and at
      // most four workgroups per compute unit (a dynamic LDS reservation that
      // brings each workgroup to a quarter of the 160 KB): 67.5 -> 71.1
      // TFLOP/s on 256 x 11,776 x 49,920 in isolation (fewer slabs of [V | C]
      // streamed at once per L2); in the pipeline 64.1 -> 66.0 TFLOP/s on the
      // 4^3-box float64 sketch (1.254 -> 1.243 s), within the run-to-run spread
      // on the 8x8-box one.  The blocked inversion's products (long K, split
      // into slices) take the same shape: 54 -> 57-60 TFLOP/s (8x8-box),
      // 57-58 -> 60 (4^3-box).  Same K order, so the same bits.
      constexpr size_t kStatic = sizeof(T) * 8 * 2 * (64 + PAD);
      constexpr size_t kCapLds = 163840 / 4 - kStatic;
      hipLaunchKernelGGL((k_gemm<T, 64, 64, 8, 2, 2, Role, CleanOnly>), grid, dim3(256), kCapLds, st, g);
      return hipGetLastError();
    }
    if (sizeof(T) == 8 && CleanOnly && Role == GemmRole::QrTrailingUpdate)
      // float64 trailing update (K = 256, C read and written): four wavefronts
      // stacked along the rows, each 16 x 64, and K chunks of 8 (58.4-59.8 ->
      // 62.1 TFLOP/s on 49,920 x 11,520 x 256 in isolation); the products keep
      // their K order, so the results are the same bits
      hipLaunchKernelGGL((k_gemm<T, 64, 64, 8, 4, 1, Role, CleanOnly>), grid, dim3(256), 0, st, g);
    else
      hipLaunchKernelGGL((k_gemm<T, 64, 64, 16, 2, 2, Role, CleanOnly>), grid, dim3(256), 0, st, g);
  }
  return hipGetLastError();
}
}  // namespace gemm_detail

template <typename T, GemmRole Role = GemmRole::Generic>
inline hipError_t gemm(const GemmArgs<T>& g, hipStream_t st) {
  return gemm_detail::launch<T, Role, false>(g, st);
}

// The same product on the clean-only instantiation when nothing needs the
// element-wise path: no mask, no triangle (except an upper-triangular B whose
// lower triangle is stored zeros) and every block's K range a whole number of
// 16-row chunks; otherwise the general kernel.
template <typename T, GemmRole Role = GemmRole::Generic>
inline hipError_t gemm_clean(const GemmArgs<T>& g, hipStream_t st) {
  const bool ok = !g.a_vmask && g.b_vcols == 0 && !g.a_upper && !g.a_lower && (!g.b_upper || g.b_lower_zero) &&
                  g.K % 16 == 0 && (g.ksplit == 0 || g.ksplit % 16 == 0);
  if (ok) return gemm_detail::launch<T, Role, true>(g, st);
  return gemm_detail::launch<T, Role, false>(g, st);
}

}  // namespace rfmls
