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
//   - triangular skipping: op(A) upper triangular (k >= i only) and/or B upper
//     triangular (k <= j only); whole zero K-tiles are skipped.
// Split-K: blockIdx.z selects the K range [z*ksplit, (z+1)*ksplit) and output
// C + z*c_zstride (each slice writes its own partial result, no atomics).
//
// Block: 256 threads = 4 waves in a 2 x 2 grid; a block computes a 64 x 64
// tile of C, each wave a 32 x 32 sub-tile as 2 x 2 MFMA 16 x 16 tiles.  K is
// staged through LDS in steps of 16.
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
  int b_upper = 0;      // B upper triangular
  int64_t ksplit = 0;   // 0 = no split
  int64_t c_zstride = 0;
};

namespace gemm_detail {

constexpr int BM = 64, BN = 64, BK = 16, PAD = 4;

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

template <typename T>
__global__ void __launch_bounds__(256) k_gemm(GemmArgs<T> g) {
  __shared__ T As[BK][BM + PAD];
  __shared__ T Bs[BK][BN + PAD];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wy = wave >> 1, wx = wave & 1;
  const int64_t i0 = (int64_t)blockIdx.y * BM;
  const int64_t j0 = (int64_t)blockIdx.x * BN;
  int64_t kbeg = 0, kend = g.K;
  if (g.ksplit > 0) {
    kbeg = (int64_t)blockIdx.z * g.ksplit;
    kend = kbeg + g.ksplit < g.K ? kbeg + g.ksplit : g.K;
  }
  if (g.a_upper && i0 > kbeg) kbeg = i0 - (i0 % BK) > kbeg ? i0 - (i0 % BK) : kbeg;
  if (g.b_upper) {
    const int64_t lim = j0 + BN;
    if (lim < kend) kend = lim;
  }
  T* C = g.C + (int64_t)blockIdx.z * g.c_zstride;

  typename Mfma<T>::acc_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = typename Mfma<T>::acc_t{0, 0, 0, 0};

  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
    // ---- stage op(A) tile (BM x BK) into As[k][i] ----
    if (!g.transA) {
      const int r = tid >> 2;          // 0..63
      const int kk = (tid & 3) * 4;    // 0,4,8,12
      const int64_t gi = i0 + r;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t gk = k0 + kk + q;
        T v = T(0);
        if (gi < g.M && gk < kend) {
          v = g.A[gi * g.lda + gk];
          if (g.a_vmask) v = vmask<T>(gi, gk, v);
        }
        As[kk + q][r] = v;
      }
    } else {
      const int kk = tid >> 4;         // 0..15
      const int r = (tid & 15) * 4;    // 0..60
      const int64_t gk = k0 + kk;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t gi = i0 + r + q;
        T v = T(0);
        if (gi < g.M && gk < kend) {
          v = g.A[gk * g.lda + gi];
          if (g.a_vmask) v = vmask<T>(gk, gi, v);
        }
        As[kk][r + q] = v;
      }
    }
    // ---- stage B tile (BK x BN) into Bs[k][j] ----
    {
      const int kk = tid >> 4;
      const int c = (tid & 15) * 4;
      const int64_t gk = k0 + kk;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t gj = j0 + c + q;
        T v = T(0);
        if (gj < g.N && gk < kend) {
          v = g.B[gk * g.ldb + gj];
          if (gj < g.b_vcols) v = vmask<T>(gk, gj, v);
        }
        Bs[kk][c + q] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kr = ks + (lane >> 4);
      T a0 = As[kr][wy * 32 + (lane & 15)];
      T a1 = As[kr][wy * 32 + 16 + (lane & 15)];
      T b0 = Bs[kr][wx * 32 + (lane & 15)];
      T b1 = Bs[kr][wx * 32 + 16 + (lane & 15)];
      acc[0][0] = Mfma<T>::op(a0, b0, acc[0][0]);
      acc[0][1] = Mfma<T>::op(a0, b1, acc[0][1]);
      acc[1][0] = Mfma<T>::op(a1, b0, acc[1][0]);
      acc[1][1] = Mfma<T>::op(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }
  // ---- epilogue: register r of each 16x16 tile is element (Mfma::row(lane, r), lane % 16) ----
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = i0 + wy * 32 + a * 16 + Mfma<T>::row(lane, r);
        const int64_t gj = j0 + wx * 32 + b * 16 + (lane & 15);
        if (gi < g.M && gj < g.N) {
          T v = g.alpha * acc[a][b][r];
          if (g.beta != T(0)) v += g.beta * C[gi * g.ldc + gj];
          C[gi * g.ldc + gj] = v;
        }
      }
}

}  // namespace gemm_detail

template <typename T>
inline hipError_t gemm(const GemmArgs<T>& g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  unsigned gz = 1;
  if (g.ksplit > 0) gz = (unsigned)((g.K + g.ksplit - 1) / g.ksplit);
  if (gz == 0) gz = 1;
  dim3 grid((unsigned)((g.N + gemm_detail::BN - 1) / gemm_detail::BN),
            (unsigned)((g.M + gemm_detail::BM - 1) / gemm_detail::BM), gz);
  hipLaunchKernelGGL(gemm_detail::k_gemm<T>, grid, dim3(256), 0, st, g);
  return hipGetLastError();
}

}  // namespace rfmls
