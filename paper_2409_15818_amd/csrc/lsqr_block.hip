// Lockstep LSQR for a block of right-hand sides (up to kBlk = 32 at a time).
//
// Each column runs exactly the single-right-hand-side recurrences of lsqr.hip
// (its own alpha, beta, rotation, stopping test); the columns only share the
// passes over the matrices:
//   Z = X V        triangular product with the packed X = R^{-1}: each 64 x 64
//                  tile of X meets a 64 x 32 block of V on the matrix cores
//                  (v_mfma_f64_16x16x4f64), so X is streamed once per
//                  iteration for all 32 columns instead of 32 times
//   U = A Z - U a  CSR SpMM: 64-row groups times LDS-staged 32-wide input windows
//                  on the matrix cores
//   Q = A^T U      the same with the transpose
//   V = X^T Q - V b
// Vectors are interleaved row-major blocks (element (i, c) at i * 32 + c).
// A column that has stopped keeps its y and x; the host polls one
// "all columns done" flag every few iterations.
#include <algorithm>
#include <cstring>

#include "common.h"
#include "lsqr_dev.h"

namespace rfmls {

constexpr int kBlk = 32;

namespace {

constexpr int kThreads = 256;
constexpr int kSpmmMaxBlocks = 2048;  // capacity of the per-column partial-sum buffers
// Producers of per-column partial sums use at most these many blocks (grid-
// stride loops), and the single-block kernels that fold the partials into the
// column scalars use 1024 threads (32 columns x 32 slices).
constexpr int kSpmmBlocks = 512;
constexpr int kRowBlocks = 1024;  // 8-row blocks: enough loads in flight for the row-wise passes
constexpr int kRedThreads = 1024;

typedef double v4d __attribute__((ext_vector_type(4)));

struct BlockState {
  LsqrDev col[kBlk];
  int all_done;
  int pad[15];
};

__device__ __forceinline__ bool all_done(const BlockState* st) { return st->all_done != 0; }

// ---------------------------------------------------------------------------
// Triangular products with 64 x 32 blocks on the matrix cores.
// Wave w computes rows 16 w .. 16 w + 15 of the 64-row output block, both
// 16-column halves.  Operand layout of v_mfma_f64_16x16x4f64: lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator register r holds
// D[l / 16 + 4 r][l % 16].
// ---------------------------------------------------------------------------
// Z = X V for a 64-row tile row: each 64 x 64 tile of X is staged in LDS with
// coalesced loads (the next tile prefetched into registers meanwhile), as is
// the matching 64 x 32 block of V; the MFMA operands are then read from LDS.
// Reading the A operand (16 rows x 4 columns per instruction) straight from
// HBM would fetch 32-byte pieces of 16 different rows per load.
template <typename TS>
__global__ void __launch_bounds__(kThreads)
    k_trmm_part(const TS* __restrict__ Xpk, int64_t nt, int64_t n, int full, const int2* __restrict__ tab,
                int C, int maxk, const double* __restrict__ V, double* __restrict__ part,
                const BlockState* __restrict__ st) {
  if (st && all_done(st)) return;
  constexpr int kPer = kTile * kTile / kThreads;  // 16 X elements per thread per tile
  __shared__ TS Xs[kTile][kTile + 1];
  __shared__ double Vs[kTile][kBlk + 1];
  const int2 e = tab[blockIdx.x];
  const int64_t I = e.x;
  const int k = e.y;
  const int64_t J0 = row_first(I, full) + (int64_t)k * C;
  const int64_t J1 = J0 + C < nt ? J0 + C : nt;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  v4d acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
  TS xr[kPer];
  double vr[kTile * kBlk / kThreads];  // 8 V elements per thread
  auto fetch = [&](int64_t J) {
    const TS* t = Xpk + ptile(I, J, nt, full) * (int64_t)(kTile * kTile);
#pragma unroll
    for (int q = 0; q < kPer; ++q) xr[q] = t[tid + q * kThreads];
#pragma unroll
    for (int q = 0; q < kTile * kBlk / kThreads; ++q) {
      const int idx = tid + q * kThreads;  // (row, col) = (idx / 32, idx % 32)
      const int64_t r = J * kTile + idx / kBlk;
      vr[q] = r < n ? V[r * kBlk + (idx % kBlk)] : 0.0;
    }
  };
  if (J0 < J1) fetch(J0);
  for (int64_t J = J0; J < J1; ++J) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int idx = tid + q * kThreads;
      Xs[idx / kTile][idx % kTile] = xr[q];
    }
#pragma unroll
    for (int q = 0; q < kTile * kBlk / kThreads; ++q) {
      const int idx = tid + q * kThreads;
      Vs[idx / kBlk][idx % kBlk] = vr[q];
    }
    __syncthreads();
    if (J + 1 < J1) fetch(J + 1);
#pragma unroll
    for (int s4 = 0; s4 < kTile / 4; ++s4) {
      const int kk = 4 * s4 + lk;
      const double a = (double)Xs[16 * w + lr][kk];
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Vs[kk][lr], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Vs[kk][16 + lr], acc1, 0, 0, 0);
    }
  }
  double* o = part + ((int64_t)I * maxk + k) * (kTile * kBlk);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 16 * w + lk + 4 * r;
    o[row * kBlk + lr] = acc0[r];
    o[row * kBlk + 16 + lr] = acc1[r];
  }
}

// P = X^T Q for a 64-column tile column J: tiles I in [k C, min((k+1) C, J+1)),
// staged in LDS like k_trmm_part (the operand is the tile read transposed).
template <typename TS>
__global__ void __launch_bounds__(kThreads)
    k_trmmT_part(const TS* __restrict__ Xpk, int64_t nt, int64_t n, int full, const int2* __restrict__ tab,
                 int C, int maxk, const double* __restrict__ Qv, double* __restrict__ part,
                 const BlockState* __restrict__ st) {
  if (st && all_done(st)) return;
  constexpr int kPer = kTile * kTile / kThreads;
  __shared__ TS Xs[kTile][kTile + 1];
  __shared__ double Qs[kTile][kBlk + 1];
  const int2 e = tab[blockIdx.x];
  const int64_t J = e.x;
  const int k = e.y;
  const int64_t I0 = (int64_t)k * C;
  const int64_t Iend = col_end(J, nt, full);
  const int64_t I1 = I0 + C < Iend ? I0 + C : Iend;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  v4d acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
  TS xr[kPer];
  double qr[kTile * kBlk / kThreads];
  auto fetch = [&](int64_t I) {
    const TS* t = Xpk + ptile(I, J, nt, full) * (int64_t)(kTile * kTile);
#pragma unroll
    for (int q = 0; q < kPer; ++q) xr[q] = t[tid + q * kThreads];
#pragma unroll
    for (int q = 0; q < kTile * kBlk / kThreads; ++q) {
      const int idx = tid + q * kThreads;
      const int64_t r = I * kTile + idx / kBlk;
      qr[q] = r < n ? Qv[r * kBlk + (idx % kBlk)] : 0.0;
    }
  };
  if (I0 < I1) fetch(I0);
  for (int64_t I = I0; I < I1; ++I) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int idx = tid + q * kThreads;
      Xs[idx / kTile][idx % kTile] = xr[q];
    }
#pragma unroll
    for (int q = 0; q < kTile * kBlk / kThreads; ++q) {
      const int idx = tid + q * kThreads;
      Qs[idx / kBlk][idx % kBlk] = qr[q];
    }
    __syncthreads();
    if (I + 1 < I1) fetch(I + 1);
#pragma unroll
    for (int s4 = 0; s4 < kTile / 4; ++s4) {
      const int kk = 4 * s4 + lk;  // row of the X tile = column of X^T
      const double a = (double)Xs[kk][16 * w + lr];
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Qs[kk][lr], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Qs[kk][16 + lr], acc1, 0, 0, 0);
    }
  }
  double* o = part + ((int64_t)J * maxk + k) * (kTile * kBlk);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 16 * w + lk + 4 * r;
    o[row * kBlk + lr] = acc0[r];
    o[row * kBlk + 16 + lr] = acc1[r];
  }
}

// out[i][c] = sum_k part[...][i][c] - coef_c prev[i][c]; per-column partial sums of squares.
// coef_c = hcoef * coef[c * cstride] (coef may be null).  Thread (i, c) with c = tid % 32.
__global__ void __launch_bounds__(kThreads)
    k_blk_tri_reduce(const double* __restrict__ part, int64_t nt, int64_t n, int full, int C, int maxk,
                     int trans, double hcoef, const double* __restrict__ coef, int cstride,
                     const double* prev, double* out, double* __restrict__ sq,
                     const BlockState* __restrict__ st) {
  if (st && all_done(st)) return;
  __shared__ double red[kThreads / kBlk][kBlk];
  const int c = threadIdx.x % kBlk;
  const int rsub = threadIdx.x / kBlk;
  double cf = hcoef;
  if (coef) cf *= coef[c * cstride];
  const bool act = !st || !st->col[c].done;
  double ss = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * (kThreads / kBlk) + rsub; i < n;
       i += (int64_t)gridDim.x * (kThreads / kBlk)) {
    const int64_t I = i / kTile;
    const int r = (int)(i % kTile);
    const int64_t nk = trans ? (col_end(I, nt, full) + C - 1) / C : (nt - row_first(I, full) + C - 1) / C;
    double s = 0.0;
    // the partials in chunk order; the loads of eight at a time are in flight together
    const double* pp = part + ((I * maxk) * kTile + r) * kBlk + c;
    int64_t kq = 0;
    for (; kq + 8 <= nk; kq += 8) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = pp[(kq + q) * kTile * kBlk];
#pragma unroll
      for (int q = 0; q < 8; ++q) s += v[q];
    }
    for (; kq < nk; ++kq) s += pp[kq * kTile * kBlk];
    if (prev && cf != 0.0) s -= cf * prev[i * kBlk + c];
    if (act) out[i * kBlk + c] = s;
    ss += s * s;
  }
  if (sq) {
    red[rsub][c] = ss;
    __syncthreads();
    if (rsub == 0) {
      double t = 0.0;
      for (int q = 0; q < kThreads / kBlk; ++q) t += red[q][c];
      sq[blockIdx.x * kBlk + c] = t;
    }
  }
}

// Entries [*b, *e) of row r in split z of nsplit: the columns in the z-th of
// nsplit ranges cut at equal-count points of the group's first row r0 (binary
// searches; malformed rows give some range, never one outside the row).
__device__ __forceinline__ void spmm_split_range(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                 int64_t r0, int64_t r, int nsplit, int z, int64_t* b_out,
                                                 int64_t* e_out) {
  const int64_t b = rp[r], e = rp[r + 1];
  const int64_t f0 = rp[r0], len0 = rp[r0 + 1] - rp[r0];
  const int32_t lo = z == 0 ? INT32_MIN : (len0 > 0 ? col[f0 + (int64_t)z * len0 / nsplit] : INT32_MAX);
  const int32_t hi = z == nsplit - 1 ? INT32_MAX : (len0 > 0 ? col[f0 + (int64_t)(z + 1) * len0 / nsplit] : INT32_MAX);
  int64_t a = b, c2 = e;
  while (a < c2) {
    const int64_t mid = (a + c2) / 2;
    if (col[mid] < lo) a = mid + 1;
    else c2 = mid;
  }
  int64_t a2 = a, c3 = e;
  if (hi != INT32_MAX) {
    while (a2 < c3) {
      const int64_t mid = (a2 + c3) / 2;
      if (col[mid] < hi) a2 = mid + 1;
      else c3 = mid;
    }
  } else {
    a2 = e;
  }
  *b_out = a;
  *e_out = a2;
}

// CSR SpMM on the matrix cores:
//   out[row][c] = sA (M Xin)[row][c] - coef_c prev[row][c],  c < 32,
// plus per-column partial sums of squares of out.  Rows go in groups of
// kSpmmGroup (64), wavefront w of a workgroup rows 16 w .. 16 w + 15; a group's
// (ascending) column indices are walked in windows of W input rows, each
// starting at a multiple of 4: the window's 32-wide input rows are staged in
// LDS, the group's entries that fall in it are scattered into a dense 64 x W
// tile (zeros elsewhere), and each wavefront multiplies its 16 x W slab by the
// W x 32 window (v_mfma_f64_16x16x4f64, two 16 x 16 output tiles).  Rows of one
// RFM box share their column runs, so the tile is nearly dense and every staged
// input row serves 64 rows through the matrix cores.  Column j always falls in
// the K step of its aligned quad j / 4, so every output is the same ordered sum
// of quads whatever W is: the window width changes no result.
//
// The walk depends only on the matrix, so k_spmm_walk runs it once per solve
// and records descriptors: per work item its windows, per window its start
// column, per window and row the row's first entry in it and their number (the
// row's entries in order until the first one outside the window).  k_spmm then
// only loads and multiplies.  Malformed input (columns out of order or out of
// range) ends a prefix early and cannot make either kernel read outside Xin or
// LDS.
//
// Split groups (nsplit > 1, for matrices with few long rows): work item
// (group, z) takes only the entries whose column lies in the z-th of nsplit
// ranges cut at equal-count points of the group's first row, and writes its
// raw sums to part[z][row][32]; k_spmm_merge adds the nsplit parts in order and
// applies the scaling, the subtraction and the sums of squares.
constexpr int kSpmmGroup = 64;
constexpr int kDescCntShift = 48;  // descriptor: first entry | count << 48

// One pass of the window walk over every work item.  Count pass: wcount[item]
// = its number of windows.  Fill pass (wptr = exclusive scan of the counts):
// window k of the item (global index wptr[item] + k) gets its start in
// wstart[k] and, for each of the group's 64 rows, the descriptor in
// wdesc[k * 64 + row].
template <int W, bool Fill>
__global__ void __launch_bounds__(kThreads)
    k_spmm_walk(const int64_t* __restrict__ rp, const int32_t* __restrict__ col, int64_t rows, int nsplit,
                int32_t* __restrict__ wcount, const int64_t* __restrict__ wptr, int32_t* __restrict__ wstart,
                int64_t* __restrict__ wdesc) {
  static_assert(W % 32 == 0 && W <= 128, "window");
  constexpr int kH = (W + 63) / 64;
  __shared__ int64_t cur[kSpmmGroup], endp[kSpmmGroup];
  __shared__ int wmin[4];
  __shared__ int w0_s;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int64_t ngroups = (rows + kSpmmGroup - 1) / kSpmmGroup;
  for (int64_t wi = blockIdx.x; wi < ngroups * nsplit; wi += gridDim.x) {
    const int64_t gi = wi / nsplit;
    const int z = (int)(wi % nsplit);
    const int64_t r0 = gi * kSpmmGroup;
    if (tid < kSpmmGroup) {
      const int64_t r = r0 + tid;
      int64_t b = r < rows ? rp[r] : 0, e = r < rows ? rp[r + 1] : 0;
      if (nsplit > 1 && r < rows) spmm_split_range(rp, col, r0, r, nsplit, z, &b, &e);
      cur[tid] = b;
      endp[tid] = e;
    }
    __syncthreads();
    if (w == 0) {
      // first window: the smallest first column of the group
      int m0 = cur[lane] < endp[lane] ? col[cur[lane]] : INT32_MAX;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const int o = __shfl_xor(m0, off, 64);
        m0 = o < m0 ? o : m0;
      }
      if (lane == 0) w0_s = m0;
    }
    __syncthreads();
    int w0 = w0_s == INT32_MAX ? INT32_MAX : (w0_s & ~3);
    int64_t k = Fill ? wptr[wi] : 0;
    while (w0 != INT32_MAX) {  // uniform
      // each row's in-window prefix: its entries in order until the first one
      // outside the window; its next column is none if the row is finished,
      // its first entry left if the window took none of it, else at least
      // w0 + W (it took entries up to the first that is not in the window,
      // whose column, the columns ascending, lies beyond it)
      const int lb = (int)((int64_t)w0 + W < (int64_t)INT32_MAX ? (int64_t)w0 + W : (int64_t)INT32_MAX - 1);
      int nxt = INT32_MAX;
      for (int rr = 0; rr < 16; ++rr) {
        const int row = 16 * w + rr;
        const int64_t base = cur[row], end = endp[row];
        int fb = W, c0 = 0;
#pragma unroll
        for (int h = 0; h < kH; ++h) {
          const int j = lane + 64 * h;
          const int64_t e = base + j;
          const bool in = j < W && e < end;
          const int cj = in ? col[e] : 0;
          if (h == 0) c0 = cj;
          const int cc = cj - w0;
          const bool ok = in && cc >= 0 && cc < W;
          const unsigned long long bad = __ballot(j < W && !ok);
          if (bad) {
            const int f = 64 * h + __builtin_ctzll(bad);
            fb = f < fb ? f : fb;
          }
        }
        int rn;
        if (base + fb >= end) rn = INT32_MAX;
        else if (fb == 0) rn = __builtin_amdgcn_readlane(c0, 0);
        else rn = lb;
        nxt = rn < nxt ? rn : nxt;
        if (lane == 0) {
          if (Fill) wdesc[k * kSpmmGroup + row] = base | ((int64_t)fb << kDescCntShift);
          cur[row] = base + fb;
        }
      }
      if (lane == 0) wmin[w] = nxt;
      if (Fill && tid == 0) wstart[k] = w0;
      __syncthreads();
      int wn = wmin[0];
#pragma unroll
      for (int q = 1; q < 4; ++q) wn = wmin[q] < wn ? wmin[q] : wn;
      w0 = wn == INT32_MAX ? INT32_MAX : (wn & ~3);
      ++k;
      __syncthreads();
    }
    if (!Fill && tid == 0) wcount[wi] = (int32_t)k;
  }
}

template <int W>
__global__ void __launch_bounds__(kThreads)
    k_spmm(const int32_t* __restrict__ col, const double* __restrict__ val, int64_t rows, int64_t ncols,
           const double* __restrict__ Xin, double sA, double hcoef, const double* __restrict__ coef, int cstride,
           const double* prev, double* out, double* __restrict__ sq, const BlockState* __restrict__ st, int nsplit,
           double* __restrict__ part, const int64_t* __restrict__ wptr, const int32_t* __restrict__ wstart,
           const int64_t* __restrict__ wdesc) {
  static_assert(W % 32 == 0 && W <= 128, "window");
  if (st && all_done(st)) return;
  __shared__ double Xs[W][kBlk];
  __shared__ double At[kSpmmGroup][W + 1];
  __shared__ double red[kThreads / 16][kBlk];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  double cf[2];
  bool act[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int c = 16 * q + lr;
    cf[q] = coef ? hcoef * coef[c * cstride] : hcoef;
    act[q] = !st || !st->col[c].done;
  }
  double ss[2] = {0.0, 0.0};
  // Window data in registers: the input rows [w0, w0 + W) (coalesced, 32
  // doubles per row) and, per wavefront, each of its 16 rows' entries in the
  // window (64 lanes over consecutive entries).  The next window's are loaded
  // while the matrix cores work on the current one.
  constexpr int kXPer = W * kBlk / kThreads;
  constexpr int kH = (W + 63) / 64;
  double xr[kXPer];
  int cj[16][kH];
  double vj[16][kH];
  int w0 = 0;
  auto load = [&](int64_t k) {
    w0 = wstart[k];
#pragma unroll
    for (int q = 0; q < kXPer; ++q) {
      const int e = tid + q * kThreads;
      const int64_t r = (int64_t)w0 + e / kBlk;
      xr[q] = (r >= 0 && r < ncols) ? Xin[r * kBlk + (e % kBlk)] : 0.0;
    }
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
      const int64_t d = wdesc[k * kSpmmGroup + 16 * w + rr];
      const int64_t base = d & ((1ll << kDescCntShift) - 1);
      const int cnt = (int)(d >> kDescCntShift);
#pragma unroll
      for (int h = 0; h < kH; ++h) {
        const int j = lane + 64 * h;
        const bool in = j < cnt;
        cj[rr][h] = in ? col[base + j] : -1;
        vj[rr][h] = in ? val[base + j] : 0.0;
      }
    }
  };
  const int64_t items = ((rows + kSpmmGroup - 1) / kSpmmGroup) * nsplit;
  // the last items first: a matrix's last rows (the RFM's interface rows, two
  // boxes' columns each) have the most windows, and blocks are dispatched in order
  for (int64_t wb = blockIdx.x; wb < items; wb += gridDim.x) {
    const int64_t wi = items - 1 - wb;
    const int64_t gi = wi / nsplit;
    const int z = (int)(wi % nsplit);
    const int64_t r0 = gi * kSpmmGroup;
    const int64_t kb = wptr[wi], ke = wptr[wi + 1];
    v4d acc[2] = {v4d{0.0, 0.0, 0.0, 0.0}, v4d{0.0, 0.0, 0.0, 0.0}};
    if (kb < ke) load(kb);
    for (int64_t k = kb; k < ke; ++k) {
      // the tile starts empty (the previous window's products are done)
      for (int e = tid; e < kSpmmGroup * W; e += kThreads) At[e / W][e % W] = 0.0;
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kXPer; ++q) {
        const int e = tid + q * kThreads;
        Xs[e / kBlk][e % kBlk] = xr[q];
      }
#pragma unroll
      for (int rr = 0; rr < 16; ++rr)
#pragma unroll
        for (int h = 0; h < kH; ++h)
          if (cj[rr][h] >= 0) At[16 * w + rr][cj[rr][h] - w0] = vj[rr][h];
      __syncthreads();
      if (k + 1 < ke) load(k + 1);
      // the wavefront's 16 x W slab times the W x 32 window
#pragma unroll 4
      for (int s4 = 0; s4 < W / 4; ++s4) {
        const double a = At[16 * w + lr][4 * s4 + lk];
        const double b0 = Xs[4 * s4 + lk][lr], b1 = Xs[4 * s4 + lk][16 + lr];
        acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b0, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b1, acc[1], 0, 0, 0);
      }
      __syncthreads();
    }
    // register r of tile q: row 16 w + lk + 4 r, column 16 q + lr
    if (nsplit > 1) {
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = r0 + 16 * w + lk + 4 * r;
          if (row < rows) part[((int64_t)z * rows + row) * kBlk + 16 * q + lr] = acc[q][r];
        }
      continue;
    }
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + 16 * w + lk + 4 * r;
        const int c = 16 * q + lr;
        if (row < rows) {
          double o = sA * acc[q][r];
          if (prev && cf[q] != 0.0) o -= cf[q] * prev[row * kBlk + c];
          if (act[q]) out[row * kBlk + c] = o;
          ss[q] += o * o;
        }
      }
  }
  if (sq) {
    // per column: the 16 lane groups (4 per wavefront) in order
#pragma unroll
    for (int q = 0; q < 2; ++q) red[4 * w + lk][16 * q + lr] = ss[q];
    __syncthreads();
    if (tid < kBlk) {
      double t = 0.0;
      for (int g = 0; g < kThreads / 16; ++g) t += red[g][tid];
      sq[blockIdx.x * kBlk + tid] = t;
    }
  }
}

// out[row][c] = sA sum_z part[z][row][c] (z in order) - cf prev[row][c] for the
// rows of a split SpMM; per-column sums of squares per block as k_spmm's.
__global__ void __launch_bounds__(kThreads)
    k_spmm_merge(const double* __restrict__ part, int nsplit, int64_t rows, double sA, double hcoef,
                 const double* __restrict__ coef, int cstride, const double* prev, double* out,
                 double* __restrict__ sq, const BlockState* __restrict__ st) {
  if (st && all_done(st)) return;
  __shared__ double red[kThreads / kBlk][kBlk];
  const int c = threadIdx.x % kBlk, rsub = threadIdx.x / kBlk;
  double cf = hcoef;
  if (coef) cf *= coef[c * cstride];
  const bool act = !st || !st->col[c].done;
  double ss = 0.0;
  for (int64_t row = (int64_t)blockIdx.x * (kThreads / kBlk) + rsub; row < rows;
       row += (int64_t)gridDim.x * (kThreads / kBlk)) {
    double a = 0.0;
    for (int z = 0; z < nsplit; ++z) a += part[((int64_t)z * rows + row) * kBlk + c];
    double o = sA * a;
    if (prev && cf != 0.0) o -= cf * prev[row * kBlk + c];
    if (act) out[row * kBlk + c] = o;
    ss += o * o;
  }
  if (sq) {
    red[rsub][c] = ss;
    __syncthreads();
    if (threadIdx.x < kBlk) {
      double t = 0.0;
      for (int q = 0; q < kThreads / kBlk; ++q) t += red[q][threadIdx.x];
      sq[blockIdx.x * kBlk + threadIdx.x] = t;
    }
  }
}

// Per-column norms from partial sums: nrm_c = sqrt(sum_b sq[b][c]) -> state field
// (field = 0: beta, 1: alpha).  Columns already stopped keep their state.
__global__ void __launch_bounds__(kRedThreads) k_blk_norms(const double* __restrict__ sq, int nsq,
                                                        BlockState* st, int field, int force) {
  if (!force && all_done(st)) return;
  __shared__ double red[kRedThreads / kBlk][kBlk];
  const int c = threadIdx.x % kBlk, rsub = threadIdx.x / kBlk;
  double t = 0.0;
  for (int b = rsub; b < nsq; b += kRedThreads / kBlk) t += sq[b * kBlk + c];
  red[rsub][c] = t;
  __syncthreads();
  if (rsub == 0) {
    double s = 0.0;
    for (int q = 0; q < kRedThreads / kBlk; ++q) s += red[q][c];
    LsqrDev& d = st->col[c];
    if (force || !d.done) {
      if (field == 0) d.beta = sqrt(s);
      else d.alpha = sqrt(s);
    }
  }
}

// vec[i][c] *= 1 / state_c (beta or alpha) for active columns
__global__ void k_blk_scale(double* vec, int64_t len, const BlockState* __restrict__ st, int field,
                            int force) {
  if (!force && all_done(st)) return;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len * kBlk;
       e += (int64_t)gridDim.x * blockDim.x) {
    const LsqrDev& d = st->col[e % kBlk];
    if (!force && d.done) continue;
    const double nv = field == 0 ? d.beta : d.alpha;
    vec[e] = nv > 0.0 ? vec[e] / nv : 0.0;
  }
}

// out = x (copy) for active columns
__global__ void k_blk_copy(const double* x, double* out, int64_t len) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len * kBlk;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = x[e];
}

__global__ void k_blk_fill(double* p, int64_t len, double v) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = v;
}

// per-column sums of squares of a len x 32 block
__global__ void __launch_bounds__(kThreads) k_blk_sumsq(const double* __restrict__ x, int64_t len,
                                                        double* __restrict__ sq) {
  __shared__ double red[kThreads / kBlk][kBlk];
  const int c = threadIdx.x % kBlk, rsub = threadIdx.x / kBlk;
  double t = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * (kThreads / kBlk) + rsub; i < len;
       i += (int64_t)gridDim.x * (kThreads / kBlk))
    t += x[i * kBlk + c] * x[i * kBlk + c];
  red[rsub][c] = t;
  __syncthreads();
  if (rsub == 0) {
    double s = 0.0;
    for (int q = 0; q < kThreads / kBlk; ++q) s += red[q][c];
    sq[blockIdx.x * kBlk + c] = s;
  }
}

__device__ void all_done_update(BlockState* st) {
  int all = 1;
  for (int c = 0; c < kBlk; ++c) all &= st->col[c].done != 0;
  st->all_done = all;
}

__global__ void k_blk_start(BlockState* st, double atol, double btol, double conlim, int64_t itmax) {
  const int c = threadIdx.x;
  if (c < kBlk) {
    LsqrDev& d = st->col[c];
    const double beta = d.beta;
    d = LsqrDev{};
    d.beta = beta;
    d.atol = atol;
    d.btol = btol;
    d.conlim = conlim;
    d.itmax = itmax;
    d.bnorm = beta;
    d.phibar = beta;
    d.istop = 7;
    if (!isfinite(beta)) {  // a non-finite right-hand side: breakdown, not "x = 0 is exact"
      d.istop = -3;
      d.done = 1;
    } else if (!(beta > 0.0)) {
      d.istop = 0;
      d.done = 1;
    }
  }
  __syncthreads();
  if (c == 0) all_done_update(st);
}

__global__ void k_blk_start2(BlockState* st) {
  const int c = threadIdx.x;
  if (c < kBlk) {
    LsqrDev& d = st->col[c];
    if (!d.done) {
      d.rhobar = d.alpha;
      d.alpha_prev = d.alpha;
      d.normr = d.beta;
      d.normar = d.alpha * d.beta;
      if (!isfinite(d.alpha)) {
        d.istop = -3;
        d.done = 1;
      } else if (!(d.alpha > 0.0)) {
        d.istop = 0;
        d.done = 1;
      }
    }
  }
  __syncthreads();
  if (c == 0) all_done_update(st);
}

// plane rotation per active column (same arithmetic as the single-column kernel)
__global__ void __launch_bounds__(kRedThreads) k_blk_rotate(BlockState* st, const double* __restrict__ wsq,
                                                         int nsq) {
  if (all_done(st)) return;
  __shared__ double red[kRedThreads / kBlk][kBlk];
  const int c = threadIdx.x % kBlk, rsub = threadIdx.x / kBlk;
  double t = 0.0;
  for (int b = rsub; b < nsq; b += kRedThreads / kBlk) t += wsq[b * kBlk + c];
  red[rsub][c] = t;
  __syncthreads();
  if (rsub != 0) return;
  double w2 = 0.0;
  for (int q = 0; q < kRedThreads / kBlk; ++q) w2 += red[q][c];
  LsqrDev& d = st->col[c];
  if (d.done) {
    d.phi_rho = 0.0;
    d.theta_rho = 0.0;
    return;
  }
  const double alpha = d.alpha, beta = d.beta;
  d.itn += 1;
  d.anorm2 += d.alpha_prev * d.alpha_prev + beta * beta;
  const double rho = hypot(d.rhobar, beta);
  if (!(rho > 0.0) || !isfinite(rho)) {
    d.istop = isfinite(rho) ? 1 : -3;
    d.done = 1;
    d.phi_rho = 0.0;
    d.theta_rho = 0.0;
    return;
  }
  const double cs = d.rhobar / rho;
  const double sn = beta / rho;
  const double theta = sn * alpha;
  d.rhobar = -cs * alpha;
  const double phi = cs * d.phibar;
  d.phibar = sn * d.phibar;
  d.phi_rho = phi / rho;
  d.theta_rho = theta / rho;
  d.ddnorm += w2 / (rho * rho);
  const double anorm = sqrt(d.anorm2);
  d.acond = anorm * sqrt(d.ddnorm);
  d.normr = d.phibar;
  d.normar = d.phibar * alpha * fabs(cs);
  d.pending = 0;
  if (d.normr == 0.0 || d.normar <= d.atol * anorm * d.normr) d.pending = 2;
  else if (d.conlim > 0.0 && d.acond >= d.conlim) d.pending = 3;
  d.alpha_prev = alpha;
}

__global__ void __launch_bounds__(kThreads)
    k_blk_update(const BlockState* __restrict__ st, const double* __restrict__ v, double* w, double* y,
                 int64_t n, double* __restrict__ ysq, double* __restrict__ wsq) {
  if (all_done(st)) return;
  __shared__ double ry[kThreads / kBlk][kBlk], rw[kThreads / kBlk][kBlk];
  const int c = threadIdx.x % kBlk, rsub = threadIdx.x / kBlk;
  const LsqrDev& d = st->col[c];
  const bool act = !d.done;
  const double a = d.phi_rho, b = d.theta_rho;
  double sy = 0.0, sw = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * (kThreads / kBlk) + rsub; i < n;
       i += (int64_t)gridDim.x * (kThreads / kBlk)) {
    const int64_t e = i * kBlk + c;
    double yi = y[e], wn = w[e];
    if (act) {
      const double wi = w[e];
      yi = yi + a * wi;
      wn = v[e] - b * wi;
      y[e] = yi;
      w[e] = wn;
    }
    sy += yi * yi;
    sw += wn * wn;
  }
  ry[rsub][c] = sy;
  rw[rsub][c] = sw;
  __syncthreads();
  if (rsub == 0) {
    double ty = 0.0, tw = 0.0;
    for (int q = 0; q < kThreads / kBlk; ++q) {
      ty += ry[q][c];
      tw += rw[q][c];
    }
    ysq[blockIdx.x * kBlk + c] = ty;
    wsq[blockIdx.x * kBlk + c] = tw;
  }
}

// consistent != 0: the system has an exact solution (backward pass), S1 is ||r|| <= btol ||b||
__global__ void __launch_bounds__(kRedThreads) k_blk_check(BlockState* st, const double* __restrict__ ysq,
                                                        int nsq, int consistent) {
  if (all_done(st)) return;
  __shared__ double red[kRedThreads / kBlk][kBlk];
  const int c = threadIdx.x % kBlk, rsub = threadIdx.x / kBlk;
  double t = 0.0;
  for (int b = rsub; b < nsq; b += kRedThreads / kBlk) t += ysq[b * kBlk + c];
  red[rsub][c] = t;
  __syncthreads();
  if (rsub == 0) {
    double y2 = 0.0;
    for (int q = 0; q < kRedThreads / kBlk; ++q) y2 += red[q][c];
    LsqrDev& d = st->col[c];
    if (!d.done) {
      d.ynorm = sqrt(y2);
      const double anorm = sqrt(d.anorm2);
      int istop = 0;
      const double rtol = consistent ? d.btol * d.bnorm : d.btol * d.bnorm + d.atol * anorm * d.ynorm;
      if (d.normr <= rtol) istop = 1;
      else if (d.pending) istop = d.pending;
      else if (d.itn >= d.itmax) istop = 7;
      if (istop) {
        d.istop = istop;
        d.done = 1;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) all_done_update(st);
}

// column-major (ld) <-> interleaved block conversions
__global__ void k_gather_block(const double* __restrict__ B, int64_t ldb, int64_t k0, int64_t nb,
                               int64_t len, double* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len * kBlk;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / kBlk, c = e % kBlk;
    out[e] = c < nb ? B[(k0 + c) * ldb + i] : 0.0;
  }
}
__global__ void k_scatter_block(const double* __restrict__ in, int64_t len, int64_t k0, int64_t nb,
                                double* __restrict__ X, int64_t ldx) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len * kBlk;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / kBlk, c = e % kBlk;
    if (c < nb) X[(k0 + c) * ldx + i] = in[e];
  }
}
__global__ void k_blk_axpy(double* x, const double* __restrict__ dx, int64_t len) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len * kBlk;
       e += (int64_t)gridDim.x * blockDim.x)
    x[e] += dx[e];
}

// out[i][c] = (x[i][c] - hb beta_c prev[i][c]) / alpha_c for active columns (0 where alpha_c <= 0);
// force: every column (set-up, before the stop flags mean anything)
__global__ void k_blk_recip_scale(const double* x, double hb, const double* prev, double* out,
                                  int64_t len, const BlockState* __restrict__ st, int force) {
  if (!force && all_done(st)) return;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len * kBlk;
       e += (int64_t)gridDim.x * blockDim.x) {
    const LsqrDev& d = st->col[e % kBlk];
    if (!force && d.done) continue;
    double o = x[e];
    if (prev && hb != 0.0) o -= hb * d.beta * prev[e];
    out[e] = d.alpha > 0.0 ? o / d.alpha : 0.0;
  }
}

// dA[e] (+)= sum_c (r[i][c] w[j][c] - lam[i][c] x[j][c]) on the pattern of A; one wavefront
// per row, lanes over the row's entries; the 32 columns of each block row are contiguous.
__global__ void __launch_bounds__(kThreads)
    k_blk_pattern_grad(const int64_t* __restrict__ rp, const int32_t* __restrict__ col, int64_t m,
                       const double* __restrict__ r, const double* __restrict__ w,
                       const double* __restrict__ lam, const double* __restrict__ x,
                       double* __restrict__ dA, int accumulate) {
  const int lane = threadIdx.x & 63;
  const int64_t wid = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  const int64_t nw = (int64_t)gridDim.x * (kThreads / 64);
  for (int64_t row = wid; row < m; row += nw) {
    const double* ri = r + row * kBlk;
    const double* li = lam + row * kBlk;
    for (int64_t e = rp[row] + lane; e < rp[row + 1]; e += 64) {
      const int64_t j = col[e];
      const double* wj = w + j * kBlk;
      const double* xj = x + j * kBlk;
      double g = 0.0;
#pragma unroll 8
      for (int c = 0; c < kBlk; ++c) g += ri[c] * wj[c] - li[c] * xj[c];
      dA[e] = accumulate ? dA[e] + g : g;
    }
  }
}

unsigned grid_for(int64_t elems) {
  const int64_t b = (elems + kThreads - 1) / kThreads;
  return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}
unsigned rows_grid(int64_t rows) {  // blocks of 8 rows x 32 columns, grid-stride beyond kRowBlocks
  const int64_t b = (rows + (kThreads / kBlk) - 1) / (kThreads / kBlk);
  return (unsigned)(b < kRowBlocks ? (b > 0 ? b : 1) : kRowBlocks);
}
unsigned spmm_grid(int64_t rows) {  // 16-row groups, grid-stride beyond kSpmmBlocks
  const int64_t b = (rows + 15) / 16;
  return (unsigned)(b < kSpmmBlocks ? (b > 0 ? b : 1) : kSpmmBlocks);
}

// SpMM launch shapes: 64-row groups; the window width (columns of the input
// block staged in LDS at a time) is chosen per matrix by the autotuner below.
// It changes neither the order of any sum nor the rows each block handles (so
// not the norm partials either), so every candidate gives bitwise the same
// result.  Grids stop at kSpmmGrid blocks (grid-stride over the groups beyond):
// up to 2048 groups one block each.
constexpr unsigned kSpmmGrid = kSpmmMaxBlocks;
struct SpmmShape {
  const void* fn;
  int group, win;
  unsigned max_blocks;  // grid cap (grid-stride over the groups beyond it)
};
// the hand-picked shape (used when tuning is off, and the tuner's reference)
SpmmShape spmm_shape(const rfmls_csr*) { return {(const void*)k_spmm<64>, kSpmmGroup, 64, kSpmmGrid}; }
static std::vector<SpmmShape> spmm_candidates(const rfmls_csr* M, int /*num_cus*/) {
  std::vector<SpmmShape> c;
  c.push_back(spmm_shape(M));
  c.push_back({(const void*)k_spmm<32>, kSpmmGroup, 32, kSpmmGrid});
  c.push_back({(const void*)k_spmm<128>, kSpmmGroup, 128, kSpmmGrid});
  return c;
}
// Split row groups of a matrix with fewer than 4 groups per compute unit and
// long rows (at least 4 windows of 64 per split) so that the grid covers the
// chip: nsplit = ceil(4 CUs / groups), at most 8.
int spmm_split(const rfmls_csr* M, int num_cus) {
  const int64_t ng = (M->m + kSpmmGroup - 1) / kSpmmGroup;
  const int64_t target = 4 * (int64_t)num_cus;
  if (ng <= 0 || ng >= target || M->nnz / M->m < 8 * 64) return 1;
  const int64_t sp = (target + ng - 1) / ng;
  const int64_t win = M->nnz / M->m / 64;  // windows of 64 columns of a row
  int64_t k = sp < 8 ? sp : 8;
  while (k > 1 && win / k < 4) --k;
  return (int)k;
}
// Window descriptors of one matrix for the window width W (built by
// spmm_build_desc, see k_spmm_walk).
struct SpmmDesc {
  int W = 0;  // 0: not built
  int nsplit = 1;
  int64_t items = 0, nwin = 0;
  int64_t* wptr = nullptr;    // items + 1 window offsets
  int32_t* wstart = nullptr;  // nwin window starts
  int64_t* wdesc = nullptr;   // nwin x 64 row descriptors
};
struct BCtx {
  rfmls_handle* h;
  const rfmls_csr* A;
  const rfmls_csr* AT;
  const rfmls_precond_t* P;
  hipStream_t st;
  double *U, *V, *W, *Y, *Z, *Q, *T, *Rr, *Xb, *Bb, *DX, *Sm, *Sn;
  double *sqA, *sqB, *sqY, *sqW, *part;
  double* spart;  // partial sums of split SpMM groups (nsplit x rows x 32)
  SpmmDesc dA, dAT;  // SpMM window descriptors of A and A^T (k_spmm_walk)
  BlockState* dst;
  IterGraph* graph = nullptr;  // captured poll interval of the loop, or null: eager launches
};

// Runs the lockstep loop: `iteration` (which enqueues one iteration on c.st) up
// to itmax times, the host polling the "all columns done" word after every
// `every` iterations; with c.graph the poll interval is captured once and replayed.
template <class F>
static rfmls_status run_loop(BCtx& c, int64_t itmax, int every, F&& iteration);

double* state_field(BlockState* s, int which) {
  // pointer to col[0].<field>; stride between columns in doubles
  LsqrDev* d = &s->col[0];
  return which == 0 ? &d->beta : &d->alpha;
}
constexpr int kStride = (int)(sizeof(LsqrDev) / sizeof(double));
static_assert(sizeof(LsqrDev) % sizeof(double) == 0, "LsqrDev must be a whole number of doubles");

rfmls_status tri_block(BCtx& c, int trans, const double* in, double* out, double hcoef,
                       const double* coef, const double* prev, double* sq, const BlockState* stp) {
  const rfmls_precond_t* P = c.P;
  const int64_t n = P->n, nt = P->nt;
  const int C = P->chunk;
  const int maxk = (int)((nt + C - 1) / C);
  const double esz = P->store == RFMLS_F64 ? 8.0 : 4.0;
  const int full = P->full;
  const double tri = full ? (double)n * (double)n : (double)n * (double)(n + 1) / 2.0;
  {
    Trace tr(c.h, full ? (trans ? "gemm_Pt" : "gemm_P") : (trans ? "trmm_Xt" : "trmm_X"),
             esz * tri + 2.0 * 8.0 * kBlk * (double)n, 2.0 * tri * kBlk);
    if (!trans) {
      if (P->store == RFMLS_F64)
        hipLaunchKernelGGL(k_trmm_part<double>, dim3((unsigned)P->ntab), dim3(kThreads), 0, c.st,
                           (const double*)P->Xpk, nt, n, full, P->tab_row, C, maxk, in, c.part, stp);
      else
        hipLaunchKernelGGL(k_trmm_part<float>, dim3((unsigned)P->ntab), dim3(kThreads), 0, c.st,
                           (const float*)P->Xpk, nt, n, full, P->tab_row, C, maxk, in, c.part, stp);
    } else {
      if (P->store == RFMLS_F64)
        hipLaunchKernelGGL(k_trmmT_part<double>, dim3((unsigned)P->ntab), dim3(kThreads), 0, c.st,
                           (const double*)P->Xpk, nt, n, full, P->tab_col, C, maxk, in, c.part, stp);
      else
        hipLaunchKernelGGL(k_trmmT_part<float>, dim3((unsigned)P->ntab), dim3(kThreads), 0, c.st,
                           (const float*)P->Xpk, nt, n, full, P->tab_col, C, maxk, in, c.part, stp);
    }
  }
  hipLaunchKernelGGL(k_blk_tri_reduce, dim3(rows_grid(n)), dim3(kThreads), 0, c.st, (const double*)c.part,
                     nt, n, full, C, maxk, trans, hcoef, coef, kStride, prev, out, sq, stp);
  RFMLS_HIP(c.h, hipGetLastError());
  return RFMLS_OK;
}

// The tuned launch shape of products with M on this handle, if a matrix of M's
// shape (rows, columns, stored entries) has been tuned: a rebuilt transpose
// (same matrix at a new address) is not tuned again.
static bool spmm_lookup(rfmls_handle* h, const rfmls_csr* M, SpmmShape* out) {
  if (!h->tune) return false;
  for (const TuneRec& t : h->tuned)
    if (t.rows == M->m && t.cols == M->n && t.nnz == M->nnz && !strcmp(t.kernel, "spmm")) {
      const std::vector<SpmmShape> cands = spmm_candidates(M, h->num_cus);
      if (t.choice >= 0 && t.choice < (int)cands.size()) {
        *out = cands[t.choice];
        return true;
      }
    }
  return false;
}

// Window descriptors of M (A or A^T of the context) for width W: a count pass
// of the window walk, the scan of the counts, one host read of the total,
// and the fill pass.  Synchronises the stream; refused while a graph is
// being captured (the solve loops prepare them before capturing).
template <int W>
static void spmm_walk_launch(BCtx& c, const rfmls_csr* M, int nsplit, unsigned grid, int32_t* cnt, int64_t* wptr,
                             int32_t* wstart, int64_t* wdesc, bool fill) {
  if (fill)
    hipLaunchKernelGGL((k_spmm_walk<W, true>), dim3(grid), dim3(kThreads), 0, c.st, M->row_ptr, M->col, M->m, nsplit,
                       cnt, (const int64_t*)wptr, wstart, wdesc);
  else
    hipLaunchKernelGGL((k_spmm_walk<W, false>), dim3(grid), dim3(kThreads), 0, c.st, M->row_ptr, M->col, M->m, nsplit,
                       cnt, (const int64_t*)wptr, wstart, wdesc);
}
static rfmls_status spmm_build_desc(BCtx& c, const rfmls_csr* M, int W, SpmmDesc* d) {
  rfmls_handle* h = c.h;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(c.st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    return fail(h, RFMLS_E_HIP, "SpMM: window descriptors requested while capturing a graph");
  const bool isA = M == c.A;
  const int nsplit = spmm_split(M, h->num_cus);
  const int64_t items = ((M->m + kSpmmGroup - 1) / kSpmmGroup) * nsplit;
  const unsigned grid = (unsigned)(items < 4096 ? (items > 0 ? items : 1) : 4096);
  void* p1;
  RFMLS_CHECK(workspace(h, isA ? WS_SPMM_WPTR_A : WS_SPMM_WPTR_AT,
                        sizeof(int64_t) * (size_t)(items + 1) + sizeof(int32_t) * (size_t)(items + 1), &p1));
  int64_t* wptr = (int64_t*)p1;
  int32_t* cnt = (int32_t*)(wptr + items + 1);
  auto walk = [&](bool fill, int32_t* ws, int64_t* wd) {
    if (W == 32) spmm_walk_launch<32>(c, M, nsplit, grid, cnt, wptr, ws, wd, fill);
    else if (W == 128) spmm_walk_launch<128>(c, M, nsplit, grid, cnt, wptr, ws, wd, fill);
    else spmm_walk_launch<64>(c, M, nsplit, grid, cnt, wptr, ws, wd, fill);
  };
  walk(false, nullptr, nullptr);
  RFMLS_CHECK(scan_counts(h, cnt, items, wptr));
  int64_t nwin = 0;
  RFMLS_HIP(h, hipMemcpyAsync(&nwin, wptr + items, sizeof(int64_t), hipMemcpyDeviceToHost, c.st));
  RFMLS_HIP(h, hipStreamSynchronize(c.st));
  void* p2;
  RFMLS_CHECK(workspace(h, isA ? WS_SPMM_WDESC_A : WS_SPMM_WDESC_AT,
                        sizeof(int64_t) * (size_t)(nwin > 0 ? nwin : 1) * kSpmmGroup +
                            sizeof(int32_t) * (size_t)(nwin > 0 ? nwin : 1) + 64,
                        &p2));
  int64_t* wdesc = (int64_t*)p2;
  int32_t* wstart = (int32_t*)(wdesc + (nwin > 0 ? nwin : 1) * kSpmmGroup);
  walk(true, wstart, wdesc);
  RFMLS_HIP(h, hipGetLastError());
  d->W = W;
  d->nsplit = nsplit;
  d->items = items;
  d->nwin = nwin;
  d->wptr = wptr;
  d->wstart = wstart;
  d->wdesc = wdesc;
  if (c.AT == c.A) c.dAT = c.dA = *d;
  return RFMLS_OK;
}

static rfmls_status spmm_launch(BCtx& c, const rfmls_csr* M, const SpmmShape& sh, const double* x, double sA,
                                double hcoef, const double* coef, const double* prev, double* out, double* sq,
                                const BlockState* stp, int* nblk);

// Autotuner of the SpMM launch shape (window width) for M: the first time a
// matrix of M's shape is used on this handle (with tuning on), every candidate of
// spmm_candidates runs on M with a zero input block of 32 columns into
// scratch (xin: M->n x 32, out: M->m x 32, sq: the partials), once to warm up
// and then three times between HIP events; the candidate with the smallest
// median is kept for M on this handle.  Synchronises the stream; never called
// while a graph is being captured.
static rfmls_status spmm_tune(BCtx& c, const rfmls_csr* M, double* xin, double* out, double* sq) {
  rfmls_handle* h = c.h;
  SpmmShape dummy;
  if (!h->tune || M->m < 1 || spmm_lookup(h, M, &dummy)) return RFMLS_OK;
  const std::vector<SpmmShape> cands = spmm_candidates(M, h->num_cus);
  hipLaunchKernelGGL(k_blk_fill, dim3(grid_for(M->n * kBlk)), dim3(kThreads), 0, c.st, xin, M->n * kBlk, 0.0);
  hipEvent_t ev[4];
  for (auto& e : ev) RFMLS_HIP(h, hipEventCreate(&e));
  std::vector<double> med(cands.size(), 0.0);
  rfmls_status st = RFMLS_OK;
  const bool trace = h->trace;
  h->trace = false;  // the trial launches are not part of any traced step
  for (size_t k = 0; k < cands.size() && st >= 0; ++k) {
    float t[3];
    st = spmm_launch(c, M, cands[k], xin, 1.0, 0.0, nullptr, nullptr, out, sq, nullptr, nullptr);
    for (int r = 0; r < 3 && st >= 0; ++r) {
      hipEventRecord(ev[0], c.st);
      st = spmm_launch(c, M, cands[k], xin, 1.0, 0.0, nullptr, nullptr, out, sq, nullptr, nullptr);
      hipEventRecord(ev[1], c.st);
      if (hipEventSynchronize(ev[1]) != hipSuccess || hipEventElapsedTime(&t[r], ev[0], ev[1]) != hipSuccess)
        st = fail(h, RFMLS_E_HIP, "SpMM autotuner: event timing failed");
    }
    if (st >= 0) {
      std::sort(t, t + 3);
      med[k] = t[1];
    }
  }
  h->trace = trace;
  for (auto& e : ev) hipEventDestroy(e);
  if (st < 0) return st;
  size_t best = 0;
  for (size_t k = 1; k < cands.size(); ++k)
    if (med[k] < med[best]) best = k;
  TuneRec rec{};
  snprintf(rec.kernel, sizeof(rec.kernel), "spmm");
  rec.rows = M->m;
  rec.cols = M->n;
  rec.nnz = M->nnz;
  rec.choice = (int)best;
  snprintf(rec.desc, sizeof(rec.desc), "group %d window %d grid %u", cands[best].group, cands[best].win,
           cands[best].max_blocks);
  rec.ms_best = med[best];
  rec.ms_default = med[0];
  rec.candidates = (int)cands.size();
  h->tuned.push_back(rec);
  return RFMLS_OK;
}

// Tunes the products with A and A^T and builds the window descriptors of the
// shapes the loop will use (before any capture of the loop).
static rfmls_status spmm_tune_both(BCtx& c) {
  RFMLS_CHECK(spmm_tune(c, c.A, c.Z, c.T, c.sqA));
  if (c.AT != c.A) RFMLS_CHECK(spmm_tune(c, c.AT, c.T, c.Sn, c.sqA));
  for (const rfmls_csr* M : {c.A, c.AT}) {
    SpmmShape sh;
    if (!spmm_lookup(c.h, M, &sh)) sh = spmm_shape(M);
    SpmmDesc* d = M == c.A ? &c.dA : &c.dAT;
    if (d->W != sh.win) RFMLS_CHECK(spmm_build_desc(c, M, sh.win, d));
  }
  return RFMLS_OK;
}

rfmls_status spmm(BCtx& c, const rfmls_csr* M, const double* x, double sA, double hcoef,
                  const double* coef, const double* prev, double* out, double* sq,
                  const BlockState* stp, int* nblk) {
  SpmmShape sh;
  if (!spmm_lookup(c.h, M, &sh)) sh = spmm_shape(M);
  return spmm_launch(c, M, sh, x, sA, hcoef, coef, prev, out, sq, stp, nblk);
}

static rfmls_status spmm_launch(BCtx& c, const rfmls_csr* M, const SpmmShape& sh, const double* x, double sA,
                                double hcoef, const double* coef, const double* prev, double* out, double* sq,
                                const BlockState* stp, int* nblk) {
  const int64_t ng = (M->m + sh.group - 1) / sh.group;
  const int nsplit = spmm_split(M, c.h->num_cus);
  const int64_t work = ng * nsplit;
  const unsigned nb = (unsigned)(work < (int64_t)sh.max_blocks ? (work > 0 ? work : 1) : sh.max_blocks);
  Trace tr(c.h, M == c.A ? "spmm_A" : "spmm_At",
           12.0 * (double)M->nnz + 8.0 * (double)(M->m + 1) +
               8.0 * kBlk * ((double)M->n + (double)M->m * (prev ? 2.0 : 1.0)),
           2.0 * kBlk * (double)M->nnz);
  int kStride_v = kStride;
  double* spart = c.spart;
  SpmmDesc* dsc = M == c.A ? &c.dA : &c.dAT;
  if (dsc->W != sh.win) RFMLS_CHECK(spmm_build_desc(c, M, sh.win, dsc));
  const int64_t* wptr = dsc->wptr;
  const int32_t* wstart = dsc->wstart;
  const int64_t* wdesc = dsc->wdesc;
  void* args[] = {(void*)&M->col, (void*)&M->val, (void*)&M->m, (void*)&M->n,
                  (void*)&x, (void*)&sA, (void*)&hcoef, (void*)&coef, (void*)&kStride_v, (void*)&prev,
                  (void*)&out, (void*)&sq, (void*)&stp, (void*)&nsplit, (void*)&spart, (void*)&wptr,
                  (void*)&wstart, (void*)&wdesc};
  RFMLS_HIP(c.h, hipLaunchKernel(sh.fn, dim3(nb), dim3(kThreads), args, 0, c.st));
  if (nsplit > 1) {
    const unsigned gm = rows_grid(M->m);
    hipLaunchKernelGGL(k_spmm_merge, dim3(gm), dim3(kThreads), 0, c.st, (const double*)spart, nsplit, M->m,
                       sA, hcoef, coef, kStride, prev, out, sq, stp);
    if (nblk) *nblk = (int)gm;
  } else if (nblk) {
    *nblk = (int)nb;
  }
  RFMLS_HIP(c.h, hipGetLastError());
  return RFMLS_OK;
}

rfmls_status poll_all(BCtx& c, int* done) {
  int* pin = (int*)((char*)c.h->pinned + 1024);
  RFMLS_HIP(c.h, hipMemcpyAsync(pin, &c.dst->all_done, sizeof(int), hipMemcpyDeviceToHost, c.st));
  RFMLS_HIP(c.h, hipStreamSynchronize(c.st));
  *done = *pin;
  return RFMLS_OK;
}

// One lockstep sweep for min ||A X y - rhs|| over the 32 columns of rhs (m x 32).
rfmls_status block_sweep(BCtx& c, const double* rhs, const rfmls_opts* o, int64_t itmax) {
  const int64_t m = c.A->m, n = c.A->n;
  const unsigned gm = grid_for(m * kBlk), gn = grid_for(n * kBlk);
  // beta_1 u_1 = rhs
  hipLaunchKernelGGL(k_blk_copy, dim3(gm), dim3(kThreads), 0, c.st, rhs, c.U, m);
  hipLaunchKernelGGL(k_blk_sumsq, dim3(rows_grid(m)), dim3(kThreads), 0, c.st, (const double*)c.U, m,
                     c.sqA);
  hipLaunchKernelGGL(k_blk_norms, dim3(1), dim3(kRedThreads), 0, c.st, (const double*)c.sqA,
                     (int)rows_grid(m), c.dst, 0, 1);
  hipLaunchKernelGGL(k_blk_start, dim3(1), dim3(64), 0, c.st, c.dst, o->atol, o->btol, o->conlim, itmax);
  hipLaunchKernelGGL(k_blk_scale, dim3(gm), dim3(kThreads), 0, c.st, c.U, m, (const BlockState*)c.dst, 0, 1);
  hipLaunchKernelGGL(k_blk_fill, dim3(gn), dim3(kThreads), 0, c.st, c.Y, n * kBlk, 0.0);
  // alpha_1 v_1 = X^T (A^T u_1)
  RFMLS_CHECK(spmm(c, c.AT, c.U, 1.0, 0.0, nullptr, nullptr, c.Q, nullptr, nullptr, nullptr));
  RFMLS_CHECK(tri_block(c, 1, c.Q, c.V, 0.0, nullptr, nullptr, c.sqB, nullptr));
  hipLaunchKernelGGL(k_blk_norms, dim3(1), dim3(kRedThreads), 0, c.st, (const double*)c.sqB,
                     (int)rows_grid(n), c.dst, 1, 0);
  hipLaunchKernelGGL(k_blk_scale, dim3(gn), dim3(kThreads), 0, c.st, c.V, n, (const BlockState*)c.dst, 1, 0);
  hipLaunchKernelGGL(k_blk_start2, dim3(1), dim3(64), 0, c.st, c.dst);
  hipLaunchKernelGGL(k_blk_copy, dim3(gn), dim3(kThreads), 0, c.st, (const double*)c.V, c.W, n);
  hipLaunchKernelGGL(k_blk_sumsq, dim3(rows_grid(n)), dim3(kThreads), 0, c.st, (const double*)c.W, n,
                     c.sqW);
  RFMLS_HIP(c.h, hipGetLastError());
  const int every = o->check_every > 0 ? o->check_every : 8;
  const BlockState* cst = c.dst;
  return run_loop(c, itmax, every, [&]() -> rfmls_status {
    RFMLS_CHECK(tri_block(c, 0, c.V, c.Z, 0.0, nullptr, nullptr, nullptr, cst));
    int nb = 0;
    RFMLS_CHECK(spmm(c, c.A, c.Z, 1.0, 1.0, state_field(c.dst, 1), c.U, c.U, c.sqA, cst, &nb));
    hipLaunchKernelGGL(k_blk_norms, dim3(1), dim3(kRedThreads), 0, c.st, (const double*)c.sqA, nb, c.dst, 0, 0);
    hipLaunchKernelGGL(k_blk_scale, dim3(gm), dim3(kThreads), 0, c.st, c.U, m, cst, 0, 0);
    RFMLS_CHECK(spmm(c, c.AT, c.U, 1.0, 0.0, nullptr, nullptr, c.Q, nullptr, cst, nullptr));
    RFMLS_CHECK(tri_block(c, 1, c.Q, c.V, 1.0, state_field(c.dst, 0), c.V, c.sqB, cst));
    hipLaunchKernelGGL(k_blk_norms, dim3(1), dim3(kRedThreads), 0, c.st, (const double*)c.sqB,
                       (int)rows_grid(n), c.dst, 1, 0);
    hipLaunchKernelGGL(k_blk_scale, dim3(gn), dim3(kThreads), 0, c.st, c.V, n, cst, 1, 0);
    hipLaunchKernelGGL(k_blk_rotate, dim3(1), dim3(kRedThreads), 0, c.st, c.dst, (const double*)c.sqW,
                       (int)rows_grid(n));
    hipLaunchKernelGGL(k_blk_update, dim3(rows_grid(n)), dim3(kThreads), 0, c.st, cst,
                       (const double*)c.V, c.W, c.Y, n, c.sqY, c.sqW);
    hipLaunchKernelGGL(k_blk_check, dim3(1), dim3(kRedThreads), 0, c.st, c.dst, (const double*)c.sqY,
                       (int)rows_grid(n), 0);
    RFMLS_HIP(c.h, hipGetLastError());
    return RFMLS_OK;
  });
}

template <class F>
static rfmls_status run_loop(BCtx& c, int64_t itmax, int every, F&& iteration) {
  rfmls_handle* h = c.h;
  int hd = 0;
  RFMLS_CHECK(poll_all(c, &hd));
  if (c.graph && !h->trace) {
    if (!c.graph->exec)
      RFMLS_CHECK(capture_graph(h, c.graph, [&]() -> rfmls_status {
        const hipStream_t s0 = c.st;
        c.st = h->stream;
        rfmls_status r = RFMLS_OK;
        for (int k = 0; k < every && r >= 0; ++k) r = iteration();
        c.st = s0;
        return r;
      }));
    for (int64_t it = 0; it < itmax && !hd; it += every) {
      RFMLS_HIP(h, hipGraphLaunch(c.graph->exec, c.st));
      RFMLS_CHECK(poll_all(c, &hd));
    }
    return RFMLS_OK;
  }
  for (int64_t it = 0; it < itmax && !hd; ++it) {
    RFMLS_CHECK(iteration());
    if ((it + 1) % every == 0) RFMLS_CHECK(poll_all(c, &hd));
  }
  return RFMLS_OK;
}

rfmls_status read_block_state(BCtx& c, BlockState* out) {
  RFMLS_HIP(c.h, hipMemcpyAsync(out, c.dst, sizeof(BlockState), hipMemcpyDeviceToHost, c.st));
  RFMLS_HIP(c.h, hipStreamSynchronize(c.st));
  return RFMLS_OK;
}

// Work blocks (5 of m x 32, 8 of n x 32), partial sums and the triangular-product
// partials, carved from one workspace slot.
static rfmls_status make_bctx(rfmls_handle* h, const rfmls_csr* A, const rfmls_csr* AT,
                              const rfmls_precond_t* P, BCtx& c) {
  const int64_t m = A->m, n = A->n;
  c.h = h;
  c.A = A;
  c.AT = AT;
  c.P = P;
  c.st = h->stream;
  const int64_t maxk = (P->nt + P->chunk - 1) / P->chunk;
  const size_t nvec = (size_t)kBlk * (size_t)(5 * m + 8 * n) + 4 * (size_t)kSpmmMaxBlocks * kBlk +
                      (size_t)P->nt * maxk * kTile * kBlk;
  void* p;
  RFMLS_CHECK(workspace(h, WS_LSQR_BLK, sizeof(double) * nvec, &p));
  double* d = (double*)p;
  auto take = [&](int64_t len) {
    double* r = d;
    d += len;
    return r;
  };
  c.U = take(m * kBlk);
  c.Rr = take(m * kBlk);
  c.Bb = take(m * kBlk);
  c.T = take(m * kBlk);
  c.Sm = take(m * kBlk);
  c.V = take(n * kBlk);
  c.W = take(n * kBlk);
  c.Y = take(n * kBlk);
  c.Z = take(n * kBlk);
  c.Q = take(n * kBlk);
  c.Xb = take(n * kBlk);
  c.DX = take(n * kBlk);
  c.Sn = take(n * kBlk);
  c.sqA = take(kSpmmMaxBlocks * kBlk);
  c.sqB = take(kSpmmMaxBlocks * kBlk);
  c.sqY = take(kSpmmMaxBlocks * kBlk);
  c.sqW = take(kSpmmMaxBlocks * kBlk);
  c.part = take(P->nt * maxk * kTile * kBlk);
  {
    const int64_t need = (int64_t)spmm_split(A, h->num_cus) * A->m > (int64_t)spmm_split(AT, h->num_cus) * AT->m
                             ? (int64_t)spmm_split(A, h->num_cus) * A->m
                             : (int64_t)spmm_split(AT, h->num_cus) * AT->m;
    void* pp;
    RFMLS_CHECK(workspace(h, WS_SPMM_PART, sizeof(double) * (size_t)need * kBlk, &pp));
    c.spart = (double*)pp;
  }
  void* ps;
  RFMLS_CHECK(workspace(h, WS_LSQR_BSTATE, sizeof(BlockState), &ps));
  c.dst = (BlockState*)ps;
  return RFMLS_OK;
}

// ---- the explicit preconditioned matrix B = A X (Alg. 1 step 4) ----
// out[j][k] = X[j][c0 + k] for k < nb (zero beyond nb, and below the diagonal
// for the triangular X = R^{-1}): a 32-column slab of X in the lockstep block
// layout, read from the packed tiles.
template <typename TS>
__global__ void k_x_slab(const TS* __restrict__ Xpk, int64_t n, int64_t nt, int full, int64_t c0, int nb,
                         double* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * kBlk;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / kBlk, c = c0 + e % kBlk;
    double v = 0.0;
    if (e % kBlk < nb && (full || j <= c))
      v = (double)Xpk[ptile(j / kTile, c / kTile, nt, full) * (int64_t)(kTile * kTile) +
                      (j % kTile) * kTile + c % kTile];
    out[e] = v;
  }
}
// B[i][c0 + k] = in[i][k] for k < nb (rows of B ldb apart)
__global__ void k_scatter_slab(const double* __restrict__ in, int64_t m, int64_t c0, int nb,
                               double* __restrict__ B, int64_t ldb) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m * kBlk;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / kBlk, k = e % kBlk;
    if (k < nb) B[i * ldb + c0 + k] = in[e];
  }
}

}  // namespace

rfmls_status run_solve_block(rfmls_handle* h, const rfmls_csr* A, const rfmls_csr* AT,
                             const rfmls_precond_t* P, const double* B, int64_t ldb, int64_t nrhs,
                             double* X, int64_t ldx, double* Rout, int64_t ldr, const rfmls_opts* o,
                             rfmls_info* info) {
  const int64_t m = A->m, n = A->n;
  const int64_t itmax = o->itmax > 0 ? o->itmax : n;
  BCtx c;
  RFMLS_CHECK(make_bctx(h, A, AT, P, c));
  RFMLS_CHECK(spmm_tune_both(c));
  IterGraph graph;  // one capture serves every sweep and column block (same buffers)
  if (o->graph) c.graph = &graph;
  const unsigned gm = grid_for(m * kBlk), gn = grid_for(n * kBlk);
  rfmls_status ret = RFMLS_OK;
  std::vector<BlockState> hs(1);
  for (int64_t k0 = 0; k0 < nrhs; k0 += kBlk) {
    const int64_t nb = nrhs - k0 < kBlk ? nrhs - k0 : kBlk;
    std::vector<rfmls_info> inf(nb);
    hipLaunchKernelGGL(k_gather_block, dim3(gm), dim3(kThreads), 0, c.st, B, ldb, k0, nb, m, c.Bb);
    // from x = 0 the first sweep takes B itself; from given starting points
    // every sweep solves for the correction from the true residual B - A X
    const bool warm = o->x_init != 0;
    std::vector<double> bsq;
    if (warm) {
      hipLaunchKernelGGL(k_gather_block, dim3(gn), dim3(kThreads), 0, c.st, (const double*)X, ldx, k0, nb,
                         n, c.Xb);
      RFMLS_CHECK(spmm(c, A, c.Xb, -1.0, -1.0, nullptr, c.Bb, c.Rr, nullptr, nullptr, nullptr));
      hipLaunchKernelGGL(k_blk_sumsq, dim3(rows_grid(m)), dim3(kThreads), 0, c.st, (const double*)c.Bb, m,
                         c.sqA);
      bsq.assign((size_t)rows_grid(m) * kBlk, 0.0);
      RFMLS_HIP(h, hipMemcpyAsync(bsq.data(), c.sqA, sizeof(double) * bsq.size(), hipMemcpyDeviceToHost,
                                  c.st));
      RFMLS_HIP(h, hipStreamSynchronize(c.st));
      for (int64_t q = 0; q < nb; ++q) {
        double t = 0.0;
        for (size_t b = 0; b < bsq.size() / kBlk; ++b) t += bsq[b * kBlk + q];
        inf[q].normb = sqrt(t);
      }
    }
    for (int sweep = 0; sweep <= o->refine; ++sweep) {
      const bool from_zero = sweep == 0 && !warm;
      RFMLS_CHECK(block_sweep(c, from_zero ? c.Bb : c.Rr, o, itmax));
      RFMLS_CHECK(read_block_state(c, hs.data()));
      int64_t itn_max = 0;
      for (int64_t q = 0; q < nb; ++q) {
        const LsqrDev& s = hs[0].col[q];
        if (s.istop < 0) return fail(h, RFMLS_E_BREAKDOWN, "non-finite value in LSQR (column %lld)", (long long)(k0 + q));
        if (sweep == 0) {
          inf[q].itn_first = s.itn;
          inf[q].istop = s.istop;
          inf[q].normr_est = s.normr;
          inf[q].normar_est = s.normar;
          inf[q].anorm_est = sqrt(s.anorm2);
          inf[q].acond_est = s.acond;
          if (!warm) inf[q].normb = s.bnorm;
          if (s.istop == 7) ret = RFMLS_W_NOCONV;
        }
        inf[q].itn += s.itn;
        inf[q].istop_last = s.istop;
        if (s.itn > itn_max) itn_max = s.itn;
      }
      // x (+)= X y ; r = b - A x
      RFMLS_CHECK(tri_block(c, 0, c.Y, from_zero ? c.Xb : c.DX, 0.0, nullptr, nullptr, nullptr, nullptr));
      if (!from_zero)
        hipLaunchKernelGGL(k_blk_axpy, dim3(gn), dim3(kThreads), 0, c.st, c.Xb, (const double*)c.DX, n);
      RFMLS_CHECK(spmm(c, A, c.Xb, -1.0, -1.0, nullptr, c.Bb, c.Rr, nullptr, nullptr, nullptr));
      if (itn_max == 0) break;
    }
    // true residual norms per column
    hipLaunchKernelGGL(k_blk_sumsq, dim3(rows_grid(m)), dim3(kThreads), 0, c.st, (const double*)c.Rr, m, c.sqA);
    RFMLS_CHECK(spmm(c, AT, c.Rr, 1.0, 0.0, nullptr, nullptr, c.Q, nullptr, nullptr, nullptr));
    hipLaunchKernelGGL(k_blk_sumsq, dim3(rows_grid(n)), dim3(kThreads), 0, c.st, (const double*)c.Q, n, c.sqB);
    std::vector<double> sa((size_t)rows_grid(m) * kBlk), sb((size_t)rows_grid(n) * kBlk);
    RFMLS_HIP(h, hipMemcpyAsync(sa.data(), c.sqA, sizeof(double) * sa.size(), hipMemcpyDeviceToHost, c.st));
    RFMLS_HIP(h, hipMemcpyAsync(sb.data(), c.sqB, sizeof(double) * sb.size(), hipMemcpyDeviceToHost, c.st));
    hipLaunchKernelGGL(k_scatter_block, dim3(gn), dim3(kThreads), 0, c.st, (const double*)c.Xb, n, k0, nb, X, ldx);
    if (Rout)
      hipLaunchKernelGGL(k_scatter_block, dim3(gm), dim3(kThreads), 0, c.st, (const double*)c.Rr, m, k0, nb, Rout, ldr);
    RFMLS_HIP(h, hipStreamSynchronize(c.st));
    for (int64_t q = 0; q < nb; ++q) {
      double ra = 0.0, rb = 0.0;
      for (size_t b = 0; b < sa.size() / kBlk; ++b) ra += sa[b * kBlk + q];
      for (size_t b = 0; b < sb.size() / kBlk; ++b) rb += sb[b * kBlk + q];
      inf[q].normr = sqrt(ra);
      inf[q].normar = sqrt(rb);
      if (info) info[k0 + q] = inf[q];
    }
  }
  return ret;
}


// Backward in lockstep blocks of 32: for each column, LSQR on the consistent
// system B^T lam = X^T g with operator M = B^T = X^T A^T (n x m), from lam = 0,
// tracking the shadow vectors vt (v = B vt) and z (lam = B z); then w = X z,
// lam = A w, dB = lam and dA += r w^T - lam x^T on A's pattern (summed over
// the right-hand sides).  Same per-column recurrences as the single-column
// backward.
rfmls_status run_backward_block(rfmls_handle* h, const rfmls_csr* A, const rfmls_csr* AT,
                                const rfmls_precond_t* P, const double* Xs, int64_t ldx,
                                const double* Rres, int64_t ldr, const double* G, int64_t ldg,
                                int64_t nrhs, double* dB, int64_t lddb, double* dAval,
                                const rfmls_opts* o, rfmls_info* info) {
  const int64_t m = A->m, n = A->n;
  const int64_t itmax = o->itmax > 0 ? o->itmax : m;
  BCtx c;
  RFMLS_CHECK(make_bctx(h, A, AT, P, c));
  RFMLS_CHECK(spmm_tune_both(c));
  IterGraph graph;
  if (o->graph) c.graph = &graph;
  // roles: un (n), vm (m), vt, wt, zz shadows (n), tmp (n), lam (m), gathered blocks
  double* un = c.V;
  double* vm = c.U;
  double* vt = c.W;
  double* wt = c.Q;
  double* zz = c.Y;
  double* tmp = c.Z;
  double* lam = c.Rr;
  double* Gb = c.Xb;
  double* Xg = c.DX;
  double* Rg = c.Bb;
  const unsigned gm = grid_for(m * kBlk), gn = grid_for(n * kBlk);
  const int every = o->check_every > 0 ? o->check_every : 8;
  const BlockState* cst = c.dst;
  rfmls_status ret = RFMLS_OK;
  std::vector<BlockState> hs(1);
  for (int64_t k0 = 0; k0 < nrhs; k0 += kBlk) {
    const int64_t nb = nrhs - k0 < kBlk ? nrhs - k0 : kBlk;
    hipLaunchKernelGGL(k_gather_block, dim3(gn), dim3(kThreads), 0, c.st, G, ldg, k0, nb, n, Gb);
    // beta_1 u_1 = X^T g
    RFMLS_CHECK(tri_block(c, 1, Gb, un, 0.0, nullptr, nullptr, c.sqB, nullptr));
    hipLaunchKernelGGL(k_blk_norms, dim3(1), dim3(kRedThreads), 0, c.st, (const double*)c.sqB,
                       (int)rows_grid(n), c.dst, 0, 1);
    hipLaunchKernelGGL(k_blk_start, dim3(1), dim3(64), 0, c.st, c.dst, o->atol, o->btol, o->conlim, itmax);
    hipLaunchKernelGGL(k_blk_scale, dim3(gn), dim3(kThreads), 0, c.st, un, n, cst, 0, 1);
    hipLaunchKernelGGL(k_blk_fill, dim3(gn), dim3(kThreads), 0, c.st, zz, n * kBlk, 0.0);
    // alpha_1 v_1 = A (X u_1);  vt_1 = u_1 / alpha_1;  w_1 = vt_1
    RFMLS_CHECK(tri_block(c, 0, un, tmp, 0.0, nullptr, nullptr, nullptr, nullptr));
    int nbk = 0;
    RFMLS_CHECK(spmm(c, A, tmp, 1.0, 0.0, nullptr, nullptr, vm, c.sqA, nullptr, &nbk));
    hipLaunchKernelGGL(k_blk_norms, dim3(1), dim3(kRedThreads), 0, c.st, (const double*)c.sqA, nbk, c.dst, 1, 0);
    hipLaunchKernelGGL(k_blk_scale, dim3(gm), dim3(kThreads), 0, c.st, vm, m, cst, 1, 0);
    hipLaunchKernelGGL(k_blk_start2, dim3(1), dim3(64), 0, c.st, c.dst);
    hipLaunchKernelGGL(k_blk_recip_scale, dim3(gn), dim3(kThreads), 0, c.st, (const double*)un, 0.0,
                       (const double*)nullptr, vt, n, cst, 1);
    hipLaunchKernelGGL(k_blk_copy, dim3(gn), dim3(kThreads), 0, c.st, (const double*)vt, wt, n);
    hipLaunchKernelGGL(k_blk_sumsq, dim3(rows_grid(n)), dim3(kThreads), 0, c.st, (const double*)wt, n, c.sqW);
    RFMLS_HIP(h, hipGetLastError());
    RFMLS_CHECK(run_loop(c, itmax, every, [&]() -> rfmls_status {
      // beta u = X^T (A^T v) - alpha u
      RFMLS_CHECK(spmm(c, AT, vm, 1.0, 0.0, nullptr, nullptr, tmp, nullptr, cst, nullptr));
      RFMLS_CHECK(tri_block(c, 1, tmp, un, 1.0, state_field(c.dst, 1), un, c.sqB, cst));
      hipLaunchKernelGGL(k_blk_norms, dim3(1), dim3(kRedThreads), 0, c.st, (const double*)c.sqB,
                         (int)rows_grid(n), c.dst, 0, 0);
      hipLaunchKernelGGL(k_blk_scale, dim3(gn), dim3(kThreads), 0, c.st, un, n, cst, 0, 0);
      // alpha v = A (X u) - beta v;  vt = (u - beta vt) / alpha
      RFMLS_CHECK(tri_block(c, 0, un, tmp, 0.0, nullptr, nullptr, nullptr, cst));
      RFMLS_CHECK(spmm(c, A, tmp, 1.0, 1.0, state_field(c.dst, 0), vm, vm, c.sqA, cst, &nbk));
      hipLaunchKernelGGL(k_blk_norms, dim3(1), dim3(kRedThreads), 0, c.st, (const double*)c.sqA, nbk, c.dst, 1, 0);
      hipLaunchKernelGGL(k_blk_scale, dim3(gm), dim3(kThreads), 0, c.st, vm, m, cst, 1, 0);
      hipLaunchKernelGGL(k_blk_recip_scale, dim3(gn), dim3(kThreads), 0, c.st, (const double*)un, 1.0,
                         (const double*)vt, vt, n, cst, 0);
      hipLaunchKernelGGL(k_blk_rotate, dim3(1), dim3(kRedThreads), 0, c.st, c.dst, (const double*)c.sqW,
                         (int)rows_grid(n));
      hipLaunchKernelGGL(k_blk_update, dim3(rows_grid(n)), dim3(kThreads), 0, c.st, cst,
                         (const double*)vt, wt, zz, n, c.sqY, c.sqW);
      hipLaunchKernelGGL(k_blk_check, dim3(1), dim3(kRedThreads), 0, c.st, c.dst, (const double*)c.sqY,
                         (int)rows_grid(n), 1);
      RFMLS_HIP(h, hipGetLastError());
      return RFMLS_OK;
    }));
    RFMLS_CHECK(read_block_state(c, hs.data()));
    for (int64_t q = 0; q < nb; ++q) {
      const LsqrDev& st = hs[0].col[q];
      if (st.istop < 0)
        return fail(h, RFMLS_E_BREAKDOWN, "non-finite value in backward LSQR (column %lld)", (long long)(k0 + q));
      if (st.istop == 7) ret = RFMLS_W_NOCONV;
      if (info) {
        rfmls_info inf{};
        inf.itn = inf.itn_first = st.itn;
        inf.istop = inf.istop_last = st.istop;
        inf.normr_est = st.normr;
        inf.normb = st.bnorm;
        info[k0 + q] = inf;
      }
    }
    // w = X z, lam = A w
    RFMLS_CHECK(tri_block(c, 0, zz, tmp, 0.0, nullptr, nullptr, nullptr, nullptr));
    RFMLS_CHECK(spmm(c, A, tmp, 1.0, 0.0, nullptr, nullptr, lam, nullptr, nullptr, nullptr));
    if (dB)
      hipLaunchKernelGGL(k_scatter_block, dim3(gm), dim3(kThreads), 0, c.st, (const double*)lam, m, k0, nb, dB, lddb);
    if (dAval) {
      hipLaunchKernelGGL(k_gather_block, dim3(gm), dim3(kThreads), 0, c.st, Rres, ldr, k0, nb, m, Rg);
      hipLaunchKernelGGL(k_gather_block, dim3(gn), dim3(kThreads), 0, c.st, Xs, ldx, k0, nb, n, Xg);
      Trace tr(h, "pattern_grad_blk", 16.0 * (double)A->nnz + 8.0 * (double)(m + 1) + 16.0 * kBlk * (double)(m + n),
               4.0 * kBlk * (double)A->nnz);
      hipLaunchKernelGGL(k_blk_pattern_grad, dim3(spmm_grid(m)), dim3(kThreads), 0, c.st, A->row_ptr,
                         A->col, m, (const double*)Rg, (const double*)tmp, (const double*)lam,
                         (const double*)Xg, dAval, k0 > 0 ? 1 : 0);
    }
    RFMLS_HIP(h, hipGetLastError());
  }
  RFMLS_HIP(h, hipStreamSynchronize(c.st));
  return ret;
}

// B = A X in slabs of 32 columns: X's slab in the block layout, one lockstep
// SpMM with A (the kernel the multi-right-hand-side solve uses), the m x 32
// result scattered into B's rows.
rfmls_status run_form_B(rfmls_handle* h, const rfmls_csr* A, const rfmls_precond_t* P, double* Bmat,
                        int64_t ldb) {
  const int64_t m = A->m, n = A->n;
  BCtx c;
  RFMLS_CHECK(make_bctx(h, A, A, P, c));
  RFMLS_CHECK(spmm_tune_both(c));
  const unsigned gn = grid_for(n * kBlk), gm = grid_for(m * kBlk);
  for (int64_t c0 = 0; c0 < n; c0 += kBlk) {
    const int nb = (int)(n - c0 < kBlk ? n - c0 : kBlk);
    if (P->store == RFMLS_F64)
      hipLaunchKernelGGL(k_x_slab<double>, dim3(gn), dim3(kThreads), 0, c.st, (const double*)P->Xpk, n,
                         P->nt, P->full, c0, nb, c.Xb);
    else
      hipLaunchKernelGGL(k_x_slab<float>, dim3(gn), dim3(kThreads), 0, c.st, (const float*)P->Xpk, n,
                         P->nt, P->full, c0, nb, c.Xb);
    RFMLS_CHECK(spmm(c, A, c.Xb, 1.0, 0.0, nullptr, nullptr, c.U, nullptr, nullptr, nullptr));
    hipLaunchKernelGGL(k_scatter_slab, dim3(gm), dim3(kThreads), 0, c.st, (const double*)c.U, m, c0, nb,
                       Bmat, ldb);
    RFMLS_HIP(h, hipGetLastError());
  }
  return RFMLS_OK;
}

}  // namespace rfmls
