// LSQR on the preconditioned operator B = A R^{-1} (Alg. 1 steps 4-6 with the
// preconditioner applied inside the iteration, Remark 3.2), textbook
// Paige-Saunders recurrences with every scalar kept on the device.
//
// Products used by one iteration:
//   z = X v            triangular product with the packed X = R^{-1}  (k_trmv_*)
//   u^ = A z - a u     SpMV over each row's column runs                (k_spmv_runs)
//   q = A^T u          the same with the explicit transpose            (k_spmv_runs)
//   v^ = X^T q - b v   transposed triangular product                   (k_trmvT_*)
// followed by the plane rotation and the updates of y and w.  Norms are
// reduced in a fixed order (per-block partials, then a fixed tree), so runs
// are bitwise reproducible.  The host only polls a device "done" flag every
// few iterations; kernels launched after the stop return immediately.
#include <mutex>

#include "common.h"
#include "lsqr_dev.h"

namespace rfmls {
namespace {

constexpr int kThreads = 256;
constexpr int kSpmvMaxBlocks = 2048;

// ---------------------------------------------------------------------------
// Triangular products with the packed tiles of X (64 x 64, upper triangle)
// ---------------------------------------------------------------------------
// z = X v: block e handles tile row I = tab[e].x, tiles J in [J_0 + k C, J_0 + (k+1) C)
// with J_0 = row_first(I) (I for the triangular packing, 0 for the full grid).
// Thread (c = lane, w = wave) accumulates rows w + 4q of the tile row against
// column c, then each row is summed across the wavefront.
template <typename TS>
__global__ void __launch_bounds__(kThreads)
    k_trmv_part(const TS* __restrict__ Xpk, int64_t nt, int64_t n, int full, const int2* __restrict__ tab,
                int C, int maxk, const double* __restrict__ v, double* __restrict__ part,
                const int* __restrict__ done) {
  if (done && *done) return;
  const int2 e = tab[blockIdx.x];
  const int64_t I = e.x;
  const int k = e.y;
  const int64_t J0 = row_first(I, full) + (int64_t)k * C;
  const int64_t J1 = J0 + C < nt ? J0 + C : nt;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  // two tiles' loads in flight per iteration (sums in the same order)
#pragma unroll 2
  for (int64_t J = J0; J < J1; ++J) {
    const TS* t = Xpk + ptile(I, J, nt, full) * (int64_t)(kTile * kTile);
    const int64_t gc = J * kTile + lane;
    const double vc = gc < n ? v[gc] : 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] += (double)t[(w + 4 * q) * kTile + lane] * vc;
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const double s = wave_sum(acc[q]);
    if (lane == 0) part[((int64_t)I * maxk + k) * kTile + w + 4 * q] = s;
  }
}

// p = X^T q: block e handles tile column J = tab[e].x, tiles I in [k C, min((k+1) C, col_end(J))).
template <typename TS>
__global__ void __launch_bounds__(kThreads)
    k_trmvT_part(const TS* __restrict__ Xpk, int64_t nt, int64_t n, int full, const int2* __restrict__ tab,
                 int C, int maxk, const double* __restrict__ qv, double* __restrict__ part,
                 const int* __restrict__ done) {
  if (done && *done) return;
  __shared__ double red[4][kTile];
  const int2 e = tab[blockIdx.x];
  const int64_t J = e.x;
  const int k = e.y;
  const int64_t I0 = (int64_t)k * C;
  const int64_t Iend = col_end(J, nt, full);
  const int64_t I1 = I0 + C < Iend ? I0 + C : Iend;
  const int lane = threadIdx.x & 63;
  // the wavefront index as a uniform value: the 16 entries of qv a wavefront
  // needs per tile are then scalar loads, with no branch for the bound test
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double acc0 = 0.0, acc1 = 0.0;  // two chains over alternate rows
#pragma unroll 2
  for (int64_t I = I0; I < I1; ++I) {
    const TS* t = Xpk + ptile(I, J, nt, full) * (int64_t)(kTile * kTile);
#pragma unroll
    for (int q = 0; q < 16; q += 2) {
      const int r = w + 4 * q;
      const int64_t gr = I * kTile + r;
      const double q0 = gr < n ? qv[gr] : 0.0;
      const double q1 = gr + 4 < n ? qv[gr + 4] : 0.0;
      acc0 += (double)t[r * kTile + lane] * q0;
      acc1 += (double)t[(r + 4) * kTile + lane] * q1;
    }
  }
  const double acc = acc0 + acc1;
  red[w][lane] = acc;
  __syncthreads();
  if (w == 0)
    part[((int64_t)J * maxk + k) * kTile + lane] =
        (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

// out[i] = sum_k part[row(i)][k] - coef * prev[i];  partial sum of squares per block.
// nk(I) = number of chunks of tile row/column I (trans: ceil(col_end(I)/C), else
// ceil((nt - row_first(I))/C)).
// A block handles tile rows I (64 outputs each, grid-stride); its four
// wavefronts sum every fourth partial of each output (independent loads in
// flight), and the four quarter sums are added in a fixed order.
constexpr int kRedMaxBlocks = 2048;

__global__ void __launch_bounds__(kThreads)
    k_tri_reduce(const double* __restrict__ part, int64_t nt, int64_t n, int full, int C, int maxk, int trans,
                 double hcoef, const double* __restrict__ dcoef, const double* prev,
                 double* out, double* __restrict__ sq, const int* __restrict__ done) {
  if (done && *done) return;
  __shared__ double scratch[kThreads / 64];
  __shared__ double quarter[kThreads / 64][kTile];
  const int r = threadIdx.x & (kTile - 1);
  const int q = threadIdx.x / kTile;
  double cf = hcoef;
  if (dcoef) cf *= *dcoef;
  double ss = 0.0;
  for (int64_t I = blockIdx.x; I < nt; I += gridDim.x) {
    const int64_t i = I * kTile + r;
    const int64_t nk = trans ? (col_end(I, nt, full) + C - 1) / C : (nt - row_first(I, full) + C - 1) / C;
    double s = 0.0;
    if (i < n)
      for (int64_t k = q; k < nk; k += kThreads / kTile) s += part[(I * maxk + k) * kTile + r];
    quarter[q][r] = s;
    __syncthreads();
    if (q == 0 && i < n) {
      double t = (quarter[0][r] + quarter[1][r]) + (quarter[2][r] + quarter[3][r]);
      if (prev && cf != 0.0) t -= cf * prev[i];
      out[i] = t;
      ss += t * t;
    }
    __syncthreads();
  }
  if (sq) {
    ss = block_sum(ss, scratch);
    if (threadIdx.x == 0) sq[blockIdx.x] = ss;
  }
}

// ---------------------------------------------------------------------------
// CSR SpMV: out[row] = sA * (A x)[row] - coef * prev[row]; half a wavefront (32
// lanes) per row, two entries per lane in flight (measured on the RFM matrix
// and its transpose: 5.2-5.9 TB/s against 3.8-4.3 for a wavefront per row).
// ---------------------------------------------------------------------------
constexpr int kSpvLanes = 32;

__global__ void __launch_bounds__(kThreads)
    k_spmv(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
           const double* __restrict__ val, int64_t rows, const double* __restrict__ x, double sA,
           double hcoef, const double* __restrict__ dcoef, const double* prev, double* out,
           double* __restrict__ sq, const int* __restrict__ done) {
  if (done && *done) return;
  __shared__ double scratch[kThreads / 64];
  const int lane = threadIdx.x & (kSpvLanes - 1);
  const int64_t sub = ((int64_t)blockIdx.x * kThreads + threadIdx.x) / kSpvLanes;
  const int64_t nsub = (int64_t)gridDim.x * (kThreads / kSpvLanes);
  double cf = hcoef;
  if (dcoef) cf *= *dcoef;
  double ss = 0.0;
  for (int64_t row = sub; row < rows; row += nsub) {
    const int64_t lo = rp[row], hi = rp[row + 1];
    double s0 = 0.0, s1 = 0.0;
    int64_t e = lo + lane;
    for (; e + kSpvLanes < hi; e += 2 * kSpvLanes) {
      s0 += val[e] * x[col[e]];
      s1 += val[e + kSpvLanes] * x[col[e + kSpvLanes]];
    }
    if (e < hi) s0 += val[e] * x[col[e]];
    double t = s0 + s1;
#pragma unroll
    for (int o = kSpvLanes / 2; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if (lane == 0) {
      double o = sA * t;
      if (prev && cf != 0.0) o -= cf * prev[row];
      out[row] = o;
      ss += o * o;
    }
  }
  if (sq) {
    ss = block_sum(ss, scratch);
    if (threadIdx.x == 0) sq[blockIdx.x] = ss;
  }
}

// ---------------------------------------------------------------------------
// Column runs.  The rows of an RFM matrix cover the basis functions of one or
// two boxes, contiguous column ranges, and the rows of its transpose a few
// blocks of collocation points.  Row i is described as at most kMaxRuns runs
// of consecutive columns: run k starts at column rcol[i kMaxRuns + k] and
// ends before entry rend[i kMaxRuns + k] of the row (counted from rp[i]); the
// SpMV then reads 8 bytes per entry (its value) instead of 12 and x in
// contiguous stretches.  nrun[i] = -1 marks a row with more runs, which takes
// the column-index path.
// ---------------------------------------------------------------------------
constexpr int kMaxRuns = 8;
// lanes per row of the run SpMV for matrices whose rows average fewer than
// 512 entries (more rows in flight per wavefront: spmv_A 0.054 -> 0.048 ms on
// the 8x8-box system's 216-entry rows, 0.060 -> 0.055 ms on the Helmholtz
// system's 446-entry rows; 4 lanes and 16 were slower); longer rows keep 32
constexpr int kSpvLanesShort = 8;

__global__ void __launch_bounds__(kThreads)
    k_find_runs(const int64_t* __restrict__ rp, const int32_t* __restrict__ col, int64_t rows,
                int32_t* __restrict__ nrun, int32_t* __restrict__ rcol, int32_t* __restrict__ rend) {
  const int lane = threadIdx.x & (kSpvLanes - 1);
  const int half = (threadIdx.x & 63) >> 5;
  const int64_t sub = ((int64_t)blockIdx.x * kThreads + threadIdx.x) / kSpvLanes;
  const int64_t nsub = (int64_t)gridDim.x * (kThreads / kSpvLanes);
  for (int64_t row = sub; row < rows; row += nsub) {
    const int64_t lo = rp[row], hi = rp[row + 1];
    int cnt = 0;  // runs found so far (uniform over the row's 32 lanes)
    for (int64_t b = lo; b < hi; b += kSpvLanes) {
      const int64_t e = b + lane;
      const bool in = e < hi;
      const int32_t c = in ? col[e] : 0;
      const int32_t pc = (in && e > lo) ? col[e - 1] : 0;
      const bool start = in && (e == lo || c != pc + 1);
      const unsigned bits = (unsigned)(__ballot(start) >> (32 * half));
      const int idx = cnt + __popc(bits & ((1u << lane) - 1u));
      if (start && idx < kMaxRuns) {
        rcol[row * kMaxRuns + idx] = c;
        if (idx > 0) rend[row * kMaxRuns + idx - 1] = (int32_t)(e - lo);
      }
      cnt += __popc(bits);
    }
    if (lane == 0) {
      if (cnt >= 1 && cnt <= kMaxRuns) rend[row * kMaxRuns + cnt - 1] = (int32_t)(hi - lo);
      nrun[row] = cnt <= kMaxRuns ? cnt : -1;
    }
  }
}

// k_spmv over column runs (rows marked -1 take the column-index path), L
// lanes per row.  A row's pointers, run count and first run are loaded
// together, and the next row's while this one is summed, so a row costs one
// memory latency instead of three.
template <int L>
__global__ void __launch_bounds__(kThreads)
    k_spmv_runs(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                const double* __restrict__ val, int64_t rows, const int32_t* __restrict__ nrun,
                const int32_t* __restrict__ rcol, const int32_t* __restrict__ rend,
                const double* __restrict__ x, double sA, double hcoef, const double* __restrict__ dcoef,
                const double* prev, double* out, double* __restrict__ sq, const int* __restrict__ done) {
  if (done && *done) return;
  __shared__ double scratch[kThreads / 64];
  const int lane = threadIdx.x & (L - 1);
  const int64_t sub = ((int64_t)blockIdx.x * kThreads + threadIdx.x) / L;
  const int64_t nsub = (int64_t)gridDim.x * (kThreads / L);
  double cf = hcoef;
  if (dcoef) cf *= *dcoef;
  double ss = 0.0;
  int64_t lo = 0, hi = 0;
  int nr = 0;
  int32_t e0 = 0, c0 = 0;
  if (sub < rows) {
    lo = rp[sub];
    hi = rp[sub + 1];
    nr = nrun[sub];
    e0 = rend[sub * kMaxRuns];
    c0 = rcol[sub * kMaxRuns];
  }
  for (int64_t row = sub; row < rows; row += nsub) {
    const int64_t nrow = row + nsub;
    int64_t nlo = 0, nhi = 0;
    int nnr = 0;
    int32_t ne0 = 0, nc0 = 0;
    if (nrow < rows) {
      nlo = rp[nrow];
      nhi = rp[nrow + 1];
      nnr = nrun[nrow];
      ne0 = rend[nrow * kMaxRuns];
      nc0 = rcol[nrow * kMaxRuns];
    }
    double s0 = 0.0, s1 = 0.0;
    if (nr < 0) {
      int64_t e = lo + lane;
      for (; e + L < hi; e += 2 * L) {
        s0 += val[e] * x[col[e]];
        s1 += val[e + L] * x[col[e + L]];
      }
      if (e < hi) s0 += val[e] * x[col[e]];
    } else {
      const double* vr = val + lo;
      int32_t off = 0;
      for (int k = 0; k < nr; ++k) {
        const int32_t end = k == 0 ? e0 : rend[row * kMaxRuns + k];
        const double* xr = x + (k == 0 ? c0 : rcol[row * kMaxRuns + k]);  // column of entry off
        // four entries per lane in flight (the transposes' rows run to
        // thousands of entries: 0.085 -> 0.064 ms on the Helmholtz A^T)
        int32_t e = off + lane;
        for (; e + 3 * L < end; e += 4 * L) {
          s0 += vr[e] * xr[e - off];
          s1 += vr[e + L] * xr[e + L - off];
          s0 += vr[e + 2 * L] * xr[e + 2 * L - off];
          s1 += vr[e + 3 * L] * xr[e + 3 * L - off];
        }
        for (; e < end; e += L) s0 += vr[e] * xr[e - off];
        off = end;
      }
    }
    double t = s0 + s1;
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if (lane == 0) {
      double o = sA * t;
      if (prev && cf != 0.0) o -= cf * prev[row];
      out[row] = o;
      ss += o * o;
    }
    lo = nlo;
    hi = nhi;
    nr = nnr;
    e0 = ne0;
    c0 = nc0;
  }
  if (sq) {
    ss = block_sum(ss, scratch);
    if (threadIdx.x == 0) sq[blockIdx.x] = ss;
  }
}

// ---------------------------------------------------------------------------
// Vector helpers
// ---------------------------------------------------------------------------
// nrm = sqrt(sum sq[0..nsq)), fixed order; every block computes it, block 0 stores it.
__device__ double reduce_partials(const double* __restrict__ sq, int nsq, double* scratch) {
  double t = 0.0;
  for (int i = threadIdx.x; i < nsq; i += blockDim.x) t += sq[i];
  return block_sum(t, scratch);
}

__global__ void __launch_bounds__(kThreads)
    k_normalize(double* vec, int64_t len, const double* __restrict__ sq, int nsq,
                double* __restrict__ nrm_out, const int* __restrict__ done) {
  if (done && *done) return;
  __shared__ double scratch[kThreads / 64];
  const double nrm = sqrt(reduce_partials(sq, nsq, scratch));
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * kThreads)
    vec[i] *= inv;
  if (blockIdx.x == 0 && threadIdx.x == 0) *nrm_out = nrm;
}

// out = (a * x + b * y) with a = ha * (*da), b = hb * (*db) (null pointers read as 1)
__global__ void k_axpby(int64_t len, double ha, const double* __restrict__ da, const double* x,
                        double hb, const double* __restrict__ db, const double* y, double* out,
                        const int* __restrict__ done) {
  if (done && *done) return;
  double a = ha, b = hb;
  if (da) a *= *da;
  if (db) b *= *db;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x) {
    double o = a * x[i];
    if (y) o += b * y[i];
    out[i] = o;
  }
}

// out = (x - hb * (*db) * y) / (*dal)   (0 where *dal is not positive)
__global__ void k_recip_scale(const double* x, double hb, const double* __restrict__ db,
                              const double* y, const double* __restrict__ dal, double* out,
                              int64_t len, const int* __restrict__ done) {
  if (done && *done) return;
  const double al = *dal;
  const double inv = al > 0.0 ? 1.0 / al : 0.0;
  double b = hb;
  if (db) b *= *db;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x) {
    double o = x[i];
    if (y && b != 0.0) o -= b * y[i];
    out[i] = o * inv;
  }
}

__global__ void k_fill(double* p, int64_t len, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// out[0] = sqrt(sum sq[0..nsq)) in the fixed order of reduce_partials (one block)
__global__ void __launch_bounds__(kThreads) k_sqrt_sum(const double* __restrict__ sq, int nsq,
                                                       double* __restrict__ out) {
  __shared__ double red[kThreads / 64];
  const double t = reduce_partials(sq, nsq, red);
  if (threadIdx.x == 0) out[0] = sqrt(t);
}

__global__ void __launch_bounds__(kThreads) k_sumsq(const double* __restrict__ x, int64_t len,
                                                    double* __restrict__ sq) {
  __shared__ double scratch[kThreads / 64];
  double t = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * kThreads)
    t += x[i] * x[i];
  t = block_sum(t, scratch);
  if (threadIdx.x == 0) sq[blockIdx.x] = t;
}

// ---------------------------------------------------------------------------
// LSQR scalars
// ---------------------------------------------------------------------------
// After beta_1 = ||b||: set up the state.
__global__ void k_lsqr_start(LsqrDev* st) {
  st->bnorm = st->beta;
  st->phibar = st->beta;
  st->anorm2 = 0.0;
  st->ddnorm = 0.0;
  st->itn = 0;
  st->istop = 7;
  st->pending = 0;
  st->done = 0;
  if (!isfinite(st->beta)) {  // a non-finite right-hand side: breakdown, not "x = 0 is exact"
    st->istop = -3;
    st->done = 1;
  } else if (!(st->beta > 0.0)) {
    st->istop = 0;
    st->done = 1;
  }
}

// After alpha_1 = ||B^T u_1||.
__global__ void k_lsqr_start2(LsqrDev* st) {
  if (st->done) return;
  st->rhobar = st->alpha;
  st->normr = st->beta;
  st->normar = st->alpha * st->beta;
  if (!isfinite(st->alpha)) {
    st->istop = -3;
    st->done = 1;
  } else if (!(st->alpha > 0.0)) {
    st->istop = 0;
    st->done = 1;
  }
}

// Plane rotation of iteration k (alpha = alpha_{k+1}, beta = beta_{k+1} are
// already in the state); wsq holds the partial sums of ||w_k||^2.
__global__ void __launch_bounds__(kThreads) k_lsqr_rotate(LsqrDev* st, const double* __restrict__ wsq,
                                                          int nsq) {
  if (st->done) return;
  __shared__ double scratch[kThreads / 64];
  const double w2 = reduce_partials(wsq, nsq, scratch);
  if (threadIdx.x != 0) return;
  const double alpha = st->alpha, beta = st->beta;
  st->itn += 1;
  st->anorm2 += st->alpha_prev * st->alpha_prev + beta * beta;
  const double rho = hypot(st->rhobar, beta);
  if (!(rho > 0.0) || !isfinite(rho)) {
    st->istop = isfinite(rho) ? 1 : -3;
    st->done = 1;
    st->phi_rho = 0.0;
    st->theta_rho = 0.0;
    return;
  }
  const double c = st->rhobar / rho;
  const double s = beta / rho;
  const double theta = s * alpha;
  st->rhobar = -c * alpha;
  const double phi = c * st->phibar;
  st->phibar = s * st->phibar;
  st->phi_rho = phi / rho;
  st->theta_rho = theta / rho;
  st->ddnorm += w2 / (rho * rho);
  const double anorm = sqrt(st->anorm2);
  st->acond = anorm * sqrt(st->ddnorm);
  st->normr = st->phibar;
  st->normar = st->phibar * alpha * fabs(c);
  st->pending = 0;
  if (st->normr == 0.0 || st->normar <= st->atol * anorm * st->normr) st->pending = 2;
  else if (st->conlim > 0.0 && st->acond >= st->conlim) st->pending = 3;
  st->alpha_prev = alpha;
}

// y += phi/rho w;  w = v - theta/rho w;  partial sums of ||y||^2 and ||w||^2.
__global__ void __launch_bounds__(kThreads)
    k_lsqr_update(const LsqrDev* __restrict__ st, const double* __restrict__ v, double* w,
                  double* y, int64_t n, double* __restrict__ ysq, double* __restrict__ wsq) {
  if (st->done) return;
  __shared__ double scratch[kThreads / 64];
  const double a = st->phi_rho, b = st->theta_rho;
  double sy = 0.0, sw = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const double wi = w[i];
    const double yi = y[i] + a * wi;
    const double wn = v[i] - b * wi;
    y[i] = yi;
    w[i] = wn;
    sy += yi * yi;
    sw += wn * wn;
  }
  sy = block_sum(sy, scratch);
  sw = block_sum(sw, scratch);
  if (threadIdx.x == 0) {
    ysq[blockIdx.x] = sy;
    wsq[blockIdx.x] = sw;
  }
}

// Stopping tests of iteration k (S1 needs ||y_k||, available only now).
__global__ void __launch_bounds__(kThreads) k_lsqr_check(LsqrDev* st, const double* __restrict__ ysq,
                                                         int nsq, int consistent) {
  if (st->done) return;
  __shared__ double scratch[kThreads / 64];
  const double y2 = reduce_partials(ysq, nsq, scratch);
  if (threadIdx.x != 0) return;
  st->ynorm = sqrt(y2);
  const double anorm = sqrt(st->anorm2);
  int istop = 0;
  const double rtol = consistent ? st->btol * st->bnorm
                                 : st->btol * st->bnorm + st->atol * anorm * st->ynorm;
  if (st->normr <= rtol) istop = 1;
  else if (st->pending) istop = st->pending;
  else if (st->itn >= st->itmax) istop = 7;
  if (istop) {
    st->istop = istop;
    st->done = 1;
  }
}

// dA[e] += r_i w_j - lam_i x_j on the pattern of A
__global__ void k_pattern_grad(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                               int64_t m, const double* __restrict__ r, const double* __restrict__ w,
                               const double* __restrict__ lam, const double* __restrict__ x,
                               double* __restrict__ dA, int accumulate) {
  const int lane = threadIdx.x & 63;
  const int64_t wid = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t row = wid; row < m; row += nw) {
    const double ri = r[row], li = lam[row];
    for (int64_t e = rp[row] + lane; e < rp[row + 1]; e += 64) {
      const int32_t j = col[e];
      const double g = ri * w[j] - li * x[j];
      dA[e] = accumulate ? dA[e] + g : g;
    }
  }
}

// ---------------------------------------------------------------------------
// Dense products with the explicit B = A R^{-1} (row-major m x n, Alg. 1 step 4).
// ---------------------------------------------------------------------------
// out[i] = sA (B v)[i] - cf prev[i], cf = hcoef (*dcoef); one wavefront per
// row, four independent partial sums per lane, a fixed-order tree across the
// wavefront; per-block sums of squares of out into sq.
__global__ void __launch_bounds__(kThreads)
    k_gemv(const double* __restrict__ B, int64_t ldb, int64_t m, int64_t n,
           const double* __restrict__ v, double sA, double hcoef, const double* __restrict__ dcoef,
           const double* prev, double* out, double* __restrict__ sq, const int* __restrict__ done) {
  if (done && *done) return;
  __shared__ double scratch[kThreads / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double cf = hcoef;
  if (dcoef) cf *= *dcoef;
  double ss = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * (kThreads / 64) + w; i < m; i += (int64_t)gridDim.x * (kThreads / 64)) {
    const double* row = B + i * ldb;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int64_t j = lane;
    for (; j + 192 < n; j += 256) {
      a0 += row[j] * v[j];
      a1 += row[j + 64] * v[j + 64];
      a2 += row[j + 128] * v[j + 128];
      a3 += row[j + 192] * v[j + 192];
    }
    for (; j < n; j += 64) a0 += row[j] * v[j];
    double t = wave_sum((a0 + a1) + (a2 + a3));
    if (lane == 0) {
      t = sA * t;
      if (prev && cf != 0.0) t -= cf * prev[i];
      out[i] = t;
      ss += t * t;
    }
  }
  if (sq) {
    ss = block_sum(ss, scratch);
    if (threadIdx.x == 0) sq[blockIdx.x] = ss;
  }
}

// part[z][j] = sum over the rows i of slice z of B[i][j] u[i]: block (x, z)
// covers the 2 kThreads columns from 2 kThreads x and rows [z rps, (z + 1) rps).
__global__ void __launch_bounds__(kThreads)
    k_gemvT_part(const double* __restrict__ B, int64_t ldb, int64_t m, int64_t n,
                 const double* __restrict__ u, int64_t rps, double* __restrict__ part,
                 const int* __restrict__ done) {
  if (done && *done) return;
  const int64_t j0 = (int64_t)blockIdx.x * 2 * kThreads + threadIdx.x, j1 = j0 + kThreads;
  const int64_t r0 = (int64_t)blockIdx.y * rps;
  const int64_t r1 = r0 + rps < m ? r0 + rps : m;
  double a0 = 0.0, a1 = 0.0;
  for (int64_t i = r0; i < r1; ++i) {
    const double ui = u[i];
    const double* row = B + i * ldb;
    if (j0 < n) a0 += row[j0] * ui;
    if (j1 < n) a1 += row[j1] * ui;
  }
  double* p = part + (int64_t)blockIdx.y * n;
  if (j0 < n) p[j0] = a0;
  if (j1 < n) p[j1] = a1;
}

// out[j] = sum_z part[z][j] (in slice order) - cf prev[j]; per-block sums of squares.
__global__ void __launch_bounds__(kThreads)
    k_gemvT_reduce(const double* __restrict__ part, int nz, int64_t n, double hcoef,
                   const double* __restrict__ dcoef, const double* prev, double* out,
                   double* __restrict__ sq, const int* __restrict__ done) {
  if (done && *done) return;
  __shared__ double scratch[kThreads / 64];
  double cf = hcoef;
  if (dcoef) cf *= *dcoef;
  double ss = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x; j < n; j += (int64_t)gridDim.x * kThreads) {
    double t = 0.0;
    for (int z = 0; z < nz; ++z) t += part[(int64_t)z * n + j];
    if (prev && cf != 0.0) t -= cf * prev[j];
    out[j] = t;
    ss += t * t;
  }
  if (sq) {
    ss = block_sum(ss, scratch);
    if (threadIdx.x == 0) sq[blockIdx.x] = ss;
  }
}

}  // namespace

// ===========================================================================
// Host drivers
// ===========================================================================
struct Ctx {
  rfmls_handle* h;
  const rfmls_csr* A;
  const rfmls_csr* AT;
  const rfmls_precond_t* P;
  const double* Bm = nullptr;  // explicit B = A R^{-1} (row-major), or null: implicit operator
  int64_t ldbm = 0;
  double* gpart = nullptr;     // slice partials of B^T u
  hipStream_t st;
  // work vectors
  double *u, *v, *w, *y, *z, *q, *t, *r, *xs;
  double *sqA, *sqB, *sqY, *sqW;
  double* hn;  // one device double for norms read by the host
  LsqrDev* dst;
  IterGraph* graph = nullptr;  // captured poll interval of the loop, or null: eager launches
  int nspmvA, nspmvAT, nvec_n, nvec_m;
  // column runs of A and A^T (null: the column-index SpMV)
  const int32_t *nrunA = nullptr, *rcolA = nullptr, *rendA = nullptr;
  const int32_t *nrunAT = nullptr, *rcolAT = nullptr, *rendAT = nullptr;
};

static unsigned spmv_blocks(int64_t rows) {
  const int64_t b = (rows + kThreads / kSpvLanes - 1) / (kThreads / kSpvLanes);
  return (unsigned)(b < kSpmvMaxBlocks ? (b > 0 ? b : 1) : kSpmvMaxBlocks);
}
static unsigned vec_blocks(int64_t len) {
  const int64_t b = (len + kThreads - 1) / kThreads;
  return (unsigned)(b < 1024 ? (b > 0 ? b : 1) : 1024);
}

int tri_reduce_blocks(int64_t n) {
  const int64_t b = ceil_div(n, kTile);
  return (int)(b < kRedMaxBlocks ? (b > 0 ? b : 1) : kRedMaxBlocks);
}

rfmls_status tri_apply(rfmls_handle* h, const rfmls_precond_t* P, int trans, const double* in,
                       double* out, double hcoef, const double* dcoef, const double* prev,
                       double* sq, const int* done) {
  const int64_t n = P->n, nt = P->nt;
  const int C = P->chunk;
  const int maxk = (int)((nt + C - 1) / C);
  hipStream_t st = h->stream;
  double* part = (double*)P->part;
  const double esz = P->store == RFMLS_F64 ? 8.0 : 4.0;
  const int full = P->full;
  const double tri_elems = full ? (double)n * (double)n : (double)n * (double)(n + 1) / 2.0;
  {
  // algorithmic: the stored entries of X once (n(n+1)/2, or n^2 for the full
  // SVD preconditioner), the input vector, the output
  Trace tr(h, full ? (trans ? "gemv_Pt" : "gemv_P") : (trans ? "trmv_Xt" : "trmv_X"),
           esz * tri_elems + 16.0 * (double)n, 2.0 * tri_elems);
  if (!trans) {
    if (P->store == RFMLS_F64)
      hipLaunchKernelGGL(k_trmv_part<double>, dim3((unsigned)P->ntab), dim3(kThreads), 0, st,
                         (const double*)P->Xpk, nt, n, full, P->tab_row, C, maxk, in, part, done);
    else
      hipLaunchKernelGGL(k_trmv_part<float>, dim3((unsigned)P->ntab), dim3(kThreads), 0, st,
                         (const float*)P->Xpk, nt, n, full, P->tab_row, C, maxk, in, part, done);
  } else {
    if (P->store == RFMLS_F64)
      hipLaunchKernelGGL(k_trmvT_part<double>, dim3((unsigned)P->ntab), dim3(kThreads), 0, st,
                         (const double*)P->Xpk, nt, n, full, P->tab_col, C, maxk, in, part, done);
    else
      hipLaunchKernelGGL(k_trmvT_part<float>, dim3((unsigned)P->ntab), dim3(kThreads), 0, st,
                         (const float*)P->Xpk, nt, n, full, P->tab_col, C, maxk, in, part, done);
  }
  }
  Trace tr2(h, "tri_reduce", 8.0 * (double)nt * maxk * kTile + 16.0 * (double)n, 0.0);
  hipLaunchKernelGGL(k_tri_reduce, dim3((unsigned)tri_reduce_blocks(n)), dim3(kThreads), 0, st, part, nt, n,
                     full, C, maxk, trans, hcoef, dcoef, prev, out, sq, done);
  RFMLS_HIP(h, hipGetLastError());
  return RFMLS_OK;
}


static rfmls_status spmv(Ctx& c, const rfmls_csr* M, const double* x, double sA, double hcoef,
                         const double* dcoef, const double* prev, double* out, double* sq,
                         const int* done, int* nblk) {
  const unsigned nb = spmv_blocks(M->m);
  const int32_t* nrun = M == c.A ? c.nrunA : c.nrunAT;
  const int32_t* rcol = M == c.A ? c.rcolA : c.rcolAT;
  const int32_t* rend = M == c.A ? c.rendA : c.rendAT;
  // algorithmic: values once (and the column indices, unless the rows are
  // described by their column runs: then a run count and at least one run per
  // row), row pointers, x gathered once, out written (and prev read when used)
  const double idx_bytes = nrun ? 4.0 * (double)M->m * (1 + 2) : 4.0 * (double)M->nnz;
  Trace tr(c.h, M == c.A ? "spmv_A" : "spmv_At",
           8.0 * (double)M->nnz + idx_bytes + 8.0 * (double)(M->m + 1) + 8.0 * (double)M->n +
               8.0 * (double)M->m * (prev ? 2.0 : 1.0),
           2.0 * (double)M->nnz);
  if (nrun && M->nnz < 512 * M->m) {
    const int64_t b = (M->m + kThreads / kSpvLanesShort - 1) / (kThreads / kSpvLanesShort);
    const unsigned nbs = (unsigned)(b < kSpmvMaxBlocks ? (b > 0 ? b : 1) : kSpmvMaxBlocks);
    hipLaunchKernelGGL(k_spmv_runs<kSpvLanesShort>, dim3(nbs), dim3(kThreads), 0, c.st, M->row_ptr, M->col, M->val,
                       M->m, nrun, rcol, rend, x, sA, hcoef, dcoef, prev, out, sq, done);
    if (nblk) *nblk = (int)nbs;
    RFMLS_HIP(c.h, hipGetLastError());
    return RFMLS_OK;
  }
  if (nrun)
    hipLaunchKernelGGL(k_spmv_runs<kSpvLanes>, dim3(nb), dim3(kThreads), 0, c.st, M->row_ptr, M->col, M->val, M->m,
                       nrun, rcol, rend, x, sA, hcoef, dcoef, prev, out, sq, done);
  else
    hipLaunchKernelGGL(k_spmv, dim3(nb), dim3(kThreads), 0, c.st, M->row_ptr, M->col, M->val, M->m,
                       x, sA, hcoef, dcoef, prev, out, sq, done);
  if (nblk) *nblk = (int)nb;
  RFMLS_HIP(c.h, hipGetLastError());
  return RFMLS_OK;
}

// Products with the explicit B (Ctx::Bm): out = B v - cf prev over the m rows,
// and out = B^T u - cf prev over the n columns (slice partials, then a
// fixed-order sum); each writes per-block sums of squares to sq and returns
// their count in *nblk.
constexpr int kGemvTSlices = 64;
static rfmls_status bmul(Ctx& c, const double* v, double hcoef, const double* dcoef,
                         const double* prev, double* out, double* sq, const int* done, int* nblk) {
  const int64_t m = c.A->m, n = c.A->n;
  const int64_t b = (m + kThreads / 64 - 1) / (kThreads / 64);
  const unsigned nb = (unsigned)(b < kSpmvMaxBlocks ? (b > 0 ? b : 1) : kSpmvMaxBlocks);
  Trace tr(c.h, "gemv_B", 8.0 * (double)m * (double)n + 8.0 * (double)n + 8.0 * (double)m * (prev ? 2.0 : 1.0),
           2.0 * (double)m * (double)n);
  hipLaunchKernelGGL(k_gemv, dim3(nb), dim3(kThreads), 0, c.st, c.Bm, c.ldbm, m, n, v, 1.0, hcoef, dcoef,
                     prev, out, sq, done);
  *nblk = (int)nb;
  RFMLS_HIP(c.h, hipGetLastError());
  return RFMLS_OK;
}
static rfmls_status btmul(Ctx& c, const double* u, double hcoef, const double* dcoef,
                          const double* prev, double* out, double* sq, const int* done, int* nblk) {
  const int64_t m = c.A->m, n = c.A->n;
  const int64_t rps = (m + kGemvTSlices - 1) / kGemvTSlices;
  const int nz = (int)((m + rps - 1) / rps);
  const unsigned nr = vec_blocks(n);
  {
    Trace tr(c.h, "gemvT_B", 8.0 * (double)m * (double)n + 8.0 * (double)m + 8.0 * (double)nz * (double)n,
             2.0 * (double)m * (double)n);
    hipLaunchKernelGGL(k_gemvT_part, dim3(ceil_div(n, 2 * kThreads), (unsigned)nz), dim3(kThreads), 0, c.st,
                       c.Bm, c.ldbm, m, n, u, rps, c.gpart, done);
    hipLaunchKernelGGL(k_gemvT_reduce, dim3(nr), dim3(kThreads), 0, c.st, (const double*)c.gpart, nz, n,
                       hcoef, dcoef, prev, out, sq, done);
  }
  *nblk = (int)nr;
  RFMLS_HIP(c.h, hipGetLastError());
  return RFMLS_OK;
}

// The pinned staging buffer: [0, 1024) uploads, [1024, 4096) downloads.  Every
// upload is followed by a stream synchronisation before the buffer is reused.
static rfmls_status upload_state(Ctx& c, const rfmls_opts* o, int64_t itmax) {
  LsqrDev* pin = (LsqrDev*)c.h->pinned;
  RFMLS_HIP(c.h, hipStreamSynchronize(c.st));
  *pin = LsqrDev{};
  pin->atol = o->atol;
  pin->btol = o->btol;
  pin->conlim = o->conlim;
  pin->itmax = itmax;
  RFMLS_HIP(c.h, hipMemcpyAsync(c.dst, pin, sizeof(LsqrDev), hipMemcpyHostToDevice, c.st));
  return RFMLS_OK;
}

static rfmls_status poll_done(Ctx& c, int* host_done) {
  int* pin = (int*)((char*)c.h->pinned + 1024);
  RFMLS_HIP(c.h, hipMemcpyAsync(pin, &c.dst->done, sizeof(int), hipMemcpyDeviceToHost, c.st));
  RFMLS_HIP(c.h, hipStreamSynchronize(c.st));
  *host_done = *pin;
  return RFMLS_OK;
}

// One LSQR iteration (Golub-Kahan step, plane rotation, updates of y and w,
// stopping tests), enqueued on c.st; nred = number of partial sums of ||v||^2.
static rfmls_status lsqr_iteration(Ctx& c, int nred) {
  rfmls_handle* h = c.h;
  const int64_t m = c.A->m, n = c.A->n;
  const int* done = &c.dst->done;
  const unsigned vbn = vec_blocks(n), vbm = vec_blocks(m);
  // beta u = A (X v) - alpha u  (or B v - alpha u)
  int nb = 0;
  if (c.Bm) {
    RFMLS_CHECK(bmul(c, c.v, 1.0, &c.dst->alpha, c.u, c.u, c.sqA, done, &nb));
  } else {
    RFMLS_CHECK(tri_apply(h, c.P, 0, c.v, c.z, 0.0, nullptr, nullptr, nullptr, done));
    RFMLS_CHECK(spmv(c, c.A, c.z, 1.0, 1.0, &c.dst->alpha, c.u, c.u, c.sqA, done, &nb));
  }
  hipLaunchKernelGGL(k_normalize, dim3(vbm), dim3(kThreads), 0, c.st, c.u, m, c.sqA, nb,
                     &c.dst->beta, done);
  // alpha v = X^T (A^T u) - beta v  (or B^T u - beta v)
  if (c.Bm) {
    RFMLS_CHECK(btmul(c, c.u, 1.0, &c.dst->beta, c.v, c.v, c.sqB, done, &nred));
  } else {
    RFMLS_CHECK(spmv(c, c.AT, c.u, 1.0, 0.0, nullptr, nullptr, c.q, nullptr, done, nullptr));
    RFMLS_CHECK(tri_apply(h, c.P, 1, c.q, c.v, 1.0, &c.dst->beta, c.v, c.sqB, done));
  }
  hipLaunchKernelGGL(k_normalize, dim3(vbn), dim3(kThreads), 0, c.st, c.v, n, c.sqB, nred,
                     &c.dst->alpha, done);
  hipLaunchKernelGGL(k_lsqr_rotate, dim3(1), dim3(kThreads), 0, c.st, c.dst, c.sqW, (int)vbn);
  hipLaunchKernelGGL(k_lsqr_update, dim3(vbn), dim3(kThreads), 0, c.st, c.dst, c.v, c.w, c.y, n,
                     c.sqY, c.sqW);
  hipLaunchKernelGGL(k_lsqr_check, dim3(1), dim3(kThreads), 0, c.st, c.dst, c.sqY, (int)vbn, 0);
  RFMLS_HIP(h, hipGetLastError());
  return RFMLS_OK;
}

// One LSQR sweep for min ||A X y - rhs||; on return c.y holds y and the state
// is in c.dst.  rhs is an m-vector (device).
static rfmls_status lsqr_sweep(Ctx& c, const double* rhs, const rfmls_opts* o, int64_t itmax) {
  rfmls_handle* h = c.h;
  const int64_t m = c.A->m, n = c.A->n;
  const int* done = &c.dst->done;
  RFMLS_CHECK(upload_state(c, o, itmax));
  const unsigned vbn = vec_blocks(n), vbm = vec_blocks(m);
  // beta_1 u_1 = rhs
  hipLaunchKernelGGL(k_axpby, dim3(vbm), dim3(kThreads), 0, c.st, m, 1.0, (const double*)nullptr,
                     rhs, 0.0, (const double*)nullptr, (const double*)nullptr, c.u,
                     (const int*)nullptr);
  hipLaunchKernelGGL(k_sumsq, dim3(vbm), dim3(kThreads), 0, c.st, c.u, m, c.sqA);
  hipLaunchKernelGGL(k_normalize, dim3(vbm), dim3(kThreads), 0, c.st, c.u, m, c.sqA, (int)vbm,
                     &c.dst->beta, (const int*)nullptr);
  hipLaunchKernelGGL(k_lsqr_start, dim3(1), dim3(1), 0, c.st, c.dst);
  hipLaunchKernelGGL(k_fill, dim3(vbn), dim3(kThreads), 0, c.st, c.y, n, 0.0);
  // alpha_1 v_1 = B^T u_1 = X^T (A^T u_1) (or the explicit B^T u_1)
  int nred = tri_reduce_blocks(n);
  if (c.Bm) {
    RFMLS_CHECK(btmul(c, c.u, 0.0, nullptr, nullptr, c.v, c.sqB, done, &nred));
  } else {
    RFMLS_CHECK(spmv(c, c.AT, c.u, 1.0, 0.0, nullptr, nullptr, c.q, nullptr, done, nullptr));
    RFMLS_CHECK(tri_apply(h, c.P, 1, c.q, c.v, 0.0, nullptr, nullptr, c.sqB, done));
  }
  hipLaunchKernelGGL(k_normalize, dim3(vbn), dim3(kThreads), 0, c.st, c.v, n, c.sqB, nred,
                     &c.dst->alpha, done);
  hipLaunchKernelGGL(k_lsqr_start2, dim3(1), dim3(1), 0, c.st, c.dst);
  // w_1 = v_1 and ||w_1||^2
  hipLaunchKernelGGL(k_axpby, dim3(vbn), dim3(kThreads), 0, c.st, n, 1.0, (const double*)nullptr,
                     c.v, 0.0, (const double*)nullptr, (const double*)nullptr, c.w, done);
  hipLaunchKernelGGL(k_sumsq, dim3(vbn), dim3(kThreads), 0, c.st, c.w, n, c.sqW);
  // alpha_prev for the ||B||_F estimate: alpha_1
  hipLaunchKernelGGL(k_axpby, dim3(1), dim3(1), 0, c.st, (int64_t)1, 1.0, (const double*)nullptr,
                     &c.dst->alpha, 0.0, (const double*)nullptr, (const double*)nullptr,
                     &c.dst->alpha_prev, (const int*)nullptr);
  const int every = o->check_every > 0 ? o->check_every : 8;
  int hd = 0;
  RFMLS_CHECK(poll_done(c, &hd));
  if (c.graph && !h->trace) {
    // the poll interval's launches recorded once per call, then replayed
    if (!c.graph->exec)
      RFMLS_CHECK(capture_graph(h, c.graph, [&]() -> rfmls_status {
        const hipStream_t s0 = c.st;
        c.st = h->stream;
        rfmls_status r = RFMLS_OK;
        for (int k = 0; k < every && r >= 0; ++k) r = lsqr_iteration(c, nred);
        c.st = s0;
        return r;
      }));
    for (int64_t it = 0; it < itmax && !hd; it += every) {
      RFMLS_HIP(h, hipGraphLaunch(c.graph->exec, c.st));
      RFMLS_CHECK(poll_done(c, &hd));
    }
    return RFMLS_OK;
  }
  for (int64_t it = 0; it < itmax && !hd; ++it) {
    RFMLS_CHECK(lsqr_iteration(c, nred));
    if ((it + 1) % every == 0) RFMLS_CHECK(poll_done(c, &hd));
  }
  return RFMLS_OK;
}

// Doubles of device memory one single-right-hand-side solve works in: the
// vectors and partial sums (make_ctx's layout) and the LSQR state after them.
static int64_t ctx_doubles(int64_t m, int64_t n) { return 4 * m + 8 * n + 4 * kSpmvMaxBlocks + 64; }
constexpr int64_t kStateDoubles = (2 * sizeof(LsqrDev) + 255) / 256 * 32;

// Bytes of the column-run descriptors of `rows` matrix rows.
static int64_t runs_bytes(int64_t rows) { return (int64_t)sizeof(int32_t) * rows * (1 + 2 * kMaxRuns); }

// base: device memory of at least ctx_doubles + kStateDoubles doubles followed
// by runs_bytes(m + n) bytes, or null for the handle's workspace
static rfmls_status make_ctx(rfmls_handle* h, const rfmls_csr* A, const rfmls_csr* AT,
                             const rfmls_precond_t* P, Ctx& c, double* base = nullptr) {
  c.h = h;
  c.A = A;
  c.AT = AT;
  c.P = P;
  c.st = h->stream;
  const int64_t m = A->m, n = A->n;
  const size_t nvec = (size_t)ctx_doubles(m, n);
  void* p = base;
  if (!base) RFMLS_CHECK(workspace(h, WS_LSQR_VEC, sizeof(double) * nvec, &p));
  double* d = (double*)p;
  c.u = d;
  d += m;
  c.r = d;
  d += m;
  c.t = d;
  d += m;
  d += m;  // spare m-vector
  c.v = d;
  d += n;
  c.w = d;
  d += n;
  c.y = d;
  d += n;
  c.z = d;
  d += n;
  c.q = d;
  d += n;
  c.xs = d;
  d += n;
  d += 2 * n;  // spare
  c.sqA = d;
  d += kSpmvMaxBlocks;
  c.sqB = d;
  d += kSpmvMaxBlocks;
  c.sqY = d;
  d += kSpmvMaxBlocks;
  c.sqW = d;
  d += kSpmvMaxBlocks;
  c.hn = d;
  void* ps = base ? (void*)(base + nvec) : nullptr;
  if (!base) RFMLS_CHECK(workspace(h, WS_LSQR_SCAL, sizeof(LsqrDev) * 2, &ps));
  c.dst = (LsqrDev*)ps;
  {
    // column runs of A and A^T, after the state in the caller's scratch or in
    // the handle's workspace
    const int64_t ra = A->m, rt = AT ? AT->m : 0;
    void* pr = base ? (void*)(base + nvec + kStateDoubles) : nullptr;
    if (!base) RFMLS_CHECK(workspace(h, WS_LSQR_RUNS, (size_t)runs_bytes(ra + rt), &pr));
    int32_t* q = (int32_t*)pr;
    auto carve = [&](const rfmls_csr* M, int64_t rows, const int32_t** nr, const int32_t** rc, const int32_t** re) {
      int32_t* n0 = q;
      int32_t* c0 = n0 + rows;
      int32_t* e0 = c0 + rows * kMaxRuns;
      q = e0 + rows * kMaxRuns;
      hipLaunchKernelGGL(k_find_runs, dim3(spmv_blocks(rows)), dim3(kThreads), 0, c.st, M->row_ptr, M->col, rows, n0,
                         c0, e0);
      *nr = n0;
      *rc = c0;
      *re = e0;
    };
    if (ra > 0) carve(A, ra, &c.nrunA, &c.rcolA, &c.rendA);
    if (rt > 0) carve(AT, rt, &c.nrunAT, &c.rcolAT, &c.rendAT);
    RFMLS_HIP(h, hipGetLastError());
  }
  return RFMLS_OK;
}

static rfmls_status read_state(Ctx& c, LsqrDev* out) {
  LsqrDev* pin = (LsqrDev*)((char*)c.h->pinned + 2048);
  RFMLS_HIP(c.h, hipMemcpyAsync(pin, c.dst, sizeof(LsqrDev), hipMemcpyDeviceToHost, c.st));
  RFMLS_HIP(c.h, hipStreamSynchronize(c.st));
  *out = *pin;
  return RFMLS_OK;
}

// ||v|| of a device vector into host (reduced on the device, 8 bytes copied
// through the pinned staging buffer)
static rfmls_status host_norm(Ctx& c, const double* v, int64_t len, double* out) {
  const unsigned nb = vec_blocks(len);
  hipLaunchKernelGGL(k_sumsq, dim3(nb), dim3(kThreads), 0, c.st, v, len, c.sqY);
  hipLaunchKernelGGL(k_sqrt_sum, dim3(1), dim3(kThreads), 0, c.st, (const double*)c.sqY, (int)nb, c.hn);
  double* pin = (double*)((char*)c.h->pinned + 3072);
  RFMLS_HIP(c.h, hipMemcpyAsync(pin, c.hn, sizeof(double), hipMemcpyDeviceToHost, c.st));
  RFMLS_HIP(c.h, hipStreamSynchronize(c.st));
  *out = *pin;
  return RFMLS_OK;
}

// One right-hand side at a time; Bm (row-major m x n, or null) is the explicit
// operator B = A R^{-1}.
static rfmls_status solve_impl(rfmls_handle* h, const rfmls_csr* A, const rfmls_csr* AT,
                               const rfmls_precond_t* P, const double* Bm, int64_t ldbm,
                               const double* B, int64_t ldb, int64_t nrhs, double* X, int64_t ldx,
                               double* Rout, int64_t ldr, const rfmls_opts* o, rfmls_info* info,
                               double* base = nullptr) {
  Ctx c;
  RFMLS_CHECK(make_ctx(h, A, AT, P, c, base));
  // the allocation-free variant launches eagerly (instantiating a graph allocates)
  IterGraph graph;
  if (o->graph && !base) c.graph = &graph;
  if (Bm) {
    void* p;
    RFMLS_CHECK(workspace(h, WS_GEMV, sizeof(double) * (size_t)kGemvTSlices * (size_t)A->n, &p));
    c.Bm = Bm;
    c.ldbm = ldbm;
    c.gpart = (double*)p;
  }
  const int64_t m = A->m, n = A->n;
  const int64_t itmax = o->itmax > 0 ? o->itmax : n;
  const unsigned vbn = vec_blocks(n), vbm = vec_blocks(m);
  rfmls_status ret = RFMLS_OK;
  for (int64_t k = 0; k < nrhs; ++k) {
    const double* b = B + k * ldb;
    double* x = X + k * ldx;
    rfmls_info inf{};
    double* rres = c.r;
    // from x = 0 the first sweep takes b itself; from a given x every sweep
    // solves for the correction from the true residual r = b - A x
    const bool warm = o->x_init != 0;
    if (warm) {
      RFMLS_CHECK(host_norm(c, b, m, &inf.normb));
      RFMLS_CHECK(spmv(c, A, x, -1.0, -1.0, nullptr, b, rres, nullptr, nullptr, nullptr));
    }
    for (int sweep = 0; sweep <= o->refine; ++sweep) {
      const bool from_zero = sweep == 0 && !warm;
      const double* rhs = from_zero ? b : rres;
      RFMLS_CHECK(lsqr_sweep(c, rhs, o, itmax));
      LsqrDev s;
      RFMLS_CHECK(read_state(c, &s));
      if (s.istop < 0) return fail(h, RFMLS_E_BREAKDOWN, "non-finite value in LSQR");
      if (sweep == 0) {
        inf.itn_first = s.itn;
        inf.istop = s.istop;
        inf.normr_est = s.normr;
        inf.normar_est = s.normar;
        inf.anorm_est = sqrt(s.anorm2);
        inf.acond_est = s.acond;
        if (!warm) inf.normb = s.bnorm;
        if (s.istop == 7) ret = RFMLS_W_NOCONV;
      }
      inf.itn += s.itn;
      inf.istop_last = s.istop;
      // x (+)= X y
      RFMLS_CHECK(tri_apply(h, P, 0, c.y, from_zero ? x : c.xs, 0.0, nullptr, nullptr, nullptr,
                            nullptr));
      if (!from_zero)
        hipLaunchKernelGGL(k_axpby, dim3(vbn), dim3(kThreads), 0, c.st, n, 1.0,
                           (const double*)nullptr, (const double*)x, 1.0, (const double*)nullptr,
                           (const double*)c.xs, x, (const int*)nullptr);
      // r = b - A x
      RFMLS_CHECK(spmv(c, A, x, -1.0, -1.0, nullptr, b, rres, nullptr, nullptr, nullptr));
      if (s.itn == 0) break;
    }
    RFMLS_CHECK(host_norm(c, rres, m, &inf.normr));
    RFMLS_CHECK(spmv(c, AT, rres, 1.0, 0.0, nullptr, nullptr, c.q, nullptr, nullptr, nullptr));
    RFMLS_CHECK(host_norm(c, c.q, n, &inf.normar));
    if (Rout)
      hipLaunchKernelGGL(k_axpby, dim3(vbm), dim3(kThreads), 0, c.st, m, 1.0, (const double*)nullptr,
                         (const double*)rres, 0.0, (const double*)nullptr, (const double*)nullptr,
                         Rout + k * ldr, (const int*)nullptr);
    if (info) info[k] = inf;
  }
  RFMLS_HIP(h, hipStreamSynchronize(c.st));
  return ret;
}

rfmls_status run_solve(rfmls_handle* h, const rfmls_csr* A, const rfmls_csr* AT,
                       const rfmls_precond_t* P, const double* B, int64_t ldb, int64_t nrhs,
                       double* X, int64_t ldx, double* Rout, int64_t ldr, const rfmls_opts* o,
                       rfmls_info* info) {
  return solve_impl(h, A, AT, P, nullptr, 0, B, ldb, nrhs, X, ldx, Rout, ldr, o, info);
}

// ---------------------------------------------------------------------------
// Allocation-free variant of the single-right-hand-side solve: its device
// scratch (the vectors, partial sums and LSQR state of make_ctx) lives in one
// file-scope array.  Each device holds its own copy of the array (allocated
// when the library's code object is loaded on that device, kept until the
// process ends); host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device, never through the
// array's name, which on the host is only a stand-in for the symbol.
// ---------------------------------------------------------------------------
namespace noalloc {
constexpr int64_t kScratchDoubles = (int64_t)1 << 22;  // 32 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxDevices = 64;
static std::mutex mu;
static double* dev_ptr[kMaxDevices] = {};
}  // namespace noalloc

// Called by rfmls_create with h->device current: record this device's
// address of the scratch array (once per device).
rfmls_status noalloc_scratch_init(rfmls_handle* h) {
  std::lock_guard<std::mutex> lk(noalloc::mu);
  if (h->device < 0 || h->device >= noalloc::kMaxDevices)
    return fail(h, RFMLS_E_ARG, "device %d out of range for the allocation-free scratch", h->device);
  if (noalloc::dev_ptr[h->device]) return RFMLS_OK;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc::scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return fail(h, RFMLS_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", h->device,
                hipGetErrorString(e));
  }
  noalloc::dev_ptr[h->device] = (double*)p;
  return RFMLS_OK;
}

int64_t noalloc_scratch_bytes() { return noalloc::kScratchDoubles * (int64_t)sizeof(double); }

int64_t noalloc_needed_bytes(int64_t m, int64_t n) {
  return (ctx_doubles(m, n) + kStateDoubles) * (int64_t)sizeof(double) + runs_bytes(m + n);
}

rfmls_status run_solve_noalloc(rfmls_handle* h, const rfmls_csr* A, const rfmls_csr* AT,
                               const rfmls_precond_t* P, const double* B, int64_t ldb, int64_t nrhs,
                               double* X, int64_t ldx, double* Rout, int64_t ldr, const rfmls_opts* o,
                               rfmls_info* info) {
  double* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(noalloc::mu);
    base = (h->device >= 0 && h->device < noalloc::kMaxDevices) ? noalloc::dev_ptr[h->device] : nullptr;
  }
  if (!base) return fail(h, RFMLS_E_HIP, "rfmls_solve_noalloc: no scratch address for device %d", h->device);
  if (noalloc_needed_bytes(A->m, A->n) > noalloc_scratch_bytes())
    return fail(h, RFMLS_E_ARG, "rfmls_solve_noalloc: m = %lld, n = %lld need %lld bytes of scratch, above the "
                "%lld-byte limit", (long long)A->m, (long long)A->n, (long long)noalloc_needed_bytes(A->m, A->n),
                (long long)noalloc_scratch_bytes());
  return solve_impl(h, A, AT, P, nullptr, 0, B, ldb, nrhs, X, ldx, Rout, ldr, o, info, base);
}

rfmls_status run_solve_explicit(rfmls_handle* h, const rfmls_csr* A, const rfmls_csr* AT,
                                const rfmls_precond_t* P, const double* Bm, int64_t ldbm,
                                const double* B, int64_t ldb, int64_t nrhs, double* X, int64_t ldx,
                                double* Rout, int64_t ldr, const rfmls_opts* o, rfmls_info* info) {
  return solve_impl(h, A, AT, P, Bm, ldbm, B, ldb, nrhs, X, ldx, Rout, ldr, o, info);
}

// Backward: LSQR on the consistent system B^T lam = c (c = X^T g), operator
// M = B^T (n x m), tracking lam = B z through the shadow vectors vt, wt (v = B vt).
rfmls_status run_backward(rfmls_handle* h, const rfmls_csr* A, const rfmls_csr* AT,
                          const rfmls_precond_t* P, const double* Xs, int64_t ldx,
                          const double* Rres, int64_t ldr, const double* G, int64_t ldg,
                          int64_t nrhs, double* dB, int64_t lddb, double* dAval,
                          const rfmls_opts* o, rfmls_info* info) {
  Ctx c;
  RFMLS_CHECK(make_ctx(h, A, AT, P, c));
  const int64_t m = A->m, n = A->n;
  const int64_t itmax = o->itmax > 0 ? o->itmax : m;
  const unsigned vbn = vec_blocks(n), vbm = vec_blocks(m);
  const int nred = tri_reduce_blocks(n);
  // roles: un = u (n-vector), vm = v (m-vector), vt/wt/zz shadows (n-vectors)
  double* un = c.z;   // n
  double* vm = c.t;   // m
  double* vt = c.w;   // n
  double* wt = c.q;   // n
  double* zz = c.y;   // n
  double* tmpn = c.xs;  // n
  double* lam = c.r;  // m
  const int* done = &c.dst->done;
  rfmls_status ret = RFMLS_OK;
  IterGraph graph;  // one capture serves every right-hand side (same buffers)
  for (int64_t k = 0; k < nrhs; ++k) {
    RFMLS_CHECK(upload_state(c, o, itmax));
    // beta_1 u_1 = c = X^T g
    RFMLS_CHECK(tri_apply(h, P, 1, G + k * ldg, un, 0.0, nullptr, nullptr, c.sqB, nullptr));
    hipLaunchKernelGGL(k_normalize, dim3(vbn), dim3(kThreads), 0, c.st, un, n, c.sqB, nred,
                       &c.dst->beta, (const int*)nullptr);
    hipLaunchKernelGGL(k_lsqr_start, dim3(1), dim3(1), 0, c.st, c.dst);
    hipLaunchKernelGGL(k_fill, dim3(vbn), dim3(kThreads), 0, c.st, zz, n, 0.0);
    // alpha_1 v_1 = M^T u_1 = A (X u_1);  vt_1 = u_1 / alpha_1
    RFMLS_CHECK(tri_apply(h, P, 0, un, tmpn, 0.0, nullptr, nullptr, nullptr, done));
    int nb = 0;
    RFMLS_CHECK(spmv(c, A, tmpn, 1.0, 0.0, nullptr, nullptr, vm, c.sqA, done, &nb));
    hipLaunchKernelGGL(k_normalize, dim3(vbm), dim3(kThreads), 0, c.st, vm, m, c.sqA, nb,
                       &c.dst->alpha, done);
    hipLaunchKernelGGL(k_lsqr_start2, dim3(1), dim3(1), 0, c.st, c.dst);
    hipLaunchKernelGGL(k_recip_scale, dim3(vbn), dim3(kThreads), 0, c.st, un, 0.0, (const double*)nullptr,
                       (const double*)nullptr, &c.dst->alpha, vt, n, done);
    hipLaunchKernelGGL(k_axpby, dim3(vbn), dim3(kThreads), 0, c.st, n, 1.0, (const double*)nullptr,
                       (const double*)vt, 0.0, (const double*)nullptr, (const double*)nullptr, wt,
                       done);
    hipLaunchKernelGGL(k_sumsq, dim3(vbn), dim3(kThreads), 0, c.st, wt, n, c.sqW);
    hipLaunchKernelGGL(k_axpby, dim3(1), dim3(1), 0, c.st, (int64_t)1, 1.0, (const double*)nullptr,
                       &c.dst->alpha, 0.0, (const double*)nullptr, (const double*)nullptr,
                       &c.dst->alpha_prev, (const int*)nullptr);
    const int every = o->check_every > 0 ? o->check_every : 8;
    int hd = 0;
    RFMLS_CHECK(poll_done(c, &hd));
    auto iteration = [&]() -> rfmls_status {
      // beta u = X^T (A^T v) - alpha u
      RFMLS_CHECK(spmv(c, AT, vm, 1.0, 0.0, nullptr, nullptr, tmpn, nullptr, done, nullptr));
      RFMLS_CHECK(tri_apply(h, P, 1, tmpn, un, 1.0, &c.dst->alpha, un, c.sqB, done));
      hipLaunchKernelGGL(k_normalize, dim3(vbn), dim3(kThreads), 0, c.st, un, n, c.sqB, nred,
                         &c.dst->beta, done);
      // alpha v = A (X u) - beta v;  vt = (u - beta vt) / alpha
      RFMLS_CHECK(tri_apply(h, P, 0, un, tmpn, 0.0, nullptr, nullptr, nullptr, done));
      RFMLS_CHECK(spmv(c, A, tmpn, 1.0, 1.0, &c.dst->beta, vm, vm, c.sqA, done, &nb));
      hipLaunchKernelGGL(k_normalize, dim3(vbm), dim3(kThreads), 0, c.st, vm, m, c.sqA, nb,
                         &c.dst->alpha, done);
      hipLaunchKernelGGL(k_recip_scale, dim3(vbn), dim3(kThreads), 0, c.st, un, 1.0,
                         (const double*)&c.dst->beta, (const double*)vt, &c.dst->alpha, vt, n, done);
      hipLaunchKernelGGL(k_lsqr_rotate, dim3(1), dim3(kThreads), 0, c.st, c.dst, c.sqW, (int)vbn);
      hipLaunchKernelGGL(k_lsqr_update, dim3(vbn), dim3(kThreads), 0, c.st, c.dst, vt, wt, zz, n,
                         c.sqY, c.sqW);
      hipLaunchKernelGGL(k_lsqr_check, dim3(1), dim3(kThreads), 0, c.st, c.dst, c.sqY, (int)vbn, 1);
      RFMLS_HIP(h, hipGetLastError());
      return RFMLS_OK;
    };
    if (o->graph && !h->trace) {
      if (!graph.exec)
        RFMLS_CHECK(capture_graph(h, &graph, [&]() -> rfmls_status {
          const hipStream_t s0 = c.st;
          c.st = h->stream;
          rfmls_status r = RFMLS_OK;
          for (int q = 0; q < every && r >= 0; ++q) r = iteration();
          c.st = s0;
          return r;
        }));
      for (int64_t it = 0; it < itmax && !hd; it += every) {
        RFMLS_HIP(h, hipGraphLaunch(graph.exec, c.st));
        RFMLS_CHECK(poll_done(c, &hd));
      }
    } else {
      for (int64_t it = 0; it < itmax && !hd; ++it) {
        RFMLS_CHECK(iteration());
        if ((it + 1) % every == 0) RFMLS_CHECK(poll_done(c, &hd));
      }
    }
    LsqrDev s;
    RFMLS_CHECK(read_state(c, &s));
    if (s.istop < 0) return fail(h, RFMLS_E_BREAKDOWN, "non-finite value in backward LSQR");
    if (s.istop == 7) ret = RFMLS_W_NOCONV;
    if (info) {
      rfmls_info inf{};
      inf.itn = inf.itn_first = s.itn;
      inf.istop = inf.istop_last = s.istop;
      inf.normr_est = s.normr;
      inf.normb = s.bnorm;
      info[k] = inf;
    }
    // w = X z (into tmpn), lam = A w
    RFMLS_CHECK(tri_apply(h, P, 0, zz, tmpn, 0.0, nullptr, nullptr, nullptr, nullptr));
    RFMLS_CHECK(spmv(c, A, tmpn, 1.0, 0.0, nullptr, nullptr, lam, nullptr, nullptr, nullptr));
    if (dB)
      hipLaunchKernelGGL(k_axpby, dim3(vbm), dim3(kThreads), 0, c.st, m, 1.0, (const double*)nullptr,
                         (const double*)lam, 0.0, (const double*)nullptr, (const double*)nullptr,
                         dB + k * lddb, (const int*)nullptr);
    if (dAval)
      hipLaunchKernelGGL(k_pattern_grad, dim3(spmv_blocks(m)), dim3(kThreads), 0, c.st, A->row_ptr,
                         A->col, m, Rres + k * ldr, (const double*)tmpn, (const double*)lam,
                         Xs + k * ldx, dAval, k > 0 ? 1 : 0);
    RFMLS_HIP(h, hipGetLastError());
  }
  RFMLS_HIP(h, hipStreamSynchronize(c.st));
  return ret;
}

}  // namespace rfmls
