// Blocked Householder QR of the sketch SA (s x n, row-major, in place):
// Alg. 1 step 3.  Only R is needed; Q is never formed.
//
// For each panel of nb columns starting at k0 (M = s - k0 rows):
//   1. k_qr_panel   unblocked Householder on the s x nb panel.  The panel is
//                   spread over G co-resident workgroups (rows held in LDS);
//                   every column needs one grid-wide reduction: the partial
//                   sums  sigma = sum_{i>j} a_ij^2  and  d_c = sum_{i>j} a_ij a_ic
//                   plus the pivot row, after which every workgroup forms the
//                   same reflector (LAPACK dlarfg convention: beta = -sign(alpha)
//                   ||(alpha, x)||, tau = (beta - alpha) / beta, v = [1; x/(alpha-beta)])
//                   and applies it to its rows.
//   2. k_gemm       W_z = V^T [V | C] over row slices z (split-K partials)
//   3. k_qr_buildT  sum the V^T V partials and build the compact-WY factor T
//                   (I - V T V^T = H_1 ... H_nb; LAPACK dlarft, forward, columnwise)
//   4. k_qr_wp      W' = T^T sum_z W_z for the trailing columns
//   5. k_gemm       C <- C - V W'
// All reductions run in a fixed order, so the factorisation is deterministic.
#include "common.h"
#include "gemm.h"

namespace rfmls {
namespace {

constexpr int kPanelThreads = 256;
constexpr int kMaxNb = 64;
constexpr int kPartStride = 2 * kMaxNb;  // per slot: [c] sums (c in [j, nb)), [64 + c] pivot row

__device__ __forceinline__ bool grid_barrier(unsigned* counter, unsigned target, int* err) {
  __syncthreads();
  __shared__ int ok;
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    int spins = 0;
    ok = 1;
    while (__hip_atomic_load(counter, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1 << 26)) {
        ok = 0;
        atomicExch(err, 1);
        break;
      }
    }
  }
  __syncthreads();
  return ok != 0;
}

// part layout: part[slot][c][g], c in [0, 2*kMaxNb), g in [0, G)
template <typename T>
__global__ void __launch_bounds__(kPanelThreads)
    k_qr_panel(T* __restrict__ P, int64_t ld, int64_t M, int nb, int rpw, T* __restrict__ tau,
               double* __restrict__ part, unsigned* __restrict__ bar, int* __restrict__ err) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* tile = reinterpret_cast<T*>(smem_raw);          // rpw x nb
  __shared__ double red[2 * kMaxNb];                 // reduced sums / pivot row
  __shared__ double grp[4][kMaxNb];                  // per row-group partials
  const int G = gridDim.x;
  const int g = blockIdx.x;
  const int tid = threadIdx.x;
  const int c = tid & 63;    // column handled by this thread
  const int rg = tid >> 6;   // row group 0..3
  const int64_t r0 = (int64_t)g * rpw;
  const int nr = (int)(M - r0 < rpw ? (M - r0 > 0 ? M - r0 : 0) : rpw);

  for (int e = tid; e < nr * nb; e += kPanelThreads) {
    const int i = e / nb, cc = e % nb;
    tile[e] = P[(r0 + i) * ld + cc];
  }
  __syncthreads();

  for (int j = 0; j < nb; ++j) {
    const int slot = j & 1;
    double* pw = part + (int64_t)slot * kPartStride * G;
    // ---- local partials over rows i > j (global panel row index) ----
    double s = 0.0;
    if (c >= j && c < nb) {
      for (int i = rg; i < nr; i += 4) {
        const int64_t gi = r0 + i;
        if (gi > j) s += (double)tile[i * nb + j] * (double)tile[i * nb + c];
      }
    }
    grp[rg][c] = s;
    __syncthreads();
    if (tid < 64 && c >= j && c < nb) {
      const double t = (grp[0][c] + grp[1][c]) + (grp[2][c] + grp[3][c]);
      pw[(int64_t)c * G + g] = t;
    }
    // pivot row j lives in block j / rpw
    const bool own_pivot = (j >= r0) && (j < r0 + nr);
    if (own_pivot && tid < 64 && c >= j && c < nb)
      pw[(int64_t)(kMaxNb + c) * G + g] = (double)tile[(j - r0) * nb + c];
    if (!grid_barrier(bar, (unsigned)((j + 1) * G), err)) return;
    // ---- reduce: wave w handles columns c = w, w+4, ... (coalesced over g) ----
    {
      const int lane = tid & 63;
      const int w = tid >> 6;
      for (int cc = j + w; cc < nb; cc += 4) {
        double t = 0.0;
        for (int gg = lane; gg < G; gg += 64) t += pw[(int64_t)cc * G + gg];
        t = wave_sum(t);
        if (lane == 0) red[cc] = t;
      }
      const int owner = j / rpw;
      if (tid < 64 && c >= j && c < nb) red[kMaxNb + c] = pw[(int64_t)(kMaxNb + c) * G + owner];
    }
    __syncthreads();
    // ---- reflector (identical in every block) ----
    const double alpha = red[kMaxNb + j];
    const double sigma = red[j];
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
    // ---- apply H_j to this block's rows i >= j, columns c > j ----
    if (c > j && c < nb && tj != 0.0) {
      const double wc = red[kMaxNb + c] + scal * red[c];
      const double f = tj * wc;
      for (int i = rg; i < nr; i += 4) {
        const int64_t gi = r0 + i;
        if (gi > j) {
          const double vi = scal * (double)tile[i * nb + j];
          tile[i * nb + c] = (T)((double)tile[i * nb + c] - vi * f);
        } else if (gi == j) {
          tile[i * nb + c] = (T)((double)tile[i * nb + c] - f);
        }
      }
    }
    __syncthreads();
    if (c == j) {
      for (int i = rg; i < nr; i += 4) {
        const int64_t gi = r0 + i;
        if (gi > j) tile[i * nb + j] = (T)(scal * (double)tile[i * nb + j]);
        else if (gi == j) tile[i * nb + j] = (T)beta;
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < nr * nb; e += kPanelThreads) {
    const int i = e / nb, cc = e % nb;
    P[(r0 + i) * ld + cc] = tile[e];
  }
}

// Build T (nb x nb upper triangular, row-major) from tau and V^T V = sum of
// nsplit partial slices Wz (each nb x ldw, leading nb columns hold V^T V).
template <typename T>
__global__ void __launch_bounds__(256)
    k_qr_buildT(const T* __restrict__ Wz, int64_t zstride, int nsplit, int64_t ldw, int nb,
                const T* __restrict__ tau, T* __restrict__ Tout) {
  __shared__ double Gm[kMaxNb][kMaxNb + 1];
  __shared__ double Tm[kMaxNb][kMaxNb + 1];
  __shared__ double tv[kMaxNb];
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * nb; e += 256) {
    const int i = e / nb, k = e % nb;
    double sacc = 0.0;
    for (int z = 0; z < nsplit; ++z) sacc += (double)Wz[(int64_t)z * zstride + (int64_t)i * ldw + k];
    Gm[i][k] = sacc;
    Tm[i][k] = 0.0;
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    const double tj = (double)tau[j];
    // t = T[0:j,0:j] * G[0:j, j]
    if (tid < j) {
      double a = 0.0;
      for (int k = tid; k < j; ++k) a += Tm[tid][k] * Gm[k][j];
      tv[tid] = a;
    }
    __syncthreads();
    if (tid < j) Tm[tid][j] = -tj * tv[tid];
    if (tid == 0) Tm[j][j] = tj;
    __syncthreads();
  }
  for (int e = tid; e < nb * nb; e += 256) Tout[e] = (T)Tm[e / nb][e % nb];
}

// W'[:, cols] = T^T * sum_z Wz[:, nb + cols], one block per 64 columns.
template <typename T>
__global__ void __launch_bounds__(256)
    k_qr_wp(const T* __restrict__ Wz, int64_t zstride, int nsplit, int64_t ldw, int nb, int64_t N,
            const T* __restrict__ Tm, T* __restrict__ Wp, int64_t ldwp) {
  __shared__ double Ws[kMaxNb][64 + 1];
  __shared__ double Ts[kMaxNb][kMaxNb + 1];
  const int tid = threadIdx.x;
  const int64_t c0 = (int64_t)blockIdx.x * 64;
  for (int e = tid; e < nb * nb; e += 256) Ts[e / nb][e % nb] = (double)Tm[e];
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
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

template <typename T>
rfmls_status qr_impl(rfmls_handle* h, int64_t s, int64_t n, T* SA, int64_t ld) {
  hipStream_t st = h->stream;
  const int nbmax = kMaxNb;
  const int64_t ksplit_rows = 4096;
  const int64_t max_split = (s + ksplit_rows - 1) / ksplit_rows;
  void *p_tau, *p_part, *p_w, *p_wp, *p_t;
  RFMLS_CHECK(workspace(h, WS_QR_TAU, sizeof(T) * nbmax, &p_tau));
  RFMLS_CHECK(workspace(h, WS_QR_PART, sizeof(double) * 2 * kPartStride * 1024, &p_part));
  RFMLS_CHECK(workspace(h, WS_QR_W, sizeof(T) * (size_t)max_split * nbmax * (size_t)n, &p_w));
  RFMLS_CHECK(workspace(h, WS_QR_WP, sizeof(T) * (size_t)nbmax * (size_t)n, &p_wp));
  RFMLS_CHECK(workspace(h, WS_QR_T, sizeof(T) * nbmax * nbmax, &p_t));
  T* tau = (T*)p_tau;
  T* W = (T*)p_w;
  T* Wp = (T*)p_wp;
  T* Tm = (T*)p_t;
  const size_t lds_budget = 150 * 1024;
  for (int64_t k0 = 0; k0 < n; k0 += nbmax) {
    const int jb = (int)(n - k0 < nbmax ? n - k0 : nbmax);
    const int64_t M = s - k0;
    // rows per block: at least 64, as many blocks as CUs allow, LDS-limited
    int64_t G = h->num_cus;
    int64_t rpw = (M + G - 1) / G;
    if (rpw < 64) {
      rpw = 64;
      G = (M + rpw - 1) / rpw;
    }
    if ((size_t)rpw * jb * sizeof(T) > lds_budget)
      return fail(h, RFMLS_E_ARG, "QR panel of %lld rows does not fit the co-resident LDS budget",
                  (long long)M);
    T* P = SA + k0 * ld + k0;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, h->barrier, 1);
    const size_t lds = (size_t)rpw * jb * sizeof(T);
    void* args[] = {(void*)&P, (void*)&ld, (void*)&M, (void*)&jb, (void*)&rpw, (void*)&tau,
                    (void*)&p_part, (void*)&h->barrier, (void*)&h->dev_flags};
    int rpw_i = (int)rpw;
    args[4] = (void*)&rpw_i;
    RFMLS_HIP(h, hipFuncSetAttribute((const void*)k_qr_panel<T>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    {
    // Householder on an M x jb panel: sum_j 4 (M - j)(jb - j) flops; panel read and written once
    const double pf = 4.0 * (double)M * jb * (jb + 1) / 2.0;
    Trace tr(h, "qr_panel", 2.0 * sizeof(T) * (double)M * jb, pf);
    RFMLS_HIP(h, hipLaunchCooperativeKernel((const void*)k_qr_panel<T>, dim3((unsigned)G),
                                            dim3(kPanelThreads), args, (unsigned)lds, st));
    }
    const int64_t ntr = n - k0 - jb;  // trailing columns
    if (ntr <= 0) continue;
    const int64_t ncols = n - k0;     // [V | C]
    const int64_t nsplit = (M + ksplit_rows - 1) / ksplit_rows;
    GemmArgs<T> g1;
    g1.M = jb;
    g1.N = ncols;
    g1.K = M;
    g1.A = P;
    g1.lda = ld;
    g1.transA = 1;
    g1.a_vmask = 1;
    g1.B = P;
    g1.ldb = ld;
    g1.b_vcols = jb;
    g1.C = W;
    g1.ldc = ncols;
    g1.alpha = T(1);
    g1.beta = T(0);
    g1.ksplit = ksplit_rows;
    g1.c_zstride = (int64_t)jb * ncols;
    {
      Trace tr(h, "qr_gemm_VtC", sizeof(T) * ((double)M * ncols + (double)nsplit * jb * ncols),
               2.0 * (double)jb * ncols * M);
      RFMLS_HIP(h, gemm<T>(g1, st));
    }
    {
    Trace tr(h, "qr_buildT_Wp", sizeof(T) * (double)(nsplit + 1) * jb * ncols, 2.0 * (double)jb * jb * ntr);
    hipLaunchKernelGGL(k_qr_buildT<T>, dim3(1), dim3(256), 0, st, W, (int64_t)jb * ncols,
                       (int)nsplit, ncols, jb, tau, Tm);
    hipLaunchKernelGGL(k_qr_wp<T>, dim3(ceil_div(ntr, 64)), dim3(256), 0, st, W,
                       (int64_t)jb * ncols, (int)nsplit, ncols, jb, ntr, Tm, Wp, ntr);
    }
    GemmArgs<T> g2;
    g2.M = M;
    g2.N = ntr;
    g2.K = jb;
    g2.A = P;
    g2.lda = ld;
    g2.transA = 0;
    g2.a_vmask = 1;
    g2.B = Wp;
    g2.ldb = ntr;
    g2.C = P + jb;
    g2.ldc = ld;
    g2.alpha = T(-1);
    g2.beta = T(1);
    {
      Trace tr(h, "qr_gemm_update", sizeof(T) * (2.0 * (double)M * ntr + (double)M * jb + (double)jb * ntr),
               2.0 * (double)M * ntr * jb);
      RFMLS_HIP(h, gemm<T>(g2, st));
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
