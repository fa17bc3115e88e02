// Count sketch SA = Phi D A (Def. 2.3): hash/sign generation, a deterministic
// bucket sort of the rows of A by h(i), and the segmented sum that writes the
// dense row-major SA.  Integer work is bit-exact; each element of SA is summed
// in float64 from +0 over its bucket's rows in ascending row order.
#include "common.h"

namespace rfmls {
namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kSignSalt = 0x5555555555555555ull;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void k_hash_sign(int64_t m, uint64_t s, uint64_t seed, int32_t* __restrict__ hash,
                            int8_t* __restrict__ sign) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const uint64_t k = (uint64_t)i + 1u;
  const uint64_t xh = mix64(seed + k * kGamma);
  const uint64_t xs = mix64((seed ^ kSignSalt) + k * kGamma);
  hash[i] = (int32_t)(((xh >> 32) * s) >> 32);
  sign[i] = (xs >> 63) ? (int8_t)-1 : (int8_t)1;
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_count(const int32_t* __restrict__ key, int64_t m, int32_t* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) atomicAdd(&count[key[i]], 1);
}

// Exclusive scan of count[0..n) into ptr[0..n] (ptr[n] = total), one block of
// 1024 threads, tiles of 1024*8 elements with a running carry.
__global__ void __launch_bounds__(1024) k_scan(const int32_t* __restrict__ count, int64_t n,
                                                int64_t* __restrict__ ptr) {
  __shared__ int64_t wsum[16];
  __shared__ int64_t carry_s;
  constexpr int kPer = 8;
  const int tid = threadIdx.x;
  if (tid == 0) carry_s = 0;
  __syncthreads();
  for (int64_t base = 0; base < n; base += 1024 * kPer) {
    int64_t loc[kPer];
    int64_t tsum = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int64_t idx = base + (int64_t)tid * kPer + k;
      loc[k] = idx < n ? count[idx] : 0;
      tsum += loc[k];
    }
    // inclusive scan of tsum across the block (wave scan then wave offsets)
    int64_t x = tsum;
    const int lane = tid & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[tid >> 6] = x;
    __syncthreads();
    int64_t woff = 0;
    for (int w = 0; w < (tid >> 6); ++w) woff += wsum[w];
    const int64_t carry = carry_s;
    int64_t run = carry + woff + x - tsum;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int64_t idx = base + (int64_t)tid * kPer + k;
      if (idx < n) ptr[idx] = run;
      run += loc[k];
    }
    __syncthreads();
    if (tid == 1023) carry_s = carry + woff + x;
    __syncthreads();
  }
  if (tid == 0) ptr[n] = carry_s;
}

__global__ void k_copy_ptr_i32(const int64_t* __restrict__ ptr, int64_t n, int32_t* __restrict__ cur) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) cur[i] = (int32_t)ptr[i];
}

__global__ void k_scatter_rows(const int32_t* __restrict__ key, int64_t m, int32_t* __restrict__ cur,
                               int32_t* __restrict__ perm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) perm[atomicAdd(&cur[key[i]], 1)] = (int32_t)i;
}

// Sort every bucket's row list ascending.  Buckets up to kSmall rows are sorted
// by one thread (insertion sort); a larger bucket is ranked by the whole block
// (rank = number of smaller entries; entries are distinct row indices).
constexpr int kSmallBucket = 64;
__global__ void __launch_bounds__(256) k_sort_buckets(const int64_t* __restrict__ ptr, int64_t s,
                                                      int32_t* __restrict__ perm,
                                                      int32_t* __restrict__ tmp) {
  const int64_t b0 = (int64_t)blockIdx.x * blockDim.x;
  const int64_t b = b0 + threadIdx.x;
  if (b < s) {
    const int64_t lo = ptr[b], hi = ptr[b + 1];
    if (hi - lo <= kSmallBucket) {
      for (int64_t i = lo + 1; i < hi; ++i) {
        const int32_t v = perm[i];
        int64_t j = i - 1;
        while (j >= lo && perm[j] > v) {
          perm[j + 1] = perm[j];
          --j;
        }
        perm[j + 1] = v;
      }
    }
  }
  const int64_t bend = b0 + blockDim.x < s ? b0 + blockDim.x : s;
  for (int64_t bb = b0; bb < bend; ++bb) {
    const int64_t lo = ptr[bb], hi = ptr[bb + 1];
    if (hi - lo <= kSmallBucket) continue;
    __syncthreads();
    for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
      const int32_t v = perm[e];
      int64_t r = 0;
      for (int64_t f = lo; f < hi; ++f) r += perm[f] < v;
      tmp[lo + r] = v;
    }
    __syncthreads();
    for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) perm[e] = tmp[e];
  }
}

// One block per sketch row j.  The bucket's rows (columns ascending within a
// row) each cover one contiguous column span; the spans, merged in order of
// their first column, map the row's touched columns onto a compact LDS window
// (at most kWin doubles).  Zeros go out first for every 16-byte segment clear
// of the window, the bucket's rows are then added into the window in ascending
// row order (a barrier between rows), and the window's segments are stored:
// the dense row is written once, with 16-byte non-temporal stores, and A's
// entries are read once.  A bucket of more than kMaxBucketRows rows or a window
// wider than kWin takes the chunked path: chunks of kWin columns, every row of
// the bucket visited per chunk.  Either way every element is summed in float64
// from +0 over the bucket's rows in ascending row order.
constexpr int kSketchThreads = 256;
constexpr int kWin = 2048;
constexpr int kMaxBucketRows = 64;

template <typename TOut>
struct SketchVec;
template <>
struct SketchVec<double> {
  static constexpr int V = 2;
  typedef double vec __attribute__((ext_vector_type(2)));
};
template <>
struct SketchVec<float> {
  static constexpr int V = 4;
  typedef float vec __attribute__((ext_vector_type(4)));
};

// Vec: the row start is 16-byte aligned (SA and ld suit 16-byte stores)
template <typename TOut, bool Vec>
__global__ void __launch_bounds__(kSketchThreads)
    k_sketch_rows(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                  const double* __restrict__ val, const int8_t* __restrict__ sign,
                  const int64_t* __restrict__ bptr, const int32_t* __restrict__ perm, int64_t n,
                  TOut* __restrict__ SA, int64_t ld) {
  constexpr int V = Vec ? SketchVec<TOut>::V : 1;
  typedef typename SketchVec<TOut>::vec vec_t;
  __shared__ double acc[kWin];
  __shared__ int32_t sp0[kMaxBucketRows], sp1[kMaxBucketRows];
  __shared__ int32_t ist[kMaxBucketRows], ien[kMaxBucketRows], ioff[kMaxBucketRows];
  __shared__ int nint_s;
  const int t = threadIdx.x;
  const int64_t j = blockIdx.x;
  const int64_t blo = bptr[j], bhi = bptr[j + 1];
  const int64_t nb = bhi - blo;
  TOut* out = SA + j * ld;
  int nint = -1;  // -1: chunked path
  if (nb <= kMaxBucketRows) {
    if (t < nb) {
      const int32_t i = perm[blo + t];
      const int64_t lo = row_ptr[i], hi = row_ptr[i + 1];
      sp0[t] = hi > lo ? col[lo] : 1;  // an empty row: an empty span
      sp1[t] = hi > lo ? col[hi - 1] : 0;
    }
    __syncthreads();
    if (t == 0) {
      // sort the spans by first column (insertion sort; a handful of rows), merge
      for (int a = 1; a < nb; ++a) {
        const int32_t x0 = sp0[a], x1 = sp1[a];
        int b2 = a - 1;
        while (b2 >= 0 && sp0[b2] > x0) {
          sp0[b2 + 1] = sp0[b2];
          sp1[b2 + 1] = sp1[b2];
          --b2;
        }
        sp0[b2 + 1] = x0;
        sp1[b2 + 1] = x1;
      }
      int k = 0, total = 0;
      for (int a = 0; a < nb; ++a) {
        if (sp1[a] < sp0[a]) continue;  // empty
        if (k > 0 && sp0[a] <= ien[k - 1] + 1) {
          if (sp1[a] > ien[k - 1]) {
            total += sp1[a] - ien[k - 1];
            ien[k - 1] = sp1[a];
          }
        } else {
          ist[k] = sp0[a];
          ien[k] = sp1[a];
          ioff[k] = total;
          total += sp1[a] - sp0[a] + 1;
          ++k;
        }
      }
      nint_s = total <= kWin ? k : -1;
    }
    __syncthreads();
    nint = nint_s;
  }
  if (nint >= 0) {
    // window position of column c, or -1
    auto wpos = [&](int64_t c) -> int {
      for (int k = 0; k < nint; ++k)
        if (c >= ist[k] && c <= ien[k]) return ioff[k] + (int)(c - ist[k]);
      return -1;
    };
    auto touches = [&](int64_t c0) {
      for (int k = 0; k < nint; ++k)
        if (c0 <= ien[k] && c0 + V - 1 >= ist[k]) return true;
      return false;
    };
    const int64_t nseg = n / V;
    // zeros for the segments clear of the window (no wait on anything below)
    for (int64_t g = t; g < nseg; g += kSketchThreads) {
      const int64_t c0 = g * V;
      if (touches(c0)) continue;
      if constexpr (Vec) {
        __builtin_nontemporal_store(vec_t{}, (vec_t*)(out + c0));
      } else {
        __builtin_nontemporal_store((TOut)0, out + c0);
      }
    }
    const int wlen = nint > 0 ? ioff[nint - 1] + ien[nint - 1] - ist[nint - 1] + 1 : 0;
    for (int w = t; w < wlen; w += kSketchThreads) acc[w] = 0.0;
    __syncthreads();
    for (int64_t q = blo; q < bhi; ++q) {
      const int32_t i = perm[q];
      const double sg = (double)sign[i];
      const int64_t lo = row_ptr[i], hi = row_ptr[i + 1];
      for (int64_t e = lo + t; e < hi; e += kSketchThreads) {
        // a column outside the row's span (a row against the ascending-column
        // contract) is dropped rather than written outside the window
        const int pw = wpos(col[e]);
        if (pw >= 0) acc[pw] += sg * val[e];
      }
      __syncthreads();
    }
    // the window's segments (a segment across two intervals is written twice, alike)
    for (int k = 0; k < nint; ++k) {
      const int64_t g0 = ist[k] / V, g1 = ien[k] / V < nseg ? ien[k] / V : nseg - 1;
      for (int64_t g = g0 + t; g <= g1; g += kSketchThreads) {
        const int64_t c0 = g * V;
        if constexpr (Vec) {
          vec_t v;
#pragma unroll
          for (int q = 0; q < V; ++q) {
            const int p = wpos(c0 + q);
            v[q] = p >= 0 ? (TOut)acc[p] : (TOut)0;
          }
          __builtin_nontemporal_store(v, (vec_t*)(out + c0));
        } else {
          const int p = wpos(c0);
          __builtin_nontemporal_store(p >= 0 ? (TOut)acc[p] : (TOut)0, out + c0);
        }
      }
    }
    // columns past the last whole segment
    for (int64_t c = nseg * V + t; c < n; c += kSketchThreads) {
      const int p = wpos(c);
      out[c] = p >= 0 ? (TOut)acc[p] : (TOut)0;
    }
    return;
  }
  // chunked path
  for (int64_t c0 = 0; c0 < n; c0 += kWin) {
    const int64_t cw = (n - c0) < kWin ? (n - c0) : kWin;
    for (int w = t; w < kWin; w += kSketchThreads) acc[w] = 0.0;
    __syncthreads();
    for (int64_t q = blo; q < bhi; ++q) {
      const int32_t i = perm[q];
      const double sg = (double)sign[i];
      const int64_t lo = row_ptr[i], hi = row_ptr[i + 1];
      for (int64_t e = lo + t; e < hi; e += kSketchThreads) {
        const int64_t c = (int64_t)col[e] - c0;
        if (c >= 0 && c < cw) acc[c] += sg * val[e];
      }
      __syncthreads();
    }
    for (int w = t; w < cw; w += kSketchThreads) out[c0 + w] = (TOut)acc[w];
    __syncthreads();
  }
}

__global__ void k_sketch_rhs(const double* __restrict__ b, int64_t nrhs, int64_t ldb,
                             const int8_t* __restrict__ sign, const int64_t* __restrict__ bptr,
                             const int32_t* __restrict__ perm, int64_t s, double* __restrict__ Sb) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= s) return;
  for (int64_t k = 0; k < nrhs; ++k) {
    double a = 0.0;
    for (int64_t q = bptr[j]; q < bptr[j + 1]; ++q) {
      const int32_t i = perm[q];
      a += (double)sign[i] * b[k * ldb + i];
    }
    Sb[k * s + j] = a;
  }
}

}  // namespace

rfmls_status launch_hash_sign(rfmls_handle* h, int64_t m, int64_t s, uint64_t seed, int32_t* hash,
                              int8_t* sign) {
  if (m == 0) return RFMLS_OK;
  Trace tr(h, "hash_sign", 5.0 * (double)m, 0.0);
  hipLaunchKernelGGL(k_hash_sign, dim3(ceil_div(m, 256)), dim3(256), 0, h->stream, m, (uint64_t)s,
                     seed, hash, sign);
  RFMLS_HIP(h, hipGetLastError());
  return RFMLS_OK;
}

// Counting sort of keys[0..m) (values in [0, nb)) into ptr[0..nb] and a
// permutation with ascending original index inside each key.  Shared by the
// sketch (key = h) and the transpose (key = column).
rfmls_status bucket_sort(rfmls_handle* h, const int32_t* key, int64_t m, int64_t nb, int64_t* ptr,
                         int32_t* perm, int32_t* scratch_count, int32_t* scratch_tmp) {
  hipStream_t st = h->stream;
  Trace tr(h, "bucket_sort", 4.0 * (double)m * 4.0 + 8.0 * (double)nb * 3.0, 0.0);
  hipLaunchKernelGGL(k_fill_i32, dim3(ceil_div(nb, 256) < 4096 ? ceil_div(nb, 256) : 4096),
                     dim3(256), 0, st, scratch_count, nb, 0);
  if (m > 0)
    hipLaunchKernelGGL(k_count, dim3(ceil_div(m, 256)), dim3(256), 0, st, key, m, scratch_count);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, scratch_count, nb, ptr);
  hipLaunchKernelGGL(k_copy_ptr_i32, dim3(ceil_div(nb, 256)), dim3(256), 0, st, ptr, nb,
                     scratch_count);
  if (m > 0) {
    hipLaunchKernelGGL(k_scatter_rows, dim3(ceil_div(m, 256)), dim3(256), 0, st, key, m,
                       scratch_count, perm);
    hipLaunchKernelGGL(k_sort_buckets, dim3(ceil_div(nb, 256)), dim3(256), 0, st, ptr, nb, perm,
                       scratch_tmp);
  }
  RFMLS_HIP(h, hipGetLastError());
  return RFMLS_OK;
}

rfmls_status scan_counts(rfmls_handle* h, const int32_t* count, int64_t n, int64_t* ptr) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, h->stream, count, n, ptr);
  RFMLS_HIP(h, hipGetLastError());
  return RFMLS_OK;
}

rfmls_status run_sketch(rfmls_handle* h, const rfmls_csr* A, int64_t s, const int32_t* hash,
                        const int8_t* sign, const double* b, int64_t nrhs, int64_t ldb, double* Sb,
                        rfmls_dtype dt, void* SA, int64_t ld) {
  void *p_count, *p_ptr, *p_perm, *p_tmp;
  RFMLS_CHECK(workspace(h, WS_SKETCH_COUNT, sizeof(int32_t) * (size_t)(s + 1), &p_count));
  RFMLS_CHECK(workspace(h, WS_SKETCH_PTR, sizeof(int64_t) * (size_t)(s + 1), &p_ptr));
  RFMLS_CHECK(workspace(h, WS_SKETCH_PERM, sizeof(int32_t) * (size_t)(A->m + 1), &p_perm));
  RFMLS_CHECK(workspace(h, WS_MISC, sizeof(int32_t) * (size_t)(A->m + 1), &p_tmp));
  int64_t* bptr = (int64_t*)p_ptr;
  int32_t* perm = (int32_t*)p_perm;
  RFMLS_CHECK(bucket_sort(h, hash, A->m, s, bptr, perm, (int32_t*)p_count, (int32_t*)p_tmp));
  {
  // algorithmic bytes: CSR read once, bucket list and signs, dense SA written once
  const double esz = dt == RFMLS_F64 ? 8.0 : 4.0;
  Trace tr(h, "sketch_rows",
           12.0 * (double)A->nnz + 8.0 * (double)(A->m + 1) + 5.0 * (double)A->m +
               8.0 * (double)(s + 1) + esz * (double)s * (double)A->n,
           (double)A->nnz);
  // 16-byte stores when every row starts 16-byte aligned
  const bool vec = (reinterpret_cast<uintptr_t>(SA) % 16 == 0) && ((int64_t)esz * ld) % 16 == 0;
  if (dt == RFMLS_F64) {
    if (vec)
      hipLaunchKernelGGL((k_sketch_rows<double, true>), dim3((unsigned)s), dim3(kSketchThreads), 0, h->stream,
                         A->row_ptr, A->col, A->val, sign, bptr, perm, A->n, (double*)SA, ld);
    else
      hipLaunchKernelGGL((k_sketch_rows<double, false>), dim3((unsigned)s), dim3(kSketchThreads), 0, h->stream,
                         A->row_ptr, A->col, A->val, sign, bptr, perm, A->n, (double*)SA, ld);
  } else {
    if (vec)
      hipLaunchKernelGGL((k_sketch_rows<float, true>), dim3((unsigned)s), dim3(kSketchThreads), 0, h->stream,
                         A->row_ptr, A->col, A->val, sign, bptr, perm, A->n, (float*)SA, ld);
    else
      hipLaunchKernelGGL((k_sketch_rows<float, false>), dim3((unsigned)s), dim3(kSketchThreads), 0, h->stream,
                         A->row_ptr, A->col, A->val, sign, bptr, perm, A->n, (float*)SA, ld);
  }
  }
  RFMLS_HIP(h, hipGetLastError());
  if (b != nullptr && Sb != nullptr && nrhs > 0) {
    hipLaunchKernelGGL(k_sketch_rhs, dim3(ceil_div(s, 256)), dim3(256), 0, h->stream, b, nrhs, ldb,
                       sign, bptr, perm, s, Sb);
    RFMLS_HIP(h, hipGetLastError());
  }
  return RFMLS_OK;
}

}  // namespace rfmls
