// Shared definitions of the rfmls HIP library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/rfmls.h"

namespace rfmls {

constexpr int kWave = 64;  // CDNA wavefront width
// grid-reduction counters of the QR panel kernel: one 256-byte line per counter
constexpr int kBarrierStride = 64;     // unsigned words between counters
constexpr int kBarrierWords = 64 * kBarrierStride;

// ---------------------------------------------------------------------------
// Handle and workspace
// ---------------------------------------------------------------------------
struct Workspace {
  void* ptr = nullptr;
  size_t bytes = 0;
};

}  // namespace rfmls

namespace rfmls {
// One autotuned launch shape: the kernel family, the shape of the operand it
// was tuned on, the candidate chosen and its time beside the hand-picked one's.
struct TuneRec {
  char kernel[16];
  int64_t rows, cols, nnz;
  int choice;
  char desc[48];
  double ms_best, ms_default;
  int candidates;
};
struct TraceRec {
  const char* name;
  hipEvent_t beg, end;
  double bytes, flops;
};
}  // namespace rfmls

struct rfmls_handle {
  int device = 0;
  bool trace = false;
  std::vector<rfmls::TraceRec> trace_recs;
  std::vector<hipEvent_t> event_pool;
  hipStream_t stream = nullptr;
  int num_cus = 0;
  std::string last_error;
  // Named, growable device scratch buffers (slot index -> buffer).
  std::vector<rfmls::Workspace> ws;
  unsigned int* barrier = nullptr;  // grid-barrier counters (device)
  int* dev_flags = nullptr;         // device error / abort flags
  void* pinned = nullptr;           // small pinned host staging buffer
  size_t pinned_bytes = 0;
  hipStream_t cap_stream = nullptr; // stream that graphs are captured on (created on first use)
  int tune = 1;                     // autotune launch shapes on first use (rfmls_tune_enable)
  int qr_panel = 0;                 // rfmls_qr_panel_mode: 0 CholeskyQR2 panels where eligible,
                                    // 1 unblocked Householder panels only, 2/3 CholeskyQR2 with its
                                    // first / second pass forced to fail (tests of the fallback)
  int qr_lookahead = 0;             // rfmls_qr_lookahead: next outer block's panels beside the trailing update
  hipStream_t la_stream = nullptr;  // their stream (created on first use) and its two events
  hipEvent_t la_event[2] = {nullptr, nullptr};
  std::vector<rfmls::TuneRec> tuned;
};

struct rfmls_precond {
  int64_t n = 0;
  int64_t nt = 0;            // number of tile rows, ceil(n / kTile)
  rfmls_dtype store = RFMLS_F64;
  // full = 0: X = R^{-1}, upper-triangular tile packing (CSQRP, Alg. 1);
  // full = 1: X = P = V_r Sigma_r^{-1}, the full nt x nt tile grid (CSSVDP, Alg. 2)
  int full = 0;
  void* Xpk = nullptr;       // packed tiles of X
  double* Rdense = nullptr;  // R (row-major n x n, float64) kept for export
  // SVD preconditioner only: singular values in the column order of P, the
  // numerical rank, the Jacobi sweeps taken and the last sweep's largest
  // |cos| between two columns
  double* sigma = nullptr;
  int64_t rank = 0;
  int sweeps = 0;
  double off = 0.0;
  int device = 0;
  // statistics of R: min|r_ii| / max|r_jj| and min_j |r_jj| / ||R[:, j]||
  double pivot_ratio = 0.0, rho_min = 0.0;
  // work decomposition of the triangular products: chunks of `chunk` tiles
  int chunk = 4;
  int64_t ntab = 0;          // number of (row-or-column, chunk) work items
  int2* tab_row = nullptr;   // X v:   (tile row I, chunk k)
  int2* tab_col = nullptr;   // X^T q: (tile column J, chunk k)
  double* part = nullptr;    // nt x ceil(nt/chunk) x kTile partial sums
};

namespace rfmls {

// Packed upper-triangular tile layout for the preconditioner: tiles of
// kTile x kTile, tile (I, J) for J >= I stored contiguously (row-major inside
// the tile), tile rows one after another.
constexpr int kTile = 64;
__host__ __device__ inline int64_t tile_index(int64_t I, int64_t J, int64_t nt) {
  // tiles before row I: sum_{r<I} (nt - r) = I*nt - I*(I-1)/2
  return I * nt - (I * (I - 1)) / 2 + (J - I);
}
// The same for either packing (full: the nt x nt grid, row after row), and
// the stored tiles of a tile row I: columns [row_first(I), nt); of a tile
// column J: rows [0, col_end(J)).
__host__ __device__ inline int64_t ptile(int64_t I, int64_t J, int64_t nt, int full) {
  return full ? I * nt + J : tile_index(I, J, nt);
}
__host__ __device__ inline int64_t row_first(int64_t I, int full) { return full ? 0 : I; }
__host__ __device__ inline int64_t col_end(int64_t J, int64_t nt, int full) { return full ? nt : J + 1; }
__host__ __device__ inline int64_t stored_tiles(int64_t nt, int full) {
  return full ? nt * nt : nt * (nt + 1) / 2;
}

// Error plumbing --------------------------------------------------------------
rfmls_status fail(rfmls_handle* h, rfmls_status st, const char* fmt, ...);

#define RFMLS_HIP(h, call)                                                           \
  do {                                                                               \
    hipError_t _e = (call);                                                          \
    if (_e != hipSuccess)                                                            \
      return ::rfmls::fail((h), RFMLS_E_HIP, "%s:%d %s: %s", __FILE__, __LINE__, #call, \
                           hipGetErrorString(_e));                                   \
  } while (0)

#define RFMLS_CHECK(expr)                \
  do {                                   \
    rfmls_status _s = (expr);            \
    if (_s < 0) return _s;               \
  } while (0)

// Workspace slot `slot` with at least `bytes` bytes (grows, never shrinks).
rfmls_status workspace(rfmls_handle* h, int slot, size_t bytes, void** out);

inline unsigned ceil_div(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// Slots of the handle workspace used by the different stages.
enum WsSlot {
  WS_SKETCH_COUNT = 0,
  WS_SKETCH_PTR,
  WS_SKETCH_PERM,
  WS_SKETCH_HASH,
  WS_SKETCH_SIGN,
  WS_QR_TAU,
  WS_QR_PART,
  WS_QR_W,
  WS_QR_WP,
  WS_QR_T,
  WS_QR_WR,
  WS_QR_INNER,
  WS_TRSM,
  WS_LSQR_VEC,
  WS_LSQR_SCAL,
  WS_LSQR_RUNS,
  WS_LSQR_PART,
  WS_LSQR_BLK,
  WS_LSQR_BSTATE,
  WS_TRANSPOSE,
  WS_X0,
  WS_GEMV,
  WS_SVD,
  WS_SPMM_PART,
  WS_SPMM_WPTR_A,
  WS_SPMM_WDESC_A,
  WS_SPMM_WPTR_AT,
  WS_SPMM_WDESC_AT,
  WS_SVD2,
  WS_APPLYQ,
  WS_MISC,
  WS_CHOLQR,
  WS_NUM_SLOTS
};

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Deterministic block sum of one double per thread (blockDim.x threads, a
// multiple of 64).  `scratch` must hold blockDim.x/64 doubles.  Every thread
// receives the result.
__device__ __forceinline__ double block_sum(double v, double* scratch) {
  v = wave_sum(v);
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) scratch[w] = v;
  __syncthreads();
  double t = 0.0;
  const int nw = blockDim.x / kWave;
  for (int i = 0; i < nw; ++i) t += scratch[i];
  return t;
}

}  // namespace rfmls

// Tracing: bracket the launches issued inside the scope with events when the
// handle's trace flag is set.  name must be a string literal.
namespace rfmls {
hipEvent_t trace_event(rfmls_handle* h);
struct Trace {
  rfmls_handle* h;
  TraceRec rec;
  Trace(rfmls_handle* hh, const char* name, double bytes, double flops) : h(hh) {
    if (!h->trace) return;
    rec.name = name;
    rec.bytes = bytes;
    rec.flops = flops;
    rec.beg = trace_event(h);
    rec.end = trace_event(h);
    hipEventRecord(rec.beg, h->stream);
  }
  ~Trace() {
    if (!h->trace) return;
    hipEventRecord(rec.end, h->stream);
    h->trace_recs.push_back(rec);
  }
};
}  // namespace rfmls

// Captured iterations: the launches of the LSQR loop between two polls of the
// device stop flag, recorded once as a HIP graph and replayed with one
// hipGraphLaunch per poll interval.  Every kernel of the loop checks the
// device "done" word first, so iterations past the stop are no-ops, exactly as
// in the eager loop.
namespace rfmls {
struct IterGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  IterGraph() = default;
  IterGraph(const IterGraph&) = delete;
  IterGraph& operator=(const IterGraph&) = delete;
  ~IterGraph() {
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
  }
};

// Records what `body` enqueues on h->stream into g.  During the capture
// h->stream is the handle's capture stream (a non-blocking stream of default
// priority, created on first use); body must enqueue kernels only.
template <class F>
rfmls_status capture_graph(rfmls_handle* h, IterGraph* g, F&& body) {
  if (!h->cap_stream) {
    hipError_t e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(h, RFMLS_E_HIP, "hipStreamCreateWithFlags: %s", hipGetErrorString(e));
  }
  hipStream_t saved = h->stream;
  hipError_t e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return fail(h, RFMLS_E_HIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  h->stream = h->cap_stream;
  rfmls_status st = body();
  hipGraph_t gr = nullptr;
  e = hipStreamEndCapture(h->cap_stream, &gr);
  h->stream = saved;
  if (st < 0) {
    if (gr) hipGraphDestroy(gr);
    return st;
  }
  if (e != hipSuccess || !gr) return fail(h, RFMLS_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  g->graph = gr;
  e = hipGraphInstantiate(&g->exec, gr, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    g->exec = nullptr;
    return fail(h, RFMLS_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  return RFMLS_OK;
}
}  // namespace rfmls

// Launch entry points implemented in the individual .hip files -----------------
namespace rfmls {
// CholeskyQR2 panel with Householder reconstruction (cholqr.hip), float64 or float32 storage
int64_t cholqr_workspace_doubles(int64_t M);
rfmls_status run_cholqr_panel(rfmls_handle* h, double* P, int64_t ld, int64_t M, double* tau, double* ws,
                              int* status, double min_ratio1, double min_ratio2);
rfmls_status run_cholqr_panel(rfmls_handle* h, float* P, int64_t ld, int64_t M, float* tau, double* ws, int* status,
                              double min_ratio1, double min_ratio2);
rfmls_status cholqr_fix(rfmls_handle* h, double* P, int64_t ld, int64_t M, const double* ws, const int* status);
rfmls_status cholqr_fix(rfmls_handle* h, float* P, int64_t ld, int64_t M, const double* ws, const int* status);
rfmls_status launch_hash_sign(rfmls_handle* h, int64_t m, int64_t s, uint64_t seed, int32_t* hash,
                              int8_t* sign);
rfmls_status run_sketch(rfmls_handle* h, const rfmls_csr* A, int64_t s, const int32_t* hash,
                        const int8_t* sign, const double* b, int64_t nrhs, int64_t ldb, double* Sb,
                        rfmls_dtype dt, void* SA, int64_t ld);
rfmls_status run_transpose(rfmls_handle* h, const rfmls_csr* A, int64_t* rp, int32_t* col,
                           double* val);
rfmls_status scan_counts(rfmls_handle* h, const int32_t* count, int64_t n, int64_t* ptr);
// Householder QR of SA (s x n); columns n .. n_room-1 (n_room <= ld) may be
// used as scratch; tau_out (n values of SA's dtype, device) receives every
// reflector's tau when given
rfmls_status run_qr(rfmls_handle* h, int64_t s, int64_t n, int64_t n_room, rfmls_dtype dt, void* SA,
                    int64_t ld, void* tau_out = nullptr);
// Y <- Q Y (Y: s x ny row-major, ldy) for the float64 QR run_qr left in P
// (s x n, ld) with its taus
rfmls_status apply_householder(rfmls_handle* h, const double* P, int64_t ld, int64_t s, int64_t n,
                               const double* tau, double* Y, int64_t ldy, int64_t ny);
rfmls_status run_build_precond(rfmls_handle* h, int64_t n, rfmls_dtype qr_dt, const void* SA,
                               int64_t ld, rfmls_dtype store, rfmls_precond_t* P, int check_rank);
// checks R (zero / non-finite pivots; with check_rank the 16 u pivot ratio; with
// check_precision the float32 column-relative pivot), records its statistics,
// then forms and packs X = R^{-1}
rfmls_status finish_precond(rfmls_handle* h, rfmls_precond_t* P, int check_rank, double unit,
                            int check_precision, int invert_f32 = 0);
// tables of the tiled products and the packed tiles of X (row-major n x n
// dense, float64) in P->store precision, for either packing (P->full)
rfmls_status pack_precond(rfmls_handle* h, rfmls_precond_t* P, const double* X);
// R (normalised, row-major n x n float64) from the top n rows of a float64 QR
// result into a new P->Rdense
rfmls_status run_extract_R(rfmls_handle* h, int64_t n, const double* SA, int64_t ld, rfmls_precond_t* P);
// CSSVDP preconditioner (Alg. 2 step 3) from the R factor in SA's top n rows
rfmls_status run_build_svd_precond(rfmls_handle* h, int64_t n, const double* SA, int64_t ld,
                                   rfmls_dtype store, double rcond, int max_sweeps,
                                   rfmls_precond_t* P);
int64_t svd_max_n();
rfmls_status put_sketched_rhs(rfmls_handle* h, int64_t s, int64_t n, int64_t nrhs, rfmls_dtype dt,
                              void* SA, int64_t ld, const double* SB);
rfmls_status sketched_solution(rfmls_handle* h, const rfmls_precond_t* P, int64_t nrhs,
                               rfmls_dtype dt, const void* SA, int64_t ld, double* X0,
                               int64_t ldx0);
// out = X in (trans 0) or X^T in (trans 1), X the stored preconditioner (R^{-1} or P),
// minus hcoef (*dcoef) prev when prev is given; per-block sums of squares of
// out into sq when given; nothing when *done is set
rfmls_status tri_apply(rfmls_handle* h, const rfmls_precond_t* P, int trans, const double* in,
                       double* out, double hcoef, const double* dcoef, const double* prev,
                       double* sq, const int* done);
rfmls_status unpack_precond(rfmls_handle* h, const rfmls_precond_t* P, double* Xdense);
rfmls_status run_solve(rfmls_handle* h, const rfmls_csr* A, const rfmls_csr* AT,
                       const rfmls_precond_t* P, const double* B, int64_t ldb, int64_t nrhs,
                       double* X, int64_t ldx, double* Rout, int64_t ldr, const rfmls_opts* o,
                       rfmls_info* info);
// allocation-free single-right-hand-side solve (device scratch in a file-scope
// array of lsqr.hip); noalloc_scratch_init records the current device's
// address of that array and is called once per handle by rfmls_create
rfmls_status noalloc_scratch_init(rfmls_handle* h);
int64_t noalloc_scratch_bytes();
int64_t noalloc_needed_bytes(int64_t m, int64_t n);
rfmls_status run_solve_noalloc(rfmls_handle* h, const rfmls_csr* A, const rfmls_csr* AT,
                               const rfmls_precond_t* P, const double* B, int64_t ldb, int64_t nrhs,
                               double* X, int64_t ldx, double* Rout, int64_t ldr, const rfmls_opts* o,
                               rfmls_info* info);
rfmls_status run_solve_explicit(rfmls_handle* h, const rfmls_csr* A, const rfmls_csr* AT,
                                const rfmls_precond_t* P, const double* Bm, int64_t ldbm,
                                const double* B, int64_t ldb, int64_t nrhs, double* X, int64_t ldx,
                                double* Rout, int64_t ldr, const rfmls_opts* o, rfmls_info* info);
rfmls_status run_form_B(rfmls_handle* h, const rfmls_csr* A, const rfmls_precond_t* P, double* Bmat,
                        int64_t ldb);
rfmls_status run_solve_block(rfmls_handle* h, const rfmls_csr* A, const rfmls_csr* AT,
                             const rfmls_precond_t* P, const double* B, int64_t ldb, int64_t nrhs,
                             double* X, int64_t ldx, double* Rout, int64_t ldr,
                             const rfmls_opts* o, rfmls_info* info);
rfmls_status run_backward_block(rfmls_handle* h, const rfmls_csr* A, const rfmls_csr* AT,
                                const rfmls_precond_t* P, const double* Xs, int64_t ldx,
                                const double* Rres, int64_t ldr, const double* G, int64_t ldg,
                                int64_t nrhs, double* dB, int64_t lddb, double* dAval,
                                const rfmls_opts* o, rfmls_info* info);
rfmls_status run_backward(rfmls_handle* h, const rfmls_csr* A, const rfmls_csr* AT,
                          const rfmls_precond_t* P, const double* Xs, int64_t ldx,
                          const double* Rres, int64_t ldr, const double* G, int64_t ldg,
                          int64_t nrhs, double* dB, int64_t lddb, double* dAval,
                          const rfmls_opts* o, rfmls_info* info);
}  // namespace rfmls
