// Internal declarations shared by the HIP translation units of librpid.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/rpid.h"

struct rpid_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cu = 0;
  // Growable device workspace, carved into regions per call.
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // Pinned host word for status read-back.
  int64_t* host_status = nullptr;
  // Uncached device memory for the cross-workgroup exchange of the pivoting
  // kernels, taken from a per-device pool and handed back by rpid_destroy.
  // Once a kernel has read it, it stays allocated until the process ends.
  void* uc = nullptr;
  size_t uc_bytes = 0;
  unsigned lupp_epoch = 0;  // tag of the LUPP exchange words of the latest launch
  // A second stream (default priority) and two events, for work inside one
  // call that can run beside the main stream's (fork and join by events).
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // Device address of this device's fixed scratch array (the allocation-free
  // sketch entry point), looked up once per device at context creation.
  void* fixed_scratch = nullptr;
};

namespace rpid {

// ---------------------------------------------------------------------------
// Error handling
// ---------------------------------------------------------------------------
#define RPID_HIP_CHECK(...)                    \
  do {                                         \
    hipError_t _e = (__VA_ARGS__);             \
    if (_e != hipSuccess) return RPID_ERR_HIP; \
  } while (0)

#define RPID_CHECK(...)             \
  do {                              \
    int _s = (__VA_ARGS__);         \
    if (_s != RPID_OK) return _s;   \
  } while (0)

// Workspace carving: aligned bump allocator over the context's buffer.
struct Carve {
  size_t off = 0;
  template <typename T>
  size_t take(size_t count) {
    off = (off + 255) & ~size_t(255);
    size_t at = off;
    off += count * sizeof(T);
    return at;
  }
};
// Grow the workspace to at least `bytes` (synchronises the stream before
// freeing the old buffer).  Called once at the top of an entry point, before
// any kernel of the call is enqueued; helpers only check their bound.
int ensure_workspace(rpid_ctx ctx, size_t bytes);
inline int ws_check(rpid_ctx ctx, size_t end) {
  return end <= ctx->ws_bytes ? RPID_OK : RPID_ERR_NOMEM;
}
template <typename T>
inline T* ws_ptr(rpid_ctx ctx, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ctx->ws) + off);
}

// ---------------------------------------------------------------------------
// Element conversion helpers (device)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float bf16_bits_to_float(uint16_t b) {
  return __uint_as_float(uint32_t(b) << 16);
}
// Round-to-nearest-even float -> bf16 bits (finite inputs).
__device__ __forceinline__ uint16_t float_to_bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return uint16_t(u >> 16);
}
template <typename T>
__device__ __forceinline__ double load_as_double(const T* p, int64_t i);
template <>
__device__ __forceinline__ double load_as_double<double>(const double* p, int64_t i) {
  return p[i];
}
template <>
__device__ __forceinline__ double load_as_double<float>(const float* p, int64_t i) {
  return (double)p[i];
}
template <>
__device__ __forceinline__ double load_as_double<uint16_t>(const uint16_t* p, int64_t i) {
  return (double)bf16_bits_to_float(p[i]);
}

// ---------------------------------------------------------------------------
// Launchers implemented in the .hip translation units
// ---------------------------------------------------------------------------
// Fill `count` 64-bit words with `value` (graph-capture friendly, no memset).
int launch_fill_u64(rpid_ctx ctx, uint64_t* p, size_t count, uint64_t value);

// LUPP on an n x k panel P(i, j) = base[i * rs + j * cs] (k steps), see lupp.hip.
template <typename T>
int lupp_panel(rpid_ctx ctx, const T* base, int64_t rs, int64_t cs, int64_t n, int64_t k,
               int64_t* J, T* Lf, int64_t ldl, T* Uf, int64_t ldu, T* diag, size_t ws_off,
               int64_t* status_dev);
// Column-pivoted Householder QR, k steps, of a sketch given as the panel
// P(i, j) = base[i * rs + j * cs] = X(j, i) (n candidates, l rows of X):
// pivots J, the k x n top of R in the original column order (Rf, ldr) and
// |R(t, t)|, see lupp.hip.
template <typename T>
int cpqr_panel(rpid_ctx ctx, const T* base, int64_t rs, int64_t cs, int64_t n, int64_t l, int64_t k,
               int64_t* J, T* Rf, int64_t ldr, T* diag, int64_t* status_dev);
// Hand the context's uncached exchange buffer back to the per-device pool
// (rpid_destroy); the buffer itself stays allocated.
void release_exchange_buffer(rpid_ctx ctx);
// Workspace bytes lupp_panel needs for an n x k panel.
size_t lupp_workspace_bytes(rpid_ctx ctx, int64_t n, int64_t k, int elem_bytes);

// X = P^T A for a "row-contiguous" left operand: P is m x l column-major (ldp),
// i.e. P^T is l x m with rows contiguous; A m x n (lda); X l x n (ldx).
// `max_split` caps the number of split-K slices (each l x n accumulators in
// the workspace at ws_off).
int sketch_f64(rpid_ctx ctx, const double* Pt, int64_t ldp, const double* A, int64_t lda,
               int64_t m, int64_t n, int64_t l, double* X, int64_t ldx, size_t ws_off,
               int64_t max_split = 16);
int sketch_f32(rpid_ctx ctx, const float* Pt, int64_t ldp, const float* A, int64_t lda,
               int64_t m, int64_t n, int64_t l, float* X, int64_t ldx, size_t ws_off,
               int64_t max_split = 16);
int sketch_e4m3(rpid_ctx ctx, const uint8_t* Pt, int64_t ldp, const uint8_t* A, int64_t lda,
                int64_t m, int64_t n, int64_t l, float* X, int64_t ldx, size_t ws_off);
int sketch_bf16(rpid_ctx ctx, const uint16_t* Pt, int64_t ldp, const uint16_t* A, int64_t lda,
                int64_t m, int64_t n, int64_t l, float* X, int64_t ldx, size_t ws_off,
                int64_t max_split = 16);
// Y^T = Omega A^T (l x m) for a column-major m x n BF16 A read in place;
// Ot = Omega^T is n x l (ldot).  RPID_ERR_UNSUPPORTED when the shape or the
// alignment does not suit the kernel (n % 64, m % 8, 16-byte alignment).
int sketch_at_bf16(rpid_ctx ctx, const uint16_t* Ot, int64_t ldot, const uint16_t* A, int64_t lda,
                   int64_t m, int64_t n, int64_t l, float* Yt, int64_t ldyt, size_t ws_off);
size_t sketch_workspace_bytes(rpid_ctx ctx, int64_t m, int64_t n, int64_t l, int elem_acc);

// Sparse and structured sketches (sparse.hip).  expand_sparse_sign writes
// the l x m sparse sign embedding (+-1 entries, unscaled) as
// out[r * rs + i * cs]; i_fast picks the faster-varying index of the write.
template <typename TE>
int expand_sparse_sign(rpid_ctx ctx, int64_t m, int64_t l, int zeta, const int32_t* rows,
                       const int8_t* signs, TE* out, int64_t rs, int64_t cs, bool i_fast);
template <typename T>
int scale_matrix(rpid_ctx ctx, int64_t rows, int64_t cols, T* X, int64_t ldx, T scale);
// The SRTT embedding transposed (m x l, ldp) in TE; inv is m int32 of scratch.
template <typename TE>
int build_srtt_t(rpid_ctx ctx, int64_t m, int64_t l, const int32_t* perm, const int8_t* phi,
                 const int32_t* sel, int32_t* inv, TE* Pt, int64_t ldp);
// X = Gamma A for a CSC matrix A (m x n, nnz stored entries); Gamma l x m.
template <typename T>
int csc_sketch(rpid_ctx ctx, int64_t m, int64_t n, int64_t nnz, const int64_t* colptr,
               const int64_t* rowidx, const T* vals, const T* Gamma, int64_t ldg, int64_t l, T* X,
               int64_t ldx);
// X = scale S A for a CSC matrix A and the sparse sign embedding S (l x m,
// zeta entries +-1 per column given by rows / signs), applied directly.
template <typename T>
int csc_sparse_sign(rpid_ctx ctx, int64_t m, int64_t n, int64_t nnz, const int64_t* colptr,
                    const int64_t* rowidx, const T* vals, const int32_t* rows, const int8_t* signs,
                    int zeta, int64_t l, T scale, T* X, int64_t ldx);
// C(:, t) = A(:, J[t]) for a CSC matrix (J null: all n columns, k = n).
template <typename T>
int csc_gather(rpid_ctx ctx, int64_t m, int64_t n, int64_t nnz, const int64_t* colptr,
               const int64_t* rowidx, const T* vals, int64_t k, const int64_t* J, T* C, int64_t ldc);
bool residual_stream_bf16(rpid_ctx ctx, int64_t m, int64_t n, int64_t r, const uint16_t* R,
                          int64_t ldr, const uint16_t* Pt, int64_t ldpt, const uint16_t* Q,
                          int64_t ldq, double* partials, int64_t* count, int* err);

// General FP64 GEMM: C = alpha op(A) op(B) + beta C, column-major.
int dgemm(rpid_ctx ctx, bool transA, bool transB, int64_t M, int64_t N, int64_t K, double alpha,
          const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
          int64_t ldc, size_t ws_off);

// Triangular solve with many right-hand sides (FP64): for every r < nrhs,
// solve op(T) x_r = b_r, op(T) = T or T^T of the k x k matrix T (ldt), with
// op(T) lower (forward) or upper (backward) triangular and optionally a unit
// diagonal.  b_r(c) = B[r * bcs + c * brs] (type TB), x_r(c) = X[r * xcs + c * xrs].
// X may alias B only when the two layouts are identical.
template <typename TB>
int tri_solve(rpid_ctx ctx, int64_t k, int64_t nrhs, const double* T, int64_t ldt, bool trans,
              bool lower_op, bool unit, const TB* B, int64_t brs, int64_t bcs, double* X,
              int64_t xrs, int64_t xcs);

// W = T^{-1} for a k x k triangular T (k <= 1024), lower or upper, unit or
// not; above 512 the scratch region at ws_tmp must also hold a
// (k/2) x (k - k/2) FP64 product and the split-K parts of two GEMMs.
int tri_inverse(rpid_ctx ctx, int64_t k, const double* T, int64_t ldt, bool lower, bool unit,
                double* W, int64_t ldw, size_t ws_tmp);

// Register-resident triangular kernels (sweep.hip), k <= 512 (one launch up
// to 160, one 2 x 2 split up to 288, repeated splits of a leading block of 128
// above); the scratch region at ws_tmp must hold sweep_scratch_bytes(k).
bool sweep_supported(int64_t k);
size_t sweep_scratch_bytes(int64_t k);
// For `batch` (1 or 2) SPD k x k matrices G_b (stride apart, lower part
// read): Cholesky G = R^T R and Winv_b = R^{-1} (upper, full matrix written).
// status[b] = 0, or j+1 for a non-positive / non-finite pivot at column j
// (the outputs are then undefined).
int chol_inverse_batched(rpid_ctx ctx, int batch, int64_t k, const double* G, int64_t ldg,
                         int64_t stride, double* Winv, int64_t ldw, int64_t wstride,
                         int64_t* status_dev, size_t ws_tmp);
// W = T^{-1} (full matrix written) for a lower or upper triangular k x k T.
int tri_inverse_sweep(rpid_ctx ctx, int64_t k, const double* T, int64_t ldt, bool lower,
                      bool unit, double* W, int64_t ldw, size_t ws_tmp);

// Cholesky G = R^T R of `batch` SPD k x k matrices (in place, upper R; the
// strict lower part is zeroed), one workgroup per matrix.  status[b] = 0 or
// j+1 for a non-positive / non-finite pivot at column j.
int cholesky_batched(rpid_ctx ctx, int batch, int64_t k, double* G, int64_t ldg,
                     int64_t stride, int64_t* status_dev);

// Small element-wise helpers (utils.hip)
template <typename TS, typename TD>
int convert_matrix(rpid_ctx ctx, int64_t rows, int64_t cols, const TS* S, int64_t lds, TD* D,
                   int64_t ldd);
// C(:, t) = A(:, J[t]) / R(t, :) = A(I[t], :); indices outside the matrix
// read as zeros (never fault).
template <typename TS, typename TD>
int gather_columns(rpid_ctx ctx, int64_t m, int64_t k, const TS* A, int64_t lda, int64_t ncols,
                   const int64_t* J, TD* C, int64_t ldc);
template <typename TS, typename TD>
int gather_rows(rpid_ctx ctx, int64_t k, int64_t n, const TS* A, int64_t lda, int64_t nrows,
                const int64_t* I, TD* R, int64_t ldr);
// D += alpha S (FP64, rows x cols)
int axpy_matrix(rpid_ctx ctx, int64_t rows, int64_t cols, double alpha, const double* S,
                int64_t lds, double* D, int64_t ldd);
// Largest eigenvalue of a symmetric positive semi-definite k x k FP64 matrix
// by power iteration (single workgroup); result written to *lam (device).
int power_iteration(rpid_ctx ctx, int64_t k, const double* G, int64_t ldg, int max_iter,
                    double rtol, double* lam);
// Y (cols x rows) = X^T for an FP64 rows x cols matrix.
// Rt(j, t) = A(I[t], j) as FP64 (Rt n x k, ldr >= n): the rows A(I, :) transposed.
template <typename TS>
int gather_rows_t(rpid_ctx ctx, int64_t k, int64_t n, const TS* A, int64_t lda, int64_t nrows,
                  const int64_t* I, double* Rt, int64_t ldr);
int transpose_f64(rpid_ctx ctx, int64_t rows, int64_t cols, const double* X, int64_t ldx,
                  double* Y, int64_t ldy);
// D = S + diag(shift) on a k x k matrix; `shift_from` (device, nullable)
// gives shift = scale * S-trace-free value computed on device: shift =
// c * sum_i S(i, i) (trace of a Gram matrix = ||C||_F^2).
int add_trace_shift(rpid_ctx ctx, int64_t k, double* G, int64_t ldg, double c);
// Set the columns J[t] of Z (k x n) to e_t.
// Z(:, J[t]) = e_t (entries of J outside [0, n) skipped).
int set_identity_columns(rpid_ctx ctx, int64_t k, int64_t n, const int64_t* J, double* Z, int64_t ldz);
// Split an FP64 matrix into `parts` BF16 terms: S = sum_p D_p (greedy RNE
// residuals); D is rows x (parts * cols) with part p in columns [p cols, (p+1) cols).
int split_bf16(rpid_ctx ctx, int64_t rows, int64_t cols, const double* S, int64_t lds, int parts,
               uint16_t* D, int64_t ldd);

}  // namespace rpid
