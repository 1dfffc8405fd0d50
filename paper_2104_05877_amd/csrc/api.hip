// C-ABI entry points of librpid (declared in include/rpid.h): argument
// validation, workspace sizing and the order of the kernels of each step.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <vector>

#include "rpid_internal.hpp"

namespace rpid {

template <typename TA>
int residual_f64(rpid_ctx ctx, int64_t m, int64_t n, int64_t r, const TA* A, int64_t lda,
                 const double* P, int64_t ldp, const double* Q, int64_t ldq, double* partials,
                 double* out2);
int residual_bf16(rpid_ctx ctx, int64_t m, int64_t n, int64_t r, const uint16_t* A, int64_t lda,
                  const uint16_t* Pt, int64_t ldpt, const uint16_t* Q, int64_t ldq,
                  double* partials, double* out2);
int pack_cols_t(rpid_ctx ctx, int64_t m, int64_t k, int parts, const uint16_t* A, int64_t lda,
                int64_t ncols, const int64_t* J, uint16_t* Pt);
int pack_split_t(rpid_ctx ctx, int64_t m, int64_t k, int parts, const double* P, int64_t ldp,
                 uint16_t* Pt);
size_t residual_partials(int64_t m, int64_t n, bool bf16);
int mlp_forward(rpid_ctx, const float*, const float*, int64_t, float*, float*);
int mlp_backward(rpid_ctx, const float*, const float*, const float*, const float*, int64_t,
                 float*, size_t);
int mlp_adam(rpid_ctx, float*, const float*, float*, float*, float, int64_t);
int mlp_features(rpid_ctx, const void*, bool, int64_t, int64_t, float*);
int mlp_pinball(rpid_ctx, const float*, const float*, int64_t, float, float*, float*);
size_t mlp_backward_workspace(int64_t B);
int sketch_fp8(rpid_ctx, const float*, int64_t, int64_t, int64_t, const float*, int64_t, int64_t,
               float*, int64_t, size_t);
size_t sketch_fp8_workspace(int64_t m, int64_t n, int64_t l);

int ensure_workspace(rpid_ctx ctx, size_t bytes) {
  if (bytes <= ctx->ws_bytes) return RPID_OK;
  if (ctx->ws) {
    RPID_HIP_CHECK(hipStreamSynchronize(ctx->stream));
    RPID_HIP_CHECK(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  size_t want = bytes + bytes / 4 + (1u << 20);
  if (hipMalloc(&ctx->ws, want) != hipSuccess) {
    ctx->ws = nullptr;
    return RPID_ERR_NOMEM;
  }
  ctx->ws_bytes = want;
  return RPID_OK;
}

static int read_status(rpid_ctx ctx, const int64_t* status_dev, int64_t* out) {
  RPID_HIP_CHECK(hipMemcpyAsync(ctx->host_status, status_dev, sizeof(int64_t),
                                hipMemcpyDeviceToHost, ctx->stream));
  RPID_HIP_CHECK(hipStreamSynchronize(ctx->stream));
  *out = *ctx->host_status;
  return RPID_OK;
}

static int read_doubles(rpid_ctx ctx, const double* dev, double* host, int count) {
  RPID_HIP_CHECK(hipMemcpyAsync(ctx->host_status, dev, sizeof(double) * count,
                                hipMemcpyDeviceToHost, ctx->stream));
  RPID_HIP_CHECK(hipStreamSynchronize(ctx->stream));
  for (int i = 0; i < count; ++i) host[i] = reinterpret_cast<double*>(ctx->host_status)[i];
  return RPID_OK;
}

static bool is_lupp_type(rpid_dtype t) { return t == RPID_F64 || t == RPID_F32; }
static size_t esize(rpid_dtype t) {
  switch (t) {
    case RPID_F64: return 8;
    case RPID_F32: return 4;
    case RPID_BF16: return 2;
    case RPID_FP8_E4M3: return 1;
  }
  return 0;
}

// Transpose-copy for the packing of Omega (element size 2, 4 or 8 bytes):
// Y(j, i) = X(i, j), X rows x cols and Y cols x rows, both column-major.
// 64 x 64 tiles through LDS; 16-byte vectors on both sides of an interior,
// aligned tile, element by element at the edges.
template <typename E>
__global__ __launch_bounds__(256) void transpose_copy_kernel(int64_t rows, int64_t cols, const E* X,
                                                             int64_t ldx, E* Y, int64_t ldy) {
  constexpr int T = 64;
  constexpr int V = 16 / (int)sizeof(E);  // elements per 16-byte vector
  constexpr int LD = T + V;               // padded LDS column
  __shared__ __attribute__((aligned(16))) E tile[T * LD];
  const int64_t bi = (int64_t)blockIdx.x * T, bj = (int64_t)blockIdx.y * T;
  const bool full = bi + T <= rows && bj + T <= cols;
  const bool vx = full && ((uintptr_t)X % 16 == 0) && (ldx * (int64_t)sizeof(E)) % 16 == 0;
  const bool vy = full && ((uintptr_t)Y % 16 == 0) && (ldy * (int64_t)sizeof(E)) % 16 == 0;
  const int tid = threadIdx.x;
  // load: tile(j, i) = X(bi + i, bj + j)
  if (vx) {
    for (int v = tid; v < T * T / V; v += 256) {
      const int j = v / (T / V), i = (v % (T / V)) * V;
      *reinterpret_cast<uint4*>(&tile[j * LD + i]) =
          *reinterpret_cast<const uint4*>(X + (bi + i) + (bj + j) * ldx);
    }
  } else {
    for (int e = tid; e < T * T; e += 256) {
      const int j = e / T, i = e % T;
      if (bi + i < rows && bj + j < cols) tile[j * LD + i] = X[(bi + i) + (bj + j) * ldx];
    }
  }
  __syncthreads();
  // store: Y(bj + j, bi + i) = tile(j, i); a vector holds V consecutive j
  if (vy) {
    for (int v = tid; v < T * T / V; v += 256) {
      const int i = v / (T / V), j = (v % (T / V)) * V;
      E buf[V];
#pragma unroll
      for (int u = 0; u < V; ++u) buf[u] = tile[(j + u) * LD + i];
      *reinterpret_cast<uint4*>(Y + (bj + j) + (bi + i) * ldy) = *reinterpret_cast<const uint4*>(buf);
    }
  } else {
    for (int e = tid; e < T * T; e += 256) {
      const int i = e / T, j = e % T;
      if (bi + i < rows && bj + j < cols) Y[(bj + j) + (bi + i) * ldy] = tile[j * LD + i];
    }
  }
}

template <typename E>
static int transpose_copy(rpid_ctx ctx, int64_t rows, int64_t cols, const E* X, int64_t ldx, E* Y,
                          int64_t ldy) {
  dim3 grid((unsigned)((rows + 63) / 64), (unsigned)((cols + 63) / 64));
  hipLaunchKernelGGL((transpose_copy_kernel<E>), grid, dim3(256), 0, ctx->stream, rows, cols, X,
                     ldx, Y, ldy);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

// W(0:k, :) += W(k:2k, :) (the two BF16 terms of a split left operand),
// written as FP64 into Wd (k x n).
__global__ void sum_halves_kernel(int64_t k, int64_t n, const float* W2, double* Wd) {
  const int64_t total = k * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % k, j = e / k;
    Wd[i + j * k] = (double)W2[i + j * 2 * k] + (double)W2[i + k + j * 2 * k];
  }
}

// ---------------------------------------------------------------------------
// CUR: Cholesky-QR passes over C (m x k) and R^T (n x k), both FP64.
// One Cholesky-QR pass over one tall FP64 matrix X (rows x k): Gram,
// Cholesky and the inverse of its factor (Wi = R^{-1}), Xq = X Wi.
static int chol_qr_one(rpid_ctx ctx, int64_t rows, int64_t k, const double* X, double* Xq, double* F,
                       double* Wi, int64_t* status_dev, size_t ws_tmp) {
  const int64_t kk = k * k;
  RPID_CHECK(dgemm(ctx, true, false, k, k, rows, 1.0, X, rows, X, rows, 0.0, F, k, ws_tmp));
  if (sweep_supported(k)) {
    RPID_CHECK(chol_inverse_batched(ctx, 1, k, F, k, kk, Wi, k, kk, status_dev, ws_tmp));
  } else {
    RPID_CHECK(cholesky_batched(ctx, 1, k, F, k, kk, status_dev));
    RPID_CHECK(tri_inverse(ctx, k, F, k, false, false, Wi, k, ws_tmp));
  }
  RPID_CHECK(dgemm(ctx, false, false, rows, k, k, 1.0, X, rows, Wi, k, 0.0, Xq, rows, ws_tmp));
  return RPID_OK;
}

// Points the context's launches at another stream for a scope.
struct StreamSwap {
  rpid_ctx ctx;
  hipStream_t saved;
  StreamSwap(rpid_ctx c, hipStream_t s) : ctx(c), saved(c->stream) { c->stream = s; }
  ~StreamSwap() { ctx->stream = saved; }
};

// After work has been forked onto the side stream, every way out of the call
// joins it back: on an early error return the main stream is made to wait for
// everything enqueued on the side so far, so the next call on the context
// cannot reuse workspace regions the side stream is still writing.
struct SideJoin {
  rpid_ctx ctx;
  bool joined = false;
  explicit SideJoin(rpid_ctx c) : ctx(c) {}
  ~SideJoin() {
    if (joined) return;
    if (hipEventRecord(ctx->ev_join, ctx->side) != hipSuccess ||
        hipStreamWaitEvent(ctx->stream, ctx->ev_join, 0) != hipSuccess)
      (void)hipStreamSynchronize(ctx->side);
  }
};

// Split-K caps of the W = Q_C^T A sketch.  Its workgroups each fill a CU for
// their whole life; with the FP64 grid capped at three quarters of the CUs
// (split 3 of the 64 column strips' 4), the R-side Cholesky-QR2 that runs
// beside it keeps a quarter of the device instead of queueing behind all of
// W (measured: FP64 CUR 2.53 -> 2.35 ms at 8192^2, k = 256; the FP32 and BF16
// sketches of W gained nothing from a cap).
static constexpr int64_t W_SPLIT_F64 = 3, W_SPLIT_F32 = 16, W_SPLIT_BF16 = 16;

// ---------------------------------------------------------------------------
template <typename TA>
static int cur_impl(rpid_ctx ctx, const TA* A, rpid_dtype a_t, int64_t m, int64_t n, int64_t lda,
                    int64_t k, const int64_t* J, int64_t* I, double* U, int64_t ldu,
                    int64_t* k_eff) {
  const bool f64 = a_t == RPID_F64;
  Carve cv;
  const size_t o_status = cv.take<int64_t>(8);
  const size_t o_C64 = cv.take<double>((size_t)m * k);
  const size_t o_C32 = f64 ? 0 : cv.take<float>((size_t)m * k);
  const size_t o_Lc = cv.take<double>((size_t)m * k);  // LUPP multipliers (discarded)
  const size_t o_Uc = cv.take<double>((size_t)k * k);
  const size_t o_Rt = cv.take<double>((size_t)n * k);
  const size_t o_C2 = cv.take<double>((size_t)m * k);
  const size_t o_Qc = cv.take<double>((size_t)m * k);
  const size_t o_Rt2 = cv.take<double>((size_t)n * k);
  const size_t o_F = cv.take<double>((size_t)4 * k * k);
  const size_t o_Wi = cv.take<double>((size_t)4 * k * k);
  const size_t o_T = cv.take<double>((size_t)3 * k * k);
  const size_t o_W = cv.take<double>((size_t)k * n);
  const size_t o_W2 = cv.take<float>((size_t)2 * k * n);
  const size_t o_Pt = cv.take<char>((size_t)m * 2 * k * 4);
  const size_t o_M = cv.take<double>((size_t)k * k);
  // scratch of the main stream (small GEMM partials, triangular kernels) and
  // of the side stream (the same, and the split-K partials of W's sketch)
  const size_t small_tmp = (size_t)64 * k * k * sizeof(double) + 4096;
  const size_t o_tmp = cv.take<char>(std::max(lupp_workspace_bytes(ctx, m, k, f64 ? 8 : 4), small_tmp));
  const size_t o_tmp2 = cv.off;
  RPID_CHECK(ensure_workspace(ctx, o_tmp2 + std::max(sketch_workspace_bytes(ctx, m, n, 2 * k, 8), small_tmp)));
  int64_t* status_dev = ws_ptr<int64_t>(ctx, o_status);
  double* C64 = ws_ptr<double>(ctx, o_C64);
  double* Rt = ws_ptr<double>(ctx, o_Rt);
  double* F = ws_ptr<double>(ctx, o_F);
  double* Wi = ws_ptr<double>(ctx, o_Wi);
  double* W = ws_ptr<double>(ctx, o_W);
  double* Tc = ws_ptr<double>(ctx, o_T);
  const int64_t kk = k * k;
  double* Tr = Tc + kk;
  double* Y = Tc + 2 * kk;

  // (S5) C = A(:, J)
  RPID_CHECK(launch_fill_u64(ctx, reinterpret_cast<uint64_t*>(I), (size_t)k, 0ull));
  RPID_CHECK(gather_columns<TA, double>(ctx, m, k, A, lda, n, J, C64, m));
  if (!f64) RPID_CHECK(gather_columns<TA, float>(ctx, m, k, A, lda, n, J, ws_ptr<float>(ctx, o_C32), m));

  // The fork point: C is ready.  The row LUPP (a cooperative launch, which
  // cannot start until every compute unit can take one of its workgroups) is
  // enqueued before the side stream's work, so it starts on an idle device
  // and the side's small kernels fit beside it.
  RPID_HIP_CHECK(hipEventRecord(ctx->ev_fork, ctx->stream));

  // (S6) row-wise LUPP on C gives I.  Its status goes to slot 4 and is read
  // with the Cholesky statuses at the end (one host synchronisation per
  // call): after a zero pivot the rest runs on the zero-filled tail of I,
  // which only reads valid rows of A.
  int64_t* lupp_status = status_dev + 4;
  if (f64) {
    RPID_CHECK(lupp_panel<double>(ctx, C64, 1, m, m, k, I, ws_ptr<double>(ctx, o_Lc), m,
                                  ws_ptr<double>(ctx, o_Uc), k, nullptr, o_tmp, lupp_status));
  } else {
    RPID_CHECK(lupp_panel<float>(ctx, ws_ptr<float>(ctx, o_C32), 1, m, m, k, I, ws_ptr<float>(ctx, o_Lc), m,
                                 ws_ptr<float>(ctx, o_Uc), k, nullptr, o_tmp, lupp_status));
  }

  // Side stream: everything that needs C but not I -- Cholesky-QR2 of C
  // (Q_C, the inverses of its two factors, Tc = their product) and
  // W = Q_C^T A -- runs beside the row LUPP.  Only C (read) is shared; the
  // side's regions and scratch are its own.
  RPID_HIP_CHECK(hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0));
  SideJoin side_join(ctx);
  {
    StreamSwap on_side(ctx, ctx->side);
    double* C2 = ws_ptr<double>(ctx, o_C2);
    double* Qc = ws_ptr<double>(ctx, o_Qc);
    RPID_CHECK(chol_qr_one(ctx, m, k, C64, C2, F, Wi, status_dev, o_tmp2));
    RPID_CHECK(chol_qr_one(ctx, m, k, C2, Qc, F + 2 * kk, Wi + 2 * kk, status_dev + 2, o_tmp2));
    RPID_CHECK(dgemm(ctx, false, false, k, k, k, 1.0, Wi, k, Wi + 2 * kk, k, 0.0, Tc, k, o_tmp2));
    // W = Q_C^T A (k x n), in the arithmetic of A's storage
    if (a_t == RPID_F64) {
      RPID_CHECK(sketch_f64(ctx, Qc, m, (const double*)A, lda, m, n, k, W, k, o_tmp2, W_SPLIT_F64));
    } else if (a_t == RPID_F32) {
      float* Pt = ws_ptr<float>(ctx, o_Pt);
      float* W32 = ws_ptr<float>(ctx, o_W2);
      RPID_CHECK(convert_matrix<double, float>(ctx, m, k, Qc, m, Pt, m));
      RPID_CHECK(sketch_f32(ctx, Pt, m, (const float*)A, lda, m, n, k, W32, k, o_tmp2, W_SPLIT_F32));
      RPID_CHECK(convert_matrix<float, double>(ctx, k, n, W32, k, W, k));
    } else {
      uint16_t* Pt = ws_ptr<uint16_t>(ctx, o_Pt);
      float* W2 = ws_ptr<float>(ctx, o_W2);
      RPID_CHECK(split_bf16(ctx, m, k, Qc, m, 2, Pt, m));
      RPID_CHECK(sketch_bf16(ctx, Pt, m, (const uint16_t*)A, lda, m, n, 2 * k, W2, 2 * k, o_tmp2, W_SPLIT_BF16));
      hipLaunchKernelGGL(sum_halves_kernel, dim3(4096), dim3(256), 0, ctx->stream, k, n, W2, W);
      RPID_HIP_CHECK(hipGetLastError());
    }
    RPID_HIP_CHECK(hipEventRecord(ctx->ev_join, ctx->stream));
  }

  // (S7) R^T = A(I, :)^T (n x k), Cholesky-QR2 into Q_R (in Rt), Tr; then,
  // with the side stream joined, M = W Q_R and U = Tc M Tr^T
  // (U = R_C^{-1} (Q_C^T A Q_R) R_R^{-T}, R_C^{-1} = W1c W2c, R_R^{-1} = W1r W2r).
  // A breakdown leaves garbage, never a fault, in what follows; the statuses
  // are checked once at the end.
  RPID_CHECK(gather_rows_t<TA>(ctx, k, n, A, lda, m, I, Rt, n));
  double* Rt2 = ws_ptr<double>(ctx, o_Rt2);
  RPID_CHECK(chol_qr_one(ctx, n, k, Rt, Rt2, F + kk, Wi + kk, status_dev + 1, o_tmp));
  RPID_CHECK(chol_qr_one(ctx, n, k, Rt2, Rt, F + 3 * kk, Wi + 3 * kk, status_dev + 3, o_tmp));
  RPID_CHECK(dgemm(ctx, false, false, k, k, k, 1.0, Wi + kk, k, Wi + 3 * kk, k, 0.0, Tr, k, o_tmp));
  RPID_HIP_CHECK(hipStreamWaitEvent(ctx->stream, ctx->ev_join, 0));
  side_join.joined = true;
  double* M = ws_ptr<double>(ctx, o_M);
  RPID_CHECK(dgemm(ctx, false, false, k, k, n, 1.0, W, k, Rt, n, 0.0, M, k, o_tmp));
  RPID_CHECK(dgemm(ctx, false, false, k, k, k, 1.0, Tc, k, M, k, 0.0, Y, k, o_tmp));
  RPID_CHECK(dgemm(ctx, false, true, k, k, k, 1.0, Y, k, Tr, k, 0.0, U, ldu, o_tmp));
  RPID_HIP_CHECK(hipMemcpyAsync(ctx->host_status, status_dev, 5 * sizeof(int64_t),
                                hipMemcpyDeviceToHost, ctx->stream));
  RPID_HIP_CHECK(hipStreamSynchronize(ctx->stream));
  const int64_t st = ctx->host_status[4];
  if (st < 0) return (int)st;
  if (k_eff) *k_eff = (st == 0) ? k : st - 1;
  if (st > 0) return (int)st;
  for (int b = 0; b < 4; ++b)
    if (ctx->host_status[b] != 0) return RPID_ERR_BREAKDOWN;
  return RPID_OK;
}

// ---------------------------------------------------------------------------
template <typename TA>
static int residual_impl(rpid_ctx ctx, int which, const TA* A, rpid_dtype a_t, int64_t m,
                         int64_t n, int64_t lda, int64_t k, const int64_t* J, const double* Z,
                         int64_t ldz, const int64_t* I, const double* U, int64_t ldu,
                         double* rel_fro, double* sums_dev) {
  const bool bf = a_t == RPID_BF16;
  constexpr int kParts = 3;  // BF16 terms of an FP64 factor
  Carve cv;
  const size_t o_out = cv.take<double>(8);
  const size_t o_P = cv.take<double>((size_t)m * k);
  // Q also holds C = A(:, J) (m x k) before the CUR form's product C U
  const size_t q_elems = (size_t)k * (which == RPID_RESIDUAL_CUR ? std::max(m, n) : n);
  const size_t o_Q = cv.take<double>(q_elems);
  const size_t o_Pb = bf ? cv.take<uint16_t>((size_t)m * kParts * k) : 0;
  const size_t o_Qb = bf ? cv.take<uint16_t>((size_t)kParts * k * n) : 0;
  const size_t o_Qs = bf ? cv.take<uint16_t>((size_t)kParts * k * n) : 0;
  const size_t o_part = cv.take<double>(residual_partials(m, n, bf) + 16);
  const size_t o_tmp = cv.off;
  RPID_CHECK(ensure_workspace(ctx, o_tmp + (size_t)64 * k * k * sizeof(double) + 4096));
  // the two sums land in the caller's device buffer when one is given
  double* out = sums_dev ? sums_dev : ws_ptr<double>(ctx, o_out);
  double* P = ws_ptr<double>(ctx, o_P);
  double* Q = ws_ptr<double>(ctx, o_Q);
  double* part = ws_ptr<double>(ctx, o_part);
  const double* Qp;
  int64_t ldq;
  if (which == RPID_RESIDUAL_ID) {
    // P = C = A(:, J), Q = Z
    if (!bf) RPID_CHECK(gather_columns<TA, double>(ctx, m, k, A, lda, n, J, P, m));
    Qp = Z;
    ldq = ldz;
  } else {
    if (which == RPID_RESIDUAL_CUR) {
      // P = C U, Q = R = A(I, :)
      RPID_CHECK(gather_columns<TA, double>(ctx, m, k, A, lda, n, J, Q, m));  // C into Q scratch
      RPID_CHECK(dgemm(ctx, false, false, m, k, k, 1.0, Q, m, U, ldu, 0.0, P, m, o_tmp));
    } else {
      // row ID: P = Z^T (Z is k x m), Q = R = A(I, :)
      RPID_CHECK(transpose_copy<double>(ctx, k, m, Z, ldz, P, m));
    }
    RPID_CHECK(gather_rows<TA, double>(ctx, k, n, A, lda, m, I, Q, k));
    Qp = Q;
    ldq = k;
  }
  if (!bf) {
    RPID_CHECK(residual_f64<TA>(ctx, m, n, k, A, lda, P, m, Qp, ldq, part, out));
  } else {
    // BF16 storage: the BF16 factor (C or R) is exact; the FP64 factor (Z or
    // C U) is split into kParts BF16 terms along r.
    // Pb is the k-contiguous (kParts k x m) transpose of P' = [P_0 .. P_{kParts-1}]
    uint16_t* Pb = ws_ptr<uint16_t>(ctx, o_Pb);
    uint16_t* Qb = ws_ptr<uint16_t>(ctx, o_Qb);
    if (which == RPID_RESIDUAL_ID) {
      RPID_CHECK(pack_cols_t(ctx, m, k, kParts, (const uint16_t*)A, lda, n, J, Pb));
      // Q' (kParts k x n): rows [p k, (p+1) k) hold term p of Z
      uint16_t* Qs = ws_ptr<uint16_t>(ctx, o_Qs);
      RPID_CHECK(split_bf16(ctx, k, n, Qp, ldq, kParts, Qs, k));  // k x (kParts n)
      // restack: term p block (k x n at column offset p n) -> rows p k of Qb
      for (int p = 0; p < kParts; ++p)
        RPID_CHECK(convert_matrix<uint16_t, uint16_t>(ctx, k, n, Qs + (int64_t)p * n * k, k,
                                                      Qb + (int64_t)p * k, kParts * k));
    } else {
      RPID_CHECK(pack_split_t(ctx, m, k, kParts, P, m, Pb));
      for (int p = 0; p < kParts; ++p)
        RPID_CHECK(gather_rows<TA, uint16_t>(ctx, k, n, A, lda, m, I, Qb + (int64_t)p * k,
                                             kParts * k));
    }
    RPID_CHECK(residual_bf16(ctx, m, n, kParts * k, (const uint16_t*)A, lda, Pb, kParts * k, Qb,
                             kParts * k, part, out));
  }
  if (sums_dev) return RPID_OK;
  double h[2];
  RPID_CHECK(read_doubles(ctx, out, h, 2));
  *rel_fro = (h[1] > 0.0) ? sqrt(h[0] / h[1]) : 0.0;
  return RPID_OK;
}

// ---------------------------------------------------------------------------
// Fixed scratch of the allocation-free sketch entry point: the packed Omega^T
// and the split-K partial sums live here instead of in the context's
// workspace.  Each device holds its own copy; host code reaches it only
// through the address hipGetSymbolAddress returns on that device (the
// array's name is a host-side stand-in).  Every call on a device shares it.
static constexpr size_t kFixedScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kFixedScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_addr;  // by device; null until looked up
}  // namespace

// This device's scratch address, looked up once per device (the device must
// be current).
static int fixed_scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_addr.size() <= device) g_scratch_addr.resize(device + 1, nullptr);
  if (!g_scratch_addr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return RPID_ERR_HIP;
    g_scratch_addr[device] = p;
  }
  *out = g_scratch_addr[device];
  return RPID_OK;
}

// Points the context's workspace at another buffer for the length of one
// call (the carving helpers read ctx->ws / ctx->ws_bytes) and restores it.
struct WorkspaceSwap {
  rpid_ctx c;
  void* ws;
  size_t bytes;
  WorkspaceSwap(rpid_ctx ctx, void* p, size_t b) : c(ctx), ws(ctx->ws), bytes(ctx->ws_bytes) {
    c->ws = p;
    c->ws_bytes = b;
  }
  ~WorkspaceSwap() {
    c->ws = ws;
    c->ws_bytes = bytes;
  }
};

// X = Omega A (Alg. 2, step 2).  With `fixed` the call takes its scratch from
// the device's fixed array (no allocation; inputs whose packed Omega^T does
// not fit are refused, and the split-K count is capped so that the partial
// sums fit), otherwise from the context's growable workspace.
static int sketch_entry(rpid_ctx ctx, const void* A, rpid_dtype a_t, int64_t m, int64_t n,
                        int64_t lda, const void* Omega, rpid_dtype o_t, int64_t l, int64_t ldo,
                        void* X, rpid_dtype x_t, int64_t ldx, bool fixed) {
  if (!ctx) return -1;
  if (!A) return -2;
  if (m < 1) return -4;
  if (n < 1) return -5;
  if (lda < m) return -6;
  if (!Omega) return -7;
  if (l < 1 || l > 1024) return -9;
  if (ldo < l) return -10;
  if (!X) return -11;
  if (ldx < l) return -13;
  const bool f64 = a_t == RPID_F64 && o_t == RPID_F64 && x_t == RPID_F64;
  const bool f32 = a_t == RPID_F32 && o_t == RPID_F32 && x_t == RPID_F32;
  const bool bf = a_t == RPID_BF16 && o_t == RPID_BF16 && x_t == RPID_F32;
  if (!(f64 || f32 || bf)) return RPID_ERR_UNSUPPORTED;
  const size_t es = esize(a_t);
  const size_t acc = f64 ? 8 : 4;
  Carve cv;
  const size_t o_pt = cv.take<char>((size_t)m * l * es + 64);
  const size_t ws_sk = cv.off;
  int64_t max_split = 16;
  if (fixed) {
    if (!ctx->fixed_scratch) return RPID_ERR_HIP;
    if (ws_sk + 512 > kFixedScratchBytes) return RPID_ERR_SCRATCH;
    // partial sums start at the next 256-byte boundary
    const size_t room = kFixedScratchBytes - ((ws_sk + 255) & ~(size_t)255);
    const int64_t fit = (int64_t)(room / ((size_t)l * n * acc));
    max_split = fit < 1 ? 1 : (fit > 16 ? 16 : fit);
  }
  RPID_HIP_CHECK(hipSetDevice(ctx->device));
  if (!fixed) RPID_CHECK(ensure_workspace(ctx, ws_sk + sketch_workspace_bytes(ctx, m, n, l, (int)acc)));
  WorkspaceSwap swap(ctx, fixed ? ctx->fixed_scratch : ctx->ws,
                     fixed ? kFixedScratchBytes : ctx->ws_bytes);
  // Pt = Omega^T, m x l column-major (rows of Omega contiguous)
  if (f64) {
    double* Pt = ws_ptr<double>(ctx, o_pt);
    RPID_CHECK(transpose_copy<double>(ctx, l, m, (const double*)Omega, ldo, Pt, m));
    return sketch_f64(ctx, Pt, m, (const double*)A, lda, m, n, l, (double*)X, ldx, ws_sk, max_split);
  }
  if (f32) {
    float* Pt = ws_ptr<float>(ctx, o_pt);
    RPID_CHECK(transpose_copy<float>(ctx, l, m, (const float*)Omega, ldo, Pt, m));
    return sketch_f32(ctx, Pt, m, (const float*)A, lda, m, n, l, (float*)X, ldx, ws_sk, max_split);
  }
  uint16_t* Pt = ws_ptr<uint16_t>(ctx, o_pt);
  RPID_CHECK(transpose_copy<uint16_t>(ctx, l, m, (const uint16_t*)Omega, ldo, Pt, m));
  return sketch_bf16(ctx, Pt, m, (const uint16_t*)A, lda, m, n, l, (float*)X, ldx, ws_sk,
                     max_split);
}

}  // namespace rpid

using namespace rpid;

extern "C" {

int rpid_version(void) { return 1; }

const char* rpid_status_string(int s) {
  if (s == RPID_OK) return "ok";
  if (s > 0) return "exactly zero pivot (rank deficiency); status-1 pivots are defined";
  switch (s) {
    case RPID_ERR_NONFINITE: return "non-finite entry in a matrix handed to pivoting";
    case RPID_ERR_HIP: return "HIP runtime call failed";
    case RPID_ERR_NOMEM: return "workspace allocation failed";
    case RPID_ERR_UNSUPPORTED: return "dtype combination or size not supported";
    case RPID_ERR_LAUNCH: return "cooperative launch could not co-schedule the grid";
    case RPID_ERR_TIMEOUT: return "device-side wait exceeded its spin limit";
    case RPID_ERR_BREAKDOWN: return "Cholesky breakdown while orthonormalising C or R^T";
    case RPID_ERR_SCRATCH: return "input larger than the fixed scratch of the allocation-free call";
    default: return "invalid argument (status = -position)";
  }
}

int rpid_create(rpid_ctx* out, int device, void* hip_stream) {
  if (!out) return -1;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return RPID_ERR_HIP;
  if (device < 0 || device >= ndev) return -2;
  RPID_HIP_CHECK(hipSetDevice(device));
  rpid_ctx c = new (std::nothrow) rpid_ctx_s();
  if (!c) return RPID_ERR_NOMEM;
  c->device = device;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    delete c;
    return RPID_ERR_HIP;
  }
  c->num_cu = prop.multiProcessorCount;
  if (hipHostMalloc((void**)&c->host_status, 64, hipHostMallocDefault) != hipSuccess) {
    delete c;
    return RPID_ERR_HIP;
  }
  if (fixed_scratch_address(device, &c->fixed_scratch) != RPID_OK) {
    (void)hipHostFree(c->host_status);
    delete c;
    return RPID_ERR_HIP;
  }
  if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
    rpid_destroy(c);
    return RPID_ERR_HIP;
  }
  *out = c;
  return RPID_OK;
}

int rpid_destroy(rpid_ctx ctx) {
  if (!ctx) return -1;
  // every release is attempted; the first failure is reported.  The uncached
  // exchange buffer goes back to the device's pool and stays allocated until
  // the process ends (device memory of that kind is never freed once a kernel
  // has read it).
  hipError_t e = hipSetDevice(ctx->device);
  const hipError_t e1 = hipStreamSynchronize(ctx->stream);
  if (e == hipSuccess) e = e1;
  if (e1 == hipSuccess) release_exchange_buffer(ctx);
  if (ctx->ws) {
    const hipError_t e2 = hipFree(ctx->ws);
    if (e == hipSuccess) e = e2;
  }
  if (ctx->host_status) {
    const hipError_t e3 = hipHostFree(ctx->host_status);
    if (e == hipSuccess) e = e3;
  }
  if (ctx->side) {
    const hipError_t e4 = hipStreamSynchronize(ctx->side);
    const hipError_t e5 = hipStreamDestroy(ctx->side);
    if (e == hipSuccess) e = e4 != hipSuccess ? e4 : e5;
  }
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  delete ctx;
  return e == hipSuccess ? RPID_OK : RPID_ERR_HIP;
}

int rpid_set_stream(rpid_ctx ctx, void* hip_stream) {
  if (!ctx) return -1;
  ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return RPID_OK;
}

// ---------------------------------------------------------------------------
int rpid_sketch(rpid_ctx ctx, const void* A, rpid_dtype a_t, int64_t m, int64_t n, int64_t lda,
                const void* Omega, rpid_dtype o_t, int64_t l, int64_t ldo, void* X, rpid_dtype x_t,
                int64_t ldx) {
  return sketch_entry(ctx, A, a_t, m, n, lda, Omega, o_t, l, ldo, X, x_t, ldx, false);
}

int rpid_sketch_noalloc(rpid_ctx ctx, const void* A, rpid_dtype a_t, int64_t m, int64_t n,
                        int64_t lda, const void* Omega, rpid_dtype o_t, int64_t l, int64_t ldo,
                        void* X, rpid_dtype x_t, int64_t ldx) {
  return sketch_entry(ctx, A, a_t, m, n, lda, Omega, o_t, l, ldo, X, x_t, ldx, true);
}

int rpid_sketch_fp8(rpid_ctx ctx, const float* A, int64_t m, int64_t n, int64_t lda,
                    const float* Omega, int64_t l, int64_t ldo, float* X, int64_t ldx) {
  if (!ctx) return -1;
  if (!A) return -2;
  if (m < 1) return -3;
  if (n < 1) return -4;
  if (lda < m) return -5;
  if (!Omega) return -6;
  if (l < 1 || l > 1024) return -7;
  if (ldo < l) return -8;
  if (!X) return -9;
  if (ldx < l) return -10;
  RPID_HIP_CHECK(hipSetDevice(ctx->device));
  const int64_t mq = (m + 511) / 512 * 512;
  RPID_CHECK(ensure_workspace(ctx, sketch_fp8_workspace(m, n, l) +
                                       sketch_workspace_bytes(ctx, mq, n, l, 4)));
  return sketch_fp8(ctx, A, m, n, lda, Omega, l, ldo, X, ldx, 0);
}

// ---------------------------------------------------------------------------
// Sketch with one plain power iteration (eq. def_power_iter, q = 1):
// Y^T = Omega A^T, then X = Y^T A.  Both products run on the sketch kernels,
// whose contraction runs along the contiguous dimension of the right factor:
// A^T is formed once (n x m), and Y^T becomes the left factor of the second
// product.  In the BF16 form Y^T (FP32) enters the second product as two
// BF16 terms (its rounding and the rounding of the remainder), stacked as
// 2 l rows whose two halves are added afterwards.
namespace {

__device__ __forceinline__ uint16_t bf16_rne_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// P (m x 2l, ldp): P(i, r) = hi(Y^T(r, i)), P(i, l + r) = lo(Y^T(r, i)) with
// hi + lo the two-term BF16 split of the FP32 value (32 x 32 LDS tiles)
__global__ __launch_bounds__(256) void split_t_bf16_kernel(int64_t l, int64_t m, const float* Yt,
                                                           int64_t ldy, uint16_t* P, int64_t ldp) {
  __shared__ float tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.y * 32, i0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t r = r0 + tx, i = i0 + yy;
    tile[yy][tx] = (r < l && i < m) ? Yt[r + i * ldy] : 0.0f;
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t i = i0 + tx, r = r0 + yy;
    if (r < l && i < m) {
      const float y = tile[tx][yy];
      const uint16_t hi = bf16_rne_bits(y);
      const uint16_t lo = bf16_rne_bits(y - __uint_as_float((uint32_t)hi << 16));
      P[i + r * ldp] = hi;
      P[i + (l + r) * ldp] = lo;
    }
  }
}

// X(r, j) = X2(r, j) + X2(l + r, j)
__global__ void add_halves_f32_kernel(int64_t l, int64_t n, const float* X2, int64_t ld2, float* X,
                                      int64_t ldx) {
  const int64_t total = l * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e % l, j = e / l;
    X[r + j * ldx] = X2[r + j * ld2] + X2[l + r + j * ld2];
  }
}

// X(r, j) = sum_b parts[b](r, j) in block order (parts: nb x l x n, FP32)
__global__ void sum_blocks_f32_kernel(int nb, int64_t l, int64_t n, const float* parts, float* X,
                                      int64_t ldx) {
  const int64_t total = l * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    float s = parts[e];
    for (int b = 1; b < nb; ++b) s += parts[(int64_t)b * total + e];
    X[e % l + (e / l) * ldx] = s;
  }
}

// U(:, J[t]) = P(:, t), k x k
__global__ void scatter_cols_f64_kernel(int64_t k, const double* P, const int64_t* J, double* U,
                                        int64_t ldu) {
  const int64_t total = k * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e % k, t = e / k;
    const int64_t j = J[t];
    if (j >= 0 && j < k) U[r + j * ldu] = P[e];
  }
}

}  // namespace

// Shapes and alignments for which the BF16 transposed-A sketch runs (the
// kernel checks them again and reports RPID_ERR_UNSUPPORTED otherwise).
static bool at_bf16_fits(const void* A, int64_t m, int64_t n, int64_t lda, int64_t l) {
  return ((uintptr_t)A % 16 == 0) && (lda * 2) % 16 == 0 && n % 64 == 0 && m % 8 == 0 &&
         64 * lda * 2 + m * 2 < ((int64_t)1 << 31) && l * n * 2 < ((int64_t)1 << 31) && l <= 1024;
}

int rpid_sketch_power1(rpid_ctx ctx, const void* A, rpid_dtype a_t, int64_t m, int64_t n,
                       int64_t lda, const void* Omega, rpid_dtype o_t, int64_t l, int64_t ldo,
                       void* X, rpid_dtype x_t, int64_t ldx) {
  if (!ctx) return -1;
  if (!A) return -2;
  if (m < 1) return -4;
  if (n < 1) return -5;
  if (lda < m) return -6;
  if (!Omega) return -7;
  if (l < 1 || l > 512) return -9;
  if (ldo < l) return -10;
  if (!X) return -11;
  if (ldx < l) return -13;
  const bool f64 = a_t == RPID_F64 && o_t == RPID_F64 && x_t == RPID_F64;
  const bool f32 = a_t == RPID_F32 && o_t == RPID_F32 && x_t == RPID_F32;
  const bool bf = a_t == RPID_BF16 && o_t == RPID_BF16 && x_t == RPID_F32;
  if (!(f64 || f32 || bf)) return RPID_ERR_UNSUPPORTED;
  RPID_HIP_CHECK(hipSetDevice(ctx->device));
  const size_t es = esize(a_t);
  const size_t acc = f64 ? 8 : 4;
  const int64_t l2 = bf ? 2 * l : l;  // rows of the second product's left factor
  Carve cv;
  const bool in_place = bf && at_bf16_fits(A, m, n, lda, l);
  const size_t o_at = in_place ? 0 : cv.take<char>((size_t)m * n * es);
  const size_t o_p1 = cv.take<char>((size_t)n * l * es);
  const size_t o_yt = cv.take<char>((size_t)l * m * acc);
  const size_t o_p2 = cv.take<char>((size_t)m * l2 * es);
  const size_t o_x2 = bf ? cv.take<float>((size_t)l2 * n) : 0;
  const size_t ws_sk = cv.off;
  RPID_CHECK(ensure_workspace(ctx, ws_sk + std::max(sketch_workspace_bytes(ctx, n, m, l, (int)acc),
                                                    sketch_workspace_bytes(ctx, m, n, l2, (int)acc))));
  char* at = ws_ptr<char>(ctx, o_at);
  char* p1 = ws_ptr<char>(ctx, o_p1);
  char* yt = ws_ptr<char>(ctx, o_yt);
  char* p2 = ws_ptr<char>(ctx, o_p2);
  if (f64) {
    RPID_CHECK(transpose_copy<double>(ctx, m, n, (const double*)A, lda, (double*)at, n));
    RPID_CHECK(transpose_copy<double>(ctx, l, n, (const double*)Omega, ldo, (double*)p1, n));
    RPID_CHECK(sketch_f64(ctx, (const double*)p1, n, (const double*)at, n, n, m, l, (double*)yt, l, ws_sk));
    RPID_CHECK(transpose_copy<double>(ctx, l, m, (const double*)yt, l, (double*)p2, m));
    return sketch_f64(ctx, (const double*)p2, m, (const double*)A, lda, m, n, l, (double*)X, ldx, ws_sk);
  }
  if (f32) {
    RPID_CHECK(transpose_copy<float>(ctx, m, n, (const float*)A, lda, (float*)at, n));
    RPID_CHECK(transpose_copy<float>(ctx, l, n, (const float*)Omega, ldo, (float*)p1, n));
    RPID_CHECK(sketch_f32(ctx, (const float*)p1, n, (const float*)at, n, n, m, l, (float*)yt, l, ws_sk));
    RPID_CHECK(transpose_copy<float>(ctx, l, m, (const float*)yt, l, (float*)p2, m));
    return sketch_f32(ctx, (const float*)p2, m, (const float*)A, lda, m, n, l, (float*)X, ldx, ws_sk);
  }
  RPID_CHECK(transpose_copy<uint16_t>(ctx, l, n, (const uint16_t*)Omega, ldo, (uint16_t*)p1, n));
  if (at_bf16_fits(A, m, n, lda, l)) {
    // Y^T = Omega A^T straight from A
    RPID_CHECK(sketch_at_bf16(ctx, (const uint16_t*)p1, n, (const uint16_t*)A, lda, m, n, l, (float*)yt, l,
                              ws_sk));
  } else {
    RPID_CHECK(transpose_copy<uint16_t>(ctx, m, n, (const uint16_t*)A, lda, (uint16_t*)at, n));
    RPID_CHECK(sketch_bf16(ctx, (const uint16_t*)p1, n, (const uint16_t*)at, n, n, m, l, (float*)yt, l, ws_sk));
  }
  dim3 grid((unsigned)((m + 31) / 32), (unsigned)((l + 31) / 32));
  hipLaunchKernelGGL(split_t_bf16_kernel, grid, dim3(256), 0, ctx->stream, l, m, (const float*)yt, l,
                     (uint16_t*)p2, m);
  RPID_HIP_CHECK(hipGetLastError());
  float* x2 = ws_ptr<float>(ctx, o_x2);
  RPID_CHECK(sketch_bf16(ctx, (const uint16_t*)p2, m, (const uint16_t*)A, lda, m, n, l2, x2, l2, ws_sk));
  int64_t blocks = (l * n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(add_halves_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, l, n, x2,
                     l2, (float*)X, ldx);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

// ---------------------------------------------------------------------------
int rpid_sketch_two_sided(rpid_ctx ctx, const void* A, rpid_dtype a_t, int64_t m, int64_t n,
                          int64_t lda, const void* Gamma, int64_t ldg, const void* Omega,
                          int64_t ldo, int64_t l, void* X, int64_t ldx, void* Yt, int64_t ldyt,
                          rpid_dtype out_t) {
  if (!ctx) return -1;
  if (!A) return -2;
  if (!(a_t == RPID_F64 || a_t == RPID_F32 || a_t == RPID_BF16)) return -3;
  if (m < 1) return -4;
  if (n < 1) return -5;
  if (lda < m) return -6;
  if (!Gamma) return -7;
  if (ldg < l) return -8;
  if (!Omega) return -9;
  if (ldo < l) return -10;
  if (l < 1 || l > 1024) return -11;
  if (!X) return -12;
  if (ldx < l) return -13;
  if (!Yt) return -14;
  if (ldyt < l) return -15;
  if (out_t != (a_t == RPID_F64 ? RPID_F64 : RPID_F32)) return -16;
  RPID_HIP_CHECK(hipSetDevice(ctx->device));
  const size_t es = esize(a_t);
  const int acc = a_t == RPID_F64 ? 8 : 4;
  const bool in_place = a_t == RPID_BF16 && at_bf16_fits(A, m, n, lda, l);
  // Row blocks of A small enough to stay in the 256 MB last-level cache
  // between the two products of a block (128 MiB, a multiple of 64 rows).
  int64_t mb = m;
  if (in_place) {
    mb = ((int64_t)128 << 20) / (n * 2);
    mb = std::max<int64_t>(64, mb / 64 * 64);
    if (mb >= m) mb = m;
  }
  const int64_t nb = (m + mb - 1) / mb;
  Carve cv;
  const size_t o_gt = cv.take<char>((size_t)m * l * es);
  const size_t o_ot = cv.take<char>((size_t)n * l * es);
  const size_t o_at = in_place ? 0 : cv.take<char>((size_t)m * n * es);
  const size_t o_parts = nb > 1 ? cv.take<float>((size_t)nb * l * n) : 0;
  const size_t ws_sk = cv.off;
  RPID_CHECK(ensure_workspace(ctx, ws_sk + std::max(sketch_workspace_bytes(ctx, m, n, l, acc),
                                                    sketch_workspace_bytes(ctx, n, m, l, acc))));
  char* gt = ws_ptr<char>(ctx, o_gt);
  char* ot = ws_ptr<char>(ctx, o_ot);
  char* at = ws_ptr<char>(ctx, o_at);
  if (a_t == RPID_F64) {
    RPID_CHECK(transpose_copy<double>(ctx, l, m, (const double*)Gamma, ldg, (double*)gt, m));
    RPID_CHECK(transpose_copy<double>(ctx, l, n, (const double*)Omega, ldo, (double*)ot, n));
    RPID_CHECK(sketch_f64(ctx, (const double*)gt, m, (const double*)A, lda, m, n, l, (double*)X, ldx, ws_sk));
    RPID_CHECK(transpose_copy<double>(ctx, m, n, (const double*)A, lda, (double*)at, n));
    return sketch_f64(ctx, (const double*)ot, n, (const double*)at, n, n, m, l, (double*)Yt, ldyt, ws_sk);
  }
  if (a_t == RPID_F32) {
    RPID_CHECK(transpose_copy<float>(ctx, l, m, (const float*)Gamma, ldg, (float*)gt, m));
    RPID_CHECK(transpose_copy<float>(ctx, l, n, (const float*)Omega, ldo, (float*)ot, n));
    RPID_CHECK(sketch_f32(ctx, (const float*)gt, m, (const float*)A, lda, m, n, l, (float*)X, ldx, ws_sk));
    RPID_CHECK(transpose_copy<float>(ctx, m, n, (const float*)A, lda, (float*)at, n));
    return sketch_f32(ctx, (const float*)ot, n, (const float*)at, n, n, m, l, (float*)Yt, ldyt, ws_sk);
  }
  const uint16_t* Ab = (const uint16_t*)A;
  RPID_CHECK(transpose_copy<uint16_t>(ctx, l, m, (const uint16_t*)Gamma, ldg, (uint16_t*)gt, m));
  RPID_CHECK(transpose_copy<uint16_t>(ctx, l, n, (const uint16_t*)Omega, ldo, (uint16_t*)ot, n));
  if (!in_place) {
    RPID_CHECK(sketch_bf16(ctx, (const uint16_t*)gt, m, Ab, lda, m, n, l, (float*)X, ldx, ws_sk));
    RPID_CHECK(transpose_copy<uint16_t>(ctx, m, n, Ab, lda, (uint16_t*)at, n));
    return sketch_bf16(ctx, (const uint16_t*)ot, n, (const uint16_t*)at, n, n, m, l, (float*)Yt, ldyt, ws_sk);
  }
  // one pass over A: each row block feeds both products back to back
  float* parts = nb > 1 ? ws_ptr<float>(ctx, o_parts) : nullptr;
  for (int64_t b = 0; b < nb; ++b) {
    const int64_t i0 = b * mb, mi = std::min(mb, m - i0);
    float* xo = nb > 1 ? parts + b * l * n : (float*)X;
    const int64_t ldxo = nb > 1 ? l : ldx;
    RPID_CHECK(sketch_bf16(ctx, (const uint16_t*)gt + i0, m, Ab + i0, lda, mi, n, l, xo, ldxo, ws_sk));
    RPID_CHECK(sketch_at_bf16(ctx, (const uint16_t*)ot, n, Ab + i0, lda, mi, n, l, (float*)Yt + i0 * ldyt,
                              ldyt, ws_sk));
  }
  if (nb > 1) {
    int64_t blocks = std::min<int64_t>((l * n + 255) / 256, 8192);
    hipLaunchKernelGGL(sum_blocks_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, (int)nb, l,
                       n, parts, (float*)X, ldx);
    RPID_HIP_CHECK(hipGetLastError());
  }
  return RPID_OK;
}

int rpid_cur_sketch(rpid_ctx ctx, const void* A, rpid_dtype a_t, int64_t m, int64_t n, int64_t lda,
                    int64_t k, const int64_t* J, const int64_t* I, double* U, int64_t ldu) {
  if (!ctx) return -1;
  if (!A) return -2;
  if (!(a_t == RPID_F64 || a_t == RPID_F32 || a_t == RPID_BF16)) return -3;
  if (m < 1) return -4;
  if (n < 1) return -5;
  if (lda < m) return -6;
  if (k < 1 || k > m || k > n || k > 1024) return -7;
  if (!J) return -8;
  if (!I) return -9;
  if (!U) return -10;
  if (ldu < k) return -11;
  RPID_HIP_CHECK(hipSetDevice(ctx->device));
  Carve cv;
  const size_t o_status = cv.take<int64_t>(8);
  const size_t o_C = cv.take<double>((size_t)m * k);
  const size_t o_S = cv.take<double>((size_t)k * k);
  const size_t o_Jp = cv.take<int64_t>((size_t)k);
  const size_t o_L = cv.take<double>((size_t)k * k);
  const size_t o_Uf = cv.take<double>((size_t)k * k);
  const size_t o_dg = cv.take<double>((size_t)k);
  const size_t o_LJ = cv.take<double>((size_t)k * k);
  const size_t o_W = cv.take<double>((size_t)k * k);
  const size_t o_WU = cv.take<double>((size_t)k * k);
  const size_t o_P = cv.take<double>((size_t)k * k);
  const size_t o_lupp = cv.off;
  const size_t o_tmp = o_lupp + lupp_workspace_bytes(ctx, k, k, 8);
  RPID_CHECK(ensure_workspace(ctx, o_tmp + (size_t)64 * k * k * sizeof(double) + 4096));
  int64_t* status_dev = ws_ptr<int64_t>(ctx, o_status);
  double* C = ws_ptr<double>(ctx, o_C);
  double* S = ws_ptr<double>(ctx, o_S);
  int64_t* Jp = ws_ptr<int64_t>(ctx, o_Jp);
  double* L = ws_ptr<double>(ctx, o_L);
  double* Uf = ws_ptr<double>(ctx, o_Uf);
  double* LJ = ws_ptr<double>(ctx, o_LJ);
  double* W = ws_ptr<double>(ctx, o_W);
  double* WU = ws_ptr<double>(ctx, o_WU);
  double* P = ws_ptr<double>(ctx, o_P);
  // S = A(I, J) in FP64
  switch (a_t) {
    case RPID_F64: RPID_CHECK(gather_columns<double, double>(ctx, m, k, (const double*)A, lda, n, J, C, m)); break;
    case RPID_F32: RPID_CHECK(gather_columns<float, double>(ctx, m, k, (const float*)A, lda, n, J, C, m)); break;
    default: RPID_CHECK(gather_columns<uint16_t, double>(ctx, m, k, (const uint16_t*)A, lda, n, J, C, m)); break;
  }
  RPID_CHECK(gather_rows<double, double>(ctx, k, k, C, m, m, I, S, k));
  // row LUPP of S: S(Jp, :) = L(Jp, :) U', so S^{-1}(:, Jp[t]) = (U'^{-1} L(Jp, :)^{-1})(:, t)
  RPID_CHECK(lupp_panel<double>(ctx, S, 1, k, k, k, Jp, L, k, Uf, k, ws_ptr<double>(ctx, o_dg), o_lupp,
                                status_dev));
  int64_t st = 0;
  RPID_CHECK(read_status(ctx, status_dev, &st));
  if (st != 0) return (int)st;
  RPID_CHECK(gather_rows<double, double>(ctx, k, k, L, k, k, Jp, LJ, k));
  RPID_CHECK(tri_inverse(ctx, k, LJ, k, true, true, W, k, o_tmp));
  RPID_CHECK(tri_inverse(ctx, k, Uf, k, false, false, WU, k, o_tmp));
  RPID_CHECK(dgemm(ctx, false, false, k, k, k, 1.0, WU, k, W, k, 0.0, P, k, o_tmp));
  const int64_t blocks = std::min<int64_t>((k * k + 255) / 256, 1024);
  hipLaunchKernelGGL(scatter_cols_f64_kernel, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, k, P, Jp, U,
                     ldu);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

// ---------------------------------------------------------------------------
// The column LUPP of rpid_select_columns and rpid_select_columns_async: the
// status goes to status_ext (a caller's device word) when given, else to the
// workspace, from where it is read back only if k_eff is given.
static int select_columns_impl(rpid_ctx ctx, const void* X, rpid_dtype x_t, int64_t l, int64_t n,
                               int64_t ldx, int64_t k, int64_t* J, void* Lf, int64_t ldl, void* Uf,
                               int64_t ldu, void* diagU, int64_t* k_eff, int64_t* status_ext) {
  if (!ctx) return -1;
  if (!X) return -2;
  if (!is_lupp_type(x_t)) return -3;
  if (l < 1) return -4;
  if (n < 1) return -5;
  if (ldx < l) return -6;
  if (k < 1 || k > l || k > n || k > 1024) return -7;
  if (!J) return -8;
  if (!Lf) return -9;
  if (ldl < n) return -10;
  if (!Uf) return -11;
  if (ldu < k) return -12;
  RPID_HIP_CHECK(hipSetDevice(ctx->device));
  const int es = (int)esize(x_t);
  Carve cv;
  const size_t o_status = cv.take<int64_t>(8);
  const size_t o_lupp = cv.off;
  RPID_CHECK(ensure_workspace(ctx, o_lupp + lupp_workspace_bytes(ctx, n, k, es)));
  int64_t* status_dev = status_ext ? status_ext : ws_ptr<int64_t>(ctx, o_status);
  // Xᵀ panel: P(i, j) = X[j + i * ldx]
  int s;
  if (x_t == RPID_F64)
    s = lupp_panel<double>(ctx, (const double*)X, ldx, 1, n, k, J, (double*)Lf, ldl, (double*)Uf,
                           ldu, (double*)diagU, o_lupp, status_dev);
  else
    s = lupp_panel<float>(ctx, (const float*)X, ldx, 1, n, k, J, (float*)Lf, ldl, (float*)Uf, ldu,
                          (float*)diagU, o_lupp, status_dev);
  if (s != RPID_OK) return s;
  if (!k_eff) return RPID_OK;
  int64_t st = 0;
  RPID_CHECK(read_status(ctx, status_dev, &st));
  if (st < 0) return (int)st;
  *k_eff = (st == 0) ? k : st - 1;
  return (int)st;
}

int rpid_select_columns(rpid_ctx ctx, const void* X, rpid_dtype x_t, int64_t l, int64_t n,
                        int64_t ldx, int64_t k, int64_t* J, void* Lf, int64_t ldl, void* Uf,
                        int64_t ldu, void* diagU, int64_t* k_eff) {
  return select_columns_impl(ctx, X, x_t, l, n, ldx, k, J, Lf, ldl, Uf, ldu, diagU, k_eff, nullptr);
}

int rpid_select_columns_async(rpid_ctx ctx, const void* X, rpid_dtype x_t, int64_t l, int64_t n,
                              int64_t ldx, int64_t k, int64_t* J, void* Lf, int64_t ldl, void* Uf,
                              int64_t ldu, void* diagU, int64_t* status_dev) {
  if (!status_dev) return -14;
  return select_columns_impl(ctx, X, x_t, l, n, ldx, k, J, Lf, ldl, Uf, ldu, diagU, nullptr,
                             status_dev);
}

// ---------------------------------------------------------------------------
int rpid_sketch_sparse_sign(rpid_ctx ctx, const void* A, rpid_dtype a_t, int64_t m, int64_t n,
                            int64_t lda, const int32_t* rows, const int8_t* signs, int64_t zeta,
                            int64_t l, double scale, void* X, rpid_dtype x_t, int64_t ldx) {
  if (!ctx) return -1;
  if (!A) return -2;
  if (m < 1) return -4;
  if (n < 1) return -5;
  if (lda < m) return -6;
  if (!rows) return -7;
  if (!signs) return -8;
  if (zeta < 1 || zeta > 64 || zeta > l) return -9;
  if (l < 1 || l > 1024) return -10;
  if (!(scale > 0.0) || !std::isfinite(scale)) return -11;
  if (!X) return -12;
  if (ldx < l) return -14;
  const bool f64 = a_t == RPID_F64 && x_t == RPID_F64;
  const bool f32 = a_t == RPID_F32 && x_t == RPID_F32;
  const bool bf = a_t == RPID_BF16 && x_t == RPID_F32;
  if (!(f64 || f32 || bf)) return RPID_ERR_UNSUPPORTED;
  RPID_HIP_CHECK(hipSetDevice(ctx->device));
  Carve cv;
  const size_t o_pt = cv.take<char>((size_t)m * l * esize(a_t));
  const size_t ws_sk = cv.off;
  RPID_CHECK(ensure_workspace(ctx, ws_sk + sketch_workspace_bytes(ctx, m, n, l, f64 ? 8 : 4)));
  // the embedding's transpose (m x l, exact +-1 entries) feeds the dense sketch
  if (f64) {
    double* pt = ws_ptr<double>(ctx, o_pt);
    RPID_CHECK(expand_sparse_sign<double>(ctx, m, l, (int)zeta, rows, signs, pt, m, 1, true));
    RPID_CHECK(sketch_f64(ctx, pt, m, (const double*)A, lda, m, n, l, (double*)X, ldx, ws_sk));
    return scale_matrix<double>(ctx, l, n, (double*)X, ldx, scale);
  }
  if (f32) {
    float* pt = ws_ptr<float>(ctx, o_pt);
    RPID_CHECK(expand_sparse_sign<float>(ctx, m, l, (int)zeta, rows, signs, pt, m, 1, true));
    RPID_CHECK(sketch_f32(ctx, pt, m, (const float*)A, lda, m, n, l, (float*)X, ldx, ws_sk));
    return scale_matrix<float>(ctx, l, n, (float*)X, ldx, (float)scale);
  }
  uint16_t* pt = ws_ptr<uint16_t>(ctx, o_pt);
  RPID_CHECK(expand_sparse_sign<uint16_t>(ctx, m, l, (int)zeta, rows, signs, pt, m, 1, true));
  RPID_CHECK(sketch_bf16(ctx, pt, m, (const uint16_t*)A, lda, m, n, l, (float*)X, ldx, ws_sk));
  return scale_matrix<float>(ctx, l, n, (float*)X, ldx, (float)scale);
}

int rpid_sketch_srtt(rpid_ctx ctx, const void* A, rpid_dtype a_t, int64_t m, int64_t n, int64_t lda,
                     const int32_t* perm, const int8_t* phi, const int32_t* sel, int64_t l, void* X,
                     rpid_dtype x_t, int64_t ldx) {
  if (!ctx) return -1;
  if (!A) return -2;
  if (m < 1) return -4;
  if (n < 1) return -5;
  if (lda < m) return -6;
  if (!perm) return -7;
  if (!phi) return -8;
  if (!sel) return -9;
  if (l < 1 || l > 1024 || l > m) return -10;
  if (!X) return -11;
  if (ldx < l) return -13;
  const bool f64 = a_t == RPID_F64 && x_t == RPID_F64;
  const bool f32 = a_t == RPID_F32 && x_t == RPID_F32;
  const bool bf = a_t == RPID_BF16 && x_t == RPID_F32;
  if (!(f64 || f32 || bf)) return RPID_ERR_UNSUPPORTED;
  RPID_HIP_CHECK(hipSetDevice(ctx->device));
  Carve cv;
  const size_t o_inv = cv.take<int32_t>((size_t)m);
  const size_t o_pt = cv.take<char>((size_t)m * l * esize(a_t));
  const size_t ws_sk = cv.off;
  RPID_CHECK(ensure_workspace(ctx, ws_sk + sketch_workspace_bytes(ctx, m, n, l, f64 ? 8 : 4)));
  int32_t* inv = ws_ptr<int32_t>(ctx, o_inv);
  if (f64) {
    double* pt = ws_ptr<double>(ctx, o_pt);
    RPID_CHECK(build_srtt_t<double>(ctx, m, l, perm, phi, sel, inv, pt, m));
    return sketch_f64(ctx, pt, m, (const double*)A, lda, m, n, l, (double*)X, ldx, ws_sk);
  }
  if (f32) {
    float* pt = ws_ptr<float>(ctx, o_pt);
    RPID_CHECK(build_srtt_t<float>(ctx, m, l, perm, phi, sel, inv, pt, m));
    return sketch_f32(ctx, pt, m, (const float*)A, lda, m, n, l, (float*)X, ldx, ws_sk);
  }
  uint16_t* pt = ws_ptr<uint16_t>(ctx, o_pt);
  RPID_CHECK(build_srtt_t<uint16_t>(ctx, m, l, perm, phi, sel, inv, pt, m));
  return sketch_bf16(ctx, pt, m, (const uint16_t*)A, lda, m, n, l, (float*)X, ldx, ws_sk);
}

static int csc_args(rpid_ctx ctx, const int64_t* colptr, const int64_t* rowidx, const void* vals,
                    rpid_dtype v_t, int64_t m, int64_t n, int64_t nnz) {
  if (!ctx) return -1;
  if (!colptr) return -2;
  if (!rowidx && nnz > 0) return -3;
  if (!vals && nnz > 0) return -4;
  if (!(v_t == RPID_F64 || v_t == RPID_F32)) return -5;
  if (m < 1) return -6;
  if (n < 1) return -7;
  if (nnz < 0) return -8;
  return RPID_OK;
}

int rpid_sketch_csc(rpid_ctx ctx, const int64_t* colptr, const int64_t* rowidx, const void* vals,
                    rpid_dtype v_t, int64_t m, int64_t n, int64_t nnz, const void* Gamma, int64_t ldg,
                    int64_t l, void* X, int64_t ldx) {
  RPID_CHECK(csc_args(ctx, colptr, rowidx, vals, v_t, m, n, nnz));
  if (!Gamma) return -9;
  if (ldg < l) return -10;
  if (l < 1 || l > 1024) return -11;
  if (!X) return -12;
  if (ldx < l) return -13;
  RPID_HIP_CHECK(hipSetDevice(ctx->device));
  if (v_t == RPID_F64)
    return csc_sketch<double>(ctx, m, n, nnz, colptr, rowidx, (const double*)vals, (const double*)Gamma,
                              ldg, l, (double*)X, ldx);
  return csc_sketch<float>(ctx, m, n, nnz, colptr, rowidx, (const float*)vals, (const float*)Gamma, ldg, l,
                           (float*)X, ldx);
}

int rpid_sketch_csc_sparse_sign(rpid_ctx ctx, const int64_t* colptr, const int64_t* rowidx,
                                const void* vals, rpid_dtype v_t, int64_t m, int64_t n, int64_t nnz,
                                const int32_t* rows, const int8_t* signs, int64_t zeta, int64_t l,
                                double scale, void* X, int64_t ldx) {
  RPID_CHECK(csc_args(ctx, colptr, rowidx, vals, v_t, m, n, nnz));
  if (!rows) return -9;
  if (!signs) return -10;
  if (zeta < 1 || zeta > 64 || zeta > l) return -11;
  if (l < 1 || l > 1024) return -12;
  if (!(scale > 0.0) || !std::isfinite(scale)) return -13;
  if (!X) return -14;
  if (ldx < l) return -15;
  RPID_HIP_CHECK(hipSetDevice(ctx->device));
  // the embedding is applied as a sparse operator: O(nnz zeta) work, nothing expanded
  if (v_t == RPID_F64)
    return csc_sparse_sign<double>(ctx, m, n, nnz, colptr, rowidx, (const double*)vals, rows, signs,
                                   (int)zeta, l, scale, (double*)X, ldx);
  return csc_sparse_sign<float>(ctx, m, n, nnz, colptr, rowidx, (const float*)vals, rows, signs, (int)zeta,
                                l, (float)scale, (float*)X, ldx);
}

int rpid_csc_gather(rpid_ctx ctx, const int64_t* colptr, const int64_t* rowidx, const void* vals,
                    rpid_dtype v_t, int64_t m, int64_t n, int64_t nnz, int64_t k, const int64_t* J,
                    void* C, int64_t ldc) {
  RPID_CHECK(csc_args(ctx, colptr, rowidx, vals, v_t, m, n, nnz));
  if (k < 1 || (!J && k != n)) return -9;
  if (!C) return -11;
  if (ldc < m) return -12;
  RPID_HIP_CHECK(hipSetDevice(ctx->device));
  if (v_t == RPID_F64)
    return csc_gather<double>(ctx, m, n, nnz, colptr, rowidx, (const double*)vals, k, J, (double*)C, ldc);
  return csc_gather<float>(ctx, m, n, nnz, colptr, rowidx, (const float*)vals, k, J, (float*)C, ldc);
}

// ---------------------------------------------------------------------------
int rpid_select_columns_cpqr(rpid_ctx ctx, const void* X, rpid_dtype x_t, int64_t l, int64_t n,
                             int64_t ldx, int64_t k, int64_t* J, void* Rf, int64_t ldr, void* diagR,
                             int64_t* k_eff) {
  if (!ctx) return -1;
  if (!X) return -2;
  if (!is_lupp_type(x_t)) return -3;
  if (l < 1 || l > 512) return -4;
  if (n < 1) return -5;
  if (ldx < l) return -6;
  if (k < 1 || k > l || k > n) return -7;
  if (!J) return -8;
  if (!Rf) return -9;
  if (ldr < k) return -10;
  RPID_HIP_CHECK(hipSetDevice(ctx->device));
  Carve cv;
  const size_t o_status = cv.take<int64_t>(8);
  RPID_CHECK(ensure_workspace(ctx, cv.off));
  int64_t* status_dev = ws_ptr<int64_t>(ctx, o_status);
  int s;
  if (x_t == RPID_F64)
    s = cpqr_panel<double>(ctx, (const double*)X, ldx, 1, n, l, k, J, (double*)Rf, ldr, (double*)diagR,
                           status_dev);
  else
    s = cpqr_panel<float>(ctx, (const float*)X, ldx, 1, n, l, k, J, (float*)Rf, ldr, (float*)diagR,
                          status_dev);
  if (s != RPID_OK) return s;
  if (!k_eff) return RPID_OK;
  int64_t st = 0;
  RPID_CHECK(read_status(ctx, status_dev, &st));
  if (st < 0) return (int)st;
  *k_eff = (st == 0) ? k : st - 1;
  return (int)st;
}

int rpid_id_coeffs_cpqr(rpid_ctx ctx, rpid_dtype r_t, int64_t k, int64_t n, const int64_t* J,
                        const void* Rf, int64_t ldr, double* Z, int64_t ldz) {
  if (!ctx) return -1;
  if (!is_lupp_type(r_t)) return -2;
  if (k < 1 || k > 1024) return -3;
  if (n < k) return -4;
  if (!J) return -5;
  if (!Rf) return -6;
  if (ldr < k) return -7;
  if (!Z) return -8;
  if (ldz < k) return -9;
  RPID_HIP_CHECK(hipSetDevice(ctx->device));
  Carve cv;
  const size_t o_R11 = cv.take<double>((size_t)k * k);
  const size_t o_W = cv.take<double>((size_t)k * k);
  const size_t o_R64 = r_t == RPID_F64 ? 0 : cv.take<double>((size_t)k * n);
  const size_t o_tmp = cv.off;
  RPID_CHECK(ensure_workspace(ctx, o_tmp + (size_t)64 * k * k * sizeof(double) + 4096));
  double* R11 = ws_ptr<double>(ctx, o_R11);
  double* Wi = ws_ptr<double>(ctx, o_W);
  const double* R64 = (const double*)Rf;
  int64_t ld64 = ldr;
  if (r_t == RPID_F64) {
    RPID_CHECK(gather_columns<double, double>(ctx, k, k, (const double*)Rf, ldr, n, J, R11, k));
  } else {
    double* Rc = ws_ptr<double>(ctx, o_R64);
    RPID_CHECK(convert_matrix<float, double>(ctx, k, n, (const float*)Rf, ldr, Rc, k));
    RPID_CHECK(gather_columns<double, double>(ctx, k, k, Rc, k, n, J, R11, k));
    R64 = Rc;
    ld64 = k;
  }
  // Z = R11^{-1} R_top, with R11 = R_top(:, J) upper triangular in pivot order
  RPID_CHECK(tri_inverse(ctx, k, R11, k, false, false, Wi, k, o_tmp));
  RPID_CHECK(dgemm(ctx, false, false, k, n, k, 1.0, Wi, k, R64, ld64, 0.0, Z, ldz, o_tmp));
  return set_identity_columns(ctx, k, n, J, Z, ldz);
}

// ---------------------------------------------------------------------------
// Z = X_1^+ X over all l rows of the sketch (X_1 = X(:, J)), by a
// Cholesky-QR2 of X_1: X_1 = Q R, Z = R^{-1} (Q^T X); Z(:, J) = I.
int rpid_id_coeffs_ls(rpid_ctx ctx, const void* X, rpid_dtype x_t, int64_t l, int64_t n, int64_t ldx,
                      int64_t k, const int64_t* J, double* Z, int64_t ldz) {
  if (!ctx) return -1;
  if (!X) return -2;
  if (!is_lupp_type(x_t)) return -3;
  if (l < 1) return -4;
  if (n < 1) return -5;
  if (ldx < l) return -6;
  if (k < 1 || k > l || k > n || k > 1024) return -7;
  if (!J) return -8;
  if (!Z) return -9;
  if (ldz < k) return -10;
  RPID_HIP_CHECK(hipSetDevice(ctx->device));
  const int64_t kk = k * k;
  Carve cv;
  const size_t o_status = cv.take<int64_t>(8);
  const size_t o_X64 = x_t == RPID_F64 ? 0 : cv.take<double>((size_t)l * n);
  const size_t o_X1 = cv.take<double>((size_t)l * k);
  const size_t o_Q = cv.take<double>((size_t)l * k);
  const size_t o_G = cv.take<double>((size_t)2 * kk);
  const size_t o_W = cv.take<double>((size_t)2 * kk);
  const size_t o_Ri = cv.take<double>((size_t)kk);
  const size_t o_Y = cv.take<double>((size_t)k * n);
  const size_t o_tmp = cv.off;
  RPID_CHECK(ensure_workspace(ctx, o_tmp + (size_t)64 * kk * sizeof(double) + 4096));
  int64_t* status_dev = ws_ptr<int64_t>(ctx, o_status);
  const double* X64 = (const double*)X;
  int64_t ld64 = ldx;
  if (x_t != RPID_F64) {
    double* Xc = ws_ptr<double>(ctx, o_X64);
    RPID_CHECK(convert_matrix<float, double>(ctx, l, n, (const float*)X, ldx, Xc, l));
    X64 = Xc;
    ld64 = l;
  }
  double* X1 = ws_ptr<double>(ctx, o_X1);
  double* Q = ws_ptr<double>(ctx, o_Q);
  double* G = ws_ptr<double>(ctx, o_G);
  double* W = ws_ptr<double>(ctx, o_W);
  double* Ri = ws_ptr<double>(ctx, o_Ri);
  double* Y = ws_ptr<double>(ctx, o_Y);
  RPID_CHECK(launch_fill_u64(ctx, reinterpret_cast<uint64_t*>(status_dev), 2, 0ull));
  RPID_CHECK(gather_columns<double, double>(ctx, l, k, X64, ld64, n, J, X1, l));
  // two Cholesky-QR passes: X1 -> Q (R1^{-1} in W), Q -> X1 (R2^{-1} in W + kk)
  const double* in = X1;
  double* out = Q;
  for (int pass = 0; pass < 2; ++pass) {
    double* Gp = G + pass * kk;
    double* Wp = W + pass * kk;
    RPID_CHECK(dgemm(ctx, true, false, k, k, l, 1.0, in, l, in, l, 0.0, Gp, k, o_tmp));
    if (sweep_supported(k)) {
      RPID_CHECK(chol_inverse_batched(ctx, 1, k, Gp, k, kk, Wp, k, kk, status_dev + pass, o_tmp));
    } else {
      RPID_CHECK(cholesky_batched(ctx, 1, k, Gp, k, kk, status_dev + pass));
      RPID_CHECK(tri_inverse(ctx, k, Gp, k, false, false, Wp, k, o_tmp));
    }
    RPID_CHECK(dgemm(ctx, false, false, l, k, k, 1.0, in, l, Wp, k, 0.0, out, l, o_tmp));
    in = out;
    out = X1;
  }
  // in = Q (orthonormal), R^{-1} = R1^{-1} R2^{-1}; Z = R^{-1} (Q^T X)
  RPID_CHECK(dgemm(ctx, false, false, k, k, k, 1.0, W, k, W + kk, k, 0.0, Ri, k, o_tmp));
  RPID_CHECK(dgemm(ctx, true, false, k, n, l, 1.0, in, l, X64, ld64, 0.0, Y, k, o_tmp));
  RPID_CHECK(dgemm(ctx, false, false, k, n, k, 1.0, Ri, k, Y, k, 0.0, Z, ldz, o_tmp));
  RPID_CHECK(set_identity_columns(ctx, k, n, J, Z, ldz));
  int64_t st[2] = {0, 0};
  RPID_HIP_CHECK(hipMemcpyAsync(ctx->host_status, status_dev, 2 * sizeof(int64_t), hipMemcpyDeviceToHost,
                                ctx->stream));
  RPID_HIP_CHECK(hipStreamSynchronize(ctx->stream));
  st[0] = ctx->host_status[0];
  st[1] = ctx->host_status[1];
  return (st[0] != 0 || st[1] != 0) ? RPID_ERR_BREAKDOWN : RPID_OK;
}

// ---------------------------------------------------------------------------
int rpid_id_coeffs(rpid_ctx ctx, const void* X, rpid_dtype x_t, int64_t l, int64_t n,
                   int64_t ldx, int64_t k, const int64_t* J, const void* Lf, int64_t ldl,
                   const void* Uf, int64_t ldu, double* Z, int64_t ldz, int refine_steps,
                   double* eta) {
  if (!ctx) return -1;
  if (!X) return -2;
  if (!is_lupp_type(x_t)) return -3;
  if (l < 1) return -4;
  if (n < 1) return -5;
  if (ldx < l) return -6;
  if (k < 1 || k > l || k > n || k > 1024) return -7;
  if (!J) return -8;
  if (!Lf) return -9;
  if (ldl < n) return -10;
  if (!Uf) return -11;
  if (ldu < k) return -12;
  if (!Z) return -13;
  if (ldz < k) return -14;
  if (refine_steps < 0 || refine_steps > 4) return -15;
  RPID_HIP_CHECK(hipSetDevice(ctx->device));
  Carve cv;
  const size_t o_LJ = cv.take<double>((size_t)k * k);
  const size_t o_Winv = cv.take<double>((size_t)k * k);
  const size_t o_WU = cv.take<double>((size_t)k * k);
  const size_t o_P = cv.take<double>((size_t)k * k);
  const size_t o_U64 = cv.take<double>((size_t)k * k);
  const size_t o_X1 = cv.take<double>((size_t)k * k);
  const size_t o_L64 = x_t == RPID_F64 ? 0 : cv.take<double>((size_t)n * k);
  const size_t o_res = refine_steps ? cv.take<double>((size_t)k * n) : 0;
  const size_t o_G = cv.take<double>((size_t)k * k);
  const size_t o_lam = cv.take<double>(8);
  const size_t o_tmp = cv.off;
  const size_t tmp_bytes = (size_t)64 * k * k * sizeof(double) + 4096;
  RPID_CHECK(ensure_workspace(ctx, o_tmp + tmp_bytes));
  double* LJ = ws_ptr<double>(ctx, o_LJ);
  double* Winv = ws_ptr<double>(ctx, o_Winv);
  const bool f64 = x_t == RPID_F64;
  // L_J = Lf(J, 0:k) in FP64 and W = L_J^{-1} (unit lower)
  if (f64)
    RPID_CHECK(gather_rows<double, double>(ctx, k, k, (const double*)Lf, ldl, n, J, LJ, k));
  else
    RPID_CHECK(gather_rows<float, double>(ctx, k, k, (const float*)Lf, ldl, n, J, LJ, k));
  RPID_CHECK(tri_inverse(ctx, k, LJ, k, true, true, Winv, k, o_tmp));
  // Z = W^T Lf^T: column j is L_J^{-T} Lf(j, :)^T, i.e. solves L_J^T z = Lf(j, :)^T
  const double* L64 = (const double*)Lf;
  int64_t ldl64 = ldl;
  if (!f64) {
    double* Lc = ws_ptr<double>(ctx, o_L64);
    RPID_CHECK(convert_matrix<float, double>(ctx, n, k, (const float*)Lf, ldl, Lc, n));
    L64 = Lc;
    ldl64 = n;
  }
  RPID_CHECK(dgemm(ctx, true, true, k, n, k, 1.0, Winv, k, L64, ldl64, 0.0, Z, ldz, o_tmp));
  RPID_CHECK(set_identity_columns(ctx, k, n, J, Z, ldz));
  if (refine_steps > 0) {
    double* U64 = ws_ptr<double>(ctx, o_U64);
    double* X1 = ws_ptr<double>(ctx, o_X1);
    double* res = ws_ptr<double>(ctx, o_res);
    double* WU = ws_ptr<double>(ctx, o_WU);
    double* Pm = ws_ptr<double>(ctx, o_P);
    if (f64) {
      RPID_CHECK(convert_matrix<double, double>(ctx, k, k, (const double*)Uf, ldu, U64, k));
      RPID_CHECK(gather_columns<double, double>(ctx, k, k, (const double*)X, ldx, n, J, X1, k));
    } else {
      RPID_CHECK(convert_matrix<float, double>(ctx, k, k, (const float*)Uf, ldu, U64, k));
      RPID_CHECK(gather_columns<float, double>(ctx, k, k, (const float*)X, ldx, n, J, X1, k));
    }
    // X_1 = (L_J U')^T, so X_1^{-1} = (W_U W)^T with W_U = U'^{-1}
    RPID_CHECK(tri_inverse(ctx, k, U64, k, false, false, WU, k, o_tmp));
    RPID_CHECK(dgemm(ctx, false, false, k, k, k, 1.0, WU, k, Winv, k, 0.0, Pm, k, o_tmp));
    for (int it = 0; it < refine_steps; ++it) {
      // res = X_k - X_1 Z (FP64, X promoted); Z += X_1^{-1} res
      if (f64)
        RPID_CHECK(convert_matrix<double, double>(ctx, k, n, (const double*)X, ldx, res, k));
      else
        RPID_CHECK(convert_matrix<float, double>(ctx, k, n, (const float*)X, ldx, res, k));
      RPID_CHECK(dgemm(ctx, false, false, k, n, k, -1.0, X1, k, Z, ldz, 1.0, res, k, o_tmp));
      RPID_CHECK(dgemm(ctx, true, false, k, n, k, 1.0, Pm, k, res, k, 1.0, Z, ldz, o_tmp));
      RPID_CHECK(set_identity_columns(ctx, k, n, J, Z, ldz));
    }
  }
  if (eta) {
    // eta^2 = 1 + ||Z_rest||_2^2 = lambda_max(Z Z^T) since Z(:, J) = I
    double* G = ws_ptr<double>(ctx, o_G);
    double* lam = ws_ptr<double>(ctx, o_lam);
    RPID_CHECK(dgemm(ctx, false, true, k, k, n, 1.0, Z, ldz, Z, ldz, 0.0, G, k, o_tmp));
    RPID_CHECK(power_iteration(ctx, k, G, k, 2000, 1e-12, lam));
    double h = 0.0;
    RPID_CHECK(read_doubles(ctx, lam, &h, 1));
    *eta = sqrt(h > 1.0 ? h : 1.0);
  }
  return RPID_OK;
}

int rpid_cur(rpid_ctx ctx, const void* A, rpid_dtype a_t, int64_t m, int64_t n, int64_t lda,
             int64_t k, const int64_t* J, int64_t* I, double* U, int64_t ldu, int64_t* k_eff) {
  if (!ctx) return -1;
  if (!A) return -2;
  if (!(a_t == RPID_F64 || a_t == RPID_F32 || a_t == RPID_BF16)) return -3;
  if (m < 1) return -4;
  if (n < 1) return -5;
  if (lda < m) return -6;
  if (k < 1 || k > m || k > n || k > 1024) return -7;
  if (!J) return -8;
  if (!I) return -9;
  if (!U) return -10;
  if (ldu < k) return -11;
  RPID_HIP_CHECK(hipSetDevice(ctx->device));
  switch (a_t) {
    case RPID_F64: return cur_impl<double>(ctx, (const double*)A, a_t, m, n, lda, k, J, I, U, ldu, k_eff);
    case RPID_F32: return cur_impl<float>(ctx, (const float*)A, a_t, m, n, lda, k, J, I, U, ldu, k_eff);
    default: return cur_impl<uint16_t>(ctx, (const uint16_t*)A, a_t, m, n, lda, k, J, I, U, ldu, k_eff);
  }
}

static int residual_entry(rpid_ctx ctx, int which, const void* A, rpid_dtype a_t, int64_t m,
                          int64_t n, int64_t lda, int64_t k, const int64_t* J, const double* Z,
                          int64_t ldz, const int64_t* I, const double* U, int64_t ldu,
                          double* rel_fro, double* sums_dev) {
  if (!ctx) return -1;
  if (which != RPID_RESIDUAL_ID && which != RPID_RESIDUAL_CUR && which != RPID_RESIDUAL_ROW_ID) return -2;
  if (!A) return -3;
  if (!(a_t == RPID_F64 || a_t == RPID_F32 || a_t == RPID_BF16)) return -4;
  if (m < 1) return -5;
  if (n < 1) return -6;
  if (lda < m) return -7;
  if (k < 1 || k > m || k > n || k > 1024) return -8;
  if (!J && which != RPID_RESIDUAL_ROW_ID) return -9;
  if (which != RPID_RESIDUAL_CUR && !Z) return -10;
  if (which != RPID_RESIDUAL_CUR && ldz < k) return -11;
  if (which != RPID_RESIDUAL_ID && !I) return -12;
  if (which == RPID_RESIDUAL_CUR && !U) return -13;
  if (which == RPID_RESIDUAL_CUR && ldu < k) return -14;
  if (!rel_fro && !sums_dev) return -15;
  RPID_HIP_CHECK(hipSetDevice(ctx->device));
  switch (a_t) {
    case RPID_F64:
      return residual_impl<double>(ctx, which, (const double*)A, a_t, m, n, lda, k, J, Z, ldz, I,
                                   U, ldu, rel_fro, sums_dev);
    case RPID_F32:
      return residual_impl<float>(ctx, which, (const float*)A, a_t, m, n, lda, k, J, Z, ldz, I, U,
                                  ldu, rel_fro, sums_dev);
    default:
      return residual_impl<uint16_t>(ctx, which, (const uint16_t*)A, a_t, m, n, lda, k, J, Z, ldz,
                                     I, U, ldu, rel_fro, sums_dev);
  }
}

int rpid_residual(rpid_ctx ctx, int which, const void* A, rpid_dtype a_t, int64_t m, int64_t n,
                  int64_t lda, int64_t k, const int64_t* J, const double* Z, int64_t ldz,
                  const int64_t* I, const double* U, int64_t ldu, double* rel_fro) {
  if (!rel_fro) return -15;
  return residual_entry(ctx, which, A, a_t, m, n, lda, k, J, Z, ldz, I, U, ldu, rel_fro, nullptr);
}

int rpid_residual_sums(rpid_ctx ctx, int which, const void* A, rpid_dtype a_t, int64_t m, int64_t n,
                       int64_t lda, int64_t k, const int64_t* J, const double* Z, int64_t ldz,
                       const int64_t* I, const double* U, int64_t ldu, double* sums) {
  if (!sums) return -15;
  return residual_entry(ctx, which, A, a_t, m, n, lda, k, J, Z, ldz, I, U, ldu, nullptr, sums);
}

// ---------------------------------------------------------------------------
int rpid_mlp_features(rpid_ctx ctx, const void* diagU, rpid_dtype x_t, int64_t L, int64_t k_eff,
                      float* feats) {
  if (!ctx) return -1;
  if (!diagU) return -2;
  if (!is_lupp_type(x_t)) return -3;
  if (L < 1 || L > 4096) return -4;
  if (k_eff < 0 || k_eff > L) return -5;
  if (!feats) return -6;
  RPID_HIP_CHECK(hipSetDevice(ctx->device));
  return mlp_features(ctx, diagU, x_t == RPID_F64, L, k_eff, feats);
}

int rpid_mlp_forward(rpid_ctx ctx, const float* W, const float* feats, int64_t B, float* yhat,
                     float* act) {
  if (!ctx) return -1;
  if (!W) return -2;
  if (!feats) return -3;
  if (B < 1) return -4;
  if (!yhat) return -5;
  RPID_HIP_CHECK(hipSetDevice(ctx->device));
  return mlp_forward(ctx, W, feats, B, yhat, act);
}

int rpid_mlp_backward(rpid_ctx ctx, const float* W, const float* feats, const float* act,
                      const float* dy, int64_t B, float* dW) {
  if (!ctx) return -1;
  if (!W) return -2;
  if (!feats) return -3;
  if (!act) return -4;
  if (!dy) return -5;
  if (B < 1) return -6;
  if (!dW) return -7;
  RPID_HIP_CHECK(hipSetDevice(ctx->device));
  RPID_CHECK(ensure_workspace(ctx, mlp_backward_workspace(B)));
  return mlp_backward(ctx, W, feats, act, dy, B, dW, 0);
}

int rpid_mlp_adam(rpid_ctx ctx, float* W, const float* dW, float* m1, float* m2, float lr,
                  int64_t t) {
  if (!ctx) return -1;
  if (!W) return -2;
  if (!dW) return -3;
  if (!m1) return -4;
  if (!m2) return -5;
  if (!(lr > 0.0f)) return -6;
  if (t < 1) return -7;
  RPID_HIP_CHECK(hipSetDevice(ctx->device));
  return mlp_adam(ctx, W, dW, m1, m2, lr, t);
}

int rpid_mlp_loss(rpid_ctx ctx, const float* yhat, const float* target, int64_t B, float tau,
                  float* dy, float* loss) {
  if (!ctx) return -1;
  if (!yhat) return -2;
  if (!target) return -3;
  if (B < 1) return -4;
  if (!(tau > 0.0f && tau < 1.0f)) return -5;
  if (!dy) return -6;
  if (!loss) return -7;
  RPID_HIP_CHECK(hipSetDevice(ctx->device));
  return mlp_pinball(ctx, yhat, target, B, tau, dy, loss);
}

}  // extern "C"
