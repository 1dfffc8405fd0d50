// Small kernels of the path: gathers of skeleton columns/rows, conversions,
// BF16 splitting of FP64 factors, triangular solves with many right-hand
// sides, and a batched single-workgroup Cholesky for k x k Gram matrices.
#include "rpid_internal.hpp"

namespace rpid {

namespace {

template <typename T>
__device__ __forceinline__ T cvt_from_double(double v);
template <>
__device__ __forceinline__ double cvt_from_double<double>(double v) {
  return v;
}
template <>
__device__ __forceinline__ float cvt_from_double<float>(double v) {
  return (float)v;
}
template <>
__device__ __forceinline__ uint16_t cvt_from_double<uint16_t>(double v) {
  return float_to_bf16_bits((float)v);
}

inline unsigned grid_for(int64_t count, int64_t per = 256, int64_t cap = 8192) {
  int64_t b = (count + per - 1) / per;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

template <typename TS, typename TD>
__global__ void convert_kernel(int64_t rows, int64_t cols, const TS* S, int64_t lds, TD* D,
                               int64_t ldd) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % rows, j = e / rows;
    D[i + j * ldd] = cvt_from_double<TD>(load_as_double<TS>(S, i + j * lds));
  }
}

// Indices outside [0, ncols) (an undefined pivot after a rank-deficient
// factorisation) read as a zero column instead of faulting.
template <typename TS, typename TD>
__global__ void gather_cols_kernel(int64_t m, int64_t k, const TS* A, int64_t lda, int64_t ncols,
                                   const int64_t* J, TD* C, int64_t ldc) {
  const int64_t total = m * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % m, t = e / m;
    const int64_t j = J[t];
    C[i + t * ldc] =
        cvt_from_double<TD>((j >= 0 && j < ncols) ? load_as_double<TS>(A, i + j * lda) : 0.0);
  }
}

template <typename TS, typename TD>
__global__ void gather_rows_kernel(int64_t k, int64_t n, const TS* A, int64_t lda, int64_t nrows,
                                   const int64_t* I, TD* R, int64_t ldr) {
  const int64_t total = k * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = e % k, j = e / k;
    const int64_t i = I[t];
    R[t + j * ldr] =
        cvt_from_double<TD>((i >= 0 && i < nrows) ? load_as_double<TS>(A, i + j * lda) : 0.0);
  }
}

__global__ void transpose_kernel(int64_t rows, int64_t cols, const double* X, int64_t ldx,
                                 double* Y, int64_t ldy) {
  __shared__ double tile[32][33];
  const int64_t bi = (int64_t)blockIdx.x * 32, bj = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = bi + tx, j = bj + r;
    if (i < rows && j < cols) tile[r][tx] = X[i + j * ldx];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t j = bj + tx, i = bi + r;
    if (i < rows && j < cols) Y[j + i * ldy] = tile[tx][r];
  }
}

__global__ void trace_shift_kernel(int64_t k, double* G, int64_t ldg, double c) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < k; i += blockDim.x) s += G[i + i * ldg];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double shift = c * red[0];
  for (int64_t i = threadIdx.x; i < k; i += blockDim.x) G[i + i * ldg] += shift;
}

__global__ void identity_cols_kernel(int64_t k, const int64_t* J, double* Z, int64_t ldz) {
  const int64_t total = k * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e % k, t = e / k;
    Z[c + J[t] * ldz] = (c == t) ? 1.0 : 0.0;
  }
}

__global__ void split_bf16_kernel(int64_t rows, int64_t cols, const double* S, int64_t lds,
                                  int parts, uint16_t* D, int64_t ldd) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % rows, j = e / rows;
    double r = S[i + j * lds];
    for (int p = 0; p < parts; ++p) {
      const uint16_t b = float_to_bf16_bits((float)r);
      D[i + (j + (int64_t)p * cols) * ldd] = b;
      r -= (double)bf16_bits_to_float(b);
    }
  }
}

// ---------------------------------------------------------------------------
// Triangular solve with many right-hand sides.  A workgroup of 256 threads
// takes 32 right-hand sides; 8 threads share one right-hand side and split
// the dot products of each block of 16 unknowns, whose partial sums are
// combined in LDS before one thread does the 16 x 16 substitution.  The 16
// rows of op(T) of the current block are staged in LDS.
// ---------------------------------------------------------------------------
constexpr int TB_ = 16;
constexpr int TS_RHS = 32;
constexpr int TS_PART = 8;

template <typename TBt>
__global__ __launch_bounds__(256) void tri_solve_kernel(int64_t k, int64_t nrhs, const double* T,
                                                        int64_t ldt, bool trans, bool lower_op,
                                                        bool unit, const TBt* B, int64_t brs,
                                                        int64_t bcs, double* X, int64_t xrs,
                                                        int64_t xcs) {
  extern __shared__ double blk[];  // TB_ x k: blk[i * k + d] = op(T)(c0 + i, d)
  __shared__ double part[TS_PART][TS_RHS][TB_ + 1];
  const int tid = threadIdx.x;
  const int rl = tid % TS_RHS;  // right-hand side within the workgroup
  const int pt = tid / TS_RHS;  // partial-sum slot
  const int64_t r = (int64_t)blockIdx.x * TS_RHS + rl;
  const bool active = r < nrhs;
  const int64_t nb = (k + TB_ - 1) / TB_;
  for (int64_t bb = 0; bb < nb; ++bb) {
    const int64_t blkid = lower_op ? bb : nb - 1 - bb;
    const int64_t c0 = blkid * TB_;
    const int bs = (int)min((int64_t)TB_, k - c0);
    __syncthreads();
    for (int64_t e = tid; e < (int64_t)TB_ * k; e += blockDim.x) {
      const int64_t i = e / k, d = e % k;
      double v = 0.0;
      if (i < bs) {
        const int64_t row = c0 + i;
        v = trans ? T[d + row * ldt] : T[row + d * ldt];
      }
      blk[e] = v;
    }
    __syncthreads();
    // partial dot products with the unknowns already solved
    double acc[TB_];
#pragma unroll
    for (int i = 0; i < TB_; ++i) acc[i] = 0.0;
    if (active) {
      const int64_t dlo = lower_op ? 0 : c0 + bs;
      const int64_t dhi = lower_op ? c0 : k;
      for (int64_t d = dlo + pt; d < dhi; d += TS_PART) {
        const double xd = X[r * xcs + d * xrs];
#pragma unroll
        for (int i = 0; i < TB_; ++i) acc[i] = fma(blk[i * k + d], xd, acc[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < TB_; ++i) part[pt][rl][i] = acc[i];
    __syncthreads();
    if (pt == 0 && active) {
      double v[TB_];
#pragma unroll
      for (int i = 0; i < TB_; ++i) {
        double s = 0.0;
#pragma unroll
        for (int p = 0; p < TS_PART; ++p) s += part[p][rl][i];
        v[i] = (i < bs) ? load_as_double<TBt>(B, r * bcs + (c0 + i) * brs) - s : 0.0;
      }
      if (lower_op) {
#pragma unroll
        for (int i = 0; i < TB_; ++i) {
          if (i < bs) {
#pragma unroll
            for (int i2 = 0; i2 < i; ++i2) v[i] = fma(-blk[i * k + c0 + i2], v[i2], v[i]);
            if (!unit) v[i] /= blk[i * k + c0 + i];
            X[r * xcs + (c0 + i) * xrs] = v[i];
          }
        }
      } else {
#pragma unroll
        for (int i = TB_ - 1; i >= 0; --i) {
          if (i < bs) {
#pragma unroll
            for (int i2 = i + 1; i2 < TB_; ++i2)
              if (i2 < bs) v[i] = fma(-blk[i * k + c0 + i2], v[i2], v[i]);
            if (!unit) v[i] /= blk[i * k + c0 + i];
            X[r * xcs + (c0 + i) * xrs] = v[i];
          }
        }
      }
    }
    __threadfence_block();
  }
}

// ---------------------------------------------------------------------------
// Cholesky of k x k SPD matrices, one 1024-thread workgroup per matrix.
// Left-looking by panels of 16 columns: the panel (rows j0..k-1) is updated
// with the finished columns (lower factor L stored in the lower triangle,
// read from global/L2), its 16 x 16 diagonal block is factored in LDS and the
// rows below are solved against it.  At the end R = L^T is written to the
// upper triangle and the strict lower triangle is zeroed.
// ---------------------------------------------------------------------------
constexpr int CB = 16;

__global__ __launch_bounds__(1024) void cholesky_kernel(int64_t k, double* Gall, int64_t ldg,
                                                        int64_t stride, int64_t* status) {
  double* G = Gall + (int64_t)blockIdx.x * stride;
  __shared__ double diag[CB][CB + 1];  // diagonal block being factored
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int64_t j0 = 0; j0 < k && !bad; j0 += CB) {
    const int bs = (int)min((int64_t)CB, k - j0);
    const int64_t nrows = k - j0;  // rows j0..k-1 of the panel
    // (1) panel update: P(i, c) = G(j0+i, j0+c) - sum_{p < j0} L(j0+i, p) L(j0+c, p)
    //     thread -> (row i, column group of 4)
    for (int64_t w = tid; w < nrows * (CB / 4); w += blockDim.x) {
      const int64_t i = w % nrows;
      const int cg = (int)(w / nrows) * 4;
      double acc[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = (cg + c < bs) ? G[(j0 + i) + (j0 + cg + c) * ldg] : 0.0;
      for (int64_t p = 0; p < j0; ++p) {
        const double lip = G[(j0 + i) + p * ldg];
#pragma unroll
        for (int c = 0; c < 4; ++c)
          if (cg + c < bs) acc[c] = fma(-lip, G[(j0 + cg + c) + p * ldg], acc[c]);
      }
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (cg + c < bs && i >= cg + c) G[(j0 + i) + (j0 + cg + c) * ldg] = acc[c];
    }
    __syncthreads();
    // (2) factor the diagonal block in LDS (lower)
    if (tid < CB * CB) {
      const int a = tid % CB, b = tid / CB;
      diag[a][b] = (a < bs && b < bs && a >= b) ? G[(j0 + a) + (j0 + b) * ldg] : 0.0;
    }
    __syncthreads();
    for (int c = 0; c < bs; ++c) {
      if (tid == 0) {
        const double d = diag[c][c];
        if (!(d > 0.0) || !isfinite(d)) {
          bad = 1;
          status[blockIdx.x] = j0 + c + 1;
        } else {
          diag[c][c] = sqrt(d);
        }
      }
      __syncthreads();
      if (bad) break;
      if (tid > c && tid < bs) diag[tid][c] /= diag[c][c];
      __syncthreads();
      if (tid < CB * CB) {
        const int a = tid % CB, b = tid / CB;
        if (b > c && a >= b && a < bs) diag[a][b] = fma(-diag[a][c], diag[b][c], diag[a][b]);
      }
      __syncthreads();
    }
    if (bad) break;
    if (tid < CB * CB) {
      const int a = tid % CB, b = tid / CB;
      if (a < bs && b < bs && a >= b) G[(j0 + a) + (j0 + b) * ldg] = diag[a][b];
    }
    // (3) rows below: L(j0+bs+i, j0:j0+bs) = P(i, :) L_jj^{-T} (forward, per row)
    for (int64_t i = tid; i < nrows - bs; i += blockDim.x) {
      const int64_t row = j0 + bs + i;
      double x[CB];
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        if (c < bs) {
          double v = G[row + (j0 + c) * ldg];
#pragma unroll
          for (int c2 = 0; c2 < c; ++c2) v = fma(-x[c2], diag[c][c2], v);
          x[c] = v / diag[c][c];
        } else {
          x[c] = 0.0;
        }
      }
#pragma unroll
      for (int c = 0; c < CB; ++c)
        if (c < bs) G[row + (j0 + c) * ldg] = x[c];
    }
    __syncthreads();
  }
  __syncthreads();
  if (!bad) {
    if (tid == 0) status[blockIdx.x] = 0;
    // R = L^T in the upper triangle, zeros below
    for (int64_t e = tid; e < k * k; e += blockDim.x) {
      const int64_t i = e % k, j = e / k;
      if (i < j) G[i + j * ldg] = G[j + i * ldg];
    }
    __syncthreads();
    for (int64_t e = tid; e < k * k; e += blockDim.x) {
      const int64_t i = e % k, j = e / k;
      if (i > j) G[i + j * ldg] = 0.0;
    }
  }
}

__global__ void axpy_kernel(int64_t rows, int64_t cols, double alpha, const double* S,
                            int64_t lds, double* D, int64_t ldd) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % rows, j = e / rows;
    D[i + j * ldd] = fma(alpha, S[i + j * lds], D[i + j * ldd]);
  }
}

// Power iteration x <- G x / ||G x|| from x0 = (1, ..., 1) (G symmetric PSD),
// stopped when the Rayleigh quotient changes by less than rtol (relative).
__global__ __launch_bounds__(1024) void power_iter_kernel(int64_t k, const double* G, int64_t ldg,
                                                          int max_iter, double rtol,
                                                          double* lam_out) {
  extern __shared__ double sh[];  // x[k], y[k]
  __shared__ double red[1024];
  __shared__ int done;
  double* x = sh;
  double* y = sh + k;
  const int tid = threadIdx.x;
  for (int64_t i = tid; i < k; i += blockDim.x) x[i] = 1.0 / sqrt((double)k);
  if (tid == 0) done = 0;
  __syncthreads();
  double lam_prev = 0.0, lam = 0.0;
  for (int it = 0; it < max_iter; ++it) {
    double part_xy = 0.0, part_yy = 0.0;
    for (int64_t i = tid; i < k; i += blockDim.x) {
      double s = 0.0;
      for (int64_t j = 0; j < k; ++j) s = fma(G[i + j * ldg], x[j], s);
      y[i] = s;
      part_xy += s * x[i];
      part_yy += s * s;
    }
    red[tid] = part_xy;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    lam = red[0];  // Rayleigh quotient x^T G x with ||x|| = 1
    __syncthreads();
    red[tid] = part_yy;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    const double ny = sqrt(red[0]);
    __syncthreads();
    if (ny == 0.0) {
      lam = 0.0;
      break;
    }
    for (int64_t i = tid; i < k; i += blockDim.x) x[i] = y[i] / ny;
    if (tid == 0 && it > 0 && fabs(lam - lam_prev) <= rtol * fabs(lam)) done = 1;
    lam_prev = lam;
    __syncthreads();
    if (done) break;
  }
  if (tid == 0) *lam_out = lam;
}

}  // namespace

int axpy_matrix(rpid_ctx ctx, int64_t rows, int64_t cols, double alpha, const double* S,
                int64_t lds, double* D, int64_t ldd) {
  hipLaunchKernelGGL(axpy_kernel, dim3(grid_for(rows * cols)), dim3(256), 0, ctx->stream, rows,
                     cols, alpha, S, lds, D, ldd);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

int power_iteration(rpid_ctx ctx, int64_t k, const double* G, int64_t ldg, int max_iter,
                    double rtol, double* lam) {
  const size_t shmem = 2 * (size_t)k * sizeof(double);
  if (shmem > 128 * 1024) return RPID_ERR_UNSUPPORTED;
  hipLaunchKernelGGL(power_iter_kernel, dim3(1), dim3(1024), shmem, ctx->stream, k, G, ldg,
                     max_iter, rtol, lam);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

template <typename TS, typename TD>
int convert_matrix(rpid_ctx ctx, int64_t rows, int64_t cols, const TS* S, int64_t lds, TD* D,
                   int64_t ldd) {
  hipLaunchKernelGGL((convert_kernel<TS, TD>), dim3(grid_for(rows * cols)), dim3(256), 0,
                     ctx->stream, rows, cols, S, lds, D, ldd);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

template <typename TS, typename TD>
int gather_columns(rpid_ctx ctx, int64_t m, int64_t k, const TS* A, int64_t lda, int64_t ncols,
                   const int64_t* J, TD* C, int64_t ldc) {
  hipLaunchKernelGGL((gather_cols_kernel<TS, TD>), dim3(grid_for(m * k)), dim3(256), 0,
                     ctx->stream, m, k, A, lda, ncols, J, C, ldc);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

template <typename TS, typename TD>
int gather_rows(rpid_ctx ctx, int64_t k, int64_t n, const TS* A, int64_t lda, int64_t nrows,
                const int64_t* I, TD* R, int64_t ldr) {
  hipLaunchKernelGGL((gather_rows_kernel<TS, TD>), dim3(grid_for(k * n)), dim3(256), 0,
                     ctx->stream, k, n, A, lda, nrows, I, R, ldr);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

int transpose_f64(rpid_ctx ctx, int64_t rows, int64_t cols, const double* X, int64_t ldx,
                  double* Y, int64_t ldy) {
  dim3 grid((unsigned)((rows + 31) / 32), (unsigned)((cols + 31) / 32));
  hipLaunchKernelGGL(transpose_kernel, grid, dim3(256), 0, ctx->stream, rows, cols, X, ldx, Y,
                     ldy);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

int add_trace_shift(rpid_ctx ctx, int64_t k, double* G, int64_t ldg, double c) {
  hipLaunchKernelGGL(trace_shift_kernel, dim3(1), dim3(256), 0, ctx->stream, k, G, ldg, c);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

int set_identity_columns(rpid_ctx ctx, int64_t k, const int64_t* J, double* Z, int64_t ldz) {
  hipLaunchKernelGGL(identity_cols_kernel, dim3(grid_for(k * k)), dim3(256), 0, ctx->stream, k, J,
                     Z, ldz);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

int split_bf16(rpid_ctx ctx, int64_t rows, int64_t cols, const double* S, int64_t lds, int parts,
               uint16_t* D, int64_t ldd) {
  hipLaunchKernelGGL(split_bf16_kernel, dim3(grid_for(rows * cols)), dim3(256), 0, ctx->stream,
                     rows, cols, S, lds, parts, D, ldd);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

template <typename TBt>
int tri_solve(rpid_ctx ctx, int64_t k, int64_t nrhs, const double* T, int64_t ldt, bool trans,
              bool lower_op, bool unit, const TBt* B, int64_t brs, int64_t bcs, double* X,
              int64_t xrs, int64_t xcs) {
  if (nrhs <= 0 || k <= 0) return RPID_OK;
  const size_t shmem = (size_t)TB_ * k * sizeof(double);
  if (shmem + sizeof(double) * TS_PART * TS_RHS * (TB_ + 1) > 160 * 1024)
    return RPID_ERR_UNSUPPORTED;
  RPID_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(tri_solve_kernel<TBt>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  hipLaunchKernelGGL((tri_solve_kernel<TBt>), dim3((unsigned)((nrhs + TS_RHS - 1) / TS_RHS)), dim3(256),
                     shmem, ctx->stream, k, nrhs, T, ldt, trans, lower_op, unit, B, brs, bcs, X,
                     xrs, xcs);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

int cholesky_batched(rpid_ctx ctx, int batch, int64_t k, double* G, int64_t ldg, int64_t stride,
                     int64_t* status_dev) {
  hipLaunchKernelGGL(cholesky_kernel, dim3(batch), dim3(1024), 0, ctx->stream, k, G, ldg, stride,
                     status_dev);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

#define RPID_INST2(TS, TD)                                                                      \
  template int convert_matrix<TS, TD>(rpid_ctx, int64_t, int64_t, const TS*, int64_t, TD*,      \
                                      int64_t);                                                  \
  template int gather_columns<TS, TD>(rpid_ctx, int64_t, int64_t, const TS*, int64_t, int64_t,  \
                                      const int64_t*, TD*, int64_t);                            \
  template int gather_rows<TS, TD>(rpid_ctx, int64_t, int64_t, const TS*, int64_t, int64_t,     \
                                   const int64_t*, TD*, int64_t);
RPID_INST2(double, double)
RPID_INST2(double, float)
RPID_INST2(float, double)
RPID_INST2(float, float)
RPID_INST2(uint16_t, double)
RPID_INST2(uint16_t, float)
RPID_INST2(uint16_t, uint16_t)
RPID_INST2(double, uint16_t)
RPID_INST2(float, uint16_t)
#undef RPID_INST2

template int tri_solve<double>(rpid_ctx, int64_t, int64_t, const double*, int64_t, bool, bool,
                               bool, const double*, int64_t, int64_t, double*, int64_t, int64_t);
template int tri_solve<float>(rpid_ctx, int64_t, int64_t, const double*, int64_t, bool, bool,
                              bool, const float*, int64_t, int64_t, double*, int64_t, int64_t);

}  // namespace rpid
