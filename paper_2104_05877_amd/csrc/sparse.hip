// Sparse and structured sketches (Sec. 2.2): the sparse sign embedding and
// sketches of a matrix given in compressed sparse column (CSC) form.
//
//  * A sparse sign embedding has zeta entries +-1 per column (times a scale);
//    its random rows and signs come from the caller.  For a dense A the
//    cheapest way to apply it on gfx950 is the dense MFMA sketch with the
//    embedding expanded to exact +-1 entries (BF16, FP32 or FP64 alike), the
//    scale applied to X afterwards; the O(nnz zeta) count of the definition
//    pays off for sparse A, where the work is the nonzeros anyway.
//  * The CSC sketch X = Gamma A runs one workgroup per column of A: every
//    thread keeps up to four rows of X(:, j) in registers and adds
//    Gamma(:, i) a_ij for the column's nonzeros in order (deterministic), so
//    Gamma's columns (contiguous) are read once per nonzero, from L2.  Row
//    indices outside [0, m) and pointer ranges outside [0, nnz) are skipped
//    rather than followed.
#include "rpid_internal.hpp"

namespace rpid {

template <typename TE>
__device__ __forceinline__ TE sign_value(int s);
template <>
__device__ __forceinline__ double sign_value<double>(int s) {
  return s > 0 ? 1.0 : (s < 0 ? -1.0 : 0.0);
}
template <>
__device__ __forceinline__ float sign_value<float>(int s) {
  return s > 0 ? 1.0f : (s < 0 ? -1.0f : 0.0f);
}
template <>
__device__ __forceinline__ uint16_t sign_value<uint16_t>(int s) {  // BF16 bits of +-1, 0
  return s > 0 ? (uint16_t)0x3F80 : (s < 0 ? (uint16_t)0xBF80 : (uint16_t)0);
}

// out[r * rs + i * cs] = 0 for r < l, i < m (i_fast: i varies fastest)
template <typename TE>
__global__ void zero_embedding_kernel(int64_t m, int64_t l, TE* out, int64_t rs, int64_t cs, bool i_fast) {
  const int64_t total = m * l;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = i_fast ? e % m : e / l;
    const int64_t r = i_fast ? e / m : e % l;
    out[r * rs + i * cs] = sign_value<TE>(0);
  }
}

// out[rows[i, s] * rs + i * cs] = signs[i, s] for i < m, s < zeta (rows
// outside [0, l) are skipped; runs after the zero fill, same stream)
template <typename TE>
__global__ void scatter_signs_kernel(int64_t m, int64_t l, int zeta, const int32_t* rows,
                                     const int8_t* signs, TE* out, int64_t rs, int64_t cs) {
  const int64_t total = m * zeta;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / zeta;
    const int32_t r = rows[e];
    if (r >= 0 && r < l) out[(int64_t)r * rs + i * cs] = sign_value<TE>(signs[e]);
  }
}

template <typename T>
__global__ void scale_kernel(int64_t rows, int64_t cols, T* X, int64_t ldx, T scale) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x)
    X[e % rows + (e / rows) * ldx] *= scale;
}

// X(:, j) = sum over the nonzeros a_ij of column j of Gamma(:, i) a_ij
// (Gamma l x m, ldg; l <= 1024, four rows per thread).
template <typename T>
__global__ __launch_bounds__(256) void csc_sketch_kernel(int64_t m, int64_t n, int64_t nnz,
                                                         const int64_t* colptr,
                                                         const int64_t* rowidx, const T* vals,
                                                         const T* Gamma, int64_t ldg, int l,
                                                         T* X, int64_t ldx) {
  const int64_t j = blockIdx.x;
  if (j >= n) return;
  const int tid = threadIdx.x;
  int64_t p0 = colptr[j], p1 = colptr[j + 1];
  p0 = p0 < 0 ? 0 : (p0 > nnz ? nnz : p0);
  p1 = p1 < p0 ? p0 : (p1 > nnz ? nnz : p1);
  T acc[4] = {T(0), T(0), T(0), T(0)};
  for (int64_t p = p0; p < p1; ++p) {
    const int64_t i = rowidx[p];
    if (i < 0 || i >= m) continue;
    const T v = vals[p];
    const T* g = Gamma + i * ldg;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int r = tid + 256 * c;
      if (r < l) acc[c] = fma(g[r], v, acc[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int r = tid + 256 * c;
    if (r < l) X[r + j * ldx] = acc[c];
  }
}

// C(:, t) = A(:, J[t]) densified (J null: every column, t = j); row indices
// outside [0, m) are skipped.
template <typename T>
__global__ __launch_bounds__(256) void csc_gather_kernel(int64_t m, int64_t n, int64_t nnz,
                                                         const int64_t* colptr,
                                                         const int64_t* rowidx, const T* vals,
                                                         int64_t k, const int64_t* J, T* C,
                                                         int64_t ldc) {
  const int64_t t = blockIdx.x;
  if (t >= k) return;
  const int64_t j = J ? J[t] : t;
  T* c = C + t * ldc;
  for (int64_t i = threadIdx.x; i < m; i += blockDim.x) c[i] = T(0);
  __syncthreads();
  if (j < 0 || j >= n) return;
  int64_t p0 = colptr[j], p1 = colptr[j + 1];
  p0 = p0 < 0 ? 0 : (p0 > nnz ? nnz : p0);
  p1 = p1 < p0 ? p0 : (p1 > nnz ? nnz : p1);
  for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
    const int64_t i = rowidx[p];
    if (i >= 0 && i < m) c[i] = vals[p];
  }
}

static unsigned grid_for(int64_t total) {
  int64_t b = (total + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (unsigned)b;
}

template <typename TE>
int expand_sparse_sign(rpid_ctx ctx, int64_t m, int64_t l, int zeta, const int32_t* rows,
                       const int8_t* signs, TE* out, int64_t rs, int64_t cs, bool i_fast) {
  hipLaunchKernelGGL((zero_embedding_kernel<TE>), dim3(grid_for(m * l)), dim3(256), 0, ctx->stream, m, l,
                     out, rs, cs, i_fast);
  RPID_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL((scatter_signs_kernel<TE>), dim3(grid_for(m * zeta)), dim3(256), 0, ctx->stream, m, l,
                     zeta, rows, signs, out, rs, cs);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}
template int expand_sparse_sign<double>(rpid_ctx, int64_t, int64_t, int, const int32_t*,
                                        const int8_t*, double*, int64_t, int64_t, bool);
template int expand_sparse_sign<float>(rpid_ctx, int64_t, int64_t, int, const int32_t*,
                                       const int8_t*, float*, int64_t, int64_t, bool);
template int expand_sparse_sign<uint16_t>(rpid_ctx, int64_t, int64_t, int, const int32_t*,
                                          const int8_t*, uint16_t*, int64_t, int64_t, bool);

template <typename T>
int scale_matrix(rpid_ctx ctx, int64_t rows, int64_t cols, T* X, int64_t ldx, T scale) {
  hipLaunchKernelGGL((scale_kernel<T>), dim3(grid_for(rows * cols)), dim3(256), 0, ctx->stream, rows,
                     cols, X, ldx, scale);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}
template int scale_matrix<double>(rpid_ctx, int64_t, int64_t, double*, int64_t, double);
template int scale_matrix<float>(rpid_ctx, int64_t, int64_t, float*, int64_t, float);

template <typename T>
int csc_sketch(rpid_ctx ctx, int64_t m, int64_t n, int64_t nnz, const int64_t* colptr,
               const int64_t* rowidx, const T* vals, const T* Gamma, int64_t ldg, int64_t l, T* X,
               int64_t ldx) {
  if (l < 1 || l > 1024 || n < 1) return RPID_ERR_UNSUPPORTED;
  hipLaunchKernelGGL((csc_sketch_kernel<T>), dim3((unsigned)n), dim3(256), 0, ctx->stream, m, n, nnz,
                     colptr, rowidx, vals, Gamma, ldg, (int)l, X, ldx);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}
template int csc_sketch<double>(rpid_ctx, int64_t, int64_t, int64_t, const int64_t*, const int64_t*,
                                const double*, const double*, int64_t, int64_t, double*, int64_t);
template int csc_sketch<float>(rpid_ctx, int64_t, int64_t, int64_t, const int64_t*, const int64_t*,
                               const float*, const float*, int64_t, int64_t, float*, int64_t);

template <typename T>
int csc_gather(rpid_ctx ctx, int64_t m, int64_t n, int64_t nnz, const int64_t* colptr,
               const int64_t* rowidx, const T* vals, int64_t k, const int64_t* J, T* C, int64_t ldc) {
  if (k < 1) return RPID_OK;
  hipLaunchKernelGGL((csc_gather_kernel<T>), dim3((unsigned)k), dim3(256), 0, ctx->stream, m, n, nnz,
                     colptr, rowidx, vals, k, J, C, ldc);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}
template int csc_gather<double>(rpid_ctx, int64_t, int64_t, int64_t, const int64_t*, const int64_t*,
                                const double*, int64_t, const int64_t*, double*, int64_t);
template int csc_gather<float>(rpid_ctx, int64_t, int64_t, int64_t, const int64_t*, const int64_t*,
                               const float*, int64_t, const int64_t*, float*, int64_t);

}  // namespace rpid
