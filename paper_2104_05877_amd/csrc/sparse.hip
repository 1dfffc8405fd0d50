// Sparse and structured sketches (Sec. 2.2): the sparse sign embedding and
// sketches of a matrix given in compressed sparse column (CSC) form.
//
//  * A sparse sign embedding has zeta entries +-1 per column (times a scale);
//    its random rows and signs come from the caller.  For a dense A the
//    cheapest way to apply it on gfx950 is the dense MFMA sketch with the
//    embedding expanded to exact +-1 entries (BF16, FP32 or FP64 alike), the
//    scale applied to X afterwards; the O(nnz zeta) count of the definition
//    pays off for sparse A, where the work is the nonzeros anyway.
//  * The SRTT embedding (subsampled randomized trigonometric transform with
//    the discrete Hartley transform) keeps l of the m transform rows, so on
//    MFMA hardware it is again cheapest as a dense l x m embedding, built from
//    its definition (sincos in FP64, stored in A's type) and fed to the dense
//    sketch.
//  * For a sparse A in CSC form the sparse sign embedding is applied as the
//    sparse operator it is (csc_sparse_sign_kernel below), O(nnz zeta).
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

// inv[perm[b]] = b for the entries of perm inside [0, m) (inv pre-filled with -1)
__global__ void invert_perm_kernel(int64_t m, const int32_t* perm, int32_t* inv) {
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < m; b += (int64_t)gridDim.x * blockDim.x) {
    const int32_t i = perm[b];
    if (i >= 0 && i < m) inv[i] = (int32_t)b;
  }
}
__global__ void fill_i32_kernel(int64_t count, int32_t* p, int32_t v) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
    p[e] = v;
}

template <typename TE>
__device__ __forceinline__ TE from_double(double v);
template <>
__device__ __forceinline__ double from_double<double>(double v) {
  return v;
}
template <>
__device__ __forceinline__ float from_double<float>(double v) {
  return (float)v;
}
template <>
__device__ __forceinline__ uint16_t from_double<uint16_t>(double v) {  // BF16, round to nearest even
  uint32_t u = __float_as_uint((float)v);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// The SRTT embedding transposed, Pt(i, r) = Gamma(r, i) = cas(2 pi sel[r] b /
// m) phi[b] / sqrt(l) with b = inv[i] the position that perm maps to row i
// (zero where inv[i] < 0); i varies fastest, so the writes are contiguous.
template <typename TE>
__global__ void srtt_build_kernel(int64_t m, int64_t l, const int32_t* inv, const int8_t* phi,
                                  const int32_t* sel, TE* Pt, int64_t ldp) {
  const int64_t total = m * l;
  const double two_pi_over_m = 6.283185307179586476925286766559 / (double)m;
  const double rs = 1.0 / sqrt((double)l);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % m, r = e / m;
    const int64_t b = inv[i];
    double v = 0.0;
    if (b >= 0) {
      int64_t a = sel[r] % m;
      if (a < 0) a += m;
      const int64_t q = (a * b) % m;
      double sn, cs;
      sincos(two_pi_over_m * (double)q, &sn, &cs);
      v = (cs + sn) * (double)phi[b] * rs;
    }
    Pt[i + r * ldp] = from_double<TE>(v);
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

// X(:, j) = scale * sum over the nonzeros a_ij of column j of S(:, i) a_ij for
// the sparse sign embedding S (zeta entries +-1 per column: rows[i zeta + s],
// signs[i zeta + s]) applied directly, O(nnz zeta) work: one wave per column
// of A keeps X(:, j) in LDS; its lanes take 64 / zeta nonzeros per round
// (lane = q zeta + s: nonzero q, entry s; four rounds' loads at once) and add
// sign * a_ij into row
// rows[i zeta + s] with LDS atomics issued nonzero by nonzero in storage
// order, so every row receives its terms in the same order on every run (LDS
// operations of one wave complete in order; the zeta rows of one column of
// S are distinct).  The additions are those of the expanded embedding (each
// term +-a_ij exact, one rounding per addition), and the scale is applied
// once at the end.  Rows of A outside [0, m), rows of S outside [0, l) and
// pointer ranges outside [0, nnz) are skipped.
template <typename T>
__global__ __launch_bounds__(256) void csc_sparse_sign_kernel(int64_t m, int64_t n, int64_t nnz,
                                                              const int64_t* colptr,
                                                              const int64_t* rowidx, const T* vals,
                                                              const int32_t* rows, const int8_t* signs,
                                                              int zeta, int l, T scale, T* X,
                                                              int64_t ldx) {
  __shared__ T acc[4][1024];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + wv;
  if (j >= n) return;
  T* a = acc[wv];
  for (int r = lane; r < l; r += 64) a[r] = T(0);
  int64_t p0 = colptr[j], p1 = colptr[j + 1];
  p0 = p0 < 0 ? 0 : (p0 > nnz ? nnz : p0);
  p1 = p1 < p0 ? p0 : (p1 > nnz ? nnz : p1);
  const int per = 64 / zeta;  // nonzeros per round
  const int q = lane / zeta, s = lane - q * zeta;
  // NR rounds at a time: all their loads are in flight together (two
  // dependent levels: the nonzeros, then their rows of S), then the adds
  constexpr int NR = 4;
  for (int64_t b = p0; b < p1; b += (int64_t)NR * per) {
    int64_t i[NR];
    T v[NR];
#pragma unroll
    for (int u = 0; u < NR; ++u) {
      const int64_t p = b + (int64_t)u * per + q;
      const bool ok = q < per && p < p1;
      i[u] = ok ? rowidx[p] : -1;
      v[u] = ok ? vals[p] : T(0);
    }
    int32_t r[NR];
    int sg[NR];
#pragma unroll
    for (int u = 0; u < NR; ++u) {
      const bool ok = i[u] >= 0 && i[u] < m;
      r[u] = ok ? rows[i[u] * zeta + s] : -1;
      sg[u] = ok ? (int)signs[i[u] * zeta + s] : 0;
    }
#pragma unroll
    for (int u = 0; u < NR; ++u) {
      const bool ok = r[u] >= 0 && r[u] < l && sg[u] != 0;
      const T c = sg[u] > 0 ? v[u] : -v[u];
      for (int qq = 0; qq < per; ++qq)
        if (ok && q == qq) atomicAdd(&a[r[u]], c);
    }
  }
  for (int r = lane; r < l; r += 64) X[r + j * ldx] = a[r] * scale;
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

template <typename TE>
int build_srtt_t(rpid_ctx ctx, int64_t m, int64_t l, const int32_t* perm, const int8_t* phi,
                 const int32_t* sel, int32_t* inv, TE* Pt, int64_t ldp) {
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(m)), dim3(256), 0, ctx->stream, m, inv, -1);
  RPID_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(invert_perm_kernel, dim3(grid_for(m)), dim3(256), 0, ctx->stream, m, perm, inv);
  RPID_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL((srtt_build_kernel<TE>), dim3(grid_for(m * l)), dim3(256), 0, ctx->stream, m, l, inv, phi,
                     sel, Pt, ldp);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}
template int build_srtt_t<double>(rpid_ctx, int64_t, int64_t, const int32_t*, const int8_t*, const int32_t*,
                                  int32_t*, double*, int64_t);
template int build_srtt_t<float>(rpid_ctx, int64_t, int64_t, const int32_t*, const int8_t*, const int32_t*,
                                 int32_t*, float*, int64_t);
template int build_srtt_t<uint16_t>(rpid_ctx, int64_t, int64_t, const int32_t*, const int8_t*, const int32_t*,
                                    int32_t*, uint16_t*, int64_t);

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
int csc_sparse_sign(rpid_ctx ctx, int64_t m, int64_t n, int64_t nnz, const int64_t* colptr,
                    const int64_t* rowidx, const T* vals, const int32_t* rows, const int8_t* signs,
                    int zeta, int64_t l, T scale, T* X, int64_t ldx) {
  if (l < 1 || l > 1024 || n < 1 || zeta < 1 || zeta > 64) return RPID_ERR_UNSUPPORTED;
  hipLaunchKernelGGL((csc_sparse_sign_kernel<T>), dim3((unsigned)((n + 3) / 4)), dim3(256), 0, ctx->stream, m,
                     n, nnz, colptr, rowidx, vals, rows, signs, zeta, (int)l, scale, X, ldx);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}
template int csc_sparse_sign<double>(rpid_ctx, int64_t, int64_t, int64_t, const int64_t*, const int64_t*,
                                     const double*, const int32_t*, const int8_t*, int, int64_t, double,
                                     double*, int64_t);
template int csc_sparse_sign<float>(rpid_ctx, int64_t, int64_t, int64_t, const int64_t*, const int64_t*,
                                    const float*, const int32_t*, const int8_t*, int, int64_t, float,
                                    float*, int64_t);

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
