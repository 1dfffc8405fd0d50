// Residual of a decomposition, ||A - P Q||_F^2 and ||A||_F^2, by explicit
// differences: a GEMM whose product tile is never stored -- the epilogue
// subtracts it from the matching tile of A, squares and sums.  P is m x r,
// Q is r x n.
//
//  * FP64 form: P, Q FP64 on FP64 MFMA (16x16x4), A promoted to FP64.
//  * BF16 form: A is BF16; P and Q are BF16 with the FP64 factor split into
//    several BF16 terms beforehand (the r dimension holds the terms), run on
//    BF16 MFMA (16x16x32) with FP32 accumulation; the epilogue works in FP64.
// Per-workgroup partial sums go to a workspace and are added in a fixed
// order (deterministic).
#include "rpid_internal.hpp"

namespace rpid {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

namespace {

// ---------------------------------------------------------------------------
// FP64 form.  Workgroup tile 64 x 64 (4 waves, each 32 x 32 = 2 x 2 MFMA
// tiles), K staged 16 at a time in LDS.
// ---------------------------------------------------------------------------
// Four waves per SIMD (the accumulators then live in VGPRs, 104 in all):
// 0.74 ms against 0.83 ms at three for the 8192^2, k = 256 FP64 residual.
template <typename TA>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
void residual_f64_kernel(int64_t m, int64_t n, int64_t r, const TA* A, int64_t lda, const double* P,
                         int64_t ldp, const double* Q, int64_t ldq, double* partials) {
  constexpr int BK = 16;
  __shared__ double Ps[BK][64 + 1];
  __shared__ double Qs[BK][64 + 1];
  __shared__ double red[2][4];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * 64, j0 = (int64_t)blockIdx.y * 64;
  const int wr = (wid & 1) * 32, wc = (wid >> 1) * 32;
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d{};
  // 4 elements of each operand per thread per K-step, fetched one step ahead
  double pn[4], qn[4];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 256 * u;
      const int ii = e % 64, kk = e / 64;
      const int64_t gi = i0 + ii, gk = k0 + kk;
      pn[u] = (gi < m && gk < r) ? P[gi + gk * ldp] : 0.0;
      const int jj = e / BK, kq = e % BK;
      const int64_t gj = j0 + jj, gq = k0 + kq;
      qn[u] = (gj < n && gq < r) ? Q[gq + gj * ldq] : 0.0;
    }
  };
  fetch(0);
  for (int64_t k0 = 0; k0 < r; k0 += BK) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 256 * u;
      Ps[e / 64][e % 64] = pn[u];
      Qs[e % BK][e / BK] = qn[u];
    }
    __syncthreads();
    if (k0 + BK < r) fetch(k0 + BK);
#pragma unroll
    for (int s = 0; s < BK / 4; ++s) {
      const int kk = s * 4 + (lane >> 4);
      double pa[2], qb[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) pa[a] = Ps[kk][wr + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < 2; ++b) qb[b] = Qs[kk][wc + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[a], qb[b], acc[a][b], 0, 0, 0);
    }
  }
  // epilogue: the FP64 MFMA leaves row (lane/16) + 4 i of each 16 x 16 tile
  // in accumulator register i: element (wr + 16a + lane/16 + 4i, wc + 16b + lane%16)
  double sd = 0.0, sa = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t gi = i0 + wr + a * 16 + (lane >> 4) + 4 * i;
        const int64_t gj = j0 + wc + b * 16 + (lane & 15);
        if (gi < m && gj < n) {
          const double av = load_as_double<TA>(A, gi + gj * lda);
          const double d = av - acc[a][b][i];
          sd = fma(d, d, sd);
          sa = fma(av, av, sa);
        }
      }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    sd += __shfl_xor(sd, off, 64);
    sa += __shfl_xor(sa, off, 64);
  }
  if (lane == 0) {
    red[0][wid] = sd;
    red[1][wid] = sa;
  }
  __syncthreads();
  if (tid == 0) {
    const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    partials[2 * b] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    partials[2 * b + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

// ---------------------------------------------------------------------------
// BF16 form.  Workgroup tile 128 x 128 (4 waves, each 64 x 64 = 4 x 4 MFMA
// tiles of 16x16x32), K staged 32 at a time in LDS.  Both operands arrive
// k-contiguous: Pt is r x m column-major (row i of P is Pt(:, i)) and Q is
// r x n column-major, so every 8 consecutive k of one row/column are one
// 16-byte load.  The next K-step's tiles are prefetched into registers
// while the current one is multiplied.
// ---------------------------------------------------------------------------
constexpr int RB_BK = 32;
constexpr int RB_PAD = RB_BK + 8;  // 80-byte LDS rows: 16-byte aligned, banks spread

__device__ __forceinline__ uint4 load8_bf16(const uint16_t* base, int64_t ld, int64_t row,
                                            int64_t nrows, int64_t k, int64_t r, bool vec_ok) {
  // elements k..k+7 of column `row` of a (r x nrows, ld) k-contiguous matrix
  uint4 v = make_uint4(0u, 0u, 0u, 0u);
  if (row >= nrows) return v;
  const uint16_t* p = base + row * ld + k;
  if (vec_ok && k + 8 <= r) return *reinterpret_cast<const uint4*>(p);
  uint16_t t[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) t[e] = (k + e < r) ? p[e] : (uint16_t)0;
  __builtin_memcpy(&v, t, 16);
  return v;
}

__global__ __launch_bounds__(256) void residual_bf16_kernel(int64_t m, int64_t n, int64_t r,
                                                            const uint16_t* A, int64_t lda,
                                                            const uint16_t* Pt, int64_t ldpt,
                                                            const uint16_t* Q, int64_t ldq,
                                                            double* partials) {
  __shared__ __attribute__((aligned(16))) uint16_t Ps[128][RB_PAD];  // Ps[row][k]
  __shared__ __attribute__((aligned(16))) uint16_t Qs[128][RB_PAD];  // Qs[col][k]
  __shared__ double red[2][4];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * 128, j0 = (int64_t)blockIdx.y * 128;
  const int wr = (wid & 1) * 64, wc = (wid >> 1) * 64;
  const bool vec_ok = ((uintptr_t)Pt % 16 == 0) && ((uintptr_t)Q % 16 == 0) && (ldpt % 8 == 0) &&
                      (ldq % 8 == 0);
  // each thread moves 2 vectors of P and 2 of Q per K-step: (row, k-octet)
  const int lr0 = tid >> 2, lk0 = (tid & 3) * 8;  // rows 0..63, then +64
  v4f acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = v4f{};
  uint4 pv[2], qv[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    pv[h] = load8_bf16(Pt, ldpt, i0 + lr0 + 64 * h, m, lk0, r, vec_ok);
    qv[h] = load8_bf16(Q, ldq, j0 + lr0 + 64 * h, n, lk0, r, vec_ok);
  }
  for (int64_t k0 = 0; k0 < r; k0 += RB_BK) {
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      *reinterpret_cast<uint4*>(&Ps[lr0 + 64 * h][lk0]) = pv[h];
      *reinterpret_cast<uint4*>(&Qs[lr0 + 64 * h][lk0]) = qv[h];
    }
    __syncthreads();
    if (k0 + RB_BK < r) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        pv[h] = load8_bf16(Pt, ldpt, i0 + lr0 + 64 * h, m, k0 + RB_BK + lk0, r, vec_ok);
        qv[h] = load8_bf16(Q, ldq, j0 + lr0 + 64 * h, n, k0 + RB_BK + lk0, r, vec_ok);
      }
    }
    v8bf pa[4], qb[4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
      __builtin_memcpy(&pa[a], &Ps[wr + a * 16 + (lane & 15)][(lane >> 4) * 8], 16);
#pragma unroll
    for (int b = 0; b < 4; ++b)
      __builtin_memcpy(&qb[b], &Qs[wc + b * 16 + (lane & 15)][(lane >> 4) * 8], 16);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pa[a], qb[b], acc[a][b], 0, 0, 0);
  }
  double sd = 0.0, sa = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t gi = i0 + wr + a * 16 + 4 * (lane >> 4) + i;
        const int64_t gj = j0 + wc + b * 16 + (lane & 15);
        if (gi < m && gj < n) {
          const double av = (double)bf16_bits_to_float(A[gi + gj * lda]);
          const double d = av - (double)acc[a][b][i];
          sd = fma(d, d, sd);
          sa = fma(av, av, sa);
        }
      }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    sd += __shfl_xor(sd, off, 64);
    sa += __shfl_xor(sa, off, 64);
  }
  if (lane == 0) {
    red[0][wid] = sd;
    red[1][wid] = sa;
  }
  __syncthreads();
  if (tid == 0) {
    const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    partials[2 * b] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    partials[2 * b + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

// Pt((c + p k), i) = A(i, J[c]) for every term p (BF16 skeleton columns,
// replicated once per term of the other factor).
__global__ void pack_cols_t_kernel(int64_t m, int64_t k, int parts, const uint16_t* A,
                                   int64_t lda, int64_t ncols, const int64_t* J, uint16_t* Pt) {
  const int64_t rr = (int64_t)parts * k;
  const int64_t total = m * rr;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e % k, i = (e / k) % m, p = e / (k * m);
    (void)p;
    const int64_t j = J[c];
    const uint16_t v = (j >= 0 && j < ncols) ? A[i + j * lda] : (uint16_t)0;
    Pt[(c + p * k) + i * rr] = v;
  }
}

// Pt((c + p k), i) = term p of the BF16 split of P(i, c) (P FP64 m x k).
__global__ void pack_split_t_kernel(int64_t m, int64_t k, int parts, const double* P,
                                    int64_t ldp, uint16_t* Pt) {
  const int64_t rr = (int64_t)parts * k;
  const int64_t total = m * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e % k, i = e / k;
    double v = P[i + c * ldp];
    for (int p = 0; p < parts; ++p) {
      const uint16_t b = float_to_bf16_bits((float)v);
      Pt[(c + p * k) + i * rr] = b;
      v -= (double)bf16_bits_to_float(b);
    }
  }
}

// out[0] = sum partials[2b], out[1] = sum partials[2b+1] in a fixed order.
__global__ __launch_bounds__(1024) void partial_sum_kernel(const double* partials, int64_t count,
                                                           double* out) {
  __shared__ double r0[1024], r1[1024];
  const int tid = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int64_t i = tid; i < count; i += 1024) {
    a += partials[2 * i];
    b += partials[2 * i + 1];
  }
  r0[tid] = a;
  r1[tid] = b;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (tid < w) {
      r0[tid] += r0[tid + w];
      r1[tid] += r1[tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[0] = r0[0];
    out[1] = r1[0];
  }
}

}  // namespace

size_t residual_partials(int64_t m, int64_t n, bool bf16) {
  const int64_t t = bf16 ? 128 : 64;
  return (size_t)((m + t - 1) / t) * ((n + t - 1) / t) * 2;
}

template <typename TA>
int residual_f64(rpid_ctx ctx, int64_t m, int64_t n, int64_t r, const TA* A, int64_t lda,
                 const double* P, int64_t ldp, const double* Q, int64_t ldq, double* partials,
                 double* out2) {
  dim3 grid((unsigned)((m + 63) / 64), (unsigned)((n + 63) / 64));
  hipLaunchKernelGGL((residual_f64_kernel<TA>), grid, dim3(256), 0, ctx->stream, m, n, r, A, lda,
                     P, ldp, Q, ldq, partials);
  RPID_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(partial_sum_kernel, dim3(1), dim3(1024), 0, ctx->stream, partials,
                     (int64_t)grid.x * grid.y, out2);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

int residual_bf16(rpid_ctx ctx, int64_t m, int64_t n, int64_t r, const uint16_t* A, int64_t lda,
                  const uint16_t* Pt, int64_t ldpt, const uint16_t* Q, int64_t ldq,
                  double* partials, double* out2) {
  int64_t count = 0;
  int err = RPID_OK;
  if (residual_stream_bf16(ctx, m, n, r, A, lda, Pt, ldpt, Q, ldq, partials, &count, &err)) {
    RPID_CHECK(err);
    hipLaunchKernelGGL(partial_sum_kernel, dim3(1), dim3(1024), 0, ctx->stream, partials, count, out2);
    RPID_HIP_CHECK(hipGetLastError());
    return RPID_OK;
  }
  dim3 grid((unsigned)((m + 127) / 128), (unsigned)((n + 127) / 128));
  hipLaunchKernelGGL(residual_bf16_kernel, grid, dim3(256), 0, ctx->stream, m, n, r, A, lda, Pt,
                     ldpt, Q, ldq, partials);
  RPID_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(partial_sum_kernel, dim3(1), dim3(1024), 0, ctx->stream, partials,
                     (int64_t)grid.x * grid.y, out2);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

int pack_cols_t(rpid_ctx ctx, int64_t m, int64_t k, int parts, const uint16_t* A, int64_t lda,
                int64_t ncols, const int64_t* J, uint16_t* Pt) {
  hipLaunchKernelGGL(pack_cols_t_kernel, dim3(4096), dim3(256), 0, ctx->stream, m, k, parts, A,
                     lda, ncols, J, Pt);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

int pack_split_t(rpid_ctx ctx, int64_t m, int64_t k, int parts, const double* P, int64_t ldp,
                 uint16_t* Pt) {
  hipLaunchKernelGGL(pack_split_t_kernel, dim3(4096), dim3(256), 0, ctx->stream, m, k, parts, P,
                     ldp, Pt);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

template int residual_f64<double>(rpid_ctx, int64_t, int64_t, int64_t, const double*, int64_t,
                                  const double*, int64_t, const double*, int64_t, double*,
                                  double*);
template int residual_f64<float>(rpid_ctx, int64_t, int64_t, int64_t, const float*, int64_t,
                                 const double*, int64_t, const double*, int64_t, double*, double*);
template int residual_f64<uint16_t>(rpid_ctx, int64_t, int64_t, int64_t, const uint16_t*, int64_t,
                                    const double*, int64_t, const double*, int64_t, double*,
                                    double*);

}  // namespace rpid
