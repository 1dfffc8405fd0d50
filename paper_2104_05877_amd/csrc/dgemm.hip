// General FP64 GEMM C = alpha op(A) op(B) + beta C (column-major), used for
// the small and skinny products of the path (Gram matrices of C and R^T,
// Q_C^T A Q_R, the refinement residual of Z, C U).  On gfx950 the FP64
// vector FMA rate equals the FP64 MFMA rate, so a register-tiled vector
// kernel reaches the same ceiling; long-K shapes (k x k results over m or n)
// are split along K into a workspace and summed in a fixed order.
#include "rpid_internal.hpp"

namespace rpid {

namespace {
constexpr int TM = 64, TN = 64, TK = 16;

struct GemmArgs {
  bool ta, tb;
  int64_t M, N, K;
  const double* A;
  int64_t lda;
  const double* B;
  int64_t ldb;
  double* C;  // output (or partials)
  int64_t ldc;
  double alpha, beta;
  int64_t kchunk;
  int64_t part_stride;  // 0: write C with alpha/beta; else partial slices
};

__device__ __forceinline__ double opA(const GemmArgs& a, int64_t i, int64_t k) {
  return a.ta ? a.A[k + i * a.lda] : a.A[i + k * a.lda];
}
__device__ __forceinline__ double opB(const GemmArgs& a, int64_t k, int64_t j) {
  return a.tb ? a.B[j + k * a.ldb] : a.B[k + j * a.ldb];
}

__global__ __launch_bounds__(256) void dgemm_kernel(GemmArgs a) {
  __shared__ double As[TK][TM + 1];
  __shared__ double Bs[TK][TN + 1];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int64_t i0 = (int64_t)blockIdx.x * TM;
  const int64_t j0 = (int64_t)blockIdx.y * TN;
  const int64_t kb = (int64_t)blockIdx.z * a.kchunk;
  const int64_t ke = min(a.K, kb + a.kchunk);
  double acc[4][4] = {};
  for (int64_t k0 = kb; k0 < ke; k0 += TK) {
    // load op(A)[i0:i0+64, k0:k0+16] and op(B)[k0:k0+16, j0:j0+64]
    for (int e = tid; e < TM * TK; e += 256) {
      int ii, kk;
      if (a.ta) {
        kk = e % TK;
        ii = e / TK;
      } else {
        ii = e % TM;
        kk = e / TM;
      }
      const int64_t gi = i0 + ii, gk = k0 + kk;
      As[kk][ii] = (gi < a.M && gk < ke) ? opA(a, gi, gk) : 0.0;
    }
    for (int e = tid; e < TN * TK; e += 256) {
      int jj, kk;
      if (a.tb) {
        jj = e % TN;
        kk = e / TN;
      } else {
        kk = e % TK;
        jj = e / TK;
      }
      const int64_t gj = j0 + jj, gk = k0 + kk;
      Bs[kk][jj] = (gj < a.N && gk < ke) ? opB(a, gk, gj) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t gi = i0 + ty + 16 * i;
    if (gi >= a.M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t gj = j0 + tx + 16 * j;
      if (gj >= a.N) continue;
      if (a.part_stride) {
        a.C[(int64_t)blockIdx.z * a.part_stride + gi + gj * a.M] = acc[i][j];
      } else {
        double* c = &a.C[gi + gj * a.ldc];
        *c = a.alpha * acc[i][j] + (a.beta == 0.0 ? 0.0 : a.beta * *c);
      }
    }
  }
}

__global__ void dgemm_reduce_kernel(const double* part, int splits, int64_t stride, int64_t M,
                                    int64_t N, double alpha, double beta, double* C, int64_t ldc) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < M * N;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % M, j = e / M;
    double s = 0.0;
    for (int t = 0; t < splits; ++t) s += part[(int64_t)t * stride + e];
    double* c = &C[i + j * ldc];
    *c = alpha * s + (beta == 0.0 ? 0.0 : beta * *c);
  }
}
}  // namespace

int dgemm(rpid_ctx ctx, bool transA, bool transB, int64_t M, int64_t N, int64_t K, double alpha,
          const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
          int64_t ldc, size_t ws_off) {
  if (M <= 0 || N <= 0) return RPID_OK;
  GemmArgs a;
  a.ta = transA;
  a.tb = transB;
  a.M = M;
  a.N = N;
  a.K = K;
  a.A = A;
  a.lda = lda;
  a.B = B;
  a.ldb = ldb;
  a.C = C;
  a.ldc = ldc;
  a.alpha = alpha;
  a.beta = beta;
  const int64_t gm = (M + TM - 1) / TM, gn = (N + TN - 1) / TN;
  int64_t splits = 1;
  const int64_t want = 2 * (int64_t)ctx->num_cu;
  if (gm * gn < want && K > 4 * TK) {
    splits = (want + gm * gn - 1) / (gm * gn);
    const int64_t maxs = (K + 255) / 256;  // at least 256 of K per split
    if (splits > maxs) splits = maxs;
    if (splits > 64) splits = 64;
    if (splits < 1) splits = 1;
  }
  a.kchunk = ((K + splits - 1) / splits + TK - 1) / TK * TK;
  if (a.kchunk < TK) a.kchunk = TK;
  splits = (K + a.kchunk - 1) / a.kchunk;
  if (splits < 1) splits = 1;
  if (splits == 1) {
    a.part_stride = 0;
    hipLaunchKernelGGL(dgemm_kernel, dim3((unsigned)gm, (unsigned)gn, 1), dim3(256), 0,
                       ctx->stream, a);
    RPID_HIP_CHECK(hipGetLastError());
    return RPID_OK;
  }
  Carve cv;
  cv.off = ws_off;
  const size_t o_part = cv.take<double>((size_t)splits * M * N);
  RPID_CHECK(ws_check(ctx, cv.off));
  double* part = ws_ptr<double>(ctx, o_part);
  a.C = part;
  a.part_stride = M * N;
  hipLaunchKernelGGL(dgemm_kernel, dim3((unsigned)gm, (unsigned)gn, (unsigned)splits), dim3(256),
                     0, ctx->stream, a);
  RPID_HIP_CHECK(hipGetLastError());
  int64_t blocks = (M * N + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(dgemm_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, part,
                     (int)splits, M * N, M, N, alpha, beta, C, ldc);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

}  // namespace rpid
