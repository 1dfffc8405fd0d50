// General FP64 GEMM C = alpha op(A) op(B) + beta C (column-major), used for
// the small and skinny products of the path (Gram matrices of C and R^T,
// Q_C^T A Q_R, the refinement residual of Z, C U).  On gfx950 the FP64
// vector FMA rate equals the FP64 MFMA rate, so a register-tiled vector
// kernel reaches the same ceiling; long-K shapes (k x k results over m or n)
// are split along K into a workspace and summed in a fixed order.
#include "rpid_internal.hpp"

namespace rpid {

namespace {
constexpr int TM = 64, TN = 64, TK = 32;

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


typedef double v4d __attribute__((ext_vector_type(4)));

// 64 x 64 output tile per workgroup; 4 waves each own a 32 x 32 quadrant
// (2 x 2 FP64 MFMA 16x16x4 tiles).  op(A) / op(B) tiles of 32 along K are
// staged in LDS (transposes resolved while staging).  The global loads run
// two K-steps ahead in two register sets, so one K-step's MFMAs (32 per
// wave) cover the latency of the loads of the step after next.
// Two waves per SIMD (the accumulators then live in VGPRs, about 250 in
// all) instead of one: the 16384^2, k = 512 decomposition, whose Cholesky-QR
// products run here, 10.4 -> 9.5 ms.
template <bool TA, bool TB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void dgemm_kernel(GemmArgs a) {
  __shared__ double As[TK][TM + 1];
  __shared__ double Bs[TK][TN + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int wr = (wid & 1) * 32, wc = (wid >> 1) * 32;
  const int64_t i0 = (int64_t)blockIdx.x * TM;
  const int64_t j0 = (int64_t)blockIdx.y * TN;
  const int64_t kb = (int64_t)blockIdx.z * a.kchunk;
  const int64_t ke = min(a.K, kb + a.kchunk);
  v4d acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = v4d{};
  // Tile loads: each thread fetches PER elements of op(A) and of op(B) per
  // K-step, along the contiguous dimension of the stored matrix: element
  // e = tid + 256 u of the tile, (i, k) = (e % TM, e / TM) for a stored A
  // (column-major, i contiguous) and (e / TK, e % TK) for a transposed one.
  constexpr int PER = TM * TK / 256;
  static_assert(256 % TM == 0 && 256 % TK == 0, "staging layout");
  auto ai = [&](int u) { return TA ? (tid + 256 * u) / TK : (tid + 256 * u) % TM; };
  auto ak = [&](int u) { return TA ? (tid + 256 * u) % TK : (tid + 256 * u) / TM; };
  auto bj = [&](int u) { return TB ? (tid + 256 * u) % TN : (tid + 256 * u) / TK; };
  auto bk = [&](int u) { return TB ? (tid + 256 * u) / TN : (tid + 256 * u) % TK; };
  struct Regs {
    double av[PER], bv[PER];
  };
  auto fetch = [&](Regs& r, int64_t k0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int64_t gi = i0 + ai(u), gk = k0 + ak(u);
      r.av[u] = (gi < a.M && gk < ke) ? (TA ? a.A[gk + gi * a.lda] : a.A[gi + gk * a.lda]) : 0.0;
      const int64_t gj = j0 + bj(u), gq = k0 + bk(u);
      r.bv[u] = (gj < a.N && gq < ke) ? (TB ? a.B[gj + gq * a.ldb] : a.B[gq + gj * a.ldb]) : 0.0;
    }
  };
  auto step = [&](const Regs& r) {
    __syncthreads();  // the previous step's LDS reads are done
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      As[ak(u)][ai(u)] = r.av[u];
      Bs[bk(u)][bj(u)] = r.bv[u];
    }
    __syncthreads();
  };
  auto multiply = [&]() {
#pragma unroll
    for (int s = 0; s < TK / 4; ++s) {
      const int kk = s * 4 + (lane >> 4);
      double pa[2], qb[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) pa[x] = As[kk][wr + x * 16 + (lane & 15)];
#pragma unroll
      for (int y = 0; y < 2; ++y) qb[y] = Bs[kk][wc + y * 16 + (lane & 15)];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[x], qb[y], acc[x][y], 0, 0, 0);
    }
  };
  Regs r0, r1;
  if (kb < ke) fetch(r0, kb);
  if (kb + TK < ke) fetch(r1, kb + TK);
  for (int64_t k0 = kb; k0 < ke; k0 += 2 * TK) {
    step(r0);
    if (k0 + 2 * TK < ke) fetch(r0, k0 + 2 * TK);
    multiply();
    if (k0 + TK >= ke) break;
    step(r1);
    if (k0 + 3 * TK < ke) fetch(r1, k0 + 3 * TK);
    multiply();
  }
  // FP64 MFMA result: register i of lane l is row (l / 16) + 4 i, column l % 16
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t gi = i0 + wr + x * 16 + (lane >> 4) + 4 * i;
        const int64_t gj = j0 + wc + y * 16 + (lane & 15);
        if (gi < a.M && gj < a.N) {
          if (a.part_stride) {
            a.C[(int64_t)blockIdx.z * a.part_stride + gi + gj * a.M] = acc[x][y][i];
          } else {
            double* c = &a.C[gi + gj * a.ldc];
            *c = a.alpha * acc[x][y][i] + (a.beta == 0.0 ? 0.0 : a.beta * *c);
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
    // eight loads in flight per round, added in the same order as one by one
    int t = 0;
    for (; t + 8 <= splits; t += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(t + u) * stride + e];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; t < splits; ++t) s += part[(int64_t)t * stride + e];
    double* c = &C[i + j * ldc];
    *c = alpha * s + (beta == 0.0 ? 0.0 : beta * *c);
  }
}
}  // namespace

static void launch_dgemm(rpid_ctx ctx, const GemmArgs& a, dim3 grid) {
  if (a.ta && a.tb)
    hipLaunchKernelGGL((dgemm_kernel<true, true>), grid, dim3(256), 0, ctx->stream, a);
  else if (a.ta)
    hipLaunchKernelGGL((dgemm_kernel<true, false>), grid, dim3(256), 0, ctx->stream, a);
  else if (a.tb)
    hipLaunchKernelGGL((dgemm_kernel<false, true>), grid, dim3(256), 0, ctx->stream, a);
  else
    hipLaunchKernelGGL((dgemm_kernel<false, false>), grid, dim3(256), 0, ctx->stream, a);
}

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
  if (gm * gn < want && K > 2 * TK) {
    splits = (want + gm * gn - 1) / (gm * gn);
    const int64_t maxs = (K + 2 * TK - 1) / (2 * TK);  // at least two K-steps per split
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
    launch_dgemm(ctx, a, dim3((unsigned)gm, (unsigned)gn, 1));
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
  launch_dgemm(ctx, a, dim3((unsigned)gm, (unsigned)gn, (unsigned)splits));
  RPID_HIP_CHECK(hipGetLastError());
  int64_t blocks = (M * N + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(dgemm_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, part,
                     (int)splits, M * N, M, N, alpha, beta, C, ldc);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

}  // namespace rpid
